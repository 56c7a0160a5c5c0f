"""GPU parity of the closed-region entry points (pft_forward_3d_regions, pft_backward_3d_regions):
F = sum_j rho_j F_j, F_j, dL/dv, dL/drho and dL/dQ against the FP64 oracle."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle as O
import paper_2104_08309_amd as pft
from gpu_util import TOL_FP32C, TOL_FP64, dev, host, nrel, special_q, step

pytestmark = pytest.mark.gpu

TOL_GRAD64 = 1e-10


def fwd(v, t, off, rho, q, mode, qdt=torch.float64):
    F, Fj, I = pft.forward_3d_regions(dev(v, torch.float64), dev(t, torch.int32), off, dev(rho, torch.float64),
                                      dev(q, qdt), mode=mode, per_region=True, intensity=True)
    torch.cuda.synchronize()
    return host(F), host(Fj), host(I)


def bwd(v, t, off, rho, q, g, mode, **kw):
    cdt = torch.complex128 if mode == "fp64" else torch.complex64
    res = pft.backward_3d_regions(dev(v, torch.float64), dev(t, torch.int32), off, dev(rho, torch.float64),
                                  dev(q, torch.float64), dev(g).to(cdt), mode=mode, **kw)
    torch.cuda.synchronize()
    return [None if x is None else host(x).astype(np.float64) for x in res]


def core_shell():
    return mg.nested_boxes(((2.0, 1.6, 1.8), (-1.0, -0.7, -0.9)), ((0.9, 0.5, 0.7), (-0.3, -0.2, 0.1)))


def test_core_shell_boxes_forward(gpu):
    """Two regions sharing the inner box's vertices; Q = 0, the axes (face normals), tiny Q."""
    v, t, off = core_shell()
    rho = np.array([3.0, -0.5])
    rng = np.random.default_rng(51)
    q = np.concatenate([rng.normal(size=(600, 3)) * 3.0, special_q(4.0), [[1e-6, 0, 0], [0, 2e-3, 1e-3]]])
    want, want_j = O.ft3d_regions(v, t, off, rho, q)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"regions core-shell forward {mode}")
        F, Fj, I = fwd(v, t, off, rho, q, mode)
        assert nrel(F, want) < tol, mode
        for j in range(2):
            assert nrel(Fj[j], want_j[j]) < tol, (mode, j)
        assert nrel(I, np.abs(want) ** 2) < 2 * tol, mode


def test_layered_sphere_sorted_size(gpu):
    """Core and two shells (level-2 icospheres, shared interface vertices), 9000 Q: the Morton-
    ordered path with region-aligned face splits; an empty region in the middle."""
    v, t, off = mg.layered_sphere(2, [0.6, 0.9, 1.2], centre=(0.3, -0.2, 0.1))
    off = np.array([off[0], off[1], off[1], off[2], off[3]])  # region 1 empty
    rho = np.array([2.0, 7.0, -1.0, 0.5])
    rng = np.random.default_rng(52)
    q = mg.q_random_ball(9000, 12.0, rng)
    want, want_j = O.ft3d_regions(v, t, off, rho, q)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"regions layered sphere forward {mode}")
        F, Fj, _ = fwd(v, t, off, rho, q, mode)
        assert nrel(F, want) < tol, mode
        assert np.all(Fj[1] == 0), mode
        for j in (0, 2, 3):
            assert nrel(Fj[j], want_j[j]) < tol, (mode, j)


def test_one_region_matches_forward_3d(gpu):
    v, t = mg.icosphere(3, 2.0)
    rng = np.random.default_rng(53)
    q = mg.q_random_ball(9000, 5.0, rng)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"regions single region vs forward_3d {mode}")
        F, _, _ = fwd(v, t, [0, len(t)], np.array([1.0]), q, mode)
        ref = host(pft.forward_3d(dev(v, torch.float64), dev(t, torch.int32), dev(q), mode=mode))
        assert nrel(F, ref) < tol, mode


def test_grad_q_single_mesh(gpu):
    """dL/dQ against the oracle's grad_Q F: generic Q, Q = 0, |Q| R below and above the
    tetrahedron-series threshold, the axes, a face normal; f32 Q in the FP32C form."""
    rng = np.random.default_rng(54)
    v, t = mg.ellipsoid_uv([3.0, 2.0, 1.5], 8, rot=np.linalg.qr(rng.normal(size=(3, 3)))[0], centre=(0.4, -0.8, 0.2))
    R = np.max(np.linalg.norm(v - v.mean(0), axis=1))
    N = np.cross(v[t[5, 1]] - v[t[5, 0]], v[t[5, 2]] - v[t[5, 0]])
    d = rng.normal(size=(40, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    q = np.concatenate([mg.q_random_ball(2000, 4.0, rng), special_q(3.0), 2.0 * N[None] / np.linalg.norm(N),
                        d[:20] * 0.3 / R, d[20:] * 0.7 / R])
    g = rng.normal(size=len(q)) + 1j * rng.normal(size=len(q))
    dq = O.ft3d_dq(v, t, q)
    for mode, tol in (("fp64", TOL_GRAD64), ("fp32c", TOL_FP32C)):
        gg = g if mode == "fp64" else g.astype(np.complex64).astype(np.complex128)
        want = np.real(np.conj(gg)[:, None] * dq)
        step(f"grad_Q single mesh {mode}")
        _, _, gq = bwd(v, t, [0, len(t)], np.array([1.0]), q, gg, mode, need_verts=False, need_rho=False)
        e = nrel(gq, want)
        print(f"{mode} grad_Q rel err {e:.3e}")
        assert e < tol, mode
        small = np.linalg.norm(q, axis=1) * R < 0.5
        assert nrel(gq[small], want[small]) < 10 * tol, mode


def test_all_gradients_with_regions(gpu):
    """dL/dv, dL/drho and dL/dQ on the layered sphere (shared interface vertices) against
    oracle.grad3d_regions; the rho-only path (forward partials) agrees with the grad_Q path."""
    v, t, off = mg.layered_sphere(1, [0.7, 1.0, 1.3], centre=(0.1, 0.2, -0.3))
    rho = np.array([1.5, -0.7, 2.2])
    rng = np.random.default_rng(55)
    q = np.concatenate([mg.q_random_ball(900, 6.0, rng), special_q(4.0)])
    g = rng.normal(size=len(q)) + 1j * rng.normal(size=len(q))
    for mode, tol in (("fp64", TOL_GRAD64), ("fp32c", TOL_FP32C)):
        gg = g if mode == "fp64" else g.astype(np.complex64).astype(np.complex128)
        wv, wr, wq = O.grad3d_regions(v, t, off, rho, q, gg)
        step(f"regions all gradients {mode}")
        gv, gr, gq = bwd(v, t, off, rho, q, gg, mode)
        assert nrel(gv, wv) < tol, mode
        assert nrel(gr, wr) < tol, mode
        assert nrel(gq, wq) < tol, mode
        step(f"regions rho-only gradient {mode}")
        _, gr2, _ = bwd(v, t, off, rho, q, gg, mode, need_verts=False, need_q=False)
        assert nrel(gr2, wr) < tol, mode


def test_autograd_regions(gpu):
    """PftRegionsFunction: torch.autograd gradients to vertices, densities and Q agree with the
    oracle for L = sum |F|^2 (grad_out = 2F, formed by torch from the library's F)."""
    v, t, off = core_shell()
    rho0 = np.array([3.0, -0.5])
    rng = np.random.default_rng(56)
    q = rng.normal(size=(300, 3)) * 2.0
    V = dev(v, torch.float64).requires_grad_(True)
    rho = dev(rho0, torch.float64).requires_grad_(True)
    Q = dev(q, torch.float64).requires_grad_(True)
    step("regions autograd fp64")
    F = pft.ft3d_regions(V, dev(t, torch.int32), off, rho, Q, mode="fp64")
    loss = torch.sum(F.real ** 2 + F.imag ** 2)
    loss.backward()
    torch.cuda.synchronize()
    Fo, _ = O.ft3d_regions(v, t, off, rho0, q)
    wv, wr, wq = O.grad3d_regions(v, t, off, rho0, q, 2.0 * Fo)
    assert nrel(host(V.grad), wv) < TOL_GRAD64
    assert nrel(host(rho.grad), wr) < TOL_GRAD64
    assert nrel(host(Q.grad), wq) < TOL_GRAD64
    step("single-mesh autograd with Q gradient fp32c")
    v1, t1 = mg.icosphere(2, 1.5)
    Q1 = dev(q, torch.float32).requires_grad_(True)
    F1 = pft.ft3d(dev(v1, torch.float32), dev(t1, torch.int32), Q1, mode="fp32c")
    torch.sum(F1.real ** 2 + F1.imag ** 2).backward()
    torch.cuda.synchronize()
    q32 = q.astype(np.float32).astype(np.float64)
    v32 = v1.astype(np.float32).astype(np.float64)
    Fo1 = O.ft3d(v32, t1, q32)
    want = np.real(np.conj(2.0 * Fo1)[:, None] * O.ft3d_dq(v32, t1, q32))
    assert nrel(host(Q1.grad).astype(np.float64), want) < TOL_FP32C


def test_config2_mesh_grad_q_full_size(gpu):
    """Config 2 (5120 faces x 262144 Q, the bench launch): FP32C dL/dQ against the FP64 form
    everywhere and both against the oracle on a sample including Q = 0."""
    cfg = mg.config2()
    v, t, q = cfg["verts"], cfg["tris"], cfg["q"]
    rng = np.random.default_rng(57)
    g = (rng.normal(size=len(q)) + 1j * rng.normal(size=len(q))).astype(np.complex64).astype(np.complex128)
    step("grad_Q config 2 fp64")
    _, _, g64 = bwd(v, t, [0, len(t)], np.array([1.0]), q, g, "fp64", need_verts=False, need_rho=False)
    step("grad_Q config 2 fp32c")
    _, _, g32 = bwd(v, t, [0, len(t)], np.array([1.0]), q, g, "fp32c", need_verts=False, need_rho=False)
    assert nrel(g32, g64) < TOL_FP32C
    idx = np.concatenate([rng.choice(len(q), 40, replace=False), [int(np.argmin(np.linalg.norm(q, axis=1)))]])
    want = np.real(np.conj(g[idx])[:, None] * O.ft3d_dq(v, t, q[idx]))
    assert nrel(g64[idx], want) < TOL_GRAD64
    assert nrel(g32[idx], want) < TOL_FP32C


def test_many_regions(gpu):
    """500 regions (small tetrahedra with random densities and positions): one face split per region
    at least, the per-region finish and the dL/drho reduction over many regions."""
    rng = np.random.default_rng(58)
    surfaces, regions = [], []
    for i in range(500):
        v, t = mg.tetrahedron(rng.normal(size=(4, 3)) * 0.4 + rng.uniform(-3, 3, size=3))
        t = mg.orient_outward(v, t)
        surfaces.append((v, t))
        regions.append([(i, +1)])
    v, t, off = mg.stack_regions(surfaces, regions)
    rho = rng.uniform(-1.0, 2.0, size=500)
    q = mg.q_random_ball(9000, 3.0, rng)
    g = rng.normal(size=len(q)) + 1j * rng.normal(size=len(q))
    want, want_j = O.ft3d_regions(v, t, off, rho, q)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"500 regions forward {mode}")
        F, Fj, _ = fwd(v, t, off, rho, q, mode)
        assert nrel(F, want) < tol, mode
        assert nrel(Fj, want_j) < tol, mode
        step(f"500 regions dL/drho {mode}")
        gg = g if mode == "fp64" else g.astype(np.complex64).astype(np.complex128)
        _, gr, _ = bwd(v, t, off, rho, q, gg, mode, need_verts=False, need_q=False)
        wr = np.array([np.sum(np.real(np.conj(gg) * want_j[j])) for j in range(500)])
        assert nrel(gr, wr) < (1e-10 if mode == "fp64" else TOL_FP32C), mode


def test_f32_inputs(gpu):
    """float32 vertices and Q through the region forward and backward: gradients come back as float32 and
    agree with the oracle at the rounded inputs."""
    v, t, off = mg.layered_sphere(1, [0.7, 1.0, 1.3], centre=(0.1, 0.2, -0.3))
    rho = np.array([1.5, -0.7, 2.2])
    rng = np.random.default_rng(59)
    q = mg.q_random_ball(900, 5.0, rng)
    g = (rng.normal(size=len(q)) + 1j * rng.normal(size=len(q))).astype(np.complex64)
    v32, q32 = v.astype(np.float32), q.astype(np.float32)
    V, T, Q, R = dev(v32), dev(t, torch.int32), dev(q32), dev(rho)
    step("regions f32 inputs")
    F = host(pft.forward_3d_regions(V, T, off, R, Q, mode="fp32c"))
    gv, gr, gq = pft.backward_3d_regions(V, T, off, R, Q, dev(g), mode="fp32c")
    torch.cuda.synchronize()
    assert gv.dtype == torch.float32 and gq.dtype == torch.float32 and gr.dtype == torch.float64
    vd, qd = v32.astype(np.float64), q32.astype(np.float64)
    want, _ = O.ft3d_regions(vd, t, off, rho, qd)
    wv, wr, wq = O.grad3d_regions(vd, t, off, rho, qd, g.astype(np.complex128))
    assert nrel(F, want) < TOL_FP32C
    assert nrel(host(gv).astype(np.float64), wv) < TOL_FP32C
    assert nrel(host(gr), wr) < TOL_FP32C
    assert nrel(host(gq).astype(np.float64), wq) < TOL_FP32C
