"""GPU parity of pft_backward_3d (vertex adjoint) and the autograd wrapper against the FP64 oracle."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle as O
import paper_2104_08309_amd as pft
from gpu_util import TOL_FP32C, dev, host, nrel, step

pytestmark = pytest.mark.gpu

TOL_GRAD64 = 1e-10


def run_bwd(v, t, q, g, mode, vdt=torch.float64):
    cdt = torch.complex128 if mode == "fp64" else torch.complex64
    r = pft.backward_3d(dev(v, vdt), dev(t, torch.int32), dev(q), dev(g).to(cdt), mode=mode)
    torch.cuda.synchronize()
    return host(r).astype(np.float64)


def test_small_meshes_random_cotangent(gpu):
    rng = np.random.default_rng(0)
    meshes = [mg.box(1.0, 1.3, 0.7, origin=(0.2, 0.1, -0.3)),
              mg.ellipsoid_uv([3.0, 2.0, 1.5], 9, centre=(0.5, -1.0, 2.0)),
              mg.icosphere(2, 2.0)]
    for i, (v, t) in enumerate(meshes):
        q = np.concatenate([mg.q_random_ball(700, 3.5, rng), [[0, 0, 0], [0, 0, 1.0], [1e-5, 0, 0]]])
        g = rng.normal(size=q.shape[0]) + 1j * rng.normal(size=q.shape[0])
        want = O.grad3d(v, t, q, g)
        step(f"bwd mesh {i} fp64")
        assert nrel(run_bwd(v, t, q, g, "fp64"), want) < TOL_GRAD64
        step(f"bwd mesh {i} fp32c")
        e = nrel(run_bwd(v, t, q, g.astype(np.complex64), "fp32c"), O.grad3d(v, t, q, g.astype(np.complex64)))
        print(f"mesh {i} fp32c grad rel err {e:.3e}")
        assert e < TOL_FP32C


def test_f32_vertices(gpu):
    v, t = mg.icosphere(2, 2.0)
    v32 = v.astype(np.float32)
    rng = np.random.default_rng(1)
    q = mg.q_random_ball(500, 3.0, rng)
    g = (rng.normal(size=500) + 1j * rng.normal(size=500)).astype(np.complex64)
    want = O.grad3d(v32.astype(np.float64), t, q, g)
    step("bwd f32 vertices fp32c")
    got = run_bwd(v32, t, q, g, "fp32c", vdt=torch.float32)
    assert nrel(got, want) < TOL_FP32C


def test_autograd_intensity_loss(gpu):
    """L = sum w (|F|^2 - I)^2 through PftFunction: gradient matches the oracle's chain rule. FP32C:
    within 1.5 e_c + 1e-5, e_c the error that the FP32C forward's F alone brings through the loss
    (the exact adjoint of the cotangent formed from it; the loss amplifies the forward's error)."""
    v0, t = mg.icosphere(3, 5.0)
    rng = np.random.default_rng(2)
    v = mg.perturb_radial(v0, 0.02, rng)
    q = mg.q_slice_z(32, 0.8)
    target = np.abs(O.ft3d(v0, t, q)) ** 2
    w = 1.0 / (q.shape[0] * O.volume3d(v0, t) ** 4)
    F = O.ft3d(v, t, q)
    want = O.grad3d(v, t, q, 4 * w * (np.abs(F) ** 2 - target) * F)
    for mode in ("fp64", "fp32c"):
        step(f"autograd loss {mode}")
        vt = dev(v).requires_grad_(True)
        Fg = pft.ft3d(vt, dev(t, torch.int32), dev(q), mode)
        loss = pft.intensity_loss(Fg.to(torch.complex128), dev(target), w)
        loss.backward()
        got = host(vt.grad)
        e = nrel(got, want)
        if mode == "fp64":
            tol = 1e-9
        else:
            F32 = host(Fg.detach()).astype(np.complex128)
            e_c = nrel(O.grad3d(v, t, q, 4 * w * (np.abs(F32) ** 2 - target) * F32), want)
            tol = 1.5 * e_c + TOL_FP32C
        print(f"autograd {mode}: rel err {e:.3e} (bar {tol:.2e})")
        assert e < tol
        # translation invariance of |F|^2: the vertex gradients sum to zero
        assert np.max(np.abs(got.sum(axis=0))) < 1e-3 * np.max(np.abs(got))


def test_deterministic_repeat(gpu):
    v, t = mg.icosphere(3, 1.0)
    rng = np.random.default_rng(3)
    q = mg.q_random_ball(2000, 6.0, rng)
    g = rng.normal(size=2000) + 1j * rng.normal(size=2000)
    for mode in ("fp64", "fp32c"):
        step(f"bwd determinism {mode}")
        a, b = run_bwd(v, t, q, g, mode), run_bwd(v, t, q, g, mode)
        assert np.array_equal(a, b)


def test_q_order_at_sorted_sizes(gpu):
    """At >= 8192 Q the FP32C adjoint visits Q in Morton order: parity against the oracle, and a
    permuted Q list (with its cotangents) gives the same gradient up to binary32 summation order."""
    rng = np.random.default_rng(12)
    v, t = mg.icosphere(1, 1.5)
    v = v + np.array([-0.2, 0.5, 0.1])
    q = mg.q_random_ball(10000, 4.0, rng)
    g = (rng.normal(size=q.shape[0]) + 1j * rng.normal(size=q.shape[0])).astype(np.complex64)
    want = O.grad3d(v, t, q, g)
    step("bwd sorted-size fp32c")
    got = run_bwd(v, t, q, g, "fp32c")
    assert nrel(got, want) < TOL_FP32C
    perm = rng.permutation(q.shape[0])
    step("bwd sorted-size fp32c permuted")
    got_p = run_bwd(v, t, q[perm], g[perm], "fp32c")
    assert nrel(got_p, got) < 1e-6
    step("bwd sorted-size fp64")
    assert nrel(run_bwd(v, t, q, g.astype(np.complex128), "fp64"), want) < TOL_GRAD64


def test_config4_full_size_sampled_vertices(gpu):
    """Icosphere L6 with radial noise, 256^2 Q slice: full adjoint on the GPU, oracle on sampled vertices."""
    cfg = mg.config4()
    v, t, q = cfg["verts"], cfg["tris"], cfg["q"]
    rng = np.random.default_rng(4)
    g = (rng.normal(size=q.shape[0]) + 1j * rng.normal(size=q.shape[0])) / q.shape[0]
    ids = rng.choice(v.shape[0], 10, replace=False)
    want = O.grad3d_vertices(v, t, q, g.astype(np.complex64), ids)
    step("config4 bwd fp32c (81920 faces x 65536 Q)")
    got = run_bwd(v, t, q, g.astype(np.complex64), "fp32c")
    e = nrel(got[ids], want)
    print(f"config4 fp32c sampled grad rel err {e:.3e}")
    assert e < TOL_FP32C
    step("config4 bwd fp64")
    got64 = run_bwd(v, t, q, g, "fp64")
    want64 = O.grad3d_vertices(v, t, q, g, ids)
    assert nrel(got64[ids], want64) < TOL_GRAD64
    # sum of all vertex gradients = Re sum_Q conj(g) i Q F(Q): the translation identity at full size
    step("config4 fwd fp64 for the identity")
    F = host(pft.forward_3d(dev(v), dev(t, torch.int32), dev(q), mode="fp64"))
    lhs = got64.sum(axis=0)
    rhs = np.real(np.sum(np.conj(g)[:, None] * 1j * q * F[:, None], axis=0))
    assert np.max(np.abs(lhs - rhs)) < 1e-9 * np.max(np.abs(got64)) * np.sqrt(v.shape[0])


def test_fp32c_moment_polynomial_ranges(gpu):
    """The FP32C adjoint and grad_Q take a face's small-phase moments from a polynomial chosen per
    wavefront by the largest centred vertex phase m among its lanes. Below 8192 Q the list order is
    kept, so each block of 64 Q on one |Q| shell makes the wavefronts of one range: shells at
    |Q| rho = 0.4 ... 2.95 (rho the largest centroid-to-vertex distance) reach every range up to the
    series/edge switch at m = 3, and a mixed block (small and large |Q| alternating) makes the small
    lanes run the highest degree. Vertex gradient and dL/dQ against the oracle."""
    v, t = mg.icosphere(2, 2.0)
    c = v[t].mean(axis=1)
    rho_f = np.linalg.norm(v[t] - c[:, None, :], axis=2).max()
    rng = np.random.default_rng(81)
    blocks = []
    for m in (0.4, 0.65, 0.95, 1.3, 1.7, 2.1, 2.6, 2.95):
        d = rng.normal(size=(128, 3))
        blocks.append(d / np.linalg.norm(d, axis=1, keepdims=True) * (m / rho_f))
    d = rng.normal(size=(128, 3))
    mags = np.where(np.arange(128) % 2 == 0, 0.3, 2.9) / rho_f
    blocks.append(d / np.linalg.norm(d, axis=1, keepdims=True) * mags[:, None])
    q = np.concatenate(blocks)
    g = (rng.normal(size=q.shape[0]) + 1j * rng.normal(size=q.shape[0])).astype(np.complex64)
    step("moment ranges: vertex adjoint fp32c")
    e = nrel(run_bwd(v, t, q, g, "fp32c"), O.grad3d(v, t, q, g))
    print(f"moment ranges: vertex gradient rel err {e:.3e}")
    assert e < TOL_FP32C
    step("moment ranges: dL/dQ fp32c")
    off = np.array([0, t.shape[0]])
    rho = np.array([1.0])
    _, _, gq = pft.backward_3d_regions(dev(v, torch.float64), dev(t, torch.int32), off, dev(rho, torch.float64),
                                       dev(q, torch.float64), dev(g), mode="fp32c", need_verts=False, need_rho=False)
    torch.cuda.synchronize()
    want = O.grad3d_regions(v, t, off, rho, q, g)[2]
    e = nrel(host(gq).astype(np.float64), want)
    print(f"moment ranges: dL/dQ rel err {e:.3e}")
    assert e < TOL_FP32C
