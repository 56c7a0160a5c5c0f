"""GPU parity of pft_forward_2d and of the batched entry points against the FP64 oracle."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle as O
import paper_2104_08309_amd as pft
from gpu_util import TOL_FP32C, TOL_FP64, dev, host, nrel, step

pytestmark = pytest.mark.gpu


def test_config1_star_polygon_full(gpu):
    cfg = mg.config1()
    v, q = cfg["verts"], cfg["q"]
    want = O.ft2d(v, q)
    step("2D config1 (64 edges x 16384 Q)")
    got = host(pft.forward_2d(dev(v), dev(q)))
    e = nrel(got, want)
    print(f"config1 fp64 rel err {e:.3e}")
    assert e < TOL_FP64
    assert abs(got[np.nonzero(np.all(q == 0, axis=1))[0][0]] - O.area2d(v)) < 1e-14


def test_2d_rectangle_hole_and_small_q(gpu):
    outer = mg.rectangle_2d(2.0, 1.5)
    inner = mg.rectangle_2d(0.5, 0.4) + np.array([0.6, 0.3])
    verts = np.concatenate([outer, inner[::-1]])
    rng = np.random.default_rng(0)
    q = np.concatenate([rng.normal(size=(700, 2)) * 5, [[0, 0], [1e-6, 0], [0, 3.0], [2.0, 0]]])
    step("2D hole")
    got = host(pft.forward_2d(dev(verts), dev(q), contour_offsets=[0, 4, 8]))
    assert nrel(got, O.ft2d(verts, q, offsets=[0, 4, 8])) < TOL_FP64
    assert nrel(got, O.ft2d(outer, q) - O.ft2d(inner, q)) < TOL_FP64


def _concat(meshes):
    vo, to, qo = [0], [0], [0]
    for m in meshes:
        vo.append(vo[-1] + m["verts"].shape[0])
        to.append(to[-1] + m["tris"].shape[0])
        qo.append(qo[-1] + m["q"].shape[0])
    V = np.concatenate([m["verts"] for m in meshes])
    T = np.concatenate([m["tris"] for m in meshes]).astype(np.int32)
    Q = np.concatenate([m["q"] for m in meshes])
    return V, T, Q, vo, to, qo


def test_small_batch_forward_backward(gpu):
    meshes = mg.batch_config(seed=7, n_meshes=9, max_faces=3000, min_q=100, max_q=700)
    meshes.append({"verts": mg.box()[0], "tris": mg.box()[1], "q": np.zeros((0, 3))})       # mesh without Q
    meshes.append({"verts": mg.icosphere(1)[0], "tris": mg.icosphere(1)[1],
                   "q": np.concatenate([[[0, 0, 0]], mg.q_random_ball(300, 2.0, np.random.default_rng(1))])})
    V, T, Q, vo, to, qo = _concat(meshes)
    rng = np.random.default_rng(2)
    G = rng.normal(size=Q.shape[0]) + 1j * rng.normal(size=Q.shape[0])
    wantF = np.concatenate([O.ft3d(m["verts"], m["tris"], m["q"]) for m in meshes])
    wantG = np.concatenate([O.grad3d(m["verts"], m["tris"], m["q"], G[qo[i]:qo[i + 1]]) if m["q"].shape[0]
                            else np.zeros_like(m["verts"]) for i, m in enumerate(meshes)])
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"batch forward {mode}")
        F = host(pft.batch_forward(dev(V), dev(T, torch.int32), dev(Q), vo, to, qo, mode=mode))
        for i in range(len(meshes)):
            s = slice(qo[i], qo[i + 1])
            if qo[i + 1] > qo[i]:
                assert nrel(F[s], wantF[s]) < tol, (mode, i)
        step(f"batch backward {mode}")
        cdt = torch.complex128 if mode == "fp64" else torch.complex64
        Gv = host(pft.batch_backward(dev(V), dev(T, torch.int32), dev(Q), vo, to, qo, dev(G).to(cdt), mode=mode))
        gtol = 1e-10 if mode == "fp64" else TOL_FP32C
        for i in range(len(meshes)):
            s = slice(vo[i], vo[i + 1])
            if qo[i + 1] > qo[i]:
                assert nrel(Gv[s], wantG[s]) < gtol, (mode, i)
            else:
                assert np.all(Gv[s] == 0)


def test_batch_matches_single_mesh_calls(gpu):
    """The persistent batched kernels and the single-mesh kernels give the same results."""
    meshes = mg.batch_config(seed=8, n_meshes=6, max_faces=6000, min_q=1000, max_q=5000)
    V, T, Q, vo, to, qo = _concat(meshes)
    step("batch fp32c vs single")
    Fb = host(pft.batch_forward(dev(V), dev(T, torch.int32), dev(Q), vo, to, qo, mode="fp32c"))
    for i, m in enumerate(meshes):
        Fs = host(pft.forward_3d(dev(m["verts"]), dev(m["tris"], torch.int32), dev(m["q"]), mode="fp32c"))
        assert nrel(Fb[qo[i]:qo[i + 1]], Fs) < 1e-6


def test_batch_edge_sharing_order(gpu):
    """The batched forward with each mesh's faces in an edge-sharing order (automatic and explicit)
    agrees with the list order; an out-of-range order entry empties that position without faulting."""
    meshes = mg.batch_config(seed=9, n_meshes=7, max_faces=5000, min_q=800, max_q=3000)
    V, T, Q, vo, to, qo = _concat(meshes)
    Vd, Td, Qd = dev(V, torch.float32), dev(T, torch.int32), dev(Q, torch.float32)
    step("batch edge-sharing order: automatic against the list order")
    Fa = host(pft.batch_forward(Vd, Td, Qd, vo, to, qo, mode="fp32c"))
    Fn = host(pft.batch_forward(Vd, Td, Qd, vo, to, qo, mode="fp32c", order=None))
    for i in range(len(meshes)):
        assert nrel(Fa[qo[i]:qo[i + 1]], Fn[qo[i]:qo[i + 1]]) < 2e-6, i
    step("batch edge-sharing order: explicit, one entry out of range")
    order, meta = pft.batch_strip_order(T, vo, to)
    j = int(to[3]) + 5
    drop = int(order[j])
    order[j] = -1
    keep = np.array([k for k in range(int(to[3]), int(to[4])) if k != drop]) - int(to[3])
    Fx = host(pft.batch_forward(Vd, Td, Qd, vo, to, qo, mode="fp32c", order=(dev(order), dev(meta))))
    m = meshes[3]
    Fk = host(pft.forward_3d(dev(m["verts"], torch.float32), dev(m["tris"][keep], torch.int32),
                             dev(m["q"], torch.float32), mode="fp32c", order=None))
    assert nrel(Fx[qo[3]:qo[4]], Fk) < 2e-6
    for i in (0, 1, 2, 4, 5, 6):
        assert nrel(Fx[qo[i]:qo[i + 1]], Fn[qo[i]:qo[i + 1]]) < 2e-6, i


def test_config5_full_size_sampled(gpu):
    """512 uneven meshes in one persistent launch (FP32C fwd + bwd); oracle on sampled meshes / Q / vertices."""
    meshes = mg.config5()
    V, T, Q, vo, to, qo = _concat(meshes)
    rng = np.random.default_rng(5)
    G = ((rng.normal(size=Q.shape[0]) + 1j * rng.normal(size=Q.shape[0])) / 1e4).astype(np.complex64)
    step(f"config5 batch fwd fp32c ({len(meshes)} meshes, {T.shape[0]} faces, {Q.shape[0]} Q)")
    F = host(pft.batch_forward(dev(V), dev(T, torch.int32), dev(Q, torch.float32), vo, to, qo, mode="fp32c"))
    step("config5 batch bwd fp32c")
    Gv = host(pft.batch_backward(dev(V), dev(T, torch.int32), dev(Q, torch.float32), vo, to, qo, dev(G),
                                 mode="fp32c"))
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(Gv))
    for i in rng.choice(len(meshes), 6, replace=False):
        m = meshes[i]
        qi = rng.choice(m["q"].shape[0], 64, replace=False)
        q32 = m["q"].astype(np.float32).astype(np.float64)
        want = O.ft3d(m["verts"], m["tris"], q32[qi])
        assert nrel(F[qo[i]:qo[i + 1]][qi], want) < TOL_FP32C, i
        ids = rng.choice(m["verts"].shape[0], 3, replace=False)
        wg = O.grad3d_vertices(m["verts"], m["tris"], q32, G[qo[i]:qo[i + 1]], ids)
        assert nrel(Gv[vo[i]:vo[i + 1]][ids], wg) < TOL_FP32C, i


def test_batch_tile_tuning(gpu):
    """The batched launches tune their tile sizes at the first call of a size bucket: the choice is
    reported, the tuning call's output is the chosen configuration's (a second call repeats it bitwise),
    and the compiled defaults (PFT_AUTOTUNE=0) agree with it to rounding."""
    import os

    meshes = mg.batch_config(seed=11, n_meshes=24, max_faces=6000, min_q=500, max_q=3000)
    V, T, Q, vo, to, qo = _concat(meshes)
    rng = np.random.default_rng(5)
    G = dev((rng.normal(size=Q.shape[0]) + 1j * rng.normal(size=Q.shape[0])).astype(np.complex64))
    Vd, Td, Qd = dev(V), dev(T, torch.int32), dev(Q)
    step("batch tuning: first calls (tune) and repeats")
    F1 = host(pft.batch_forward(Vd, Td, Qd, vo, to, qo, mode="fp32c"))
    G1 = host(pft.batch_backward(Vd, Td, Qd, vo, to, qo, G, mode="fp32c"))
    F2 = host(pft.batch_forward(Vd, Td, Qd, vo, to, qo, mode="fp32c"))
    G2 = host(pft.batch_backward(Vd, Td, Qd, vo, to, qo, G, mode="fp32c"))
    info = pft.tuning_info()
    assert "batch_forward[" in info and "batch_backward[" in info, info
    assert np.array_equal(F1.view(np.uint8), F2.view(np.uint8))
    assert np.array_equal(G1.view(np.uint8), G2.view(np.uint8))
    step("batch tuning: compiled defaults")
    os.environ["PFT_AUTOTUNE"] = "0"
    try:
        F0 = host(pft.batch_forward(Vd, Td, Qd, vo, to, qo, mode="fp32c"))
        G0 = host(pft.batch_backward(Vd, Td, Qd, vo, to, qo, G, mode="fp32c"))
    finally:
        del os.environ["PFT_AUTOTUNE"]
    assert nrel(F0, F1) < 1e-6 and nrel(G0, G1) < 1e-6
    want = O.ft3d(meshes[0]["verts"], meshes[0]["tris"], meshes[0]["q"])
    assert nrel(F1[qo[0]:qo[1]], want) < TOL_FP32C
