"""The FP32C phase range: at |Q| rho <= PFT_FP32C_PHASE_MAX (rho the largest face centroid-to-vertex
distance) the binary32 form meets the FP32C bar against the oracle; beyond it every FP32C entry point
writes NaN at that Q (and the adjoints' gradients turn NaN), while the binary64 form stays finite."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle as O
import paper_2104_08309_amd as pft
from gpu_util import TOL_FP32C, TOL_FP64, dev, host, nrel, step

pytestmark = pytest.mark.gpu


def big_box():
    """A 40 x 36 x 44 box, rotated and off the origin: faces of extent about 30."""
    rng = np.random.default_rng(11)
    rot = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    v, t = mg.box(40.0, 36.0, 44.0, origin=(5.0, -3.0, 2.0))
    return v @ rot.T, t


def q_split(lim, n_in, n_out, seed):
    """n_in random Q with |Q| <= 0.97 lim and n_out with 1.05 lim <= |Q| <= 1.5 lim."""
    rng = np.random.default_rng(seed)
    q_in = mg.q_random_ball(n_in, 0.97 * lim, rng)
    d = rng.normal(size=(n_out, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q_out = d * rng.uniform(1.05 * lim, 1.5 * lim, size=(n_out, 1))
    return q_in, q_out


def test_q_limit_matches_face_extent(gpu):
    v, t = big_box()
    lim = pft.fp32c_q_limit(v, t)
    g = v[t].mean(axis=1)
    rho = np.sqrt(((v[t] - g[:, None, :]) ** 2).sum(axis=2)).max()
    assert lim == pytest.approx(128.0 / rho, rel=1e-12)


def test_forward_in_range_accurate_out_of_range_nan(gpu):
    v, t = big_box()
    lim = pft.fp32c_q_limit(v, t)
    q_in, q_out = q_split(lim, 900, 100, 1)
    q = np.concatenate([q_in, q_out])
    want = O.ft3d(v, t, q_in)
    step("phase range fp32c forward")
    F, I = pft.forward_3d(dev(v), dev(t, torch.int32), dev(q), mode="fp32c", intensity=True)
    F, I = host(F), host(I)
    n = q_in.shape[0]
    assert np.all(np.isfinite(F[:n])) and np.all(np.isfinite(I[:n]))
    assert nrel(F[:n], want) < TOL_FP32C
    assert np.all(np.isnan(F[n:].real)) and np.all(np.isnan(F[n:].imag)) and np.all(np.isnan(I[n:]))
    step("phase range fp64 forward")
    F64 = host(pft.forward_3d(dev(v), dev(t, torch.int32), dev(q), mode="fp64"))
    assert np.all(np.isfinite(F64))
    assert nrel(F64[:n], want) < TOL_FP64
    step("phase range fp32c forward without allocation")
    Fn = host(pft.forward_3d_noalloc(dev(v), dev(t, torch.int32), dev(q), mode="fp32c"))
    assert np.all(np.isfinite(Fn[:n])) and np.all(np.isnan(Fn[n:]))


def test_adjoint_and_loss(gpu):
    v, t = big_box()
    lim = pft.fp32c_q_limit(v, t)
    q_in, q_out = q_split(lim, 500, 1, 2)
    rng = np.random.default_rng(3)
    g = rng.normal(size=q_in.shape[0]) + 1j * rng.normal(size=q_in.shape[0])
    step("phase range fp32c adjoint, every Q in range")
    G = host(pft.backward_3d(dev(v), dev(t, torch.int32), dev(q_in), dev(g).to(torch.complex64), mode="fp32c"))
    assert nrel(G, O.grad3d(v, t, q_in, g)) < TOL_FP32C
    step("phase range fp32c adjoint, one Q beyond")
    q = np.concatenate([q_in, q_out])
    g1 = np.concatenate([g, [1.0 + 0.5j]])
    G = host(pft.backward_3d(dev(v), dev(t, torch.int32), dev(q), dev(g1).to(torch.complex64), mode="fp32c"))
    assert np.all(np.isnan(G))
    step("phase range fp64 adjoint, one Q beyond")
    G = host(pft.backward_3d(dev(v), dev(t, torch.int32), dev(q), dev(g1), mode="fp64"))
    assert np.all(np.isfinite(G))
    step("phase range fp32c intensity loss, one Q beyond")
    target = dev(np.ones(q.shape[0]))
    L, Gv = pft.intensity_loss_3d(dev(v), dev(t, torch.int32), dev(q), target, mode="fp32c")
    assert np.isnan(float(L)) and np.all(np.isnan(host(Gv)))
    L, Gv = pft.intensity_loss_3d(dev(v), dev(t, torch.int32), dev(q_in), target[: q_in.shape[0]], mode="fp32c")
    assert np.isfinite(float(L)) and np.all(np.isfinite(host(Gv)))


def test_poly_regions_and_batch(gpu):
    vq, quads = mg.box_quads(40.0, 40.0, 40.0, origin=(-20.0, -15.0, -25.0))
    rho_q = 20.0 * np.sqrt(2.0)
    lim_q = 128.0 / rho_q
    q_in, q_out = q_split(lim_q, 300, 20, 4)
    q = np.concatenate([q_in, q_out])
    n = q_in.shape[0]
    step("phase range fp32c polygon forward")
    F = host(pft.forward_3d_poly(dev(vq), quads, dev(q), mode="fp32c"))
    assert nrel(F[:n], O.ft3d_poly(vq, quads, q_in)) < TOL_FP32C
    assert np.all(np.isnan(F[n:]))

    v, t = big_box()
    lim = pft.fp32c_q_limit(v, t)
    q_in, q_out = q_split(lim, 300, 20, 5)
    q = np.concatenate([q_in, q_out])
    step("phase range fp32c regions forward")
    F = host(pft.forward_3d_regions(dev(v), dev(t, torch.int32), [0, t.shape[0]], dev(np.array([2.0])), dev(q),
                                    mode="fp32c"))
    assert nrel(F[:n], 2.0 * O.ft3d(v, t, q_in)) < TOL_FP32C
    assert np.all(np.isnan(F[n:]))

    # a batch of the big box and a small sphere: only the big box's Q beyond its own bound are NaN
    vs, ts = mg.icosphere(2, 1.0)
    qs = mg.q_random_ball(200, 1.5 * lim, np.random.default_rng(6))  # far inside the sphere's bound
    V = np.concatenate([v, vs])
    T = np.concatenate([t, ts]).astype(np.int32)
    Q = np.concatenate([q, qs])
    vo, to, qo = [0, v.shape[0], V.shape[0]], [0, t.shape[0], T.shape[0]], [0, q.shape[0], Q.shape[0]]
    step("phase range fp32c batch forward")
    F = host(pft.batch_forward(dev(V), dev(T, torch.int32), dev(Q), vo, to, qo, mode="fp32c"))
    assert nrel(F[:n], O.ft3d(v, t, q_in)) < TOL_FP32C
    assert np.all(np.isnan(F[n:q.shape[0]]))
    assert nrel(F[q.shape[0]:], O.ft3d(vs, ts, qs)) < TOL_FP32C
