"""GPU parity of pft_forward_3d (both arithmetic forms) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle as O
import paper_2104_08309_amd as pft
from paper_2104_08309_amd import _lib
from gpu_util import TOL_FP32C, TOL_FP64, dev, host, maxrel, nrel, special_q, step

pytestmark = pytest.mark.gpu


def run(v, t, q, mode, vdt=torch.float64, qdt=torch.float64, intensity=False):
    r = pft.forward_3d(dev(v, vdt), dev(t, torch.int32), dev(q, qdt), mode=mode, intensity=intensity)
    torch.cuda.synchronize()
    if intensity:
        return host(r[0]), host(r[1])
    return host(r)


def test_box_all_forms_and_degenerate_q(gpu):
    v, t = mg.box(1.0, 1.3, 0.7, origin=(0.3, -0.2, 0.1))
    rng = np.random.default_rng(0)
    q = np.concatenate([rng.normal(size=(600, 3)) * 4.0, special_q(3.0), [[1e-6, 0, 0], [0, 0, 2.0]]])
    want = O.ft3d(v, t, q)
    step("box fp64")
    assert nrel(run(v, t, q, "fp64"), want) < TOL_FP64
    step("box fp32c")
    got = run(v, t, q, "fp32c")
    assert nrel(got, want) < TOL_FP32C and maxrel(got, want) < TOL_FP32C


def test_ragged_tiles_ellipsoid(gpu):
    """288 faces (4.5 LDS tiles) and 1000 Q (3.9 blocks): ragged tails on both axes."""
    rng = np.random.default_rng(1)
    v, t = mg.ellipsoid_uv([3.0, 2.0, 1.5], 9, rot=np.linalg.qr(rng.normal(size=(3, 3)))[0], centre=(1.0, 2.0, -1.0))
    assert t.shape[0] == 288
    q = np.concatenate([mg.q_random_ball(990, 3.0, rng), special_q(2.0, 3)])
    want = O.ft3d(v, t, q)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"ellipsoid {mode}")
        got = run(v, t, q, mode)
        assert nrel(got, want) < tol, mode


def test_input_dtypes(gpu):
    v, t = mg.icosphere(2, 2.0)
    rng = np.random.default_rng(2)
    q = mg.q_random_ball(700, 4.0, rng)
    v32, q32 = v.astype(np.float32), q.astype(np.float32)
    want32 = O.ft3d(v32.astype(np.float64), t, q32.astype(np.float64))
    step("dtypes fp64 mode, f32 inputs")
    assert nrel(run(v32, t, q32, "fp64", torch.float32, torch.float32), want32) < TOL_FP64
    step("dtypes fp32c mode, f32 inputs")
    assert nrel(run(v32, t, q32, "fp32c", torch.float32, torch.float32), want32) < TOL_FP32C
    step("dtypes fp32c mode, mixed")
    want = O.ft3d(v32.astype(np.float64), t, q)
    assert nrel(run(v32, t, q, "fp32c", torch.float32, torch.float64), want) < TOL_FP32C


def test_intensity_output(gpu):
    v, t = mg.icosphere(2, 2.0)
    q = mg.q_random_ball(500, 3.0, np.random.default_rng(3))
    for mode in ("fp64", "fp32c"):
        step(f"intensity {mode}")
        F, I = run(v, t, q, mode, intensity=True)
        assert np.allclose(I, np.abs(F.astype(np.complex128)) ** 2, rtol=1e-6 if mode == "fp32c" else 1e-14)


def test_empty_and_degenerate_meshes(gpu):
    q = mg.q_random_ball(300, 2.0, np.random.default_rng(4))
    q[0] = 0
    # no faces at all
    v0 = np.zeros((3, 3))
    for mode in ("fp64", "fp32c"):
        step(f"empty mesh {mode}")
        got = pft.forward_3d(dev(v0), torch.zeros((0, 3), dtype=torch.int32, device="cuda:0"), dev(q), mode=mode)
        assert torch.count_nonzero(got).item() == 0
    # zero-area faces and an out-of-range index contribute nothing
    v, t = mg.box(1.0, 1.0, 1.0)
    v2 = np.concatenate([v, [[0.5, 0.5, 0.5]]])
    t2 = np.concatenate([t, [[0, 1, 1], [8, 8, 8], [0, 8, 0], [0, 1, 99]]]).astype(np.int32)
    want = O.ft3d(v, t, q)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"degenerate faces {mode}")
        assert nrel(run(v2, t2, q, mode), want) < tol
    step("validate_mesh")
    bad, rep = pft.validate_mesh(dev(t2, torch.int32), v2.shape[0])
    assert bad == 1 and rep == 3


def test_strict_index_validation(gpu, monkeypatch):
    """With PFT_VALIDATE=1 an out-of-range triangle index is an argument error (checked on the
    device before any work) in the forward, the adjoint and the region entry points."""
    v, t = mg.box(1.0, 1.0, 1.0)
    t2 = np.concatenate([t, [[0, 1, 99]]]).astype(np.int32)
    q = mg.q_random_ball(50, 2.0, np.random.default_rng(5))
    V, T2, Q = dev(v), dev(t2, torch.int32), dev(q)
    g = torch.ones(len(q), dtype=torch.complex128, device="cuda:0")
    one = torch.ones(1, dtype=torch.float64, device="cuda:0")
    monkeypatch.setenv("PFT_VALIDATE", "1")
    step("PFT_VALIDATE=1 rejects a bad index")
    for call in (lambda: pft.forward_3d(V, T2, Q, mode="fp64"),
                 lambda: pft.backward_3d(V, T2, Q, g, mode="fp64"),
                 lambda: pft.forward_3d_regions(V, T2, [0, len(t2)], one, Q, mode="fp64"),
                 lambda: pft.backward_3d_regions(V, T2, [0, len(t2)], one, Q, g, mode="fp64")):
        with pytest.raises(_lib.PftError, match="out of range"):
            call()
    step("PFT_VALIDATE=1 accepts a valid mesh")
    assert nrel(host(pft.forward_3d(V, dev(t, torch.int32), Q, mode="fp64")), O.ft3d(v, t, q)) < TOL_FP64
    monkeypatch.delenv("PFT_VALIDATE")
    step("without PFT_VALIDATE the bad face is empty")
    assert nrel(host(pft.forward_3d(V, T2, Q, mode="fp64")), O.ft3d(v, t, q)) < TOL_FP64


def test_edge_sharing_order(gpu):
    """forward_3d in an edge-sharing face order (automatic and explicit) against the oracle and the list
    order; the cached order follows in-place changes of the triangle tensor; an out-of-range order
    entry drops that position's face without faulting."""
    rng = np.random.default_rng(71)
    v, t = mg.ellipsoid_uv([3.0, 2.0, 1.5], 12, rot=np.linalg.qr(rng.normal(size=(3, 3)))[0], centre=(0.4, -0.2, 0.3))
    q = np.concatenate([mg.q_random_ball(9000, 4.0, rng), special_q(3.0)])
    want = O.ft3d(v, t, q)
    V, Q = dev(v, torch.float32), dev(q, torch.float32)
    T = dev(t, torch.int32)
    step("edge-sharing order: automatic")
    Fa = host(pft.forward_3d(V, T, Q, mode="fp32c"))
    Fn = host(pft.forward_3d(V, T, Q, mode="fp32c", order=None))
    want32 = O.ft3d(v.astype(np.float32).astype(np.float64), t, q.astype(np.float32).astype(np.float64))
    assert nrel(Fa, want32) < TOL_FP32C and nrel(Fn, want32) < TOL_FP32C
    assert nrel(Fa, Fn) < 2e-6
    step("edge-sharing order: in-place change of the triangles")
    perm = rng.permutation(len(t))
    T.copy_(dev(t[perm][:, [1, 2, 0]], torch.int32))
    assert nrel(host(pft.forward_3d(V, T, Q, mode="fp32c")), want32) < TOL_FP32C
    step("edge-sharing order: explicit, with one position out of range")
    order, meta = pft.strip_order(t)
    drop = int(order[len(order) // 2])
    order[len(order) // 2] = -1
    keep = np.array([i for i in range(len(t)) if i != drop])
    Fx = host(pft.forward_3d(V, dev(t, torch.int32), Q, mode="fp32c",
                             order=(dev(order), dev(meta))))
    # the surface is open without that face, where the small-|Q| branch (whose threshold differs
    # between the forms) no longer agrees with the surface sum: compare with the list-order kernel
    Fk = host(pft.forward_3d(V, dev(t[keep], torch.int32), Q, mode="fp32c", order=None))
    assert nrel(Fx, Fk) < 2e-6
    step("edge-sharing order: binary64 ignores it")
    F64 = host(pft.forward_3d(dev(v), dev(t, torch.int32), dev(q), mode="fp64", order=(dev(order * 0 + np.arange(len(t), dtype=np.int32)), dev(meta))))
    assert nrel(F64, want) < TOL_FP64


def test_q_order_reuse(gpu):
    """Q visiting orders computed once (q_order) and passed in: the forward gives bitwise the values of
    an in-call sort for any permutation (each Q is evaluated on its own), the adjoint bitwise the same
    for the same order and within rounding for another; the cache follows in-place changes of Q."""
    rng = np.random.default_rng(72)
    v, t = mg.icosphere(3, 1.5)
    V, T = dev(v, torch.float32), dev(t, torch.int32)
    Q = dev(mg.q_random_ball(20000, 5.0, rng), torch.float32)
    g = dev(rng.normal(size=20000) + 1j * rng.normal(size=20000), torch.complex64)
    step("q order: forward with the cached order, an in-call sort and a reversed order")
    Fa = host(pft.forward_3d(V, T, Q, mode="fp32c"))
    Fn = host(pft.forward_3d(V, T, Q, mode="fp32c", q_order=None))
    rev = torch.arange(Q.shape[0] - 1, -1, -1, dtype=torch.int64, device=Q.device).to(torch.uint32)
    Fr = host(pft.forward_3d(V, T, Q, mode="fp32c", q_order=rev))
    assert np.array_equal(Fa.view(np.uint8), Fn.view(np.uint8))
    assert np.array_equal(Fr.view(np.uint8), Fn.view(np.uint8))
    step("q order: adjoint")
    Ga = host(pft.backward_3d(V, T, Q, g, mode="fp32c"))
    Gn = host(pft.backward_3d(V, T, Q, g, mode="fp32c", q_order=None))
    Gr = host(pft.backward_3d(V, T, Q, g, mode="fp32c", q_order=rev))
    assert np.array_equal(Ga.view(np.uint8), Gn.view(np.uint8))
    assert nrel(Gr, Gn) < 1e-6
    step("q order: in-place change of Q")
    Q.mul_(0.5)
    F2 = host(pft.forward_3d(V, T, Q, mode="fp32c"))
    F2n = host(pft.forward_3d(V, T, Q, mode="fp32c", q_order=None))
    assert np.array_equal(F2.view(np.uint8), F2n.view(np.uint8))


def test_empty_q_list(gpu):
    v, t = mg.box()
    step("nq = 0")
    out = pft.forward_3d(dev(v), dev(t, torch.int32), torch.zeros((0, 3), dtype=torch.float64, device="cuda:0"))
    assert out.shape == (0,)


def test_deterministic_repeat(gpu):
    v, t = mg.icosphere(3, 1.0)
    q = mg.q_random_ball(3000, 8.0, np.random.default_rng(5))
    for mode in ("fp64", "fp32c"):
        step(f"determinism {mode}")
        a, b = run(v, t, q, mode), run(v, t, q, mode)
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_q_order_invariance_at_sorted_sizes(gpu):
    """At >= 8192 Q the kernels visit Q in Morton order and write F back to the caller's index: parity
    against the oracle, and a permuted Q list gives the same values permuted (bitwise: each Q is
    evaluated independently of the others)."""
    rng = np.random.default_rng(11)
    v, t = mg.icosphere(2, 2.0)
    v = v + np.array([0.4, -0.3, 0.2])
    q = np.concatenate([mg.q_random_ball(12000, 4.0, rng), special_q(3.0)])
    want = O.ft3d(v, t, q)
    perm = rng.permutation(q.shape[0])
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"sorted-size parity {mode} ({q.shape[0]} Q)")
        got = run(v, t, q, mode)
        assert nrel(got, want) < tol, mode
        step(f"sorted-size permuted {mode}")
        got_p = run(v, t, q[perm], mode)
        assert np.array_equal(got_p, got[perm]), mode


def test_config2_full_size_sampled(gpu):
    """Icosphere L4 (5120 faces), full 64^3 grid on the GPU; oracle on a seeded sample incl. 0, axes, diagonal."""
    cfg = mg.config2()
    v, t, q = cfg["verts"], cfg["tris"], cfg["q"]
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(q.shape[0], 1200, replace=False),
                          np.nonzero(np.sum(q != 0, axis=1) <= 1)[0][::8],                  # 0 and the axes
                          np.nonzero((q[:, 0] == q[:, 1]) & (q[:, 1] == q[:, 2]))[0]])      # the diagonal
    want = O.ft3d(v, t, q[idx])
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"config2 {mode} (262144 Q)")
        got = run(v, t, q, mode)
        assert np.all(np.isfinite(got))
        e = nrel(got[idx], want)
        print(f"config2 {mode}: rel err {e:.3e}, max rel {maxrel(got[idx], want):.3e}")
        assert e < tol


def test_large_q_instance_both_orders(gpu):
    """From 2^20 Q on, the FP32C forward holds 3 Q per thread instead of 2 (another kernel instance and
    other face splits): both face orders against the oracle on a sample, and the same Q evaluated in a
    list just below the threshold (the 2-Q instance) agree to rounding."""
    v, t = mg.icosphere(3, 2.0)
    v = v + np.array([0.2, -0.1, 0.3])
    rng = np.random.default_rng(21)
    nq = (1 << 20) + 1000
    q = np.concatenate([special_q(3.0), mg.q_random_ball(nq - special_q(3.0).shape[0], 6.0, rng)])
    idx = np.concatenate([np.arange(special_q(3.0).shape[0]), rng.choice(nq, 200, replace=False)])
    want = O.ft3d(v, t, q[idx].astype(np.float32).astype(np.float64))
    V, T, Q = dev(v), dev(t, torch.int32), dev(q, torch.float32)
    step(f"large-Q instance, edge-sharing order ({nq} Q)")
    Fe = host(pft.forward_3d(V, T, Q, mode="fp32c"))
    assert np.all(np.isfinite(Fe))
    assert nrel(Fe[idx], want) < TOL_FP32C
    step(f"large-Q instance, list order ({nq} Q)")
    Fl = host(pft.forward_3d(V, T, Q, mode="fp32c", order=None))
    assert nrel(Fl[idx], want) < TOL_FP32C
    assert nrel(Fl, Fe) < 2e-6
    m = (1 << 20) - 1000
    step(f"2-Q instance on the first {m} of the same Q")
    Fs = host(pft.forward_3d(V, T, dev(q[:m], torch.float32), mode="fp32c"))
    assert nrel(Fs, Fe[:m]) < 2e-6


def test_config3_full_size_sampled(gpu):
    """Union of 20 balls (~1e5 faces) on the full 128^3 grid (FP32C, c64 + |F|^2); oracle on a sample."""
    cfg = mg.config3()
    v, t, q = cfg["verts"], cfg["tris"], cfg["q"]
    assert abs(t.shape[0] - 100_000) <= 5000
    step("config3 fp32c (2097152 Q)")
    F, I = run(v, t, q, "fp32c", qdt=torch.float32, intensity=True)
    assert np.all(np.isfinite(F))
    rng = np.random.default_rng(3)
    idx = np.concatenate([[np.nonzero(np.all(q == 0, axis=1))[0][0]], rng.choice(q.shape[0], 100, replace=False)])
    want = O.ft3d(v, t, q[idx].astype(np.float32).astype(np.float64))
    e = nrel(F[idx], want)
    print(f"config3 fp32c: rel err {e:.3e}")
    assert e < TOL_FP32C
    assert np.allclose(I[idx], np.abs(F[idx].astype(np.complex128)) ** 2, rtol=1e-5)


def test_near_normal_face_series_both_precisions(gpu):
    """Q within 1 degree of a box face's normal takes the face's simplex series (relative test
    |Q_perp| < 0.02 |Q.n|). Its centred vertex phases grow like |Q_perp| times the face size: up to
    |Q| = 20 they stay within the binary32 polynomial's half radian, from |Q| = 80 some lanes take
    the binary64 series. Each magnitude group against the oracle."""
    v, t = mg.box(1.0, 1.3, 0.7, origin=(0.3, -0.2, 0.1))
    rng = np.random.default_rng(83)
    groups = []
    for s in (5.0, 20.0, 80.0, 120.0):
        qs = []
        for axis in range(3):
            d = rng.uniform(-0.012, 0.012, size=(64, 3))
            d[:, axis] = rng.choice([-1.0, 1.0], size=64)
            qs.append(d / np.linalg.norm(d, axis=1, keepdims=True) * s)
        groups.append(np.concatenate(qs))
    q = np.concatenate(groups)
    want = O.ft3d(v, t, q)
    step("near-normal series fp32c")
    got = run(v, t, q, "fp32c")
    for i, s in enumerate((5.0, 20.0, 80.0, 120.0)):
        sl = slice(i * 192, (i + 1) * 192)
        e = nrel(got[sl], want[sl])
        print(f"|Q| = {s}: rel err {e:.3e}")
        assert e < TOL_FP32C, s
