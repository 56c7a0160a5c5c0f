"""GPU parity of pft_forward_3d_poly (planar polygon faces) against the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

import meshgen as mg
import oracle as O
import paper_2104_08309_amd as pft
from gpu_util import TOL_FP32C, TOL_FP64, dev, host, maxrel, nrel, special_q, step

pytestmark = pytest.mark.gpu


def run(v, faces, q, mode, vdt=torch.float64, qdt=torch.float64):
    r = pft.forward_3d_poly(dev(v, vdt), faces, dev(q, qdt), mode=mode)
    torch.cuda.synchronize()
    return host(r)


def test_box_quads_and_degenerate_q(gpu):
    """Six quads; Q on the axes (along face normals: the fan series) and Q = 0, tiny Q."""
    v, f = mg.box_quads(1.0, 1.3, 0.7, origin=(0.3, -0.2, 0.1))
    rng = np.random.default_rng(41)
    q = np.concatenate([rng.normal(size=(500, 3)) * 4.0, special_q(3.0), [[1e-6, 0, 0], [0, 0, 2.0]]])
    want = O.ft3d_poly(v, f, q)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"poly box {mode}")
        got = run(v, f, q, mode)
        assert nrel(got, want) < tol and maxrel(got, want) < tol, mode


def test_prism_over_large_polygon(gpu):
    """A prism over a 40-gon (40-vertex caps and quads): long vertex loops, several tiles."""
    poly = mg.star_polygon(seed=6, n=40, rmin=0.7, rmax=1.1)
    v, f = mg.prism_polygon(poly, 1.4, -0.3)
    rng = np.random.default_rng(42)
    q = np.concatenate([mg.q_random_ball(900, 6.0, rng), special_q(4.0)])
    want = O.ft3d_poly(v, f, q)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"poly 40-gon prism {mode}")
        assert nrel(run(v, f, q, mode), want) < tol, mode


def test_mixed_faces_sorted_size(gpu):
    """Quads and triangles (planar lat-long ellipsoid), 12000 Q (Morton-ordered path), f32 inputs too."""
    rng = np.random.default_rng(43)
    v, f = mg.ellipsoid_quads([3.0, 2.0, 1.5], 10, 16, rot=np.linalg.qr(rng.normal(size=(3, 3)))[0],
                              centre=(0.4, -0.8, 0.2))
    q = mg.q_random_ball(12000, 3.0, rng)
    want = O.ft3d_poly(v, f, q)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"poly ellipsoid {mode}")
        assert nrel(run(v, f, q, mode), want) < tol, mode
    v32, q32 = v.astype(np.float32), q.astype(np.float32)
    want32 = O.ft3d_poly(v32.astype(np.float64), f, q32.astype(np.float64))
    step("poly ellipsoid fp32c, f32 inputs")
    assert nrel(run(v32, f, q32, "fp32c", torch.float32, torch.float32), want32) < TOL_FP32C


def test_matches_triangle_path(gpu):
    """The polygon kernels and the triangle kernels on the fan triangulation agree."""
    rng = np.random.default_rng(44)
    v, f = mg.ellipsoid_quads([2.0, 2.5, 1.0], 8, 12)
    tri = np.array([[x[0], x[l], x[l + 1]] for x in f for l in range(1, len(x) - 1)], dtype=np.int32)
    q = mg.q_random_ball(2000, 4.0, rng)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"poly vs triangles {mode}")
        a = run(v, f, q, mode)
        b = host(pft.forward_3d(dev(v, torch.float64), dev(tri, torch.int32), dev(q, torch.float64), mode=mode))
        assert nrel(a, b) < tol, mode


def test_empty_and_degenerate_faces(gpu):
    """A zero-area face and an out-of-range index contribute 0; an empty Q list is a no-op."""
    v, f = mg.box_quads(1.0, 1.0, 1.0)
    v = np.concatenate([v, [[5.0, 5.0, 5.0]]])
    f = f + [[8, 8, 8], [0, 1, 99]]
    q = np.array([[0.3, -0.2, 0.5], [1.0, 2.0, -0.5]])
    want = O.ft3d_poly(v[:8], f[:6], q)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"poly degenerate faces {mode}")
        assert nrel(run(v, f, q, mode), want) < tol, mode
    step("poly empty Q")
    assert run(v, f, np.zeros((0, 3)), "fp32c").shape == (0,)
