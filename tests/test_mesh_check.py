"""pft_check_mesh (host): what the 3D section requires of the boundary -- a closed surface of
consistently oriented triangles -- counted edge by edge, on closed meshes and on meshes broken in
each way the counts name."""
import numpy as np
import pytest

import meshgen as mg
import paper_2104_08309_amd as pft
from paper_2104_08309_amd import _lib

ZERO = {"bad_index": 0, "repeated_vertex": 0, "open_edges": 0, "nonmanifold_edges": 0, "misoriented_edges": 0}


@pytest.mark.parametrize("mesh", ["icosphere", "box", "union", "ellipsoid"])
def test_closed_meshes_pass(mesh):
    if mesh == "icosphere":
        v, t = mg.icosphere(3, 1.0)
    elif mesh == "box":
        v, t = mg.box(1.0, 2.0, 0.5)
    elif mesh == "union":
        v, t = mg.union_of_spheres(np.array([[0.0, 0, 0], [1.2, 0.3, 0]]), np.array([1.0, 0.8]), h=0.25)
    else:
        v, t = mg.ellipsoid_uv([3.0, 2.0, 1.5], 9)
    assert pft.check_mesh(t, len(v)) == ZERO
    # reversing every face keeps the surface closed and consistent (it only turns it inward)
    assert pft.check_mesh(t[:, ::-1], len(v)) == ZERO


def test_each_defect_is_counted():
    v, t = mg.icosphere(2, 1.0)
    nv = len(v)
    assert pft.check_mesh(t[1:], nv) == dict(ZERO, open_edges=3)
    flipped = t.copy()
    flipped[5] = flipped[5][::-1]
    assert pft.check_mesh(flipped, nv) == dict(ZERO, misoriented_edges=3)
    extra = np.concatenate([t, t[7:8, ::-1]])
    assert pft.check_mesh(extra, nv) == dict(ZERO, nonmanifold_edges=3)
    bad = np.concatenate([t, [[0, 1, nv + 4], [-1, 2, 3]]])
    assert pft.check_mesh(bad, nv)["bad_index"] == 2
    rep = np.concatenate([t, [[3, 3, 4]]])
    r = pft.check_mesh(rep, nv)
    assert r["repeated_vertex"] == 1 and r["open_edges"] == 0
    # two separate closed components are fine; one of them opened is not
    both = np.concatenate([t, t + nv])
    assert pft.check_mesh(both, 2 * nv) == ZERO
    assert pft.check_mesh(np.concatenate([t, (t + nv)[1:]]), 2 * nv)["open_edges"] == 3


def test_validation():
    lib = _lib.load()
    rep = _lib.PftMeshCheck()
    assert lib.pft_check_mesh(None, -1, 3, rep) == _lib.PFT_EINVAL
    assert lib.pft_check_mesh(None, 2, 3, rep) == _lib.PFT_EINVAL
    assert lib.pft_check_mesh(None, 0, 3, None) == _lib.PFT_EINVAL
    assert lib.pft_check_mesh(None, 0, 3, rep) == _lib.PFT_OK


def _rho_by_definition(v, t):
    """Largest distance from a triangle's centroid to one of its corners, face by face."""
    best = 0.0
    for f in t:
        p = v[f]
        g = p.mean(axis=0)
        best = max(best, max(np.linalg.norm(p[k] - g) for k in range(3)))
    return best


@pytest.mark.parametrize("mesh", ["icosphere", "box", "ellipsoid", "hull"])
def test_fp32c_q_limit(mesh):
    """pft_fp32c_q_limit (host) is PFT_FP32C_PHASE_MAX over the largest face extent."""
    rng = np.random.default_rng(4)
    if mesh == "icosphere":
        v, t = mg.icosphere(3, 50.0)
    elif mesh == "box":
        v, t = mg.box(40.0, 3.0, 7.0, origin=(1.0, 2.0, 3.0))
    elif mesh == "ellipsoid":
        v, t = mg.ellipsoid_uv([30.0, 20.0, 15.0], 9, centre=(5.0, 0.0, -5.0))
    else:
        v, t = mg.convex_hull_mesh(rng.normal(size=(32, 3)) * 40.0)
    assert pft.fp32c_q_limit(v, t) == pytest.approx(128.0 / _rho_by_definition(v, t), rel=1e-12)
    # float32 vertices: the limit of the rounded vertices
    import ctypes
    v32 = np.ascontiguousarray(v, dtype=np.float32)
    t32 = np.ascontiguousarray(t, dtype=np.int32)
    lim = ctypes.c_double()
    assert _lib.load().pft_fp32c_q_limit(v32.ctypes.data, _lib.PFT_F32, len(v32), t32.ctypes.data, len(t32),
                                         ctypes.byref(lim)) == 0
    assert lim.value == pytest.approx(128.0 / _rho_by_definition(v32.astype(np.float64), t), rel=1e-12)


def test_fp32c_q_limit_edge_cases():
    import ctypes
    lib = _lib.load()
    assert pft.fp32c_q_limit(np.zeros((0, 3)), np.zeros((0, 3), dtype=np.int32)) == float("inf")
    v, t = mg.box(2.0, 2.0, 2.0)
    # a face with an out-of-range index is empty in the transform and skipped here
    far = np.concatenate([v, [[1e6, 0.0, 0.0]]])
    assert pft.fp32c_q_limit(far, np.concatenate([t, [[0, 1, 99]]])) == pytest.approx(pft.fp32c_q_limit(v, t))
    # a face with extent always counts, even when degenerate (zero area)
    line = np.concatenate([v, [[10.0, 0.0, 0.0]]])
    assert pft.fp32c_q_limit(line, np.concatenate([t, [[0, 8, 0]]])) < pft.fp32c_q_limit(v, t)
    lim = ctypes.c_double()
    vv = np.ascontiguousarray(v)
    tt = np.ascontiguousarray(t, dtype=np.int32)
    assert lib.pft_fp32c_q_limit(vv.ctypes.data, _lib.PFT_F64, len(vv), tt.ctypes.data, len(tt), None) == _lib.PFT_EINVAL
    assert lib.pft_fp32c_q_limit(None, _lib.PFT_F64, len(vv), tt.ctypes.data, len(tt), ctypes.byref(lim)) == \
        _lib.PFT_EINVAL
    assert lib.pft_fp32c_q_limit(vv.ctypes.data, _lib.PFT_F64, -1, tt.ctypes.data, len(tt), ctypes.byref(lim)) == \
        _lib.PFT_EINVAL
    assert lib.pft_fp32c_q_limit(vv.ctypes.data, 7, len(vv), tt.ctypes.data, len(tt), ctypes.byref(lim)) == \
        _lib.PFT_EUNSUPPORTED
