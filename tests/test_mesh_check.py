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
