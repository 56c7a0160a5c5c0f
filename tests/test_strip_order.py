"""The host edge-sharing face order (pft_strip_order): a permutation; per position a cyclic rotation of the
face's vertex list, optionally traversed in reverse (b, a, c); and links that name an edge the two
consecutive faces really share: edge 0 of the face is edge 1 of its predecessor."""
import numpy as np
import pytest

import meshgen as mg
from paper_2104_08309_amd import _lib, api

LINK, REFLECT = 4, 8


def traversal(tris, order, meta, i):
    f = tris[order[i]]
    r = int(meta[i]) & 3
    assert r < 3
    a = [int(f[r]), int(f[(r + 1) % 3]), int(f[(r + 2) % 3])]
    return [a[1], a[0], a[2]] if int(meta[i]) & REFLECT else a


def check_order(tris, order, meta, nv):
    nf = len(tris)
    assert sorted(order.tolist()) == list(range(nf))
    assert np.all((meta & ~np.uint8(3 | LINK | REFLECT)) == 0)
    for i in range(nf):
        a = traversal(tris, order, meta, i)
        f = [int(x) for x in tris[order[i]]]
        rev = f[::-1]
        if int(meta[i]) & REFLECT:  # the reversed orientation
            assert any(a == rev[k:] + rev[:k] for k in range(3))
        else:  # a cyclic rotation of the listed vertices: same orientation
            assert any(a == f[k:] + f[:k] for k in range(3))
        if int(meta[i]) & LINK:
            assert i > 0
            b = traversal(tris, order, meta, i - 1)
            assert {a[0], a[1]} == {b[1], b[2]}
            assert all(0 <= x < nv for x in a + b) and len(set(a)) == 3 and len(set(b)) == 3
    return float(np.mean((meta & LINK) > 0))


@pytest.mark.parametrize("level", [0, 2, 4])
def test_icosphere_chains(level):
    v, t = mg.icosphere(level, 1.0)
    order, meta = api.strip_order(t)
    frac = check_order(t, order, meta, len(v))
    assert frac > (0.9 if level >= 2 else 0.6)


def test_union_mesh_and_bad_faces():
    """A marching-tetrahedra union mesh, plus faces with out-of-range and repeated indices (placed
    unlinked) and a duplicated face listed backwards (three faces on an edge)."""
    v, t = mg.union_of_spheres(np.array([[0.0, 0, 0], [1.2, 0.3, 0]]), np.array([1.0, 0.8]), h=0.25)
    t2 = np.concatenate([t, [[0, 1, 10 ** 6], [3, 3, 4], t[7][::-1]]]).astype(np.int32)
    order, meta = api.strip_order(t2, nv=len(v))
    frac = check_order(t2, order, meta, len(v))
    assert frac > 0.8
    pos = {int(o): i for i, o in enumerate(order)}
    for bad in (len(t), len(t) + 1):
        assert meta[pos[bad]] & LINK == 0


def test_validation():
    lib = _lib.load()
    assert lib.pft_strip_order(None, 4, 10, None, None) == _lib.PFT_EINVAL
    assert lib.pft_strip_order(None, -1, 10, None, None) == _lib.PFT_EINVAL
    assert lib.pft_strip_order(None, 0, 10, None, None) == _lib.PFT_OK


def test_batch_order_stays_within_each_mesh():
    """batch_strip_order: each mesh's range holds a permutation of its own triangles, offset by its first
    triangle, with valid links inside the range and none across a range boundary."""
    meshes = [mg.icosphere(2, 1.0), mg.box(), mg.icosphere(1, 2.0)]
    tris = np.concatenate([t for _, t in meshes]).astype(np.int32)
    to = np.cumsum([0] + [len(t) for _, t in meshes])
    vo = np.cumsum([0] + [len(v) for v, _ in meshes])
    order, meta = api.batch_strip_order(tris, vo, to)
    for i, (v, t) in enumerate(meshes):
        a, b = int(to[i]), int(to[i + 1])
        local_order = order[a:b] - a
        assert meta[a] & LINK == 0
        check_order(t, local_order, meta[a:b], len(v))
