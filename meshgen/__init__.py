"""Seeded synthetic inputs for the polygon / polyhedron Fourier transform.

This module builds geometry and reciprocal-space sample points only: meshes,
polygons and Q lists. It holds none of the transform's arithmetic and is
shared by the tests, the benchmark and the oracle's callers. Every generator is
deterministic given its seed (``numpy.random.default_rng``).

Conventions
-----------
* 3D meshes are ``(verts [V,3] float64, tris [F,3] int32)``, 0-based, closed,
  with each triangle counter-clockwise seen from outside (outward normal by the
  right-hand rule), the orientation the paper's 3D section asks for.
* 2D polygons are ``verts [V,2] float64`` traversed counter-clockwise.
* Q grids are FFT-style: ``q_k = -qmax + 2*qmax*k/n`` for ``k = 0..n-1`` so
  that Q = 0 and the coordinate axes are on the grid.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "fft_axis", "q_grid_2d", "q_grid_3d", "q_slice_z", "q_random_ball",
    "star_polygon", "rectangle_2d", "box", "tetrahedron", "icosahedron",
    "icosphere", "subdivide", "perturb_radial", "orient_outward",
    "ellipsoid_uv", "convex_hull_mesh", "union_of_spheres",
    "union_of_spheres_config", "batch_config", "read_netgen_surfacemesh",
    "box_quads", "prism_polygon", "ellipsoid_quads", "sphere_quadrature",
    "stack_regions", "layered_sphere", "nested_boxes",
    "config1", "config2", "config3", "config4", "config5",
]


# ----------------------------------------------------------------------------
# Q sample sets
# ----------------------------------------------------------------------------
def fft_axis(n: int, qmax: float) -> np.ndarray:
    """FFT-style axis of n points on [-qmax, qmax): contains 0 when n is even."""
    return -qmax + 2.0 * qmax * np.arange(n, dtype=np.float64) / n


def q_grid_2d(n: int, qmax: float) -> np.ndarray:
    """n*n grid of 2D Q vectors, row-major over (qx, qy). Shape [n*n, 2]."""
    ax = fft_axis(n, qmax)
    qx, qy = np.meshgrid(ax, ax, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel()], axis=1)


def q_grid_3d(n: int, qmax: float) -> np.ndarray:
    """n^3 grid of 3D Q vectors, row-major over (qx, qy, qz). Shape [n^3, 3]."""
    ax = fft_axis(n, qmax)
    qx, qy, qz = np.meshgrid(ax, ax, ax, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)


def q_slice_z(n: int, qmax: float, qz: float = 0.0) -> np.ndarray:
    """n*n grid in the (qx, qy) plane at fixed qz. Shape [n*n, 3]."""
    q2 = q_grid_2d(n, qmax)
    return np.concatenate([q2, np.full((q2.shape[0], 1), qz)], axis=1)


def q_random_ball(n: int, qmax: float, rng: np.random.Generator) -> np.ndarray:
    """n Q vectors with uniform direction and |Q| = qmax * U^(1/3) (uniform in the ball)."""
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = qmax * rng.random(n) ** (1.0 / 3.0)
    return d * r[:, None]


def sphere_quadrature(n_theta: int, n_phi: int):
    """Product quadrature on the unit sphere: Gauss-Legendre in cos(theta) x uniform in phi.

    Returns (dirs [n_theta * n_phi, 3], weights [n_theta * n_phi]) with the
    weights summing to 1, so sum_j w_j f(s_j) approximates the average of f
    over directions; exact for spherical harmonics of degree < 2 n_theta with
    |m| < n_phi.
    """
    x, wx = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * math.pi * (np.arange(n_phi) + 0.5) / n_phi
    st = np.sqrt(1.0 - x * x)
    dirs = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)), np.outer(x, np.ones(n_phi))], axis=-1)
    w = np.outer(0.5 * wx, np.full(n_phi, 1.0 / n_phi))
    return dirs.reshape(-1, 3), w.reshape(-1)


# ----------------------------------------------------------------------------
# 2D shapes
# ----------------------------------------------------------------------------
def star_polygon(seed: int = 1, n: int = 64, rmin: float = 0.5, rmax: float = 1.0) -> np.ndarray:
    """Random star-shaped polygon: angles ~ U[0, 2pi) sorted, radii ~ U[rmin, rmax]."""
    rng = np.random.default_rng(seed)
    th = np.sort(rng.random(n) * 2.0 * math.pi)
    r = rmin + (rmax - rmin) * rng.random(n)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def rectangle_2d(a: float, b: float) -> np.ndarray:
    """Rectangle [0,a] x [0,b], counter-clockwise from the origin corner."""
    return np.array([[0.0, 0.0], [a, 0.0], [a, b], [0.0, b]])


# ----------------------------------------------------------------------------
# 3D meshes
# ----------------------------------------------------------------------------
def _face_normals(verts: np.ndarray, tris: np.ndarray) -> np.ndarray:
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    return np.cross(b - a, c - a)


def orient_outward(verts: np.ndarray, tris: np.ndarray, centre=None) -> np.ndarray:
    """Flip triangles of a star-shaped (about ``centre``) mesh so normals point outward."""
    if centre is None:
        centre = verts.mean(axis=0)
    n = _face_normals(verts, tris)
    g = verts[tris].mean(axis=1) - centre
    flip = np.einsum("ij,ij->i", n, g) < 0
    out = tris.copy()
    out[flip, 1], out[flip, 2] = tris[flip, 2], tris[flip, 1]
    return out


def box(a: float = 1.0, b: float = 1.0, c: float = 1.0, origin=(0.0, 0.0, 0.0)):
    """Axis-aligned box [0,a]x[0,b]x[0,c] + origin as 12 outward triangles."""
    o = np.asarray(origin, dtype=np.float64)
    v = np.array([[x, y, z] for z in (0.0, c) for y in (0.0, b) for x in (0.0, a)]) + o
    # vertex index = ix + 2*iy + 4*iz
    quads = [
        (0, 2, 3, 1),  # z = 0, normal -z
        (4, 5, 7, 6),  # z = c, normal +z
        (0, 1, 5, 4),  # y = 0, normal -y
        (2, 6, 7, 3),  # y = b, normal +y
        (0, 4, 6, 2),  # x = 0, normal -x
        (1, 3, 7, 5),  # x = a, normal +x
    ]
    t = []
    for p0, p1, p2, p3 in quads:
        t.append((p0, p1, p2))
        t.append((p0, p2, p3))
    return v, np.array(t, dtype=np.int32)


def tetrahedron(pts=None):
    """A tetrahedron as 4 outward triangles (default: a generic, non-regular one)."""
    if pts is None:
        pts = np.array([[0.1, -0.2, 0.05], [1.3, 0.1, -0.1], [0.2, 0.9, 0.15], [0.4, 0.3, 1.1]])
    pts = np.asarray(pts, dtype=np.float64)
    tris = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], dtype=np.int32)
    return pts, orient_outward(pts, tris)


def icosahedron():
    """Regular icosahedron with vertices (0, +-1, +-phi) and cyclic permutations, circumradius 1."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int32)
    return v, orient_outward(v, f, centre=np.zeros(3))


def subdivide(verts: np.ndarray, tris: np.ndarray, project_radius=None):
    """1 -> 4 midpoint subdivision; optionally project new vertices onto a sphere.

    Orientation is preserved. Midpoints of shared edges are created once.
    """
    nv = verts.shape[0]
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=0)
    key = np.sort(e, axis=1)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    mid = 0.5 * (verts[uniq[:, 0]] + verts[uniq[:, 1]])
    if project_radius is not None:
        mid *= project_radius / np.linalg.norm(mid, axis=1, keepdims=True)
    nf = tris.shape[0]
    m01 = nv + inv[:nf]
    m12 = nv + inv[nf:2 * nf]
    m20 = nv + inv[2 * nf:]
    a, b, c = tris[:, 0], tris[:, 1], tris[:, 2]
    new = np.concatenate([
        np.stack([a, m01, m20], 1), np.stack([m01, b, m12], 1),
        np.stack([m20, m12, c], 1), np.stack([m01, m12, m20], 1),
    ], axis=0).astype(np.int32)
    return np.concatenate([verts, mid], axis=0), new


def icosphere(level: int, radius: float = 1.0):
    """Icosphere: icosahedron subdivided ``level`` times, vertices projected to radius.

    Level L has 20*4^L triangles and 10*4^L + 2 vertices.
    """
    v, f = icosahedron()
    for _ in range(level):
        v, f = subdivide(v, f, project_radius=1.0)
    return v * radius, f


def perturb_radial(verts: np.ndarray, sigma_rel: float, rng: np.random.Generator) -> np.ndarray:
    """Scale each vertex radially (about the origin) by (1 + sigma_rel * N(0,1))."""
    s = 1.0 + sigma_rel * rng.normal(size=verts.shape[0])
    return verts * s[:, None]


def _rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# ----------------------------------------------------------------------------
# 3D meshes with planar polygon faces (lists of CCW vertex indices)
# ----------------------------------------------------------------------------
def box_quads(a: float = 1.0, b: float = 1.0, c: float = 1.0, origin=(0.0, 0.0, 0.0)):
    """Axis-aligned box [0,a]x[0,b]x[0,c] + origin as 6 outward quads (face 0: z = 0, face 1: z = c)."""
    o = np.asarray(origin, dtype=np.float64)
    v = np.array([[x, y, z] for z in (0.0, c) for y in (0.0, b) for x in (0.0, a)]) + o
    faces = [[0, 2, 3, 1], [4, 5, 7, 6], [0, 1, 5, 4], [2, 6, 7, 3], [0, 4, 6, 2], [1, 3, 7, 5]]
    return v, faces


def stack_regions(surfaces, regions):
    """One vertex / triangle list for several closed regions.

    ``surfaces`` is a list of (verts, tris) closed outward surfaces; ``regions`` lists, per
    region, the surfaces that bound it as (surface index, +1 outward or -1 reversed). A surface
    shared by two regions keeps one copy of its vertices. Returns (verts, tris, region_offsets)
    with region j's triangles at region_offsets[j] .. region_offsets[j+1].
    """
    base, verts = [], []
    n = 0
    for v, _ in surfaces:
        base.append(n)
        verts.append(np.asarray(v, dtype=np.float64))
        n += len(v)
    tris, offsets = [], [0]
    for reg in regions:
        for si, sign in reg:
            t = np.asarray(surfaces[si][1], dtype=np.int64) + base[si]
            tris.append(t if sign > 0 else t[:, ::-1])
        offsets.append(offsets[-1] + sum(len(surfaces[si][1]) for si, _ in reg))
    tv = np.concatenate(verts) if verts else np.zeros((0, 3))
    tt = np.concatenate(tris).astype(np.int32) if tris else np.zeros((0, 3), dtype=np.int32)
    return tv, tt, np.array(offsets, dtype=np.int64)


def layered_sphere(level: int, radii, centre=(0.0, 0.0, 0.0)):
    """Concentric icospheres of increasing radii as regions: a core (inside radii[0]) and shells
    (between radii[j-1] and radii[j]), each bounded by its outer sphere and the reversed inner one."""
    surfaces = []
    for r in radii:
        v, t = icosphere(level, r)
        surfaces.append((v + np.asarray(centre, dtype=np.float64), t))
    regions = [[(0, +1)]] + [[(j, +1), (j - 1, -1)] for j in range(1, len(radii))]
    return stack_regions(surfaces, regions)


def nested_boxes(outer, inner):
    """A box inside a box as two regions (core = inner box, shell = outer minus inner).
    ``outer`` and ``inner`` are ((a, b, c), origin)."""
    surfaces = [box(*outer[0], origin=outer[1]), box(*inner[0], origin=inner[1])]
    return stack_regions(surfaces, [[(1, +1)], [(0, +1), (1, -1)]])


def prism_polygon(poly2d: np.ndarray, h: float, z0: float = 0.0):
    """Right prism over a counter-clockwise simple polygon (in the xy plane) from z0 to z0 + h:
    bottom and top nu-gons and nu side quads, all outward."""
    p = np.asarray(poly2d, dtype=np.float64)
    n = p.shape[0]
    v = np.concatenate([np.c_[p, np.full(n, z0)], np.c_[p, np.full(n, z0 + h)]])
    faces = [list(range(n - 1, -1, -1)), list(range(n, 2 * n))]
    for i in range(n):
        j = (i + 1) % n
        faces.append([i, j, n + j, n + i])
    return v, faces


def ellipsoid_quads(semi_axes, n_lat: int, n_lon: int, rot=None, centre=(0.0, 0.0, 0.0)):
    """Latitude-longitude ellipsoid with planar faces: quads between circles of latitude of the unit
    sphere (isosceles trapezoids, so planar), triangle fans at the poles, then scaled by the semi-axes
    (an affine map keeps faces planar), rotated and moved. Returns (verts, faces) of 4-gons and 3-gons,
    2 * n_lon triangles and (n_lat - 3) * n_lon quads."""
    th = np.linspace(0.0, math.pi, n_lat + 1)[1:-1]
    ph = 2.0 * math.pi * np.arange(n_lon) / n_lon
    ring = np.array([[math.sin(t) * math.cos(f), math.sin(t) * math.sin(f), math.cos(t)] for t in th for f in ph])
    v = np.concatenate([[[0.0, 0.0, 1.0]], ring, [[0.0, 0.0, -1.0]]])
    top, bot = 0, v.shape[0] - 1
    idx = lambda i, j: 1 + i * n_lon + (j % n_lon)
    faces = []
    for j in range(n_lon):
        faces.append([top, idx(0, j), idx(0, j + 1)])
    for i in range(n_lat - 3):
        for j in range(n_lon):
            faces.append([idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)])
    for j in range(n_lon):
        faces.append([bot, idx(n_lat - 3, j + 1), idx(n_lat - 3, j)])
    v = v * np.asarray(semi_axes, dtype=np.float64)
    if rot is not None:
        v = v @ np.asarray(rot).T
    return v + np.asarray(centre, dtype=np.float64), faces


def ellipsoid_uv(semi_axes, n_lat: int, rot=None, centre=(0.0, 0.0, 0.0)):
    """UV-tessellated ellipsoid: n_lat latitude bands, 2*n_lat longitudes, pole fans.

    Triangle count = 4*n_lat*(n_lat-1).
    """
    n_lon = 2 * n_lat
    th = np.arange(1, n_lat) * math.pi / n_lat          # interior latitudes
    ph = np.arange(n_lon) * 2.0 * math.pi / n_lon
    T, P = np.meshgrid(th, ph, indexing="ij")
    ring = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    v = np.concatenate([[[0.0, 0.0, 1.0]], ring, [[0.0, 0.0, -1.0]]], axis=0)
    top, bot = 0, v.shape[0] - 1

    def idx(i, j):  # ring i (0..n_lat-2), lon j
        return 1 + i * n_lon + (j % n_lon)

    t = []
    for j in range(n_lon):
        t.append((top, idx(0, j), idx(0, j + 1)))
        t.append((bot, idx(n_lat - 2, j + 1), idx(n_lat - 2, j)))
    for i in range(n_lat - 2):
        for j in range(n_lon):
            a, b = idx(i, j), idx(i, j + 1)
            c, d = idx(i + 1, j), idx(i + 1, j + 1)
            t.append((a, c, d))
            t.append((a, d, b))
    tris = np.array(t, dtype=np.int32)
    tris = orient_outward(v, tris, centre=np.zeros(3))
    v = v * np.asarray(semi_axes, dtype=np.float64)
    if rot is not None:
        v = v @ np.asarray(rot).T
    return v + np.asarray(centre, dtype=np.float64), tris


def convex_hull_mesh(points: np.ndarray):
    """Convex hull of a point cloud as an outward triangle mesh on the hull vertices."""
    from scipy.spatial import ConvexHull

    h = ConvexHull(points)
    used = np.unique(h.simplices)
    remap = -np.ones(points.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    v = points[used]
    t = remap[h.simplices].astype(np.int32)
    return v, orient_outward(v, t, centre=v.mean(axis=0))


# ----------------------------------------------------------------------------
# union of balls: boundary by marching tetrahedra on the signed distance field
# ----------------------------------------------------------------------------
# Kuhn (Freudenthal) split of the unit cube into 6 tetrahedra along the main
# diagonal; corner index = ix + 2*iy + 4*iz. The split is the same in every
# cell, so shared cube faces are cut along the same diagonal and the surface
# is closed.
_KUHN = np.array([
    [0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7],
    [0, 2, 6, 7], [0, 4, 5, 7], [0, 4, 6, 7],
], dtype=np.int64)


def _sdf_union(p: np.ndarray, centres: np.ndarray, radii: np.ndarray, chunk: int = 1 << 18) -> np.ndarray:
    out = np.empty(p.shape[0])
    for s in range(0, p.shape[0], chunk):
        q = p[s:s + chunk]
        d = np.sqrt(((q[:, None, :] - centres[None, :, :]) ** 2).sum(-1)) - radii[None, :]
        out[s:s + chunk] = d.min(axis=1)
    return out


def union_of_spheres(centres, radii, h: float, margin: float = 2.0, bisect_iters: int = 30):
    """Closed outward triangle mesh of the boundary of a union of balls.

    Marching tetrahedra (Kuhn split) on the grid of step ``h``; surface
    vertices sit on grid edges with a sign change, located by bisection on the
    exact signed distance min_i(|x - c_i| - r_i). Returns (verts, tris).
    """
    centres = np.asarray(centres, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)
    lo = (centres - radii[:, None]).min(0) - margin * h
    hi = (centres + radii[:, None]).max(0) + margin * h
    n = np.ceil((hi - lo) / h).astype(np.int64) + 1
    axes = [lo[k] + h * np.arange(n[k]) for k in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    f = _sdf_union(nodes, centres, radii)
    f[f == 0.0] = 1e-12 * h  # no node exactly on the surface
    inside = f < 0.0

    def nid(ix, iy, iz):
        return (ix * n[1] + iy) * n[2] + iz

    ix, iy, iz = np.meshgrid(np.arange(n[0] - 1), np.arange(n[1] - 1), np.arange(n[2] - 1), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    corner = np.stack([nid(ix + (c & 1), iy + ((c >> 1) & 1), iz + ((c >> 2) & 1)) for c in range(8)], 1)
    # keep only cells with a sign change
    cin = inside[corner]
    keep = cin.any(1) & ~cin.all(1)
    corner = corner[keep]
    tets = corner[:, _KUHN].reshape(-1, 4)
    tin = inside[tets]
    k = tin.sum(1)
    tets, tin, k = tets[(k > 0) & (k < 4)], tin[(k > 0) & (k < 4)], k[(k > 0) & (k < 4)]

    # sort each tet's nodes: inside ones first (stable), remembering parity
    order = np.argsort(~tin, axis=1, kind="stable")
    st = np.take_along_axis(tets, order, 1)

    edge_keys = []
    tri_edges = []  # list of (m, 3, 2) arrays of node pairs (inside, outside)

    def add(sel, pairs_list):
        tri_edges.append(np.stack([np.stack([st[sel, a], st[sel, b]], 1) for a, b in pairs_list], 1))

    s1, s2, s3 = k == 1, k == 2, k == 3
    # one inside node (0), outside 1,2,3
    add(s1, [(0, 1), (0, 2), (0, 3)])
    # three inside (0,1,2), outside 3
    add(s3, [(0, 3), (1, 3), (2, 3)])
    # two inside (0,1), outside (2,3): quad e02, e03, e13, e12
    add(s2, [(0, 2), (0, 3), (1, 3)])
    add(s2, [(0, 2), (1, 3), (1, 2)])
    te = np.concatenate(tri_edges, 0)  # (T, 3, 2) node pairs (in, out)
    flat = te.reshape(-1, 2)
    key = np.sort(flat, axis=1)
    uk, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    # locate the zero crossing on each unique grid edge
    a_in = np.where(inside[uk[:, 0]], uk[:, 0], uk[:, 1])
    b_out = np.where(inside[uk[:, 0]], uk[:, 1], uk[:, 0])
    pa, pb = nodes[a_in], nodes[b_out]
    lo_t = np.zeros(uk.shape[0])
    hi_t = np.ones(uk.shape[0])
    for _ in range(bisect_iters):
        mid = 0.5 * (lo_t + hi_t)
        fm = _sdf_union(pa + mid[:, None] * (pb - pa), centres, radii)
        ins = fm < 0.0
        lo_t = np.where(ins, mid, lo_t)
        hi_t = np.where(ins, hi_t, mid)
    tt = 0.5 * (lo_t + hi_t)
    verts = pa + tt[:, None] * (pb - pa)
    tris = inv.reshape(-1, 3).astype(np.int64)
    # orient each triangle so its normal points from the inside nodes to the outside ones
    tri_tet_in = te[:, :, 0]
    tri_tet_out = te[:, :, 1]
    cin_ = nodes[tri_tet_in].mean(1)
    cout_ = nodes[tri_tet_out].mean(1)
    nrm = _face_normals(verts, tris)
    flip = np.einsum("ij,ij->i", nrm, cout_ - cin_) < 0
    t2 = tris.copy()
    t2[flip, 1], t2[flip, 2] = tris[flip, 2], tris[flip, 1]
    return verts, t2.astype(np.int32)


def union_of_spheres_config(seed: int = 3, n_spheres: int = 20, box_side: float = 200.0,
                            rmin: float = 20.0, rmax: float = 60.0, target_faces: int = 100_000,
                            tol: float = 0.05, h0: float = 4.0, max_iter: int = 12):
    """Random union of balls meshed to about ``target_faces`` triangles (grid step tuned)."""
    rng = np.random.default_rng(seed)
    c = (rng.random((n_spheres, 3)) - 0.5) * box_side
    r = rmin + (rmax - rmin) * rng.random(n_spheres)
    h = h0
    best = None
    for _ in range(max_iter):
        v, t = union_of_spheres(c, r, h)
        nf = t.shape[0]
        if best is None or abs(nf - target_faces) < abs(best[1].shape[0] - target_faces):
            best = (v, t, h)
        if abs(nf - target_faces) <= tol * target_faces:
            break
        h *= math.sqrt(nf / target_faces)  # faces ~ area / h^2
    v, t, h = best
    return {"verts": v, "tris": t, "centres": c, "radii": r, "h": h}


# ----------------------------------------------------------------------------
# batched set of uneven meshes
# ----------------------------------------------------------------------------
def _log_uniform(rng, lo, hi):
    return math.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * rng.random())


def batch_config(seed: int = 5, n_meshes: int = 512, min_faces: int = 200, max_faces: int = 20_000,
                 min_q: int = 4096, max_q: int = 65536, qmax: float = 0.5,
                 hull_points=(32, 4000), scale=1.0):
    """Uneven batch: random ellipsoids and subdivided convex hulls, each with its own Q list."""
    rng = np.random.default_rng(seed)
    meshes = []
    for _ in range(n_meshes):
        if rng.random() < 0.5:
            T = _log_uniform(rng, min_faces, max_faces)
            n_lat = max(3, int(round(math.sqrt(T / 4.0))))
            ax = 10.0 + 40.0 * rng.random(3)
            rot = _rotation(rng)
            cen = (rng.random(3) - 0.5) * 40.0
            v, t = ellipsoid_uv(ax * scale, n_lat, rot=rot, centre=cen * scale)
            kind = "ellipsoid"
        else:
            npts = int(round(_log_uniform(rng, *hull_points)))
            rad = (10.0 + 40.0 * rng.random()) * scale
            d = rng.normal(size=(npts, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            pts = d * (rad * rng.random(npts) ** (1.0 / 3.0))[:, None]
            v, t = convex_hull_mesh(pts)
            while t.shape[0] < min_faces:
                v, t = subdivide(v, t)
            kind = "hull"
        nq = int(round(_log_uniform(rng, min_q, max_q)))
        q = q_random_ball(nq, qmax, rng)
        meshes.append({"verts": v, "tris": t.astype(np.int32), "q": q, "kind": kind})
    return meshes


# ----------------------------------------------------------------------------
# netgen surface mesh text reader (test helper)
# ----------------------------------------------------------------------------
def read_netgen_surfacemesh(text: str):
    """Parse netgen 'surfacemesh' text: header, point count, xyz lines, element count, 1-based triangles."""
    lines = [ln.strip() for ln in text.strip().splitlines() if ln.strip()]
    if lines[0] != "surfacemesh":
        raise ValueError("not a netgen surfacemesh")
    npt = int(lines[1])
    pts = np.array([[float(x) for x in ln.split()] for ln in lines[2:2 + npt]])
    nel = int(lines[2 + npt])
    el = np.array([[int(x) for x in ln.split()] for ln in lines[3 + npt:3 + npt + nel]], dtype=np.int32)
    return pts, el - 1


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
def config1():
    """Star polygon (64 vertices) and a 128^2 Q grid over [-20,20]^2; FP64."""
    return {"verts": star_polygon(seed=1, n=64), "q": q_grid_2d(128, 20.0)}


def config2():
    """Icosphere level 4 (5120 faces), R = 50, 64^3 Q grid over [-0.5,0.5]^3."""
    v, t = icosphere(4, 50.0)
    return {"verts": v, "tris": t, "q": q_grid_3d(64, 0.5), "radius": 50.0}


def config3(target_faces: int = 100_000):
    """Union of 20 balls (~1e5 faces), 128^3 Q grid over [-0.3,0.3]^3."""
    d = union_of_spheres_config(seed=3, target_faces=target_faces)
    d["q"] = q_grid_3d(128, 0.3)
    return d


def config4():
    """Icosphere level 6 with 2% radial noise, 256^2 Q slice at Qz = 0 over [-0.4,0.4]^2."""
    v0, t = icosphere(6, 50.0)
    rng = np.random.default_rng(4)
    v = perturb_radial(v0, 0.02, rng)
    return {"verts": v, "verts0": v0, "tris": t, "q": q_slice_z(256, 0.4), "radius": 50.0}


def config5(n_meshes: int = 512):
    """512 uneven meshes with 200-20000 faces and 4096-65536 random Q each."""
    return batch_config(seed=5, n_meshes=n_meshes)
