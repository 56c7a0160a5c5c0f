"""Pins of the polygon-face oracle (oracle.ft3d_poly): eq. sum_elements_3d with nu_m edges per face."""
import json
import os

import numpy as np

import meshgen as mg
import oracle as O
from conftest import GOLDEN


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def test_prism_whole_rectangular_faces():
    """The paper's prism example works with whole rectangular faces: eq. prism_direct and the face
    terms I_{z=c}, I_{z=0} are single quad faces here (no triangulation)."""
    g = json.load(open(os.path.join(GOLDEN, "prism_3d.json")))
    v, f = mg.box_quads(g["a"], g["b"], g["c"])
    q = np.array([r["q"] for r in g["rows"]])
    assert rel(O.ft3d_poly(v, f, q), np.array([complex(*r["integral"]) for r in g["rows"]])) < 1e-13
    I = O.ft3d_poly_face_terms(v, f, q)
    assert rel(I[:, 1], np.array([complex(*r["I_top"]) for r in g["rows"]])) < 1e-13
    assert rel(I[:, 0], np.array([complex(*r["I_bottom"]) for r in g["rows"]])) < 1e-13


def test_box_axes_and_small_q():
    """Q along the axes (parallel to face normals: the fan-series branch; perpendicular to edges:
    sinc(0)), Q = 0 and a tiny Q against the separable closed form."""
    a, b, c, o = 1.3, 0.7, 1.1, (0.2, -0.4, 0.3)
    v, f = mg.box_quads(a, b, c, origin=o)

    def f1(L, qq, x0):
        return L if qq == 0.0 else (np.exp(1j * qq * (x0 + L)) - np.exp(1j * qq * x0)) / (1j * qq)

    q = np.array([[0, 0, 2.5], [1.7, 0, 0], [0, -0.9, 3.0], [0, 0, 0], [2e-3, 1e-3, -1e-3], [1.2, -0.7, 2.2]])
    want = np.array([f1(a, Q[0], o[0]) * f1(b, Q[1], o[1]) * f1(c, Q[2], o[2]) for Q in q])
    # the closed form itself cancels at the tiny Q (about 1e-13 there)
    assert rel(O.ft3d_poly(v, f, q), want) < 1e-12


def test_prism_over_polygon_is_2d_transform_times_axial_integral():
    """A right prism over a star polygon (nu-gon caps, quad sides): F(Q) = F_2D(Qx, Qy) *
    (exp(i Qz (z0 + h)) - exp(i Qz z0)) / (i Qz), the 2D transform from the independent 2D oracle."""
    poly = mg.star_polygon(seed=4, n=11, rmin=0.6, rmax=1.2) + np.array([0.3, -0.2])
    h, z0 = 1.7, -0.4
    v, f = mg.prism_polygon(poly, h, z0)
    rng = np.random.default_rng(3)
    q = np.concatenate([rng.normal(size=(60, 3)) * 2.5, [[0.0, 0.0, 1.3], [1.1, -0.6, 0.0], [0.0, 0.0, 0.0]]])
    F2 = O.ft2d(poly, q[:, :2])
    ax = np.array([h if Q == 0.0 else (np.exp(1j * Q * (z0 + h)) - np.exp(1j * Q * z0)) / (1j * Q) for Q in q[:, 2]])
    assert rel(O.ft3d_poly(v, f, q), F2 * ax) < 1e-12


def test_matches_fan_triangulation():
    """Planar quad/triangle ellipsoid: the polygon form equals the triangle form on its fan
    triangulation (an exact identity for planar faces), incl. Q near face normals."""
    rng = np.random.default_rng(5)
    v, f = mg.ellipsoid_quads([3.0, 2.0, 1.5], 8, 12, rot=np.linalg.qr(rng.normal(size=(3, 3)))[0],
                              centre=(0.5, -1.0, 0.3))
    tri = np.array([[x[0], x[l], x[l + 1]] for x in f for l in range(1, len(x) - 1)])
    P = v[f[30]]
    n = np.cross(P[1] - P[0], P[2] - P[0])
    q = np.concatenate([mg.q_random_ball(80, 3.0, rng), [2.0 * n / np.linalg.norm(n), [0, 0, 0], [1e-4, 0, 0]]])
    assert rel(O.ft3d_poly(v, f, q), O.ft3d(v, tri, q)) < 1e-13
