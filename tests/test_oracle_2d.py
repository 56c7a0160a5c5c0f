"""Pins of the 2D oracle (oracle.ft2d) against what the paper and mathematics fix."""
import json
import math
import os

import numpy as np
import pytest

import meshgen as mg
import oracle as O
from indep import quad_tri_fan
from conftest import GOLDEN


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def test_rectangle_edge_terms_match_worked_example():
    """Each of the four printed edge terms of eq. rectangle_sum, edge by edge."""
    g = json.load(open(os.path.join(GOLDEN, "rectangle_2d.json")))
    v = mg.rectangle_2d(g["a"], g["b"])
    for row in g["rows"]:
        terms = O.ft2d_edge_terms(v, np.array([row["q"]]))[0]
        want = np.array([complex(*t) for t in row["edge_terms"]])
        assert rel(terms, want) < 1e-13


def test_rectangle_closed_form():
    """eq. rectangle_integral and FT_Rect (paper) = oracle F(Q), incl. Q on the axes."""
    g = json.load(open(os.path.join(GOLDEN, "rectangle_2d.json")))
    v = mg.rectangle_2d(g["a"], g["b"])
    q = np.array([r["q"] for r in g["rows"]])
    F = O.ft2d(v, q)
    for i, row in enumerate(g["rows"]):
        assert abs(F[i] - complex(*row["integral"])) < 1e-13 * abs(complex(*row["integral"])) + 1e-15
        assert abs(F[i] - complex(*row["ft_rect"])) < 1e-13 * abs(complex(*row["ft_rect"])) + 1e-15
    # on the axes the separable integral is a * (e^{i Qy b}-1)/(i Qy) etc.
    a, b = g["a"], g["b"]
    qa = np.array([[0.0, 1.3], [2.2, 0.0], [0.0, -0.004]])
    F = O.ft2d(v, qa)
    want = [a * (np.exp(1j * 1.3 * b) - 1) / (1j * 1.3), b * (np.exp(1j * 2.2 * a) - 1) / (1j * 2.2),
            a * (np.exp(-1j * 0.004 * b) - 1) / (-1j * 0.004)]
    assert rel(F, np.array(want)) < 1e-12


def test_area_at_q0_and_small_q_continuity():
    v = mg.star_polygon(seed=1, n=64)
    A = O.area2d(v)
    assert O.ft2d(v, np.zeros((1, 2)))[0] == pytest.approx(A, rel=1e-15)
    # shoelace vs an independent triangle-fan sum
    two_a = sum((v[i][0] - v[0][0]) * (v[i + 1][1] - v[0][1]) - (v[i][1] - v[0][1]) * (v[i + 1][0] - v[0][0])
                for i in range(1, len(v) - 1))
    assert A == pytest.approx(0.5 * two_a, rel=1e-14)
    # both sides of the series threshold agree (R ~ 1, tau = 1e-2)
    rng = np.random.default_rng(0)
    d = rng.normal(size=(20, 2))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q = d * np.geomspace(1e-4, 3e-1, 20)[:, None]
    F_lo = O.ft2d(v, q, tau_vol=1.0)     # series for all of these
    F_hi = O.ft2d(v, q, tau_vol=1e-9)    # edge sums for all of these
    assert rel(F_lo[q[:, 0] ** 2 + q[:, 1] ** 2 > 1e-4], F_hi[q[:, 0] ** 2 + q[:, 1] ** 2 > 1e-4]) < 1e-11


def test_brute_force_quadrature_star_polygon():
    v = mg.star_polygon(seed=1, n=64)
    rng = np.random.default_rng(1)
    q = rng.normal(size=(12, 2)) * 3.0
    F = O.ft2d(v, q)
    # the star polygon is star-shaped about the origin: integrate the fan from the origin
    want = np.array([quad_tri_fan(np.concatenate([[[0.0, 0.0]], v, v[:1]]), Q, n=40) for Q in q])
    assert rel(F, want) < 1e-12


def test_invariants_2d():
    v = mg.star_polygon(seed=3, n=40)
    rng = np.random.default_rng(2)
    q = rng.normal(size=(50, 2)) * 4
    F = O.ft2d(v, q)
    # Hermitian symmetry
    assert rel(O.ft2d(v, -q), np.conj(F)) < 1e-13
    # translation: F_{r+t}(Q) = exp(iQ.t) F(Q)
    t = np.array([0.37, -1.2])
    assert rel(O.ft2d(v + t, q), np.exp(1j * q @ t) * F) < 1e-13
    # rotation: F_{R r}(Q) = F(R^T Q)
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    assert rel(O.ft2d(v @ Rm.T, q), O.ft2d(v, q @ Rm)) < 1e-13
    # scaling: F_{s r}(Q) = s^2 F(s Q)
    s = 1.9
    assert rel(O.ft2d(s * v, q), s * s * O.ft2d(v, s * q)) < 1e-13
    # orientation flip gives -F
    assert rel(O.ft2d(v[::-1], q), -F) < 1e-13


def test_hole_is_difference_of_contours():
    outer = mg.rectangle_2d(2.0, 1.5)
    inner = mg.rectangle_2d(0.5, 0.4) + np.array([0.6, 0.3])
    verts = np.concatenate([outer, inner[::-1]])  # hole traversed clockwise
    rng = np.random.default_rng(3)
    q = rng.normal(size=(30, 2)) * 3
    F = O.ft2d(verts, q, offsets=[0, 4, 8])
    assert rel(F, O.ft2d(outer, q) - O.ft2d(inner, q)) < 1e-13
    assert O.ft2d(verts, np.zeros((1, 2)), offsets=[0, 4, 8])[0].real == pytest.approx(3.0 - 0.2, rel=1e-14)


def test_edge_perpendicular_to_q_is_not_dropped():
    """Q.d = 0 for two edges of the rectangle: removable, sinc(0) = 1 (the printed code would drop them)."""
    v = mg.rectangle_2d(1.0, 2.0)
    F = O.ft2d(v, np.array([[0.0, 0.8]]))[0]
    want = 1.0 * (np.exp(1j * 0.8 * 2.0) - 1) / (1j * 0.8)
    assert abs(F - want) < 1e-14
