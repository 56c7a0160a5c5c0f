"""Pins of the orientation-averaged intensity (oracle.orientation_average) and of its direction quadrature."""
import math

import numpy as np

import meshgen as mg
import oracle as O
from indep import sphere_ft


def tet_moments(verts, tris):
    """Volume, centroid and radius of gyration of a closed mesh from closed-form tetrahedron moments.

    Fan of tetrahedra (0, a, b, c): signed volume V_t = a.(b x c)/6, first moment V_t (a+b+c)/4,
    second moment of |r|^2: V_t/20 (|a|^2 + |b|^2 + |c|^2 + |a+b+c|^2).
    """
    v = np.asarray(verts, dtype=np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    vt = np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    V = vt.sum()
    s = a + b + c
    first = (vt[:, None] * s / 4.0).sum(0)
    second = (vt / 20.0 * (np.sum(a * a, 1) + np.sum(b * b, 1) + np.sum(c * c, 1) + np.sum(s * s, 1))).sum()
    cen = first / V
    return V, cen, second / V - cen @ cen


def test_quadrature_moments():
    """sum w = 1 and the first even moments of the direction over the sphere: <x^2> = 1/3,
    <x^4> = 1/5, <x^2 y^2> = 1/15, odd moments vanish (exact for the product rule's degree)."""
    d, w = mg.sphere_quadrature(5, 10)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15)
    for k in range(3):
        assert abs((w * d[:, k] ** 2).sum() - 1.0 / 3.0) < 1e-14
        assert abs((w * d[:, k] ** 4).sum() - 1.0 / 5.0) < 1e-14
        assert abs((w * d[:, k]).sum()) < 1e-15
        assert abs((w * d[:, k] ** 3).sum()) < 1e-15
    assert abs((w * d[:, 0] ** 2 * d[:, 1] ** 2).sum() - 1.0 / 15.0) < 1e-14
    assert abs((w * d[:, 1] ** 2 * d[:, 2] ** 2).sum() - 1.0 / 15.0) < 1e-14


def test_guinier_law():
    """I(q) = V^2 (1 - q^2 Rg^2 / 3 + O(q^4)): the q^2 coefficient (Richardson over q and 2q)
    against the radius of gyration from tetrahedron moments, on an off-centre rotated ellipsoid."""
    rng = np.random.default_rng(21)
    rot = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    v, t = mg.ellipsoid_uv([3.0, 2.0, 1.5], 9, rot=rot, centre=(1.0, -2.0, 0.5))
    V, _, rg2 = tet_moments(v, t)
    assert abs(O.orientation_average(v, t, [0.0], *mg.sphere_quadrature(3, 6))[0] - V * V) < 1e-12 * V * V
    d, w = mg.sphere_quadrature(6, 12)
    q = 0.01
    I = O.orientation_average(v, t, [q, 2 * q], d, w)
    A = (1.0 - I / (V * V)) / np.array([q, 2 * q]) ** 2
    coef = A[0] - (A[1] - A[0]) / 3.0
    assert abs(coef - rg2 / 3.0) < 1e-7 * rg2


def test_box_against_closed_form_average():
    """The same quadrature applied to the separable closed-form transform of a box."""
    a, b, c, o = 1.3, 0.7, 1.1, np.array([0.2, -0.4, 0.3])
    v, t = mg.box(a, b, c, origin=tuple(o))
    d, w = mg.sphere_quadrature(7, 14)
    qabs = np.array([0.0, 0.4, 1.7, 3.5, 6.0])

    def f(L, qq, x0):
        small = np.abs(qq) < 1e-12
        qs = np.where(small, 1.0, qq)
        return np.where(small, L, (np.exp(1j * qs * (x0 + L)) - np.exp(1j * qs * x0)) / (1j * qs))

    want = []
    for qa in qabs:
        Q = qa * d
        F = f(a, Q[:, 0], o[0]) * f(b, Q[:, 1], o[1]) * f(c, Q[:, 2], o[2])
        want.append(np.sum(w * np.abs(F) ** 2))
    got = O.orientation_average(v, t, qabs, d, w)
    assert np.max(np.abs(got - np.array(want)) / np.array(want)) < 1e-12


def test_icosphere_converges_to_the_sphere():
    """|F|^2 of the sphere (the paper's sphere form, scaled) is direction independent; icosphere
    averages approach it against the volume-matched radius (about 16x per subdivision level here)."""
    d, w = mg.sphere_quadrature(6, 12)
    qabs = np.linspace(0.3, 6.0, 8)
    errs = []
    for level in (2, 3):
        v, t = mg.icosphere(level, 1.0)
        V = tet_moments(v, t)[0]
        r_eff = (3.0 * V / (4.0 * math.pi)) ** (1.0 / 3.0)
        want = np.abs(sphere_ft(qabs, r_eff)) ** 2
        got = O.orientation_average(v, t, qabs, d, w)
        errs.append(float(np.linalg.norm(got - want) / np.linalg.norm(want)))
    assert errs[0] < 5e-5 and errs[1] < 3e-6
    assert errs[1] < errs[0] / 8.0
