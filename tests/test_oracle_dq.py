"""Pins of grad_Q F (oracle.ft3d_dq): the Q-derivative of the volume integral, i * integral of r exp(iQ.r)."""
import math

import numpy as np

import meshgen as mg
import oracle as O
from indep import quad_tet_moment, tetfan_dF_dQ
from test_oracle_orient import tet_moments


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def box_dq(a, b, c, o, Q):
    """Separable closed form: F = f(a, Qx, ox) f(b, Qy, oy) f(c, Qz, oz), f(L, q, x0) = integral of
    exp(iqx) over [x0, x0 + L], differentiated factor by factor."""
    def f(L, q, x0):
        x1 = x0 + L
        return L if q == 0.0 else (np.exp(1j * q * x1) - np.exp(1j * q * x0)) / (1j * q)

    def df(L, q, x0):
        x1 = x0 + L
        if abs(q) * max(abs(x0), abs(x1)) < 0.1:  # the quotients cancel: sum_n i^(n+1) q^n (x1^(n+2) - x0^(n+2)) / (n! (n+2))
            return sum(1j ** (n + 1) * q ** n * (x1 ** (n + 2) - x0 ** (n + 2)) / (math.factorial(n) * (n + 2))
                       for n in range(14))
        e1, e0 = np.exp(1j * q * x1), np.exp(1j * q * x0)
        return (x1 * e1 - x0 * e0) / q + 1j * (e1 - e0) / q ** 2
    L, x0 = (a, b, c), o
    fs = [f(L[k], Q[k], x0[k]) for k in range(3)]
    ds = [df(L[k], Q[k], x0[k]) for k in range(3)]
    return np.array([ds[0] * fs[1] * fs[2], fs[0] * ds[1] * fs[2], fs[0] * fs[1] * ds[2]])


def test_box_closed_form():
    """On and off the axes (face-series branch, sinc(0)), a tiny Q (tetrahedron series) and Q = 0."""
    a, b, c, o = 1.3, 0.7, 1.1, (0.2, -0.4, 0.3)
    v, t = mg.box(a, b, c, origin=o)
    q = np.array([[1.2, -0.7, 2.2], [0.0, 0.0, 2.5], [1.7, 0.0, 0.0], [0.0, -0.9, 3.0], [4.0, 3.0, -5.0],
                  [2e-3, 1e-3, -1e-3], [0.0, 0.0, 0.0]])
    want = np.array([box_dq(a, b, c, o, Q) for Q in q])
    assert rel(O.ft3d_dq(v, t, q), want) < 1e-12


def test_tetrahedron_quadrature():
    """Collapsed Gauss-Legendre quadrature of i r exp(iQ.r) over a single tetrahedron."""
    v, t = mg.tetrahedron()
    v = v + np.array([0.3, -0.5, 0.2])
    q = np.array([[1.2, -0.8, 2.0], [-2.5, 0.3, 0.7], [0.4, 3.1, -1.0], [0.05, -0.02, 0.03]])
    want = np.array([1j * quad_tet_moment(v[0], v[1], v[2], v[3], Q) for Q in q])
    assert rel(O.ft3d_dq(v, t, q), want) < 1e-10


def test_tetrahedron_fan_with_doubled_node():
    """Exact per-tetrahedron moments from the matrix exponential, fan from a point other than the
    oracle's centre, at Q along a face normal, generic Q and small Q."""
    v, t = mg.icosphere(1, 1.3)
    v = v * np.array([1.0, 0.8, 1.2]) + np.array([0.7, -0.4, 0.2])
    N = np.cross(v[t[0, 1]] - v[t[0, 0]], v[t[0, 2]] - v[t[0, 0]])
    q = np.array([[1.1, -2.0, 0.6], [0.0, 0.0, 3.3], 2.5 * N / np.linalg.norm(N), [2e-3, 1e-3, -3e-3], [0.2, 0.1, 0.0]])
    assert rel(O.ft3d_dq(v, t, q), tetfan_dF_dQ(v, t, q, origin=[0.1, 0.2, -0.1])) < 1e-11


def test_central_differences_of_the_transform():
    rng = np.random.default_rng(11)
    v, t = mg.ellipsoid_uv([1.5, 1.0, 0.8], 5, rot=np.linalg.qr(rng.normal(size=(3, 3)))[0], centre=(0.4, 0.2, -0.3))
    q = rng.normal(size=(6, 3)) * 2.0
    h = 1e-5
    fd = np.stack([(O.ft3d(v, t, q + h * e) - O.ft3d(v, t, q - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    assert rel(O.ft3d_dq(v, t, q), fd) < 1e-8


def test_zero_is_i_volume_times_centroid():
    rng = np.random.default_rng(12)
    v, t = mg.ellipsoid_uv([2.0, 1.0, 1.5], 6, rot=np.linalg.qr(rng.normal(size=(3, 3)))[0], centre=(1.0, -2.0, 0.5))
    V, cen, _ = tet_moments(v, t)
    assert rel(O.ft3d_dq(v, t, np.zeros((1, 3)))[0], 1j * V * cen) < 1e-13


def test_scaling_identity():
    """F of the mesh scaled by s is s^3 F(sQ); d/ds at s = 1: sum_k v_k.dF/dv_k = 3F + Q.grad_Q F."""
    v, t = mg.icosphere(1, 1.0)
    v = v * np.array([1.2, 0.9, 1.0]) + np.array([0.3, 0.1, -0.2])
    rng = np.random.default_rng(13)
    q = np.concatenate([rng.normal(size=(5, 3)) * 2.5, [[0.01, -0.02, 0.015]]])
    J = O.dft3d_dverts(v, t, q)
    lhs = np.einsum("qvk,vk->q", J, v)
    rhs = 3.0 * O.ft3d(v, t, q) + np.einsum("qk,qk->q", q, O.ft3d_dq(v, t, q))
    assert rel(rhs, lhs) < 1e-11


def test_translation_and_branch_continuity():
    """Shifting the mesh by a multiplies F by exp(iQ.a) and adds i a F to the gradient; the
    two branches agree on both sides of the series threshold."""
    v, t = mg.icosphere(2, 1.0)
    v = v * np.array([1.0, 0.8, 1.2])
    a = np.array([0.7, -1.1, 0.4])
    rng = np.random.default_rng(14)
    q = rng.normal(size=(5, 3)) * 1.7
    g0, F0 = O.ft3d_dq(v, t, q), O.ft3d(v, t, q)
    ph = np.exp(1j * (q @ a))
    assert rel(O.ft3d_dq(v + a, t, q), ph[:, None] * (g0 + 1j * a[None, :] * F0[:, None])) < 1e-12
    R = np.max(np.linalg.norm(v - v.mean(0), axis=1))
    d = rng.normal(size=(4, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    for qr in (0.3, 0.5, 0.8):
        qq = d * qr / R
        assert rel(O.ft3d_dq(v, t, qq, tau_dq=0.0), O.ft3d_dq(v, t, qq, tau_dq=1e9)) < 1e-13
