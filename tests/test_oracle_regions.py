"""Pins of the piecewise-constant density transform (oracle.ft3d_regions) and its gradients."""
import numpy as np
import pytest

import meshgen as mg
import oracle as O
from test_oracle_dq import box_dq


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


def box_f(a, b, c, o, Q):
    def f(L, q, x0):
        return L if q == 0.0 else (np.exp(1j * q * (x0 + L)) - np.exp(1j * q * x0)) / (1j * q)
    return f(a, Q[0], o[0]) * f(b, Q[1], o[1]) * f(c, Q[2], o[2])


Q_SET = np.array([[1.2, -0.7, 2.2], [0.0, 0.0, 2.5], [1.7, 0.0, 0.0], [4.0, 3.0, -5.0], [2e-3, 1e-3, -1e-3],
                  [0.0, 0.0, 0.0]])


def test_box_cut_in_two_with_equal_density():
    """Two adjacent boxes of equal density: the shared wall appears in both regions with opposite
    orientations and cancels, leaving the closed form of the whole box."""
    o = (0.2, -0.4, 0.3)
    v1, t1 = mg.box(0.5, 0.7, 1.1, origin=o)
    v2, t2 = mg.box(0.8, 0.7, 1.1, origin=(o[0] + 0.5, o[1], o[2]))
    v, t, off = mg.stack_regions([(v1, t1), (v2, t2)], [[(0, +1)], [(1, +1)]])
    F, Fj = O.ft3d_regions(v, t, off, [2.5, 2.5], Q_SET)
    want = np.array([2.5 * box_f(1.3, 0.7, 1.1, o, Q) for Q in Q_SET])
    assert rel(F, want) < 1e-12
    assert rel(Fj[0], [box_f(0.5, 0.7, 1.1, o, Q) for Q in Q_SET]) < 1e-12


def test_core_and_shell_boxes():
    """Core density 3 inside a shell of density -0.5: F = -0.5 F_outer + 3.5 F_inner."""
    outer, inner = ((2.0, 1.6, 1.8), (-1.0, -0.7, -0.9)), ((0.9, 0.5, 0.7), (-0.3, -0.2, 0.1))
    v, t, off = mg.nested_boxes(outer, inner)
    rho = np.array([3.0, -0.5])
    F, Fj = O.ft3d_regions(v, t, off, rho, Q_SET)
    fo = np.array([box_f(*outer[0], outer[1], Q) for Q in Q_SET])
    fi = np.array([box_f(*inner[0], inner[1], Q) for Q in Q_SET])
    assert rel(F, -0.5 * fo + 3.5 * fi) < 1e-12
    assert rel(Fj[1], fo - fi) < 1e-12


def test_gradients_against_closed_forms_and_differences():
    """dL/drho_j and dL/dQ for L = sum_Q w |F|^2 on the core-shell boxes (closed forms), dL/dv by
    central differences of the same loss through ft3d_regions."""
    outer, inner = ((2.0, 1.6, 1.8), (-1.0, -0.7, -0.9)), ((0.9, 0.5, 0.7), (-0.3, -0.2, 0.1))
    v, t, off = mg.nested_boxes(outer, inner)
    rho = np.array([3.0, -0.5])
    q = Q_SET[:5]
    w = np.array([0.7, 1.3, 0.4, 2.0, 1.1])
    fo = np.array([box_f(*outer[0], outer[1], Q) for Q in q])
    fi = np.array([box_f(*inner[0], inner[1], Q) for Q in q])
    F = rho[1] * fo + (rho[0] - rho[1]) * fi
    g = 2.0 * w * F  # dL/dReF + i dL/dImF
    gv, gr, gq = O.grad3d_regions(v, t, off, rho, q, g)
    # dL/drho: F_core = fi, F_shell = fo - fi
    assert rel(gr, [np.sum(np.real(np.conj(g) * fi)), np.sum(np.real(np.conj(g) * (fo - fi)))]) < 1e-12
    dF = np.array([rho[1] * box_dq(*outer[0], outer[1], Q) + (rho[0] - rho[1]) * box_dq(*inner[0], inner[1], Q)
                   for Q in q])
    assert rel(gq, np.real(np.conj(g)[:, None] * dF)) < 1e-12

    def loss(vv):
        FF, _ = O.ft3d_regions(vv, t, off, rho, q)
        return float(np.sum(w * np.abs(FF) ** 2))
    h = 1e-6
    for vid in (0, 5, 9, 14):
        for k in range(3):
            e = np.zeros_like(v)
            e[vid, k] = h
            fd = (loss(v + e) - loss(v - e)) / (2 * h)
            assert abs(gv[vid, k] - fd) < 1e-7 * max(1.0, np.max(np.abs(gv)))


def test_layered_sphere_volumes_and_empty_region():
    v, t, off = mg.layered_sphere(1, [0.5, 0.8, 1.0])
    F, Fj = O.ft3d_regions(v, t, off, [1.0, 2.0, 3.0], np.zeros((1, 3)))
    vols = [O.volume3d(v, t[off[j]:off[j + 1]]) for j in range(3)]
    assert np.allclose(Fj[:, 0].real, vols, rtol=1e-13) and vols[1] > 0 and vols[2] > 0
    assert abs(F[0] - (vols[0] + 2 * vols[1] + 3 * vols[2])) < 1e-12 * abs(F[0])
    off2 = np.array([0, 0, len(t)])
    F2, Fj2 = O.ft3d_regions(v, t, off2, [5.0, 1.0], Q_SET[:2])
    assert np.all(Fj2[0] == 0) and rel(F2, O.ft3d(v, t, Q_SET[:2])) < 1e-13
    with pytest.raises(ValueError):
        O.ft3d_regions(v, t, [0, 10], [1.0], Q_SET[:1])
