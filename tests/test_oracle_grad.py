"""Pins of the oracle's vertex gradient (oracle.grad3d / dft3d_dverts)."""
import numpy as np

import meshgen as mg
import oracle as O
from indep import tetfan_dF_dv


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _mesh():
    v, t = mg.icosphere(1, 1.0)
    return v * np.array([1.0, 0.8, 1.2]) + np.array([0.05, -0.1, 0.2]), t


def test_jacobian_vs_central_differences():
    v, t = _mesh()
    rng = np.random.default_rng(0)
    q = np.concatenate([rng.normal(size=(6, 3)) * 2.0, [[0.0, 0.0, 1.5], [1e-3, 0.0, 0.0]]])
    J = O.dft3d_dverts(v, t, q)
    h = 1e-5
    for k in [0, 5, 17, 33]:
        for c in range(3):
            vp, vm = v.copy(), v.copy()
            vp[k, c] += h
            vm[k, c] -= h
            fd = (O.ft3d(vp, t, q) - O.ft3d(vm, t, q)) / (2 * h)
            assert np.max(np.abs(J[:, k, c] - fd)) < 1e-8 * max(1.0, np.max(np.abs(fd)))


def test_jacobian_vs_matrix_exponential_divided_differences():
    """dF/dv_k = sum_m N_m exp[iQ.a, iQ.b, iQ.c, iQ.v_k] evaluated independently with expm."""
    for v, t in [mg.tetrahedron(), _mesh()]:
        rng = np.random.default_rng(3)
        q = np.concatenate([rng.normal(size=(5, 3)) * 2.5, [[0.0, 0.0, 0.0], [0.0, 2.0, 0.0]]])
        assert rel(O.dft3d_dverts(v, t, q), tetfan_dF_dv(v, t, q)) < 1e-12


def test_volume_gradient_at_q0():
    v, t = _mesh()
    J = O.dft3d_dverts(v, t, np.zeros((1, 3)))[0]
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    N = np.cross(b - a, c - a)
    want = np.zeros_like(v)
    for k in range(3):
        np.add.at(want, t[:, k], N / 6.0)
    assert rel(J.real, want) < 1e-13 and np.max(np.abs(J.imag)) < 1e-15


def test_translation_identity():
    """Translating every vertex by dt multiplies F by exp(iQ.dt): sum_k dF/dv_k = i Q F."""
    v, t = _mesh()
    rng = np.random.default_rng(1)
    q = rng.normal(size=(10, 3)) * 3
    J = O.dft3d_dverts(v, t, q)
    F = O.ft3d(v, t, q)
    assert rel(J.sum(axis=1), 1j * q * F[:, None]) < 1e-12


def test_intensity_loss_gradient_fd_and_zero_sum():
    v, t = _mesh()
    rng = np.random.default_rng(2)
    q = rng.normal(size=(30, 3)) * 2
    target = np.abs(O.ft3d(v * 1.03, t, q)) ** 2
    w = 1.0 / q.shape[0]

    def loss(vv):
        F = O.ft3d(vv, t, q)
        return float(np.sum(w * (np.abs(F) ** 2 - target) ** 2))

    F = O.ft3d(v, t, q)
    g = 4 * w * (np.abs(F) ** 2 - target) * F   # dL/dReF + i dL/dImF
    G = O.grad3d(v, t, q, g)
    # translation invariance of |F|^2 => gradients sum to zero
    assert np.max(np.abs(G.sum(axis=0))) < 1e-12 * np.max(np.abs(G))
    h = 1e-6
    for k in [2, 11, 40]:
        for c in range(3):
            vp, vm = v.copy(), v.copy()
            vp[k, c] += h
            vm[k, c] -= h
            fd = (loss(vp) - loss(vm)) / (2 * h)
            assert abs(G[k, c] - fd) < 1e-7 * max(1.0, np.max(np.abs(G)))


def test_selected_vertices_match_full_gradient():
    v, t = _mesh()
    rng = np.random.default_rng(5)
    q = rng.normal(size=(40, 3)) * 2
    g = rng.normal(size=40) + 1j * rng.normal(size=40)
    G = O.grad3d(v, t, q, g)
    ids = [0, 7, 19, 41]
    assert rel(O.grad3d_vertices(v, t, q, g, ids), G[ids]) < 1e-13


def test_vertex_moment_branch_continuity():
    v, t = _mesh()
    rng = np.random.default_rng(6)
    d = rng.normal(size=(30, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q = d * np.geomspace(0.05, 5.0, 30)[:, None]
    J1 = O.dft3d_dverts(v, t, q, tau_face=0.2)
    J2 = O.dft3d_dverts(v, t, q, tau_face=3.0)
    assert rel(J1, J2) < 1e-10
