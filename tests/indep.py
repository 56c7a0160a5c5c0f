"""Independent evaluations of the polygon / polyhedron transform, for pinning the oracle.

None of these share code or formulas with ``oracle/``:
* ``tetfan_ft3d``   -- the volume as a fan of tetrahedra from a point o, each
  tetrahedron integrated exactly as 6|T| times the divided difference of exp
  at the nodes i Q.(o, a, b, c), read off the matrix exponential of the 4x4
  bidiagonal (Opitz) matrix with scipy.linalg.expm.
* ``quad_tet`` / ``quad_tri_fan`` -- tensor Gauss-Legendre quadrature on the
  collapsed (Duffy) cube mapped onto each simplex.
* ``sphere_ft``     -- the paper's unit-sphere formula scaled to radius R.
* ``tetfan_dF_dQ`` / ``quad_tet_moment`` -- grad_Q F = i * integral of r exp(iQ.r):
  per tetrahedron the barycentric moments as divided differences with a
  doubled node (expm), or Gauss-Legendre quadrature of r exp(iQ.r).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm
from scipy.special import gamma, jv


def dd_exp(nodes) -> complex:
    """Divided difference exp[z_0, ..., z_k] via expm of the bidiagonal matrix (Opitz)."""
    k = len(nodes)
    M = np.diag(np.asarray(nodes, dtype=np.complex128)) + np.diag(np.ones(k - 1, dtype=np.complex128), 1)
    return complex(expm(M)[0, k - 1])


def tetfan_ft3d(verts, tris, q, origin=None) -> np.ndarray:
    """F(Q) = sum over faces of the signed tetrahedron (o, a, b, c), exact per tetrahedron."""
    v = np.asarray(verts, dtype=np.float64)
    o = v.mean(axis=0) if origin is None else np.asarray(origin, dtype=np.float64)
    out = np.zeros(len(q), dtype=np.complex128)
    for qi, Q in enumerate(np.asarray(q, dtype=np.float64)):
        s = 0.0 + 0.0j
        for t in tris:
            a, b, c = v[t[0]], v[t[1]], v[t[2]]
            six_vol = float(np.dot(a - o, np.cross(b - o, c - o)))
            s += six_vol * dd_exp([1j * Q @ o, 1j * Q @ a, 1j * Q @ b, 1j * Q @ c])
        out[qi] = s
    return out


def tetfan_dF_dv(verts, tris, q) -> np.ndarray:
    """dF/dv_k = sum_{m ∋ k} N_m exp[iQ.a, iQ.b, iQ.c, iQ.v_k] (node k doubled), via expm. [nq, nv, 3]."""
    v = np.asarray(verts, dtype=np.float64)
    out = np.zeros((len(q), v.shape[0], 3), dtype=np.complex128)
    for qi, Q in enumerate(np.asarray(q, dtype=np.float64)):
        for t in tris:
            a, b, c = v[t[0]], v[t[1]], v[t[2]]
            N = np.cross(b - a, c - a)
            ph = [1j * Q @ a, 1j * Q @ b, 1j * Q @ c]
            for k in range(3):
                out[qi, t[k]] += N * dd_exp(ph + [ph[k]])
    return out


def tetfan_dF_dQ(verts, tris, q, origin=None) -> np.ndarray:
    """grad_Q F = i sum over tetrahedra (o, a, b, c) of sum_j r_j 6|T| exp[iQ.o, iQ.a, iQ.b, iQ.c, iQ.r_j]
    (the integral of lambda_j exp(iQ.r) over T is 6|T| times the divided difference with node j
    doubled). [nq, 3] complex."""
    v = np.asarray(verts, dtype=np.float64)
    o = v.mean(axis=0) if origin is None else np.asarray(origin, dtype=np.float64)
    out = np.zeros((len(q), 3), dtype=np.complex128)
    for qi, Q in enumerate(np.asarray(q, dtype=np.float64)):
        for t in tris:
            pts = [o, v[t[0]], v[t[1]], v[t[2]]]
            six_vol = float(np.dot(pts[1] - o, np.cross(pts[2] - o, pts[3] - o)))
            nodes = [1j * Q @ p for p in pts]
            for j, p in enumerate(pts):
                out[qi] += 1j * six_vol * dd_exp(nodes + [nodes[j]]) * p
    return out


def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def quad_tet(a, b, c, d, Q, n=24) -> complex:
    """Integral of exp(iQ.r) over the tetrahedron (a, b, c, d) by collapsed Gauss-Legendre (signed)."""
    x, w = _gl01(n)
    U, V, W = np.meshgrid(x, x, x, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    s1 = U
    s2 = V * (1 - U)
    s3 = W * (1 - U) * (1 - V)
    jac = (1 - U) ** 2 * (1 - V)
    P = (a[None, None, None, :] + s1[..., None] * (b - a) + s2[..., None] * (c - a) + s3[..., None] * (d - a))
    six_vol = float(np.dot(b - a, np.cross(c - a, d - a)))
    f = np.exp(1j * (P @ Q))
    return complex(six_vol * np.sum(WU * WV * WW * jac * f))


def quad_tet_moment(a, b, c, d, Q, n=24) -> np.ndarray:
    """Integral of r exp(iQ.r) over the tetrahedron (a, b, c, d) by collapsed Gauss-Legendre (signed). [3]."""
    x, w = _gl01(n)
    U, V, W = np.meshgrid(x, x, x, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    s1 = U
    s2 = V * (1 - U)
    s3 = W * (1 - U) * (1 - V)
    jac = (1 - U) ** 2 * (1 - V)
    P = (a[None, None, None, :] + s1[..., None] * (b - a) + s2[..., None] * (c - a) + s3[..., None] * (d - a))
    six_vol = float(np.dot(b - a, np.cross(c - a, d - a)))
    f = (WU * WV * WW * jac * np.exp(1j * (P @ Q)))[..., None] * P
    return six_vol * np.sum(f.reshape(-1, 3), axis=0)


def quad_tri_fan(verts2d, Q, n=30) -> complex:
    """Integral of exp(iQ.r) over a polygon as a fan of triangles from its first vertex (signed)."""
    v = np.asarray(verts2d, dtype=np.float64)
    x, w = _gl01(n)
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    s1, s2 = U, V * (1 - U)
    jac = 1 - U
    tot = 0.0 + 0.0j
    a = v[0]
    for i in range(1, len(v) - 1):
        b, c = v[i], v[i + 1]
        two_a = (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0])
        P = a + s1[..., None] * (b - a) + s2[..., None] * (c - a)
        tot += two_a * np.sum(WU * WV * jac * np.exp(1j * (P @ Q)))
    return complex(tot)


def sphere_ft(qabs, R) -> np.ndarray:
    """Paper's unit-sphere form (4 pi/3) Gamma(5/2) J_{3/2}(Q) / (Q/2)^{3/2}, scaled: F_R(Q) = R^3 F_1(Q R)."""
    qabs = np.asarray(qabs, dtype=np.float64)
    x = qabs * R
    with np.errstate(invalid="ignore", divide="ignore"):
        f1 = (4 * math.pi / 3) * gamma(2.5) * jv(1.5, x) / (x / 2) ** 1.5
    return np.where(x == 0, 4 * math.pi / 3 * R ** 3, R ** 3 * f1)
