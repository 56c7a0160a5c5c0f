"""Planted mistakes in the oracle must be caught by its pins.

Each case below edits a private copy of the oracle's source on the CPU (a
flipped sign, a dropped term, a wrong index, a transposed operand, a wrong
factorial), loads it as a separate module and runs a compact battery of pins
that do not depend on the oracle itself: the paper's printed rectangle and
prism values, closed forms, brute-force quadrature and the matrix-exponential
tetrahedron fan of tests/indep.py. The unmodified oracle passes the battery;
every modified copy must fail at least one pin. The committed oracle is never
changed.
"""
import importlib.util
import json
import os
import sys

import numpy as np
import pytest

import meshgen as mg
from conftest import GOLDEN, ROOT
from indep import dd_exp, quad_tet, quad_tet_moment, quad_tri_fan, tetfan_ft3d
from test_oracle_dq import box_dq

ORACLE_SRC = os.path.join(ROOT, "oracle", "pft_oracle.py")


def _load(src: str, name: str):
    spec = importlib.util.spec_from_loader(name, loader=None)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[name] = mod  # dataclass-free module, but keep it importable by name while it runs
    try:
        exec(compile(src, f"<{name}>", "exec"), mod.__dict__)
    finally:
        sys.modules.pop(name, None)
    return mod


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


# ---------------------------------------------------------------------------
# the pin battery: each returns the relative error of one pinned fact
# ---------------------------------------------------------------------------
def _pin_rect_edges(O):
    g = json.load(open(os.path.join(GOLDEN, "rectangle_2d.json")))
    v = mg.rectangle_2d(g["a"], g["b"])
    err = 0.0
    for row in g["rows"]:
        terms = O.ft2d_edge_terms(v, np.array([row["q"]]))[0]
        err = max(err, _rel(terms, np.array([complex(*t) for t in row["edge_terms"]])))
    return err


def _pin_rect_integral(O):
    g = json.load(open(os.path.join(GOLDEN, "rectangle_2d.json")))
    v = mg.rectangle_2d(g["a"], g["b"])
    q = np.array([r["q"] for r in g["rows"]])
    return _rel(O.ft2d(v, q), np.array([complex(*r["integral"]) for r in g["rows"]]))


def _pin_polygon_quadrature(O):
    # star polygon off the origin (translation phase), general Q and one small-|Q| point (series branch)
    v = mg.star_polygon(seed=3, n=9) + np.array([0.4, -0.3])
    q = np.array([[1.3, -0.7], [-2.1, 0.4], [0.0, 3.0], [2e-3, 1e-3]])
    want = np.array([quad_tri_fan(v, Q) for Q in q])
    return _rel(O.ft2d(v, q), want)


def _pin_prism(O):
    g = json.load(open(os.path.join(GOLDEN, "prism_3d.json")))
    v, t = mg.box(g["a"], g["b"], g["c"])
    q = np.array([r["q"] for r in g["rows"]])
    e = _rel(O.ft3d(v, t, q), np.array([complex(*r["integral"]) for r in g["rows"]]))
    I = O.ft3d_face_terms(v, t, q)
    # box() lists the z = 0 face as triangles 0, 1 and the z = c face as triangles 2, 3
    e = max(e, _rel(I[:, 2] + I[:, 3], np.array([complex(*r["I_top"]) for r in g["rows"]])))
    e = max(e, _rel(I[:, 0] + I[:, 1], np.array([complex(*r["I_bottom"]) for r in g["rows"]])))
    return e


def _box_closed(a, b, c, o, Q):
    def f(L, q, x0):
        return L if q == 0.0 else (np.exp(1j * q * (x0 + L)) - np.exp(1j * q * x0)) / (1j * q)
    return f(a, Q[0], o[0]) * f(b, Q[1], o[1]) * f(c, Q[2], o[2])


def _pin_box_axes_and_zero(O):
    # Q along the axes is parallel to face normals (face-series branch) and perpendicular to edges (sinc(0));
    # Q = 0 is the volume; a tiny Q takes the fan-of-tetrahedra series
    a, b, c, o = 1.1, 0.8, 1.4, (0.3, -0.2, 0.5)
    v, t = mg.box(a, b, c, origin=o)
    q = np.array([[0.0, 0.0, 2.0], [1.7, 0.0, 0.0], [0.0, -2.4, 0.9], [0.0, 0.0, 0.0], [3e-3, -2e-3, 1e-3]])
    want = np.array([_box_closed(a, b, c, o, Q) for Q in q])
    return _rel(O.ft3d(v, t, q), want)


def _pin_tet_quadrature(O):
    a, b, c, d = (np.array(x, dtype=float) for x in ([0.1, 0.0, 0.2], [1.3, 0.1, -0.1], [0.2, 1.1, 0.3],
                                                      [0.4, 0.3, 1.2]))
    # outward orientation of the four faces
    v = np.stack([a, b, c, d])
    t = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]])
    q = np.array([[1.2, -0.8, 2.0], [-2.5, 0.3, 0.7], [0.4, 3.1, -1.0]])
    want = np.array([quad_tet(a, b, c, d, Q) for Q in q])
    return _rel(O.ft3d(v, t, q), want)


def _pin_tetfan(O):
    v, t = mg.icosphere(1, 1.3)
    v = v + np.array([0.7, -0.4, 0.2])
    N = np.cross(v[t[0, 1]] - v[t[0, 0]], v[t[0, 2]] - v[t[0, 0]])
    q = np.array([[1.1, -2.0, 0.6], [0.0, 0.0, 3.3], 2.5 * N / np.linalg.norm(N), [2e-3, 1e-3, -3e-3]])
    return _rel(O.ft3d(v, t, q), tetfan_ft3d(v, t, q))


def _pin_gradient(O):
    v, t = mg.icosphere(0, 1.1)
    v = v + np.array([0.2, 0.1, -0.3])
    rng = np.random.default_rng(5)
    q = np.concatenate([rng.normal(size=(4, 3)) * 1.5, [[1e-3, 2e-3, -1e-3]]])
    g = rng.normal(size=len(q)) + 1j * rng.normal(size=len(q))
    # dF/dv_k = sum over incident faces of N_m exp[iQ.a, iQ.b, iQ.c, iQ.v_k] (node k doubled)
    want = np.zeros_like(v)
    for qi, Q in enumerate(q):
        for tri in t:
            A, B, C = v[tri[0]], v[tri[1]], v[tri[2]]
            Nm = np.cross(B - A, C - A)
            ph = [1j * Q @ A, 1j * Q @ B, 1j * Q @ C]
            for k in range(3):
                want[tri[k]] += np.real(np.conj(g[qi]) * Nm * dd_exp(ph + [ph[k]]))
    return _rel(O.grad3d(v, t, q, g), want)


def _pin_dq_box(O):
    # grad_Q F of a box: off-axis, along a face normal, and a small Q (tetrahedron-series branch)
    a, b, c, o = 1.3, 0.7, 1.1, (0.2, -0.4, 0.3)
    v, t = mg.box(a, b, c, origin=o)
    q = np.array([[1.2, -0.7, 2.2], [0.0, 0.0, 2.5], [4.0, 3.0, -5.0], [0.05, 0.02, -0.03]])
    return _rel(O.ft3d_dq(v, t, q), np.array([box_dq(a, b, c, o, Q) for Q in q]))


def _pin_dq_tet_quadrature(O):
    v, t = mg.tetrahedron()
    v = v + np.array([0.3, -0.5, 0.2])
    q = np.array([[1.2, -0.8, 2.0], [0.4, 3.1, -1.0], [0.05, -0.02, 0.03]])
    want = np.array([1j * quad_tet_moment(v[0], v[1], v[2], v[3], Q) for Q in q])
    return _rel(O.ft3d_dq(v, t, q), want)


def _pin_regions_core_shell(O):
    outer, inner = ((2.0, 1.6, 1.8), (-1.0, -0.7, -0.9)), ((0.9, 0.5, 0.7), (-0.3, -0.2, 0.1))
    v, t, off = mg.nested_boxes(outer, inner)
    q = np.array([[1.2, -0.7, 2.2], [0.0, 0.0, 2.5]])
    F, _ = O.ft3d_regions(v, t, off, [3.0, -0.5], q)
    want = np.array([-0.5 * _box_closed(*outer[0], outer[1], Q) + 3.5 * _box_closed(*inner[0], inner[1], Q)
                     for Q in q])
    return _rel(F, want)


def _pin_poly_prism(O):
    # a prism over a non-convex polygon whose first three vertices turn clockwise (a reflex vertex at
    # index 1): polygon faces against the 2D transform times the axial integral, including Q along
    # the axis (the caps' series branch) and in the plane
    poly = np.array([[0.0, 0.0], [1.0, 0.4], [2.0, 0.0], [2.0, 2.0], [0.0, 2.0]]) + np.array([0.3, -0.2])
    h, z0 = 1.3, -0.4
    v, f = mg.prism_polygon(poly, h, z0)
    q = np.array([[1.1, -0.7, 0.9], [0.0, 0.0, 1.7], [2.3, 0.4, 0.0], [-0.5, 1.9, -1.2]])
    F2 = O.ft2d(poly, q[:, :2])
    ax = np.array([h if Q == 0.0 else (np.exp(1j * Q * (z0 + h)) - np.exp(1j * Q * z0)) / (1j * Q) for Q in q[:, 2]])
    return _rel(O.ft3d_poly(v, f, q), F2 * ax)


def _pin_orient_box(O):
    # the direction quadrature applied to the box's separable closed form
    a, b, c, o = 1.3, 0.7, 1.1, (0.2, -0.4, 0.3)
    v, t = mg.box(a, b, c, origin=o)
    d, w = mg.sphere_quadrature(5, 10)
    qabs = np.array([0.0, 0.9, 2.5])
    want = [float(np.sum(w * np.abs([_box_closed(a, b, c, o, qa * s) for s in d]) ** 2)) for qa in qabs]
    return _rel(O.orientation_average(v, t, qabs, d, w), want)


PINS = [_pin_rect_edges, _pin_rect_integral, _pin_polygon_quadrature, _pin_prism, _pin_box_axes_and_zero,
        _pin_tet_quadrature, _pin_tetfan, _pin_gradient, _pin_dq_box, _pin_dq_tet_quadrature,
        _pin_regions_core_shell, _pin_poly_prism, _pin_orient_box]
TOL = {_pin_polygon_quadrature: 1e-9, _pin_tet_quadrature: 1e-9, _pin_dq_tet_quadrature: 1e-9}


def _failures(O):
    bad = []
    for pin in PINS:
        try:
            err = pin(O)
            ok = np.isfinite(err) and err < TOL.get(pin, 1e-11)
        except Exception:  # a mutation that breaks the evaluation is caught too
            ok = False
        if not ok:
            bad.append(pin.__name__)
    return bad


# ---------------------------------------------------------------------------
# planted mistakes: (name, exact source fragment, replacement)
# ---------------------------------------------------------------------------
MUTATIONS = [
    ("2d edge normal sign", "qn_d = qg[:, 0:1] * d[None, :, 1] - qg[:, 1:2] * d[None, :, 0]",
     "qn_d = qg[:, 0:1] * d[None, :, 1] + qg[:, 1:2] * d[None, :, 0]"),
    ("2d edge start instead of midpoint", "np.exp(1j * (qg @ m.T)) * _sinc(eta)",
     "np.exp(1j * (qg @ ra.T)) * _sinc(eta)"),
    ("2d full instead of half edge phase", "        eta = 0.5 * (qg @ d.T)\n        term",
     "        eta = (qg @ d.T)\n        term"),
    ("2d translation phase sign", "out[gen] = np.exp(1j * (qg @ t)) * np.sum(term, axis=1)",
     "out[gen] = np.exp(-1j * (qg @ t)) * np.sum(term, axis=1)"),
    ("2d worked-example edge term sign", "return -(qn_d / Q2) * 1j * np.exp(1j * (q @ m.T)) * _sinc(eta)",
     "return (qn_d / Q2) * 1j * np.exp(1j * (q @ m.T)) * _sinc(eta)"),
    ("3d in-plane normal operands transposed", "nxd = np.cross(fc.nhat, fc.d[l])                        # n x d_l",
     "nxd = np.cross(fc.d[l], fc.nhat)"),
    ("3d dropped edge", "        for l in range(3):\n            nxd = np.cross(fc.nhat",
     "        for l in range(2):\n            nxd = np.cross(fc.nhat"),
    ("3d sinc of the midpoint instead of the edge", "            eta = 0.5 * (q @ fc.d[l].T)\n            acc",
     "            eta = 0.5 * (q @ fc.m[l].T)\n            acc"),
    ("3d edge phase at the start vertex", "acc += coef * 1j * np.exp(1j * (q @ fc.m[l].T)) * _sinc(eta)",
     "acc += coef * 1j * np.exp(1j * (q @ fc.v[l].T)) * _sinc(eta)"),
    ("3d face series factorial", "ser = simplex_exp_series(delta, dim=2)", "ser = simplex_exp_series(delta, dim=3)"),
    ("3d flux sign (the paper's printed sign)", "I = (-1j * (qq @ fc.nhat.T) / Q2[idx[s:e]][:, None]) * J",
     "I = (1j * (qq @ fc.nhat.T) / Q2[idx[s:e]][:, None]) * J"),
    ("3d translation phase sign", "out[idx[s:e]] = np.exp(1j * (qq @ t)) * np.sum(I, axis=1)",
     "out[idx[s:e]] = np.exp(-1j * (qq @ t)) * np.sum(I, axis=1)"),
    ("3d volume sign at Q = 0", "out[zero] = volume3d(v, tris)", "out[zero] = -volume3d(v, tris)"),
    ("3d small-Q tetrahedron weight", 'six_v = np.einsum("ij,ij->i", fc.N, a)',
     'six_v = 0.5 * np.einsum("ij,ij->i", fc.N, a)'),
    ("series phase sign", "s = s + (1j ** n) * h[n] / math.factorial(n + dim)",
     "s = s + ((-1j) ** n) * h[n] / math.factorial(n + dim)"),
    ("complete homogeneous recurrence index", "cur.append(cur[j - 1] + x * prev[j])",
     "cur.append(cur[j - 1] + x * prev[j - 1])"),
    ("series truncated", "if (n > 2 and bound < tol) or n >= 400:", "if (n > 2 and bound < 1e-3) or n >= 400:"),
    ("gradient barycentric corner shifted", "beta = np.cross(N, fc.d[(k + 1) % 3]) / np.where(fc.ok, N2, 1.0)[:, None]",
     "beta = np.cross(N, fc.d[(k + 2) % 3]) / np.where(fc.ok, N2, 1.0)[:, None]"),
    ("gradient node not doubled", "B[qi, fi, k] = pre * simplex_exp_series(delta + [delta[k]], dim=3)",
     "B[qi, fi, k] = pre * simplex_exp_series(delta + [delta[(k + 1) % 3]], dim=3)"),
    ("gradient dsinc term dropped", "- 1j * s[:, :, None] * 0.5 * u[(l + 2) % 3][None, :, :]))",
     "- 0.0 * s[:, :, None] * 0.5 * u[(l + 2) % 3][None, :, :]))"),
    ("gradient conjugate dropped", 'Rw += np.real(np.einsum("q,qfk->fk", np.conj(go[s:e]), B))',
     'Rw += np.real(np.einsum("q,qfk->fk", go[s:e], B))'),
    ("grad_Q: volume term dropped", "gF[idx[s:e]] = surf / q2[:, None] - qq * (Fc[idx[s:e]] / q2)[:, None]",
     "gF[idx[s:e]] = surf / q2[:, None]"),
    ("grad_Q: surface term sign", "surf += (qn * B[:, :, k]) @ vk", "surf -= (qn * B[:, :, k]) @ vk"),
    ("grad_Q: tetrahedron moment factorial", "mom = vol6[None, :] * simplex_exp_series(ph + [ph[k + 1]], dim=4)",
     "mom = vol6[None, :] * simplex_exp_series(ph + [ph[k + 1]], dim=3)"),
    ("grad_Q: doubled node shifted", "mom = vol6[None, :] * simplex_exp_series(ph + [ph[k + 1]], dim=4)",
     "mom = vol6[None, :] * simplex_exp_series(ph + [ph[k]], dim=4)"),
    ("grad_Q: translation term sign", "return ph_t[:, None] * (gF + 1j * t[None, :] * Fc[:, None])",
     "return ph_t[:, None] * (gF - 1j * t[None, :] * Fc[:, None])"),
    ("regions: densities dropped", "return (rho[:, None] * Fj).sum(axis=0), Fj", "return Fj.sum(axis=0), Fj"),
    ("polygon: edges traversed backwards", "P1 = np.roll(P, -1, axis=1)", "P1 = np.roll(P, 1, axis=1)"),
    ("polygon: closing edge dropped", "            for l in range(nu):\n                nxd = np.cross(nhat, d[:, l, :])",
     "            for l in range(nu - 1):\n                nxd = np.cross(nhat, d[:, l, :])"),
    ("polygon: unsigned fan-triangle areas",
     'two_a = np.einsum("ij,ij->i", np.cross(b - a, c - a), nhat[fi])   # signed 2 A_t',
     "two_a = np.linalg.norm(np.cross(b - a, c - a), axis=1)"),
    ("polygon: edge phase at the start vertex", "m = 0.5 * (P + P1)                                       # m_l",
     "m = P"),
    ("orientation: quadrature weights dropped", "out[i] = float(np.sum(weights * np.abs(F) ** 2))",
     "out[i] = float(np.mean(np.abs(F) ** 2))"),
    ("orientation: modulus not squared", "out[i] = float(np.sum(weights * np.abs(F) ** 2))",
     "out[i] = float(np.sum(weights * np.abs(F)))"),
]


def test_battery_passes_on_the_oracle():
    O = _load(open(ORACLE_SRC).read(), "oracle_control")
    assert _failures(O) == []


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new):
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, f"mutation site not found uniquely: {old!r}"
    O = _load(src.replace(old, new), "oracle_mutant")
    assert _failures(O), f"no pin caught the planted mistake: {name}"
