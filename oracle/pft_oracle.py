"""FP64 CPU oracle: direct Fourier transform of polygons (2D) and closed triangle meshes (3D).

TEST INFRASTRUCTURE ONLY -- imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library. Plain NumPy in
float64 / complex128, vectorised over (Q, face) blocks; no blocking, fusion or
reordering beyond what the formulas state.

Transform convention (paper, eq. for FT_V and the 2D area integral):
    F(Q) = integral over the region of exp(+i Q.r),   F(0) = area / volume.
Meshes: triangles counter-clockwise seen from outside (paper, 3D section and
the appendix code's element convention). Polygons: counter-clockwise contours;
a clockwise contour subtracts (a hole).

Readings of the paper used here (each also justified in the test suite):
* The edge-sum of eq. sum_elements_3d carries the in-plane edge normal as
  n x d_l, which points into the face for a counter-clockwise contour; the 2D
  derivation (eq. line_normal) needs the outward normal d_l x n. The oracle
  uses the outward one, so F(0) = +volume and the prism example's face terms
  are reproduced.
* The edge sum runs over the nu_m edges l = 0..nu_m-1 with r_{nu_m} = r_0.
* The factored phase in the midpoint form is the edge midpoint
  (r_{l+1} + r_l)/2.
* Removable singularities are evaluated by series of the same integrals:
  Q = 0 gives the area / volume; small |Q| uses the fan of simplices from the
  centroid; Q nearly parallel to a face normal uses the face's own simplex
  series; Q perpendicular to an edge uses sinc(0) = 1.
"""
from __future__ import annotations

import math

import numpy as np

# series thresholds (dimensionless phase spreads)
TAU_FACE = 1.0   # face series when |Q_perp| * L_m < TAU_FACE (L_m = longest edge of face m)
TAU_VOL = 1e-2   # fan-of-simplices series when |Q| * R < TAU_VOL (R = max distance from the centroid)
TAU_DQ = 0.5     # fan-of-tetrahedra series for grad_Q F when |Q| * R < TAU_DQ
CHUNK_ELEMS = 1 << 20  # (Q x face) elements per block


# ----------------------------------------------------------------------------
# small helpers
# ----------------------------------------------------------------------------
def area2d(verts: np.ndarray, offsets=None) -> float:
    """Signed area of one or more closed contours (shoelace formula; CCW positive)."""
    v = np.asarray(verts, dtype=np.float64)
    tot = 0.0
    for s, e in _contours(v.shape[0], offsets):
        x, y = v[s:e, 0], v[s:e, 1]
        tot += 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))
    return tot


def volume3d(verts: np.ndarray, tris: np.ndarray) -> float:
    """Signed volume enclosed by a closed, outward triangle mesh: sum of a.(b x c)/6."""
    v = np.asarray(verts, dtype=np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    return float(np.sum(np.einsum("ij,ij->i", a, np.cross(b, c)))) / 6.0


def _contours(nv, offsets):
    if offsets is None:
        return [(0, nv)]
    off = list(offsets)
    return [(off[i], off[i + 1]) for i in range(len(off) - 1)]


def hsym(xs, n_max: int):
    """Complete homogeneous symmetric polynomials h_0 .. h_{n_max} of the variables ``xs``.

    Recurrence over variables: h_n(x_1..x_j) = h_n(x_1..x_{j-1}) + x_j h_{n-1}(x_1..x_j).
    """
    xs = [np.asarray(x) for x in xs]
    shape = np.broadcast(*xs).shape
    dt = np.result_type(*xs, np.float64)
    prev = [np.ones(shape, dtype=dt) for _ in range(len(xs) + 1)]  # h_0^{(j)} = 1
    out = [prev[-1].copy()]
    for _ in range(1, n_max + 1):
        cur = [np.zeros(shape, dtype=dt)]  # h_n^{(0)} = 0 for n >= 1
        for j, x in enumerate(xs, start=1):
            cur.append(cur[j - 1] + x * prev[j])
        out.append(cur[-1])
        prev = cur
    return out


def _n_terms(xmax: float, nvars: int, dim: int, tol: float = 1e-20) -> int:
    """Number of series terms so that C(n+k-1,k-1) xmax^n / (n+dim)! < tol."""
    n = 0
    while True:
        bound = math.comb(n + nvars - 1, nvars - 1) * xmax ** n / math.factorial(n + dim)
        if (n > 2 and bound < tol) or n >= 400:
            return n
        n += 1


def simplex_exp_series(xs, dim: int) -> np.ndarray:
    """sum_n i^n h_n(xs) / (n+dim)!  for real phases xs (len(xs) = dim + 1 for a simplex).

    For a d-simplex S with vertex phases f_j = Q.v_j, the integral of exp(i f)
    over S equals d! |S| times this sum (simplex moment formula: the integral
    of f^n over S is |S| d! n!/(n+d)! h_n(f_0..f_d)); it is also the divided
    difference of exp at the nodes i f_j.
    """
    xs = [np.asarray(x, dtype=np.float64) for x in xs]
    xmax = max(float(np.max(np.abs(x))) if x.size else 0.0 for x in xs)
    K = _n_terms(xmax, len(xs), dim)
    h = hsym(xs, K)
    s = np.zeros(np.broadcast(*xs).shape, dtype=np.complex128)
    for n in range(K, -1, -1):  # smallest terms first
        s = s + (1j ** n) * h[n] / math.factorial(n + dim)
    return s


def _sinc(x):
    """sin(x)/x with sinc(0) = 1."""
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))


def _dsinc(x):
    """d/dx sinc(x) = (x cos x - sin x)/x^2; Taylor series for |x| < 0.5."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 0.5
    xs = np.where(small, x, 0.0)
    ser = np.zeros_like(x)
    for k in range(8, 0, -1):  # sum_k (-1)^k 2k x^(2k-1) / (2k+1)!
        ser = ser + ((-1) ** k) * 2 * k * xs ** (2 * k - 1) / math.factorial(2 * k + 1)
    xb = np.where(small, 1.0, x)
    direct = (xb * np.cos(xb) - np.sin(xb)) / (xb * xb)
    return np.where(small, ser, direct)


def _blocks(nq: int, nf: int):
    step = max(1, CHUNK_ELEMS // max(nf, 1))
    for s in range(0, nq, step):
        yield s, min(nq, s + step)


# ----------------------------------------------------------------------------
# 2D: polygon
# ----------------------------------------------------------------------------
def ft2d_edge_terms(verts: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Per-edge contour integrals of F.n ds for one closed contour, absolute coordinates.

    Edge l runs from r_l to r_{l+1} (wrapping). Eq. line_integral_generic in
    its midpoint form: -(Q.n_l)|d_l|/Q^2 * i exp(i Q.m_l) sinc(Q.d_l/2), with
    n_l |d_l| = (dy, -dx) from eq. line_normal. Returns [nq, n_edges] complex.
    Q = 0 is not defined here (the integrand's field has 1/Q^2).
    """
    r = np.asarray(verts, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    r1 = np.roll(r, -1, axis=0)
    d = r1 - r
    m = 0.5 * (r + r1)
    Q2 = np.sum(q * q, axis=1)[:, None]
    qn_d = q[:, 0:1] * d[None, :, 1] - q[:, 1:2] * d[None, :, 0]
    eta = 0.5 * (q @ d.T)
    return -(qn_d / Q2) * 1j * np.exp(1j * (q @ m.T)) * _sinc(eta)


def ft2d(verts: np.ndarray, q: np.ndarray, offsets=None, tau_vol: float = TAU_VOL) -> np.ndarray:
    """F(Q) of a polygon (one or more contours; CCW adds, CW subtracts). [nq] complex128.

    Parity pins: rectangle closed form eq. rectangle_integral and its worked
    edge terms eq. rectangle_sum; shoelace area at Q = 0; fan-triangle brute force.
    """
    v = np.asarray(verts, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 2)
    nq = q.shape[0]
    t = v.mean(axis=0)
    r = v - t
    R = float(np.max(np.linalg.norm(r, axis=1))) if r.size else 0.0
    cont = _contours(v.shape[0], offsets)
    # edges of every contour, relative to the centroid t
    ra = np.concatenate([r[s:e] for s, e in cont])
    rb = np.concatenate([np.roll(r[s:e], -1, axis=0) for s, e in cont])
    d = rb - ra
    m = 0.5 * (ra + rb)
    out = np.empty(nq, dtype=np.complex128)
    Q2 = np.sum(q * q, axis=1)
    qa = np.sqrt(Q2)
    zero = Q2 == 0.0
    small = (~zero) & (qa * R < tau_vol)
    gen = ~(zero | small)
    out[zero] = area2d(v, offsets)
    if np.any(small):
        qs = q[small]
        fa, fb = qs @ ra.T, qs @ rb.T
        two_a = ra[:, 0] * rb[:, 1] - ra[:, 1] * rb[:, 0]  # 2 x signed area of (t, r_l, r_l+1)
        ser = simplex_exp_series([np.zeros_like(fa), fa, fb], dim=2)
        out[small] = np.exp(1j * (qs @ t)) * np.sum(two_a[None, :] * ser, axis=1)
    if np.any(gen):
        qg = q[gen]
        qn_d = qg[:, 0:1] * d[None, :, 1] - qg[:, 1:2] * d[None, :, 0]   # (Q.n_l)|d_l|
        eta = 0.5 * (qg @ d.T)
        term = -(qn_d / Q2[gen][:, None]) * 1j * np.exp(1j * (qg @ m.T)) * _sinc(eta)
        out[gen] = np.exp(1j * (qg @ t)) * np.sum(term, axis=1)
    return out


# ----------------------------------------------------------------------------
# 3D: closed triangle mesh
# ----------------------------------------------------------------------------
class _Faces:
    """Per-face geometry in the coordinates given (no re-centring)."""

    def __init__(self, verts, tris):
        v = np.asarray(verts, dtype=np.float64)
        t = np.asarray(tris, dtype=np.int64)
        self.v = [v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]]           # a, b, c
        a, b, c = self.v
        self.N = np.cross(b - a, c - a)                          # 2 A n_hat
        self.nN = np.linalg.norm(self.N, axis=1)                 # 2 A
        self.ok = self.nN > 0.0
        self.nhat = np.where(self.ok[:, None], self.N / np.where(self.ok, self.nN, 1.0)[:, None], 0.0)
        self.g = (a + b + c) / 3.0
        self.d = [b - a, c - b, a - c]                           # d_l = r_{l+1} - r_l
        self.m = [0.5 * (a + b), 0.5 * (b + c), 0.5 * (c + a)]   # edge midpoints
        self.L = np.sqrt(np.max(np.stack([np.sum(dd * dd, 1) for dd in self.d]), axis=0))


def _face_integrals(fc: _Faces, q: np.ndarray, tau_face: float) -> np.ndarray:
    """J_m(Q) = integral of exp(i Q.r) over each triangle. [nq, nf] complex.

    Edge branch: in-plane 2D result (eq. line_integral_generic, midpoint form)
    with Q -> Q_perp and the outward in-plane edge normal d_l x n:
        J = sum_l [Q_perp.(n x d_l)/Q_perp^2] i exp(i Q.m_l) sinc(Q.d_l/2).
    Series branch (|Q_perp| L < tau_face): J = 2A exp(i Q.g) sum_n i^n h_n(delta)/(n+2)!,
    delta_k = Q.(v_k - g).
    """
    nq, nf = q.shape[0], fc.N.shape[0]
    Qpar = q @ fc.nhat.T                                            # Q.n
    Qperp = q[:, None, :] - Qpar[:, :, None] * fc.nhat[None, :, :]
    Qperp2 = np.sum(Qperp * Qperp, axis=2)
    series = (Qperp2 * fc.L[None, :] ** 2 < tau_face ** 2) & fc.ok[None, :]
    edge = (~series) & fc.ok[None, :]
    J = np.zeros((nq, nf), dtype=np.complex128)
    if np.any(edge):
        acc = np.zeros((nq, nf), dtype=np.complex128)
        safe = np.where(edge, Qperp2, 1.0)
        for l in range(3):
            nxd = np.cross(fc.nhat, fc.d[l])                        # n x d_l
            coef = np.einsum("qfk,fk->qf", Qperp, nxd) / safe       # Q_perp.(n x d_l)/Q_perp^2
            eta = 0.5 * (q @ fc.d[l].T)
            acc += coef * 1j * np.exp(1j * (q @ fc.m[l].T)) * _sinc(eta)
        J = np.where(edge, acc, J)
    if np.any(series):
        qi, fi = np.nonzero(series)
        qq = q[qi]
        g = fc.g[fi]
        delta = [np.sum(qq * (fc.v[k][fi] - g), axis=1) for k in range(3)]
        ser = simplex_exp_series(delta, dim=2)
        J[qi, fi] = fc.nN[fi] * np.exp(1j * np.sum(qq * g, axis=1)) * ser
    return J


def face_integrals(verts, tris, q, tau_face: float = TAU_FACE) -> np.ndarray:
    """Integral of exp(i Q.r) over each triangle, absolute coordinates. [nq, nf] complex."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    fc = _Faces(verts, tris)
    out = np.empty((q.shape[0], fc.N.shape[0]), dtype=np.complex128)
    for s, e in _blocks(q.shape[0], fc.N.shape[0]):
        out[s:e] = _face_integrals(fc, q[s:e], tau_face)
    return out


def ft3d_face_terms(verts, tris, q, tau_face: float = TAU_FACE) -> np.ndarray:
    """Per-face flux integrals I_m = (-i Q.n_m / Q^2) J_m (eq. single_area_integral). [nq, nf].

    Summed over a closed mesh they give F(Q) (eq. sum_elements_3d). Absolute
    coordinates; Q = 0 is excluded (1/Q^2).
    """
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    fc = _Faces(verts, tris)
    J = face_integrals(verts, tris, q, tau_face)
    Q2 = np.sum(q * q, axis=1)[:, None]
    return (-1j * (q @ fc.nhat.T) / Q2) * J


def ft3d(verts, tris, q, tau_face: float = TAU_FACE, tau_vol: float = TAU_VOL) -> np.ndarray:
    """F(Q) = volume integral of exp(i Q.r) inside a closed outward triangle mesh. [nq] complex128.

    Re-centred on the vertex mean t: F(Q) = exp(i Q.t) sum_m I_m(Q) in centred
    coordinates. Q = 0 gives the signed volume; |Q| R < tau_vol sums the
    tetrahedra (t, a_m, b_m, c_m) by their simplex series.

    Parity pins: prism closed form eq. prism_direct and the face terms
    I_{z=c}, I_{z=0}; sphere form factor (convergence); tetra-fan divided
    differences via a matrix exponential; brute-force quadrature; invariants.
    """
    v = np.asarray(verts, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    t = v.mean(axis=0)
    r = v - t
    fc = _Faces(r, tris)
    R = float(np.max(np.linalg.norm(r, axis=1)))
    nq = q.shape[0]
    out = np.empty(nq, dtype=np.complex128)
    Q2 = np.sum(q * q, axis=1)
    zero = Q2 == 0.0
    small = (~zero) & (np.sqrt(Q2) * R < tau_vol)
    gen = ~(zero | small)
    out[zero] = volume3d(v, tris)
    if np.any(small):
        qs = q[small]
        a, b, c = fc.v
        six_v = np.einsum("ij,ij->i", fc.N, a)  # 6 x signed volume of (t, a, b, c) = N.a
        for s, e in _blocks(qs.shape[0], a.shape[0]):
            qq = qs[s:e]
            ser = simplex_exp_series([np.zeros((e - s, a.shape[0])), qq @ a.T, qq @ b.T, qq @ c.T], dim=3)
            out[np.nonzero(small)[0][s:e]] = np.exp(1j * (qq @ t)) * np.sum(six_v[None, :] * ser, axis=1)
    if np.any(gen):
        qg = q[gen]
        idx = np.nonzero(gen)[0]
        for s, e in _blocks(qg.shape[0], fc.N.shape[0]):
            qq = qg[s:e]
            J = _face_integrals(fc, qq, tau_face)
            I = (-1j * (qq @ fc.nhat.T) / Q2[idx[s:e]][:, None]) * J
            out[idx[s:e]] = np.exp(1j * (qq @ t)) * np.sum(I, axis=1)
    return out


# ----------------------------------------------------------------------------
# 3D: closed mesh of planar polygon faces (eq. sum_elements_3d for general nu_m)
# ----------------------------------------------------------------------------
def _poly_faces(faces):
    faces = [np.asarray(f, dtype=np.int64).reshape(-1) for f in faces]
    for f in faces:
        if f.size < 3:
            raise ValueError("a face needs at least 3 vertices")
    return faces


def _poly_face_integrals(r, faces, q, tau_face):
    """J_m(Q) = integral of exp(i Q.r) over each planar polygon face, coordinates as given, and the
    unit normals. Returns (J [nq, nf] complex, nhat [nf, 3]).

    Edge branch: the in-plane 2D result (eq. line_integral_generic, midpoint form) with Q -> Q_perp
    and the outward in-plane edge normal d_l x n, over the nu_m edges:
        J = sum_l [Q_perp.(n x d_l)/Q_perp^2] i exp(i Q.m_l) sinc(Q.d_l/2).
    Series branch (|Q_perp| L < tau_face): the fan triangles (r_0, r_l, r_{l+1}) with signed areas,
    each 2A_t exp(i Q.g_t) sum_n i^n h_n(delta)/(n+2)!.
    """
    nq, nf = q.shape[0], len(faces)
    J = np.zeros((nq, nf), dtype=np.complex128)
    nhat_all = np.zeros((nf, 3))
    by_nu = {}
    for idx, f in enumerate(faces):
        by_nu.setdefault(f.size, []).append(idx)
    for nu, ids in by_nu.items():
        ids = np.asarray(ids)
        P = r[np.stack([faces[i] for i in ids])]                 # [nf_g, nu, 3]
        P1 = np.roll(P, -1, axis=1)
        Narea = 0.5 * np.sum(np.cross(P, P1), axis=1)            # area vector A n
        A = np.linalg.norm(Narea, axis=1)
        ok = A > 0.0
        nhat = np.where(ok[:, None], Narea / np.where(ok, A, 1.0)[:, None], 0.0)
        nhat_all[ids] = nhat
        d = P1 - P                                               # d_l = r_{l+1} - r_l
        m = 0.5 * (P + P1)                                       # m_l
        L = np.sqrt(np.max(np.sum(d * d, axis=2), axis=1))
        Qpar = q @ nhat.T
        Qperp = q[:, None, :] - Qpar[:, :, None] * nhat[None, :, :]
        Qperp2 = np.sum(Qperp * Qperp, axis=2)
        series = (Qperp2 * L[None, :] ** 2 < tau_face ** 2) & ok[None, :]
        edge = (~series) & ok[None, :]
        Jg = np.zeros((nq, ids.size), dtype=np.complex128)
        if np.any(edge):
            safe = np.where(edge, Qperp2, 1.0)
            acc = np.zeros((nq, ids.size), dtype=np.complex128)
            for l in range(nu):
                nxd = np.cross(nhat, d[:, l, :])
                coef = np.einsum("qfk,fk->qf", Qperp, nxd) / safe
                eta = 0.5 * (q @ d[:, l, :].T)
                acc += coef * 1j * np.exp(1j * (q @ m[:, l, :].T)) * _sinc(eta)
            Jg = np.where(edge, acc, Jg)
        if np.any(series):
            qi, fi = np.nonzero(series)
            qq = q[qi]
            ser = np.zeros(qi.size, dtype=np.complex128)
            for l in range(1, nu - 1):
                a, b, c = P[fi, 0], P[fi, l], P[fi, l + 1]
                g = (a + b + c) / 3.0
                two_a = np.einsum("ij,ij->i", np.cross(b - a, c - a), nhat[fi])   # signed 2 A_t
                delta = [np.sum(qq * (x - g), axis=1) for x in (a, b, c)]
                ser += two_a * np.exp(1j * np.sum(qq * g, axis=1)) * simplex_exp_series(delta, dim=2)
            Jg[qi, fi] = ser
        J[:, ids] = Jg
    return J, nhat_all


def ft3d_poly_face_terms(verts, faces, q, tau_face: float = TAU_FACE) -> np.ndarray:
    """Per-face flux integrals I_m = (-i Q.n_m / Q^2) J_m of planar polygon faces (eq.
    single_area_integral), absolute coordinates, Q = 0 excluded. [nq, nf]."""
    v = np.asarray(verts, dtype=np.float64)
    faces = _poly_faces(faces)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    J, nhat = _poly_face_integrals(v, faces, q, tau_face)
    Q2 = np.sum(q * q, axis=1)[:, None]
    return (-1j * (q @ nhat.T) / Q2) * J


def ft3d_poly(verts, faces, q, tau_face: float = TAU_FACE, tau_vol: float = TAU_VOL) -> np.ndarray:
    """F(Q) of the volume enclosed by planar polygon faces, each a counter-clockwise (seen from
    outside) list of vertex indices. [nq] complex128.

    eq. sum_elements_3d with nu_m edges per face (the in-plane edge normal taken outward, as in
    ``ft3d``): F = exp(i Q.t) sum_m (-i Q.n_m / Q^2) J_m in coordinates centred on the vertex mean t,
    J_m from ``_poly_face_integrals``. Q = 0 gives the volume and |Q| R < tau_vol the
    tetrahedron-fan series over the fan triangles, as in ``ft3d``.
    Parity pins: the paper's prism face terms I_{z=c}, I_{z=0} for whole rectangular faces and
    eq. prism_direct, prisms over polygons (the 2D transform times the axial integral), and
    agreement with ``ft3d`` on fan triangulations.
    """
    v = np.asarray(verts, dtype=np.float64)
    faces = _poly_faces(faces)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    t = v.mean(axis=0)
    r = v - t
    R = float(np.max(np.linalg.norm(r, axis=1)))
    tri = np.array([[f[0], f[l], f[l + 1]] for f in faces for l in range(1, f.size - 1)], dtype=np.int64)
    out = np.empty(q.shape[0], dtype=np.complex128)
    Q2 = np.sum(q * q, axis=1)
    zero = Q2 == 0.0
    small = (~zero) & (np.sqrt(Q2) * R < tau_vol)
    gen = ~(zero | small)
    out[zero] = volume3d(v, tri)
    if np.any(small):
        out[small] = ft3d(v, tri, q[small], tau_face, tau_vol)  # the same fan-of-tetrahedra series
    if np.any(gen):
        qg = q[gen]
        idx = np.nonzero(gen)[0]
        for s0, e0 in _blocks(qg.shape[0], max(len(faces), 1) * 4):
            qq = qg[s0:e0]
            J, nhat = _poly_face_integrals(r, faces, qq, tau_face)
            I = (-1j * (qq @ nhat.T) / Q2[idx[s0:e0]][:, None]) * J
            out[idx[s0:e0]] = np.exp(1j * (qq @ t)) * np.sum(I, axis=1)
    return out


# ----------------------------------------------------------------------------
# 3D gradient with respect to the vertices
# ----------------------------------------------------------------------------
def _vertex_moments(fc: _Faces, q: np.ndarray, tau_face: float) -> np.ndarray:
    """B_{m,k}(Q) = integral over triangle m of lambda_k exp(i Q.r) dA. [nq, nf, 3] complex.

    lambda_k is the barycentric (hat) function of corner k. Moving corner k of
    face m by dv changes the enclosed volume integral by n_m.dv B_{m,k}
    (transport theorem with the boundary velocity lambda_k dv).

    Edge branch: lambda_k = 1/3 + beta_k.(r - g), beta_k = N x d_{k+1} / |N|^2,
    and the integral of (r - g) exp(i Q.(r - g)) is -i grad_Q of the centred face
    integral J_c = i |N| S / |P|^2, S = sum_l (P.d_l) sinc(Q.d_l/2) exp(i Q.(m_l - g)),
    P = Q x N (the edge form of the face integral), differentiated in closed form.
    Series branch: B = 2A exp(i Q.g) sum_n i^n h_n(delta_a, delta_b, delta_c, delta_k)/(n+3)!.
    """
    nq, nf = q.shape[0], fc.N.shape[0]
    N, nN = fc.N, fc.nN
    N2 = nN * nN
    u = [fc.v[k] - fc.g for k in range(3)]
    P = np.cross(q[:, None, :], N[None, :, :])
    P2 = np.sum(P * P, axis=2)
    series = (P2 * fc.L[None, :] ** 2 < (tau_face ** 2) * N2[None, :]) & fc.ok[None, :]
    edge = (~series) & fc.ok[None, :]
    B = np.zeros((nq, nf, 3), dtype=np.complex128)
    phase_g = np.exp(1j * (q @ fc.g.T))
    if np.any(edge):
        P2s = np.where(edge, P2, 1.0)
        S = np.zeros((nq, nf), dtype=np.complex128)
        gS = np.zeros((nq, nf, 3), dtype=np.complex128)
        for l in range(3):
            dl = fc.d[l]
            w = np.einsum("qfk,fk->qf", P, dl)                      # P.d_l
            eta = 0.5 * (q @ dl.T)
            E = np.exp(1j * (q @ (-0.5 * u[(l + 2) % 3]).T))        # exp(i Q.(m_l - g))
            s, sp = _sinc(eta), _dsinc(eta)
            S += w * s * E
            nxd = np.cross(N, dl)                                   # grad_Q (P.d_l) = N x d_l
            gS += E[:, :, None] * (nxd[None, :, :] * s[:, :, None]
                                   + w[:, :, None] * (sp[:, :, None] * 0.5 * dl[None, :, :]
                                                      - 1j * s[:, :, None] * 0.5 * u[(l + 2) % 3][None, :, :]))
        QN = q @ N.T
        gP2 = 2.0 * (N2[None, :, None] * q[:, None, :] - QN[:, :, None] * N[None, :, :])
        Jc = 1j * nN[None, :] * S / P2s
        Mc = nN[None, :, None] * (gS / P2s[:, :, None] - S[:, :, None] * gP2 / (P2s * P2s)[:, :, None])
        for k in range(3):
            beta = np.cross(N, fc.d[(k + 1) % 3]) / np.where(fc.ok, N2, 1.0)[:, None]
            Bk = phase_g * (Jc / 3.0 + np.einsum("qfk,fk->qf", Mc, beta))
            B[:, :, k] = np.where(edge, Bk, 0.0)
    if np.any(series):
        qi, fi = np.nonzero(series)
        qq = q[qi]
        delta = [np.sum(qq * u[k][fi], axis=1) for k in range(3)]
        pre = nN[fi] * phase_g[qi, fi]
        for k in range(3):
            B[qi, fi, k] = pre * simplex_exp_series(delta + [delta[k]], dim=3)
    return B


def face_vertex_moments(verts, tris, q, tau_face: float = TAU_FACE) -> np.ndarray:
    """Integral of lambda_k exp(i Q.r) over each triangle (absolute coordinates). [nq, nf, 3]."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    fc = _Faces(verts, tris)
    return _vertex_moments(fc, q, tau_face)


def dft3d_dverts(verts, tris, q, tau_face: float = TAU_FACE) -> np.ndarray:
    """Jacobian dF(Q)/dv_k for every Q and vertex. [nq, nv, 3] complex (small inputs only)."""
    v = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    t = v.mean(axis=0)
    fc = _Faces(v - t, tris)
    B = _vertex_moments(fc, q, tau_face) * np.exp(1j * (q @ t))[:, None, None]
    out = np.zeros((q.shape[0], v.shape[0], 3), dtype=np.complex128)
    for k in range(3):
        contrib = B[:, :, k][:, :, None] * fc.nhat[None, :, :]      # n_m B_{m,k}
        for comp in range(3):
            np.add.at(out[:, :, comp], (slice(None), tris[:, k]), contrib[:, :, comp])
    return out


def _grad_faces(fc, tris, q, grad_out, t, tau_face, face_sel=None):
    """Per-face, per-corner real weights R_{m,k} = Re sum_Q conj(g_Q) B_{m,k}(Q) / |N_m|."""
    nf = fc.N.shape[0]
    Rw = np.zeros((nf, 3))
    go = np.asarray(grad_out, dtype=np.complex128).reshape(-1)
    for s, e in _blocks(q.shape[0], nf):
        qq = q[s:e]
        B = _vertex_moments(fc, qq, tau_face) * np.exp(1j * (qq @ t))[:, None, None]
        Rw += np.real(np.einsum("q,qfk->fk", np.conj(go[s:e]), B))
    return Rw


def _sub_faces(fc: _Faces, sel):
    sub = _Faces.__new__(_Faces)
    sub.v = [x[sel] for x in fc.v]
    sub.N, sub.nN, sub.ok, sub.nhat, sub.g = fc.N[sel], fc.nN[sel], fc.ok[sel], fc.nhat[sel], fc.g[sel]
    sub.d = [x[sel] for x in fc.d]
    sub.m = [x[sel] for x in fc.m]
    sub.L = fc.L[sel]
    return sub


def grad3d(verts, tris, q, grad_out, tau_face: float = TAU_FACE) -> np.ndarray:
    """dL/dv [nv, 3] for a real loss L with grad_out(Q) = dL/dReF(Q) + i dL/dImF(Q).

    dL/dv_k = sum_Q Re(conj(grad_out(Q)) dF(Q)/dv_k), dF/dv_k = sum_{m ∋ k} n_m B_{m,k}(Q).
    Parity pins: central finite differences of ``ft3d``; dV/dv_k = sum_m N_m/6 at Q = 0;
    the translation identity sum_k dF/dv_k = i Q F.
    """
    v = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    t = v.mean(axis=0)
    fc = _Faces(v - t, tris)
    Rw = _grad_faces(fc, tris, q, grad_out, t, tau_face)
    out = np.zeros((v.shape[0], 3))
    for k in range(3):
        np.add.at(out, tris[:, k], fc.nhat * Rw[:, k][:, None])
    return out


def grad3d_vertices(verts, tris, q, grad_out, vids, tau_face: float = TAU_FACE) -> np.ndarray:
    """dL/dv for the selected vertices only (faces incident to them). [len(vids), 3]."""
    v = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    vids = np.asarray(vids, dtype=np.int64)
    t = v.mean(axis=0)
    fc = _Faces(v - t, tris)
    sel = np.nonzero(np.isin(tris, vids).any(axis=1))[0]
    sub = _sub_faces(fc, sel)
    Rw = _grad_faces(sub, tris[sel], q, grad_out, t, tau_face)
    out = np.zeros((vids.size, 3))
    pos = {int(x): i for i, x in enumerate(vids)}
    for j, m in enumerate(sel):
        for k in range(3):
            i = pos.get(int(tris[m, k]))
            if i is not None:
                out[i] += sub.nhat[j] * Rw[j, k]
    return out


# ----------------------------------------------------------------------------
# 3D gradient with respect to Q
# ----------------------------------------------------------------------------
def ft3d_dq(verts, tris, q, tau_face: float = TAU_FACE, tau_dq: float = TAU_DQ) -> np.ndarray:
    """grad_Q F(Q) = i * volume integral of r exp(i Q.r) inside a closed outward mesh. [nq, 3] complex.

    Not in the paper; it follows from the same divergence theorem. With the field
    x_a (-i Q / Q^2) exp(i Q.r), whose divergence is x_a exp(i Q.r) - i Q_a exp(i Q.r) / Q^2,
        integral of r exp(i Q.r) dV = sum_m (-i Q.n_m / Q^2) integral over m of r exp(i Q.r) dA
                                      + (i Q / Q^2) F(Q),
    and r is linear on a face (r = sum_k lambda_k r_k), so the face integral is
    sum_k r_k B_{m,k}(Q) with the barycentric moments B of ``_vertex_moments``. Hence, in
    coordinates centred on the vertex mean t,
        grad F_c = sum_m (Q.n_m / Q^2) sum_k r_{m,k} B_{m,k} - (Q / Q^2) F_c,
        grad F   = exp(i Q.t) (grad F_c + i t F_c).
    |Q| R < tau_dq (the two terms cancel as (|Q| R)^-3 there) and Q = 0: the tetrahedra
    (t, a, b, c), whose barycentric moments are 6|T| sum_n i^n h_n(0, f_a, f_b, f_c, f_k)/(n+4)!
    (node k doubled, f = Q.(v - t)), so grad F_c = i sum_T sum_k r_k times that moment.
    Parity pins: separable closed form of a box's derivative, collapsed Gauss-Legendre
    quadrature of r exp(i Q.r) on a tetrahedron, the matrix-exponential tetrahedron fan with
    a doubled node, central differences of ``ft3d`` in Q, grad F(0) = i V x centroid, and the
    scaling identity Q.grad_Q F = sum_k v_k.dF/dv_k - 3F.
    """
    v = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    t = v.mean(axis=0)
    r = v - t
    fc = _Faces(r, tris)
    R = float(np.max(np.linalg.norm(r, axis=1)))
    nq = q.shape[0]
    gF = np.zeros((nq, 3), dtype=np.complex128)
    Fc = np.zeros(nq, dtype=np.complex128)
    Q2 = np.sum(q * q, axis=1)
    small = np.sqrt(Q2) * R < tau_dq
    a, b, c = fc.v
    if np.any(small):
        qs = q[small]
        idx = np.nonzero(small)[0]
        vol6 = np.einsum("ij,ij->i", a, fc.N)  # 6 x signed volume of (t, a, b, c)
        for s, e in _blocks(qs.shape[0], a.shape[0]):
            qq = qs[s:e]
            ph = [np.zeros((e - s, a.shape[0])), qq @ a.T, qq @ b.T, qq @ c.T]
            Fc[idx[s:e]] = np.sum(vol6[None, :] * simplex_exp_series(ph, dim=3), axis=1)
            acc = np.zeros((e - s, 3), dtype=np.complex128)
            for k, vk in enumerate((a, b, c)):
                mom = vol6[None, :] * simplex_exp_series(ph + [ph[k + 1]], dim=4)
                acc += mom @ vk
            gF[idx[s:e]] = 1j * acc
    gen = ~small
    if np.any(gen):
        qg = q[gen]
        idx = np.nonzero(gen)[0]
        for s, e in _blocks(qg.shape[0], a.shape[0]):
            qq = qg[s:e]
            q2 = Q2[idx[s:e]]
            B = _vertex_moments(fc, qq, tau_face)                   # [nq, nf, 3]
            qn = qq @ fc.nhat.T                                     # Q.n_m
            Fc[idx[s:e]] = np.sum(-1j * qn * np.sum(B, axis=2), axis=1) / q2
            surf = np.zeros((e - s, 3), dtype=np.complex128)
            for k, vk in enumerate((a, b, c)):
                surf += (qn * B[:, :, k]) @ vk
            gF[idx[s:e]] = surf / q2[:, None] - qq * (Fc[idx[s:e]] / q2)[:, None]
    ph_t = np.exp(1j * (q @ t))
    return ph_t[:, None] * (gF + 1j * t[None, :] * Fc[:, None])


# ----------------------------------------------------------------------------
# Piecewise-constant density over closed regions
# ----------------------------------------------------------------------------
def _regions(region_offsets, nf):
    off = [int(x) for x in region_offsets]
    if not off or off[0] != 0 or off[-1] != nf or any(off[i + 1] < off[i] for i in range(len(off) - 1)):
        raise ValueError("region_offsets must rise from 0 to the number of triangles")
    return [(off[j], off[j + 1]) for j in range(len(off) - 1)]


def ft3d_regions(verts, tris, region_offsets, rho, q):
    """F(Q) = sum_j rho_j F_j(Q) for a density rho_j constant on closed region j, whose outward
    boundary is triangles region_offsets[j] .. region_offsets[j+1]. Returns (F [nq], F_j [nreg, nq]).

    Plain definition: the integral of rho(r) exp(i Q.r) is the density-weighted sum of the
    regions' transforms (``ft3d`` of each region's boundary). A face shared by two regions
    appears once in each, with opposite orientations.
    Parity pins: a box cut into two boxes of equal density equals the whole box; a box inside
    a box (core and shell) against the separable closed forms.
    """
    tris = np.asarray(tris, dtype=np.int64)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    rho = np.asarray(rho, dtype=np.float64).reshape(-1)
    regs = _regions(region_offsets, tris.shape[0])
    if rho.size != len(regs):
        raise ValueError("one density per region")
    Fj = np.stack([ft3d(verts, tris[s:e], q) if e > s else np.zeros(q.shape[0], dtype=np.complex128)
                   for s, e in regs]) if regs else np.zeros((0, q.shape[0]), dtype=np.complex128)
    return (rho[:, None] * Fj).sum(axis=0), Fj


def grad3d_regions(verts, tris, region_offsets, rho, q, grad_out):
    """Gradients of a real loss L(F) with F = sum_j rho_j F_j, given grad_out = dL/dReF + i dL/dImF:
        dL/dv      = sum_j rho_j grad3d(region j)                    [nv, 3]
        dL/drho_j  = sum_Q Re(conj(grad_out) F_j)                   [nreg]
        dL/dQ      = Re(conj(grad_out) sum_j rho_j grad_Q F_j)      [nq, 3]
    """
    v = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    rho = np.asarray(rho, dtype=np.float64).reshape(-1)
    go = np.asarray(grad_out, dtype=np.complex128).reshape(-1)
    regs = _regions(region_offsets, tris.shape[0])
    gv = np.zeros((v.shape[0], 3))
    gr = np.zeros(len(regs))
    gq = np.zeros((q.shape[0], 3), dtype=np.complex128)
    for j, (s, e) in enumerate(regs):
        if e == s:
            continue
        tj = tris[s:e]
        gv += rho[j] * grad3d(v, tj, q, go)
        gr[j] = float(np.sum(np.real(np.conj(go) * ft3d(v, tj, q))))
        gq += rho[j] * ft3d_dq(v, tj, q)
    return gv, gr, np.real(np.conj(go)[:, None] * gq)


# ----------------------------------------------------------------------------
# Orientation average of the intensity (the scattering quantity of the paper's
# introduction: a randomly oriented particle scatters <|F(Q)|^2> over directions)
# ----------------------------------------------------------------------------
def orientation_average(verts, tris, qabs, dirs, weights) -> np.ndarray:
    """I(q_i) = sum_j w_j |F(q_i s_j)|^2 for the direction quadrature (s_j, w_j). [nqa] float64.

    Plain definition: the transform of ``ft3d`` at every (magnitude, direction)
    pair, squared in modulus and summed with the weights.
    Parity pins: Guinier's small-q law I = V^2 (1 - q^2 Rg^2 / 3 + O(q^4)) with V
    and Rg from closed-form tetrahedron moments; the same quadrature applied to
    the closed-form transform of a box; convergence of icosphere meshes to the
    sphere's |F|^2.
    """
    qabs = np.asarray(qabs, dtype=np.float64).reshape(-1)
    dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    weights = np.asarray(weights, dtype=np.float64).reshape(-1)
    out = np.zeros(qabs.shape[0])
    for i, q in enumerate(qabs):
        F = ft3d(verts, tris, q * dirs)
        out[i] = float(np.sum(weights * np.abs(F) ** 2))
    return out

