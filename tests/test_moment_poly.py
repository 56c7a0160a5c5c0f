"""The fitted polynomials of exp(ix) behind the binary32 adjoint's barycentric moments
(csrc/moment_poly.h): each one's error on its phase range, the bound that error puts on the
moments of a triangle (3D section, the face integrals of the vertex gradient), and that the
header is what its generator writes."""
import math
import os
import re
import subprocess
import sys

import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2104_08309_amd", "csrc")


def _header():
    with open(os.path.join(CSRC, "moment_poly.h")) as fh:
        return fh.read()


def _polys():
    src = _header()
    out = []
    pat = (r"static constexpr float M = ([0-9.]+)f;\s+static constexpr int N = (\d+);\s+"
           r"static constexpr float cj\[N \+ 1\] = \{([^}]*)\};\s+static constexpr float cy\[N \+ 1\] = \{([^}]*)\};")
    for m in re.finditer(pat, src):
        vals = lambda g: np.array([float(x.strip().rstrip("f")) for x in g.split(",")], np.float64)
        out.append((float(m.group(1)), int(m.group(2)), vals(m.group(3)), vals(m.group(4))))
    err = float(re.search(r"kMomentPolyErr = ([0-9.e+-]+);", src).group(1))
    count = int(re.search(r"kMomentPolyBuckets = (\d+);", src).group(1))
    assert len(out) == count
    return out, err


def _exact(d0, d1, nmax=60):
    """Barycentric moments of the simplex from the Taylor series to convergence (binary64)."""
    d2 = -d0 - d1
    e2 = d0 * d1 + d2 * (d0 + d1)
    e3 = d0 * d1 * d2
    H = [1.0, 0.0, -e2, e3]
    for n in range(4, nmax + 1):
        H.append(-e2 * H[n - 2] + e3 * H[n - 3])
    a0, a1 = [1.0], [1.0]
    for n in range(1, nmax + 1):
        a0.append(H[n] + d0 * a0[-1])
        a1.append(H[n] + d1 * a1[-1])
    J = sum((1j ** n) * H[n] / math.factorial(n + 2) for n in range(nmax + 1))
    Y0 = sum((1j ** n) * a0[n] / math.factorial(n + 3) for n in range(nmax + 1))
    Y1 = sum((1j ** n) * a1[n] / math.factorial(n + 3) for n in range(nmax + 1))
    return J, Y0, Y1


def _quadrature(d, f):
    """Simplex average of f(phi) with phi = lambda . d by a dense barycentric grid (for the
    closed-form check of the moments, independent of the series)."""
    n = 400
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = i + j < n
    l0 = (i[keep] + 1.0 / 3.0) / n
    l1 = (j[keep] + 1.0 / 3.0) / n
    # lower triangles of the grid (centroids) and upper ones
    up = i[keep] + j[keep] < n - 1
    u0 = (i[keep][up] + 2.0 / 3.0) / n
    u1 = (j[keep][up] + 2.0 / 3.0) / n
    L0 = np.concatenate([l0, u0])
    L1 = np.concatenate([l1, u1])
    L2 = 1.0 - L0 - L1
    phi = L0 * d[0] + L1 * d[1] + L2 * d[2]
    w = 0.5 / len(phi)
    return [np.sum(f(phi)) * w, np.sum(L0 * f(phi)) * w, np.sum(L1 * f(phi)) * w]


def test_buckets_cover_the_series_branch():
    polys, _ = _polys()
    Ms = [p[0] for p in polys]
    assert Ms == sorted(Ms) and len(set(Ms)) == len(Ms)
    with open(os.path.join(CSRC, "pft_internal.h")) as fh:
        smax = float(re.search(r"#define PFT_SERIES_MAX_PHASE ([0-9.]+)", fh.read()).group(1))
    assert Ms[-1] >= smax
    for M in Ms:
        assert float(np.float32(M)) == M  # the lanes compare binary32 phases with M exactly


def test_polynomials_fit_exp_on_their_range():
    polys, eps = _polys()
    for M, N, cj, cy in polys:
        n = np.arange(N + 1)
        fact = np.array([math.factorial(k) for k in range(N + 4)], np.float64)
        aj = cj * fact[n + 2] / fact[n]
        ay = cy * fact[n + 3] / fact[n]
        # both tables come from one set of coefficients a_n (each rounded to binary32 once)
        np.testing.assert_allclose(aj, ay, rtol=2e-7)
        x = np.linspace(-M, M, 40001)
        q = sum((1j ** k) * aj[k] * x ** k for k in range(N + 1))
        assert np.max(np.abs(q - np.exp(1j * x))) <= eps, M


def test_moment_error_within_the_bound():
    """J within eps/2 and Y_k within eps/6 for triangles whose largest centred phase is at
    most M (phases of random triangles scaled to the bucket edges)."""
    polys, eps = _polys()
    rng = np.random.default_rng(7)
    for M, N, cj, cy in polys:
        worst_j = worst_y = 0.0
        for t in range(60):
            d = rng.normal(size=3)
            d -= d.mean()
            d *= M / np.max(np.abs(d)) * (1.0 if t % 3 == 0 else rng.uniform(0.2, 1.0))
            d0, d1 = d[0], d[1]
            d2 = -d0 - d1
            e2 = d0 * d1 + d2 * (d0 + d1)
            e3 = d0 * d1 * d2
            H = [1.0, 0.0, -e2, e3]
            for k in range(4, N + 1):
                H.append(-e2 * H[k - 2] + e3 * H[k - 3])
            a0, a1 = [1.0], [1.0]
            for k in range(1, N + 1):
                a0.append(H[k] + d0 * a0[-1])
                a1.append(H[k] + d1 * a1[-1])
            J = sum((1j ** k) * cj[k] * H[k] for k in range(N + 1))
            Y0 = sum((1j ** k) * cy[k] * a0[k] for k in range(N + 1))
            Y1 = sum((1j ** k) * cy[k] * a1[k] for k in range(N + 1))
            EJ, EY0, EY1 = _exact(d0, d1)
            worst_j = max(worst_j, abs(J - EJ))
            worst_y = max(worst_y, abs(Y0 - EY0), abs(Y1 - EY1))
        assert worst_j <= eps / 2 and worst_y <= eps / 6, (M, worst_j, worst_y)


def test_face_polynomial():
    """The forward's near-degenerate face integral: the fit on [-M, M] and J within err/2 of the
    converged series for triangles whose largest centred phase is at most M."""
    src = _header()
    m = re.search(r"struct FacePoly \{\s+static constexpr float M = ([0-9.]+)f;\s+static constexpr int N = (\d+);\s+"
                  r"static constexpr float cj\[N \+ 1\] = \{([^}]*)\};", src)
    M, N = float(m.group(1)), int(m.group(2))
    cj = np.array([float(x.strip().rstrip("f")) for x in m.group(3).split(",")], np.float64)
    eps = float(re.search(r"kFacePolyErr = ([0-9.e+-]+);", src).group(1))
    n = np.arange(N + 1)
    a = cj * np.array([math.factorial(k + 2) / math.factorial(k) for k in n])
    x = np.linspace(-M, M, 40001)
    q = sum((1j ** k) * a[k] * x ** k for k in range(N + 1))
    assert np.max(np.abs(q - np.exp(1j * x))) <= eps
    rng = np.random.default_rng(8)
    worst = 0.0
    for t in range(60):
        d = rng.normal(size=3)
        d -= d.mean()
        d *= M / np.max(np.abs(d)) * (1.0 if t % 3 == 0 else rng.uniform(0.05, 1.0))
        e2 = d[0] * d[1] + d[2] * (d[0] + d[1])
        e3 = d[0] * d[1] * d[2]
        H = [1.0, 0.0, -e2, e3]
        for k in range(4, N + 1):
            H.append(-e2 * H[k - 2] + e3 * H[k - 3])
        J = sum((1j ** k) * cj[k] * H[k] for k in range(N + 1))
        worst = max(worst, abs(J - _exact(d[0], d[1])[0]))
    assert worst <= eps / 2, worst


def test_exact_moments_against_quadrature():
    """The series the bound is measured against is the simplex average itself."""
    for d in ([0.4, -1.1, 0.7], [2.0, -0.5, -1.5], [0.0, 0.0, 0.0]):
        d = np.array(d)
        E = _exact(d[0], d[1])
        Qd = _quadrature(d, lambda p: np.exp(1j * p))
        for a, b in zip(E, Qd):
            assert abs(a - b) < 2e-5


def test_header_is_the_generator_output():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_moment_poly.py")], capture_output=True,
                         text=True, check=True).stdout
    assert out.strip() == _header().strip()
