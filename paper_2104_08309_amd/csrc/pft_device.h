// Device-side building blocks shared by the forward, adjoint and batched
// kernels: Q loading, turn-based sine / cosine, sinc, and the per-(Q, face)
// evaluations of the transform in its edge-sum and series forms.
//
// Notation (per triangle a, b, c, counter-clockwise seen from outside):
//   N = (b - a) x (c - a) = 2 A n,  g = (a + b + c)/3,  u_k = v_k - g,
//   d_l = v_{l+1} - v_l (edges),  m_l = (v_l + v_{l+1})/2 (edge midpoints),
//   P = Q x N,  psi_k = Q.u_k / 2,  eta_l = Q.d_l / 2 = psi_{l+1} - psi_l.
// Since m_l - g = -u_{l+2}/2, the edge phase relative to the face origin is
// exp(-i psi_{l+2}).
//
// Per face, the divergence theorem gives the flux term (3D section of the
// paper: eq. single_area_integral with the in-plane integral from the 2D
// edge formula in its midpoint / sinc form, outward in-plane edge normal):
//   T_m(Q) = |Q|^2 I_m = (Q.N)/|P|^2 exp(i Q.g) S_m,
//   S_m = sum_l (P.d_l) sinc(eta_l) exp(-i psi_{l+2}),
// and F(Q) = exp(i Q.t) sum_m T_m / |Q|^2 for a mesh re-centred on t.
// Where |P| -> 0 (Q along the face normal) the edge form is 0/0; there the
// face integral is evaluated by its simplex series
//   T_m = -i (Q.N) exp(i Q.g) sum_n i^n h_n(delta_a, delta_b, delta_c)/(n+2)!,
// delta_k = Q.u_k, h_n the complete homogeneous symmetric polynomial.
#pragma once

#include "pft_internal.h"

// binary64 building blocks are also compiled for the host (CPU unit checks of the device math)
#define PFT_HD __host__ __device__

namespace pft {

constexpr float kTwoPiF = 6.28318530717958647692f;
constexpr float kInv2PiF = 0.15915494309189533577f;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kInv2PiD = 0.15915494309189533577;

PFT_HD __forceinline__ void load_q3(const void* q, int qdtype, int64_t i, double* Q) {
  if (qdtype == PFT_F64) {
    const double* p = static_cast<const double*>(q) + 3 * i;
    Q[0] = p[0];
    Q[1] = p[1];
    Q[2] = p[2];
  } else {
    const float* p = static_cast<const float*>(q) + 3 * i;
    Q[0] = (double)p[0];
    Q[1] = (double)p[1];
    Q[2] = (double)p[2];
  }
}

// Cotangent of F relative to a mesh re-centred on t: the face integrals of the
// centred mesh carry exp(-iQ.t) relative to the absolute ones, so
// conj(g) B_abs = conj(g exp(-iQ.t)) B_centred. Returns g exp(-iQ.t).
PFT_HD __forceinline__ void centred_cotangent(double gr, double gi, const double* Q, const double* t, double& hr,
                                              double& hi) {
  double st, ct;
  sincos(Q[0] * t[0] + Q[1] * t[1] + Q[2] * t[2], &st, &ct);
  hr = gr * ct + gi * st;
  hi = gi * ct - gr * st;
}

// Partial sums written by one kernel and read once by the next: streaming
// (non-temporal) accesses keep them from displacing the face records in L2.
__device__ __forceinline__ void store_stream(double2* p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
__device__ __forceinline__ double2 load_stream(const double2* p) {
  return make_double2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}

// Sum of the forward's binary64 partials (one per face split) of the visited Q number qi, in split order.
__device__ __forceinline__ void fwd_partial_sum(const FwdArgs& a, int64_t qi, double& xr, double& xi) {
  xr = xi = 0.0;
  for (int s = 0; s < a.splits; ++s) {
    const double2 v = load_stream(a.partial + (int64_t)s * a.nq + qi);
    xr += v.x;
    xi += v.y;
  }
}

// sin(2 pi x), cos(2 pi x) for x in turns (hardware transcendental unit; valid for |x| <= 256).
__device__ __forceinline__ float sin_turns(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_turns(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

// sin(2 pi x) / x for x in turns, i.e. 2 pi sinc(2 pi x). At the removable point
// x = 0 the product is 0 * inf = NaN, and the IEEE minimum with 2 pi (which
// returns the non-NaN operand) yields the limit 2 pi; elsewhere the quotient is
// at most 2 pi, so the minimum leaves it unchanged.
__device__ __forceinline__ float sinc2pi_turns(float x) { return fminf(sin_turns(x) * rcp_f(x), kTwoPiF); }

// The same function as a polynomial in y = x^2 for |x| <= kSincPolyMax = 1/2 turn: the minimax fit of
// degree 5 in y (Remez exchange on the absolute error over y in [0, 1/4]; fit error 3.9e-7), with the
// coefficients rounded to binary32. Evaluated by Horner's rule in binary32 the error stays below 1e-6,
// i.e. 1.6e-7 of the value 2 pi at x = 0 -- the size of the hardware sine's own error divided by x -- with
// no transcendental instruction and no removable point. Beyond 1/2 turn the caller uses sinc2pi_turns.
constexpr float kSincPolyMax = 0.5f;
__device__ __forceinline__ float sinc2pi_poly(float x) {
  const float y = x * x;
  float p = fmaf(-12.473669052124023f, y, 41.344398498535156f);
  p = fmaf(p, y, -76.61480712890625f);
  p = fmaf(p, y, 81.5999755859375f);
  p = fmaf(p, y, -41.341590881347656f);
  return fmaf(p, y, 6.283185005187988f);
}
// sinc2pi_poly's value `c` at x where it applies, the sine-quotient form beyond.
__device__ __forceinline__ float sinc2pi_wide(float x, float c) {
  return fabsf(x) > kSincPolyMax ? sin_turns(x) * rcp_f(x) : c;
}

// 1/n! for n = 0..95, correctly rounded binary64 (device constant memory; a
// host copy for host builds of the binary64 math).
#define PFT_INV_FACT_VALUES \
    1.0, 1.0, 0.5, 0.16666666666666666, 0.041666666666666664, 0.008333333333333333, 0.001388888888888889, \
    0.0001984126984126984, 2.48015873015873e-05, 2.7557319223985893e-06, 2.755731922398589e-07, \
    2.505210838544172e-08, 2.08767569878681e-09, 1.6059043836821613e-10, 1.1470745597729725e-11, \
    7.647163731819816e-13, 4.779477332387385e-14, 2.8114572543455206e-15, 1.5619206968586225e-16, \
    8.22063524662433e-18, 4.110317623312165e-19, 1.9572941063391263e-20, 8.896791392450574e-22, \
    3.868170170630684e-23, 1.6117375710961184e-24, 6.446950284384474e-26, 2.4795962632247976e-27, \
    9.183689863795546e-29, 3.279889237069838e-30, 1.1309962886447716e-31, 3.7699876288159054e-33, \
    1.216125041553518e-34, 3.8003907548547434e-36, 1.151633562077195e-37, 3.387157535521162e-39, \
    9.67759295863189e-41, 2.6882202662866363e-42, 7.265460179153071e-44, 1.911963205040282e-45, \
    4.902469756513544e-47, 1.2256174391283858e-48, 2.9893108271424046e-50, 7.117406731291439e-52, \
    1.6552108677421951e-53, 3.7618428812322616e-55, 8.359650847182804e-57, 1.817315401561479e-58, \
    3.866628513960594e-60, 8.055476070751236e-62, 1.643974708316579e-63, 3.287949416633158e-65, \
    6.446959640457172e-67, 1.2397999308571486e-68, 2.3392451525606576e-70, 4.331935467704922e-72, \
    7.876246304918039e-74, 1.4064725544496498e-75, 2.4674957095607893e-77, 4.254302947518602e-79, \
    7.2106829618959365e-81, 1.2017804936493226e-82, 1.9701319568021682e-84, 3.1776321883905942e-86, \
    5.043860616493007e-88, 7.881032213270323e-90, 1.2124664943492804e-91, 1.8370704459837581e-93, \
    2.74189618803546e-95, 4.0322002765227353e-97, 5.843768516699616e-99, 8.34824073814231e-101, \
    1.1758085546679308e-102, 1.633067437038793e-104, 2.2370786808750587e-106, 3.023079298479809e-108, \
    4.030772397973079e-110, 5.30364789206984e-112, 6.887854405285506e-114, 8.830582570878855e-116, \
    1.117795262136564e-117, 1.397244077670705e-119, 1.7249926884823517e-121, 2.103649620100429e-123, \
    2.53451761457883e-125, 3.0172828744986073e-127, 3.5497445582336554e-129, 4.127609951434483e-131, \
    4.7443792545223946e-133, 5.3913400619572666e-135, 6.057685462873333e-137, 6.730761625414815e-139, \
    7.396441346609687e-141, 8.039610159358355e-143, 8.64474210683694e-145, 9.196534156209511e-147, \
    9.680562269694223e-149
constexpr int kInvFactCount = 96;
__constant__ const double kInvFactD[kInvFactCount] = {PFT_INV_FACT_VALUES};
static const double kInvFactH[kInvFactCount] = {PFT_INV_FACT_VALUES};

PFT_HD __forceinline__ double inv_fact(int n) {
#if defined(__HIP_DEVICE_COMPILE__)
  return kInvFactD[n];
#else
  return kInvFactH[n];
#endif
}

// Complete homogeneous series with centred arguments (d0 + d1 + d2 = 0):
// sum_{n>=0} i^n h_n(d0, d1, d2) / (n + 2)!, binary64.
// h_n obeys h_n = -e2 h_{n-2} + e3 h_{n-3} (generating function
// 1 / prod(1 - d_k t) = 1 / (1 + e2 t^2 - e3 t^3) when e1 = 0). Terms are added
// four at a time (one of each power of i) until the bound m^n / (2 n!) on the
// next term, m = max |d_k| (|h_n| <= m^n (n+1)(n+2)/2), falls below `tol` times
// the partial sum, or n reaches 84.
PFT_HD inline void face_series_f64(double d0, double d1, double d2, double& sr, double& si, double tol) {
  const double e2 = d0 * d1 + d0 * d2 + d1 * d2;
  const double e3 = d0 * d1 * d2;
  const double m = fmax(fabs(d0), fmax(fabs(d1), fabs(d2)));
  const double m4 = (m * m) * (m * m);
  // n = 0..3: h = 1, 0, -e2, e3
  double h1 = 0.0, h2 = -e2, h3 = e3;  // h_{n-3}, h_{n-2}, h_{n-1} at n = 4
  sr = 0.5 - h2 * inv_fact(4);
  si = -h3 * inv_fact(5);
  double mn = m4;  // m^n
  for (int n = 4; n < 88; n += 4) {
    const double a = -e2 * h2 + e3 * h1;  // h_n
    const double b = -e2 * h3 + e3 * h2;  // h_{n+1}
    const double c = -e2 * a + e3 * h3;   // h_{n+2}
    const double d = -e2 * b + e3 * a;    // h_{n+3}
    sr += a * inv_fact(n + 2) - c * inv_fact(n + 4);
    si += b * inv_fact(n + 3) - d * inv_fact(n + 5);
    h1 = b;
    h2 = c;
    h3 = d;
    mn *= m4;
    if (mn * 0.5 * inv_fact(n + 4) < tol * (fabs(sr) + fabs(si))) break;
  }
}

// Simplex series of a tetrahedron with one vertex at the origin:
// sum_n i^n h_n(x_a, x_b, x_c) / (n + 3)!, binary64, with
// h_n = e1 h_{n-1} - e2 h_{n-2} + e3 h_{n-3}; four terms per step as above, until
// the bound m^n / (2 n!) on the next term falls below 1e-17 of the partial sum
// (n at most 89).
PFT_HD inline void tet_series_f64(double xa, double xb, double xc, double& sr, double& si) {
  const double e1 = xa + xb + xc;
  const double e2 = xa * xb + xa * xc + xb * xc;
  const double e3 = xa * xb * xc;
  const double m = fmax(fabs(xa), fmax(fabs(xb), fabs(xc)));
  const double m4 = (m * m) * (m * m);
  double h1 = 0.0, h2 = 0.0, h3 = 1.0;  // h_{n-3}, h_{n-2}, h_{n-1} at n = 1
  sr = 1.0 / 6.0;
  si = 0.0;
  double mn = m;  // m^n
  for (int n = 1; n < 89; n += 4) {
    const double a = e1 * h3 - e2 * h2 + e3 * h1;  // h_n     (i^n = i)
    const double b = e1 * a - e2 * h3 + e3 * h2;   // h_{n+1} (-1)
    const double c = e1 * b - e2 * a + e3 * h3;    // h_{n+2} (-i)
    const double d = e1 * c - e2 * b + e3 * a;     // h_{n+3} (+1)
    si += a * inv_fact(n + 3) - c * inv_fact(n + 5);
    sr += d * inv_fact(n + 6) - b * inv_fact(n + 4);
    h1 = b;
    h2 = c;
    h3 = d;
    mn *= m4;
    if (mn * 0.5 * inv_fact(n + 4) < 1e-17 * (fabs(sr) + fabs(si))) break;
  }
}

__device__ constexpr double kZeroOrigin[3] = {0.0, 0.0, 0.0};

// Contribution N.a * series of the tetrahedron (o, a, b, c) for a small-|Q| lane, o an apex given relative
// to the mesh centre t (the sum over a closed surface is then the volume integral of exp(iQ.(r - o))).
PFT_HD __forceinline__ void tet_term_f64(const Face64& F, const double* Q, double& xr, double& xi,
                                         const double* o) {
  double a[3], b[3], c[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = F.g[k] + F.u0[k] - o[k];
    b[k] = F.g[k] + F.u1[k] - o[k];
    c[k] = F.g[k] - F.u0[k] - F.u1[k] - o[k];
  }
  const double six_v = F.N[0] * a[0] + F.N[1] * a[1] + F.N[2] * a[2];
  const double xa = Q[0] * a[0] + Q[1] * a[1] + Q[2] * a[2];
  const double xb = Q[0] * b[0] + Q[1] * b[1] + Q[2] * b[2];
  const double xc = Q[0] * c[0] + Q[1] * c[1] + Q[2] * c[2];
  double sr, si;
  tet_series_f64(xa, xb, xc, sr, si);
  xr += six_v * sr;
  xi += six_v * si;
}

}  // namespace pft
