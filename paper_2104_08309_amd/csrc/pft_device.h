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

// sin(2 pi x), cos(2 pi x) for x in turns (hardware transcendental unit; valid for |x| <= 256).
__device__ __forceinline__ float sin_turns(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_turns(float x) { return __builtin_amdgcn_cosf(x); }
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

// sin(2 pi x) / x for x in turns, i.e. 2 pi sinc(2 pi x). At the removable point
// x = 0 the product is 0 * inf = NaN, and the IEEE minimum with 2 pi (which
// returns the non-NaN operand) yields the limit 2 pi; elsewhere the quotient is
// at most 2 pi, so the minimum leaves it unchanged.
__device__ __forceinline__ float sinc2pi_turns(float x) { return fminf(sin_turns(x) * rcp_f(x), kTwoPiF); }

// Complete homogeneous series with centred arguments (d0 + d1 + d2 = 0):
// sum_{n>=0} i^n h_n(d0, d1, d2) / (n + 2)!, binary64, terms added until they
// fall below 1e-17 of the partial sum (at most 80 terms).
// h_n obeys h_n = -e2 h_{n-2} + e3 h_{n-3} (generating function
// 1 / prod(1 - d_k t) = 1 / (1 + e2 t^2 - e3 t^3) when e1 = 0).
PFT_HD inline void face_series_f64(double d0, double d1, double d2, double& sr, double& si) {
  const double e2 = d0 * d1 + d0 * d2 + d1 * d2;
  const double e3 = d0 * d1 * d2;
  const double m = fmax(fabs(d0), fmax(fabs(d1), fabs(d2)));
  double hm3 = 0.0, hm2 = 1.0, hm1 = 0.0;  // h_{n-3}, h_{n-2}, h_{n-1} at n = 2
  double inv = 1.0 / 24.0;                 // 1/(n+2)! at n = 2
  sr = 0.5;
  si = 0.0;
  double mn = m * m;  // m^n; m^n (n+1)(n+2)/2 / (n+2)! bounds |h_n| / (n+2)!
  for (int n = 2; n < 80; ++n) {
    const double h = -e2 * hm2 + e3 * hm3;
    const double term = h * inv;
    switch (n & 3) {
      case 0: sr += term; break;
      case 1: si += term; break;
      case 2: sr -= term; break;
      default: si -= term; break;
    }
    hm3 = hm2;
    hm2 = hm1;
    hm1 = h;
    const double bound = mn * 0.5 * (n + 1) * (n + 2) * inv;
    if (n >= 4 && bound < 1e-17 * (fabs(sr) + fabs(si))) break;
    mn *= m;
    inv /= (double)(n + 3);
  }
}

// Simplex series of a tetrahedron with one vertex at the origin:
// sum_n i^n h_n(x_a, x_b, x_c) / (n + 3)!, binary64, with
// h_n = e1 h_{n-1} - e2 h_{n-2} + e3 h_{n-3}.
PFT_HD inline void tet_series_f64(double xa, double xb, double xc, double& sr, double& si) {
  const double e1 = xa + xb + xc;
  const double e2 = xa * xb + xa * xc + xb * xc;
  const double e3 = xa * xb * xc;
  const double m = fmax(fabs(xa), fmax(fabs(xb), fabs(xc)));
  double hm3 = 0.0, hm2 = 0.0, hm1 = 1.0;  // h_{n-3}, h_{n-2}, h_{n-1} at n = 1
  double inv = 1.0 / 24.0;                 // 1/(n+3)! at n = 1
  sr = 1.0 / 6.0;
  si = 0.0;
  double mn = 1.0;
  for (int n = 1; n < 80; ++n) {
    const double h = e1 * hm1 - e2 * hm2 + e3 * hm3;
    const double term = h * inv;
    switch (n & 3) {
      case 0: sr += term; break;
      case 1: si += term; break;
      case 2: sr -= term; break;
      default: si -= term; break;
    }
    hm3 = hm2;
    hm2 = hm1;
    hm1 = h;
    mn *= m;
    const double bound = mn * 0.5 * (n + 1) * (n + 2) * inv;
    if (n >= 3 && bound < 1e-17 * (fabs(sr) + fabs(si))) break;
    inv /= (double)(n + 4);
  }
}

// Contribution N.a * series of the tetrahedron (t, a, b, c) for a small-|Q| lane.
PFT_HD __forceinline__ void tet_term_f64(const Face64& F, const double* Q, double& xr, double& xi) {
  double a[3], b[3], c[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = F.g[k] + F.u0[k];
    b[k] = F.g[k] + F.u1[k];
    c[k] = F.g[k] - F.u0[k] - F.u1[k];
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
