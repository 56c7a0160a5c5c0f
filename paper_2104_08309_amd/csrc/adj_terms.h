// Per-(Q, face) terms of the adjoint (barycentric moments of each face),
// binary64 and FP32-compensated forms, shared by the single-mesh and batched
// kernels. The formulas are stated at the top of bwd3d.hip.
#pragma once

#include "moment_poly.h"
#include "pft_device.h"

namespace pft {

// ---------------------------------------------------------------------------
// binary64
// ---------------------------------------------------------------------------
PFT_HD __forceinline__ double dsinc_series(double x) {
  // d/dx sin(x)/x = sum_k (-1)^k 2k x^(2k-1) / (2k+1)!, |x| < 0.5
  const double x2 = x * x;
  return x * (-1.0 / 3.0 + x2 * (1.0 / 30.0 + x2 * (-1.0 / 840.0 + x2 * (1.0 / 45360.0 +
             x2 * (-1.0 / 3991680.0 + x2 * (1.0 / 518918400.0))))));
}

// Barycentric moments of a triangle from its centred vertex phases
// d0 + d1 + d2 = 0 (d_k = Q.(v_k - g)):
//   Y_k = sum_n i^n h_n(d0, d1, d2, d_k) / (n+3)!   (k = 0, 1),
//   J   = sum_n i^n h_n(d0, d1, d2) / (n+2)!         (so Y_2 = J - Y_0 - Y_1),
// with H_n = h_n(d0, d1, d2) = -e2 H_{n-2} + e3 H_{n-3} and
// h_n(d0, d1, d2, d_k) = H_n + d_k h_{n-1}(d0, d1, d2, d_k). Terms are added four
// at a time until m^n / n! < tol (m = max |d_k|; the next term of Y is below
// (1/6) m^n / n!, of J below (1/2) m^n / n!), or n reaches NMAX. The loop is
// unrolled, so the factorial coefficients are compile-time constants folded into
// the instructions rather than values held in registers.
template <typename T>
PFT_HD constexpr T inv_fact_c(int n) {
  constexpr double t[kInvFactCount] = {PFT_INV_FACT_VALUES};
  return T(t[n]);
}

template <typename T, int NMAX>
PFT_HD __forceinline__ void bary_moments(T d0, T d1, T m, T tol, T* yr, T* yi, T& jr, T& ji) {
  const T d2 = -d0 - d1;
  const T e2 = d0 * d1 + d2 * (d0 + d1);
  const T e3 = d0 * d1 * d2;
  const T m2 = m * m, m4 = m2 * m2;
  // n = 1..4 written out: H_1 = 0, H_2 = -e2, H_3 = e3, H_4 = e2^2
  const T H2 = -e2, H3 = e3, H4 = e2 * e2;
  T a0 = d0, a1 = d1;  // h_{n}(d0,d1,d2,d0), h_{n}(d0,d1,d2,d1) at n = 1
  T y0i = inv_fact_c<T>(4) * a0, y1i = inv_fact_c<T>(4) * a1;
  a0 = H2 + d0 * a0;
  a1 = H2 + d1 * a1;
  T y0r = T(1.0 / 6.0) - inv_fact_c<T>(5) * a0, y1r = T(1.0 / 6.0) - inv_fact_c<T>(5) * a1;
  jr = T(0.5) - inv_fact_c<T>(4) * H2;
  a0 = H3 + d0 * a0;
  a1 = H3 + d1 * a1;
  y0i -= inv_fact_c<T>(6) * a0;
  y1i -= inv_fact_c<T>(6) * a1;
  ji = -inv_fact_c<T>(5) * H3;
  a0 = H4 + d0 * a0;
  a1 = H4 + d1 * a1;
  y0r += inv_fact_c<T>(7) * a0;
  y1r += inv_fact_c<T>(7) * a1;
  jr += inv_fact_c<T>(6) * H4;
  T Hm3 = H2, Hm2 = H3, Hm1 = H4;  // H_{n-3}, H_{n-2}, H_{n-1} at n = 5
  T mn = m * m4;                   // m^n at the start of each chunk
  if (!(mn * inv_fact_c<T>(5) < tol)) {
#pragma unroll
    for (int n = 5; n < NMAX; n += 4) {
      // i^n cycles (+i, -1, -i, +1) over n = 1, 2, 3, 4 (mod 4)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T H = -e2 * Hm2 + e3 * Hm3;
        a0 = H + d0 * a0;
        a1 = H + d1 * a1;
        const T c3 = inv_fact_c<T>(n + r + 3), c2 = inv_fact_c<T>(n + r + 2);
        if (r == 0) {
          y0i += c3 * a0; y1i += c3 * a1; ji += c2 * H;
        } else if (r == 1) {
          y0r -= c3 * a0; y1r -= c3 * a1; jr -= c2 * H;
        } else if (r == 2) {
          y0i -= c3 * a0; y1i -= c3 * a1; ji -= c2 * H;
        } else {
          y0r += c3 * a0; y1r += c3 * a1; jr += c2 * H;
        }
        Hm3 = Hm2;
        Hm2 = Hm1;
        Hm1 = H;
      }
      mn *= m4;
      if (mn * inv_fact_c<T>(n + 4) < tol) break;
    }
  }
  yr[0] = y0r; yi[0] = y0i;
  yr[1] = y1r; yi[1] = y1i;
}

// The same moments in binary32 from a polynomial q(x) = sum_n i^n a_n x^n of exp(ix)
// fitted on [-M, M] (moment_poly.h): J = sum_n i^n a_n n! H_n / (n+2)! and
// Y_k = sum_n i^n a_n n! h_n(d0, d1, d2, d_k) / (n+3)!, exact for q, so the error is
// the simplex average of q - exp(ix) at phases within [-M, M] (J within err/2, Y_k
// within err/6) for every lane with max |d_k| <= M. The degree is fixed by P.
template <class P>
__device__ __forceinline__ void bary_moments_poly(float d0, float d1, float* yr, float* yi, float& jr, float& ji) {
  static_assert(P::N >= 5, "the first five terms are written out");
  const float d2 = -d0 - d1;
  const float e2 = d0 * d1 + d2 * (d0 + d1);
  const float e3 = d0 * d1 * d2;
  // n = 0..4 written out: H_0 = 1, H_1 = 0, H_2 = -e2, H_3 = e3, H_4 = e2^2
  const float H2 = -e2, H3 = e3, H4 = e2 * e2;
  float a0 = d0, a1 = d1;  // h_1(d0,d1,d2,d_k) = d_k (H_1 = 0)
  float y0r = P::cy[0], y1r = P::cy[0];
  jr = P::cj[0];
  float y0i = P::cy[1] * a0, y1i = P::cy[1] * a1;
  a0 = H2 + d0 * a0;
  a1 = H2 + d1 * a1;
  y0r -= P::cy[2] * a0;
  y1r -= P::cy[2] * a1;
  jr -= P::cj[2] * H2;
  a0 = H3 + d0 * a0;
  a1 = H3 + d1 * a1;
  y0i -= P::cy[3] * a0;
  y1i -= P::cy[3] * a1;
  ji = -P::cj[3] * H3;
  a0 = H4 + d0 * a0;
  a1 = H4 + d1 * a1;
  y0r += P::cy[4] * a0;
  y1r += P::cy[4] * a1;
  jr += P::cj[4] * H4;
  float Hm3 = H2, Hm2 = H3, Hm1 = H4;  // H_{n-3}, H_{n-2}, H_{n-1} at n = 5
#pragma unroll
  for (int n = 5; n <= P::N; ++n) {
    const float H = -e2 * Hm2 + e3 * Hm3;
    a0 = H + d0 * a0;
    a1 = H + d1 * a1;
    const float c3 = P::cy[n], c2 = P::cj[n];
    // i^n cycles (+i, -1, -i, +1) over n = 1, 2, 3, 0 (mod 4)
    if ((n & 3) == 1) {
      y0i += c3 * a0; y1i += c3 * a1; ji += c2 * H;
    } else if ((n & 3) == 2) {
      y0r -= c3 * a0; y1r -= c3 * a1; jr -= c2 * H;
    } else if ((n & 3) == 3) {
      y0i -= c3 * a0; y1i -= c3 * a1; ji -= c2 * H;
    } else {
      y0r += c3 * a0; y1r += c3 * a1; jr += c2 * H;
    }
    Hm3 = Hm2;
    Hm2 = Hm1;
    Hm1 = H;
  }
  yr[0] = y0r; yi[0] = y0i;
  yr[1] = y1r; yi[1] = y1i;
}

// Binary32 moments for the lanes that take the series branch (max |d_k| = m <= 3):
// the wavefront takes the lowest-degree polynomial whose range covers the largest m
// among its active lanes (a wavefront-uniform choice, so no lane waits on another's
// branch), after at most three comparisons.
static_assert(kSeriesMaxPhase <= kMomentPolyMaxPhase, "the series branch must stay within the fitted range");
__device__ __forceinline__ void bary_moments_f32(float d0, float d1, float m, float* yr, float* yi, float& jr,
                                                 float& ji) {
  static_assert(kMomentPolyBuckets == 7, "the dispatch below names seven polynomials");
  if (__any(m > MomentPoly3::M)) {
    if (__any(m > MomentPoly5::M))
      bary_moments_poly<MomentPoly6>(d0, d1, yr, yi, jr, ji);
    else if (__any(m > MomentPoly4::M))
      bary_moments_poly<MomentPoly5>(d0, d1, yr, yi, jr, ji);
    else
      bary_moments_poly<MomentPoly4>(d0, d1, yr, yi, jr, ji);
  } else if (__any(m > MomentPoly1::M)) {
    if (__any(m > MomentPoly2::M))
      bary_moments_poly<MomentPoly3>(d0, d1, yr, yi, jr, ji);
    else
      bary_moments_poly<MomentPoly2>(d0, d1, yr, yi, jr, ji);
  } else {
    if (__any(m > MomentPoly0::M))
      bary_moments_poly<MomentPoly1>(d0, d1, yr, yi, jr, ji);
    else
      bary_moments_poly<MomentPoly0>(d0, d1, yr, yi, jr, ji);
  }
}

// Edge form of the barycentric moments (|Q.(v - g)| beyond the series range):
// the moment of corner k relative to exp(iQ.g), normalised by 2A, is
// X_k * inv with inv = 1/|P|^2 (P = Q x N), and S is the face's edge sum, so
// that X_0 + X_1 + X_2 = i S and the normalised face integral is i S inv. The
// moments come from the closed-form Q-derivative of the edge sum.
PFT_HD __forceinline__ void edge_moments_f64(const Face64& f, const double* G, const double* Q, double Px, double Py,
                                             double Pz, double q0, double q1, double inv, double* Xr, double* Xi,
                                             double& Sr, double& Si) {
  const double q2 = -q0 - q1;
  const double p0 = 0.5 * q0, p1 = 0.5 * q1, p2 = 0.5 * q2;
  double s0, c0, s1, c1;
  sincos(p0, &s0, &c0);
  sincos(p1, &s1, &c1);
  const double c2 = c0 * c1 - s0 * s1;
  const double s2 = -(s0 * c1 + c0 * s1);
  const double pi0 = Px * f.u0[0] + Py * f.u0[1] + Pz * f.u0[2];
  const double pi1 = Px * f.u1[0] + Py * f.u1[1] + Pz * f.u1[2];
  const double pi2 = -pi0 - pi1;
  const double w[3] = {pi1 - pi0, pi2 - pi1, pi0 - pi2};
  const double eta[3] = {p1 - p0, p2 - p1, p0 - p2};
  const double sn[3] = {s1 * c0 - c1 * s0, s2 * c1 - c2 * s1, s0 * c2 - c0 * s2};
  const double cs[3] = {c1 * c0 + s1 * s0, c2 * c1 + s2 * s1, c0 * c2 + s0 * s2};
  // e_l = exp(-i psi_{l+2})
  const double er[3] = {c2, c0, c1};
  const double ei[3] = {-s2, -s0, -s1};
  double ar[3], ai[3], br[3], bi[3], cr[3], ci[3];
  Sr = 0.0;
  Si = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double x = eta[l];
    double sg, dsg;
    if (fabs(x) < 0.1) {
      const double x2 = x * x;
      sg = 1.0 + x2 * (-1.0 / 6.0 + x2 * (1.0 / 120.0 + x2 * (-1.0 / 5040.0 + x2 * (1.0 / 362880.0))));
    } else {
      sg = sn[l] / x;
    }
    dsg = fabs(x) < 0.5 ? dsinc_series(x) : (cs[l] - sg) / x;
    cr[l] = sg * er[l];
    ci[l] = sg * ei[l];
    ar[l] = w[l] * cr[l];
    ai[l] = w[l] * ci[l];
    br[l] = w[l] * dsg * er[l];
    bi[l] = w[l] * dsg * ei[l];
    Sr += ar[l];
    Si += ai[l];
  }
  // Gram matrix of the edges, G = {d0.d0, d1.d1, d2.d2, d0.d1, d1.d2, d2.d0}
  const double Gm[3][3] = {{G[0], G[3], G[5]}, {G[3], G[1], G[4]}, {G[5], G[4], G[2]}};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int kp = (k + 1) % 3, km = (k + 2) % 3;
    double xr = -0.5 * Si, xi = 0.5 * Sr;  // (i/2) S
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      xr += Gm[kp][l] * cr[l];
      xi += Gm[kp][l] * ci[l];
    }
    xr += 0.5 * (br[km] - br[k]);
    xi += 0.5 * (bi[km] - bi[k]);
    xr += 0.5 * ai[kp];   // -(i/2) a_{k+1}
    xi -= 0.5 * ar[kp];
    const double s = 2.0 * w[kp] * inv;
    Xr[k] = xr - s * Sr;
    Xi[k] = xi - s * Si;
  }
}

PFT_HD __forceinline__ void adj_term_f64(const Face64& f, const double* G, const double* Q, double gr,
                                             double gi, double* R) {
  const double Px = Q[1] * f.N[2] - Q[2] * f.N[1];
  const double Py = Q[2] * f.N[0] - Q[0] * f.N[2];
  const double Pz = Q[0] * f.N[1] - Q[1] * f.N[0];
  const double P2 = Px * Px + Py * Py + Pz * Pz;
  const double phi = Q[0] * f.g[0] + Q[1] * f.g[1] + Q[2] * f.g[2];
  double sf, cf;
  sincos(phi, &sf, &cf);
  // z = conj(g) exp(i Q.g)
  const double zr = gr * cf + gi * sf;
  const double zi = gr * sf - gi * cf;
  const double q0 = Q[0] * f.u0[0] + Q[1] * f.u0[1] + Q[2] * f.u0[2];
  const double q1 = Q[0] * f.u1[0] + Q[1] * f.u1[1] + Q[2] * f.u1[2];
  const double q2 = -q0 - q1;
  if (f.thr < 0.0) {  // empty face
    R[0] = R[1] = R[2] = 0.0;
    return;
  }
  const double m = fmax(fabs(q0), fmax(fabs(q1), fabs(q2)));
  if (m <= kSeriesMaxPhase) {
    // barycentric moments by their series (no cancellation for |delta| <= 3)
    double yr[2], yi[2], jr, ji;
    bary_moments<double, 33>(q0, q1, m, 1e-17, yr, yi, jr, ji);
    R[0] = zr * yr[0] - zi * yi[0];
    R[1] = zr * yr[1] - zi * yi[1];
    R[2] = (zr * jr - zi * ji) - R[0] - R[1];
    return;
  }
  const double inv = 1.0 / P2;
  double Xr[3], Xi[3], Sr, Si;
  edge_moments_f64(f, G, Q, Px, Py, Pz, q0, q1, inv, Xr, Xi, Sr, Si);
#pragma unroll
  for (int k = 0; k < 3; ++k) R[k] = (zr * Xr[k] - zi * Xi[k]) * inv;
}

// ---------------------------------------------------------------------------
// FP32-compensated
// ---------------------------------------------------------------------------
// sin(x)/x for |x| < 1 (Taylor series to x^10)
__device__ __forceinline__ float sinc_series_f(float x) {
  const float x2 = x * x;
  return 1.0f + x2 * (-1.0f / 6.0f + x2 * (1.0f / 120.0f + x2 * (-1.0f / 5040.0f + x2 * (1.0f / 362880.0f +
         x2 * (-1.0f / 39916800.0f)))));
}

// d/dx sin(x)/x for |x| < 1 (Taylor series to x^11)
__device__ __forceinline__ float dsinc_series_f(float x) {
  const float x2 = x * x;
  return x * (-1.0f / 3.0f + x2 * (1.0f / 30.0f + x2 * (-1.0f / 840.0f + x2 * (1.0f / 45360.0f +
             x2 * (-1.0f / 3991680.0f + x2 * (1.0f / 518918400.0f))))));
}

// Edge form of the barycentric moments in binary32, as edge_moments_f64:
// moment k (normalised by 2A, relative to exp(iQ.g)) = X_k * inv, inv = 1/|P|^2,
// and the face integral i S inv. Sinc and its derivative use their Taylor
// series for |x| < 1 (the hardware sine loses relative accuracy at small
// arguments) and quotients beyond.
__device__ __forceinline__ void edge_moments_fp32c(const Face32B& f, float Px, float Py, float Pz, float q0, float q1,
                                                   float inv, float* Xr, float* Xi, float& Sr, float& Si) {
  const float w0 = Px * f.d0[0] + Py * f.d0[1] + Pz * f.d0[2];
  const float w1 = Px * f.d1[0] + Py * f.d1[1] + Pz * f.d1[2];
  const float w[3] = {w0, w1, -w0 - w1};
  const float p0 = q0 * (0.5f * kInv2PiF), p1 = q1 * (0.5f * kInv2PiF), p2 = -p0 - p1;  // psi_k in turns
  const float s0 = sin_turns(p0), c0 = cos_turns(p0);
  const float s1 = sin_turns(p1), c1 = cos_turns(p1);
  const float c2 = c0 * c1 - s0 * s1;
  const float s2 = -(s0 * c1 + c0 * s1);
  const float eta[3] = {p1 - p0, p2 - p1, p0 - p2};  // turns
  const float cs[3] = {c1 * c0 + s1 * s0, c2 * c1 + s2 * s1, c0 * c2 + s0 * s2};
  const float er[3] = {c2, c0, c1};
  const float ei[3] = {-s2, -s0, -s1};
  float ar[3], ai[3], br[3], bi[3], cr[3], ci[3];
  Sr = 0.0f;
  Si = 0.0f;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const float xt = eta[l];
    const float x = kTwoPiF * xt;                  // radians
    const float rx = rcp_f(xt) * kInv2PiF;         // 1/x
    const bool near0 = fabsf(x) < 1.0f;
    const float sg = near0 ? sinc_series_f(x) : sin_turns(xt) * rx;
    const float dsg = near0 ? dsinc_series_f(x) : (cs[l] - sg) * rx;
    cr[l] = sg * er[l];
    ci[l] = sg * ei[l];
    ar[l] = w[l] * cr[l];
    ai[l] = w[l] * ci[l];
    const float wd = w[l] * dsg;
    br[l] = wd * er[l];
    bi[l] = wd * ei[l];
    Sr += ar[l];
    Si += ai[l];
  }
  const float Gm[3][3] = {{f.G[0], f.G[3], f.G[5]}, {f.G[3], f.G[1], f.G[4]}, {f.G[5], f.G[4], f.G[2]}};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int kp = (k + 1) % 3, km = (k + 2) % 3;
    float xr = -0.5f * Si, xi = 0.5f * Sr;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      xr += Gm[kp][l] * cr[l];
      xi += Gm[kp][l] * ci[l];
    }
    xr += 0.5f * (br[km] - br[k]);
    xi += 0.5f * (bi[km] - bi[k]);
    xr += 0.5f * ai[kp];
    xi -= 0.5f * ar[kp];
    const float s = 2.0f * w[kp] * inv;
    Xr[k] = xr - s * Sr;
    Xi[k] = xi - s * Si;
  }
}

__device__ __forceinline__ void adj_term_fp32c(const Face32B& f, float qx, float qy, float qz, float Q2,
                                               const double* Qd, float gr, float gi, float* R) {
  const float N0 = f.N[0], N1 = f.N[1], N2 = f.N[2];
  const float Px = qy * N2 - qz * N1;
  const float Py = qz * N0 - qx * N2;
  const float Pz = qx * N1 - qy * N0;
  const float P2 = Px * Px + Py * Py + Pz * Pz;
  const double ph = Qd[0] * f.gt[0] + Qd[1] * f.gt[1] + Qd[2] * f.gt[2];
  const float r = (float)(ph - rint(ph));
  const float cf = cos_turns(r), sf = sin_turns(r);
  const float zr = gr * cf + gi * sf;
  const float zi = gr * sf - gi * cf;
  const float q0 = qx * f.u0[0] + qy * f.u0[1] + qz * f.u0[2];  // delta_k = Q.u_k
  const float q1 = qx * f.u1[0] + qy * f.u1[1] + qz * f.u1[2];
  const float q2 = -q0 - q1;
  const float m = fmaxf(fabsf(q0), fmaxf(fabsf(q1), fabsf(q2)));
  // (an empty face has an all-zero record: m = 0, finite weights, times N = 0 later)
  if (m <= (float)kSeriesMaxPhase) {
    // barycentric moments in binary32 from the fitted polynomial of exp(ix) (every
    // term is bounded for |delta| <= 3; no cancellation with the face's size in Q)
    float yr[2], yi[2], jr, ji;
    bary_moments_f32(q0, q1, m, yr, yi, jr, ji);
    R[0] = zr * yr[0] - zi * yi[0];
    R[1] = zr * yr[1] - zi * yi[1];
    R[2] = (zr * jr - zi * ji) - R[0] - R[1];
    return;
  }
  const float inv = rcp_f(fmaxf(P2, 1e-30f));
  float Xr[3], Xi[3], Sr, Si;
  edge_moments_fp32c(f, Px, Py, Pz, q0, q1, inv, Xr, Xi, Sr, Si);
#pragma unroll
  for (int k = 0; k < 3; ++k) R[k] = (zr * Xr[k] - zi * Xi[k]) * inv;
}

// ---------------------------------------------------------------------------
// Wavefront sum in binary64 (shuffles through the LDS crossbar).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a block of NT threads in binary64 and a fixed order; every thread
// must call it and every thread gets the total. lds holds NT / 64 doubles.
template <int NT>
__device__ __forceinline__ double block_total(double v, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_total(v);
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t += lds[w];
  return t;
}

// ---------------------------------------------------------------------------
// binary64 adjoint, one block's share: `nt` face records in LDS (with their
// edge Gram matrices) against the reordered Q records [qb, qe), kQPTB Q per
// thread per pass. Each thread adds its weights for face j to its own
// binary64 slots acc[3 j + k][thread] (zeroed by the caller); adj_block_sum
// reduces the slots once the range is done.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void adj_tile_f64(const Face64* tile, const double (*gtile)[8], int nt, int64_t qb,
                                             int64_t qe, const QRec64* __restrict__ rec, double (*acc)[kBlock]) {
  constexpr int P = kQPTB;
  const int tid = threadIdx.x;
  for (int64_t q0 = qb; q0 < qe; q0 += (int64_t)kBlock * P) {
    double Qd[P][3];
    double hr[P], hi[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t qi = q0 + (int64_t)p * kBlock + tid;
      Qd[p][0] = Qd[p][1] = Qd[p][2] = 0.0;
      hr[p] = hi[p] = 0.0;
      if (qi < qe) {
        const QRec64 r = rec[qi];
        Qd[p][0] = r.q[0];
        Qd[p][1] = r.q[1];
        Qd[p][2] = r.q[2];
        hr[p] = r.hr;
        hi[p] = r.hi;
      }
    }
#pragma unroll 1
    for (int j = 0; j < nt; ++j) {
      double S[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int p = 0; p < P; ++p) {
        double R[3];
        adj_term_f64(tile[j], gtile[j], Qd[p], hr[p], hi[p], R);
        S[0] += R[0];
        S[1] += R[1];
        S[2] += R[2];
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[3 * j + k][tid] += S[k];
    }
  }
}

// ---------------------------------------------------------------------------
// FP32C adjoint, one block's share: `nt` face records in LDS against the
// reordered Q records [qb, qe), kQPTB Q per thread per pass. Each thread adds
// its weights for face j to its own binary32 slots acc[3 j + k][thread] (zeroed
// by the caller); adj_block_sum32 reduces the slots once the range is done, so
// no cross-lane traffic happens per face.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void adj_tile_fp32c(const Face32B* tile, int nt, int64_t qb, int64_t qe,
                                               const QRec32* __restrict__ rec, float (*acc)[kBlock]) {
  constexpr int P = kQPTB;
  const int tid = threadIdx.x;
  for (int64_t q0 = qb; q0 < qe; q0 += (int64_t)kBlock * P) {
    double Qd[P][3];
    float qx[P], qy[P], qz[P], Q2[P], hr[P], hi[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int64_t qi = q0 + (int64_t)p * kBlock + tid;
      Qd[p][0] = Qd[p][1] = Qd[p][2] = 0.0;
      hr[p] = hi[p] = 0.0f;
      if (qi < qe) {
        const QRec32 r = rec[qi];
        Qd[p][0] = r.q[0];
        Qd[p][1] = r.q[1];
        Qd[p][2] = r.q[2];
        hr[p] = r.hr;
        hi[p] = r.hi;
      }
      qx[p] = (float)Qd[p][0];
      qy[p] = (float)Qd[p][1];
      qz[p] = (float)Qd[p][2];
      Q2[p] = qx[p] * qx[p] + qy[p] * qy[p] + qz[p] * qz[p];
    }
#pragma unroll 1
    for (int j = 0; j < nt; ++j) {
      float S[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int p = 0; p < P; ++p) {
        float R[3];
        adj_term_fp32c(tile[j], qx[p], qy[p], qz[p], Q2[p], Qd[p], hr[p], hi[p], R);
        S[0] += R[0];
        S[1] += R[1];
        S[2] += R[2];
      }
      // private slots: a plain read-modify-write (an LDS atomic add is far slower)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[3 * j + k][tid] += S[k];
    }
  }
}

// Sum of the per-thread slots of adj_tile_fp32c / adj_tile_f64 for each of the
// nt * 3 weights, in binary64 and a fixed order; wave w handles weights w,
// w + 4, ... and lane 0 writes out[v]. Call after a barrier.
template <typename T>
__device__ __forceinline__ void adj_block_sum(T (*acc)[kBlock], int nt, double* out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int v = wave; v < nt * 3; v += kBlock / 64) {
    double x = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) x += (double)acc[v][lane + 64 * i];
    x = wave_total(x);
    if (lane == 0) out[v] = x;
  }
}

}  // namespace pft
