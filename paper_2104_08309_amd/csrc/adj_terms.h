// Per-(Q, face) terms of the adjoint (barycentric moments of each face),
// binary64 and FP32-compensated forms, shared by the single-mesh and batched
// kernels. The formulas are stated at the top of bwd3d.hip.
#pragma once

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

// Barycentric simplex series: sum_n i^n h_n(d0, d1, d2, dk) / (n+3)!, d0 + d1 + d2 = 0.
// h4_n = H_n + dk h4_{n-1} where H_n = h_n(d0, d1, d2) = -e2 H_{n-2} + e3 H_{n-3}.
PFT_HD inline void bary_series_f64(double e2, double e3, double m, double dk, double& yr, double& yi) {
  double Hm3 = 0.0, Hm2 = 0.0, Hm1 = 1.0;  // H_{n-3}, H_{n-2}, H_{n-1} at n = 1 (H_0 = 1)
  double h4 = 1.0;                         // h4_0
  double inv = 1.0 / 24.0;                 // 1/(n+3)! at n = 1
  yr = 1.0 / 6.0;
  yi = 0.0;
  const double mm = fmax(m, fabs(dk));
  double mn = 1.0;
  for (int n = 1; n < 90; ++n) {
    const double H = -e2 * Hm2 + e3 * Hm3;
    h4 = H + dk * h4;
    const double term = h4 * inv;
    switch (n & 3) {
      case 0: yr += term; break;
      case 1: yi += term; break;
      case 2: yr -= term; break;
      default: yi -= term; break;
    }
    Hm3 = Hm2;
    Hm2 = Hm1;
    Hm1 = H;
    mn *= mm;
    // |h4_n| <= C(n+3, 3) mm^n
    const double bound = mn * (double)((n + 1) * (n + 2) * (n + 3)) / 6.0 * inv;
    if (n >= 3 && bound < 1e-17 * (fabs(yr) + fabs(yi))) break;
    inv /= (double)(n + 4);
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
  if (P2 < f.thr) {
    const double e2 = q0 * q1 + q0 * q2 + q1 * q2;
    const double e3 = q0 * q1 * q2;
    const double m = fmax(fabs(q0), fmax(fabs(q1), fabs(q2)));
    const double dk[3] = {q0, q1, q2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double yr, yi;
      bary_series_f64(e2, e3, m, dk[k], yr, yi);
      R[k] = zr * yr - zi * yi;
    }
    return;
  }
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
  double Sr = 0.0, Si = 0.0;
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
  const double inv = 1.0 / P2;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int kp = (k + 1) % 3, km = (k + 2) % 3;
    double Xr = -0.5 * Si, Xi = 0.5 * Sr;  // (i/2) S
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      Xr += Gm[kp][l] * cr[l];
      Xi += Gm[kp][l] * ci[l];
    }
    Xr += 0.5 * (br[km] - br[k]);
    Xi += 0.5 * (bi[km] - bi[k]);
    Xr += 0.5 * ai[kp];   // -(i/2) a_{k+1}
    Xi -= 0.5 * ar[kp];
    const double s = 2.0 * w[kp] * inv;
    Xr -= s * Sr;
    Xi -= s * Si;
    R[k] = (zr * Xr - zi * Xi) * inv;
  }
}

// ---------------------------------------------------------------------------
// FP32-compensated
// ---------------------------------------------------------------------------
// Barycentric series in binary32, fixed number of terms chosen from the
// largest |delta| of the lane (the series is only taken for |delta| <= 3).
__device__ __forceinline__ void bary_series_f32(float e2, float e3, int nterms, float d0, float d1, float d2,
                                                float* yr, float* yi) {
  // 1/(n+3)! for n = 0..23
  constexpr float kInvF[24] = {
      1.6666667e-01f, 4.1666668e-02f, 8.3333338e-03f, 1.3888889e-03f, 1.9841270e-04f, 2.4801588e-05f,
      2.7557319e-06f, 2.7557319e-07f, 2.5052108e-08f, 2.0876757e-09f, 1.6059044e-10f, 1.1470746e-11f,
      7.6471636e-13f, 4.7794773e-14f, 2.8114573e-15f, 1.5619207e-16f, 8.2206352e-18f, 4.1103176e-19f,
      1.9572941e-20f, 8.8967911e-22f, 3.8681702e-23f, 1.6117376e-24f, 6.4469503e-26f, 2.4795963e-27f};
  float Hm3 = 0.0f, Hm2 = 0.0f, Hm1 = 1.0f;
  float h0 = 1.0f, h1 = 1.0f, h2 = 1.0f;
  float r0 = kInvF[0], r1 = kInvF[0], r2 = kInvF[0];
  float i0 = 0.0f, i1 = 0.0f, i2 = 0.0f;
  for (int n = 1; n < nterms; ++n) {
    const float H = -e2 * Hm2 + e3 * Hm3;
    h0 = H + d0 * h0;
    h1 = H + d1 * h1;
    h2 = H + d2 * h2;
    const float c = kInvF[n];
    const int ph = n & 3;
    const float sgn = (ph < 2) ? c : -c;
    if (ph & 1) {
      i0 += sgn * h0;
      i1 += sgn * h1;
      i2 += sgn * h2;
    } else {
      r0 += sgn * h0;
      r1 += sgn * h1;
      r2 += sgn * h2;
    }
    Hm3 = Hm2;
    Hm2 = Hm1;
    Hm1 = H;
  }
  yr[0] = r0; yr[1] = r1; yr[2] = r2;
  yi[0] = i0; yi[1] = i1; yi[2] = i2;
}

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
  const float p0 = qx * f.h0[0] + qy * f.h0[1] + qz * f.h0[2];  // psi_k in turns
  const float p1 = qx * f.h1[0] + qy * f.h1[1] + qz * f.h1[2];
  const float p2 = -p0 - p1;
  const float kFourPi = 2.0f * kTwoPiF;
  const float q0 = kFourPi * p0, q1 = kFourPi * p1, q2 = -q0 - q1;  // delta_k = Q.u_k
  const float m = fmaxf(fabsf(q0), fmaxf(fabsf(q1), fabsf(q2)));
  if (f.thr < 0.0f) {  // empty face
    R[0] = R[1] = R[2] = 0.0f;
    return;
  }
  if (P2 < fmaxf(f.thr, f.kap * Q2) && m <= 3.0f) {
    const float e2 = q0 * q1 + q0 * q2 + q1 * q2;
    const float e3 = q0 * q1 * q2;
    // terms for a truncation error below 1e-9 of the leading 1/6 at the lane's largest |delta|
    const int nterms = m < 0.35f ? 9 : (m < 0.8f ? 12 : (m < 1.2f ? 14 : (m < 1.6f ? 16 : 21)));
    float yr[3], yi[3];
    bary_series_f32(e2, e3, nterms, q0, q1, q2, yr, yi);
    R[0] = zr * yr[0] - zi * yi[0];
    R[1] = zr * yr[1] - zi * yi[1];
    R[2] = zr * yr[2] - zi * yi[2];
    return;
  }
  const float w0 = Px * f.d0[0] + Py * f.d0[1] + Pz * f.d0[2];
  const float w1 = Px * f.d1[0] + Py * f.d1[1] + Pz * f.d1[2];
  const float w[3] = {w0, w1, -w0 - w1};
  const float s0 = sin_turns(p0), c0 = cos_turns(p0);
  const float s1 = sin_turns(p1), c1 = cos_turns(p1);
  const float c2 = c0 * c1 - s0 * s1;
  const float s2 = -(s0 * c1 + c0 * s1);
  const float eta[3] = {p1 - p0, p2 - p1, p0 - p2};  // turns
  const float cs[3] = {c1 * c0 + s1 * s0, c2 * c1 + s2 * s1, c0 * c2 + s0 * s2};
  const float er[3] = {c2, c0, c1};
  const float ei[3] = {-s2, -s0, -s1};
  float ar[3], ai[3], br[3], bi[3], cr[3], ci[3];
  float Sr = 0.0f, Si = 0.0f;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const float xt = eta[l];
    const float x = kTwoPiF * xt;                  // radians
    const float rx = rcp_f(xt) * kInv2PiF;         // 1/x
    // sinc and its derivative: Taylor series for |x| < 1 (the hardware sine loses
    // relative accuracy at small arguments), quotients beyond
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
  const float inv = rcp_f(fmaxf(P2, 1e-30f));
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int kp = (k + 1) % 3, km = (k + 2) % 3;
    float Xr = -0.5f * Si, Xi = 0.5f * Sr;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      Xr += Gm[kp][l] * cr[l];
      Xi += Gm[kp][l] * ci[l];
    }
    Xr += 0.5f * (br[km] - br[k]);
    Xi += 0.5f * (bi[km] - bi[k]);
    Xr += 0.5f * ai[kp];
    Xi -= 0.5f * ar[kp];
    const float s = 2.0f * w[kp] * inv;
    Xr -= s * Sr;
    Xi -= s * Si;
    R[k] = (zr * Xr - zi * Xi) * inv;
  }
}

// ---------------------------------------------------------------------------
// One block's share of the adjoint: the faces staged in LDS (`nt` of them)
// against the Q range [qb, qe), one Q per thread per pass. For each face the
// three real weights of the 256 Q of a pass are summed across each wavefront
// by lane shuffles and lane 0 adds them to that wavefront's binary64 slot in
// `wacc[wave][3 j + k]` (zeroed by the caller). Faces are visited one at a
// time, so the working set stays that of a single (Q, face) term.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int MODE>
__device__ __forceinline__ void adj_tile_accumulate(const unsigned char* smem_tile, const double (*gtile)[8], int nt,
                                                    const double* tc, int64_t qb, int64_t qe, const void* q,
                                                    int qdtype, const void* grad_out,
                                                    double (*wacc)[kTileFB * 3]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t q0 = qb; q0 < qe; q0 += kBlock) {
    const int64_t qi = q0 + tid;
    double Qd[3] = {0.0, 0.0, 0.0};
    double hr = 0.0, hi = 0.0;
    if (qi < qe) {
      load_q3(q, qdtype, qi, Qd);
      double gr, gi;
      if (MODE == PFT_FP64) {
        const double2 g = static_cast<const double2*>(grad_out)[qi];
        gr = g.x;
        gi = g.y;
      } else {
        const float2 g = static_cast<const float2*>(grad_out)[qi];
        gr = (double)g.x;
        gi = (double)g.y;
      }
      centred_cotangent(gr, gi, Qd, tc, hr, hi);
    }
    if (MODE == PFT_FP64) {
      const Face64* tile = reinterpret_cast<const Face64*>(smem_tile);
#pragma unroll 1
      for (int j = 0; j < nt; ++j) {
        double R[3];
        adj_term_f64(tile[j], gtile[j], Qd, hr, hi, R);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double v = wave_sum(R[k]);
          if (lane == 0) wacc[wave][3 * j + k] += v;
        }
      }
    } else {
      const Face32B* tile = reinterpret_cast<const Face32B*>(smem_tile);
      const float qx = (float)Qd[0], qy = (float)Qd[1], qz = (float)Qd[2];
      const float Q2 = qx * qx + qy * qy + qz * qz;
#pragma unroll 1
      for (int j = 0; j < nt; ++j) {
        float R[3];
        adj_term_fp32c(tile[j], qx, qy, qz, Q2, Qd, (float)hr, (float)hi, R);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float v = wave_sum(R[k]);
          if (lane == 0) wacc[wave][3 * j + k] += (double)v;
        }
      }
    }
  }
}

}  // namespace pft
