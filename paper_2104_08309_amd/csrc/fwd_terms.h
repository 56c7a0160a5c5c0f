// Per-(Q, face) terms of the forward transform, binary64 and FP32-compensated
// forms, shared by the single-mesh and batched kernels (formulas in pft_device.h).
#pragma once

#include "pft_device.h"

namespace pft {

// ---------------------------------------------------------------------------
// binary64 per-(Q, face) term T_m (see pft_device.h for the formula)
// ---------------------------------------------------------------------------
PFT_HD __forceinline__ double sinc_f64(double x, double sinx) {
  // sinx = sin(x) from the vertex phase products; Taylor series near 0 where
  // the quotient loses relative accuracy.
  const double x2 = x * x;
  if (fabs(x) < 0.1) {
    return 1.0 + x2 * (-1.0 / 6.0 + x2 * (1.0 / 120.0 + x2 * (-1.0 / 5040.0 + x2 * (1.0 / 362880.0))));
  }
  return sinx / x;
}

PFT_HD __forceinline__ void face_term_f64(const Face64& f, const double* Q, double& Tr, double& Ti) {
  const double QN = Q[0] * f.N[0] + Q[1] * f.N[1] + Q[2] * f.N[2];
  const double Px = Q[1] * f.N[2] - Q[2] * f.N[1];
  const double Py = Q[2] * f.N[0] - Q[0] * f.N[2];
  const double Pz = Q[0] * f.N[1] - Q[1] * f.N[0];
  const double P2 = Px * Px + Py * Py + Pz * Pz;
  const double phi = Q[0] * f.g[0] + Q[1] * f.g[1] + Q[2] * f.g[2];
  double sf, cf;
  sincos(phi, &sf, &cf);
  const double q0 = Q[0] * f.u0[0] + Q[1] * f.u0[1] + Q[2] * f.u0[2];  // delta_0 = 2 psi_0
  const double q1 = Q[0] * f.u1[0] + Q[1] * f.u1[1] + Q[2] * f.u1[2];
  if (P2 < f.thr) {
    double sr, si;
    face_series_f64(q0, q1, -q0 - q1, sr, si);
    // T = -i (Q.N) exp(i phi) s
    Tr = QN * (cf * si + sf * sr);
    Ti = -QN * (cf * sr - sf * si);
    return;
  }
  const double p0 = 0.5 * q0, p1 = 0.5 * q1, p2 = -p0 - p1;
  double s0, c0, s1, c1;
  sincos(p0, &s0, &c0);
  sincos(p1, &s1, &c1);
  const double c2 = c0 * c1 - s0 * s1;      // exp(i psi_2) = conj(exp(i psi_0) exp(i psi_1))
  const double s2 = -(s0 * c1 + c0 * s1);
  // w_l = P.d_l = pi_{l+1} - pi_l with pi_k = P.u_k
  const double pi0 = Px * f.u0[0] + Py * f.u0[1] + Pz * f.u0[2];
  const double pi1 = Px * f.u1[0] + Py * f.u1[1] + Pz * f.u1[2];
  const double pi2 = -pi0 - pi1;
  const double w0 = pi1 - pi0, w1 = pi2 - pi1, w2 = pi0 - pi2;
  // sinc(eta_l), eta_l = psi_{l+1} - psi_l, sin(eta_l) = Im(exp(i psi_{l+1}) exp(-i psi_l))
  const double a0 = w0 * sinc_f64(p1 - p0, s1 * c0 - c1 * s0);
  const double a1 = w1 * sinc_f64(p2 - p1, s2 * c1 - c2 * s1);
  const double a2 = w2 * sinc_f64(p0 - p2, s0 * c2 - c0 * s2);
  // edge l carries exp(-i psi_{l+2})
  const double Sr = a0 * c2 + a1 * c0 + a2 * c1;
  const double Si = -(a0 * s2 + a1 * s0 + a2 * s1);
  const double co = QN / fmax(P2, 1e-300);
  const double Ur = co * cf, Ui = co * sf;
  Tr = Ur * Sr - Ui * Si;
  Ti = Ur * Si + Ui * Sr;
}

// ---------------------------------------------------------------------------
// FP32-compensated per-(Q, face) term
// ---------------------------------------------------------------------------
// Edge-sum form of the FP32-compensated face term. Sets `need_series` when the
// pair is near-degenerate (Q close to the face normal) so that the caller
// replaces the result with face_series_fp32c; keeping the branch out of this
// function leaves straight-line code that the compiler can interleave across
// the several Q a thread evaluates.
__device__ __forceinline__ void face_term_fp32c(const Face32& f, float qx, float qy, float qz, float Q2,
                                                const double* Qd, float& Tr, float& Ti, bool& need_series,
                                                float& phase_out) {
  const float N0 = f.N[0], N1 = f.N[1], N2 = f.N[2];
  const float QN = qx * N0 + qy * N1 + qz * N2;
  const float Px = qy * N2 - qz * N1;
  const float Py = qz * N0 - qx * N2;
  const float Pz = qx * N1 - qy * N0;
  const float P2 = Px * Px + Py * Py + Pz * Pz;
  const float w0 = Px * f.d0[0] + Py * f.d0[1] + Pz * f.d0[2];
  const float w1 = Px * f.d1[0] + Py * f.d1[1] + Pz * f.d1[2];
  const float w2 = -w0 - w1;
  // half-vertex phases psi_k in turns
  const float p0 = qx * f.h0[0] + qy * f.h0[1] + qz * f.h0[2];
  const float p1 = qx * f.h1[0] + qy * f.h1[1] + qz * f.h1[2];
  const float p2 = -p0 - p1;
  // 2 pi sinc(eta_l), eta_l = psi_{l+1} - psi_l (turns)
  const float a0 = w0 * sinc2pi_turns(p1 - p0);
  const float a1 = w1 * sinc2pi_turns(p2 - p1);
  const float a2 = w2 * sinc2pi_turns(p0 - p2);
  // face origin phase Q.g in turns, reduced to [-1/2, 1/2] in binary64; the edge
  // midpoint phases are Q.m_l = Q.g - psi_{l+2}
  const double ph = Qd[0] * f.gt[0] + Qd[1] * f.gt[1] + Qd[2] * f.gt[2];
  const float r = (float)(ph - rint(ph));
  const float t0 = r - p2, t1 = r - p0, t2 = r - p1;
  const float Sr = a0 * cos_turns(t0) + a1 * cos_turns(t1) + a2 * cos_turns(t2);
  const float Si = a0 * sin_turns(t0) + a1 * sin_turns(t1) + a2 * sin_turns(t2);
  const float co = QN * rcp_f(fmaxf(P2, 1e-30f));
  Tr = co * Sr;
  Ti = co * Si;
  need_series = P2 < fmaxf(f.thr, f.kap * Q2);
  phase_out = r;  // the series fix-up forms exp(i Q.g) itself (rare path)
}

// Q nearly along the face normal: binary64 simplex series of the face,
// T = -i (Q.N) exp(i Q.g) sum_n i^n h_n(delta) / (n+2)!.
__device__ __forceinline__ void face_series_fp32c(const Face64* __restrict__ fa, const double* Qd, float r,
                                               float& Tr, float& Ti) {
  const float cf = cos_turns(r), sf = sin_turns(r);
  const Face64 F = *fa;
  const double QNd = Qd[0] * F.N[0] + Qd[1] * F.N[1] + Qd[2] * F.N[2];
  const double q0 = Qd[0] * F.u0[0] + Qd[1] * F.u0[1] + Qd[2] * F.u0[2];
  const double q1 = Qd[0] * F.u1[0] + Qd[1] * F.u1[1] + Qd[2] * F.u1[2];
  double sr, si;
  face_series_f64(q0, q1, -q0 - q1, sr, si);
  Tr = (float)(QNd * ((double)cf * si + (double)sf * sr));
  Ti = (float)(-QNd * ((double)cf * sr - (double)sf * si));
}

__device__ __forceinline__ void kahan_add(float& sum, float& comp, float x) {
  const float y = x - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

}  // namespace pft
