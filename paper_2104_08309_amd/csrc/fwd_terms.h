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
    face_series_f64(q0, q1, -q0 - q1, sr, si, 1e-17);
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
// the several Q a thread evaluates. The quantities the series needs (the
// half-vertex phases, Q.N and the reduced face phase) are returned in `sd`.
struct SeriesInputs {
  float p0, p1;  // half-vertex phases psi_0, psi_1 in turns
  float QN;      // Q . N
  float r;       // face origin phase Q.g in turns, reduced to [-1/2, 1/2]
};

__device__ __forceinline__ void face_term_fp32c(const Face32& f, float qx, float qy, float qz, float Q2,
                                                const double* Qd, float& Tr, float& Ti, bool& need_series,
                                                SeriesInputs& sd) {
  const float QN = qx * f.N[0] + qy * f.N[1] + qz * f.N[2];
  // in-plane components of Q (times |N|); P = Q x N = s2 e1 - s1 e2
  const float s1 = qx * f.E1[0] + qy * f.E1[1] + qz * f.E1[2];
  const float s2 = qx * f.E2[0] + qy * f.E2[1] + qz * f.E2[2];
  const float P2 = s1 * s1 + s2 * s2;
  // edge weights w_l = P . d_l (over 2 pi)
  const float w0 = s2 * f.al[0] + s1 * f.be[0];
  const float w1 = s2 * f.al[1] + s1 * f.be[1];
  const float w2 = -w0 - w1;
  // half-vertex phases psi_k in turns
  const float p0 = s1 * f.ga[0] + s2 * f.de[0];
  const float p1 = s1 * f.ga[1] + s2 * f.de[1];
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
  sd.p0 = p0;
  sd.p1 = p1;
  sd.QN = QN;
  sd.r = r;
}

// Q nearly along the face normal: simplex series of the face in binary64,
// T = -i (Q.N) exp(i Q.g) sum_n i^n h_n(delta) / (n+2)!, delta_k = 4 pi psi_k,
// from the binary32 phases of the edge form (their rounding is that of the
// edge form's own inputs). Terms stop at 1e-10 of the sum, far below binary32
// resolution.
__device__ __forceinline__ void face_series_fp32c(const SeriesInputs& sd, float& Tr, float& Ti) {
  constexpr double kFourPi = 12.566370614359172954;
  const double q0 = kFourPi * (double)sd.p0, q1 = kFourPi * (double)sd.p1;
  double sr, si;
  face_series_f64(q0, q1, -q0 - q1, sr, si, 1e-10);
  const double cf = (double)cos_turns(sd.r), sf = (double)sin_turns(sd.r);
  const double QN = (double)sd.QN;
  Tr = (float)(QN * (cf * si + sf * sr));
  Ti = (float)(-QN * (cf * sr - sf * si));
}

// The same face term with one edge term taken from the previous face: in an
// edge-sharing order (consecutive faces share an edge, Face32::link) the
// shared edge's sinc(eta) exp(2 pi i t) is the same for both faces (the
// midpoint is the same, and sinc is even in eta, whose sign flips with the
// edge's direction); only its weight w = P.d belongs to each face. E holds
// the previous face's terms of its edges 1 and 2 (re, im, re, im) and is
// replaced by this face's; with reuse = 0 all three edge terms are computed.
__device__ __forceinline__ void face_term_fp32c_shared(const Face32& f, float qx, float qy, float qz, float Q2,
                                                       const double* Qd, bool reuse, float* E, float& Tr,
                                                       float& Ti, bool& need_series, SeriesInputs& sd) {
  const float QN = qx * f.N[0] + qy * f.N[1] + qz * f.N[2];
  const float s1 = qx * f.E1[0] + qy * f.E1[1] + qz * f.E1[2];
  const float s2 = qx * f.E2[0] + qy * f.E2[1] + qz * f.E2[2];
  const float P2 = s1 * s1 + s2 * s2;
  const float w0 = s2 * f.al[0] + s1 * f.be[0];
  const float w1 = s2 * f.al[1] + s1 * f.be[1];
  const float w2 = -w0 - w1;
  const float p0 = s1 * f.ga[0] + s2 * f.de[0];
  const float p1 = s1 * f.ga[1] + s2 * f.de[1];
  const float p2 = -p0 - p1;
  const double ph = Qd[0] * f.gt[0] + Qd[1] * f.gt[1] + Qd[2] * f.gt[2];
  const float r = (float)(ph - rint(ph));
  const float t0 = r - p2, t1 = r - p0, t2 = r - p1;
  float e0r, e0i;
  if (reuse) {
    const bool one = f.link == 1u;
    e0r = one ? E[0] : E[2];
    e0i = one ? E[1] : E[3];
  } else {
    const float c0 = sinc2pi_turns(p1 - p0);
    e0r = c0 * cos_turns(t0);
    e0i = c0 * sin_turns(t0);
  }
  const float c1 = sinc2pi_turns(p2 - p1), c2 = sinc2pi_turns(p0 - p2);
  E[0] = c1 * cos_turns(t1);
  E[1] = c1 * sin_turns(t1);
  E[2] = c2 * cos_turns(t2);
  E[3] = c2 * sin_turns(t2);
  const float Sr = w0 * e0r + w1 * E[0] + w2 * E[2];
  const float Si = w0 * e0i + w1 * E[1] + w2 * E[3];
  const float co = QN * rcp_f(fmaxf(P2, 1e-30f));
  Tr = co * Sr;
  Ti = co * Si;
  need_series = P2 < fmaxf(f.thr, f.kap * Q2);
  sd.p0 = p0;
  sd.p1 = p1;
  sd.QN = QN;
  sd.r = r;
}

// One LDS tile of FP32C face records against the NQ Q points of a thread:
// adds each face's term to tr[k], ti[k] (plain binary32 inside the tile). The
// edge form is evaluated for every lane (no per-Q branch, so the NQ streams
// interleave); pairs flagged near-degenerate are replaced by the series, and
// lanes with small[k] set are left for the caller's small-|Q| path.
// SHARE: the records are in edge-sharing order; E[k] carries the previous
// face's edge terms across faces and tiles, prev_ok says whether there is a
// previous (non-empty) face of the same face range to take them from.
template <int NQ, bool SHARE>
__device__ __forceinline__ void fwd_tile_fp32c(const Face32* tile, int nt, const float* qx, const float* qy,
                                               const float* qz, const float* Q2, const double (*Qd)[3],
                                               const bool* small, float* tr, float* ti, float (*E)[4],
                                               bool& prev_ok) {
  for (int j = 0; j < nt; ++j) {
    float Tr[NQ], Ti[NQ];
    SeriesInputs sd[NQ];
    bool ser[NQ];
    if (SHARE) {
      const bool reuse = prev_ok && tile[j].link != 0u;
#pragma unroll
      for (int k = 0; k < NQ; ++k)
        face_term_fp32c_shared(tile[j], qx[k], qy[k], qz[k], Q2[k], Qd[k], reuse, E[k], Tr[k], Ti[k], ser[k],
                               sd[k]);
      prev_ok = tile[j].thr >= 0.0f;
    } else {
#pragma unroll
      for (int k = 0; k < NQ; ++k)
        face_term_fp32c(tile[j], qx[k], qy[k], qz[k], Q2[k], Qd[k], Tr[k], Ti[k], ser[k], sd[k]);
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      if (ser[k] && !small[k]) face_series_fp32c(sd[k], Tr[k], Ti[k]);
      tr[k] += Tr[k];
      ti[k] += Ti[k];
    }
  }
}

__device__ __forceinline__ void kahan_add(float& sum, float& comp, float x) {
  const float y = x - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

}  // namespace pft
