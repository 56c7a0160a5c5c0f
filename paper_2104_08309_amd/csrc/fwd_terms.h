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
// Per (Q, face), in binary32 on the record's face-local quantities:
//   QN = Q.N, s_j = Q.(|N| e_j), |P|^2 = s1^2 + s2^2, w_l = P.d_l (w_2 = -w_0 - w_1),
//   half-vertex phases p_k = Q.u_k / (4 pi) in turns (p_2 = -p_0 - p_1),
//   eta_l = p_{l+1} - p_l, edge midpoint phase t_l = r - p_{l+2} with r = Q.g / (2 pi),
//   E_l = 2 pi sinc(2 pi eta_l) exp(2 pi i t_l),  T = (QN / |P|^2) sum_l w_l E_l,
// the face term (Q.N)/|P|^2 exp(iQ.g) S of the 3D section written in turns. The
// 2 pi sinc comes from sinc2pi_poly (no transcendental instruction) and the
// midpoint exponentials from the hardware sine and cosine of turns.
//
// The origin phase r is formed in binary64 and reduced to [-1/2, 1/2] before it
// is rounded to binary32. In an edge-sharing order (Face32::flags) edge 0 is the
// previous record's edge 1, whose E is carried in registers: it depends only on
// the edge (its midpoint, and |eta| since the sinc is even). Near-degenerate
// pairs (Q nearly along the face normal, and empty faces) are replaced by the
// face's simplex series in binary64.

// Inputs of the binary64 series fix-up for one pair.
struct SeriesInputs {
  float p0, p1;  // half-vertex phases psi_0, psi_1 in turns
  float QN;      // Q . N
  float r;       // face origin phase Q.g in turns (any integer offset)
};

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

// What one thread carries from face to face within a face range.
template <int NQ>
struct FwdCarry {
  float er[NQ], ei[NQ];  // E of the previous record's edge 1
  bool prev;             // there is a previous record in this range (uniform)
  __device__ __forceinline__ void reset() { prev = false; }
};

// One face record against a thread's NQ Q points: adds each term to tr[k], ti[k]
// (lanes with small[k] set are left for the caller's small-|Q| path).
template <int NQ, bool SHARE>
__device__ __forceinline__ void fwd_face_fp32c(const Face32& f, const float* qx, const float* qy, const float* qz,
                                               const float* Q2, const double (*Qd)[3], const bool* small, float* tr,
                                               float* ti, FwdCarry<NQ>& c) {
  const uint32_t flags = __builtin_amdgcn_readfirstlane(f.flags);
  const bool linked = SHARE && c.prev && (flags & kFaceLinked) != 0u;
  float QN[NQ], P2[NQ], w0[NQ], w1[NQ], p0[NQ], p1[NQ], r[NQ], c1[NQ], c2[NQ];
  float m = 0.0f;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    QN[k] = qx[k] * f.N[0] + qy[k] * f.N[1] + qz[k] * f.N[2];
    const float s1 = qx[k] * f.E1[0] + qy[k] * f.E1[1] + qz[k] * f.E1[2];
    const float s2 = qx[k] * f.E2[0] + qy[k] * f.E2[1] + qz[k] * f.E2[2];
    P2[k] = s1 * s1 + s2 * s2;
    w0[k] = s2 * f.al[0] + s1 * f.be[0];
    w1[k] = s2 * f.al[1] + s1 * f.be[1];
    p0[k] = s1 * f.ga[0] + s2 * f.de[0];
    p1[k] = s1 * f.ga[1] + s2 * f.de[1];
    // eta_1 = p_2 - p_1 and eta_2 = p_0 - p_2 with p_2 = -p_0 - p_1
    const float x1 = fmaf(-2.0f, p1[k], -p0[k]), x2 = fmaf(2.0f, p0[k], p1[k]);
    c1[k] = sinc2pi_poly(x1);
    c2[k] = sinc2pi_poly(x2);
    m = fmaxf(m, fmaxf(fabsf(x1), fabsf(x2)));
  }
  if (__builtin_expect(m > kSincPolyMax, 0)) {  // long edges at large |Q|: the sine quotient
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      c1[k] = sinc2pi_wide(fmaf(-2.0f, p1[k], -p0[k]), c1[k]);
      c2[k] = sinc2pi_wide(fmaf(2.0f, p0[k], p1[k]), c2[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const double ph = Qd[k][0] * f.gt[0] + Qd[k][1] * f.gt[1] + Qd[k][2] * f.gt[2];
    r[k] = (float)(ph - rint(ph));
  }
  float e0r[NQ], e0i[NQ];
  if (linked) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      e0r[k] = c.er[k];
      e0i[k] = c.ei[k];
    }
  } else {  // edge 0 too (first face of a chain, or the list order)
    float c0[NQ];
    float m0 = 0.0f;
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const float x0 = p1[k] - p0[k];
      c0[k] = sinc2pi_poly(x0);
      m0 = fmaxf(m0, fabsf(x0));
    }
    if (__builtin_expect(m0 > kSincPolyMax, 0)) {
#pragma unroll
      for (int k = 0; k < NQ; ++k) c0[k] = sinc2pi_wide(p1[k] - p0[k], c0[k]);
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const float t0 = r[k] + p0[k] + p1[k];
      e0r[k] = c0[k] * cos_turns(t0);
      e0i[k] = c0[k] * sin_turns(t0);
    }
  }
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const float t1 = r[k] - p0[k], t2 = r[k] - p1[k];
    const float e1r = c1[k] * cos_turns(t1), e1i = c1[k] * sin_turns(t1);
    const float e2r = c2[k] * cos_turns(t2), e2i = c2[k] * sin_turns(t2);
    const float w2 = -(w0[k] + w1[k]);
    const float Sr = w0[k] * e0r[k] + w1[k] * e1r + w2 * e2r;
    const float Si = w0[k] * e0i[k] + w1[k] * e1i + w2 * e2i;
    const float co = QN[k] * rcp_f(P2[k]);
    float Tr = co * Sr, Ti = co * Si;
    // |Q_perp| L < tau or |Q_perp| < tau_rel |Q| (and every pair of an empty face): the series
    if (P2[k] < fmaf(f.kap, Q2[k], f.thr) && !small[k]) {
      SeriesInputs sd;
      sd.p0 = p0[k];
      sd.p1 = p1[k];
      sd.QN = QN[k];
      sd.r = r[k];
      face_series_fp32c(sd, Tr, Ti);
    }
    tr[k] += Tr;
    ti[k] += Ti;
    c.er[k] = e1r;
    c.ei[k] = e1i;
  }
  c.prev = true;
}

// One LDS tile of FP32C face records against the NQ Q points of a thread
// (plain binary32 sums inside the tile). SHARE: the records are in an
// edge-sharing order; `c` carries the shared edge's term and the origin phase
// across faces and tiles of one face range (reset it at the range's start).
template <int NQ, bool SHARE>
__device__ __forceinline__ void fwd_tile_fp32c(const Face32* tile, int nt, const float* qx, const float* qy,
                                               const float* qz, const float* Q2, const double (*Qd)[3],
                                               const bool* small, float* tr, float* ti, FwdCarry<NQ>& c) {
  for (int j = 0; j < nt; ++j) fwd_face_fp32c<NQ, SHARE>(tile[j], qx, qy, qz, Q2, Qd, small, tr, ti, c);
}

__device__ __forceinline__ void kahan_add(float& sum, float& comp, float x) {
  const float y = x - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

}  // namespace pft
