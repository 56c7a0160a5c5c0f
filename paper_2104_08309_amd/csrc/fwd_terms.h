// Per-(Q, face) terms of the forward transform, binary64 and FP32-compensated
// forms, shared by the single-mesh and batched kernels (formulas in pft_device.h).
#pragma once

#include "moment_poly.h"
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
// Per (Q, face), in binary32 on the record's face-local quantities (Face32):
//   QN = Q.N' = Q.n/2, s_j = Q.e_j/2, |P'|^2 = s1^2 + s2^2 = |P|^2 / (4|N|^2),
//   w_l = s2 al_l + s1 be_l = P.d_l / (4 pi |N|) (w_2 = -w_0 - w_1),
//   edge half-phases eta_l = Q.d_l / (4 pi) = s1 al_l - s2 be_l in turns,
//   half-vertex phases p_k = Q.u_k / (4 pi) (p_2 = -p_0 - p_1, eta_l = p_{l+1} - p_l),
//   edge midpoint phase t_l = r - p_{l+2} with r = Q.g / (2 pi),
//   E_l = 2 pi sinc(2 pi eta_l) exp(2 pi i t_l),  T = (QN / |P'|^2) sum_l w_l E_l,
// the face term (Q.N)/|P|^2 exp(iQ.g) S of the 3D section written in turns. The
// 2 pi sinc comes from sinc2pi_poly (no transcendental instruction) and the
// midpoint exponentials from the hardware sine and cosine of turns.
//
// Where the midpoint phases come from. In an edge-sharing order (Face32::flags)
// edge 0 of a linked face is the previous record's edge 1: the same segment, so
// the same midpoint. Its phase t_0 = r + p_0 + p_1 is carried in registers
// (reduced to [-1/2, 1/2] turn), and the two new midpoint phases follow from it
// and the face's own half-vertex phases without the origin phase:
//   t_1 = t_0 - (2 p_0 + p_1) = t_0 - eta_2,   t_2 = t_0 + (-p_0 - 2 p_1) = t_0 + eta_1.
// Each carried step rounds once in binary32 (at most 2^-25 turn for a phase in
// [-1/2, 1/2]), so the chain is re-anchored every kAnchor faces: there, and at
// every face that does not follow its predecessor across an edge, the origin
// phase r = Q.g / (2 pi) is formed in binary64 and reduced to [-1/2, 1/2]
// before it is rounded to binary32. The edge term sinc(eta) exp(i Q.m) of the
// carried edge is carried too (its sinc and the cosine and sine of its
// midpoint phase): it depends only on the edge, since the sinc is even.
// Near-degenerate pairs (Q nearly along the face normal, and empty faces) are
// replaced by the face's simplex series (binary32 through a fitted polynomial at
// small phases, binary64 beyond).

// The FP32C forward sums tau_rel times each face term (Face32::N); partial sums are divided by it once.
constexpr double kInvSumScale32 = 1.0 / kTauRel32;

#ifndef PFT_ANCHOR
#define PFT_ANCHOR kTileF32
#endif
constexpr int kAnchor = PFT_ANCHOR;  // faces between binary64 origin phases in a chain (divides kTileF32)
static_assert(kTileF32 % kAnchor == 0 && kAnchor % 2 == 0, "anchor interval: even, and divides the face tile");

// Inputs of the series fix-up for one pair.
struct SeriesInputs {
  float p0, p1;  // half-vertex phases psi_0, psi_1 in turns
  float QN;      // Q . N, times whatever factor the caller's sums carry (the term is linear in it)
  float r;       // face origin phase Q.g in turns (any integer offset)
};

// The face integral J = sum_n i^n h_n(d) / (n+2)! (normalised by twice the area) in
// binary32 from the polynomial P of exp(ix) fitted on [-P::M, P::M]: J = sum_n i^n
// a_n n! h_n(d) / (n+2)!, within P's fit error / 2 of the exact J for every
// triangle with max |d_k| <= P::M (the simplex average of the fit error).
template <class P>
__device__ __forceinline__ void face_integral_poly(float d0, float d1, float& jr, float& ji) {
  static_assert(P::N >= 5, "the first five terms are written out");
  const float d2 = -d0 - d1;
  const float e2 = d0 * d1 + d2 * (d0 + d1);
  const float e3 = d0 * d1 * d2;
  // H_0 = 1, H_1 = 0, H_2 = -e2, H_3 = e3, H_4 = e2^2, H_n = -e2 H_{n-2} + e3 H_{n-3}
  const float H2 = -e2, H3 = e3, H4 = e2 * e2;
  jr = P::cj[0] - P::cj[2] * H2;
  jr += P::cj[4] * H4;
  ji = -P::cj[3] * H3;
  float Hm3 = H2, Hm2 = H3, Hm1 = H4;
#pragma unroll
  for (int n = 5; n <= P::N; ++n) {
    const float H = -e2 * Hm2 + e3 * Hm3;
    const float c = P::cj[n];
    if ((n & 3) == 1) {
      ji += c * H;
    } else if ((n & 3) == 2) {
      jr -= c * H;
    } else if ((n & 3) == 3) {
      ji -= c * H;
    } else {
      jr += c * H;
    }
    Hm3 = Hm2;
    Hm2 = Hm1;
    Hm1 = H;
  }
}

// Q nearly along the face normal: the face's simplex series,
// T = -i (Q.N) exp(i Q.g) sum_n i^n h_n(delta) / (n+2)!, delta_k = 4 pi psi_k,
// from the binary32 phases of the edge form (their rounding is that of the
// edge form's own inputs). A lane whose largest |delta_k| is within the fitted
// polynomial's range (always so for |Q_perp| L < 0.1, and for the relative test
// while 0.02 |Q| rho stays below it) evaluates it in binary32, within 1e-7 of J;
// a lane beyond it sums the series in binary64 to 1e-10 of the sum. The choice is
// per lane, so a Q's value does not depend on the other lanes of its wavefront.
__device__ __forceinline__ void face_series_fp32c(const SeriesInputs& sd, float& Tr, float& Ti) {
  constexpr float kFourPiF = 12.566370614359172954f;
  const float d0 = kFourPiF * sd.p0, d1 = kFourPiF * sd.p1;
  const float m = fmaxf(fabsf(d0), fmaxf(fabsf(d1), fabsf(d0 + d1)));
  if (m <= FacePoly::M) {
    float sr, si;
    face_integral_poly<FacePoly>(d0, d1, sr, si);
    const float cf = cos_turns(sd.r), sf = sin_turns(sd.r);
    Tr = sd.QN * (cf * si + sf * sr);
    Ti = -sd.QN * (cf * sr - sf * si);
    return;
  }
  constexpr double kFourPi = 12.566370614359172954;
  const double q0 = kFourPi * (double)sd.p0, q1 = kFourPi * (double)sd.p1;
  double sr, si;
  face_series_f64(q0, q1, -q0 - q1, sr, si, 1e-10);
  const double cf = (double)cos_turns(sd.r), sf = (double)sin_turns(sd.r);
  const double QN = (double)sd.QN;
  Tr = (float)(QN * (cf * si + sf * sr));
  Ti = (float)(-QN * (cf * sr - sf * si));
}

// What one thread carries from face to face within a face range: the edge 1 of
// the previous record, as its 2 pi sinc(2 pi eta), the cosine and sine of its
// midpoint phase, and that phase in turns reduced to [-1/2, 1/2].
template <int NQ>
struct FwdCarry {
  float c[NQ], cs[NQ], sn[NQ], t[NQ];
  bool prev;             // there is a previous record in this range (uniform)
  __device__ __forceinline__ void reset() { prev = false; }
};

// The binary64 Q of a thread's NQ points held as binary32 pairs: Q = hi + lo with
// hi = (float)Q (the binary32 Q of the edge arithmetic) and lo = (float)(Q - hi),
// i.e. Q to 48 bits (relative error <= 2^-48), for the binary64 origin phase at
// the anchors, in half the registers of a binary64 copy.
template <int NQ>
struct QLow {
  float lo[NQ][3];
  __device__ __forceinline__ void set(int k, const double* Q, float hx, float hy, float hz) {
    lo[k][0] = (float)(Q[0] - (double)hx);
    lo[k][1] = (float)(Q[1] - (double)hy);
    lo[k][2] = (float)(Q[2] - (double)hz);
  }
  __device__ __forceinline__ double qd(float hi, int k, int j) const { return (double)hi + (double)lo[k][j]; }
  // The same inside the face loop: the empty asm statement makes the pair opaque at the anchor, so the
  // compiler forms the binary64 value there instead of hoisting nine binary64 registers out of the loop.
  __device__ __forceinline__ double qd_here(float hi, int k, int j) const {
    float h = hi, l = lo[k][j];
    asm volatile("" : "+v"(h), "+v"(l));
    return (double)h + (double)l;
  }
};

// The same low parts kept in a wavefront's slice of LDS (64 * 3 * NQ floats, lane-major so a wavefront's
// access is one conflict-free row) instead of nine registers: only the anchors, the chain starts and the
// small-|Q| fan read them. Each lane reads only what it wrote itself.
template <int NQ>
struct QLowLds {
  float* lo;  // this wavefront's slice
  int lane;
  __device__ __forceinline__ void set(int k, const double* Q, float hx, float hy, float hz) {
    lo[(k * 3 + 0) * 64 + lane] = (float)(Q[0] - (double)hx);
    lo[(k * 3 + 1) * 64 + lane] = (float)(Q[1] - (double)hy);
    lo[(k * 3 + 2) * 64 + lane] = (float)(Q[2] - (double)hz);
  }
  __device__ __forceinline__ double qd(float hi, int k, int j) const {
    return (double)hi + (double)lo[(k * 3 + j) * 64 + lane];
  }
  __device__ __forceinline__ double qd_here(float hi, int k, int j) const { return qd(hi, k, j); }
};

// Orders a wavefront's LDS accesses around a tile it stages for itself: its stores are complete before
// any lane reads, and its earlier reads before it overwrites (a wavefront's LDS instructions execute in
// order; the fence also keeps the compiler from moving accesses across it).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Largest |Q| over the wavefront's lanes (every lane gets the same value).
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// Whether any edge half-phase |eta| = |Q.d| / (4 pi) of a wavefront can exceed
// the polynomial sinc's range: |d| <= 2 rho for a face whose vertices lie within
// rho of its centroid, so |eta| <= qmax rho / (2 pi). A wavefront that passes
// this test never meets an argument beyond kSincPolyMax (1e-3 of margin for
// rounding) and skips the per-lane range test; each lane's value is the same
// either way.
__device__ __forceinline__ bool sinc_range_test_needed(float qmax, double rho) {
  return (double)qmax * rho * kInv2PiD > 0.999 * (double)kSincPolyMax;
}

// S = sum_l w_l sinc_l e^{2 pi i t_l} of one face and Q from the carried edge 0 (its sinc c0 and
// exponential e0) and the new edges 1 and 2, with w_2 = -(w_0 + w_1).
__device__ __forceinline__ void edge_sum(float w0, float w1, float c0, float c1, float c2, float e0c, float e0s,
                                         float e1c, float e1s, float e2c, float e2s, float& Sr, float& Si) {
  const float a0 = w0 * c0, a1 = w1 * c1, a2 = (w0 + w1) * c2;
  Sr = a0 * e0c + a1 * e1c - a2 * e2c;
  Si = a0 * e0s + a1 * e1s - a2 * e2s;
}

// One face record against a thread's NQ Q points: adds each term to tr[k], ti[k]
// (lanes with small[k] set are left for the caller's small-|Q| path). CHECK:
// test each edge half-phase against the polynomial sinc's range; anchor: form
// the origin phase in binary64 even when the face is linked. `cin` holds the
// previous record's edge 1 (edge 0 of a linked face); the face's own edge 1 goes
// to `cout` (SHARE only; the two may be the same object).
template <int NQ, bool SHARE, bool CHECK, bool TC, class QL>
__device__ __forceinline__ void fwd_face_fp32c(const Face32& f, const float* qx, const float* qy, const float* qz,
                                               const QL& ql, const bool* small, float* tr,
                                               float* ti, bool anchor, FwdCarry<NQ>& cin, FwdCarry<NQ>& cout) {
  const uint32_t flags = __builtin_amdgcn_readfirstlane(f.flags);
  const bool linked = SHARE && cin.prev && (flags & kFaceLinked) != 0u;
  float QN[NQ], P2[NQ], w0[NQ], w1[NQ], x1[NQ], x2[NQ], c1[NQ], c2[NQ];
  float m = 0.0f;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    QN[k] = qx[k] * f.N[0] + qy[k] * f.N[1] + qz[k] * f.N[2];
    const float s1 = qx[k] * f.E1[0] + qy[k] * f.E1[1] + qz[k] * f.E1[2];
    const float s2 = qx[k] * f.E2[0] + qy[k] * f.E2[1] + qz[k] * f.E2[2];
    P2[k] = s1 * s1 + s2 * s2;
    w0[k] = s2 * f.al[0] + s1 * f.be[0];
    w1[k] = s2 * f.al[1] + s1 * f.be[1];
    // edge half-phases eta_1, eta_2 (eta_0 = -eta_1 - eta_2)
    x1[k] = s1 * f.al[1] - s2 * f.be[1];
    x2[k] = s1 * f.al[2] - s2 * f.be[2];
    c1[k] = sinc2pi_poly(x1[k]);
    c2[k] = sinc2pi_poly(x2[k]);
    if (CHECK) m = fmaxf(m, fmaxf(fabsf(x1[k]), fabsf(x2[k])));
  }
  if (CHECK && __builtin_expect(m > kSincPolyMax, 0)) {  // long edges at large |Q|: the sine quotient
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      c1[k] = sinc2pi_wide(x1[k], c1[k]);
      c2[k] = sinc2pi_wide(x2[k], c2[k]);
    }
  }
  // Edge 0 where it is not the carried edge: its midpoint phase t_0 = r + p_0 + p_1 = r + (eta_2 - eta_1)/3
  // from the binary64 origin phase (also at an anchor, replacing the carried phase), and its term when
  // unlinked.
  if (!linked || anchor) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const double ph =
          ql.qd_here(qx[k], k, 0) * f.gt[0] + ql.qd_here(qy[k], k, 1) * f.gt[1] + ql.qd_here(qz[k], k, 2) * f.gt[2];
      const float r = (float)(ph - rint(ph));
      cin.t[k] = r + (x2[k] - x1[k]) * (1.0f / 3.0f);
    }
    if (!linked) {  // first face of a chain, or the list order
      float m0 = 0.0f;
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        const float x0 = -(x1[k] + x2[k]);
        cin.c[k] = sinc2pi_poly(x0);
        if (CHECK) m0 = fmaxf(m0, fabsf(x0));
        cin.cs[k] = cos_turns(cin.t[k]);
        cin.sn[k] = sin_turns(cin.t[k]);
      }
      if (CHECK && __builtin_expect(m0 > kSincPolyMax, 0)) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) cin.c[k] = sinc2pi_wide(-(x1[k] + x2[k]), cin.c[k]);
      }
    }
  }
  float Sr[NQ], Si[NQ], co[NQ], t1[NQ];
  bool need[NQ];
  bool any = false;
  if constexpr (TC) {
    // The face's transcendental instructions back to back. On this target every switch between
    // transcendental and ordinary vector instructions costs issue cycles, so one run of 5 NQ is cheaper
    // than the several shorter ones the compiler forms by itself; the scheduling barriers keep it from
    // interleaving them (at the price of a few more live registers).
    float t2[NQ], e1c[NQ], e1s[NQ], e2c[NQ], e2s[NQ], rp[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      // t_1 = t_0 - eta_2, t_2 = t_0 + eta_1
      t1[k] = cin.t[k] - x2[k];
      t2[k] = cin.t[k] + x1[k];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      e1c[k] = cos_turns(t1[k]);
      e1s[k] = sin_turns(t1[k]);
      e2c[k] = cos_turns(t2[k]);
      e2s[k] = sin_turns(t2[k]);
      rp[k] = rcp_f(P2[k]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      edge_sum(w0[k], w1[k], cin.c[k], c1[k], c2[k], cin.cs[k], cin.sn[k], e1c[k], e1s[k], e2c[k], e2s[k], Sr[k], Si[k]);
      co[k] = QN[k] * rp[k];
      // |Q_perp| L < tau or |Q_perp| < tau_rel |Q| (and every pair of an empty face): the series
      need[k] = P2[k] < fmaf(QN[k], QN[k], f.thr) && !small[k];
      any |= need[k];
      if (SHARE) {
        cout.c[k] = c1[k];
        cout.cs[k] = e1c[k];
        cout.sn[k] = e1s[k];
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      t1[k] = cin.t[k] - x2[k];
      const float t2 = cin.t[k] + x1[k];
      const float e1c = cos_turns(t1[k]), e1s = sin_turns(t1[k]);
      const float e2c = cos_turns(t2), e2s = sin_turns(t2);
      edge_sum(w0[k], w1[k], cin.c[k], c1[k], c2[k], cin.cs[k], cin.sn[k], e1c, e1s, e2c, e2s, Sr[k], Si[k]);
      co[k] = QN[k] * rcp_f(P2[k]);
      need[k] = P2[k] < fmaf(QN[k], QN[k], f.thr) && !small[k];
      any |= need[k];
      if (SHARE) {
        cout.c[k] = c1[k];
        cout.cs[k] = e1c;
        cout.sn[k] = e1s;
      }
    }
  }
  // one branch per face for the rare lanes that need the series (of any of their NQ points)
  if (__builtin_expect(any, 0)) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      if (need[k]) {
        // half-vertex phases from the edge half-phases: p_0 = (2 eta_2 + eta_1)/3, p_1 = -(2 eta_1 + eta_2)/3
        SeriesInputs sd;
        sd.p0 = (2.0f * x2[k] + x1[k]) * (1.0f / 3.0f);
        sd.p1 = -(2.0f * x1[k] + x2[k]) * (1.0f / 3.0f);
        sd.QN = QN[k] * f.nN;  // tau_rel Q.N through the record's own N', as in the edge form
        sd.r = t1[k] + sd.p0;
        face_series_fp32c(sd, Sr[k], Si[k]);  // tau_rel times the face term, like the edge form's
        co[k] = 1.0f;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    tr[k] = fmaf(co[k], Sr[k], tr[k]);
    ti[k] = fmaf(co[k], Si[k], ti[k]);
    if (SHARE) cout.t[k] = t1[k] - rintf(t1[k]);
  }
  cout.prev = true;
}

// One LDS tile of FP32C face records against the NQ Q points of a thread
// (plain binary32 sums inside the tile). SHARE: the records are in an
// edge-sharing order; `c` carries the shared edge's term and midpoint phase
// across faces and tiles of one face range (reset it at the range's start).
// The origin phase is formed in binary64 at every kAnchor-th face of a tile (of kTileF32 faces).
// Faces go in pairs that pass the carry between two register sets, so no copy
// of it is needed from one face to the next. TC: each face's transcendental
// instructions in one run (fwd_face_fp32c).
template <int NQ, bool SHARE, bool CHECK, bool TC, class QL>
__device__ __forceinline__ void fwd_tile_fp32c(const Face32* tile, int nt, const float* qx, const float* qy,
                                               const float* qz, const QL& ql,
                                               const bool* small, float* tr, float* ti, FwdCarry<NQ>& c) {
  FwdCarry<NQ> d;
  int j = 0;
  for (; j + 2 <= nt; j += 2) {
    fwd_face_fp32c<NQ, SHARE, CHECK, TC>(tile[j], qx, qy, qz, ql, small, tr, ti, (j % kAnchor) == 0, c, d);
    fwd_face_fp32c<NQ, SHARE, CHECK, TC>(tile[j + 1], qx, qy, qz, ql, small, tr, ti, false, d, c);
  }
  if (j < nt) {
    fwd_face_fp32c<NQ, SHARE, CHECK, TC>(tile[j], qx, qy, qz, ql, small, tr, ti, (j % kAnchor) == 0, c, d);
    c = d;
  }
}

__device__ __forceinline__ void kahan_add(float& sum, float& comp, float x) {
  const float y = x - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

}  // namespace pft
