// Per-(Q, face) terms of grad_Q F, binary64 and FP32-compensated forms.
//
// grad_Q F = i * volume integral of r exp(iQ.r). With the field
// x_a (-iQ/|Q|^2) exp(iQ.r), whose divergence is x_a exp(iQ.r) - iQ_a exp(iQ.r)/|Q|^2,
// the divergence theorem turns the volume integral into face integrals of
// r exp(iQ.r) plus (iQ/|Q|^2) F; r is linear on a face, r = sum_k lambda_k v_k,
// so the face integral of r exp(iQ.r) is sum_k v_k times the barycentric
// moment of corner k (the moments of the vertex adjoint). In coordinates
// centred on the mesh centre t, with c_m = (Q.N_m) exp(iQ.g_m) and the moments
// Y_k normalised by 2A relative to exp(iQ.g_m) (J = Y_0 + Y_1 + Y_2):
//   A = sum_m c_m sum_k (v_k - t) Y_k,   B = sum_m c_m J,
//   F_c = -i B / |Q|^2,   grad F_c = (A + iQ B / |Q|^2) / |Q|^2,
//   grad F = exp(iQ.t) (grad F_c + i t F_c).
// The two parts cancel as (|Q| R)^-2 at small |Q| R; there the tetrahedra
// (t, a, b, c) give F_c and grad F_c directly by their series.
#pragma once

#include "adj_terms.h"

namespace pft {

// Tetrahedron with one vertex at the origin and vertex phases x = (x_a, x_b, x_c):
//   S   = sum_n i^n h_n(x_a, x_b, x_c) / (n+3)!,
//   T_k = sum_n i^n h_n(x_a, x_b, x_c, x_k) / (n+4)!   (node k doubled),
// so the integral of exp(iQ.r) over it is 6|T| S and that of lambda_k exp(iQ.r)
// is 6|T| T_k. H_n = h_n(x_a, x_b, x_c) = e1 H_{n-1} - e2 H_{n-2} + e3 H_{n-3} and
// h_n(x, x_k) = H_n + x_k h_{n-1}(x, x_k). Both terms of index n are below
// m^n / n! (m = max |x|); four terms are added per step until that bound on
// the next index is below 1e-18 (the sums are near 1/6 and 1/24 here).
PFT_HD inline void tet_moments_f64(const double* x, double& sr, double& si, double* tr, double* ti) {
  const double e1 = x[0] + x[1] + x[2];
  const double e2 = x[0] * x[1] + x[0] * x[2] + x[1] * x[2];
  const double e3 = x[0] * x[1] * x[2];
  const double m = fmax(fabs(x[0]), fmax(fabs(x[1]), fabs(x[2])));
  const double m4 = (m * m) * (m * m);
  double Hm3 = 0.0, Hm2 = 0.0, Hm1 = 1.0;  // H_{n-3}, H_{n-2}, H_{n-1} at n = 1
  double a[3] = {1.0, 1.0, 1.0};           // h_{n-1}(x, x_k) at n = 1
  sr = 1.0 / 6.0;
  si = 0.0;
  for (int k = 0; k < 3; ++k) tr[k] = 1.0 / 24.0, ti[k] = 0.0;
  double mn = m;  // m^n at the start of each step
  for (int n = 1; n < 85; n += 4) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double H = e1 * Hm1 - e2 * Hm2 + e3 * Hm3;
      const double cs = inv_fact(n + r + 3), ct = inv_fact(n + r + 4);
#pragma unroll
      for (int k = 0; k < 3; ++k) a[k] = H + x[k] * a[k];
      // i^(n+r) with n = 1 (mod 4): +i, -1, -i, +1
      if (r == 0) {
        si += cs * H;
        for (int k = 0; k < 3; ++k) ti[k] += ct * a[k];
      } else if (r == 1) {
        sr -= cs * H;
        for (int k = 0; k < 3; ++k) tr[k] -= ct * a[k];
      } else if (r == 2) {
        si -= cs * H;
        for (int k = 0; k < 3; ++k) ti[k] -= ct * a[k];
      } else {
        sr += cs * H;
        for (int k = 0; k < 3; ++k) tr[k] += ct * a[k];
      }
      Hm3 = Hm2;
      Hm2 = Hm1;
      Hm1 = H;
    }
    mn *= m4;
    if (mn * inv_fact(n + 4) < 1e-18) break;
  }
}

// Small |Q| R: the tetrahedron (o, a, b, c) of face F (o an apex relative to t) adds 6|T| S to F and
// i sum_k v_k 6|T| T_k to grad F, both about o (dq_apex moves them to t).
PFT_HD __forceinline__ void dq_tet_f64(const Face64& F, const double* Q, double* Gr, double* Gi, double& Fr,
                                       double& Fi, const double* o) {
  double v[3][3];
  for (int c = 0; c < 3; ++c) {
    v[0][c] = F.g[c] + F.u0[c] - o[c];
    v[1][c] = F.g[c] + F.u1[c] - o[c];
    v[2][c] = F.g[c] - F.u0[c] - F.u1[c] - o[c];
  }
  const double six_v = F.N[0] * v[0][0] + F.N[1] * v[0][1] + F.N[2] * v[0][2];
  double x[3];
  for (int k = 0; k < 3; ++k) x[k] = Q[0] * v[k][0] + Q[1] * v[k][1] + Q[2] * v[k][2];
  double sr, si, tr[3], ti[3];
  tet_moments_f64(x, sr, si, tr, ti);
  Fr += six_v * sr;
  Fi += six_v * si;
  for (int c = 0; c < 3; ++c) {
    const double mr = v[0][c] * tr[0] + v[1][c] * tr[1] + v[2][c] * tr[2];
    const double mi = v[0][c] * ti[0] + v[1][c] * ti[1] + v[2][c] * ti[2];
    Gr[c] -= six_v * mi;  // i (mr + i mi)
    Gi[c] += six_v * mr;
  }
}

// The fan sums about an apex o, moved to coordinates about t: F = exp(iQ.o) F_o and
// grad F = exp(iQ.o) (grad F_o + i o F_o).
PFT_HD __forceinline__ void dq_apex(const double* Q, const double* o, double* Gr, double* Gi, double& Fr,
                                    double& Fi) {
  double so, co;
  sincos(Q[0] * o[0] + Q[1] * o[1] + Q[2] * o[2], &so, &co);
  for (int c = 0; c < 3; ++c) {
    const double ur = Gr[c] - o[c] * Fi, ui = Gi[c] + o[c] * Fr;
    Gr[c] = co * ur - so * ui;
    Gi[c] = co * ui + so * ur;
  }
  const double fr = co * Fr - so * Fi;
  Fi = co * Fi + so * Fr;
  Fr = fr;
}

// binary64 surface term of face f: A += c sum_k (v_k - t) Y_k, B += c J.
PFT_HD __forceinline__ void dq_term_f64(const Face64& f, const double* G, const double* Q, double* Ar, double* Ai,
                                        double& Br, double& Bi) {
  if (f.thr < 0.0) return;  // empty face
  const double Px = Q[1] * f.N[2] - Q[2] * f.N[1];
  const double Py = Q[2] * f.N[0] - Q[0] * f.N[2];
  const double Pz = Q[0] * f.N[1] - Q[1] * f.N[0];
  const double P2 = Px * Px + Py * Py + Pz * Pz;
  double sf, cf;
  sincos(Q[0] * f.g[0] + Q[1] * f.g[1] + Q[2] * f.g[2], &sf, &cf);
  const double QN = Q[0] * f.N[0] + Q[1] * f.N[1] + Q[2] * f.N[2];
  const double q0 = Q[0] * f.u0[0] + Q[1] * f.u0[1] + Q[2] * f.u0[2];
  const double q1 = Q[0] * f.u1[0] + Q[1] * f.u1[1] + Q[2] * f.u1[2];
  const double m = fmax(fabs(q0), fmax(fabs(q1), fabs(q0 + q1)));
  double yr[2], yi[2], jr, ji;
  if (m <= kSeriesMaxPhase) {
    bary_moments<double, 33>(q0, q1, m, 1e-17, yr, yi, jr, ji);
  } else {
    const double inv = 1.0 / P2;
    double Xr[3], Xi[3], Sr, Si;
    edge_moments_f64(f, G, Q, Px, Py, Pz, q0, q1, inv, Xr, Xi, Sr, Si);
    yr[0] = Xr[0] * inv;
    yi[0] = Xi[0] * inv;
    yr[1] = Xr[1] * inv;
    yi[1] = Xi[1] * inv;
    jr = -Si * inv;
    ji = Sr * inv;
  }
  const double cr = QN * cf, ci = QN * sf;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    // v_2 - t, v_0 - v_2 and v_1 - v_2 (Y_2 = J - Y_0 - Y_1)
    const double p2 = f.g[c] - f.u0[c] - f.u1[c];
    const double e0 = 2.0 * f.u0[c] + f.u1[c];
    const double e1 = f.u0[c] + 2.0 * f.u1[c];
    const double vr = p2 * jr + e0 * yr[0] + e1 * yr[1];
    const double vi = p2 * ji + e0 * yi[0] + e1 * yi[1];
    Ar[c] += cr * vr - ci * vi;
    Ai[c] += cr * vi + ci * vr;
  }
  Br += cr * jr - ci * ji;
  Bi += cr * ji + ci * jr;
}

// FP32C surface term of face f (record of the FP32C adjoint), the same sums in binary32.
__device__ __forceinline__ void dq_term_fp32c(const Face32B& f, float qx, float qy, float qz, const double* Qd,
                                              float* Ar, float* Ai, float& Br, float& Bi) {
  const float N0 = f.N[0], N1 = f.N[1], N2 = f.N[2];
  const float Px = qy * N2 - qz * N1;
  const float Py = qz * N0 - qx * N2;
  const float Pz = qx * N1 - qy * N0;
  const float P2 = Px * Px + Py * Py + Pz * Pz;
  const double ph = Qd[0] * f.gt[0] + Qd[1] * f.gt[1] + Qd[2] * f.gt[2];
  const float r = (float)(ph - rint(ph));
  const float cf = cos_turns(r), sf = sin_turns(r);
  const float QN = qx * N0 + qy * N1 + qz * N2;
  const float q0 = qx * f.u0[0] + qy * f.u0[1] + qz * f.u0[2];
  const float q1 = qx * f.u1[0] + qy * f.u1[1] + qz * f.u1[2];
  const float m = fmaxf(fabsf(q0), fmaxf(fabsf(q1), fabsf(q0 + q1)));
  // (an empty face has an all-zero record: N = 0 makes its terms 0)
  float yr[2], yi[2], jr, ji;
  if (m <= (float)kSeriesMaxPhase) {
    bary_moments_f32(q0, q1, m, yr, yi, jr, ji);
  } else {
    const float inv = rcp_f(fmaxf(P2, 1e-30f));
    float Xr[3], Xi[3], Sr, Si;
    edge_moments_fp32c(f, Px, Py, Pz, q0, q1, inv, Xr, Xi, Sr, Si);
    yr[0] = Xr[0] * inv;
    yi[0] = Xi[0] * inv;
    yr[1] = Xr[1] * inv;
    yi[1] = Xi[1] * inv;
    jr = -Si * inv;
    ji = Sr * inv;
  }
  const float cr = QN * cf, ci = QN * sf;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float e0 = 2.0f * f.u0[c] + f.u1[c];
    const float e1 = f.u0[c] + 2.0f * f.u1[c];
    const float vr = f.c2[c] * jr + e0 * yr[0] + e1 * yr[1];
    const float vi = f.c2[c] * ji + e0 * yi[0] + e1 * yi[1];
    Ar[c] += cr * vr - ci * vi;
    Ai[c] += cr * vi + ci * vr;
  }
  Br += cr * jr - ci * ji;
  Bi += cr * ji + ci * jr;
}

}  // namespace pft
