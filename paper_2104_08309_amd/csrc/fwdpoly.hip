// Forward 3D transform of a closed mesh of planar polygon faces: eq.
// sum_elements_3d with nu_m edges per face, evaluated natively (nu edge terms
// per face instead of 3 (nu - 2) for a triangulation).
//
// Per face, with u_k = r_k - g (g the vertex mean), N = sum_k u_k x u_{k+1}
// = 2 A n, P = Q x N, psi_k = Q.u_k / 2:
//   T = (Q.N / |P|^2) exp(iQ.g) sum_k (P.d_k) sinc(psi_{k+1} - psi_k) exp(i (psi_k + psi_{k+1})),
// the edge k running from vertex k to k+1 (wrapping), whose midpoint phase
// relative to g is psi_k + psi_{k+1}. Where Q is nearly along n the face is
// the sum of its fan triangles (r_0, r_l, r_{l+1}), each by its simplex series
// with its signed area. The layout follows fwd3d.hip: a Q tile per block, a
// range of face tiles per blockIdx.y, records staged in LDS per tile (faces
// and their vertex records are contiguous), binary64 partials per split.
#include "fwd_terms.h"

namespace pft {
namespace {

// ---------------------------------------------------------------------------
// binary64
// ---------------------------------------------------------------------------
// fan-triangle series of a polygon face: sum_t 2A_t exp(iQ.g_t) series(delta_t), relative to exp(iQ.g)
__device__ void poly_fan_series_f64(const FaceP64& F, const VtxP64* V, const double* Q, double& jr, double& ji) {
  jr = ji = 0.0;
  const double* a = V[0].u;
  const double qa = Q[0] * a[0] + Q[1] * a[1] + Q[2] * a[2];
  for (int l = 1; l + 1 < F.nv; ++l) {
    const double* b = V[l].u;
    const double* c = V[l + 1].u;
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double two_a = (cr[0] * F.N[0] + cr[1] * F.N[1] + cr[2] * F.N[2]) * F.invN;
    const double qb = Q[0] * b[0] + Q[1] * b[1] + Q[2] * b[2];
    const double qc = Q[0] * c[0] + Q[1] * c[1] + Q[2] * c[2];
    const double qt = (qa + qb + qc) / 3.0;  // phase of the triangle's centroid relative to g
    double sr, si;
    face_series_f64(qa - qt, qb - qt, qc - qt, sr, si, 1e-17);
    double st, ct;
    sincos(qt, &st, &ct);
    jr += two_a * (ct * sr - st * si);
    ji += two_a * (ct * si + st * sr);
  }
}

__device__ void poly_term_f64(const FaceP64& F, const VtxP64* V, const double* Q, double& Tr, double& Ti) {
  const double QN = Q[0] * F.N[0] + Q[1] * F.N[1] + Q[2] * F.N[2];
  const double Px = Q[1] * F.N[2] - Q[2] * F.N[1];
  const double Py = Q[2] * F.N[0] - Q[0] * F.N[2];
  const double Pz = Q[0] * F.N[1] - Q[1] * F.N[0];
  const double P2 = Px * Px + Py * Py + Pz * Pz;
  double sf, cf;
  sincos(Q[0] * F.g[0] + Q[1] * F.g[1] + Q[2] * F.g[2], &sf, &cf);
  double Sr = 0.0, Si = 0.0, co;
  if (P2 < F.thr) {
    // T = -i (Q.n) exp(iQ.g) J
    double jr, ji;
    poly_fan_series_f64(F, V, Q, jr, ji);
    co = QN * F.invN;
    Sr = ji;
    Si = -jr;
  } else {
    const double* u0 = V[0].u;
    const double psi0 = 0.5 * (Q[0] * u0[0] + Q[1] * u0[1] + Q[2] * u0[2]);
    const double pi0 = Px * u0[0] + Py * u0[1] + Pz * u0[2];
    double s0, c0;
    sincos(psi0, &s0, &c0);
    double psi_a = psi0, pi_a = pi0, s_a = s0, c_a = c0;
    for (int k = 1; k <= F.nv; ++k) {
      double psi_b, pi_b, s_b, c_b;
      if (k < F.nv) {
        const double* u = V[k].u;
        psi_b = 0.5 * (Q[0] * u[0] + Q[1] * u[1] + Q[2] * u[2]);
        pi_b = Px * u[0] + Py * u[1] + Pz * u[2];
        sincos(psi_b, &s_b, &c_b);
      } else {
        psi_b = psi0;
        pi_b = pi0;
        s_b = s0;
        c_b = c0;
      }
      // edge a -> b: w = P.d, sinc(psi_b - psi_a), exp(i (psi_a + psi_b))
      const double w = pi_b - pi_a;
      const double sg = sinc_f64(psi_b - psi_a, s_b * c_a - c_b * s_a);
      const double er = c_a * c_b - s_a * s_b, ei = s_a * c_b + c_a * s_b;
      Sr += w * sg * er;
      Si += w * sg * ei;
      psi_a = psi_b;
      pi_a = pi_b;
      s_a = s_b;
      c_a = c_b;
    }
    co = QN / fmax(P2, 1e-300);
  }
  const double Ur = co * cf, Ui = co * sf;
  Tr = Ur * Sr - Ui * Si;
  Ti = Ur * Si + Ui * Sr;
}

// small |Q|: the fan of tetrahedra (t, a, b, c) over the face's fan triangles, as tet_term_f64
__device__ void poly_tet_f64(const FaceP64& F, const VtxP64* V, const double* Q, double& xr, double& xi) {
  double a[3];
  for (int c = 0; c < 3; ++c) a[c] = F.g[c] + V[0].u[c];
  const double xa = Q[0] * a[0] + Q[1] * a[1] + Q[2] * a[2];
  for (int l = 1; l + 1 < F.nv; ++l) {
    double b[3], c[3];
    for (int k = 0; k < 3; ++k) {
      b[k] = F.g[k] + V[l].u[k];
      c[k] = F.g[k] + V[l + 1].u[k];
    }
    const double six_v = a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
                         a[2] * (b[0] * c[1] - b[1] * c[0]);
    const double xb = Q[0] * b[0] + Q[1] * b[1] + Q[2] * b[2];
    const double xc = Q[0] * c[0] + Q[1] * c[1] + Q[2] * c[2];
    double sr, si;
    tet_series_f64(xa, xb, xc, sr, si);
    xr += six_v * sr;
    xi += six_v * si;
  }
}

template <typename FR, typename VR>
__device__ __forceinline__ void stage_tile(const PolyTile& tl, const FR* fsrc, const VR* vsrc, FR* fdst, VR* vdst) {
  const int nfb = (tl.f1 - tl.f0) * (int)sizeof(FR) / 16;
  const int nvb = (tl.v1 - tl.v0) * (int)sizeof(VR);
  const uint4* fs = reinterpret_cast<const uint4*>(fsrc + tl.f0);
  uint4* fd = reinterpret_cast<uint4*>(fdst);
  for (int i = threadIdx.x; i < nfb; i += kBlock) fd[i] = fs[i];
  // vertex records: 4-byte words (VtxP32 is 24 B, so a tile may start off a 16-byte boundary)
  const uint32_t* vs = reinterpret_cast<const uint32_t*>(vsrc + tl.v0);
  uint32_t* vd = reinterpret_cast<uint32_t*>(vdst);
  for (int i = threadIdx.x; i < nvb / 4; i += kBlock) vd[i] = vs[i];
}

__global__ __launch_bounds__(kBlock) void fwdpoly_fp64_kernel(FwdArgs a, PolyArgs p) {
  __shared__ FaceP64 fh[kTileFP];
  __shared__ VtxP64 vr[kTileV];
  const int64_t qi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = qi < a.nq;
  double Q[3] = {0.0, 0.0, 0.0};
  if (active) load_q3(a.q, a.qdtype, a.perm ? (int64_t)a.perm[qi] : qi, Q);
  const double Q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
  const bool small = sqrt(Q2) * a.info[0].R < a.tau0;
  const int64_t t_begin = (int64_t)blockIdx.y * p.tiles_per_split;
  const int64_t t_end = min(p.ntiles, t_begin + p.tiles_per_split);
  double xr = 0.0, xi = 0.0;
  for (int64_t t = t_begin; t < t_end; ++t) {
    const PolyTile tl = p.tiles[t];
    __syncthreads();
    stage_tile(tl, p.f64, p.v64, fh, vr);
    __syncthreads();
    for (int j = 0; j < tl.f1 - tl.f0; ++j) {
      const FaceP64 F = fh[j];
      const VtxP64* V = vr + (F.v0 - tl.v0);
      if (!small) {
        double Tr, Ti;
        poly_term_f64(F, V, Q, Tr, Ti);
        xr += Tr;
        xi += Ti;
      } else {
        poly_tet_f64(F, V, Q, xr, xi);
      }
    }
  }
  if (active) store_stream(a.partial + (int64_t)blockIdx.y * a.nq + qi, make_double2(xr, xi));
}

// ---------------------------------------------------------------------------
// FP32-compensated: the vertex loop in binary32 turns (hardware sin / cos),
// the face origin phase reduced in binary64, the fan series from the binary32
// phases (each fan triangle in binary32 through the fitted polynomial of exp(ix)
// when its centred phases stay within its range, in binary64 otherwise; chosen
// per lane and triangle), Kahan sums across tiles.
// ---------------------------------------------------------------------------
__device__ void poly_series_fp32c(const FaceP32& F, const VtxP32* V, float s1, float s2, float QN, float r,
                                  float& Tr, float& Ti) {
  constexpr double kFourPi = 12.566370614359172954;
  const VtxP32 v0 = V[0];
  const double pa = kFourPi * (double)(s1 * v0.ga + s2 * v0.de);  // Q.u_0 in radians
  double jr = 0.0, ji = 0.0;
  for (int l = 1; l + 1 < F.nv; ++l) {
    const VtxP32 vb = V[l], vc = V[l + 1];
    const double pb = kFourPi * (double)(s1 * vb.ga + s2 * vb.de);
    const double pc = kFourPi * (double)(s1 * vc.ga + s2 * vc.de);
    const double two_a = ((double)vb.x - v0.x) * ((double)vc.y - v0.y) - ((double)vc.x - v0.x) * ((double)vb.y - v0.y);
    const double qt = (pa + pb + pc) / 3.0;
    const float da = (float)(pa - qt), db = (float)(pb - qt);
    double sr, si, st, ct;
    if (fmaxf(fabsf(da), fmaxf(fabsf(db), fabsf(da + db))) <= FacePoly::M && fabs(qt) <= 1.0) {
      // small phases: binary32 face integral and binary32 sine / cosine of the fan triangle's centroid phase
      float fr, fi;
      face_integral_poly<FacePoly>(da, db, fr, fi);
      const float q32 = (float)qt * kInv2PiF;
      sr = fr;
      si = fi;
      st = sin_turns(q32);
      ct = cos_turns(q32);
    } else {
      face_series_f64(pa - qt, pb - qt, pc - qt, sr, si, 1e-10);
      sincos(qt, &st, &ct);
    }
    jr += two_a * (ct * sr - st * si);
    ji += two_a * (ct * si + st * sr);
  }
  // T = -i (Q.n) exp(2 pi i r) J
  const double cf = (double)cos_turns(r), sf = (double)sin_turns(r);
  const double qn = (double)QN * (double)F.invN;
  const double ur = cf * jr - sf * ji, ui = cf * ji + sf * jr;
  Tr = (float)(qn * ui);
  Ti = (float)(-qn * ur);
}

template <int NQ>
__device__ __forceinline__ void poly_tile_fp32c(const FaceP32* fh, const VtxP32* vr, int nfaces, int vbase,
                                                const float* qx, const float* qy, const float* qz, const float* Q2,
                                                const double (*Qd)[3], const bool* small, float* tr, float* ti) {
  for (int j = 0; j < nfaces; ++j) {
    const FaceP32 F = fh[j];
    const VtxP32* V = vr + (F.v0 - vbase);
    float s1[NQ], s2[NQ], QN[NQ], P2[NQ], r[NQ], p0[NQ], pa[NQ], Sr[NQ], Si[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      QN[k] = qx[k] * F.N[0] + qy[k] * F.N[1] + qz[k] * F.N[2];
      s1[k] = qx[k] * F.E1[0] + qy[k] * F.E1[1] + qz[k] * F.E1[2];
      s2[k] = qx[k] * F.E2[0] + qy[k] * F.E2[1] + qz[k] * F.E2[2];
      P2[k] = s1[k] * s1[k] + s2[k] * s2[k];
      const double ph = Qd[k][0] * F.gt[0] + Qd[k][1] * F.gt[1] + Qd[k][2] * F.gt[2];
      r[k] = (float)(ph - rint(ph));
      p0[k] = s1[k] * V[0].ga + s2[k] * V[0].de;
      pa[k] = p0[k];
      Sr[k] = Si[k] = 0.0f;
    }
    for (int m = 1; m <= F.nv; ++m) {
      const VtxP32 ea = V[m - 1];                   // edge m-1 -> m
      const VtxP32 vb = V[m < F.nv ? m : 0];
      float pb[NQ], x[NQ], c[NQ], big = 0.0f;
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        pb[k] = m < F.nv ? s1[k] * vb.ga + s2[k] * vb.de : p0[k];
        x[k] = pb[k] - pa[k];
        c[k] = sinc2pi_poly(x[k]);
        big = fmaxf(big, fabsf(x[k]));
      }
      // the sine quotient for this lane's edges beyond the polynomial's range (a lane's value does not
      // depend on the other lanes of its wavefront)
      if (__builtin_expect(big > kSincPolyMax, 0)) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) c[k] = sinc2pi_wide(x[k], c[k]);
      }
#pragma unroll
      for (int k = 0; k < NQ; ++k) {
        const float w = s2[k] * ea.al + s1[k] * ea.be;
        const float aw = w * c[k];
        const float t = r[k] + pa[k] + pb[k];
        Sr[k] += aw * cos_turns(t);
        Si[k] += aw * sin_turns(t);
        pa[k] = pb[k];
      }
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const float co = QN[k] * rcp_f(fmaxf(P2[k], 1e-30f));
      float Tr = co * Sr[k], Ti = co * Si[k];
      if (P2[k] < fmaxf(F.thr, F.kap * Q2[k]) && !small[k]) poly_series_fp32c(F, V, s1[k], s2[k], QN[k], r[k], Tr, Ti);
      tr[k] += Tr;
      ti[k] += Ti;
    }
  }
}

__global__ __launch_bounds__(kBlock) void fwdpoly_fp32c_kernel(FwdArgs a, PolyArgs p) {
  __shared__ FaceP32 fh[kTileFP];
  __shared__ VtxP32 vr[kTileV];
  const int64_t qbase = (int64_t)blockIdx.x * (kBlock * kQPTPoly) + threadIdx.x;
  const double R = a.info[0].R;
  double Qd[kQPTPoly][3];
  float qx[kQPTPoly], qy[kQPTPoly], qz[kQPTPoly], Q2[kQPTPoly];
  bool small[kQPTPoly], active[kQPTPoly];
  bool any_small = false;
#pragma unroll
  for (int k = 0; k < kQPTPoly; ++k) {
    const int64_t qi = qbase + (int64_t)k * kBlock;
    active[k] = qi < a.nq;
    Qd[k][0] = Qd[k][1] = Qd[k][2] = 0.0;
    if (active[k]) load_q3(a.q, a.qdtype, a.perm ? (int64_t)a.perm[qi] : qi, Qd[k]);
    qx[k] = (float)Qd[k][0];
    qy[k] = (float)Qd[k][1];
    qz[k] = (float)Qd[k][2];
    Q2[k] = qx[k] * qx[k] + qy[k] * qy[k] + qz[k] * qz[k];
    const double Q2d = Qd[k][0] * Qd[k][0] + Qd[k][1] * Qd[k][1] + Qd[k][2] * Qd[k][2];
    small[k] = sqrt(Q2d) * R < a.tau0;
    any_small |= small[k];
  }
  const int64_t t_begin = (int64_t)blockIdx.y * p.tiles_per_split;
  const int64_t t_end = min(p.ntiles, t_begin + p.tiles_per_split);
  float sr[kQPTPoly], si[kQPTPoly], cr[kQPTPoly], ci[kQPTPoly];
  double xr[kQPTPoly], xi[kQPTPoly];
#pragma unroll
  for (int k = 0; k < kQPTPoly; ++k) sr[k] = si[k] = cr[k] = ci[k] = 0.0f, xr[k] = xi[k] = 0.0;
  for (int64_t t = t_begin; t < t_end; ++t) {
    const PolyTile tl = p.tiles[t];
    __syncthreads();
    stage_tile(tl, p.f32, p.v32, fh, vr);
    __syncthreads();
    float tr[kQPTPoly], ti[kQPTPoly];
#pragma unroll
    for (int k = 0; k < kQPTPoly; ++k) tr[k] = ti[k] = 0.0f;
    poly_tile_fp32c<kQPTPoly>(fh, vr, tl.f1 - tl.f0, tl.v0, qx, qy, qz, Q2, Qd, small, tr, ti);
#pragma unroll
    for (int k = 0; k < kQPTPoly; ++k) {
      kahan_add(sr[k], cr[k], tr[k]);
      kahan_add(si[k], ci[k], ti[k]);
    }
    if (any_small) {
#pragma unroll
      for (int k = 0; k < kQPTPoly; ++k)
        if (small[k])
          for (int f = tl.f0; f < tl.f1; ++f) {
            const FaceP64 F = p.f64[f];
            poly_tet_f64(F, p.v64 + F.v0, Qd[k], xr[k], xi[k]);
          }
    }
  }
#pragma unroll
  for (int k = 0; k < kQPTPoly; ++k) {
    if (active[k]) {
      const double2 v = small[k] ? make_double2(xr[k], xi[k])
                                 : make_double2((double)sr[k] - (double)cr[k], (double)si[k] - (double)ci[k]);
      store_stream(a.partial + (int64_t)blockIdx.y * a.nq + qbase + (int64_t)k * kBlock, v);
    }
  }
}

}  // namespace

hipError_t launch_fwdpoly_fp64(const FwdArgs& a, const PolyArgs& p, hipStream_t s) {
  dim3 grid((unsigned)((a.nq + kBlock - 1) / kBlock), (unsigned)a.splits);
  fwdpoly_fp64_kernel<<<grid, kBlock, 0, s>>>(a, p);
  return hipGetLastError();
}

hipError_t launch_fwdpoly_fp32c(const FwdArgs& a, const PolyArgs& p, hipStream_t s) {
  dim3 grid((unsigned)((a.nq + kBlock * kQPTPoly - 1) / (kBlock * kQPTPoly)), (unsigned)a.splits);
  fwdpoly_fp32c_kernel<<<grid, kBlock, 0, s>>>(a, p);
  return hipGetLastError();
}

}  // namespace pft
