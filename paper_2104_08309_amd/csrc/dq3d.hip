// grad_Q F and closed regions of constant density.
//
// dq3d_*_kernel: the forward's layout (a Q tile per block, faces streamed
// through LDS, the face range split over blockIdx.y, Q visited in Morton
// order) evaluating, per Q, the face sums A (3 complex) and B of dq_terms.h;
// lanes with |Q| R < tau sum the tetrahedron fan instead. Each split writes
// its four binary64 partials.
//
// Finish kernels: per Q and per region j (the splits of a region cover only
// its faces), the partials of the region's splits are added in a fixed order,
// giving F_j and grad F_j; the density-weighted sums F = sum_j rho_j F_j and
// dL/dQ = Re(conj(g) sum_j rho_j grad F_j) are formed in registers, and
// dL/drho_j = sum_Q Re(conj(g) F_j) is reduced per block (binary64, fixed
// order) and then over blocks.
#include "dq_terms.h"
#include "fwd_terms.h"

namespace pft {
namespace {

constexpr int kFinishBlock = 256;

__device__ __forceinline__ void split_range(const DqArgs& a, int64_t& b, int64_t& e) {
  if (a.split_face) {
    b = a.split_face[blockIdx.y];
    e = a.split_face[blockIdx.y + 1];
  } else {
    b = (int64_t)blockIdx.y * a.faces_per_split;
    e = min(a.nf, b + a.faces_per_split);
  }
}

__device__ __forceinline__ double2* dq_slot(const DqArgs& a, int comp, int64_t qi) {
  return a.partial + ((int64_t)blockIdx.y * 4 + comp) * a.nq + qi;
}

// ---------------------------------------------------------------------------
// binary64: one Q per thread; face records and their Gram matrices in LDS
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void dq3d_fp64_kernel(DqArgs a) {
  __shared__ Face64 tile[kTileF];
  __shared__ double gtile[kTileF][8];
  const int64_t qi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = qi < a.nq;
  double Q[3] = {0.0, 0.0, 0.0};
  if (active) load_q3(a.q, a.qdtype, a.perm ? (int64_t)a.perm[qi] : qi, Q);
  const double4 geo = a.split_geo ? a.split_geo[blockIdx.y] : make_double4(0.0, 0.0, 0.0, a.info[0].R);
  const double o[3] = {geo.x, geo.y, geo.z};
  const bool small = sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]) * geo.w < a.tau;
  int64_t f_begin, f_end;
  split_range(a, f_begin, f_end);
  double Ar[3] = {0.0, 0.0, 0.0}, Ai[3] = {0.0, 0.0, 0.0}, Br = 0.0, Bi = 0.0;
  for (int64_t t0 = f_begin; t0 < f_end; t0 += kTileF) {
    const int nt = (int)min((int64_t)kTileF, f_end - t0);
    __syncthreads();
    {
      const uint4* src = reinterpret_cast<const uint4*>(a.f64 + t0);
      uint4* dst = reinterpret_cast<uint4*>(tile);
      for (int i = threadIdx.x; i < nt * (int)(sizeof(Face64) / 16); i += kBlock) dst[i] = src[i];
      const double* gs = a.gram + t0 * 8;
      for (int i = threadIdx.x; i < nt * 8; i += kBlock) gtile[i / 8][i % 8] = gs[i];
    }
    __syncthreads();
    if (!small) {
      for (int j = 0; j < nt; ++j) dq_term_f64(tile[j], gtile[j], Q, Ar, Ai, Br, Bi);
    } else {
      for (int j = 0; j < nt; ++j) dq_tet_f64(tile[j], Q, Ar, Ai, Br, Bi, o);
    }
  }
  if (small && a.split_geo) dq_apex(Q, o, Ar, Ai, Br, Bi);
  if (active) {
    for (int c = 0; c < 3; ++c) store_stream(dq_slot(a, c, qi), make_double2(Ar[c], Ai[c]));
    store_stream(dq_slot(a, 3, qi), make_double2(Br, Bi));
  }
}

// ---------------------------------------------------------------------------
// FP32C: kQPTDQ Q per thread (strided by the block size), binary32 sums per
// LDS tile, Kahan across tiles; small-|Q| lanes take the binary64 tetrahedron
// fan over the split after the tile loop.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void dq3d_fp32c_kernel(DqArgs a) {
  constexpr int P = kQPTDQ;
  __shared__ Face32B tile[kTileF];
  const int64_t qbase = (int64_t)blockIdx.x * (kBlock * P) + threadIdx.x;
  const double4 geo = a.split_geo ? a.split_geo[blockIdx.y] : make_double4(0.0, 0.0, 0.0, a.info[0].R);
  const double R = geo.w;
  const double o[3] = {geo.x, geo.y, geo.z};
  double Qd[P][3];
  float qx[P], qy[P], qz[P];
  bool small[P], active[P];
  bool any_small = false;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int64_t qi = qbase + (int64_t)k * kBlock;
    active[k] = qi < a.nq;
    Qd[k][0] = Qd[k][1] = Qd[k][2] = 0.0;
    if (active[k]) load_q3(a.q, a.qdtype, a.perm ? (int64_t)a.perm[qi] : qi, Qd[k]);
    qx[k] = (float)Qd[k][0];
    qy[k] = (float)Qd[k][1];
    qz[k] = (float)Qd[k][2];
    small[k] = sqrt(Qd[k][0] * Qd[k][0] + Qd[k][1] * Qd[k][1] + Qd[k][2] * Qd[k][2]) * R < a.tau;
    any_small |= small[k];
  }
  int64_t f_begin, f_end;
  split_range(a, f_begin, f_end);
  // running sums and compensations: A_x, A_y, A_z, B as (re, im) pairs
  float sum[P][8], cmp[P][8];
#pragma unroll
  for (int k = 0; k < P; ++k)
#pragma unroll
    for (int c = 0; c < 8; ++c) sum[k][c] = cmp[k][c] = 0.0f;
  for (int64_t t0 = f_begin; t0 < f_end; t0 += kTileF) {
    const int nt = (int)min((int64_t)kTileF, f_end - t0);
    __syncthreads();
    {
      const uint4* src = reinterpret_cast<const uint4*>(a.f32 + t0);
      uint4* dst = reinterpret_cast<uint4*>(tile);
      for (int i = threadIdx.x; i < nt * (int)(sizeof(Face32B) / 16); i += kBlock) dst[i] = src[i];
    }
    __syncthreads();
    float Ar[P][3], Ai[P][3], Br[P], Bi[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      Ar[k][0] = Ar[k][1] = Ar[k][2] = Ai[k][0] = Ai[k][1] = Ai[k][2] = 0.0f;
      Br[k] = Bi[k] = 0.0f;
    }
    for (int j = 0; j < nt; ++j) {
      const Face32B f = tile[j];
#pragma unroll
      for (int k = 0; k < P; ++k) dq_term_fp32c(f, qx[k], qy[k], qz[k], Qd[k], Ar[k], Ai[k], Br[k], Bi[k]);
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        kahan_add(sum[k][2 * c], cmp[k][2 * c], Ar[k][c]);
        kahan_add(sum[k][2 * c + 1], cmp[k][2 * c + 1], Ai[k][c]);
      }
      kahan_add(sum[k][6], cmp[k][6], Br[k]);
      kahan_add(sum[k][7], cmp[k][7], Bi[k]);
    }
  }
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int64_t qi = qbase + (int64_t)k * kBlock;
    double v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = (double)sum[k][c] - (double)cmp[k][c];
    if (any_small && small[k]) {
      double Gr[3] = {0.0, 0.0, 0.0}, Gi[3] = {0.0, 0.0, 0.0}, Fr = 0.0, Fi = 0.0;
      for (int64_t f = f_begin; f < f_end; ++f) dq_tet_f64(a.f64[f], Qd[k], Gr, Gi, Fr, Fi, o);
      if (a.split_geo) dq_apex(Qd[k], o, Gr, Gi, Fr, Fi);
      for (int c = 0; c < 3; ++c) v[2 * c] = Gr[c], v[2 * c + 1] = Gi[c];
      v[6] = Fr;
      v[7] = Fi;
    }
    if (active[k])
      for (int c = 0; c < 4; ++c) store_stream(dq_slot(a, c, qi), make_double2(v[2 * c], v[2 * c + 1]));
  }
}

// ---------------------------------------------------------------------------
// finish kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 load_cot(const void* g, int c128, int64_t i) {
  if (c128) return static_cast<const double2*>(g)[i];
  const float2 v = static_cast<const float2*>(g)[i];
  return make_double2(v.x, v.y);
}

__device__ __forceinline__ void store_complex(void* p, int c128, int64_t i, double re, double im) {
  if (c128)
    static_cast<double2*>(p)[i] = make_double2(re, im);
  else
    static_cast<float2*>(p)[i] = make_float2((float)re, (float)im);
}

__global__ __launch_bounds__(kFinishBlock) void regions_finish_kernel(FwdArgs a, RegionArgs r, int out_c128) {
  __shared__ double lds[kFinishBlock / 64];
  const int64_t qi = (int64_t)blockIdx.x * kFinishBlock + threadIdx.x;
  const bool valid = qi < a.nq;
  const int64_t dst = valid ? (a.perm ? (int64_t)a.perm[qi] : qi) : 0;
  double Q[3] = {0.0, 0.0, 0.0};
  if (valid) load_q3(a.q, a.qdtype, dst, Q);
  const MeshInfo mi = a.info[0];
  const double Q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
  const double qabs = sqrt(Q2);
  double st, ct;
  sincos(Q[0] * mi.t[0] + Q[1] * mi.t[1] + Q[2] * mi.t[2], &st, &ct);
  const double2 g = (valid && r.grad_out) ? load_cot(r.grad_out, out_c128, dst) : make_double2(0.0, 0.0);
  double Fr = 0.0, Fi = 0.0;
  for (int j = 0; j < r.nreg; ++j) {
    double xr = 0.0, xi = 0.0;
    if (valid)
      for (int s = r.region_split[j]; s < r.region_split[j + 1]; ++s) {
        const double2 v = load_stream(a.partial + (int64_t)s * a.nq + qi);
        xr += v.x;
        xi += v.y;
      }
    if (!(qabs * (r.region_R ? r.region_R[j] : mi.R) < a.tau0)) {  // this region's small-|Q| test
      xr /= Q2;
      xi /= Q2;
    }
    if (!out_c128 && fp32c_phase_out_of_range(qabs, mi)) xr = xi = quiet_nan();  // beyond the FP32C phase range
    const double fr = ct * xr - st * xi, fi = ct * xi + st * xr;
    if (valid && r.out_regions) store_complex(r.out_regions, out_c128, (int64_t)j * a.nq + dst, fr, fi);
    const double rho = r.rho[j];
    Fr += rho * fr;
    Fi += rho * fi;
    if (r.rho_part) {
      const double t = block_total<kFinishBlock>(g.x * fr + g.y * fi, lds);  // Re(conj(g) F_j)
      if (threadIdx.x == 0) r.rho_part[(int64_t)blockIdx.x * r.nreg + j] = t;
    }
  }
  if (!valid) return;
  if (a.out) store_complex(a.out, out_c128, dst, Fr, Fi);
  if (a.intensity) {
    if (out_c128)
      static_cast<double*>(a.intensity)[dst] = Fr * Fr + Fi * Fi;
    else
      static_cast<float*>(a.intensity)[dst] = (float)(Fr * Fr + Fi * Fi);
  }
}

__global__ __launch_bounds__(kFinishBlock) void dq_finish_kernel(DqArgs a, RegionArgs r, int go_c128, void* grad_q,
                                                                 int gq_dtype) {
  __shared__ double lds[kFinishBlock / 64];
  const int64_t qi = (int64_t)blockIdx.x * kFinishBlock + threadIdx.x;
  const bool valid = qi < a.nq;
  const int64_t dst = valid ? (a.perm ? (int64_t)a.perm[qi] : qi) : 0;
  double Q[3] = {0.0, 0.0, 0.0};
  if (valid) load_q3(a.q, a.qdtype, dst, Q);
  const MeshInfo mi = a.info[0];
  const double Q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
  const double qabs = sqrt(Q2);
  double st, ct;
  sincos(Q[0] * mi.t[0] + Q[1] * mi.t[1] + Q[2] * mi.t[2], &st, &ct);
  const double2 g = valid ? load_cot(r.grad_out, go_c128, dst) : make_double2(0.0, 0.0);
  double gq[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < r.nreg; ++j) {
    double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (valid)
      for (int s = r.region_split[j]; s < r.region_split[j + 1]; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double2 x = load_stream(a.partial + ((int64_t)s * 4 + c) * a.nq + qi);
          v[2 * c] += x.x;
          v[2 * c + 1] += x.y;
        }
    // centred F_c and grad F_c
    double fcr, fci, gcr[3], gci[3];
    if (qabs * (r.region_R ? r.region_R[j] : mi.R) < a.tau) {  // this region's small-|Q| test
      fcr = v[6];
      fci = v[7];
      for (int c = 0; c < 3; ++c) gcr[c] = v[2 * c], gci[c] = v[2 * c + 1];
    } else {
      const double iq2 = 1.0 / Q2;
      fcr = v[7] * iq2;  // -i B / |Q|^2
      fci = -v[6] * iq2;
      for (int c = 0; c < 3; ++c) {
        // (A + i Q B / |Q|^2) / |Q|^2
        gcr[c] = (v[2 * c] - Q[c] * v[7] * iq2) * iq2;
        gci[c] = (v[2 * c + 1] + Q[c] * v[6] * iq2) * iq2;
      }
    }
    if (!go_c128 && fp32c_phase_out_of_range(qabs, mi)) {  // beyond the FP32C phase range
      fcr = fci = quiet_nan();
      for (int c = 0; c < 3; ++c) gcr[c] = gci[c] = quiet_nan();
    }
    const double rho = r.rho[j];
    for (int c = 0; c < 3; ++c) {
      // grad F = exp(iQ.t) (grad F_c + i t F_c)
      const double ur = gcr[c] - mi.t[c] * fci, ui = gci[c] + mi.t[c] * fcr;
      const double wr = ct * ur - st * ui, wi = ct * ui + st * ur;
      gq[c] += rho * (g.x * wr + g.y * wi);
    }
    if (r.rho_part) {
      const double fr = ct * fcr - st * fci, fi = ct * fci + st * fcr;
      const double t = block_total<kFinishBlock>(g.x * fr + g.y * fi, lds);
      if (threadIdx.x == 0) r.rho_part[(int64_t)blockIdx.x * r.nreg + j] = t;
    }
  }
  if (!valid || !grad_q) return;
  for (int c = 0; c < 3; ++c) {
    if (gq_dtype == PFT_F64)
      static_cast<double*>(grad_q)[dst * 3 + c] = gq[c];
    else
      static_cast<float*>(grad_q)[dst * 3 + c] = (float)gq[c];
  }
}

// One block per region: the per-block sums in a fixed order.
__global__ __launch_bounds__(kFinishBlock) void rho_reduce_kernel(const double* part, int64_t nblocks, int nreg,
                                                                  double* out) {
  __shared__ double lds[kFinishBlock / 64];
  const int j = blockIdx.x;
  double v = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += kFinishBlock) v += part[b * nreg + j];
  v = block_total<kFinishBlock>(v, lds);
  if (threadIdx.x == 0) out[j] = v;
}

// One block per region: the mean of its face centroids, then the largest corner distance from it.
__global__ __launch_bounds__(kFinishBlock) void region_radii_kernel(const Face64* f64, const int64_t* off,
                                                                    double* region_R, double4* region_geo) {
  __shared__ double lds[kFinishBlock / 64];
  const int j = blockIdx.x;
  const int64_t b = off[j], e = off[j + 1];
  double c[3];
  for (int k = 0; k < 3; ++k) {
    double v = 0.0;
    for (int64_t m = b + threadIdx.x; m < e; m += kFinishBlock) v += f64[m].g[k];
    c[k] = block_total<kFinishBlock>(v, lds) / (double)max<int64_t>(e - b, 1);
  }
  double r2 = 0.0;
  for (int64_t m = b + threadIdx.x; m < e; m += kFinishBlock) {
    const Face64& f = f64[m];
    for (int q = 0; q < 3; ++q) {
      double d2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double u = q == 0 ? f.u0[k] : (q == 1 ? f.u1[k] : -f.u0[k] - f.u1[k]);
        const double x = f.g[k] + u - c[k];
        d2 += x * x;
      }
      r2 = fmax(r2, d2);
    }
  }
  // block maximum (fixed order)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) r2 = fmax(r2, __shfl_xor(r2, o, 64));
  __syncthreads();
  if (lane == 0) lds[wave] = r2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int w = 0; w < kFinishBlock / 64; ++w) mx = fmax(mx, lds[w]);
    region_R[j] = sqrt(mx);
    region_geo[j] = make_double4(c[0], c[1], c[2], sqrt(mx));
  }
}

__global__ __launch_bounds__(256) void split_radii_kernel(const int32_t* region_split, int nreg,
                                                          const double4* region_geo, double4* split_geo) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nreg) return;
  for (int sp = region_split[j]; sp < region_split[j + 1]; ++sp) split_geo[sp] = region_geo[j];
}

__global__ __launch_bounds__(256) void face_weights_kernel(const int64_t* off, int nreg, const double* rho,
                                                           int64_t nf, double* w) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  // the region j with off[j] <= m < off[j+1] (empty regions are skipped by the search)
  int lo = 0, hi = nreg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (off[mid] <= m)
      lo = mid;
    else
      hi = mid - 1;
  }
  w[m] = rho[lo];
}

}  // namespace

inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

int64_t finish_blocks(int64_t nq) { return (nq + kFinishBlock - 1) / kFinishBlock; }

hipError_t launch_dq3d_fp64(const DqArgs& a, hipStream_t s) {
  if (a.splits <= 0 || a.nq <= 0) return hipSuccess;
  dim3 grid((unsigned)((a.nq + kBlock - 1) / kBlock), (unsigned)a.splits);
  dq3d_fp64_kernel<<<grid, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_dq3d_fp32c(const DqArgs& a, hipStream_t s) {
  if (a.splits <= 0 || a.nq <= 0) return hipSuccess;
  dim3 grid((unsigned)((a.nq + kBlock * kQPTDQ - 1) / (kBlock * kQPTDQ)), (unsigned)a.splits);
  dq3d_fp32c_kernel<<<grid, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_regions_finish(const FwdArgs& a, const RegionArgs& r, int out_c128, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  regions_finish_kernel<<<(unsigned)finish_blocks(a.nq), kFinishBlock, 0, s>>>(a, r, out_c128);
  return hipGetLastError();
}

hipError_t launch_dq_finish(const DqArgs& a, const RegionArgs& r, int go_c128, void* grad_q, int gq_dtype,
                            hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  dq_finish_kernel<<<(unsigned)finish_blocks(a.nq), kFinishBlock, 0, s>>>(a, r, go_c128, grad_q, gq_dtype);
  return hipGetLastError();
}

hipError_t launch_rho_reduce(const double* rho_part, int64_t nblocks, int nreg, double* grad_rho, hipStream_t s) {
  if (nreg <= 0) return hipSuccess;
  rho_reduce_kernel<<<(unsigned)nreg, kFinishBlock, 0, s>>>(rho_part, nblocks, nreg, grad_rho);
  return hipGetLastError();
}

hipError_t launch_region_radii(const Face64* f64, const int64_t* d_region_off, int nreg,
                               const int32_t* d_region_split, double* region_R, double4* region_geo,
                               double4* split_geo, hipStream_t s) {
  if (nreg <= 0) return hipSuccess;
  region_radii_kernel<<<(unsigned)nreg, kFinishBlock, 0, s>>>(f64, d_region_off, region_R, region_geo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  split_radii_kernel<<<(unsigned)((nreg + 255) / 256), 256, 0, s>>>(d_region_split, nreg, region_geo, split_geo);
  return hipGetLastError();
}

hipError_t launch_face_weights(const int64_t* d_region_off, int nreg, const double* rho, int64_t nf, double* w,
                               hipStream_t s) {
  if (nf <= 0 || nreg <= 0) return hipSuccess;
  face_weights_kernel<<<grid_for(nf), 256, 0, s>>>(d_region_off, nreg, rho, nf, w);
  return hipGetLastError();
}

}  // namespace pft
