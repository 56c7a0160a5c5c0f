// Adjoint of the 3D transform with respect to the vertices.
//
// Moving the closed surface with a velocity field changes F(Q) by the surface
// integral of exp(iQ.r) (velocity . n) dA (transport theorem applied to the
// volume integral that defines F). A vertex v_k moves the points of each
// incident triangle with its barycentric weight lambda_k, so
//   dF/dv_k = sum_{m ∋ k} n_m B_{m,k},   B_{m,k} = integral over m of lambda_k exp(iQ.r) dA,
// and for a real loss with g(Q) = dL/dReF + i dL/dImF:
//   dL/dv_k = sum_{m ∋ k} N_m R_{m,k},   R_{m,k} = Re sum_Q conj(g(Q)) B_{m,k}(Q) / |N_m|.
//
// Writing Bt_k = B_{m,k} / |N_m| = exp(iQ.g) Y_k, Y_k is evaluated either
//  (series)    Y_k = sum_n i^n h_n(delta_a, delta_b, delta_c, delta_k) / (n+3)!,
//              the barycentric moment of the simplex (node k doubled); the binary32
//              form replaces 1/n! by the coefficients of a polynomial of exp(ix)
//              fitted on the lanes' phase range and stops at its degree, or
//  (edge form) from lambda_k = 1/3 + beta_k.(r - g), beta_k = N x d_{k+1} / |N|^2,
//              and the centred face integral J_c = i |N| S / |P|^2 differentiated in Q:
//              |P|^2 Y_k = (i/2) S + sum_l (d_{k+1}.d_l) sinc_l e_l
//                          + (w_{k-1} sinc'_{k-1} e_{k-1} - w_k sinc'_k e_k) / 2
//                          - (i/2) w_{k+1} sinc_{k+1} e_{k+1} - 2 S w_{k+1} / |P|^2,
//              with w_l = P.d_l, e_l = exp(-i psi_{l+2}), S = sum_l w_l sinc_l e_l.
// The series is used where |Q_perp| L is small (it has no cancellation there;
// the edge form cancels like 1/(|Q_perp| L)^2).
//
// Layout: a block owns a tile of faces (records in LDS) and loops over a
// range of Q (a Q-split), kQPTB Q per thread per pass; the grid is one-
// dimensional over (face tile, Q-split) pairs (adj_block).
// Each thread adds its weights to private slots in LDS (one per face and
// corner; binary64 or binary32 by form), and a fixed-order binary64 block sum
// at the end writes the per-split partials. The Q list is reordered and paired
// with its cotangent g exp(-iQ.t) beforehand (qorder.hip).
#include <hipcub/hipcub.hpp>

#include "adj_terms.h"

namespace pft {
namespace {

// (face tile, Q-split) of this block. Blocks go to the dies in turn (block b to die b mod kXcds); when the
// split count is a multiple of kXcds, each die takes its own qsplits / kXcds Q-splits across all face tiles,
// so each Q record is fetched into one die's L2 only (face tile fastest within a die).
__device__ __forceinline__ void adj_block(const BwdArgs& a, int64_t ftiles, int64_t& ft, int64_t& qs) {
  const int64_t b = blockIdx.x;
  if (a.qsplits % kXcds == 0) {
    const int64_t rank = b / kXcds;
    ft = rank % ftiles;
    qs = (b % kXcds) * (a.qsplits / kXcds) + rank / ftiles;
  } else {
    ft = b % ftiles;
    qs = b / ftiles;
  }
}

__global__ __launch_bounds__(kBlock) void bwd3d_fp64_kernel(BwdArgs a, const double* gram) {
  __shared__ Face64 tile[kTileFB];
  __shared__ double gtile[kTileFB][8];
  __shared__ double acc[kTileFB * 3][kBlock];
  const int tid = threadIdx.x;
  int64_t ft, qs;
  adj_block(a, (a.nf + kTileFB - 1) / kTileFB, ft, qs);
  const int64_t f0 = ft * kTileFB;
  const int nt = (int)min((int64_t)kTileFB, a.nf - f0);
  for (int i = tid; i < nt * (int)(sizeof(Face64) / 16); i += kBlock)
    reinterpret_cast<uint4*>(tile)[i] = reinterpret_cast<const uint4*>(a.f64 + f0)[i];
  for (int i = tid; i < nt * 8; i += kBlock) gtile[i / 8][i % 8] = gram[(f0 + i / 8) * 8 + i % 8];
  for (int v = 0; v < nt * 3; ++v) acc[v][tid] = 0.0;
  __syncthreads();
  const int64_t qb = qs * a.q_per_split;
  const int64_t qe = min(a.nq, qb + a.q_per_split);
  adj_tile_f64(tile, gtile, nt, qb, qe, a.rec64, acc);
  __syncthreads();
  adj_block_sum(acc, nt, a.partial + (qs * a.nf + f0) * 3);
}

__global__ __launch_bounds__(kBlock) void bwd3d_fp32c_kernel(BwdArgs a) {
  __shared__ Face32B tile[kTileFB32];
  __shared__ float acc[kTileFB32 * 3][kBlock];
  const int tid = threadIdx.x;
  int64_t ft, qs;
  adj_block(a, (a.nf + kTileFB32 - 1) / kTileFB32, ft, qs);
  const int64_t f0 = ft * kTileFB32;
  const int nt = (int)min((int64_t)kTileFB32, a.nf - f0);
  for (int i = tid; i < nt * (int)(sizeof(Face32B) / 16); i += kBlock)
    reinterpret_cast<uint4*>(tile)[i] = reinterpret_cast<const uint4*>(a.f32 + f0)[i];
  for (int v = 0; v < nt * 3; ++v) acc[v][tid] = 0.0f;
  __syncthreads();
  const int64_t qb = qs * a.q_per_split;
  const int64_t qe = min(a.nq, qb + a.q_per_split);
  adj_tile_fp32c(tile, nt, qb, qe, a.rec, acc);
  __syncthreads();
  adj_block_sum(acc, nt, a.partial + (qs * a.nf + f0) * 3);
}

__global__ __launch_bounds__(256) void gram64_kernel(const Face64* f64, int64_t nf, double* gram) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  const Face64 f = f64[m];
  double d0[3], d1[3], d2[3];
  for (int k = 0; k < 3; ++k) {
    d0[k] = f.u1[k] - f.u0[k];
    d1[k] = -f.u0[k] - 2.0 * f.u1[k];
    d2[k] = 2.0 * f.u0[k] + f.u1[k];
  }
  auto dot = [](const double* x, const double* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
  double* G = gram + m * 8;
  G[0] = dot(d0, d0);
  G[1] = dot(d1, d1);
  G[2] = dot(d2, d2);
  G[3] = dot(d0, d1);
  G[4] = dot(d1, d2);
  G[5] = dot(d2, d0);
  G[6] = G[7] = 0.0;
}

// ---------------------------------------------------------------------------
// reduction over splits, per-corner vectors, vertex gather
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void face_contrib_kernel(const double* partial, int qsplits, const Face64* f64,
                                                           const double* face_w, int64_t nf, double* contrib) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // corner slot 3m + k
  if (i >= nf * 3) return;
  const int64_t m = i / 3;
  double R = 0.0;
  for (int s = 0; s < qsplits; ++s) R += partial[(int64_t)s * nf * 3 + i];
  if (face_w) R *= face_w[m];  // density of the face's region
  const Face64& f = f64[m];
  contrib[i * 3 + 0] = f.N[0] * R;
  contrib[i * 3 + 1] = f.N[1] * R;
  contrib[i * 3 + 2] = f.N[2] * R;
}

__global__ __launch_bounds__(256) void incidence_keys_kernel(const int32_t* tris, int64_t nf, const int64_t* vert_off,
                                                             const int32_t* face_mesh, int64_t nv_total,
                                                             uint32_t* keys, uint32_t* vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf * 3) return;
  const int64_t m = i / 3;
  int64_t base = 0, nv = nv_total;
  if (vert_off) {
    const int32_t mesh = face_mesh[m];
    base = vert_off[mesh];
    nv = vert_off[mesh + 1] - base;
  }
  const int32_t a = tris[3 * m], b = tris[3 * m + 1], c = tris[3 * m + 2];
  const bool ok = a >= 0 && b >= 0 && c >= 0 && a < nv && b < nv && c < nv;
  const int32_t v = tris[i];
  keys[i] = ok ? (uint32_t)(base + v) : (uint32_t)nv_total;
  vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void gather_kernel(const uint32_t* keys, const uint32_t* vals, int64_t nslots,
                                                     const double* contrib, int64_t nv, void* grad, int vdtype) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  // [lo, hi) = slots whose key is v (keys sorted ascending)
  int64_t lo = 0, hi = nslots;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (keys[mid] < (uint32_t)v) lo = mid + 1; else hi = mid;
  }
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int64_t i = lo; i < nslots && keys[i] == (uint32_t)v; ++i) {
    const int64_t s = vals[i];
    gx += contrib[s * 3 + 0];
    gy += contrib[s * 3 + 1];
    gz += contrib[s * 3 + 2];
  }
  if (vdtype == PFT_F64) {
    double* g = static_cast<double*>(grad) + v * 3;
    g[0] = gx; g[1] = gy; g[2] = gz;
  } else {
    float* g = static_cast<float*>(grad) + v * 3;
    g[0] = (float)gx; g[1] = (float)gy; g[2] = (float)gz;
  }
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_gram64(const Face64* f64, int64_t nf, double* gram, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  gram64_kernel<<<grid_for(nf), 256, 0, s>>>(f64, nf, gram);
  return hipGetLastError();
}

hipError_t launch_bwd3d_fp64(const BwdArgs& a, const double* gram, hipStream_t s) {
  const int64_t blocks = (a.nf + kTileFB - 1) / kTileFB * a.qsplits;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  bwd3d_fp64_kernel<<<(unsigned)blocks, kBlock, 0, s>>>(a, gram);
  return hipGetLastError();
}

hipError_t launch_bwd3d_fp32c(const BwdArgs& a, hipStream_t s) {
  const int64_t blocks = (a.nf + kTileFB32 - 1) / kTileFB32 * a.qsplits;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  bwd3d_fp32c_kernel<<<(unsigned)blocks, kBlock, 0, s>>>(a);
  return hipGetLastError();
}


hipError_t launch_bwd_face_contrib(const double* partial, int qsplits, const Face64* f64, const double* face_w,
                                   int64_t nf, double* contrib, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  face_contrib_kernel<<<grid_for(nf * 3), 256, 0, s>>>(partial, qsplits, f64, face_w, nf, contrib);
  return hipGetLastError();
}

hipError_t launch_incidence_keys(const int32_t* tris, int64_t nf, const int64_t* d_vert_off,
                                 const int32_t* d_face_mesh, int64_t nv_total, uint32_t* keys, uint32_t* vals,
                                 hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  incidence_keys_kernel<<<grid_for(nf * 3), 256, 0, s>>>(tris, nf, d_vert_off, d_face_mesh, nv_total, keys, vals);
  return hipGetLastError();
}

hipError_t sort_incidence(uint32_t* keys_in, uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out, int64_t n,
                          int64_t nv_total, void* temp, size_t* temp_bytes, hipStream_t s) {
  int end_bit = 1;
  while (end_bit < 32 && ((uint64_t)1 << end_bit) <= (uint64_t)nv_total) ++end_bit;
  return hipcub::DeviceRadixSort::SortPairs(temp, *temp_bytes, keys_in, keys_out, vals_in, vals_out, (int)n, 0,
                                            end_bit, s);
}

hipError_t launch_gather_vertices(const uint32_t* keys_sorted, const uint32_t* vals_sorted, int64_t nslots,
                                  const double* contrib, int64_t nv, void* grad, int vdtype, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  gather_kernel<<<grid_for(nv), 256, 0, s>>>(keys_sorted, vals_sorted, nslots, contrib, nv, grad, vdtype);
  return hipGetLastError();
}

}  // namespace pft
