// Batched transform of many independent meshes in one persistent launch.
//
// The host cuts every mesh into work items -- (mesh, Q-tile, face chunk) for
// the forward, described by runs of equal-size items (BatchGroupFwd), (mesh,
// face tile of <= kTileFB faces, Q chunk) for the adjoint -- and orders them
// by decreasing cost (longest processing time first). A
// grid sized to the GPU's resident capacity pulls items from a device counter
// until the list is exhausted (the FP32C forward per wavefront, the others per
// block); every puller reaches the exit test on each iteration, so the grid
// always drains. Each item writes its own
// partial slot, and a finish kernel adds the partials of each Q (or face) in a
// fixed order, so results do not depend on which block ran which item.
#include "adj_terms.h"
#include "fwd_terms.h"

namespace pft {
namespace {

// Fetch the next work item index for the whole block (vector atomic from one lane).
__device__ __forceinline__ int64_t next_item(uint32_t* counter, int* slot) {
  if (threadIdx.x == 0) *slot = (int)atomicAdd(counter, 1u);
  __syncthreads();
  const int64_t it = *slot;
  __syncthreads();
  return it;
}

// Work item `idx` of the forward from its group (binary search over the groups' first items; with a
// wavefront-uniform idx the search runs on scalar loads).
__device__ __forceinline__ BatchItemFwd group_item(const BatchGroupFwd* __restrict__ g, int n_groups, int64_t idx) {
  int lo = 0, hi = n_groups;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (g[mid].first <= idx) lo = mid; else hi = mid;
  }
  const BatchGroupFwd G = g[lo];
  const int64_t k = idx - G.first;
  const int64_t dc = k / G.ntq, dt = k - dc * G.ntq;
  BatchItemFwd it;
  it.mesh = G.mesh;
  it.chunk = 0;
  it.q0 = G.q_base + dt * G.qtile;
  it.nq = G.nq;
  it.pad = 0;
  it.f0 = G.f_base + dc * G.cf;
  it.nf = G.nf;
  it.part = G.part_base + dc * G.part_stride + dt * G.qtile;
  return it;
}

// The binary64 batched forward: blocks pull (mesh, Q-tile of kBlock Q, face chunk) items, one Q per
// thread, the chunk's faces staged through LDS for the whole block.
__global__ __launch_bounds__(kBlock) void batch_fwd_fp64_kernel(const BatchGroupFwd* __restrict__ groups,
                                                               int n_groups, int64_t n_items, uint32_t* counter,
                                                               const Face64* __restrict__ f64, const void* q,
                                                               int qdtype, const uint32_t* __restrict__ perm,
                                                               double2* partial, const MeshInfo* __restrict__ info,
                                                               double tau0) {
  __shared__ Face64 tile[kTileF];
  __shared__ int slot;
  for (;;) {
    const int64_t idx = next_item(counter, &slot);
    if (idx >= n_items) break;
    const BatchItemFwd it = group_item(groups, n_groups, idx);
    const int lane = threadIdx.x;
    const int64_t f_end = it.f0 + it.nf;
    const double R = info[it.mesh].R;
    const bool active = lane < it.nq;
    double Qd[3] = {0.0, 0.0, 0.0};
    if (active) load_q3(q, qdtype, perm ? (int64_t)perm[it.q0 + lane] : it.q0 + lane, Qd);
    const double Q2d = Qd[0] * Qd[0] + Qd[1] * Qd[1] + Qd[2] * Qd[2];
    const bool small = sqrt(Q2d) * R < tau0;
    double xr = 0.0, xi = 0.0;
    for (int64_t t0 = it.f0; t0 < f_end; t0 += kTileF) {
      const int nt = (int)min((int64_t)kTileF, f_end - t0);
      __syncthreads();
      for (int i = lane; i < nt * (int)(sizeof(Face64) / 16); i += kBlock)
        reinterpret_cast<uint4*>(tile)[i] = reinterpret_cast<const uint4*>(f64 + t0)[i];
      __syncthreads();
      if (!small) {
        for (int j = 0; j < nt; ++j) {
          double Tr, Ti;
          face_term_f64(tile[j], Qd, Tr, Ti);
          xr += Tr;
          xi += Ti;
        }
      } else {
        for (int j = 0; j < nt; ++j) tet_term_f64(tile[j], Qd, xr, xi, kZeroOrigin);
      }
    }
    if (active) store_stream(partial + it.part + lane, make_double2(xr, xi));
  }
}

// The next work item of a wavefront (lane 0 takes it from the counter; the value is read back as a
// wavefront-uniform scalar, so the item's fields load into scalar registers).
__device__ __forceinline__ int64_t wave_next_item(uint32_t* counter) {
  int idx = 0;
  if ((threadIdx.x & 63) == 0) idx = (int)atomicAdd(counter, 1u);
  return (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(idx);
}

// The FP32C batched forward: every wavefront is an independent worker. It pulls (mesh, Q-tile of 64 QPT
// Q, face chunk) items from the counter (longest first), holds QPT Q per lane (strided by 64), streams the
// chunk's faces through its own LDS tile with wavefront-local ordering and writes its binary64 partials;
// no block barrier anywhere, so a wavefront never waits for the others of its block. QPT = 3 runs at
// kBatchFwdWaves waves per SIMD, QPT = 1 and 2 one wavefront more (at 2 a few per-item values spill,
// outside the face loop; measured 6 % faster on the 512-mesh batch than at kBatchFwdWaves).
template <bool SHARE, int QPT>
__global__ __launch_bounds__(kBlock, QPT >= 3 ? kBatchFwdWaves : kBatchFwdWaves + 1) void batch_fwd_fp32c_kernel(
    const BatchGroupFwd* __restrict__ groups, int n_groups, int64_t n_items, uint32_t* counter,
    const Face64* __restrict__ f64,
    const Face32* __restrict__ f32, const void* q, int qdtype, const uint32_t* __restrict__ perm, double2* partial,
    const MeshInfo* __restrict__ info, double tau0) {
  __shared__ Face32 tiles[kBlock / 64][kTileF32];
  __shared__ float qlo[kBlock / 64][3 * QPT * 64];
  const int lane = (int)(threadIdx.x & 63);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  Face32* tile = tiles[w];
  for (;;) {
    const int64_t idx = wave_next_item(counter);
    if (idx >= n_items) break;
    const BatchItemFwd it = group_item(groups, n_groups, idx);
    const int64_t f_end = it.f0 + it.nf;
    const MeshInfo& mi = info[it.mesh];
    const double R = mi.R;
    QLowLds<QPT> ql;
    ql.lo = qlo[w];
    ql.lane = lane;
    float qx[QPT], qy[QPT], qz[QPT], Q2[QPT];
    bool small[QPT], active[QPT];
    bool any_small = false;
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
      const int qo = lane + k * 64;
      active[k] = qo < it.nq;
      double Qd[3] = {0.0, 0.0, 0.0};
      if (active[k]) load_q3(q, qdtype, perm ? (int64_t)perm[it.q0 + qo] : it.q0 + qo, Qd);
      qx[k] = (float)Qd[0];
      qy[k] = (float)Qd[1];
      qz[k] = (float)Qd[2];
      ql.set(k, Qd, qx[k], qy[k], qz[k]);
      Q2[k] = qx[k] * qx[k] + qy[k] * qy[k] + qz[k] * qz[k];
      const double Q2d = Qd[0] * Qd[0] + Qd[1] * Qd[1] + Qd[2] * Qd[2];
      small[k] = sqrt(Q2d) * R < tau0;
      any_small |= small[k];
    }
    float qmax = 0.0f;
#pragma unroll
    for (int k = 0; k < QPT; ++k) qmax = fmaxf(qmax, sqrtf(Q2[k]));
    const bool check = __builtin_amdgcn_readfirstlane((int)sinc_range_test_needed(wave_max(qmax), mi.rho)) != 0;
    float sr[QPT], si[QPT], cr[QPT], ci[QPT];
#pragma unroll
    for (int k = 0; k < QPT; ++k) sr[k] = si[k] = cr[k] = ci[k] = 0.0f;
    FwdCarry<QPT> carry;  // shared edge term from the previous face of the item
    carry.reset();
    for (int64_t t0 = it.f0; t0 < f_end; t0 += kTileF32) {
      const int nt = (int)min((int64_t)kTileF32, f_end - t0);
      wave_lds_fence();
      for (int i = lane; i < nt * (int)(sizeof(Face32) / 16); i += 64)
        reinterpret_cast<uint4*>(tile)[i] = reinterpret_cast<const uint4*>(f32 + t0)[i];
      wave_lds_fence();
      float tr[QPT], ti[QPT];
#pragma unroll
      for (int k = 0; k < QPT; ++k) tr[k] = ti[k] = 0.0f;
      // transcendentals in one run per face at 2 Q per thread (measured neutral at 1; at 3 the run
      // would add register pressure to a variant that already spills)
      if (check)
        fwd_tile_fp32c<QPT, SHARE, true, (QPT == 2)>(tile, nt, qx, qy, qz, ql, small, tr, ti, carry);
      else
        fwd_tile_fp32c<QPT, SHARE, false, (QPT == 2)>(tile, nt, qx, qy, qz, ql, small, tr, ti, carry);
#pragma unroll
      for (int k = 0; k < QPT; ++k) {
        kahan_add(sr[k], cr[k], tr[k]);
        kahan_add(si[k], ci[k], ti[k]);
      }
    }
    // small-|Q| lanes: the binary64 tetrahedron fan over the item's faces, after the surface sums
    double xr[QPT], xi[QPT];
#pragma unroll
    for (int k = 0; k < QPT; ++k) xr[k] = xi[k] = 0.0;
    if (any_small) {
#pragma unroll
      for (int k = 0; k < QPT; ++k)
        if (small[k]) {
          const double Qd[3] = {ql.qd(qx[k], k, 0), ql.qd(qy[k], k, 1), ql.qd(qz[k], k, 2)};
          for (int64_t j = it.f0; j < f_end; ++j) tet_term_f64(f64[j], Qd, xr[k], xi[k], kZeroOrigin);
        }
    }
    const int l = (int)__lane_id();  // anew, so no lane index is kept live across the face loop
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
      if (l + k * 64 < it.nq) {
        const double2 v = small[k] ? make_double2(xr[k], xi[k])
                                   : make_double2(((double)sr[k] - (double)cr[k]) * kInvSumScale32,
                                                  ((double)si[k] - (double)ci[k]) * kInvSumScale32);
        store_stream(partial + it.part + l + k * 64, v);
      }
    }
  }
}

// One thread per Q of the batch: add the face-chunk partials of its mesh, apply
// exp(iQ.t) / |Q|^2, write F (and |F|^2).
__global__ __launch_bounds__(256) void batch_fwd_finish_kernel(const double2* partial, const int64_t* q_off,
                                                               int64_t n_meshes, const int64_t* q_part,
                                                               const int32_t* q_chunks, const MeshInfo* info,
                                                               const void* q, int qdtype,
                                                               const uint32_t* perm, int64_t nq_total,
                                                               double tau0, int out_c128, void* out,
                                                               void* intensity) {
  const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= nq_total) return;
  const int64_t dst = perm ? (int64_t)perm[qi] : qi;  // the permutation keeps each mesh's range
  int64_t lo = 0, hi = n_meshes;  // last mesh with q_off[mesh] <= qi
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (q_off[mid] <= qi) lo = mid; else hi = mid;
  }
  const int64_t mesh = lo;
  const int64_t nqm = q_off[mesh + 1] - q_off[mesh];
  const int64_t j = qi - q_off[mesh];
  double xr = 0.0, xi = 0.0;
  for (int c = 0; c < q_chunks[mesh]; ++c) {
    const double2 v = load_stream(partial + q_part[mesh] + (int64_t)c * nqm + j);
    xr += v.x;
    xi += v.y;
  }
  double Q[3];
  load_q3(q, qdtype, dst, Q);
  const MeshInfo mi = info[mesh];
  const double Q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
  if (!(sqrt(Q2) * mi.R < tau0)) {
    xr /= Q2;
    xi /= Q2;
  }
  double st, ct;
  sincos(Q[0] * mi.t[0] + Q[1] * mi.t[1] + Q[2] * mi.t[2], &st, &ct);
  double Fr = ct * xr - st * xi;
  double Fi = ct * xi + st * xr;
  if (!out_c128 && fp32c_phase_out_of_range(sqrt(Q2), mi)) Fr = Fi = quiet_nan();  // beyond the FP32C phase range
  if (out_c128) {
    static_cast<double2*>(out)[dst] = make_double2(Fr, Fi);
    if (intensity) static_cast<double*>(intensity)[dst] = Fr * Fr + Fi * Fi;
  } else {
    static_cast<float2*>(out)[dst] = make_float2((float)Fr, (float)Fi);
    if (intensity) static_cast<float*>(intensity)[dst] = (float)(Fr * Fr + Fi * Fi);
  }
}

__global__ __launch_bounds__(kBlock) void batch_bwd_fp64_kernel(const BatchItemBwd* __restrict__ items,
                                                               int64_t n_items, uint32_t* counter,
                                                               const Face64* __restrict__ f64,
                                                               const double* __restrict__ gram,
                                                               const QRec64* __restrict__ rec, double* partial) {
  __shared__ Face64 tile[kTileFB];
  __shared__ double gtile[kTileFB][8];
  __shared__ double acc[kTileFB * 3][kBlock];
  __shared__ int slot;
  const int tid = threadIdx.x;
  for (;;) {
    const int64_t idx = next_item(counter, &slot);
    if (idx >= n_items) break;
    const BatchItemBwd it = items[idx];
    const int nt = it.nf;
    for (int i = tid; i < nt * (int)(sizeof(Face64) / 16); i += kBlock)
      reinterpret_cast<uint4*>(tile)[i] = reinterpret_cast<const uint4*>(f64 + it.f0)[i];
    for (int i = tid; i < nt * 8; i += kBlock) gtile[i / 8][i % 8] = gram[(it.f0 + i / 8) * 8 + i % 8];
    for (int v = 0; v < nt * 3; ++v) acc[v][tid] = 0.0;
    __syncthreads();
    adj_tile_f64(tile, gtile, nt, it.q0, it.q0 + it.nq, rec, acc);
    __syncthreads();
    adj_block_sum(acc, nt, partial + it.part * 3);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void batch_bwd_fp32c_kernel(const BatchItemBwd* __restrict__ items,
                                                                int64_t n_items, uint32_t* counter,
                                                                const Face32B* __restrict__ f32b,
                                                                const QRec32* __restrict__ rec, double* partial) {
  __shared__ Face32B tile[kTileFB32];
  __shared__ float acc[kTileFB32 * 3][kBlock];
  __shared__ int slot;
  const int tid = threadIdx.x;
  for (;;) {
    const int64_t idx = next_item(counter, &slot);
    if (idx >= n_items) break;
    const BatchItemBwd it = items[idx];
    const int nt = it.nf;
    for (int i = tid; i < nt * (int)(sizeof(Face32B) / 16); i += kBlock)
      reinterpret_cast<uint4*>(tile)[i] = reinterpret_cast<const uint4*>(f32b + it.f0)[i];
    for (int v = 0; v < nt * 3; ++v) acc[v][tid] = 0.0f;
    __syncthreads();
    adj_tile_fp32c(tile, nt, it.q0, it.q0 + it.nq, rec, acc);
    __syncthreads();
    adj_block_sum(acc, nt, partial + it.part * 3);
    __syncthreads();
  }
}

// Per face corner: sum the Q-chunk partials of its mesh and form N_m R_{m,k}.
__global__ __launch_bounds__(256) void batch_bwd_reduce_kernel(const double* partial, const int64_t* face_base,
                                                               const int32_t* face_nchunks, const int64_t* tri_off,
                                                               const int32_t* face_mesh, const Face64* f64,
                                                               int64_t nf_total, double* contrib) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // corner slot 3m + k
  if (i >= nf_total * 3) return;
  const int64_t m = i / 3;
  const int k = (int)(i % 3);
  const int32_t mesh = face_mesh[m];
  const int64_t nfm = tri_off[mesh + 1] - tri_off[mesh];
  const int64_t fl = m - tri_off[mesh];
  double R = 0.0;
  for (int c = 0; c < face_nchunks[mesh]; ++c) R += partial[(face_base[mesh] + (int64_t)c * nfm + fl) * 3 + k];
  const Face64& f = f64[m];
  contrib[i * 3 + 0] = f.N[0] * R;
  contrib[i * 3 + 1] = f.N[1] * R;
  contrib[i * 3 + 2] = f.N[2] * R;
}

}  // namespace

int batch_fwd_blocks_per_cu(int mode, bool share, int qpt) {
  int nb = 0;
  if (mode == PFT_FP64)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_fwd_fp64_kernel, kBlock, 0);
  else if (share)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, qpt >= 3 ? batch_fwd_fp32c_kernel<true, 3> : qpt == 2 ? batch_fwd_fp32c_kernel<true, 2>
                                                                  : batch_fwd_fp32c_kernel<true, 1>,
        kBlock, 0);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, qpt >= 3 ? batch_fwd_fp32c_kernel<false, 3> : qpt == 2 ? batch_fwd_fp32c_kernel<false, 2>
                                                                   : batch_fwd_fp32c_kernel<false, 1>,
        kBlock, 0);
  return nb > 0 ? nb : 1;
}

int batch_bwd_blocks_per_cu(int mode) {
  int nb = 0;
  if (mode == PFT_FP64)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_bwd_fp64_kernel, kBlock, 0);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_bwd_fp32c_kernel, kBlock, 0);
  return nb > 0 ? nb : 1;
}

hipError_t launch_batch_fwd(int mode, const BatchGroupFwd* groups, int n_groups, int64_t n_items, uint32_t* counter,
                            const Face64* f64, const Face32* f32, const void* q, int qdtype, const uint32_t* perm,
                            double2* partial, const MeshInfo* info, double tau0, int grid, hipStream_t s,
                            bool share, int qpt) {
  if (n_items <= 0) return hipSuccess;
#define PFT_BATCH_FWD(SH, QP) \
  batch_fwd_fp32c_kernel<SH, QP><<<grid, kBlock, 0, s>>>(groups, n_groups, n_items, counter, f64, f32, q, qdtype, perm, \
                                                          partial, info, tau0)
  if (mode == PFT_FP64)
    batch_fwd_fp64_kernel<<<grid, kBlock, 0, s>>>(groups, n_groups, n_items, counter, f64, q, qdtype, perm, partial, info,
                                                  tau0);
  else if (share)
    qpt >= 3 ? PFT_BATCH_FWD(true, 3) : qpt == 2 ? PFT_BATCH_FWD(true, 2) : PFT_BATCH_FWD(true, 1);
  else
    qpt >= 3 ? PFT_BATCH_FWD(false, 3) : qpt == 2 ? PFT_BATCH_FWD(false, 2) : PFT_BATCH_FWD(false, 1);
#undef PFT_BATCH_FWD
  return hipGetLastError();
}

hipError_t launch_batch_fwd_finish(const double2* partial, const int64_t* d_q_off, int64_t n_meshes,
                                   const int64_t* d_q_part, const int32_t* d_q_chunks, const MeshInfo* info,
                                   const void* q, int qdtype, const uint32_t* perm, int64_t nq_total, double tau0,
                                   int out_c128, void* out, void* intensity, hipStream_t s) {
  if (nq_total <= 0) return hipSuccess;
  batch_fwd_finish_kernel<<<(unsigned)((nq_total + 255) / 256), 256, 0, s>>>(
      partial, d_q_off, n_meshes, d_q_part, d_q_chunks, info, q, qdtype, perm, nq_total, tau0, out_c128, out,
      intensity);
  return hipGetLastError();
}

hipError_t launch_batch_bwd(int mode, const BatchItemBwd* items, int64_t n_items, uint32_t* counter,
                            const Face64* f64, const double* gram, const Face32B* f32b, const QRec32* rec,
                            const QRec64* rec64, double* partial, int grid, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (mode == PFT_FP64)
    batch_bwd_fp64_kernel<<<grid, kBlock, 0, s>>>(items, n_items, counter, f64, gram, rec64, partial);
  else
    batch_bwd_fp32c_kernel<<<grid, kBlock, 0, s>>>(items, n_items, counter, f32b, rec, partial);
  return hipGetLastError();
}

hipError_t launch_batch_bwd_reduce(const double* partial, const int64_t* d_face_base, const int32_t* d_face_nchunks,
                                   const int64_t* d_tri_off, const int32_t* d_face_mesh, const Face64* f64,
                                   int64_t nf_total, double* contrib, hipStream_t s) {
  if (nf_total <= 0) return hipSuccess;
  batch_bwd_reduce_kernel<<<(unsigned)((nf_total * 3 + 255) / 256), 256, 0, s>>>(
      partial, d_face_base, d_face_nchunks, d_tri_off, d_face_mesh, f64, nf_total, contrib);
  return hipGetLastError();
}

}  // namespace pft
