// Q ordering.
//
// Each Q is evaluated independently, so the kernels may visit the Q list in any
// order. Their cost per (Q, face) follows the worst lane of a wavefront: the
// adjoint's series runs until its largest vertex phase |Q.(v - g)| has
// converged, and the forward's near-degenerate branch (Q nearly along a face
// normal) runs whenever one lane needs it. Wavefronts of nearby Q waste less
// work than wavefronts spanning a grid row or a random set. The Q points are
// sorted by mesh, then by the Morton code of their coordinates quantised
// inside the bounding box of all Q (10 bits per axis; 5 for a single mesh,
// which keeps the sort key at 16 bits); the forward reads Q
// through the permutation and writes F back to the caller's order, the FP32C
// adjoint gathers Q with their centred cotangents into QRec32 records.
#include <hipcub/hipcub.hpp>

#include "pft_device.h"

namespace pft {
namespace {

constexpr int kBoxBlocks = 256;

__global__ __launch_bounds__(256) void qbox_partial_kernel(const void* q, int qdtype, int64_t nq, double* partial) {
  __shared__ double red[6][256];
  const int tid = threadIdx.x;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + tid; i < nq; i += (int64_t)gridDim.x * blockDim.x) {
    double Q[3];
    load_q3(q, qdtype, i, Q);
    for (int k = 0; k < 3; ++k) {
      lo[k] = fmin(lo[k], Q[k]);
      hi[k] = fmax(hi[k], Q[k]);
    }
  }
  for (int k = 0; k < 3; ++k) {
    red[k][tid] = lo[k];
    red[3 + k][tid] = hi[k];
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s)
      for (int k = 0; k < 3; ++k) {
        red[k][tid] = fmin(red[k][tid], red[k][tid + s]);
        red[3 + k][tid] = fmax(red[3 + k][tid], red[3 + k][tid + s]);
      }
    __syncthreads();
  }
  if (tid < 6) partial[blockIdx.x * 6 + tid] = red[tid][0];
}

__global__ __launch_bounds__(256) void qbox_final_kernel(const double* partial, int nb, double* box) {
  __shared__ double red[6][256];
  const int tid = threadIdx.x;
  for (int k = 0; k < 6; ++k) red[k][tid] = tid < nb ? partial[tid * 6 + k] : (k < 3 ? INFINITY : -INFINITY);
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s)
      for (int k = 0; k < 3; ++k) {
        red[k][tid] = fmin(red[k][tid], red[k][tid + s]);
        red[3 + k][tid] = fmax(red[3 + k][tid], red[3 + k][tid + s]);
      }
    __syncthreads();
  }
  if (tid < 6) box[tid] = red[tid][0];
}

// spread the low 10 bits of x to every third bit
__device__ __forceinline__ uint64_t spread3(uint32_t x) {
  uint64_t v = x & 0x3ffu;
  v = (v | (v << 16)) & 0x30000ffull;
  v = (v | (v << 8)) & 0x300f00full;
  v = (v | (v << 4)) & 0x30c30c3ull;
  v = (v | (v << 2)) & 0x9249249ull;
  return v;
}

__device__ __forceinline__ int64_t mesh_of(const int64_t* q_off, int64_t n_meshes, int64_t i) {
  if (!q_off) return 0;
  int64_t lo = 0, hi = n_meshes;  // last mesh with q_off[mesh] <= i
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (q_off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void qkey_kernel(const void* q, int qdtype, int64_t nq, const double* box,
                                                   const int64_t* q_off, int64_t n_meshes, uint64_t* keys,
                                                   uint32_t* vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  double Q[3];
  load_q3(q, qdtype, i, Q);
  uint64_t code = 0;
  for (int k = 0; k < 3; ++k) {
    const double ext = box[3 + k] - box[k];
    double u = ext > 0.0 ? (Q[k] - box[k]) / ext * 1024.0 : 0.0;
    u = fmin(fmax(u, 0.0), 1023.0);  // NaN coordinates map to 0 (fmax returns the non-NaN operand)
    code |= spread3((uint32_t)u) << k;
  }
  keys[i] = ((uint64_t)mesh_of(q_off, n_meshes, i) << 30) | code;
  vals[i] = (uint32_t)i;
}

// One mesh: a 15-bit Morton code (5 bits per axis). 16-bit keys let the radix
// sort use its one-sweep passes at every size above 1e5 (its merge-based path,
// taken for wider keys up to 2^20 items, costs several times more).
__global__ __launch_bounds__(256) void qkey16_kernel(const void* q, int qdtype, int64_t nq, const double* box,
                                                     uint16_t* keys, uint32_t* vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  double Q[3];
  load_q3(q, qdtype, i, Q);
  uint64_t code = 0;
  for (int k = 0; k < 3; ++k) {
    const double ext = box[3 + k] - box[k];
    double u = ext > 0.0 ? (Q[k] - box[k]) / ext * 32.0 : 0.0;
    u = fmin(fmax(u, 0.0), 31.0);
    code |= spread3((uint32_t)u) << k;
  }
  keys[i] = (uint16_t)code;
  vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void qrec32_kernel(const void* q, int qdtype, const float2* grad_out, int64_t nq,
                                                     const uint32_t* perm, const MeshInfo* info,
                                                     const int64_t* q_off, int64_t n_meshes, QRec32* rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int64_t j = perm[i];
  double Q[3];
  load_q3(q, qdtype, j, Q);
  const float2 g = grad_out[j];
  const MeshInfo& mi = info[mesh_of(q_off, n_meshes, j)];
  double hr, hi;
  centred_cotangent((double)g.x, (double)g.y, Q, mi.t, hr, hi);
  // beyond the FP32C phase range: a NaN cotangent, so every vertex gradient is NaN
  if (fp32c_phase_out_of_range(sqrt(Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2]), mi)) hr = hi = quiet_nan();
  QRec32 r;
  r.q[0] = Q[0];
  r.q[1] = Q[1];
  r.q[2] = Q[2];
  r.hr = (float)hr;
  r.hi = (float)hi;
  rec[i] = r;
}

__global__ __launch_bounds__(256) void qrec64_kernel(const void* q, int qdtype, const double2* grad_out, int64_t nq,
                                                     const uint32_t* perm, const MeshInfo* info,
                                                     const int64_t* q_off, int64_t n_meshes, QRec64* rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int64_t j = perm[i];
  double Q[3];
  load_q3(q, qdtype, j, Q);
  const double2 g = grad_out[j];
  QRec64 r;
  centred_cotangent(g.x, g.y, Q, info[mesh_of(q_off, n_meshes, j)].t, r.hr, r.hi);
  r.q[0] = Q[0];
  r.q[1] = Q[1];
  r.q[2] = Q[2];
  r.pad = 0.0;
  rec[i] = r;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int qorder_end_bit(int64_t n_meshes) {
  int end_bit = 30;
  while (end_bit < 64 && ((uint64_t)1 << (end_bit - 30)) < (uint64_t)std::max<int64_t>(n_meshes, 1)) ++end_bit;
  return end_bit;
}

hipError_t qorder_sort_bytes(int64_t nq, int64_t n_meshes, size_t* bytes) {
  *bytes = 0;
  if (n_meshes <= 1)
    return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const uint16_t*)nullptr, (uint16_t*)nullptr,
                                              (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)nq, 0, 15);
  return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                            (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)nq, 0,
                                            qorder_end_bit(n_meshes));
}

hipError_t launch_qorder(const void* q, int qdtype, int64_t nq, const int64_t* d_q_off, int64_t n_meshes,
                         const QOrderScratch& w, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  const int nb = (int)std::min<int64_t>(kBoxBlocks, (nq + 255) / 256);
  qbox_partial_kernel<<<nb, 256, 0, s>>>(q, qdtype, nq, w.box_partial);
  qbox_final_kernel<<<1, 256, 0, s>>>(w.box_partial, nb, w.box);
  size_t tb = w.sort_bytes;
  if (n_meshes <= 1) {
    uint16_t* k16 = reinterpret_cast<uint16_t*>(w.keys);
    uint16_t* k16s = reinterpret_cast<uint16_t*>(w.keys_sorted);
    qkey16_kernel<<<grid_for(nq), 256, 0, s>>>(q, qdtype, nq, w.box, k16, w.vals);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipcub::DeviceRadixSort::SortPairs(w.sort_temp, tb, k16, k16s, w.vals, w.perm, (int)nq, 0, 15, s);
  }
  qkey_kernel<<<grid_for(nq), 256, 0, s>>>(q, qdtype, nq, w.box, d_q_off, n_meshes, w.keys, w.vals);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipcub::DeviceRadixSort::SortPairs(w.sort_temp, tb, w.keys, w.keys_sorted, w.vals, w.perm, (int)nq, 0,
                                            qorder_end_bit(n_meshes), s);
}

hipError_t launch_qrec32_gather(const void* q, int qdtype, const void* grad_out, int64_t nq, const uint32_t* perm,
                                const MeshInfo* info, const int64_t* d_q_off, int64_t n_meshes, QRec32* rec,
                                hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  qrec32_kernel<<<grid_for(nq), 256, 0, s>>>(q, qdtype, static_cast<const float2*>(grad_out), nq, perm, info,
                                             d_q_off, n_meshes, rec);
  return hipGetLastError();
}

hipError_t launch_qrec64_gather(const void* q, int qdtype, const void* grad_out, int64_t nq, const uint32_t* perm,
                                const MeshInfo* info, const int64_t* d_q_off, int64_t n_meshes, QRec64* rec,
                                hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  qrec64_kernel<<<grid_for(nq), 256, 0, s>>>(q, qdtype, static_cast<const double2*>(grad_out), nq, perm, info,
                                             d_q_off, n_meshes, rec);
  return hipGetLastError();
}

}  // namespace pft
