// Orientation average of the scattered intensity,
//   I(q) = sum_j w_j |F(q s_j)|^2,
// the powder / solution-scattering quantity that motivates the method (the
// paper's introduction): the transform over a direction quadrature (s_j, w_j)
// at each magnitude q, then a weighted sum over directions.
#include "pft_internal.h"

namespace pft {
namespace {

// Q[i * ndir + j] = qabs[i] * dirs[j] (binary64)
__global__ __launch_bounds__(256) void qdirs_kernel(const double* qabs, int64_t nqa, const double* dirs, int64_t ndir,
                                                    double* Q) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nqa * ndir) return;
  const int64_t i = k / ndir, j = k - i * ndir;
  const double q = qabs[i];
  Q[3 * k + 0] = q * dirs[3 * j + 0];
  Q[3 * k + 1] = q * dirs[3 * j + 1];
  Q[3 * k + 2] = q * dirs[3 * j + 2];
}

// out[i] = sum_j w_j I[i * ndir + j] in binary64, one block per magnitude: each
// thread sums a strided share of the directions, then a fixed-order tree.
template <typename T>
__global__ __launch_bounds__(256) void dir_sum_kernel(const T* I, const double* w, int64_t nqa, int64_t ndir,
                                                      double* out) {
  __shared__ double red[256];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int64_t j = tid; j < ndir; j += 256) acc += w[j] * (double)I[i * ndir + j];
  red[tid] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) out[i] = red[0];
}

}  // namespace

hipError_t launch_qdirs(const double* qabs, int64_t nqa, const double* dirs, int64_t ndir, double* Q, hipStream_t s) {
  const int64_t n = nqa * ndir;
  if (n <= 0) return hipSuccess;
  qdirs_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(qabs, nqa, dirs, ndir, Q);
  return hipGetLastError();
}

hipError_t launch_dir_sum(const void* I, int idtype, const double* w, int64_t nqa, int64_t ndir, double* out,
                          hipStream_t s) {
  if (nqa <= 0) return hipSuccess;
  if (idtype == PFT_F64)
    dir_sum_kernel<double><<<(unsigned)nqa, 256, 0, s>>>(static_cast<const double*>(I), w, nqa, ndir, out);
  else
    dir_sum_kernel<float><<<(unsigned)nqa, 256, 0, s>>>(static_cast<const float*>(I), w, nqa, ndir, out);
  return hipGetLastError();
}

}  // namespace pft
