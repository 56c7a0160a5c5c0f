// Intensity loss and its cotangent in one pass over the forward's partials.
//
// For L = sum_Q w(Q) (|F(Q)|^2 - I(Q))^2 the cotangent of the adjoint is
// g = dL/dRe F + i dL/dIm F = 4 w (|F|^2 - I) F. With F = exp(iQ.t) F_c (F_c the
// transform of the mesh centred on t), the adjoint's centred cotangent is
// g exp(-iQ.t) = 4 w (|F|^2 - I) F_c, and |F| = |F_c|: neither needs the
// translation phase. The finish kernel below adds the forward's partials of
// each Q in a fixed order (as the forward's finish), forms F_c, the loss term
// and the cotangent in binary64, writes the adjoint's Q record in the visiting
// order (so no separate gather is needed), optionally F and |F|^2 at the
// caller's index, and reduces the loss per block; a single block then adds the
// block sums in order.
#include "adj_terms.h"

namespace pft {
namespace {

constexpr int kLossBlock = 256;

__global__ __launch_bounds__(kLossBlock) void loss_finish_kernel(FwdArgs a, const double* weight, const double* target,
                                                                 int c128, QRec32* rec, QRec64* rec64,
                                                                 double* loss_part) {
  __shared__ double lds[kLossBlock / 64];
  const int64_t qi = (int64_t)blockIdx.x * kLossBlock + threadIdx.x;
  const bool valid = qi < a.nq;
  double term = 0.0;
  if (valid) {
    const int64_t dst = a.perm ? (int64_t)a.perm[qi] : qi;
    double Q[3];
    load_q3(a.q, a.qdtype, dst, Q);
    double xr, xi;
    fwd_partial_sum(a, qi, xr, xi);
    const MeshInfo mi = a.info[0];
    const double Q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
    if (!(sqrt(Q2) * mi.R < a.tau0)) {
      xr /= Q2;
      xi /= Q2;
    }
    // beyond the FP32C phase range: NaN F, loss term and cotangent
    if (!c128 && fp32c_phase_out_of_range(sqrt(Q2), mi)) xr = xi = quiet_nan();
    const double I = xr * xr + xi * xi;
    const double w = weight ? weight[dst] : 1.0;
    const double r = I - target[dst];
    term = w * r * r;
    const double hr = 4.0 * w * r * xr, hi = 4.0 * w * r * xi;
    if (c128) {
      QRec64 R;
      R.q[0] = Q[0];
      R.q[1] = Q[1];
      R.q[2] = Q[2];
      R.pad = 0.0;
      R.hr = hr;
      R.hi = hi;
      rec64[qi] = R;
    } else {
      QRec32 R;
      R.q[0] = Q[0];
      R.q[1] = Q[1];
      R.q[2] = Q[2];
      R.hr = (float)hr;
      R.hi = (float)hi;
      rec[qi] = R;
    }
    if (a.out) {
      double st, ct;
      sincos(Q[0] * mi.t[0] + Q[1] * mi.t[1] + Q[2] * mi.t[2], &st, &ct);
      const double Fr = ct * xr - st * xi, Fi = ct * xi + st * xr;
      if (c128)
        static_cast<double2*>(a.out)[dst] = make_double2(Fr, Fi);
      else
        static_cast<float2*>(a.out)[dst] = make_float2((float)Fr, (float)Fi);
    }
    if (a.intensity) {
      if (c128)
        static_cast<double*>(a.intensity)[dst] = I;
      else
        static_cast<float*>(a.intensity)[dst] = (float)I;
    }
  }
  const double t = block_total<kLossBlock>(term, lds);
  if (threadIdx.x == 0) loss_part[blockIdx.x] = t;
}

// One block: the per-block sums in a fixed order.
__global__ __launch_bounds__(kLossBlock) void sum_blocks_kernel(const double* part, int64_t n, double* out) {
  __shared__ double lds[kLossBlock / 64];
  double v = 0.0;
  for (int64_t b = threadIdx.x; b < n; b += kLossBlock) v += part[b];
  v = block_total<kLossBlock>(v, lds);
  if (threadIdx.x == 0) out[0] = v;
}

}  // namespace

int64_t loss_blocks(int64_t nq) { return (nq + kLossBlock - 1) / kLossBlock; }

hipError_t launch_loss_finish(const FwdArgs& a, const double* weight, const double* target, int c128, QRec32* rec,
                              QRec64* rec64, double* loss_part, double* loss, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  const int64_t nb = loss_blocks(a.nq);
  loss_finish_kernel<<<(unsigned)nb, kLossBlock, 0, s>>>(a, weight, target, c128, rec, rec64, loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  sum_blocks_kernel<<<1, kLossBlock, 0, s>>>(loss_part, nb, loss);
  return hipGetLastError();
}

}  // namespace pft
