// Forward 3D transform of a closed triangle mesh: F(Q) for a list of Q.
//
// Layout: Q-tiles of threads (binary64: one Q per thread; FP32C: kQPT Q per
// thread, each wavefront of a block on its own share of the faces), faces
// streamed through LDS in tiles of kTileF records and broadcast to the
// wavefront. Each block's sums over its face range are binary64 partials; the
// finish kernel adds a Q's partials in a fixed order and applies
// exp(i Q.t) / |Q|^2. The faces are split when there are too few Q to fill
// the GPU (over blockIdx.y in binary64; in FP32C the split is part of the
// one-dimensional block index).
//
// Two arithmetic forms:
//  * fwd3d_fp64_kernel  -- IEEE binary64 throughout.
//  * fwd3d_fp32c_kernel -- edge arithmetic in binary32 on face-local
//    coordinates, the face origin phase Q.g reduced in binary64 and
//    evaluated in turns, the near-degenerate series branch in binary64, the
//    sum over faces blocked per LDS tile and compensated (Kahan) across tiles.
//    With the records in an edge-sharing order (Face32::flags) a face takes
//    the term of the edge it shares with its predecessor from registers.
#include "fwd3d_fp32c.h"

namespace pft {
namespace {

__global__ __launch_bounds__(kBlock) void fwd3d_fp64_kernel(FwdArgs a) {
  __shared__ Face64 tile[kTileF];
  const int64_t qi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = qi < a.nq;
  double Q[3] = {0.0, 0.0, 0.0};
  if (active) load_q3(a.q, a.qdtype, a.perm ? (int64_t)a.perm[qi] : qi, Q);
  const double Q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
  // the split's region (centre o relative to t, radius) when the splits follow regions, else the mesh
  const double4 geo = a.split_geo ? a.split_geo[blockIdx.y] : make_double4(0.0, 0.0, 0.0, a.info[0].R);
  const double o[3] = {geo.x, geo.y, geo.z};
  const bool small = sqrt(Q2) * geo.w < a.tau0;
  int64_t f_begin, f_end;
  split_faces(a, blockIdx.y, f_begin, f_end);
  double xr = 0.0, xi = 0.0;
  for (int64_t t0 = f_begin; t0 < f_end; t0 += kTileF) {
    const int nt = (int)min((int64_t)kTileF, f_end - t0);
    __syncthreads();
    {
      const uint4* src = reinterpret_cast<const uint4*>(a.f64 + t0);
      uint4* dst = reinterpret_cast<uint4*>(tile);
      for (int i = threadIdx.x; i < nt * (int)(sizeof(Face64) / 16); i += kBlock) dst[i] = src[i];
    }
    __syncthreads();
    if (!small) {
      for (int j = 0; j < nt; ++j) {
        double Tr, Ti;
        face_term_f64(tile[j], Q, Tr, Ti);
        xr += Tr;
        xi += Ti;
      }
    } else {
      for (int j = 0; j < nt; ++j) tet_term_f64(tile[j], Q, xr, xi, o);
    }
  }
  if (small && a.split_geo) apex_phase(Q, o, xr, xi);
  if (active) store_stream(a.partial + (int64_t)blockIdx.y * a.nq + qi, make_double2(xr, xi));
}

// Sum the splits in order, apply exp(i Q.t) and 1/|Q|^2, write F and |F|^2 at
// the caller's index of the visited Q.
__global__ __launch_bounds__(256) void fwd3d_finish_kernel(FwdArgs a, int out_c128) {
  const int64_t qi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= a.nq) return;
  const int64_t dst = a.perm ? (int64_t)a.perm[qi] : qi;
  double Q[3];
  load_q3(a.q, a.qdtype, dst, Q);
  double xr, xi;
  fwd_partial_sum(a, qi, xr, xi);
  const MeshInfo mi = a.info[0];
  const double Q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
  const bool small = sqrt(Q2) * mi.R < a.tau0;
  if (!small) {
    xr /= Q2;
    xi /= Q2;
  }
  double st, ct;
  sincos(Q[0] * mi.t[0] + Q[1] * mi.t[1] + Q[2] * mi.t[2], &st, &ct);
  double Fr = ct * xr - st * xi;
  double Fi = ct * xi + st * xr;
  if (!out_c128 && fp32c_phase_out_of_range(sqrt(Q2), mi)) Fr = Fi = quiet_nan();  // beyond the FP32C phase range
  if (out_c128) {
    if (a.out) static_cast<double2*>(a.out)[dst] = make_double2(Fr, Fi);
    if (a.intensity) static_cast<double*>(a.intensity)[dst] = Fr * Fr + Fi * Fi;
  } else {
    if (a.out) static_cast<float2*>(a.out)[dst] = make_float2((float)Fr, (float)Fi);
    if (a.intensity) static_cast<float*>(a.intensity)[dst] = (float)(Fr * Fr + Fi * Fi);
  }
}

}  // namespace

hipError_t launch_fwd3d_fp64(const FwdArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.nq + kBlock - 1) / kBlock), (unsigned)a.splits);
  fwd3d_fp64_kernel<<<grid, kBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_fwd3d_fp32c(const FwdArgs& a, hipStream_t s) {
  const int64_t qtiles = (a.nq + kFwdQTile - 1) / kFwdQTile;
  const int64_t blocks = (qtiles + kXcds - 1) / kXcds * kXcds * a.splits;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  if (!a.share_edges) return launch_fwd3d_fp32c_list(a, s);
  fwd3d_fp32c_kernel<true><<<(unsigned)blocks, kFwdBlock, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_fwd3d_finish(const FwdArgs& a, int out_c128, hipStream_t s) {
  fwd3d_finish_kernel<<<(unsigned)((a.nq + 255) / 256), 256, 0, s>>>(a, out_c128);
  return hipGetLastError();
}

}  // namespace pft
