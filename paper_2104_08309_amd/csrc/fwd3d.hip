// Forward 3D transform of a closed triangle mesh: F(Q) for a list of Q.
//
// Layout: Q-tiles of threads (binary64: one Q per thread; FP32C: QPT Q per
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
#include "fwd_terms.h"

namespace pft {
namespace {

// The tetrahedron fan about an apex o (relative to t) gives the integral of exp(iQ.(r - o)); times
// exp(iQ.o) it is relative to t like the surface sums.
__device__ __forceinline__ void apex_phase(const double* Q, const double* o, double& xr, double& xi) {
  double so, co;
  sincos(Q[0] * o[0] + Q[1] * o[1] + Q[2] * o[2], &so, &co);
  const double r = co * xr - so * xi;
  xi = co * xi + so * xr;
  xr = r;
}

// Face range of split `sp`: from the split table when the splits follow region boundaries, else equal
// ranges.
__device__ __forceinline__ void split_faces(const FwdArgs& a, int64_t sp, int64_t& b, int64_t& e) {
  if (a.split_face) {
    b = a.split_face[sp];
    e = a.split_face[sp + 1];
  } else {
    b = sp * a.faces_per_split;
    e = min(a.nf, b + a.faces_per_split);
  }
}

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

// The FP32C forward. A block holds one Q-tile of kQT = 64 QPT Q, the same in each of its
// kFwdSplitWaves wavefronts (lane l holds the tile's Q l, l + 64, ...; QPT per thread, so each face
// record read from LDS serves QPT independent instruction streams), and one face split. The grid is
// one-dimensional and its blocks go to the dies in turn (block b to die b mod kXcds), so the block
// index is read as (die, rank on the die) and the k-th group of `splits` blocks a die receives holds
// every split of one Q-tile: a Q-tile's Q and permutation entries are fetched into that die's L2 once
// and served from there to its other splits (the Q-tile count is padded to a multiple of kXcds; the
// padding blocks exit at once).
// Each wavefront takes its own contiguous share of the split's faces and streams them through its own
// LDS tile of kTileF32 records, with wavefront-local ordering only: no block barrier after the start.
// A wavefront that is done leaves its binary64 partials in its own tile and counts itself done; the
// last of the block's wavefronts adds their partials of each Q in wavefront order and writes them (one
// partial per Q and block), and the others exit at once. SHARE: the records are in an
// edge-sharing order and each face takes one edge term from its predecessor in the wavefront's range
// (two edge terms per face instead of three). Small-|Q| lanes (|Q| R < tau0, R the split's radius) take
// the binary64 tetrahedron fan about the split's apex.
template <bool SHARE, int QPT>
__global__ __launch_bounds__(kFwdBlock, fwd_waves(QPT)) void fwd3d_fp32c_kernel(FwdArgs a) {
  constexpr int kQT = fwd_qtile(QPT);
  __shared__ Face32 tiles[kFwdSplitWaves][kTileF32];
  __shared__ float qlo[kFwdSplitWaves][3 * QPT * 64];
  __shared__ uint32_t done;  // wavefronts of the block that have left their partials
  static_assert(sizeof(Face32) * kTileF32 >= sizeof(double2) * QPT * 64, "a wavefront's partials fit its tile");
  // (Q-tile, split) of this block from its die and rank on the die
  const uint32_t rank = blockIdx.x / kXcds;
  const uint32_t qtile = blockIdx.x % kXcds + kXcds * (rank / (uint32_t)a.splits);
  const uint32_t sp = rank % (uint32_t)a.splits;
  if ((int64_t)qtile * kQT >= a.nq) return;  // padding of the Q-tile count (whole block)
  if (threadIdx.x == 0) done = 0u;
  __syncthreads();
  // the wavefront index as a wavefront-uniform (scalar) value, so the face range and tile addresses
  // derived from it stay in scalar registers
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = (int)(threadIdx.x & 63);
  Face32* tile = tiles[w];
  const double4 geo = a.split_geo ? a.split_geo[sp] : make_double4(0.0, 0.0, 0.0, a.info[0].R);
  const double R = geo.w;
  const double o[3] = {geo.x, geo.y, geo.z};
  int64_t f_begin, f_end;
  split_faces(a, sp, f_begin, f_end);
  {  // this wavefront's share
    const int64_t per = (f_end - f_begin + kFwdSplitWaves - 1) / kFwdSplitWaves;
    const int64_t b = min(f_end, f_begin + w * per);
    f_end = min(f_end, b + per);
    f_begin = b;
  }
  const int64_t qbase = (int64_t)qtile * kQT + lane;
  QLowLds<QPT> ql;
  ql.lo = qlo[w];
  ql.lane = lane;
  float qx[QPT], qy[QPT], qz[QPT], Q2[QPT];
  bool small[QPT], active[QPT];
  bool any_small = false;
#pragma unroll
  for (int k = 0; k < QPT; ++k) {
    const int64_t qi = qbase + (int64_t)k * 64;
    active[k] = qi < a.nq;
    double Qd[3] = {0.0, 0.0, 0.0};
    if (active[k]) load_q3(a.q, a.qdtype, a.perm ? (int64_t)a.perm[qi] : qi, Qd);
    qx[k] = (float)Qd[0];
    qy[k] = (float)Qd[1];
    qz[k] = (float)Qd[2];
    ql.set(k, Qd, qx[k], qy[k], qz[k]);
    Q2[k] = qx[k] * qx[k] + qy[k] * qy[k] + qz[k] * qz[k];
    const double Q2d = Qd[0] * Qd[0] + Qd[1] * Qd[1] + Qd[2] * Qd[2];
    small[k] = sqrt(Q2d) * R < a.tau0;
    any_small |= small[k];
  }
  float qmax = 0.0f;
#pragma unroll
  for (int k = 0; k < QPT; ++k) qmax = fmaxf(qmax, sqrtf(Q2[k]));
  const bool check = __builtin_amdgcn_readfirstlane((int)sinc_range_test_needed(wave_max(qmax), a.info[0].rho)) != 0;
  float sr[QPT], si[QPT], cr[QPT], ci[QPT];
#pragma unroll
  for (int k = 0; k < QPT; ++k) sr[k] = si[k] = cr[k] = ci[k] = 0.0f;
  FwdCarry<QPT> carry;  // shared edge term from the previous face (SHARE)
  carry.reset();         // no previous face at the start of the range
  for (int64_t t0 = f_begin; t0 < f_end; t0 += kTileF32) {
    const int nt = (int)min((int64_t)kTileF32, f_end - t0);
    // the wavefront's previous tile has been read (its LDS reads were issued in order before these
    // writes); its writes are complete before any lane reads the tile
    wave_lds_fence();
    {
      const uint4* src = reinterpret_cast<const uint4*>(a.f32 + t0);
      uint4* d = reinterpret_cast<uint4*>(tile);
      for (int i = lane; i < nt * (int)(sizeof(Face32) / 16); i += 64) d[i] = src[i];
    }
    wave_lds_fence();
    float tr[QPT], ti[QPT];
#pragma unroll
    for (int k = 0; k < QPT; ++k) tr[k] = ti[k] = 0.0f;
    if (check)
      fwd_tile_fp32c<QPT, SHARE, true, SHARE>(tile, nt, qx, qy, qz, ql, small, tr, ti, carry);
    else
      fwd_tile_fp32c<QPT, SHARE, false, SHARE>(tile, nt, qx, qy, qz, ql, small, tr, ti, carry);
#pragma unroll
    for (int k = 0; k < QPT; ++k) {
      kahan_add(sr[k], cr[k], tr[k]);
      kahan_add(si[k], ci[k], ti[k]);
    }
  }
  // small-|Q| lanes: the binary64 tetrahedron fan over the range's faces, after the surface sums (the
  // rare wavefronts that hold such a lane pay for it; the others keep no binary64 sums live above)
  double xr[QPT], xi[QPT];
#pragma unroll
  for (int k = 0; k < QPT; ++k) xr[k] = xi[k] = 0.0;
  if (any_small) {
#pragma unroll
    for (int k = 0; k < QPT; ++k)
      if (small[k]) {
        const double Qd[3] = {ql.qd(qx[k], k, 0), ql.qd(qy[k], k, 1), ql.qd(qz[k], k, 2)};
        for (int64_t j = f_begin; j < f_end; ++j) tet_term_f64(a.f64[j], Qd, xr[k], xi[k], o);
        if (a.split_geo) apex_phase(Qd, o, xr[k], xi[k]);
      }
  }
  // this wavefront's partials into its own tile (it reads no more records)
  wave_lds_fence();
  double2* red = reinterpret_cast<double2*>(tiles[w]);
#pragma unroll
  for (int k = 0; k < QPT; ++k)
    red[k * 64 + lane] = small[k] ? make_double2(xr[k], xi[k])
                                  : make_double2(((double)sr[k] - (double)cr[k]) * kInvSumScale32,
                                                 ((double)si[k] - (double)ci[k]) * kInvSumScale32);
  // count this wavefront done once its partials are visible to the block; the last one adds them all
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  int last = 0;
  if (lane == 0) last = atomicAdd(&done, 1u) == (uint32_t)(kFwdSplitWaves - 1) ? 1 : 0;
  if (__builtin_amdgcn_readfirstlane(last) == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  // the lane index anew (from the lane mask, not threadIdx), so no Q index is kept live across the loop
  const int l = (int)__lane_id();
#pragma unroll
  for (int k = 0; k < QPT; ++k) {
    const int64_t qi = (int64_t)qtile * kQT + k * 64 + l;
    double2 v = reinterpret_cast<const double2*>(tiles[0])[k * 64 + l];
    for (int u = 1; u < kFwdSplitWaves; ++u) {
      const double2 x = reinterpret_cast<const double2*>(tiles[u])[k * 64 + l];
      v.x += x.x;
      v.y += x.y;
    }
    if (qi < a.nq) store_stream(a.partial + (int64_t)sp * a.nq + qi, v);
  }
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
  if (a.qpt != kQPT && a.qpt != kQPTLarge) return hipErrorInvalidValue;
  const int64_t qtiles = (a.nq + fwd_qtile(a.qpt) - 1) / fwd_qtile(a.qpt);
  const int64_t blocks = (qtiles + kXcds - 1) / kXcds * kXcds * a.splits;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  const bool large = a.qpt == kQPTLarge && kQPTLarge != kQPT;
  if (a.share_edges) {
    if (large)
      fwd3d_fp32c_kernel<true, kQPTLarge><<<(unsigned)blocks, kFwdBlock, 0, s>>>(a);
    else
      fwd3d_fp32c_kernel<true, kQPT><<<(unsigned)blocks, kFwdBlock, 0, s>>>(a);
  } else {
    if (large)
      fwd3d_fp32c_kernel<false, kQPTLarge><<<(unsigned)blocks, kFwdBlock, 0, s>>>(a);
    else
      fwd3d_fp32c_kernel<false, kQPT><<<(unsigned)blocks, kFwdBlock, 0, s>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_fwd3d_finish(const FwdArgs& a, int out_c128, hipStream_t s) {
  fwd3d_finish_kernel<<<(unsigned)((a.nq + 255) / 256), 256, 0, s>>>(a, out_c128);
  return hipGetLastError();
}

}  // namespace pft
