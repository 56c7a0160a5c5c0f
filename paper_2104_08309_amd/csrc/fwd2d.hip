// Forward 2D transform of a polygon (one or more closed contours), binary64.
//
// 2D section of the paper: with the field F = -iQ exp(iQ.r)/Q^2 (whose
// divergence is exp(iQ.r)), the area integral becomes a sum over contour
// edges of the flux through each edge (eq. line_integral_generic), whose
// exponential difference is written in midpoint form as
//   (exp(iQ.r_{l+1}) - exp(iQ.r_l)) / (Q.d_l) = i exp(iQ.m_l) sinc(Q.d_l/2),
// and with (Q.n_l)|d_l| = Qx dy - Qy dx for the outward normal of a
// counter-clockwise edge (eq. line_normal):
//   F(Q) = -(i/|Q|^2) sum_l (Qx dy_l - Qy dx_l) exp(iQ.m_l) sinc(Q.d_l/2).
// Coordinates are relative to the vertex mean t; F gets exp(iQ.t) at the end.
// For |Q| R < tau0 the area is summed as the fan of triangles (t, r_l, r_{l+1})
// through their simplex series, which is exact at Q = 0 (signed area).
#include "pft_device.h"

namespace pft {
namespace {

// Block layout: kQ2D Q points x kGroups2D edge groups; the thread of (Q, group g) sums the edges
// g, g + kGroups2D, ... of each LDS tile, and the groups' sums are added in the order g = 0, 1, ...
// so that a polygon of a few dozen edges still gives every CU several waves.
constexpr int kGroups2D = 8;
constexpr int kQ2D = kBlock / kGroups2D;

__device__ __forceinline__ void edge_term_2d(const Edge2D& e, double Qx, double Qy, double& xr, double& xi) {
  const double dx = e.b[0] - e.a[0], dy = e.b[1] - e.a[1];
  const double mx = 0.5 * (e.a[0] + e.b[0]), my = 0.5 * (e.a[1] + e.b[1]);
  const double eta = 0.5 * (Qx * dx + Qy * dy);
  double sinc;
  if (fabs(eta) < 0.1) {
    const double x2 = eta * eta;
    sinc = 1.0 + x2 * (-1.0 / 6.0 + x2 * (1.0 / 120.0 + x2 * (-1.0 / 5040.0 + x2 * (1.0 / 362880.0))));
  } else {
    sinc = sin(eta) / eta;
  }
  double sm, cm;
  sincos(Qx * mx + Qy * my, &sm, &cm);
  const double wgt = (Qx * dy - Qy * dx) * sinc;
  // -i * wgt * exp(i Q.m)
  xr += wgt * sm;
  xi -= wgt * cm;
}

// Triangle (t, a, b) of the fan by its simplex series: 2 |T| sum_n i^n h_n(0, Q.a, Q.b) / (n+2)!.
__device__ __forceinline__ void fan_term_2d(const Edge2D& e, double Qx, double Qy, double& xr, double& xi) {
  const double two_a = e.a[0] * e.b[1] - e.a[1] * e.b[0];
  const double xa = Qx * e.a[0] + Qy * e.a[1];
  const double xb = Qx * e.b[0] + Qy * e.b[1];
  // h_n = e1 h_{n-1} - e2 h_{n-2}
  const double e1 = xa + xb, e2 = xa * xb;
  const double m = fmax(fabs(xa), fabs(xb));
  double hm2 = 0.0, hm1 = 1.0, inv = 1.0 / 6.0, sr = 0.5, si = 0.0, mn = 1.0;
  for (int n = 1; n < 80; ++n) {
    const double h = e1 * hm1 - e2 * hm2;
    const double term = h * inv;
    switch (n & 3) {
      case 0: sr += term; break;
      case 1: si += term; break;
      case 2: sr -= term; break;
      default: si -= term; break;
    }
    hm2 = hm1;
    hm1 = h;
    mn *= m;
    if (n >= 2 && mn * (n + 1) * inv < 1e-17 * (fabs(sr) + fabs(si))) break;
    inv /= (double)(n + 3);
  }
  xr += two_a * sr;
  xi += two_a * si;
}

__global__ __launch_bounds__(kBlock) void fwd2d_kernel(const Edge2D* edges, int64_t ne, const MeshInfo* info,
                                                       const double* q, int64_t nq, double tau0, double* out) {
  __shared__ Edge2D tile[kTileE];
  __shared__ double2 part[kGroups2D][kQ2D];
  const int lq = threadIdx.x % kQ2D, grp = threadIdx.x / kQ2D;
  const int64_t qi = (int64_t)blockIdx.x * kQ2D + lq;
  const bool active = qi < nq;
  const double Qx = active ? q[2 * qi] : 0.0;
  const double Qy = active ? q[2 * qi + 1] : 0.0;
  const double Q2 = Qx * Qx + Qy * Qy;
  const MeshInfo mi = info[0];
  const bool small = sqrt(Q2) * mi.R < tau0;
  double xr = 0.0, xi = 0.0;
  for (int64_t t0 = 0; t0 < ne; t0 += kTileE) {
    const int nt = (int)min((int64_t)kTileE, ne - t0);
    __syncthreads();
    for (int i = threadIdx.x; i < nt * 2; i += kBlock)
      reinterpret_cast<uint4*>(tile)[i] = reinterpret_cast<const uint4*>(edges + t0)[i];
    __syncthreads();
    if (!small) {
      for (int j = grp; j < nt; j += kGroups2D) edge_term_2d(tile[j], Qx, Qy, xr, xi);
    } else {
      for (int j = grp; j < nt; j += kGroups2D) fan_term_2d(tile[j], Qx, Qy, xr, xi);
    }
  }
  part[grp][lq] = make_double2(xr, xi);
  __syncthreads();
  if (grp != 0 || !active) return;
  xr = xi = 0.0;
  for (int g = 0; g < kGroups2D; ++g) {
    xr += part[g][lq].x;
    xi += part[g][lq].y;
  }
  if (!small) {
    xr /= Q2;
    xi /= Q2;
  }
  double st, ct;
  sincos(Qx * mi.t[0] + Qy * mi.t[1], &st, &ct);
  out[2 * qi] = ct * xr - st * xi;
  out[2 * qi + 1] = ct * xi + st * xr;
}

}  // namespace

hipError_t launch_fwd2d(const Edge2D* edges, int64_t ne, const MeshInfo* info, double, const double* q, int64_t nq,
                        double tau0, double* out, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  fwd2d_kernel<<<(unsigned)((nq + kQ2D - 1) / kQ2D), kBlock, 0, s>>>(edges, ne, info, q, nq, tau0, out);
  return hipGetLastError();
}

}  // namespace pft
