// Prologue kernels: per-mesh centre and radius, per-face and per-edge records.
//
// The records carry the geometry each (Q, face) evaluation needs, relative to
// local origins, so that the hot loops see small coordinates: the mesh is
// re-centred on its vertex mean t, each face on its centroid g. Everything here
// runs once per call in binary64 and is O(V + F).
#include "pft_internal.h"

namespace pft {
namespace {

constexpr double kInv2Pi = 0.15915494309189533577;
constexpr double kInv4Pi = 0.07957747154594766788;

__device__ inline void load_vertex(const void* verts, int vdtype, int dim, int64_t i, double* out) {
  if (vdtype == PFT_F64) {
    const double* v = static_cast<const double*>(verts) + i * dim;
    for (int k = 0; k < dim; ++k) out[k] = v[k];
  } else {
    const float* v = static_cast<const float*>(verts) + i * dim;
    for (int k = 0; k < dim; ++k) out[k] = (double)v[k];
  }
}

// One block of kInfoBlock threads per mesh: t = vertex mean, R = max |v - t|. Each thread takes every
// kInfoBlock-th vertex; the per-thread values are combined by a fixed butterfly within each wavefront and
// then wavefront by wavefront in order, so the result does not depend on timing.
constexpr int kInfoBlock = 1024;

__device__ __forceinline__ double info_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double info_wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__global__ __launch_bounds__(kInfoBlock) void mesh_info_kernel(const void* verts, int vdtype, int dim,
                                                              int64_t nv_single, const int64_t* vert_off,
                                                              MeshInfo* info) {
  constexpr int kWaves = kInfoBlock / 64;
  __shared__ double red[kWaves][3];
  const int64_t mesh = blockIdx.x;
  const int64_t v0 = vert_off ? vert_off[mesh] : 0;
  const int64_t v1 = vert_off ? vert_off[mesh + 1] : nv_single;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t i = v0 + tid; i < v1; i += kInfoBlock) {
    double p[3] = {0.0, 0.0, 0.0};
    load_vertex(verts, vdtype, dim, i, p);
    for (int k = 0; k < 3; ++k) s[k] += p[k];
  }
  for (int k = 0; k < 3; ++k) s[k] = info_wave_sum(s[k]);
  if (lane == 0)
    for (int k = 0; k < 3; ++k) red[w][k] = s[k];
  __syncthreads();
  const int64_t n = v1 - v0;
  double t[3];
  for (int k = 0; k < 3; ++k) {
    double a = 0.0;
    for (int u = 0; u < kWaves; ++u) a += red[u][k];
    t[k] = n > 0 ? a / (double)n : 0.0;
  }
  __syncthreads();  // every thread has read the sums before red is reused
  double r2 = 0.0;
  for (int64_t i = v0 + tid; i < v1; i += kInfoBlock) {
    double p[3] = {0.0, 0.0, 0.0};
    load_vertex(verts, vdtype, dim, i, p);
    double d2 = 0.0;
    for (int k = 0; k < dim; ++k) d2 += (p[k] - t[k]) * (p[k] - t[k]);
    r2 = fmax(r2, d2);
  }
  r2 = info_wave_max(r2);
  if (lane == 0) red[w][0] = r2;
  __syncthreads();
  if (tid == 0) {
    double r = 0.0;
    for (int u = 0; u < kWaves; ++u) r = fmax(r, red[u][0]);
    MeshInfo m;
    for (int k = 0; k < 3; ++k) m.t[k] = t[k];
    m.R = sqrt(r);
    m.rho = 0.0;  // raised by the face prologue
    m.pad = 0.0;
    info[mesh] = m;
  }
}

__device__ inline void make_face64(const double* a, const double* b, const double* c, double tau, Face64& f) {
  double g[3], u0[3], u1[3], e0[3], e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    g[k] = (a[k] + b[k] + c[k]) / 3.0;
    u0[k] = a[k] - g[k];
    u1[k] = b[k] - g[k];
    e0[k] = b[k] - a[k];
    e1[k] = c[k] - b[k];
    e2[k] = a[k] - c[k];
  }
  // N = (b - a) x (c - a) = e0 x (-e2)
  double N[3] = {e0[1] * (c[2] - a[2]) - e0[2] * (c[1] - a[1]),
                 e0[2] * (c[0] - a[0]) - e0[0] * (c[2] - a[2]),
                 e0[0] * (c[1] - a[1]) - e0[1] * (c[0] - a[0])};
  double N2 = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
  double L2 = 0.0;
  L2 = fmax(L2, e0[0] * e0[0] + e0[1] * e0[1] + e0[2] * e0[2]);
  L2 = fmax(L2, e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  L2 = fmax(L2, e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
  for (int k = 0; k < 3; ++k) {
    f.g[k] = g[k];
    f.u0[k] = u0[k];
    f.u1[k] = u1[k];
    f.N[k] = N[k];
  }
  f.thr = (N2 > 0.0 && L2 > 0.0) ? tau * tau * N2 / L2 : -1.0;
  f.pad[0] = L2;
  f.pad[1] = N2;
  f.pad[2] = 0.0;
}

__device__ inline void empty_face64(Face64& f) {
  for (int k = 0; k < 3; ++k) f.g[k] = f.u0[k] = f.u1[k] = f.N[k] = 0.0;
  f.thr = -1.0;
  f.pad[0] = f.pad[1] = f.pad[2] = 0.0;
}

// Largest squared distance from a face record's centroid to its vertices (u0, u1, -u0 - u1).
__device__ inline double face_extent2(const Face64& f) {
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double w = -f.u0[k] - f.u1[k];
    d0 += f.u0[k] * f.u0[k];
    d1 += f.u1[k] * f.u1[k];
    d2 += w * w;
  }
  return fmax(d0, fmax(d1, d2));
}

// Raise info[mesh].rho to sqrt(ext2) over the lanes of the wavefront. Every lane
// of the wavefront must reach this call (lanes without a face pass ext2 = 0);
// the lanes of the first lane's mesh are reduced to one atomic, any other lane
// (a wavefront that straddles two meshes of a batch) raises its own. rho >= 0,
// so its binary64 pattern orders like an unsigned integer.
__device__ inline void raise_rho(MeshInfo* info, int64_t mesh, double ext2) {
  const int64_t mesh0 = __shfl(mesh, 0);
  double r = mesh == mesh0 ? ext2 : 0.0;
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off));
  if ((threadIdx.x & 63) == 0 && r > 0.0)
    atomicMax(reinterpret_cast<unsigned long long*>(&info[mesh0].rho), (unsigned long long)__double_as_longlong(sqrt(r)));
  if (mesh != mesh0 && ext2 > 0.0)
    atomicMax(reinterpret_cast<unsigned long long*>(&info[mesh].rho),
              (unsigned long long)__double_as_longlong(sqrt(ext2)));
}

// The edge-sharing flags of position m kept in Face64::pad[2] for the FP32C record
// builder: 1 = linked to the previous position, 2 = traversal reversed. The Face64
// record itself keeps the outward (rotated) vertex order.
__device__ __forceinline__ int order_code(const uint8_t* meta, int64_t m) {
  if (!meta) return 0;
  return ((meta[m] & kMetaLink) ? 1 : 0) | ((meta[m] & kMetaReflect) ? 2 : 0);
}

__global__ __launch_bounds__(256) void face64_kernel(const void* verts, int vdtype, int64_t nv, const int32_t* tris,
                                                     int64_t nf, MeshInfo* info, double tau, Face64* out,
                                                     const int32_t* order, const uint8_t* meta) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double ext2 = 0.0;
  if (m < nf) {
    // the face at this position of the (optional) edge-sharing order, its vertex list rotated
    const int64_t src = order ? (int64_t)order[m] : m;
    const int rot = meta ? (meta[m] & 3) : 0;
    const int code = order_code(meta, m);
    Face64 f;
    const bool in_list = src >= 0 && src < nf && rot < 3;
    const int32_t ia = in_list ? tris[3 * src + rot] : -1;
    const int32_t ib = in_list ? tris[3 * src + (rot + 1) % 3] : -1;
    const int32_t ic = in_list ? tris[3 * src + (rot + 2) % 3] : -1;
    if (ia < 0 || ib < 0 || ic < 0 || ia >= nv || ib >= nv || ic >= nv) {
      empty_face64(f);
    } else {
      double a[3], b[3], c[3];
      load_vertex(verts, vdtype, 3, ia, a);
      load_vertex(verts, vdtype, 3, ib, b);
      load_vertex(verts, vdtype, 3, ic, c);
      const MeshInfo mi = info[0];
      for (int k = 0; k < 3; ++k) {
        a[k] -= mi.t[k];
        b[k] -= mi.t[k];
        c[k] -= mi.t[k];
      }
      make_face64(a, b, c, tau, f);
      f.pad[2] = (double)code;
      ext2 = face_extent2(f);
    }
    out[m] = f;
  }
  raise_rho(info, 0, ext2);
}

// One thread per polygon face: vertex mean g, area vector N = sum_k u_k x u_{k+1}
// (u_k = r_k - g; exact for a planar face), longest edge, vertex offsets. A face
// with an out-of-range index or zero area becomes empty (all-zero records).
__global__ __launch_bounds__(256) void poly64_kernel(const void* verts, int vdtype, int64_t nv,
                                                     const int64_t* face_off, const int32_t* face_verts, int64_t nf,
                                                     MeshInfo* info, double tau, FaceP64* fout,
                                                     VtxP64* vout) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double ext2 = 0.0;
  if (m < nf) {
    const int64_t b = face_off[m], e = face_off[m + 1];
    const int n = (int)(e - b);
    bool ok = n >= 3;
    for (int64_t k = b; k < e; ++k) ok = ok && face_verts[k] >= 0 && face_verts[k] < nv;
    const MeshInfo mi = info[0];
    FaceP64 f;
    f.v0 = (int32_t)b;
    f.nv = n;
    f.pad[0] = f.pad[1] = 0;
    double g[3] = {0.0, 0.0, 0.0};
    if (ok) {
      for (int64_t k = b; k < e; ++k) {
        double r[3];
        load_vertex(verts, vdtype, 3, face_verts[k], r);
        for (int c = 0; c < 3; ++c) g[c] += r[c] - mi.t[c];
      }
      for (int c = 0; c < 3; ++c) g[c] /= (double)n;
    }
    double N[3] = {0.0, 0.0, 0.0}, L2 = 0.0;
    double u0[3] = {0.0, 0.0, 0.0}, uprev[3] = {0.0, 0.0, 0.0};
    for (int64_t k = b; k < e; ++k) {
      double u[3] = {0.0, 0.0, 0.0};
      if (ok) {
        load_vertex(verts, vdtype, 3, face_verts[k], u);
        for (int c = 0; c < 3; ++c) u[c] -= mi.t[c] + g[c];
        ext2 = fmax(ext2, u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      }
      VtxP64 r;
      r.u[0] = u[0];
      r.u[1] = u[1];
      r.u[2] = u[2];
      r.pad = 0.0;
      vout[k] = r;
      if (k == b) {
        for (int c = 0; c < 3; ++c) u0[c] = u[c];
      } else {
        N[0] += uprev[1] * u[2] - uprev[2] * u[1];
        N[1] += uprev[2] * u[0] - uprev[0] * u[2];
        N[2] += uprev[0] * u[1] - uprev[1] * u[0];
        double d2 = 0.0;
        for (int c = 0; c < 3; ++c) d2 += (u[c] - uprev[c]) * (u[c] - uprev[c]);
        L2 = fmax(L2, d2);
      }
      for (int c = 0; c < 3; ++c) uprev[c] = u[c];
    }
    if (n >= 1) {  // closing edge
      N[0] += uprev[1] * u0[2] - uprev[2] * u0[1];
      N[1] += uprev[2] * u0[0] - uprev[0] * u0[2];
      N[2] += uprev[0] * u0[1] - uprev[1] * u0[0];
      double d2 = 0.0;
      for (int c = 0; c < 3; ++c) d2 += (u0[c] - uprev[c]) * (u0[c] - uprev[c]);
      L2 = fmax(L2, d2);
    }
    const double N2 = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
    ok = ok && N2 > 0.0 && L2 > 0.0;
    for (int c = 0; c < 3; ++c) {
      f.g[c] = ok ? g[c] : 0.0;
      f.N[c] = ok ? N[c] : 0.0;
    }
    f.thr = ok ? tau * tau * N2 / L2 : -1.0;
    f.invN = ok ? 1.0 / sqrt(N2) : 0.0;
    fout[m] = f;
    if (!ok) ext2 = 0.0;
  }
  raise_rho(info, 0, ext2);
}

// FP32C polygon records: orthonormal in-plane basis (e1 along the first edge of
// non-zero length, e2 = n x e1) and the per-vertex coefficients.
__global__ __launch_bounds__(256) void poly32_kernel(const FaceP64* fin, const VtxP64* vin, int64_t nf,
                                                     double tau_rel, FaceP32* fout, VtxP32* vout) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  const FaceP64 f = fin[m];
  const bool ok = f.thr >= 0.0;
  const double N2 = f.N[0] * f.N[0] + f.N[1] * f.N[1] + f.N[2] * f.N[2];
  const double nN = sqrt(N2);
  double e1[3] = {0.0, 0.0, 0.0}, e2[3] = {0.0, 0.0, 0.0};
  if (ok) {
    for (int k = 0; k < f.nv; ++k) {
      const VtxP64 a = vin[f.v0 + k], b = vin[f.v0 + (k + 1) % f.nv];
      double d[3] = {b.u[0] - a.u[0], b.u[1] - a.u[1], b.u[2] - a.u[2]};
      const double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (dl > 0.0) {
        for (int c = 0; c < 3; ++c) e1[c] = d[c] / dl;
        break;
      }
    }
    // e2 = n x e1
    e2[0] = (f.N[1] * e1[2] - f.N[2] * e1[1]) / nN;
    e2[1] = (f.N[2] * e1[0] - f.N[0] * e1[2]) / nN;
    e2[2] = (f.N[0] * e1[1] - f.N[1] * e1[0]) / nN;
  }
  FaceP32 r;
  for (int c = 0; c < 3; ++c) {
    r.gt[c] = f.g[c] * kInv2Pi;
    r.N[c] = (float)f.N[c];
    r.E1[c] = (float)(nN * e1[c]);
    r.E2[c] = (float)(nN * e2[c]);
  }
  r.thr = ok ? (float)f.thr : -1.0f;  // the binary64 records were built with this form's threshold
  r.kap = ok ? (float)(tau_rel * tau_rel * N2) : -1.0f;
  r.invN = (float)f.invN;
  r.v0 = f.v0;
  r.nv = f.nv;
  r.pad[0] = r.pad[1] = 0;
  fout[m] = r;
  for (int k = 0; k < f.nv; ++k) {
    const VtxP64 a = vin[f.v0 + k], b = vin[f.v0 + (k + 1) % f.nv];
    VtxP32 v;
    if (ok) {
      const double d[3] = {b.u[0] - a.u[0], b.u[1] - a.u[1], b.u[2] - a.u[2]};
      const double x = e1[0] * a.u[0] + e1[1] * a.u[1] + e1[2] * a.u[2];
      const double y = e2[0] * a.u[0] + e2[1] * a.u[1] + e2[2] * a.u[2];
      v.ga = (float)(x * kInv4Pi / nN);
      v.de = (float)(y * kInv4Pi / nN);
      v.al = (float)((e1[0] * d[0] + e1[1] * d[1] + e1[2] * d[2]) * kInv2Pi);
      v.be = (float)(-(e2[0] * d[0] + e2[1] * d[1] + e2[2] * d[2]) * kInv2Pi);
      v.x = (float)x;
      v.y = (float)y;
    } else {
      v.ga = v.de = v.al = v.be = v.x = v.y = 0.0f;
    }
    vout[f.v0 + k] = v;
  }
}

__global__ __launch_bounds__(256) void face_mesh_kernel(const int64_t* tri_off, int64_t n_meshes, int64_t nf_total,
                                                        int32_t* face_mesh) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf_total) return;
  // last mesh i with tri_off[i] <= f (meshes may be empty)
  int64_t lo = 0, hi = n_meshes;  // invariant: tri_off[lo] <= f < tri_off[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if (tri_off[mid] <= f) lo = mid; else hi = mid;
  }
  face_mesh[f] = (int32_t)lo;
}

__global__ __launch_bounds__(256) void face64_batch_kernel(const void* verts, int vdtype, const int32_t* tris,
                                                           const int64_t* vert_off, const int64_t* tri_off,
                                                           const int32_t* face_mesh, int64_t nf_total,
                                                           MeshInfo* info, double tau, Face64* out,
                                                           const int32_t* order, const uint8_t* meta) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double ext2 = 0.0;
  const int32_t mesh = m < nf_total ? face_mesh[m] : -1;
  if (m < nf_total) {
    const int64_t vb = vert_off[mesh];
    const int64_t nv = vert_off[mesh + 1] - vb;
    // the face at this position of the (optional) edge-sharing order (within its mesh), rotated
    const int64_t src = order ? (int64_t)order[m] : m;
    const int rot = meta ? (meta[m] & 3) : 0;
    const int code = order_code(meta, m);
    const bool in_list = src >= 0 && src < nf_total && rot < 3;
    const int32_t ia = in_list ? tris[3 * src + rot] : -1;
    const int32_t ib = in_list ? tris[3 * src + (rot + 1) % 3] : -1;
    const int32_t ic = in_list ? tris[3 * src + (rot + 2) % 3] : -1;
    Face64 f;
    if (ia < 0 || ib < 0 || ic < 0 || ia >= nv || ib >= nv || ic >= nv) {
      empty_face64(f);
    } else {
      double a[3], b[3], c[3];
      load_vertex(verts, vdtype, 3, vb + ia, a);
      load_vertex(verts, vdtype, 3, vb + ib, b);
      load_vertex(verts, vdtype, 3, vb + ic, c);
      const MeshInfo mi = info[mesh];
      for (int k = 0; k < 3; ++k) {
        a[k] -= mi.t[k];
        b[k] -= mi.t[k];
        c[k] -= mi.t[k];
      }
      make_face64(a, b, c, tau, f);
      f.pad[2] = (double)code;
      ext2 = face_extent2(f);
    }
    out[m] = f;
  }
  raise_rho(info, mesh, ext2);
}


// A caller's Q visiting order made safe to index with: entries out of range
// become the position itself (a wrong order then gives wrong values, never an
// out-of-bounds access).
__global__ __launch_bounds__(256) void clamp_perm_kernel(const uint32_t* in, int64_t n, uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t v = in[i];
  out[i] = (int64_t)v < n ? v : (uint32_t)i;
}

__global__ __launch_bounds__(256) void iota_u32_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void face32_kernel(const Face64* in, int64_t nf, double tau, double tau_rel,
                                                     Face32* out) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  const Face64 f = in[m];
  Face32 r;
  const double L2 = f.pad[0], N2 = f.pad[1];
  const bool ok = f.thr >= 0.0;
  const int code = (int)f.pad[2];
  // linked only to a non-empty predecessor (an empty record carries no edge term)
  const bool link = ok && (code & 1) && m > 0 && in[m - 1].thr >= 0.0;
  const bool refl = (code & 2) != 0;
  // traversal order (a, b, c), or (b, a, c) reversed; the normal of the traversal
  double u0[3], u1[3], Nt[3], d0[3], d1[3], e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    u0[k] = refl ? f.u1[k] : f.u0[k];
    u1[k] = refl ? f.u0[k] : f.u1[k];
    Nt[k] = refl ? -f.N[k] : f.N[k];
    d0[k] = u1[k] - u0[k];
    d1[k] = -u0[k] - 2.0 * u1[k];
  }
  for (int k = 0; k < 3; ++k) r.gt[k] = f.g[k] * kInv2Pi;
  auto dot = [](const double* x, const double* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
  const double nN = sqrt(N2), nd0 = sqrt(dot(d0, d0));
  if (ok && nd0 > 0.0) {
    double d2[3];
    for (int k = 0; k < 3; ++k) {
      e1[k] = d0[k] / nd0;
      d2[k] = -d0[k] - d1[k];
    }
    // e2 = n x e1 = (N x d0) / (|N| |d0|), with the traversal's normal
    e2[0] = (Nt[1] * d0[2] - Nt[2] * d0[1]) / (nN * nd0);
    e2[1] = (Nt[2] * d0[0] - Nt[0] * d0[2]) / (nN * nd0);
    e2[2] = (Nt[0] * d0[1] - Nt[1] * d0[0]) / (nN * nd0);
    for (int k = 0; k < 3; ++k) {
      r.N[k] = (float)(0.5 * tau_rel * f.N[k] / nN);
      r.E1[k] = (float)(0.5 * e1[k]);
      r.E2[k] = (float)(0.5 * e2[k]);
    }
    const double* d[3] = {d0, d1, d2};
    for (int l = 0; l < 3; ++l) {
      r.al[l] = (float)(dot(e1, d[l]) * kInv2Pi);
      r.be[l] = (float)(-dot(e2, d[l]) * kInv2Pi);
    }
    r.thr = (float)(0.25 * tau * tau / L2);
    r.nN = (float)(2.0 * nN);
    r.flags = link ? kFaceLinked : 0u;
  } else {
    // empty face: every weight is zero; thr > 0 sends every pair to the series, whose term is
    // Q.N = 0 times a finite sum, so its contribution is exactly zero (the edge form would be 0/0)
    for (int k = 0; k < 3; ++k) r.N[k] = r.E1[k] = r.E2[k] = r.al[k] = r.be[k] = 0.0f;
    r.thr = 1.0f;
    r.nN = 0.0f;
    r.flags = 0u;
  }
  out[m] = r;
}

__global__ __launch_bounds__(256) void face32b_kernel(const Face64* in, int64_t nf, double tau, double tau_rel,
                                                      Face32B* out) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  const Face64 f = in[m];
  Face32B r;
  const double L2 = f.pad[0], N2 = f.pad[1];
  const bool ok = f.thr >= 0.0;
  double d0[3], d1[3], d2[3];
  for (int k = 0; k < 3; ++k) {
    d0[k] = f.u1[k] - f.u0[k];
    d1[k] = -f.u0[k] - 2.0 * f.u1[k];
    d2[k] = 2.0 * f.u0[k] + f.u1[k];
    r.gt[k] = f.g[k] * kInv2Pi;
    // an empty face gets an all-zero record: its weights stay finite and the
    // vertex gather multiplies them by N = 0
    r.N[k] = ok ? (float)f.N[k] : 0.0f;
    r.d0[k] = ok ? (float)d0[k] : 0.0f;
    r.d1[k] = ok ? (float)d1[k] : 0.0f;
    r.u0[k] = ok ? (float)f.u0[k] : 0.0f;
    r.u1[k] = ok ? (float)f.u1[k] : 0.0f;
  }
  auto dot = [](const double* x, const double* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
  r.G[0] = ok ? (float)dot(d0, d0) : 0.0f;
  r.G[1] = ok ? (float)dot(d1, d1) : 0.0f;
  r.G[2] = ok ? (float)dot(d2, d2) : 0.0f;
  r.G[3] = ok ? (float)dot(d0, d1) : 0.0f;
  r.G[4] = ok ? (float)dot(d1, d2) : 0.0f;
  r.G[5] = ok ? (float)dot(d2, d0) : 0.0f;
  r.thr = ok ? (float)(tau * tau * N2 / L2) : -1.0f;
  r.kap = ok ? (float)(tau_rel * tau_rel * N2) : -1.0f;
  for (int k = 0; k < 3; ++k) r.c2[k] = ok ? (float)(f.g[k] - f.u0[k] - f.u1[k]) : 0.0f;
  out[m] = r;
}

__global__ __launch_bounds__(256) void edges2d_kernel(const double* verts, int64_t nv, const int64_t* off,
                                                      int64_t ncont, const MeshInfo* info, Edge2D* edges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  int64_t start = 0, end = nv;
  if (off) {
    int64_t lo = 0, hi = ncont;  // last contour c with off[c] <= i
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) / 2;
      if (off[mid] <= i) lo = mid; else hi = mid;
    }
    start = off[lo];
    end = off[lo + 1];
  }
  const int64_t j = (i + 1 < end) ? i + 1 : start;
  const MeshInfo mi = info[0];
  Edge2D e;
  e.a[0] = verts[2 * i] - mi.t[0];
  e.a[1] = verts[2 * i + 1] - mi.t[1];
  e.b[0] = verts[2 * j] - mi.t[0];
  e.b[1] = verts[2 * j + 1] - mi.t[1];
  edges[i] = e;
}

__global__ __launch_bounds__(256) void validate_kernel(const int32_t* tris, int64_t nf, int64_t nv,
                                                       unsigned long long* counts) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nf) return;
  const int32_t a = tris[3 * m], b = tris[3 * m + 1], c = tris[3 * m + 2];
  const int bad = (a < 0 || a >= nv) + (b < 0 || b >= nv) + (c < 0 || c >= nv);
  if (bad) atomicAdd(&counts[0], (unsigned long long)bad);
  if (a == b || b == c || c == a) atomicAdd(&counts[1], 1ull);
}

__global__ __launch_bounds__(256) void zero_u32_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_mesh_info(const void* verts, int vdtype, const int64_t* d_vert_off, int64_t n_meshes,
                            MeshInfo* info, hipStream_t s) {
  mesh_info_kernel<<<(unsigned)n_meshes, kInfoBlock, 0, s>>>(verts, vdtype, 3, 0, d_vert_off, info);
  return hipGetLastError();
}

hipError_t launch_mesh_info_single(const void* verts, int vdtype, int dim, int64_t nv, MeshInfo* info,
                                   hipStream_t s) {
  mesh_info_kernel<<<1, kInfoBlock, 0, s>>>(verts, vdtype, dim, nv, nullptr, info);
  return hipGetLastError();
}

hipError_t launch_face64(const void* verts, int vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                         MeshInfo* info, double tau, Face64* out, hipStream_t s, const int32_t* order,
                         const uint8_t* meta) {
  if (nf <= 0) return hipSuccess;
  face64_kernel<<<grid_for(nf), 256, 0, s>>>(verts, vdtype, nv, tris, nf, info, tau, out, order, meta);
  return hipGetLastError();
}

hipError_t launch_poly_records(const void* verts, int vdtype, int64_t nv, const int64_t* face_off,
                               const int32_t* face_verts, int64_t nf, MeshInfo* info, double tau, FaceP64* f64,
                               VtxP64* v64, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  poly64_kernel<<<grid_for(nf), 256, 0, s>>>(verts, vdtype, nv, face_off, face_verts, nf, info, tau, f64, v64);
  return hipGetLastError();
}

hipError_t launch_poly_records32(const FaceP64* f64, const VtxP64* v64, int64_t nf, double tau_rel, FaceP32* f32,
                                 VtxP32* v32, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  poly32_kernel<<<grid_for(nf), 256, 0, s>>>(f64, v64, nf, tau_rel, f32, v32);
  return hipGetLastError();
}

hipError_t launch_face32(const Face64* f64, int64_t nf, double tau, double tau_rel, Face32* out, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  face32_kernel<<<grid_for(nf), 256, 0, s>>>(f64, nf, tau, tau_rel, out);
  return hipGetLastError();
}

hipError_t launch_face32b(const Face64* f64, int64_t nf, double tau, double tau_rel, Face32B* out, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  face32b_kernel<<<grid_for(nf), 256, 0, s>>>(f64, nf, tau, tau_rel, out);
  return hipGetLastError();
}

hipError_t launch_fill_face_mesh(const int64_t* d_tri_off, int64_t n_meshes, int64_t nf_total, int32_t* face_mesh,
                                 hipStream_t s) {
  if (nf_total <= 0) return hipSuccess;
  face_mesh_kernel<<<grid_for(nf_total), 256, 0, s>>>(d_tri_off, n_meshes, nf_total, face_mesh);
  return hipGetLastError();
}

hipError_t launch_face64_batch(const void* verts, int vdtype, const int32_t* tris, const int64_t* d_vert_off,
                               const int64_t* d_tri_off, const int32_t* d_face_mesh, int64_t nf_total,
                               MeshInfo* info, double tau, Face64* out, hipStream_t s,
                               const int32_t* order, const uint8_t* meta) {
  if (nf_total <= 0) return hipSuccess;
  face64_batch_kernel<<<grid_for(nf_total), 256, 0, s>>>(verts, vdtype, tris, d_vert_off, d_tri_off, d_face_mesh,
                                                         nf_total, info, tau, out, order, meta);
  return hipGetLastError();
}

hipError_t launch_edges2d(const double* verts, int64_t nv, const int64_t* d_off, int64_t ncont, MeshInfo* info,
                          Edge2D* edges, hipStream_t s) {
  mesh_info_kernel<<<1, kInfoBlock, 0, s>>>(verts, PFT_F64, 2, nv, nullptr, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nv <= 0) return e;
  edges2d_kernel<<<grid_for(nv), 256, 0, s>>>(verts, nv, d_off, ncont, info, edges);
  return hipGetLastError();
}

hipError_t launch_validate(const int32_t* tris, int64_t nf, int64_t nv, unsigned long long* counts, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  validate_kernel<<<grid_for(nf), 256, 0, s>>>(tris, nf, nv, counts);
  return hipGetLastError();
}

hipError_t launch_clamp_perm(const uint32_t* in, int64_t n, uint32_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  clamp_perm_kernel<<<grid_for(n), 256, 0, s>>>(in, n, out);
  return hipGetLastError();
}

hipError_t launch_iota_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  iota_u32_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  zero_u32_kernel<<<grid_for(n), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

}  // namespace pft
