// Internal declarations shared by the libpft HIP sources: per-face / per-edge
// records written by the prologue kernels, tuning constants, and the launcher
// functions that the C ABI layer calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pft.h"

namespace pft {

// ---------------------------------------------------------------------------
// Tuning constants
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;        // threads per block for the Q-parallel kernels
#ifndef PFT_TILEF
#define PFT_TILEF 64
#endif
constexpr int kTileF = PFT_TILEF;  // faces staged in LDS per tile (binary64 forward and grad_Q)
#ifndef PFT_TILEF32
#define PFT_TILEF32 64
#endif
// faces per LDS tile of an FP32C forward wavefront (also the binary64 re-anchoring interval of its carried
// phases); 6 KiB of records plus 2.25 KiB of Q low parts per wavefront, so the LDS holds more wavefronts
// than the 5 per SIMD the registers allow
constexpr int kTileF32 = PFT_TILEF32;
constexpr int kTileFB = 8;         // faces per block in the binary64 adjoint
#ifndef PFT_QPT
#define PFT_QPT 2
#endif
#ifndef PFT_QPT_LARGE
#define PFT_QPT_LARGE 3
#endif
#ifndef PFT_FWD_LARGE_NQ
#define PFT_FWD_LARGE_NQ (1 << 20)
#endif
// Q per thread in the FP32C forward: kQPT (5 waves per SIMD) below kFwdLargeNq Q, where the face splits
// and the tail matter more, kQPTLarge (4 waves per SIMD; fewer face-record reads and per-face branches
// per pair) from kFwdLargeNq Q on. Each Q's arithmetic is the same in both, so is its value.
constexpr int kQPT = PFT_QPT;
constexpr int kQPTLarge = PFT_QPT_LARGE;
constexpr int64_t kFwdLargeNq = PFT_FWD_LARGE_NQ;
inline int fwd_qpt(int64_t nq) { return nq >= kFwdLargeNq ? kQPTLarge : kQPT; }
__host__ __device__ constexpr int fwd_waves(int qpt) { return qpt >= 3 ? 4 : 5; }  // waves per SIMD
#ifndef PFT_FWD_BLOCK_WAVES
#define PFT_FWD_BLOCK_WAVES 4
#endif
constexpr int kFwdSplitWaves = PFT_FWD_BLOCK_WAVES;  // wavefronts of an FP32C forward block, each on its own faces
constexpr int kFwdBlock = 64 * kFwdSplitWaves;       // threads of an FP32C forward block
__host__ __device__ constexpr int fwd_qtile(int qpt) { return 64 * qpt; }  // Q of an FP32C forward block
constexpr int kXcds = 8;                             // accelerator dies (each with its own L2) of the target
#ifndef PFT_BATCH_FWD_WAVES
#define PFT_BATCH_FWD_WAVES 4
#endif
// the same for the batched FP32C forward at 3 Q per thread (at 1 and 2 Q, one wavefront more)
constexpr int kBatchFwdWaves = PFT_BATCH_FWD_WAVES;
#ifndef PFT_QPT_BATCH
#define PFT_QPT_BATCH 2
#endif
constexpr int kQPTBatch = PFT_QPT_BATCH;  // Q per thread in the batched FP32C forward
#ifndef PFT_QPTB
#define PFT_QPTB 3
#endif
constexpr int kQPTB = PFT_QPTB;    // Q per thread per pass in the adjoint
#ifndef PFT_TILEFB32
#define PFT_TILEFB32 8
#endif
constexpr int kTileFB32 = PFT_TILEFB32;  // faces per block in the FP32C adjoint
#ifndef PFT_QPT_DQ
#define PFT_QPT_DQ 2
#endif
constexpr int kQPTDQ = PFT_QPT_DQ;  // Q per thread in the FP32C grad_Q kernel
constexpr int kTileE = 64;         // 2D edges staged in LDS per tile

// Series thresholds (dimensionless). A (Q, face) pair uses the face's simplex
// series instead of the edge sum when |Q_perp| L_face < tau (absolute test) or
// |Q_perp| < tau_rel |Q| (relative test, guards the rounding of Q x N in FP32).
constexpr double kTauF64 = 0.05;     // forward and adjoint, FP64 mode
constexpr double kTauF32 = 0.1;      // forward, FP32C mode (series in FP64)
constexpr double kTauRel32 = 0.02;   // forward, FP32C mode, relative test
constexpr double kTauB32 = 1.5;      // (record field of the FP32C adjoint; empty-face flag)
// The adjoint evaluates each face's barycentric moments by their series (binary64)
// or by a polynomial of exp(ix) fitted on [-3, 3] (binary32, moment_poly.h) when the
// largest centred vertex phase |Q.(v_k - g)| is at most this, by the
// differentiated edge sums otherwise (there |Q_perp| L > 4.5).
#ifndef PFT_SERIES_MAX_PHASE
#define PFT_SERIES_MAX_PHASE 3.0
#endif
constexpr double kSeriesMaxPhase = PFT_SERIES_MAX_PHASE;
constexpr double kTauRelB32 = 0.05;  // adjoint, FP32C mode, relative test
// Whole-mesh series (fan of tetrahedra from the vertex mean) when |Q| R < tau0.
constexpr double kTau0F64 = 0.01;
constexpr double kTau0F32 = 0.2;
// grad_Q F: the surface form cancels as (|Q| R)^-2 at small |Q| R; below this
// the tetrahedron fan (binary64 series) is used in both forms.
constexpr double kTauDQ = 0.5;
// Closed regions in FP32C: the surface sum of a small region cancels by a factor of about 45 / (|Q| R_j)
// for a tetrahedron (R_j the region's own radius), so below |Q| R_j = 2 its binary64 tetrahedron fan about
// the region's centre is used (the forward and grad_Q alike); for regions of the size of the whole set
// this covers a negligible share of a Q grid.
constexpr double kTauRegion32 = 2.0;
// 2D fan series when |Q| R < tau0.
constexpr double kTau02D = 0.01;

// ---------------------------------------------------------------------------
// Records
// ---------------------------------------------------------------------------
// Per-mesh quantities (device): vertex mean t, radius R = max |v - t|, and
// rho, the largest distance from a face's centroid (vertex mean) to one of its
// vertices over the mesh's faces (the face prologue raises it from 0; the
// FP32C phase-range check reads it).
struct MeshInfo {
  double t[3];
  double R;
  double rho;
  double pad;
};

// FP32C phase range. The binary32 form takes every phase it evaluates relative
// to a face origin: the half-vertex phases Q.u/2 (u = vertex - face centroid),
// the edge half-differences Q.(b - a)/2 and the midpoint phases, all in turns.
// With |Q| rho <= kPhaseMax32 radians each of them is at most
// kPhaseMax32 / (2 pi) + 1/2 < 21 turns, inside the hardware sine's domain and
// rounded to within 2^-20 turn (6e-6 rad) in binary32. The FP32C finish steps
// write NaN (F, |F|^2, the loss term, the cotangent records) for every Q beyond
// it; the binary64 form has no such bound.
constexpr double kPhaseMax32 = PFT_FP32C_PHASE_MAX;
__host__ __device__ __forceinline__ bool fp32c_phase_out_of_range(double qabs, const MeshInfo& mi) {
  return qabs * mi.rho > kPhaseMax32;
}
__host__ __device__ __forceinline__ double quiet_nan() { return __builtin_nan(""); }

// FP64 face record: geometry relative to the mesh centre t.
struct alignas(16) Face64 {
  double g[3];    // centroid
  double u0[3];   // a - g
  double u1[3];   // b - g          (c - g = -u0 - u1)
  double N[3];    // (b - a) x (c - a) = 2 A n
  double thr;     // series when |Q x N|^2 < thr  (tau^2 |N|^2 / L^2; -1 for an empty face)
  double pad[3];
};
static_assert(sizeof(Face64) == 128, "Face64 layout");

// FP32C forward face record (staged in LDS). The in-plane geometry is held in
// an orthonormal basis e1, e2 of the face plane (e1 along b - a, e2 = n x e1,
// with a, b, c the vertices in the record's traversal order and n that order's
// unit normal). With the half components sigma_j = Q . e_j / 2 of the in-plane
// part of Q, and the edge coefficients al_l = (e1 . d_l)/(2 pi), be_l = -(e2 . d_l)/(2 pi):
//   eta_l = Q . d_l / (4 pi) = sigma1 al_l - sigma2 be_l      (edge half-phase, turns)
//   w'_l = sigma2 al_l + sigma1 be_l = (P . d_l) / (4 pi |N|)  (P = Q x N; the edge weight)
//   |P|^2 / (4 |N|^2) = sigma1^2 + sigma2^2,   tau_rel (Q . n) / 2 = Q . N'  (N' = tau_rel N / (2 |N|)),
// so tau_rel times the face term (Q.N)/|P|^2 sum_l (P.d_l) E_l equals (Q.N')/(sigma1^2 + sigma2^2)
// sum_l w'_l E_l: the kernels sum that and divide by tau_rel once per partial sum. The factor tau_rel
// (the relative series threshold) lets one fused multiply-add form the series test
// |P'|^2 < (Q.N')^2 + thr, i.e. |Q_perp| < tau_rel |Q.n| or |Q_perp| L < tau.
// In an edge-sharing order the traversal may be the reverse of the outward
// (counter-clockwise) one, so that the edge shared with the next face is edge
// 1: the edge sum is the same for both traversals (each edge's P . d and
// sinc are unchanged when both the normal and the edge flip), and N' below
// stays the outward normal, so the face term is unchanged.
struct alignas(16) Face32 {
  double gt[3];   // centroid / (2 pi), binary64: face origin phase in turns is Q . gt
  float N[3];     // N' = tau_rel N / (2 |N|), N the outward (b - a) x (c - a) of the counter-clockwise traversal
  float E1[3];    // e1 / 2
  float E2[3];    // e2 / 2
  float al[3];    // (e1 . d_l) / (2 pi), l = 0, 1, 2 (d_0 = b - a, d_1 = c - b, d_2 = a - c)
  float be[3];    // -(e2 . d_l) / (2 pi)
  float thr;      // tau^2 / (4 L^2) (1 for an empty face: its series term is Q.N = 0 times a sum)
  float nN;       // 2 |N|: the series branch takes tau_rel Q . N as nN (Q . N'), scaled like the edge terms
  uint32_t flags; // kFaceLinked: edge 0 is the previous record's edge 1 (edge-sharing order)
};
static_assert(sizeof(Face32) == 96, "Face32 layout");
constexpr uint32_t kFaceLinked = 1u;
// Edge-sharing order metadata (pft_strip_order, one byte per position): the face's
// vertex list rotated by (meta & 3), edge 0 shared with the previous position's
// edge 1 if (meta & kMetaLink), and the traversal reversed (b, a, c) if (meta & kMetaReflect).
constexpr unsigned kMetaLink = 4u;
constexpr unsigned kMetaReflect = 8u;

// FP32C adjoint face record.
struct alignas(16) Face32B {
  double gt[3];   // centroid / (2 pi)
  float N[3];
  float d0[3];    // b - a
  float d1[3];    // c - b
  float u0[3];    // a - g: vertex phase delta_0 = Q . u0
  float u1[3];    // b - g
  float G[6];     // d0.d0, d1.d1, d2.d2, d0.d1, d1.d2, d2.d0
  float thr;      // tau_b^2 |N|^2 / L^2 (-1 for an empty face, whose record is otherwise all zero)
  float kap;      // tau_relb^2 |N|^2
  float c2[3];    // c - t (vertex c relative to the mesh centre; used by grad_Q F)
};
static_assert(sizeof(Face32B) == 128, "Face32B layout");

// One Q of the FP32C adjoint's reordered list (qorder.hip): the Q vector and the
// centred cotangent g(Q) exp(-iQ.t) of the mesh that owns it.
struct alignas(16) QRec32 {
  double q[3];
  float hr, hi;
};
static_assert(sizeof(QRec32) == 32, "QRec32 layout");
// The same for the binary64 adjoint (cotangent in binary64).
struct alignas(16) QRec64 {
  double q[3];
  double pad;
  double hr, hi;
};
static_assert(sizeof(QRec64) == 48, "QRec64 layout");


// 2D edge record (FP64), relative to the polygon's vertex mean.
struct alignas(16) Edge2D {
  double a[2];    // start vertex
  double b[2];    // end vertex
};

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files). All enqueue on `s` and return the
// HIP status of the launch.
// ---------------------------------------------------------------------------
// prologue.hip
hipError_t launch_mesh_info(const void* verts, int vdtype, const int64_t* d_vert_off, int64_t n_meshes,
                            MeshInfo* info, hipStream_t s);
hipError_t launch_mesh_info_single(const void* verts, int vdtype, int dim, int64_t nv, MeshInfo* info,
                                   hipStream_t s);
// With order / meta (device, [nf]; NULL: the list order), record m is face order[m] with its
// vertex list rotated by meta[m] & 3, and pad[2] holds the link meta[m] >> 2 (0, 1 or 2).
hipError_t launch_face64(const void* verts, int vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                         MeshInfo* info, double tau, Face64* out, hipStream_t s,
                         const int32_t* order = nullptr, const uint8_t* meta = nullptr);
hipError_t launch_face32(const Face64* f64, int64_t nf, double tau, double tau_rel, Face32* out, hipStream_t s);
hipError_t launch_face32b(const Face64* f64, int64_t nf, double tau, double tau_rel, Face32B* out, hipStream_t s);
hipError_t launch_face64_batch(const void* verts, int vdtype, const int32_t* tris, const int64_t* d_vert_off,
                               const int64_t* d_tri_off, const int32_t* d_face_mesh, int64_t nf_total,
                               MeshInfo* info, double tau, Face64* out, hipStream_t s,
                               const int32_t* order = nullptr, const uint8_t* meta = nullptr);
hipError_t launch_fill_face_mesh(const int64_t* d_tri_off, int64_t n_meshes, int64_t nf_total, int32_t* face_mesh,
                                 hipStream_t s);
hipError_t launch_edges2d(const double* verts, int64_t nv, const int64_t* d_off, int64_t ncont, MeshInfo* info,
                          Edge2D* edges, hipStream_t s);
hipError_t launch_validate(const int32_t* tris, int64_t nf, int64_t nv, unsigned long long* counts, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s);
hipError_t launch_iota_u32(uint32_t* p, int64_t n, hipStream_t s);
// out[i] = in[i] if in[i] < n, else i (a caller's Q order made safe to index with).
hipError_t launch_clamp_perm(const uint32_t* in, int64_t n, uint32_t* out, hipStream_t s);

// ---------------------------------------------------------------------------
// Planar polygon faces (fwdpoly.hip): a face header plus one record per vertex
// (the edge from vertex k to k+1, wrapping, belongs to vertex k). Faces are
// processed in tiles of consecutive faces holding at most kTileV vertices.
// ---------------------------------------------------------------------------
constexpr int kTileV = 256;       // vertex records per polygon tile (and the largest face)
constexpr int kTileFP = 64;       // faces per polygon tile
#ifndef PFT_QPT_POLY
#define PFT_QPT_POLY 3
#endif
constexpr int kQPTPoly = PFT_QPT_POLY;  // Q per thread in the FP32C polygon forward

struct alignas(16) FaceP64 {      // relative to the mesh centre t
  double g[3];                    // vertex mean of the polygon
  double N[3];                    // area vector sum_k u_k x u_{k+1} = 2 A n
  double thr;                     // series when |Q x N|^2 < thr (tau^2 |N|^2 / L^2; -1 for an empty face)
  double invN;                    // 1 / |N| (0 for an empty face)
  int32_t v0;                     // first vertex record
  int32_t nv;                     // vertex count
  int32_t pad[2];
};
static_assert(sizeof(FaceP64) == 80, "FaceP64 layout");

struct alignas(16) VtxP64 {
  double u[3];                    // r_k - g
  double pad;
};
static_assert(sizeof(VtxP64) == 32, "VtxP64 layout");

struct alignas(16) FaceP32 {      // FP32C: in-plane basis as in Face32
  double gt[3];                   // g / (2 pi): face origin phase in turns is Q . gt
  float N[3];                     // 2 A n
  float E1[3];                    // |N| e1 (e1 along the first non-degenerate edge)
  float E2[3];                    // |N| e2, e2 = n x e1
  float thr;                      // tau^2 |N|^2 / L^2 (-1 for an empty face)
  float kap;                      // tau_rel^2 |N|^2
  float invN;                     // 1 / |N|
  int32_t v0;                     // first vertex record
  int32_t nv;                     // vertex count
  int32_t pad[2];
};
static_assert(sizeof(FaceP32) == 96, "FaceP32 layout");

struct VtxP32 {
  float ga, de;                   // half-vertex phase psi_k = Q.u_k / 2 in turns = s1 ga + s2 de
  float al, be;                   // edge k -> k+1: P . d_k / (2 pi) = s2 al + s1 be
  float x, y;                     // in-plane coordinates e1 . u_k, e2 . u_k (fan areas of the series)
};
static_assert(sizeof(VtxP32) == 24, "VtxP32 layout");

struct PolyTile {                 // faces [f0, f1) with vertex records [v0, v1)
  int32_t f0, f1, v0, v1;
};

struct PolyArgs {
  const FaceP64* f64;
  const VtxP64* v64;
  const FaceP32* f32;
  const VtxP32* v32;
  const PolyTile* tiles;
  int64_t ntiles;
  int64_t tiles_per_split;
};

// prologue.hip: records of polygon faces (face_off: device CSR offsets into face_verts)
hipError_t launch_poly_records(const void* verts, int vdtype, int64_t nv, const int64_t* face_off,
                               const int32_t* face_verts, int64_t nf, MeshInfo* info, double tau, FaceP64* f64,
                               VtxP64* v64, hipStream_t s);
// (the binary64 records must have been built with the FP32C threshold tau)
hipError_t launch_poly_records32(const FaceP64* f64, const VtxP64* v64, int64_t nf, double tau_rel, FaceP32* f32,
                                 VtxP32* v32, hipStream_t s);

// fwd3d.hip
struct FwdArgs {
  const Face64* f64;
  const Face32* f32;
  const MeshInfo* info;
  int64_t nf;
  const void* q;
  int qdtype;
  int64_t nq;
  int splits;
  int64_t faces_per_split;
  const uint32_t* perm;  // visiting order of Q (NULL: the caller's order); partials follow it
  const int64_t* split_face;  // [splits + 1] face range of each split (NULL: faces_per_split each)
  double2* partial;   // [splits][nq] when splits > 1
  void* out;
  void* intensity;
  double tau0;
  int share_edges = 0;  // FP32C: records are in edge-sharing order (Face32::link), reuse the shared edge's term
  int qpt = kQPT;       // FP32C: Q per thread (kQPT or kQPTLarge, fwd_qpt), set with the splits
  // [splits] (x, y, z) the centre of the split's region relative to t, w its radius: the small-|Q| test of
  // a split uses that radius and its tetrahedron fan that apex (NULL: the mesh's R, apex t)
  const double4* split_geo = nullptr;
};
hipError_t launch_fwd3d_fp64(const FwdArgs& a, hipStream_t s);
hipError_t launch_fwd3d_fp32c(const FwdArgs& a, hipStream_t s);
hipError_t launch_fwd3d_finish(const FwdArgs& a, int out_c128, hipStream_t s);

// Closed regions of constant density (dq3d.hip): region j owns the splits
// region_split[j] .. region_split[j+1] of the face-split partials.
struct RegionArgs {
  const int32_t* region_split;  // [nreg + 1] (device)
  int nreg;
  const double* rho;            // [nreg] densities (device)
  void* out_regions;            // [nreg][nq] per-region F (NULL: not written)
  const void* grad_out;         // [nq] cotangent for dL/drho and dL/dQ (NULL: forward only)
  double* rho_part;             // [blocks][nreg] per-block sums of Re(conj(g) F_j) (NULL: not formed)
  const double* region_R;       // [nreg] each region's own radius for the small-|Q| test (NULL: the mesh's R)
};
// F = sum_j rho_j F_j (and F_j, |F|^2, dL/drho partials) from forward partials.
hipError_t launch_regions_finish(const FwdArgs& a, const RegionArgs& r, int out_c128, hipStream_t s);
// dL/drho_j = sum over blocks of rho_part[.][j], fixed order.
hipError_t launch_rho_reduce(const double* rho_part, int64_t nblocks, int nreg, double* grad_rho, hipStream_t s);
int64_t finish_blocks(int64_t nq);
// rho of the region owning each face (region offsets on the device).
// Radius of each region about its own centre (the mean of its face centroids), from the binary64
// records: region_R[j]; and split_geo[s] = (centre relative to t, radius) of the region owning split s.
hipError_t launch_region_radii(const Face64* f64, const int64_t* d_region_off, int nreg,
                               const int32_t* d_region_split, double* region_R, double4* region_geo,
                               double4* split_geo, hipStream_t s);
hipError_t launch_face_weights(const int64_t* d_region_off, int nreg, const double* rho, int64_t nf, double* w,
                               hipStream_t s);

// loss.hip: L = sum_Q w (|F|^2 - I)^2 from the forward's partials (a.out and a.intensity
// optional), the adjoint's Q records with the cotangent 4 w (|F|^2 - I) F_c (rec for FP32C,
// rec64 for FP64) in the visiting order, per-block loss sums and their fixed-order total.
int64_t loss_blocks(int64_t nq);
hipError_t launch_loss_finish(const FwdArgs& a, const double* weight, const double* target, int c128, QRec32* rec,
                              QRec64* rec64, double* loss_part /*[loss_blocks(nq)]*/, double* loss, hipStream_t s);

// grad_Q F (dq3d.hip): per Q, the face sums A = sum_m (Q.N_m) e^{iQ.g_m} (sum over corners of
// (v_k - t) times the normalised barycentric moments) and B = sum_m (Q.N_m) e^{iQ.g_m} J_m/2A,
// or, for |Q| R < tau, the tetrahedron-fan grad F_c and F_c directly.
struct DqArgs {
  const MeshInfo* info;
  const Face64* f64;
  const double* gram;       // FP64: [nf][8] edge Gram matrices
  const Face32B* f32;       // FP32C records
  int64_t nf;
  const void* q;
  int qdtype;
  int64_t nq;
  const uint32_t* perm;
  int splits;
  int64_t faces_per_split;
  const int64_t* split_face;
  double2* partial;         // [splits][4][nq]: A_x, A_y, A_z, B
  double tau;
  const double4* split_geo = nullptr;  // as FwdArgs::split_geo
};
hipError_t launch_dq3d_fp64(const DqArgs& a, hipStream_t s);
hipError_t launch_dq3d_fp32c(const DqArgs& a, hipStream_t s);
// dL/dQ = Re(conj(g) sum_j rho_j grad F_j) into grad_q ([nq][3] of gq_dtype, may be NULL), and
// the dL/drho partials when r.rho_part is set.
hipError_t launch_dq_finish(const DqArgs& a, const RegionArgs& r, int go_c128, void* grad_q, int gq_dtype,
                            hipStream_t s);
// fwdpoly.hip: the forward over polygon faces (FwdArgs's face fields unused; splits over tiles)
hipError_t launch_fwdpoly_fp64(const FwdArgs& a, const PolyArgs& p, hipStream_t s);
hipError_t launch_fwdpoly_fp32c(const FwdArgs& a, const PolyArgs& p, hipStream_t s);

// bwd3d.hip
struct BwdArgs {
  const MeshInfo* info;  // mesh centre t: the cotangent is taken relative to the centred mesh
  const Face64* f64;
  const Face32B* f32;
  int64_t nf;
  const void* q;
  int qdtype;
  int64_t nq;
  const void* grad_out;
  const QRec32* rec;    // FP32C: reordered Q with their centred cotangents (launch_qrec32_gather)
  const QRec64* rec64;  // FP64: the same in binary64 (launch_qrec64_gather)
  int qsplits;
  int64_t q_per_split;
  double* partial;    // [qsplits][nf][3]
};
hipError_t launch_gram64(const Face64* f64, int64_t nf, double* gram /*[nf][8]*/, hipStream_t s);
hipError_t launch_bwd3d_fp64(const BwdArgs& a, const double* gram, hipStream_t s);
hipError_t launch_bwd3d_fp32c(const BwdArgs& a, hipStream_t s);

// qorder.hip: a permutation of the Q list (by mesh, then by the Morton code of
// Q) that groups nearby Q into wavefronts; each mesh's Q keep their index range
// (d_q_off: CSR offsets of Q per mesh, or NULL for one mesh). perm[i] is the
// caller's index of the i-th visited Q.
struct QOrderScratch {   // device temporaries of launch_qorder
  double* box_partial;   // [256 * 6]
  double* box;           // [6]
  uint64_t* keys;        // [nq]
  uint64_t* keys_sorted; // [nq]
  uint32_t* vals;        // [nq]
  uint32_t* perm;        // [nq] result
  void* sort_temp;       // [sort_bytes]
  size_t sort_bytes;
};
hipError_t qorder_sort_bytes(int64_t nq, int64_t n_meshes, size_t* bytes);
hipError_t launch_qorder(const void* q, int qdtype, int64_t nq, const int64_t* d_q_off, int64_t n_meshes,
                         const QOrderScratch& w, hipStream_t s);
// rec[i] = Q[perm[i]] with its centred cotangent g exp(-iQ.t), t the centre of the owning mesh.
hipError_t launch_qrec32_gather(const void* q, int qdtype, const void* grad_out, int64_t nq, const uint32_t* perm,
                                const MeshInfo* info, const int64_t* d_q_off, int64_t n_meshes, QRec32* rec,
                                hipStream_t s);
// The same with a binary64 cotangent (grad_out complex128).
hipError_t launch_qrec64_gather(const void* q, int qdtype, const void* grad_out, int64_t nq, const uint32_t* perm,
                                const MeshInfo* info, const int64_t* d_q_off, int64_t n_meshes, QRec64* rec,
                                hipStream_t s);
// Sum the per-split adjoint weights, form per-corner vectors N_m R_{m,k} and
// gather them per vertex through the sorted incidence list.
hipError_t launch_bwd_face_contrib(const double* partial, int qsplits, const Face64* f64, const double* face_w, int64_t nf,
                                   double* contrib /*[nf*3][3]*/, hipStream_t s);
hipError_t launch_incidence_keys(const int32_t* tris, int64_t nf, const int64_t* d_vert_off,
                                 const int32_t* d_face_mesh, int64_t nv_total, uint32_t* keys, uint32_t* vals,
                                 hipStream_t s);
hipError_t sort_incidence(uint32_t* keys_in, uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out, int64_t n,
                          int64_t nv_total, void* temp, size_t* temp_bytes, hipStream_t s);
hipError_t launch_gather_vertices(const uint32_t* keys_sorted, const uint32_t* vals_sorted, int64_t nslots,
                                  const double* contrib, int64_t nv, void* grad, int vdtype, hipStream_t s);

// fwd2d.hip
hipError_t launch_fwd2d(const Edge2D* edges, int64_t ne, const MeshInfo* info, double area_hint, const double* q,
                        int64_t nq, double tau0, double* out, hipStream_t s);

// batch.hip
struct BatchItemFwd {   // one (mesh, Q-tile, face-chunk) work item
  int32_t mesh;
  int32_t chunk;        // face-chunk index within the mesh
  int64_t q0;           // first global Q index of the tile
  int32_t nq;           // Q in the tile (<= kBlock for FP64, <= 64 * (Q per thread) for FP32C)
  int32_t pad;
  int64_t f0;           // first global face index of the chunk
  int64_t nf;           // faces in the chunk
  int64_t part;         // partial slot base (in units of Q): partial[part + Q offset in the tile]
};
// A run of equal-size forward work items of one mesh: item k of the group is the (k / ntq)-th of its face
// chunks and the (k % ntq)-th of its Q-tiles. The host orders the groups by decreasing item size and
// numbers the items group after group (`first`); a puller finds an item's group by binary search, so the
// item list itself is never stored.
struct BatchGroupFwd {
  int64_t first;        // index of the group's first item in the global work order
  int64_t f_base;       // first global face of its first chunk
  int64_t q_base;       // first global Q of its first Q-tile
  int64_t part_base;    // partial slot of its first item
  int64_t part_stride;  // partial slots per face chunk (the mesh's Q count)
  int32_t mesh;
  int32_t ntq;          // Q-tiles per chunk in the group
  int32_t cf;           // faces between consecutive chunks
  int32_t qtile;        // Q between consecutive Q-tiles
  int32_t nf;           // faces of each item
  int32_t nq;           // Q of each item
};
struct BatchItemBwd {   // one (mesh, face-tile, Q-chunk) work item
  int32_t mesh;
  int32_t qchunk;
  int64_t f0;           // first global face index of the tile
  int32_t nf;           // faces in the tile (<= kTileFB for FP64, <= kTileFB32 for FP32C)
  int32_t pad;
  int64_t q0;           // first global Q index of the chunk
  int64_t nq;           // Q in the chunk
  int64_t part;         // partial slot base (in units of face corners): partial[(part + j) * 3 + k]
};
int batch_fwd_blocks_per_cu(int mode, bool share = false, int qpt = 1);
int batch_bwd_blocks_per_cu(int mode);
hipError_t launch_batch_fwd(int mode, const BatchGroupFwd* groups, int n_groups, int64_t n_items, uint32_t* counter,
                            const Face64* f64, const Face32* f32, const void* q, int qdtype, const uint32_t* perm,
                            double2* partial, const MeshInfo* info, double tau0, int grid, hipStream_t s,
                            bool share = false, int qpt = 1);
hipError_t launch_batch_fwd_finish(const double2* partial, const int64_t* d_q_off, int64_t n_meshes,
                                   const int64_t* d_q_part, const int32_t* d_q_chunks, const MeshInfo* info,
                                   const void* q, int qdtype, const uint32_t* perm, int64_t nq_total, double tau0,
                                   int out_c128, void* out, void* intensity, hipStream_t s);
hipError_t launch_batch_bwd(int mode, const BatchItemBwd* items, int64_t n_items, uint32_t* counter,
                            const Face64* f64, const double* gram, const Face32B* f32b, const QRec32* rec,
                            const QRec64* rec64, double* partial, int grid, hipStream_t s);
hipError_t launch_batch_bwd_reduce(const double* partial, const int64_t* d_face_base, const int32_t* d_face_nchunks,
                                   const int64_t* d_tri_off, const int32_t* d_face_mesh, const Face64* f64,
                                   int64_t nf_total, double* contrib, hipStream_t s);

// orient.hip
hipError_t launch_qdirs(const double* qabs, int64_t nqa, const double* dirs, int64_t ndir, double* Q, hipStream_t s);
hipError_t launch_dir_sum(const void* I, int idtype, const double* w, int64_t nqa, int64_t ndir, double* out,
                          hipStream_t s);

// Profiling hooks (api.cpp)
void prof_begin(const char* name, hipStream_t s);
void prof_end(const char* name, hipStream_t s);

}  // namespace pft

// ---------------------------------------------------------------------------
// Allocation-free forward (api.cpp, noalloc.hip)
// ---------------------------------------------------------------------------
namespace pft {
// Record `msg` as the calling thread's last error and return `st`.
pft_status set_error(pft_status st, const char* msg);
// pft_forward_3d with its temporaries carved from a fixed device buffer of `cap` bytes that
// scratch_fn supplies after the arguments have been checked (sizes beyond the buffer give EINVAL).
pft_status forward3d_noalloc(pft_status (*scratch_fn)(void**), size_t cap, const void* verts, int vdtype,
                             int64_t nv, const int32_t* tris, int64_t nf, const void* q, int qdtype, int64_t nq,
                             int mode, void* out, void* intensity, void* stream);
}  // namespace pft
