/*
 * pft.h -- C ABI of libpft: direct Fourier transform of polygonal areas and
 * closed triangulated volumes on AMD Instinct MI355X (gfx950).
 *
 * Method: B. B. Maranville, "An implementation of an efficient direct Fourier
 * transform of polygonal areas and volumes". The transform is
 *
 *     F(Q) = integral over the region of exp(+i Q.r) dA   (2D polygon)
 *     F(Q) = integral over the region of exp(+i Q.r) dV   (3D closed mesh)
 *
 * (paper: definition of FT_V and the 2D area integral). The divergence theorem
 * turns it into sums over polygon edges (2D section, eq. line_integral_generic
 * and its midpoint form) and, in 3D, into sums over faces of in-plane edge
 * sums (3D section, eq. single_area_integral and eq. sum_elements_3d). No
 * normalisation: F(0) is the area / volume. Q is in reciprocal units of the
 * vertex coordinates.
 *
 * Common conventions for every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller, contiguous,
 *    row-major, unless the argument is documented as a HOST pointer. The
 *    library never allocates or frees caller memory.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *    legacy default stream) and is asynchronous; outputs are valid once the
 *    stream has reached that point. Temporary device memory comes from a
 *    workspace the library keeps per (device, stream), reused by later calls on
 *    that stream and grown through the stream-ordered allocator when needed;
 *    pft_release_workspace frees it. Calls from several host threads on one
 *    stream are serialised while they enqueue.
 *  - Return value: PFT_OK after synchronous argument validation and a
 *    successful launch, or an error code; the message is available from
 *    pft_last_error() on the calling thread. Device-side faults surface at the
 *    caller's next synchronisation, as for any HIP work.
 *  - Counts of zero are valid: nq == 0 does nothing; nf == 0 (empty mesh)
 *    writes zeros.
 *  - Complex outputs are interleaved (re, im) pairs.
 *  - NaN / Inf in inputs propagate to the affected outputs.
 *  - Triangle indices outside [0, nv) never cause an out-of-bounds access: the
 *    face is treated as empty (contributes zero); pft_validate_mesh counts them
 *    on the device and pft_check_mesh checks a mesh on the host (indices, closed,
 *    consistently oriented). With PFT_VALIDATE=1 in the environment (read at
 *    each call), pft_forward_3d, pft_backward_3d, pft_intensity_loss_3d,
 *    pft_orientation_average and the region entry points run that check on
 *    their mesh first (synchronously; each region on its own), also require a
 *    non-negative enclosed volume, and return PFT_EINVAL if the mesh fails.
 *  - Results do not depend on the order of faces in the list except through
 *    floating-point rounding, and are bitwise reproducible for fixed inputs
 *    and sizes (fixed reduction order, no floating-point atomics).
 */
#ifndef PFT_H
#define PFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PFT_OK = 0,
  PFT_EINVAL = -1,        /* invalid argument (null pointer, negative count, misalignment, bad offsets) */
  PFT_EUNSUPPORTED = -2,  /* unsupported mode / dtype combination */
  PFT_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
  PFT_ENOMEM = -4         /* stream-ordered temporary allocation failed */
} pft_status;

/* Arithmetic of the transform.
 * PFT_FP64  : every step in IEEE binary64; complex128 outputs.
 * PFT_FP32C : "FP32-compensated": the mesh is re-centred on its vertex mean and
 *             each face on its centroid in binary64; the per-(Q, face) edge
 *             arithmetic then runs in binary32 on small local coordinates,
 *             with the face's origin phase Q.g and the mesh phase Q.t taken in
 *             binary64, the near-degenerate branches (Q nearly along a face
 *             normal, |Q| R small) evaluated in binary64, and the sum over
 *             faces accumulated with compensation; complex64 outputs. */
typedef enum { PFT_FP64 = 0, PFT_FP32C = 1 } pft_mode;

/* FP32C phase range (radians). The binary32 form takes every phase it
 * evaluates relative to a face origin, so its accuracy depends on |Q| rho, rho
 * being the largest distance from a face's centroid to one of its vertices
 * (over the mesh; for a batch, over each mesh). For |Q| rho <= PFT_FP32C_PHASE_MAX
 * every binary32 phase is under 21 turns and rounded to within 6e-6 rad; at
 * each Q beyond it the FP32C entry points write NaN instead of a value of
 * unknown accuracy: F and |F|^2 of the forward calls (each region's F and the
 * dL/drho sums of the region calls, dL/dQ of pft_backward_3d_regions), the loss
 * term of pft_intensity_loss_3d (so the loss and every gradient entry are NaN),
 * and that Q's cotangent in the adjoints (every vertex gradient is NaN).
 * PFT_FP64 has no such bound. pft_fp32c_q_limit gives the bound on |Q| for a
 * host mesh; the device check computes rho in binary64 from the centred mesh,
 * so a Q within rounding of the bound may fall on either side. */
#define PFT_FP32C_PHASE_MAX 128.0

/* Real element type of an input array. */
typedef enum { PFT_F32 = 0, PFT_F64 = 1 } pft_dtype;

/*
 * pft_forward_2d -- F(Q) of a polygon with one or more closed contours
 * (2D section: divergence theorem with the field -iQ exp(iQ.r)/Q^2, edge normal
 * eq. line_normal, edge integral eq. line_integral_generic in its midpoint /
 * sinc form). FP64 only.
 *
 *  verts            [nv][2] float64, contour vertices in traversal order.
 *  contour_offsets  HOST int64 [ncontours + 1], non-decreasing, first 0, last nv;
 *                   contour c is verts[offsets[c] .. offsets[c+1]). NULL means a
 *                   single contour of all nv vertices (ncontours is ignored).
 *                   Counter-clockwise contours add, clockwise ones subtract
 *                   (holes). A contour with fewer than 3 vertices encloses no area.
 *  q                [nq][2] float64.
 *  out              [nq] complex128 (interleaved float64 pairs), overwritten.
 * Errors: EINVAL for null pointers with non-zero counts, negative counts,
 * misaligned pointers (8 B), or offsets that are not non-decreasing from 0 to nv.
 */
pft_status pft_forward_2d(const double* verts, int64_t nv, const int64_t* contour_offsets, int64_t ncontours,
                          const double* q, int64_t nq, double* out, void* stream);

/*
 * pft_forward_3d -- F(Q) of the volume enclosed by a closed triangle mesh
 * (3D section: eq. divergence3d split over faces, eq. single_area_integral,
 * eq. sum_elements_3d with the outward in-plane edge normal, edge sums in the
 * midpoint / sinc form).
 *
 *  verts    [nv][3] of vdtype. tris [nf][3] int32, 0-based, each triangle
 *           counter-clockwise seen from outside (outward normal by the
 *           right-hand rule). The mesh must be closed (every edge shared by two
 *           faces with opposite directions); an inward mesh gives -F, an open
 *           mesh gives an origin-dependent value. Zero-area faces contribute 0.
 *  q        [nq][3] of qdtype.
 *  mode     PFT_FP64 : out is [nq] complex128, intensity (optional) [nq] float64.
 *           PFT_FP32C: out is [nq] complex64,  intensity (optional) [nq] float32.
 *  out      overwritten. intensity: NULL or |F(Q)|^2, overwritten.
 * Errors: EINVAL (null pointers with non-zero counts, negative counts,
 * misalignment to the element size), EUNSUPPORTED (unknown mode / dtype).
 */
pft_status pft_forward_3d(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                          const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, void* out, void* intensity,
                          void* stream);

/*
 * pft_strip_order -- an edge-sharing order of a triangle mesh's faces (HOST
 * function, no GPU work): consecutive faces share an edge wherever the greedy
 * chains over the edge adjacency allow. Each face is traversed from a cyclic
 * rotation of its vertex list, reversed where needed, so that its edge 0
 * (v0 -> v1) is the edge it shares with the previous face and its edge 1
 * (v1 -> v2) the edge it shares with the next one; the face term of a triangle
 * is the same for both traversals (3D section: each edge's term keeps its
 * value when the normal and the edge both flip), and the library keeps the
 * outward normal for Q.N. For pft_forward_3d_ordered; the order depends only on
 * the connectivity, so it is computed once per mesh.
 *
 *  tris   [nf][3] int32 (HOST).
 *  order  [nf] int32 (HOST), written: a permutation of 0 .. nf-1.
 *  meta   [nf] uint8 (HOST), written: rotation r (0..2) in bits 0-1, bit 2
 *         set if edge 0 (after the rotation) is edge 1 of the previous face
 *         (after its own rotation and reversal), bit 3 set if the traversal is
 *         reversed: (v_r, v_r+1, v_r+2) becomes (v_r+1, v_r, v_r+2).
 *  Faces with an out-of-range or repeated index are placed without a link.
 * Errors: EINVAL for negative counts or NULL pointers with nf > 0.
 */
pft_status pft_strip_order(const int32_t* tris, int64_t nf, int64_t nv, int32_t* order, uint8_t* meta);

/*
 * pft_q_order -- the order in which the kernels visit a Q list: sorted by the
 * Morton code of Q (nearby Q share wavefronts; below 8192 Q, the list order).
 * Each Q's F does not depend on the order; the adjoint's sums over Q follow it.
 * Computing it once and passing it to pft_forward_3d_ordered and
 * pft_backward_3d_ordered saves the sort in every call on the same Q.
 *  q      [nq][3] of qdtype (DEVICE).
 *  order  [nq] uint32 (DEVICE), written: a permutation of 0 .. nq-1.
 * Errors: EINVAL for NULL pointers with nq > 0, misalignment or nq > 2^32 - 1.
 */
pft_status pft_q_order(const void* q, pft_dtype qdtype, int64_t nq, uint32_t* order, void* stream);

/*
 * pft_forward_3d_ordered -- pft_forward_3d with the faces taken in an
 * edge-sharing order (pft_strip_order, copied to the device) and/or the Q
 * visited in a given order (pft_q_order). The sum over faces is unchanged
 * (eq. sum_elements_3d; only the rounding order differs); in the
 * FP32-compensated form the term sinc(Q.d/2) exp(iQ.m) of an edge shared with
 * the previous face is reused, so a face costs two edge terms instead of three.
 *
 *  Arguments as pft_forward_3d, plus
 *  face_order  NULL (the list order) or [nf] int32 (DEVICE), a permutation
 *              of 0 .. nf-1 (an entry out of range makes that position an
 *              empty face);
 *  face_meta   NULL with face_order, else [nf] uint8 (DEVICE), as written by
 *              pft_strip_order. A wrong link or reversal gives a wrong result,
 *              never an out-of-bounds access.
 *  q_order     NULL (sorted here) or [nq] uint32 (DEVICE), a permutation of
 *              0 .. nq-1 (an entry out of range is replaced by its position).
 * Errors: as pft_forward_3d; EINVAL also for only one of face_order,
 * face_meta given.
 */
pft_status pft_forward_3d_ordered(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                  const int32_t* face_order, const uint8_t* face_meta, const void* q,
                                  pft_dtype qdtype, int64_t nq, pft_mode mode, void* out, void* intensity,
                                  const uint32_t* q_order, void* stream);

/*
 * pft_forward_3d_noalloc -- pft_forward_3d for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the call allocates and frees nothing. Its
 * temporaries (mesh centre, per-face records, per-split partial sums) live in
 * a device array of fixed size, 64 MiB on each GPU the library runs on, held
 * until the process ends. The Q are visited in the list order, the face splits
 * are as many as fit beside the records, and the PFT_VALIDATE check (which
 * synchronises) is not run. The caller still passes inputs and outputs.
 *
 *  Arguments, outputs and results as pft_forward_3d (equal up to the rounding
 *  order of the face sum).
 *  Limits: the records take 240 bytes per face in PFT_FP32C (128 in PFT_FP64)
 *  and each Q at least 16 bytes, within 64 MiB (e.g. 99 460 faces with
 *  2 097 152 Q in PFT_FP32C).
 *  Concurrency: every call on one GPU uses that GPU's one array, so calls that
 *  overlap on a GPU (other streams or host threads) race; calls on one stream
 *  are ordered.
 * Errors: as pft_forward_3d; EINVAL also for a mesh or Q list too large for
 * the array (the message gives the sizes).
 */
pft_status pft_forward_3d_noalloc(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                  const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, void* out,
                                  void* intensity, void* stream);

/*
 * pft_forward_3d_poly -- F(Q) of the volume enclosed by planar polygon faces
 * (3D section: eq. sum_elements_3d with nu_m edges per face, evaluated natively:
 * nu edge terms per face).
 *
 *  verts        [nv][3] of vdtype (DEVICE).
 *  face_offsets HOST int64 [nf + 1], non-decreasing from 0; face i is
 *               face_verts[face_offsets[i] .. face_offsets[i+1]), 3 to 256
 *               vertices, counter-clockwise seen from outside. Faces must be
 *               planar (the normal is taken from the polygon's area vector) and
 *               simple; the mesh closed as in pft_forward_3d.
 *  face_verts   DEVICE int32, 0-based vertex indices. A face with an
 *               out-of-range index or zero area contributes 0.
 *  q, mode, out, intensity as in pft_forward_3d.
 * Errors: as pft_forward_3d; EINVAL also for bad offsets, a face with fewer
 * than 3 or more than 256 vertices, or more than 2^31 - 1 vertex references.
 */
pft_status pft_forward_3d_poly(const void* verts, pft_dtype vdtype, int64_t nv, const int64_t* face_offsets,
                               const int32_t* face_verts, int64_t nf, const void* q, pft_dtype qdtype, int64_t nq,
                               pft_mode mode, void* out, void* intensity, void* stream);

/*
 * pft_orientation_average -- orientation-averaged intensity of a closed mesh,
 *     I(q_i) = sum_j w_j |F(q_i s_j)|^2,
 * the powder / solution-scattering quantity that motivates the method (the
 * paper's introduction), with F as in pft_forward_3d evaluated at every
 * (magnitude, direction) pair in the given arithmetic form.
 *
 *  Mesh arguments as in pft_forward_3d.
 *  qabs     [nqa] float64 magnitudes |Q| (DEVICE).
 *  dirs     [ndir][3] float64 unit directions s_j (DEVICE).
 *  weights  [ndir] float64 quadrature weights w_j (DEVICE); for the average
 *           over the sphere they sum to 1 (a product Gauss-Legendre x uniform
 *           quadrature is exact for spherical harmonics up to its degree).
 *  mode     PFT_FP64 or PFT_FP32C for the transform; the weighted sum is
 *           formed in binary64 in a fixed order either way.
 *  out      [nqa] float64 (DEVICE), overwritten; 0 when ndir == 0.
 *  face_order, face_meta  NULL, or an edge-sharing face order as for
 *           pft_forward_3d_ordered (DEVICE; both or neither).
 * Temporaries: nqa * ndir Q points (24 B each) and intensities.
 * Errors: as pft_forward_3d; EINVAL also for nqa > 2^31 - 1,
 * nqa * ndir * 3 beyond int64, or only one of face_order, face_meta given.
 */
pft_status pft_orientation_average(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                   const double* qabs, int64_t nqa, const double* dirs, const double* weights,
                                   int64_t ndir, pft_mode mode, double* out, const int32_t* face_order,
                                   const uint8_t* face_meta, void* stream);

/*
 * pft_backward_3d -- adjoint of pft_forward_3d with respect to the vertices.
 * The paper gives the forward transform only; the derivative follows from the
 * same volume integral: moving the boundary with velocity field u changes F by
 * the surface integral of exp(iQ.r) (u . n) dA, and a vertex moves the points
 * of its incident faces with their barycentric (hat) weight, so
 *     dF(Q)/dv_k = sum over faces m containing k of n_m * integral over m of lambda_k exp(iQ.r) dA.
 *
 *  Mesh and q arguments as in pft_forward_3d.
 *  grad_out    [nq] complex, dL/dRe F(Q) + i dL/dIm F(Q) for a real loss L
 *              (complex128 in PFT_FP64 mode, complex64 in PFT_FP32C mode).
 *  grad_verts  [nv][3] of vdtype, OVERWRITTEN with
 *              dL/dv_k = sum_Q Re(conj(grad_out(Q)) dF(Q)/dv_k).
 * Errors: as pft_forward_3d.
 */
pft_status pft_backward_3d(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                           const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, const void* grad_out,
                           void* grad_verts, void* stream);

/*
 * pft_backward_3d_ordered -- pft_backward_3d visiting the Q in a given order
 * (pft_q_order) instead of sorting them in the call.
 *  q_order  NULL (sorted here) or [nq] uint32 (DEVICE), a permutation of
 *           0 .. nq-1 (an entry out of range is replaced by its position).
 * Errors: as pft_backward_3d.
 */
pft_status pft_backward_3d_ordered(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                   const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, const void* grad_out,
                                   void* grad_verts, const uint32_t* q_order, void* stream);

/*
 * pft_intensity_loss_3d -- the intensity loss
 *     L = sum_Q w(Q) (|F(Q)|^2 - I(Q))^2
 * and its vertex gradient in one call: the forward of pft_forward_3d, the
 * cotangent dL/dRe F + i dL/dIm F = 4 w (|F|^2 - I) F formed on the device in
 * binary64 as the partial sums are finished, and the adjoint of
 * pft_backward_3d, sharing one set of face records and one Q order. For
 * fitting a mesh to a measured intensity (the scattering use of the
 * transform); the paper gives the forward only.
 *
 *  Mesh, q and mode arguments as in pft_forward_3d.
 *  weight      NULL (w = 1) or [nq] float64 (DEVICE).
 *  target      [nq] float64 I(Q) (DEVICE).
 *  loss        DEVICE float64 scalar, overwritten with L (summed in binary64
 *              in a fixed order).
 *  out         NULL or [nq] complex F(Q) (complex128 for PFT_FP64, complex64 for PFT_FP32C).
 *  grad_verts  NULL or [nv][3] of vdtype, OVERWRITTEN with dL/dv.
 *  face_order, face_meta  NULL, or an edge-sharing face order for the FP32C
 *              forward as for pft_forward_3d_ordered (DEVICE; both or neither).
 * Errors: as pft_forward_3d; EINVAL also for loss NULL, target NULL with
 * nq > 0, or only one of face_order, face_meta given.
 */
pft_status pft_intensity_loss_3d(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                 const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode, const double* weight,
                                 const double* target, double* loss, void* out, void* grad_verts,
                                 const int32_t* face_order, const uint8_t* face_meta, void* stream);

/*
 * pft_forward_3d_regions -- F(Q) of a density that is constant on each of
 * several closed regions: F = sum_j rho_j F_j, F_j the transform of region j
 * (the "constant quantity over a volume" of the method, taken piecewise).
 *
 *  verts, vdtype, nv, q, qdtype, nq, mode, intensity as in pft_forward_3d.
 *  tris            [nf][3] int32 (DEVICE): the outward boundaries of the
 *                  regions, region j owning triangles region_offsets[j] ..
 *                  region_offsets[j+1]). A surface shared by two regions is
 *                  listed in both, with opposite orientations (it may reuse
 *                  the same vertices). Each region must be closed.
 *  region_offsets  HOST int64 [nreg + 1], non-decreasing from 0 to nf.
 *  nreg            number of regions, 0 .. 4096 (nreg = 0 gives F = 0).
 *  rho             [nreg] float64 densities (DEVICE).
 *  out             [nq] complex (complex128 for PFT_FP64, complex64 for PFT_FP32C).
 *  out_regions     NULL or [nreg][nq] complex of the same type: F_j, which is
 *                  also dF/drho_j.
 *  face_order, face_meta  NULL, or an edge-sharing order as for
 *                  pft_forward_3d_ordered that keeps every face within its
 *                  region's range (DEVICE; both or neither; used by FP32C).
 * Temporaries: about (nreg + 40) * nq * 16 bytes of partial sums.
 * Errors: as pft_forward_3d; EINVAL also for bad offsets, offsets that do not
 * end at nf, nreg outside 0 .. 4096, rho NULL with nreg > 0, or only one of
 * face_order, face_meta given.
 */
pft_status pft_forward_3d_regions(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                  const int64_t* region_offsets, int64_t nreg, const double* rho, const void* q,
                                  pft_dtype qdtype, int64_t nq, pft_mode mode, void* out, void* out_regions,
                                  void* intensity, const int32_t* face_order, const uint8_t* face_meta,
                                  void* stream);

/*
 * pft_backward_3d_regions -- gradients of a real loss L(F) with
 * F = sum_j rho_j F_j (pft_forward_3d_regions), given
 * grad_out = dL/dRe F + i dL/dIm F:
 *     dL/dv_k    = sum_Q Re(conj(g) sum_j rho_j dF_j/dv_k)  (as pft_backward_3d, faces weighted by their density),
 *     dL/drho_j  = sum_Q Re(conj(g) F_j),
 *     dL/dQ      = Re(conj(g) grad_Q F),  grad_Q F = i * integral of rho r exp(iQ.r) dV.
 * The paper gives none of these; grad_Q F follows from the divergence theorem
 * with the field x_a (-iQ/|Q|^2) exp(iQ.r) and the barycentric moments of the
 * faces (r is linear on a face), and from the tetrahedron fan for |Q| R < 0.5.
 * With one region of density 1 this is the Q-gradient of pft_forward_3d.
 *
 *  Mesh, region, q and mode arguments as in pft_forward_3d_regions.
 *  grad_out    [nq] complex (complex128 for PFT_FP64, complex64 for PFT_FP32C).
 *  grad_verts  NULL or [nv][3] of vdtype, OVERWRITTEN.
 *  grad_rho    NULL or [nreg] float64, OVERWRITTEN.
 *  grad_q      NULL or [nq][3] of qdtype, OVERWRITTEN.
 * Outputs that are NULL are not computed. Temporaries: as the adjoint for
 * grad_verts; (nreg + 40) * nq * 64 bytes for grad_q.
 * Errors: as pft_forward_3d_regions.
 */
pft_status pft_backward_3d_regions(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                                   const int64_t* region_offsets, int64_t nreg, const double* rho, const void* q,
                                   pft_dtype qdtype, int64_t nq, pft_mode mode, const void* grad_out,
                                   void* grad_verts, double* grad_rho, void* grad_q, void* stream);

/*
 * A batch of independent closed meshes, each with its own Q list, stored as
 * concatenations. Offsets are HOST int64 arrays of length n_meshes + 1,
 * non-decreasing from 0; mesh i owns verts[vert_offsets[i] .. vert_offsets[i+1]),
 * tris[tri_offsets[i] .. tri_offsets[i+1]) with indices LOCAL to mesh i, and
 * q[q_offsets[i] .. q_offsets[i+1]). Outputs follow q_offsets (forward) and
 * vert_offsets (backward).
 */
typedef struct {
  int64_t n_meshes;
  const int64_t* vert_offsets; /* HOST [n_meshes + 1] */
  const int64_t* tri_offsets;  /* HOST [n_meshes + 1] */
  const int64_t* q_offsets;    /* HOST [n_meshes + 1] */
  const void* verts;           /* DEVICE [total_nv][3] of vdtype */
  pft_dtype vdtype;
  const int32_t* tris;         /* DEVICE [total_nf][3], local indices */
  const void* q;               /* DEVICE [total_nq][3] of qdtype */
  pft_dtype qdtype;
} pft_mesh_batch;

/*
 * pft_batch_forward -- pft_forward_3d for every mesh of a batch in one
 * persistent launch: (mesh, Q-tile, face-chunk) work items ordered by cost,
 * pulled from a device work counter by a grid sized to the GPU.
 *  out        [total_nq] complex (complex128 for PFT_FP64, complex64 for PFT_FP32C).
 *  intensity  NULL or [total_nq] |F|^2 (float64 / float32).
 * Errors: as pft_forward_3d, plus EINVAL for offsets that are not non-decreasing from 0.
 */
pft_status pft_batch_forward(const pft_mesh_batch* batch, pft_mode mode, void* out, void* intensity, void* stream);

/*
 * pft_batch_forward_ordered -- pft_batch_forward with each mesh's faces in an
 * edge-sharing order (pft_strip_order of the mesh, offset by its first
 * triangle), so that the FP32C forward reuses shared edge terms as
 * pft_forward_3d_ordered does.
 *  face_order  [total_nf] int32 (DEVICE): position m (in mesh i's triangle
 *              range) holds a triangle of the same mesh; an entry out of
 *              range makes that position an empty face.
 *  face_meta   [total_nf] uint8 (DEVICE), as written by pft_strip_order.
 * Errors: as pft_batch_forward; EINVAL also for face_order or face_meta NULL.
 */
pft_status pft_batch_forward_ordered(const pft_mesh_batch* b, const int32_t* face_order, const uint8_t* face_meta,
                                     pft_mode mode, void* out, void* intensity, void* stream);

/*
 * pft_batch_backward -- pft_backward_3d for every mesh of a batch.
 *  grad_out    [total_nq] complex (complex128 / complex64 by mode).
 *  grad_verts  [total_nv][3] of vdtype, overwritten.
 */
pft_status pft_batch_backward(const pft_mesh_batch* batch, pft_mode mode, const void* grad_out, void* grad_verts,
                              void* stream);

/*
 * pft_check_mesh -- what the method requires of a triangle mesh, checked on the
 * host (3D section: the boundary is a closed polygonal surface whose faces run
 * counter-clockwise seen from outside). An open surface makes the sum over
 * faces depend on the origin, and faces of inconsistent orientation subtract
 * where they should add. HOST function, no GPU work.
 *
 *  tris    [nf][3] int32 (HOST).
 *  report  HOST, written: the counts below; a mesh passes when all are zero.
 * The enclosed volume's sign (negative for an inward mesh, which gives -F) needs
 * the vertices: F(0) is that volume. With PFT_VALIDATE=1 in the environment the
 * 3D entry points run this check on their (device) mesh, each region on its
 * own, and also reject a negative volume, returning EINVAL with the counts.
 * Errors: EINVAL for negative counts or NULL pointers.
 */
typedef struct {
  int64_t bad_index;          /* faces with an index outside [0, nv) */
  int64_t repeated_vertex;    /* faces listing a vertex twice */
  int64_t open_edges;         /* edges of exactly one face: the surface has a boundary */
  int64_t nonmanifold_edges;  /* edges of more than two faces */
  int64_t misoriented_edges;  /* edges that both of their faces run in the same direction */
} pft_mesh_check;
pft_status pft_check_mesh(const int32_t* tris, int64_t nf, int64_t nv, pft_mesh_check* report);

/*
 * pft_fp32c_q_limit -- the largest |Q| at which the FP32C form evaluates a
 * triangle mesh: PFT_FP32C_PHASE_MAX / rho, rho the largest distance from a
 * face's centroid to one of its vertices (faces with an index outside [0, nv)
 * are skipped, as the transform skips them); +infinity when no face has extent.
 * HOST function, no GPU work: verts [nv][3] of vdtype, tris [nf][3] int32 and
 * q_limit are host pointers.
 * Errors: EINVAL for negative counts or NULL pointers (verts may be NULL when
 * nv is 0, tris when nf is 0), EUNSUPPORTED for an unknown vertex dtype.
 */
pft_status pft_fp32c_q_limit(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris, int64_t nf,
                             double* q_limit);

/*
 * pft_validate_mesh -- count triangle indices outside [0, nv) and faces with a
 * repeated vertex. Synchronous: blocks until the check has run on `stream`.
 * Both outputs are HOST pointers (either may be NULL).
 */
pft_status pft_validate_mesh(const int32_t* tris, int64_t nf, int64_t nv, int64_t* n_bad_index,
                             int64_t* n_repeated_vertex, void* stream);

/* Message for the last non-OK status returned on the calling thread ("" if none). */
const char* pft_last_error(void);

/* Free the per-stream workspaces of the current device and return cached
 * stream-ordered memory to the system (synchronises the device). */
pft_status pft_release_workspace(void);

/*
 * Kernel timing, for measurement. When enabled, each entry point records HIP
 * events on its stream around its main compute kernel(s); pft_profile_read
 * synchronises on the recorded events and returns, for the kernel family
 * `name` ("fwd3d_fp32c", "fwd3d_fp64", "bwd3d_fp32c", "bwd3d_fp64", "fwd2d_fp64",
 * "batch_fwd", "batch_bwd"), the number of launches and their summed
 * duration in milliseconds since the last reset. HOST pointers.
 */
pft_status pft_profile_enable(int enable);
pft_status pft_profile_reset(void);
pft_status pft_profile_read(const char* name, int64_t* launches, double* total_ms);

/*
 * Tile sizes of the batched launches (the batched forward's Q per thread and
 * faces per work item, the batched adjoint's Q per work item) are chosen at run
 * time per (GPU, form, size bucket of meshes, faces and face*Q pairs): the
 * first pft_batch_forward / pft_batch_backward call with a new key runs each
 * candidate once on its input, times it (that call synchronises), keeps the
 * fastest and produces its output with it; later calls with the key reuse the
 * choice. PFT_AUTOTUNE=0 in the environment selects the compiled defaults.
 * pft_tuning_info returns one line per choice made in this process (key,
 * choice and each candidate's time); the text is valid until the next call on
 * the same thread.
 */
const char* pft_tuning_info(void);

/* Library version string. */
const char* pft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PFT_H */
