/*
 * facetransfer: transfer of halo data across 3:1 resolution transitions of a
 * block-structured 3D Cartesian spacetree mesh, on AMD Instinct MI355X
 * (gfx950).  Implements the interpolation and restriction of Stokes,
 * Weinzierl, Zhang and Li, "Fast Higher-Order Interpolation and Restriction
 * in ExaHyPE Avoiding Non-physical Reflections" (arXiv 2504.15814):
 * the d-linear tensor-product baseline and the second- and third-order
 * Taylor schemes, applied as one operator per face.
 *
 * ---------------------------------------------------------------------------
 * Data layout (the paper stores face data "AoS lexicographically", Section
 * 4.1; everything else below is this library's convention)
 * ---------------------------------------------------------------------------
 * A face buffer belongs to one face of a patch of p^3 cells with halo depth k
 * (Section 2).  Orientation o in 0..5 names the normal axis a = o mod 3; the
 * tangential axes b < c are the other two, in increasing order.  The buffer
 * holds 2k cells along a and p along b and c; cell (i0, i1, i2) (indices
 * along physical axes 0, 1, 2) has cell number (i2*e1 + i1)*e0 + i0 where
 * e_a = 2k and e_b = e_c = p, and unknown u of that cell is element
 * cell*U + u.  Normal index [0, k) is the - side of the face, [k, 2k) the +
 * side.  For o < 3 the fine patch lies on the + side, for o >= 3 on the -
 * side.
 *
 * A hanging (fine) face is one of the 3x3 subfaces of its coarse face
 * (three-partitioning, Section 2); subface s = sb + 3*sc with sb, sc in 0..2
 * covers coarse columns [sb*p/3, (sb+1)*p/3) x [sc*p/3, (sc+1)*p/3) of the
 * coarse face.  Coarse and fine face buffers have the same shape.  When p is
 * not a multiple of 3 (Section 5.3 times such sizes) a coarse column may
 * straddle two fine faces: interpolation writes the fine face's own cells,
 * and restriction writes the coarse columns whose centres lie on the fine
 * face (every coarse centre lies on exactly one fine face, on one of its
 * fine centres); the averaging restriction of a straddling column takes
 * that fine column instead of the mean of three.
 *
 * Interpolation (Q^f = P Q^c, Section 2) reads both halves of the coarse
 * face buffer and writes the fine face buffer's coarse-side half (its halo).
 * Restriction (Q^c = R Q^f, Section 2) reads the fine face buffer (both
 * halves) and writes the part of the coarse face buffer's fine-side half that
 * lies under the subface.  Both apply only the 1/9 segment of P or R that
 * belongs to the subface, the same operator for every unknown.
 *
 * Schemes (Section 3, Appendix C): FT_DLINEAR is the tensor-product baseline
 * (1D linear interpolation per axis with linear extrapolation at the face
 * edges; restriction by averaging).  FT_TAYLOR2 / FT_TAYLOR3 evaluate, at
 * every target centre, a Taylor polynomial of degree 2 / 3 about the nearest
 * source cell, fitted by least squares with the constant pinned to that
 * cell's value over a 3x3x3 box stencil (plus the two-away axial points for
 * degree 3), shifted toward the face interior at face edges.  Coinciding
 * centres are copied bit for bit.
 *
 * Supported sizes: 6 <= p <= 48; k in {2, 3} for every
 * scheme and k = 1 (the finite-volume halo of Section 2) for FT_DLINEAR; there
 * the single fine ghost layer is interpolated between coarse layer 0 and the
 * coarse face's fine-side layer, and the coarse halo layer is extrapolated
 * through the fine face's inner layer and its halo layer; 1 <= U <= 4096.
 *
 * ---------------------------------------------------------------------------
 * Ownership, streams and errors
 * ---------------------------------------------------------------------------
 * Every data pointer passed to an apply call is DEVICE memory owned by the
 * caller.  Operators are owned by the library until destroyed; they are
 * immutable after build and may be shared across threads and streams.
 * Apply calls are asynchronous on the given HIP stream (NULL = the null
 * stream), allocate nothing and never synchronise, so they may be captured
 * into a HIP graph.
 *
 * All entry points return FT_OK or an error code and never throw; a message
 * for the last failure on the calling thread is available from
 * transfer_last_error().  Argument checks happen on the host before anything
 * is launched.  Per-face descriptors live in device memory and are checked
 * by the kernels: a face whose orientation, subface or offsets are out of
 * range (offset < 0 or offset + 2k*p*p*U > the buffer's element count) is
 * skipped, writes nothing, and is counted in the operator's device error
 * counter (transfer_operator_errors).
 *
 * Aliasing: source and destination buffers must not overlap, except that
 * several restriction faces may write disjoint segments of the same coarse
 * face, and several interpolation faces may read the same coarse face.
 */
#ifndef FACETRANSFER_H
#define FACETRANSFER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define FT_OK 0
#define FT_ERR_INVALID 1     /* bad argument (null pointer, range, mismatch) */
#define FT_ERR_UNSUPPORTED 2 /* valid but unsupported (p, k, scheme, dtype)  */
#define FT_ERR_HIP 3         /* HIP runtime failure                           */
#define FT_ERR_NOMEM 4       /* device or host allocation failed              */

/* Directions. */
#define FT_INTERPOLATE 0
#define FT_RESTRICT 1

/* Schemes. */
#define FT_DLINEAR 1
#define FT_TAYLOR2 2
#define FT_TAYLOR3 3

/* Element types of face buffers and how the operator is applied.
 * FT_F64:        float64 storage, float64 arithmetic.
 * FT_F32:        float32 storage; interpolation sums in float32 with float32
 *                weights on the vector ALUs, restriction sums in float64
 *                (extrapolation weights have a large 1-norm, so cancellation
 *                decides the accuracy there).
 * FT_F32_BF16X3: float32 storage; interpolation on the matrix cores: weights
 *                and data are split into bfloat16 parts (x = x0 + x1 + x2
 *                exactly, W = W0 + W1 + W2) and W0 x0 + W0 x1 + W1 x0 is
 *                accumulated in float32 (each dropped product is at most
 *                2^-16 of |w x|: error <= about 3 * 2^-16 of sum |w x| per
 *                output).  Restriction as FT_F32.
 * FT_F32_BF16X6: as FT_F32_BF16X3 plus the compensating products
 *                W0 x2 + W1 x1 + W2 x0 of the split residuals (dropped terms
 *                <= 3 * 2^-24 of sum |w x|, i.e. float32 rounding level).
 *                Restriction as FT_F32.
 * FT_F64_TO_F32: restriction only, face buffers only: float64 fine data,
 *                float64 sums, float32 coarse faces (each output is the
 *                FT_F64 result rounded once to float32).  Restriction's
 *                extrapolation rows (Section 3: coarse layers without a
 *                coinciding fine cell; weights of 1-norm up to about 400)
 *                amplify the rounding of float32-stored fine data to about
 *                1e-5 of the field; with float64 fine data the coarse faces
 *                carry only their own float32 rounding, and interpolation
 *                from them in FT_F32 or FT_F32_BF16X6 into float32 fine halo
 *                buffers keeps a restrict-then-interpolate step within about
 *                1e-6 of float64. */
#define FT_F64 0
#define FT_F32 1
#define FT_F32_BF16X3 2
#define FT_F32_BF16X6 3
#define FT_F64_TO_F32 4

/* Build flags. */
#define FT_BUILD_HOST_ONLY 1 /* build the weight tables on the host only; the
                                operator can be inspected but not applied  */
#define FT_BUILD_2D 2        /* two-dimensional faces (see below)           */

/* Two dimensions (Sections 2-3 state the method for any dimension): with
 * FT_BUILD_2D the operator works on faces of two-dimensional patches (p^2
 * cells, halo depth k).  Orientation o in 0..3 names the normal axis
 * a = o mod 2; the tangential axis is the other one; the fine patch lies on
 * the + side for o < 2.  A face buffer holds 2k cells along a and p along the
 * tangential axis, cell (i0, i1) at cell number i1*e0 + i0 (axis 0 fastest,
 * unknowns innermost), normal index [0, k) on the - side.  Subface s in 0..2
 * covers coarse columns [s*p/3, (s+1)*p/3).  The stencils are the 3 x 3
 * box (plus the two-away axial points for degree 3).  interpolate_faces and
 * restrict_faces take such operators in every dtype; plans and the patch
 * calls below take three-dimensional operators only. */

typedef struct ft_operator ft_operator;

/* Build the transfer operator for one (direction, scheme, p, k).
 * The Taylor fits and d-linear weights are assembled in extended precision on
 * the host and rounded to float64 (and float32) weight tables, one dense block
 * per class of expansion cell (Section 3: the matrices are precomputed once
 * instead of per call), then copied to the current HIP device unless
 * FT_BUILD_HOST_ONLY is set.
 * out: receives the handle (library-owned; release with
 *      destroy_transfer_operator).
 * Errors: FT_ERR_INVALID (null out, unknown direction / scheme),
 *         FT_ERR_UNSUPPORTED (p, k outside the supported set, k = 1 with a
 *         Taylor scheme),
 *         FT_ERR_NOMEM, FT_ERR_HIP. */
int build_transfer_operator(int direction, int scheme, int p, int k, int flags,
                            ft_operator** out);

/* Release an operator; NULL is accepted and ignored.  The caller must make
 * sure no launch that uses it is still pending. */
int destroy_transfer_operator(ft_operator* op);

/* Interpolate fine halo layers from coarse face data (Section 2, Q^f = P Q^c;
 * Section 3, Taylor expansion about the containing coarse cell).
 * op            : an FT_INTERPOLATE operator built for the device in use.
 * n_faces       : number of hanging faces (0 is a no-op).
 * orientation   : device int8[n_faces], 0..5.
 * subface       : device int8[n_faces], 0..8.
 * coarse_offset : device int64[n_faces], element offset of each face's coarse
 *                 face buffer inside `coarse`.
 * fine_offset   : device int64[n_faces], element offset of each fine face
 *                 buffer inside `fine`.
 * unknowns      : U, unknowns per cell (AoS, innermost).
 * dtype         : FT_F64, FT_F32, FT_F32_BF16X3 or FT_F32_BF16X6 (the last
 *                 three store float32).
 * coarse        : device, coarse_elems elements, read only.
 * fine          : device, fine_elems elements; only the halo (coarse-side)
 *                 half of each referenced fine face buffer is written.
 * stream        : hipStream_t (NULL for the null stream).
 * Errors (host-side, nothing launched): FT_ERR_INVALID, FT_ERR_UNSUPPORTED;
 * FT_ERR_HIP if the launch fails. */
int interpolate_faces(const ft_operator* op, int64_t n_faces, const int8_t* orientation,
                      const int8_t* subface, const int64_t* coarse_offset,
                      const int64_t* fine_offset, int unknowns, int dtype,
                      const void* coarse, int64_t coarse_elems, void* fine,
                      int64_t fine_elems, void* stream);

/* Restrict fine face data into the coarse face's fine-side half (Section 2,
 * Q^c = R Q^f; Section 3, Taylor expansion about the fine cell nearest each
 * coarse centre: injection where they coincide, extrapolation elsewhere).
 * Arguments as for interpolate_faces, with `fine` read only and `coarse`
 * written: per face, the (p/3)^2 * k cells of the coarse face's fine-side half
 * that lie under the subface.  dtype may also be FT_F64_TO_F32: `fine` then
 * holds float64 (fine_elems of them) and `coarse` float32. */
int restrict_faces(const ft_operator* op, int64_t n_faces, const int8_t* orientation,
                   const int8_t* subface, const int64_t* coarse_offset,
                   const int64_t* fine_offset, int unknowns, int dtype, const void* fine,
                   int64_t fine_elems, void* coarse, int64_t coarse_elems, void* stream);

/* Operator facts, written to info[0..n_info) (host memory):
 * [0] direction  [1] scheme  [2] p  [3] k
 * [4] rows per expansion cell (interpolation 9k, restriction k; 2D: 3k, k)
 * [5] expansion cells per subface ((p/3)^2; 2D: p/3)
 * [6] number of distinct weight blocks  [7] largest block width (stencil)
 * [8] nonzero weights in one subface segment (orientation 0, subface 4;
 *     2D: subface 1)
 * [9] bytes of the float64 weight tables
 * [10] dimension (3, or 2 with FT_BUILD_2D)
 * Errors: FT_ERR_INVALID for a null op / info or n_info < 1. */
int transfer_operator_info(const ft_operator* op, int64_t* info, int n_info);

/* Export the 1/9 segment of the operator for one (orientation, subface) in
 * physical cell numbering, as COO triplets into caller-owned host arrays of
 * `capacity` entries: rows[] are destination cell numbers, cols[] source cell
 * numbers, vals[] float64 weights.  *n_entries receives the count (also when
 * capacity is too small, in which case nothing is written and
 * FT_ERR_INVALID is returned).  Host only; needs no device. */
int transfer_operator_segment(const ft_operator* op, int orientation, int subface,
                              int64_t capacity, int64_t* rows, int64_t* cols, double* vals,
                              int64_t* n_entries);

/* ---------------------------------------------------------------------------
 * Patches: the transfer fused with the patch halos
 * ---------------------------------------------------------------------------
 * Section 2: every patch of p^3 cells carries a halo of depth k on its faces
 * (not on edges or vertices), refreshed at the start of a time step from the
 * face-connected neighbours: a plain copy between patches of one level, the
 * transfer across a resolution transition.  The face buffers above are the 2k
 * layers around one face; the calls below read and write them in place
 * inside the patches, so no face buffer has to be assembled and scattered.
 *
 * Patch layout: a box of P = p + 2k cells per axis whose interior is
 * [k, k + p) on every axis; cell (i0, i1, i2) is cell number (i2*P + i1)*P + i0
 * (axis 0 fastest) and unknown u of it is element cell*U + u.  Edge and vertex
 * cells of the box exist in storage and are never read or written.
 *
 * Patch faces are numbered f = a + 3*upper (f < 3: the face at the lower
 * boundary along axis a; f >= 3: the upper one).  The face view of face f is
 * the 2k x p x p box of cells around it: normal cells [0, 2k) (f < 3) or
 * [p, p + 2k) (f >= 3), tangential cells [k, k + p).  In storage order its
 * cells are those of a face buffer of that face (layer 0 on the - side).  The
 * half of the view inside the patch is its inner half, the other its outer
 * (halo) half.  At a transition face of orientation o the fine patch's face
 * is f = o and the coarse patch's face is f = (o + 3) mod 6.
 *
 * Per-item descriptors live in device memory and are checked by the kernels
 * against the element counts; an item out of range is skipped and counted
 * (the transfer in the operator's counter, the copies in *skipped when that
 * device pointer is not NULL). */
#define FT_HALF_INNER 1
#define FT_HALF_OUTER 2
#define FT_HALF_BOTH 3

/* Interpolate into the halo of each fine patch straight from its coarse
 * patch: the same arithmetic as interpolate_faces on the face views (the
 * coarse patch's face view, both halves, is read; the fine patch's outer
 * half of face o is written).
 * coarse_offset / fine_offset: element offsets of the coarse and fine
 * patches (their cell (0, 0, 0)).  Other arguments as for interpolate_faces.
 * `coarse` and `fine` may be the same array (one pool of patches): a call
 * reads coarse face views and writes fine halos, which are disjoint as long
 * as no (fine patch, orientation) pair is listed twice. */
int interpolate_patches(const ft_operator* op, int64_t n_faces, const int8_t* orientation,
                        const int8_t* subface, const int64_t* coarse_offset,
                        const int64_t* fine_offset, int unknowns, int dtype,
                        const void* coarse, int64_t coarse_elems, void* fine,
                        int64_t fine_elems, void* stream);

/* Restrict from each fine patch into the halo of its coarse patch: the same
 * arithmetic as restrict_faces on the face views (the fine patch's face view
 * of face o, both halves, is read; in the coarse patch's outer half of face
 * (o + 3) mod 6 the (p/3)^2 * k cells under the subface are written).
 * Offsets as for interpolate_patches; `fine` and `coarse` may be one array. */
int restrict_patches(const ft_operator* op, int64_t n_faces, const int8_t* orientation,
                     const int8_t* subface, const int64_t* coarse_offset,
                     const int64_t* fine_offset, int unknowns, int dtype, const void* fine,
                     int64_t fine_elems, void* coarse, int64_t coarse_elems, void* stream);

/* Copy the chosen halves (FT_HALF_*) of face view face[i] of the patch at
 * patch_offset[i] into the face buffer at face_offset[i] (Section 2: the
 * face data of a patch are its boundary layers and the halo facing them).
 * p >= 1, 1 <= k <= p, 1 <= U <= 4096; dtype selects the element size only
 * (FT_F64: 8 bytes, the float32 modes: 4 bytes; values are copied bit for
 * bit).  face: device int8[n], 0..5; offsets: device int64[n].  patches and
 * faces must not overlap.  skipped: device int, or NULL. */
int gather_patch_faces(int p, int k, int64_t n, const int8_t* face, const int64_t* patch_offset,
                       const int64_t* face_offset, int halves, int unknowns, int dtype,
                       const void* patches, int64_t patch_elems, void* faces,
                       int64_t face_elems, int* skipped, void* stream);

/* The reverse of gather_patch_faces: the chosen halves of each face buffer
 * are written into face view face[i] of its patch. */
int scatter_patch_faces(int p, int k, int64_t n, const int8_t* face, const int64_t* patch_offset,
                        const int64_t* face_offset, int halves, int unknowns, int dtype,
                        const void* faces, int64_t face_elems, void* patches,
                        int64_t patch_elems, int* skipped, void* stream);

/* Same-level halo exchange (Section 2: where both neighbours have one
 * resolution the halo is a copy).  Pair i: the patch at lower_offset[i]
 * touches the patch at upper_offset[i] across its upper face along axis[i]
 * (device int8, 0..2).  The lower patch's upper halo receives the upper
 * patch's first k interior layers, and the upper patch's lower halo the lower
 * patch's last k interior layers.  Both patches live in `patches`; a call
 * reads interiors and writes halos, so pairs may share patches, but each halo
 * (patch, face) must be written by at most one pair. */
int copy_patch_halos(int p, int k, int64_t n_pairs, const int8_t* axis,
                     const int64_t* lower_offset, const int64_t* upper_offset, int unknowns,
                     int dtype, void* patches, int64_t patch_elems, int* skipped, void* stream);

/* ---------------------------------------------------------------------------
 * Plans: uneven mixes in one launch
 * ---------------------------------------------------------------------------
 * A plan groups batches of hanging faces that use different operators
 * (direction, scheme, p, k) over one coarse and one fine buffer, with one
 * element type and one unknown count, and runs them as one persistent
 * launch: a fixed grid of waves walks all (face, anchor) work items.  With
 * FT_PLAN_RESTRICT_FIRST every restriction batch completes before any
 * interpolation batch starts (two launches), as one time step needs when
 * the interpolated faces read coarse data that the restriction writes
 * (Section 2: halos are refreshed before the compute kernel).  Without it,
 * all batches must be independent (no face writes what another reads). */
#define FT_PLAN_RESTRICT_FIRST 1
/* FT_PLAN_PATCHES: every batch addresses patches (the layout of the patch
 * calls above): coarse_offset / fine_offset are patch offsets and `coarse` /
 * `fine` are patch pools, which may be the same array. */
#define FT_PLAN_PATCHES 2

typedef struct ft_plan ft_plan;
typedef struct ft_graph ft_graph;

/* One batch of a plan (host struct; the arrays it points to are DEVICE
 * memory, laid out as for interpolate_faces / restrict_faces). */
typedef struct ft_plan_batch {
  const ft_operator* op;
  int64_t n_faces;
  const int8_t* orientation;
  const int8_t* subface;
  const int64_t* coarse_offset;
  const int64_t* fine_offset;
} ft_plan_batch;

/* Build a plan over n_batches batches (the batches[] array is copied; the
 * operators, device arrays and buffers must stay valid while the plan or a
 * graph captured from it is used).
 * dtype as for interpolate_faces; restriction batches of the FT_F32_BF16X*
 * types run as FT_F32.  FT_F64_TO_F32 (restriction batches only, face
 * buffers only) takes a float64 `fine` and a float32 `coarse` array.  The schedule starts at a default and can be tuned
 * with transfer_plan_autotune.  Allocates its small device segment tables.
 * Errors: FT_ERR_INVALID (null pointers, n_batches < 1, operators of another
 * device), FT_ERR_UNSUPPORTED (dtype, unknowns), FT_ERR_NOMEM, FT_ERR_HIP. */
int build_transfer_plan(const ft_plan_batch* batches, int n_batches, int unknowns, int dtype,
                        void* coarse, int64_t coarse_elems, void* fine, int64_t fine_elems,
                        int flags, ft_plan** out);

/* Run the plan asynchronously on `stream` (no allocation, no host
 * synchronisation: capturable). */
int run_transfer_plan(const ft_plan* plan, void* stream);

/* One fused launch over `n_batches` batches, as build_transfer_plan +
 * run_transfer_plan with the default schedule would run them, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): this call allocates
 * nothing.  The batches' segment table goes into a fixed workspace of the
 * library in device memory (one per device, held until the process ends,
 * room for 128 non-empty batches per phase, 20 KiB), written by a small
 * kernel on `stream` before the transfer kernels.  Arguments, checks and
 * results are those of build_transfer_plan / run_transfer_plan (bitwise
 * equal to the plan's outputs); nothing needs to be zero beforehand.
 * Asynchronous on `stream`.  Calls on one device share the workspace: calls
 * that overlap in time (on different streams, without ordering between
 * them) race and must not be issued; calls on one stream are safe.
 * Errors: as build_transfer_plan, plus FT_ERR_UNSUPPORTED for more than 128
 * non-empty batches in one phase (FT_PLAN_RESTRICT_FIRST puts restriction
 * batches in phase 0 and interpolation batches in phase 1; otherwise every
 * batch is in phase 0). */
int run_transfer_batches(const ft_plan_batch* batches, int n_batches, int unknowns, int dtype,
                         void* coarse, int64_t coarse_elems, void* fine, int64_t fine_elems,
                         int flags, void* stream);

/* Schedule of a plan, packed as waves_per_block | blocks_per_cu << 8 |
 * xcd_remap << 16 | heavy_first << 17 | persistent << 18 (waves_per_block
 * in {1, 2, 4}, blocks_per_cu in 1..64).  persistent = 1: a grid of
 * blocks_per_cu blocks per compute unit walks all work items with a grid
 * stride; persistent = 0: one wave per work item (blocks_per_cu unused).
 * xcd_remap gives every XCD a contiguous range of items; heavy_first orders
 * the batches by decreasing cost per item.  Every schedule computes bitwise
 * identical results (each output's summation order is fixed by the
 * operator). */
int transfer_plan_set_schedule(ft_plan* plan, int64_t schedule);
int transfer_plan_get_schedule(const ft_plan* plan, int64_t* schedule);

/* Autotuner: run the plan `reps` times under each candidate schedule (after
 * one warm-up run), time it with HIP events on `stream`, keep the fastest,
 * and report it and its mean time in milliseconds.  The candidates are the
 * one-wave-per-item schedules (2 or 4 waves per block, xcd_remap and
 * heavy_first on or off); persistent schedules stay available through
 * transfer_plan_set_schedule.  The runs write the plan's outputs like
 * run_transfer_plan.  Synchronises the stream. */
int transfer_plan_autotune(ft_plan* plan, void* stream, int reps, int64_t* best_schedule,
                           double* best_ms);

int destroy_transfer_plan(ft_plan* plan);

/* Capture `steps` consecutive runs of the plan into one HIP graph on a
 * library-owned stream and instantiate it.  The graph holds the plan's
 * device segment tables (uploaded once, in both segment orders, when the
 * plan is built): it stays valid after the plan's schedule changes and after
 * destroy_transfer_plan, as long as the operators and buffers live. */
int transfer_plan_capture(const ft_plan* plan, int steps, ft_graph** out);

/* As transfer_plan_capture for a step made of several plans: each of the
 * `steps` captured steps runs plans[0], ..., plans[n_plans - 1] in order
 * (for instance an FT_F64_TO_F32 restriction plan and then a float32
 * interpolation plan that reads its coarse faces).  The plans array is
 * read during the call only; all plans must belong to the current device.
 * The graph holds every plan's segment tables.
 * Errors: FT_ERR_INVALID (NULL pointers, n_plans < 1, steps < 1, plans of
 * another device), FT_ERR_NOMEM, FT_ERR_HIP. */
int transfer_plans_capture(const ft_plan* const* plans, int n_plans, int steps, ft_graph** out);

/* Launch a captured graph on `stream`. */
int transfer_graph_launch(const ft_graph* graph, void* stream);

int destroy_transfer_graph(ft_graph* graph);

/* Read (and optionally reset) the operator's device count of skipped faces.
 * Synchronises the device; not for use inside graph capture. */
int transfer_operator_errors(const ft_operator* op, int64_t* n_skipped, int reset);

/* Message for the last failure on the calling thread ("" if none). */
const char* transfer_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int transfer_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FACETRANSFER_H */
