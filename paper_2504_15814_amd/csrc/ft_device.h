// Device bodies of the transfer: one (face, expansion anchor) work item per
// wave.  Shared by the per-batch kernels and the fused plan kernel.
//
// apply_item: vector-ALU form (Section 2: the 1/9 segment of P or R per
// hanging face, the same operator for every unknown; Section 4.2: vectorise
// over the unknowns of the AoS halo).  The 64 lanes of the wave run over
// unknowns, so every operator weight is wave-uniform: the weights stream
// through the scalar cache into SGPRs and each loaded source value feeds R
// fused multiply-adds held in VGPR accumulators.  Source loads and
// destination stores are contiguous over the unknowns of a cell (AoS).  The
// rotation / mirroring onto the reference face (Section 4.1) is not
// materialised: the wave derives the physical strides of its face from the
// orientation and walks the reference-frame stencil through them.
//
// mfma_item: float32 interpolation on the matrix cores.  Per anchor the
// operator application is a small dense contraction Y (rows x unknowns) =
// W (rows x stencil) . X (stencil x unknowns) (Section 6 suggests block
// formats so that GEMM-type kernels apply), computed with
// v_mfma_f32_32x32x16_bf16: M = the <= 27 fine rows of the anchor (padded to
// 32), N = 32 unknowns per tile, K = 16 stencil points per step.  Float32 data
// and the operator are split into bfloat16 parts (x = x0 + x1 + x2 exactly,
// W = W0 + W1 + W2) and W0x0 + W0x1 + W1x0 (3 terms) or also W0x2 + W1x1 +
// W2x0 (6 terms, compensating the split residuals) are accumulated in
// float32.  The exact-copy row is written from the source value itself.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "ft_internal.h"

namespace ft {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Read-only data reached through pointers that were themselves read from
// memory (an operator view, its tables, a plan's descriptor arrays) is
// accessed through the constant address space: wave-uniform reads then go
// through the scalar cache (s_load) instead of per-lane flat loads.
#define FT_CONST __attribute__((address_space(4)))
template <typename P>
__device__ __forceinline__ const FT_CONST P* cptr(const P* p) {
  return (const FT_CONST P*)p;
}

// Logical block number.  Hardware dispatches block i to XCD i % 8.
// xcd_remap 1: each XCD receives a contiguous range of logical blocks, so
// neighbouring anchors of one face share that XCD's L2.  xcd_remap 2: each
// XCD receives runs of kXcdRun consecutive logical blocks (16 anchors with
// four waves per block), so the anchors of a face mostly share one L2 while
// the eight XCDs work on neighbouring faces at any time.
constexpr int kXcdRun = 4;
__device__ inline int64_t logical_block(int xcd_remap) {
  const int64_t b = blockIdx.x;
  if (!xcd_remap) return b;
  if (xcd_remap == 2) {
    const int64_t full = gridDim.x / (8 * kXcdRun) * (8 * kXcdRun);
    if (b >= full) return b;
    const int64_t j = b / 8;  // the j-th block dispatched to XCD b % 8
    return (j / kXcdRun) * (8 * kXcdRun) + (b % 8) * kXcdRun + j % kXcdRun;
  }
  const int64_t nb = gridDim.x;
  const int64_t per = nb / 8;
  const int64_t full = per * 8;
  if (b >= full) return b;
  return (b % 8) * per + b / 8;
}

// Geometry of one (face, anchor) work item: where its stencil cells and its
// destination rows live.  Returns false when the item has nothing to do: a
// bad descriptor (counted once per face) or, with p not a multiple of 3, an
// anchor of the E x E grid that holds no column of this subface.  With p not
// a multiple of 3 some interpolation rows also belong to the neighbouring
// fine face (not stored; see `full`).
struct ItemGeom {
  int64_t so, dof;         // element offsets of the source / destination face or patch
  int anchor_cell;         // source cell of the anchor at normal coordinate 0
  int nstride, sb, sc;     // source strides: normal (signed), tangential b and c
  int dst_cell0, dstride;  // destination cell of row 0, signed normal stride
  int db, dc;              // destination tangential strides
  int dst_b, dst_c;        // destination column of row tb = tc = 0
  int cls, width, start;   // anchor class and its weight block
  int axis;                // normal axis of the face
};

template <int DIR, int EC, int DIM>
__device__ __forceinline__ bool item_geometry(
    const FT_CONST DevOp* op, const int face, const int e, const int layout,
    const FT_CONST int8_t* orientation, const FT_CONST int8_t* subface,
    const FT_CONST int64_t* src_offset, const FT_CONST int64_t* dst_offset, const int U,
    const int64_t src_elems, const int64_t dst_elems, int* __restrict__ errors, ItemGeom* g) {
  const int lane = threadIdx.x & 63;
  const int E = EC > 0 ? EC : op->E;
  const int eb = DIM == 3 ? e % E : e, ec = DIM == 3 ? e / E : 0;
  const int p = op->p, k = op->k;

  const int o = __builtin_amdgcn_readfirstlane((int)orientation[face]);
  const int s = __builtin_amdgcn_readfirstlane((int)subface[face]);
  // Elements one item may touch: a face buffer, or a whole patch box.
  const int P = p + 2 * k;
  const int64_t item_elems =
      (layout == kFaceBuffers ? (int64_t)(2 * k * p) * (DIM == 3 ? p : 1) : (int64_t)P * P * P) *
      U;
  const int64_t so = src_offset[face];
  const int64_t dof = dst_offset[face];
  const bool bad = o < 0 || o > (DIM == 3 ? 5 : 3) || s < 0 || s > (DIM == 3 ? 8 : 2) || so < 0 ||
                   dof < 0 || so > src_elems - item_elems || dof > dst_elems - item_elems;
  if (bad) {
    if (e == 0 && lane == 0) atomicAdd(errors, 1);
    return false;
  }
  FaceView sv, dv;
  if (DIM == 3)
    transfer_views(DIR, layout, o, p, k, &sv, &dv);
  else
    sv = dv = buffer_view2d(o % 2, p, k);
  int nbase, nsign;
  normal_map_side(DIR, o < (DIM == 3 ? 3 : 2), k, &nbase, &nsign);
  const int sb = DIM == 3 ? s % 3 : s, sc = DIM == 3 ? s / 3 : 0;

  // Anchor columns in the source face (anc) and first destination columns
  // (dst: the fine column of row tb = 0, or the coarse target column).
  int anc_b, anc_c = 0, dst_b, dst_c = 0;
  if (DIR == 0) {
    anc_b = interp_anchor0(sb, p) + eb;
    dst_b = 3 * anc_b - sb * p;
    if (DIM == 3) {
      anc_c = interp_anchor0(sc, p) + ec;
      dst_c = 3 * anc_c - sc * p;
    }
    if (!interp_anchor_valid(anc_b, sb, p) || (DIM == 3 && !interp_anchor_valid(anc_c, sc, p)))
      return false;
  } else {
    dst_b = restrict_anchor0(sb, p) + eb;
    anc_b = 3 * dst_b + 1 - sb * p;
    if (DIM == 3) {
      dst_c = restrict_anchor0(sc, p) + ec;
      anc_c = 3 * dst_c + 1 - sc * p;
    }
    if (!restrict_anchor_valid(dst_b, sb, p) || (DIM == 3 && !restrict_anchor_valid(dst_c, sc, p)))
      return false;
  }
  const int cls = axis_class(anc_b, p) * kAxisClasses + (DIM == 3 ? axis_class(anc_c, p) : 0);
  g->so = so;
  g->dof = dof;
  g->cls = cls;
  g->width = op->width[cls];
  g->start = op->start[cls];
  g->anchor_cell = sv.base + anc_b * sv.sb + anc_c * sv.sc + nbase * sv.sa;
  g->nstride = nsign * sv.sa;
  g->sb = sv.sb;
  g->sc = sv.sc;
  g->dst_cell0 = dv.base + nbase * dv.sa + dst_b * dv.sb + dst_c * dv.sc;
  g->dstride = nsign * dv.sa;
  g->db = dv.sb;
  g->dc = dv.sc;
  g->dst_b = dst_b;
  g->dst_c = dst_c;
  g->axis = DIM == 3 ? o % 3 : o % 2;
  return true;
}

// Destination cell of row r of an item, and whether the row is this fine
// face's (interpolation with p not a multiple of 3 has rows of the
// neighbouring fine face at the subface edges).
template <int DIR, int DIM>
__device__ __forceinline__ int row_cell(const ItemGeom& g, const int r, const int p, bool* mine) {
  if (DIR == 0) {
    const int gl = DIM == 3 ? r / 9 : r / 3, tb = DIM == 3 ? (r / 3) % 3 : r % 3;
    const int tc = DIM == 3 ? r % 3 : 0;
    *mine = (unsigned)(g.dst_b + tb) < (unsigned)p &&
            (DIM == 2 || (unsigned)(g.dst_c + tc) < (unsigned)p);
    return g.dst_cell0 + gl * g.dstride + tb * g.db + tc * g.dc;
  }
  *mine = true;
  return g.dst_cell0 + r * g.dstride;
}

// Interpolation rows are r = g * 9 + tb * 3 + tc (normal layer g, tangential
// offsets tb, tc).  store_row<R, X>(i) is the row stored i-th, so that
// consecutive stores go to adjacent cells: with X = 0 layer by layer, the
// three cells along b back to back (b is axis 0, adjacent in memory, when
// the normal is axis 1 or 2); with X = 1, for faces whose normal is axis 0,
// the k layers of one column back to back.  Against row order, float64
// interpolation 3-7 % and float32 4-10 % faster (same-machine A/B); one order per
// normal axis, three store sequences, was slower than these two.
template <int R, int X>
__device__ __forceinline__ constexpr int store_row(const int i) {
  if (R % 9 != 0) return i;
  constexpr int G = R / 9;
  if (X) return (i % G) * 9 + ((i / G) % 3) * 3 + i / (3 * G);  // tc, tb, g fastest
  return (i / 9) * 9 + (i % 3) * 3 + (i / 3) % 3;               // g, tc, tb fastest
}

// DIR 0: interpolation (src = coarse, dst = fine).  DIR 1: restriction
// (src = fine, dst = coarse).  R rows per anchor; EC anchors per axis (0 = read
// from the operator); COPY is the exact-copy row (its source is stencil entry
// 0 of every block) or -1.  T source storage, A accumulator, W weight type,
// TD destination storage (float32 for restriction of float64 fine data into
// float32 coarse faces, else T).
// DIM 3, or 2 for two-dimensional faces (2k x p cells; no third axis, the
// anchor index e runs over the p/3 coarse columns of the subface).
template <int DIR, int R, int EC, int COPY, typename T, typename A, typename W, int DIM = 3,
          typename TD = T>
__device__ __forceinline__ void apply_item(
    const DevOp* __restrict__ op_, const int face, const int e, const int layout,
    const int8_t* __restrict__ orientation_, const int8_t* __restrict__ subface_,
    const int64_t* __restrict__ src_offset_, const int64_t* __restrict__ dst_offset_, const int U,
    const T* __restrict__ src, const int64_t src_elems, TD* __restrict__ dst,
    const int64_t dst_elems, const W* __restrict__ weights_, int* __restrict__ errors) {
  const FT_CONST DevOp* op = cptr(op_);
  const FT_CONST int8_t* orientation = cptr(orientation_);
  const FT_CONST int8_t* subface = cptr(subface_);
  const FT_CONST int64_t* src_offset = cptr(src_offset_);
  const FT_CONST int64_t* dst_offset = cptr(dst_offset_);
  const FT_CONST W* weights = cptr(weights_);
  // Stencil loads in flight per wave before their FMAs: eight in float32
  // (interpolation 4-7 % faster), four in float64 (eight no faster).
  constexpr int kGroup = sizeof(A) == 4 ? 8 : 4;
  const int lane = threadIdx.x & 63;
  const int p = op->p;
  ItemGeom g;
  if (!item_geometry<DIR, EC, DIM>(op, face, e, layout, orientation, subface, src_offset,
                                   dst_offset, U, src_elems, dst_elems, errors, &g))
    return;
  const int width = g.width;
  const int anchor_cell = g.anchor_cell;
  const int nstride = g.nstride;
  const int dst_b = g.dst_b, dst_c = g.dst_c;

  const T* __restrict__ sp = src + g.so;
  TD* __restrict__ dp = dst + g.dof;
  const FT_CONST int* pts = cptr(op->stencil) + g.start;
  const FT_CONST W* wts = weights + (int64_t)g.start * R;

  for (int u0 = 0; u0 < U; u0 += 64) {
    const int u = u0 + lane;
    const bool act = u < U;
    const int uu = act ? u : U - 1;  // idle lanes re-read a valid element
    A acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = A(0);
    A copy_val = A(0);
    int q = 0;
    for (; q + kGroup <= width; q += kGroup) {
      A x[kGroup];
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        int n, db, dc;
        unpack_point(pts[q + j], &n, &db, &dc);
        const int cell = anchor_cell + n * nstride + db * g.sb + dc * g.sc;
        x[j] = A(sp[(int64_t)cell * U + uu]);
      }
      if (COPY >= 0 && q == 0) copy_val = x[0];
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const FT_CONST W* w = wts + (q + j) * R;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (r != COPY) acc[r] = fma(A(w[r]), x[j], acc[r]);
      }
    }
    for (; q < width; ++q) {
      int n, db, dc;
      unpack_point(pts[q], &n, &db, &dc);
      const int cell = anchor_cell + n * nstride + db * g.sb + dc * g.sc;
      const A x = A(sp[(int64_t)cell * U + uu]);
      if (COPY >= 0 && q == 0) copy_val = x;
      const FT_CONST W* w = wts + q * R;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r != COPY) acc[r] = fma(A(w[r]), x, acc[r]);
    }
    if (!act) continue;
    // Interpolation anchors whose fine cells all belong to this fine face
    // (every anchor when 3 divides p) store straight through; the others skip
    // the cells of the neighbouring fine face.
    const bool full =
        DIR == 1 || (dst_b >= 0 && dst_b + 2 < p && (DIM == 2 || (dst_c >= 0 && dst_c + 2 < p)));
    auto store_rows = [&](auto check, auto xo) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int r = DIR == 0 && DIM == 3 ? store_row<R, decltype(xo)::value>(i) : i;
        bool mine;
        const int dcell = row_cell<DIR, DIM>(g, r, p, &mine);
        if (decltype(check)::value && !mine) continue;
        // Streaming (non-temporal) stores: the written halo is not re-read by
        // this launch.
        __builtin_nontemporal_store(TD(r == COPY ? copy_val : acc[r]), &dp[(int64_t)dcell * U + u]);
      }
    };
    if (DIR == 0 && DIM == 3 && g.axis == 0) {
      if (full)
        store_rows(std::false_type{}, std::integral_constant<int, 1>{});
      else
        store_rows(std::true_type{}, std::integral_constant<int, 1>{});
    } else {
      if (full)
        store_rows(std::false_type{}, std::integral_constant<int, 0>{});
      else
        store_rows(std::true_type{}, std::integral_constant<int, 0>{});
    }
  }
}

// Order this wave's LDS writes before its reads of what other lanes wrote
// (the slice is private to the wave, so no block barrier is needed).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Copy n values into LDS, lanes over the values, eight loads in flight per
// lane before their LDS writes.
template <typename A, typename Load>
__device__ __forceinline__ void stage_lds(A* __restrict__ to, const int n, const int lane,
                                          Load load) {
  constexpr int kBatch = 8;
  for (int j0 = 0; j0 < n; j0 += 64 * kBatch) {
    A v[kBatch];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int j = j0 + 64 * i + lane;
      v[i] = j < n ? load(j) : A(0);
    }
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int j = j0 + 64 * i + lane;
      if (j < n) to[j] = v[i];
    }
  }
}

// Few unknowns per cell (Section 6: for PDEs with few unknowns the
// application strategy decides the speed): with lanes over unknowns most of
// the wave would idle and every load and store would move a few bytes.
// Here the anchor's weight block (width x R, contiguous) and all its
// (stencil point, unknown) source values are loaded at once, lanes over the
// values, into the wave's LDS slice: ws[q * R + r], then xs[q * U + u].
// Then lanes run over (row, unknown) outputs and each sums its row over the
// stencil in stencil order: the same fused multiply-add chain as
// apply_item, so both bodies give bitwise equal results.  The slice holds
// width * (R + U) values of A.  Types as for apply_item.
template <int DIR, int R, int COPY, typename T, typename A, typename W, int DIM = 3,
          typename TD = T>
__device__ __forceinline__ void small_item(
    const DevOp* __restrict__ op_, const int face, const int e, const int layout,
    const int8_t* __restrict__ orientation_, const int8_t* __restrict__ subface_,
    const int64_t* __restrict__ src_offset_, const int64_t* __restrict__ dst_offset_, const int U,
    const T* __restrict__ src, const int64_t src_elems, TD* __restrict__ dst,
    const int64_t dst_elems, const W* __restrict__ weights, int* __restrict__ errors,
    A* __restrict__ slice) {
  const FT_CONST DevOp* op = cptr(op_);
  const int lane = threadIdx.x & 63;
  const int p = op->p;
  ItemGeom g;
  if (!item_geometry<DIR, 0, DIM>(op, face, e, layout, cptr(orientation_), cptr(subface_),
                                  cptr(src_offset_), cptr(dst_offset_), U, src_elems, dst_elems,
                                  errors, &g))
    return;
  const T* __restrict__ sp = src + g.so;
  TD* __restrict__ dp = dst + g.dof;
  const int* __restrict__ pts = op_->stencil + g.start;
  const W* __restrict__ wts = weights + (int64_t)g.start * R;
  const int width = g.width;
  A* __restrict__ ws = slice;
  A* __restrict__ xs = slice + width * R;

  stage_lds(ws, width * R, lane, [&](int j) { return A(wts[j]); });
  stage_lds(xs, width * U, lane, [&](int j) {
    const int q = j / U, u = j - q * U;
    int n, db, dc;
    unpack_point(pts[q], &n, &db, &dc);
    const int cell = g.anchor_cell + n * g.nstride + db * g.sb + dc * g.sc;
    return A(sp[(int64_t)cell * U + u]);
  });
  wave_lds_sync();
  const int n_out = R * U;
  for (int o = lane; o < n_out; o += 64) {
    const int r = o / U, u = o - r * U;
    bool mine;
    const int dcell = row_cell<DIR, DIM>(g, r, p, &mine);
    A acc = A(0);
    if (r == COPY) {
      acc = xs[u];  // the exact copy of stencil entry 0
    } else {
      for (int q = 0; q < width; ++q) acc = fma(ws[q * R + r], xs[q * U + u], acc);
    }
    if (mine) __builtin_nontemporal_store(TD(acc), &dp[(int64_t)dcell * U + u]);
  }
}

// Float32 interpolation on the matrix cores (see the file comment).
template <int R, int EC, int TERMS, int DIM = 3>
__device__ __forceinline__ void mfma_item(
    const DevOp* __restrict__ op_, const int face, const int e, const int layout,
    const int8_t* __restrict__ orientation_,
    const int8_t* __restrict__ subface_, const int64_t* __restrict__ src_offset_,
    const int64_t* __restrict__ dst_offset_, const int U, const float* __restrict__ src,
    const int64_t src_elems, float* __restrict__ dst, const int64_t dst_elems,
    int* __restrict__ errors) {
  const FT_CONST DevOp* op = cptr(op_);
  const FT_CONST int8_t* orientation = cptr(orientation_);
  const FT_CONST int8_t* subface = cptr(subface_);
  const FT_CONST int64_t* src_offset = cptr(src_offset_);
  const FT_CONST int64_t* dst_offset = cptr(dst_offset_);
  // Row (g, tb, tc) = (1, 1, 1) (3D, R >= 18) or (g, tb) = (1, 1) (2D, R >= 6) is
  // the coarse centre itself when k >= 2; with k = 1 no row is a copy.
  constexpr int COPY = DIM == 3 ? (R >= 18 ? 13 : -1) : (R >= 6 ? 4 : -1);
  const int lane = threadIdx.x & 63;
  const int p = op->p;
  ItemGeom g;
  if (!item_geometry<0, EC, DIM>(op, face, e, layout, orientation, subface, src_offset,
                                 dst_offset, U, src_elems, dst_elems, errors, &g))
    return;
  const int cls = g.cls;
  const int width = g.width;
  const int start = g.start;
  const int nsteps = (width + kMfmaK - 1) / kMfmaK;
  const int anchor_cell = g.anchor_cell;
  const int nstride = g.nstride;
  const int dst_b = g.dst_b, dst_c = g.dst_c;

  const FT_CONST bf16x8* wt = cptr(reinterpret_cast<const bf16x8*>(op->wbf16));
  const FT_CONST int* pts = cptr(op->stencil) + start;
  int copy_cell = anchor_cell;
  if (COPY >= 0) {
    int n, db, dc;
    unpack_point(pts[0], &n, &db, &dc);  // the copy source is entry 0
    copy_cell = anchor_cell + n * nstride + db * g.sb + dc * g.sc;
  }

  const float* __restrict__ sp = src + g.so;
  float* __restrict__ dp = dst + g.dof;
  for (int u0 = 0; u0 < U; u0 += 64) {
    // Lanes run over 64 unknowns: every stencil cell is one coalesced load.
    // The B operands of the two 32-unknown tiles are then formed in
    // registers: for a k-step (16 stencil points) each lane packs its 8 + 8
    // bfloat16 values, and v_permlane32_swap exchanges the upper half-wave of
    // the first 8 with the lower half-wave of the second 8, which yields
    // B[8h + i][col] in lane 32 h + col for unknowns u0 + col (tile 0) and
    // u0 + 32 + col (tile 1).
    const int uu = min(u0 + lane, U - 1);
    f32x16 acc0 = {}, acc1 = {};
    for (int st_i = 0; st_i < nsteps; ++st_i) {
      const bf16x8 w0 = wt[mfma_a_index(cls, st_i, 0, lane) / 8];
      const bf16x8 w1 = wt[mfma_a_index(cls, st_i, 1, lane) / 8];
      bf16x8 w2;
      if (TERMS == 6) w2 = wt[mfma_a_index(cls, st_i, 2, lane) / 8];
      float x[kMfmaK];
#pragma unroll
      for (int j = 0; j < kMfmaK; ++j) {
        const int q = kMfmaK * st_i + j;
        x[j] = 0.0f;
        if (q < width) {
          int n, db, dc;
          unpack_point(pts[q], &n, &db, &dc);
          const int cell = anchor_cell + n * nstride + db * g.sb + dc * g.sc;
          x[j] = sp[(int64_t)cell * U + uu];
        }
      }
      // Split x = x0 + x1 + x2 (bfloat16 parts), packed per 8 stencil points.
      bf16x8 p0[2], p1[2], p2[2];
#pragma unroll
      for (int j = 0; j < kMfmaK; ++j) {
        const __bf16 a0 = (__bf16)x[j];
        const float r1 = x[j] - (float)a0;
        const __bf16 a1 = (__bf16)r1;
        p0[j / 8][j % 8] = a0;
        p1[j / 8][j % 8] = a1;
        if (TERMS == 6) p2[j / 8][j % 8] = (__bf16)(r1 - (float)a1);
      }
      auto to_tiles = [](bf16x8 lo, bf16x8 hi, bf16x8* t0, bf16x8* t1) {
        u32x4 a = __builtin_bit_cast(u32x4, lo), b = __builtin_bit_cast(u32x4, hi);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const auto sw = __builtin_amdgcn_permlane32_swap(a[r], b[r], false, false);
          a[r] = sw[0];
          b[r] = sw[1];
        }
        *t0 = __builtin_bit_cast(bf16x8, a);
        *t1 = __builtin_bit_cast(bf16x8, b);
      };
      bf16x8 b0a, b0b, b1a, b1b, b2a, b2b;
      to_tiles(p0[0], p0[1], &b0a, &b0b);
      to_tiles(p1[0], p1[1], &b1a, &b1b);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, b0a, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, b0b, acc1, 0, 0, 0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, b1a, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, b1b, acc1, 0, 0, 0);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, b0a, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, b0b, acc1, 0, 0, 0);
      if (TERMS == 6) {
        to_tiles(p2[0], p2[1], &b2a, &b2b);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, b2a, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, b2b, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, b1a, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, b1b, acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2, b0a, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w2, b0b, acc1, 0, 0, 0);
      }
    }
    // In lane 32 h + col, accumulator v of tile t holds row 8 (v / 4) + 4 h +
    // v % 4 for unknown u0 + 32 t + col.  v_permlane32_swap of (acc0[v], acc1[v]) leaves the
    // h = 0 row in the first result and the h = 1 row in the second, each with
    // lanes over the 64 unknowns u0 + lane: whole cells, without LDS.
    float rows[32];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int m = 8 * (v / 4) + (v % 4);
      const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(acc0[v]),
                                                       __float_as_uint(acc1[v]), false, false);
      rows[m] = __uint_as_float(sw[0]);
      rows[m + 4] = __uint_as_float(sw[1]);
    }
    const int u = u0 + lane;
    if (u < U) {
      const float xc = COPY >= 0 ? sp[(int64_t)copy_cell * U + u] : 0.0f;
      // Anchors whose fine cells all belong to this fine face (every anchor
      // when 3 divides p) store straight through; the others skip the cells
      // of the neighbouring fine face.
      const bool full = dst_b >= 0 && dst_b + 2 < p && (DIM == 2 || (dst_c >= 0 && dst_c + 2 < p));
      auto store_rows = [&](auto check, auto xo) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int m = DIM == 3 ? store_row<R, decltype(xo)::value>(i) : i;
          bool mine;
          const int dcell = row_cell<0, DIM>(g, m, p, &mine);
          if (decltype(check)::value && !mine) continue;
          __builtin_nontemporal_store(m == COPY ? xc : rows[m], &dp[(int64_t)dcell * U + u]);
        }
      };
      if (DIM == 3 && g.axis == 0) {
        if (full)
          store_rows(std::false_type{}, std::integral_constant<int, 1>{});
        else
          store_rows(std::true_type{}, std::integral_constant<int, 1>{});
      } else {
        if (full)
          store_rows(std::false_type{}, std::integral_constant<int, 0>{});
        else
          store_rows(std::true_type{}, std::integral_constant<int, 0>{});
      }
    }
  }
}

}  // namespace ft
