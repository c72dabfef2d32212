// gfx950 kernels applying the face-transfer operators (Section 2 of Stokes et
// al., arXiv 2504.15814: the 1/9 segment of P or R per hanging face, the same
// operator for every unknown; Section 4.2: vectorise over the unknowns of the
// AoS halo).
//
// Work unit: one wave per (face, expansion anchor).  An anchor is one coarse
// column of the subface for interpolation (its k*9 fine ghost cells are the
// block's rows) or one coarse target column for restriction (its k layers are
// the rows).  The 64 lanes of the wave run over unknowns, so every operator
// weight is wave-uniform: the weights stream through the scalar cache into
// SGPRs and each loaded source value feeds R fused multiply-adds held in
// VGPR accumulators.  Source loads and destination stores are contiguous over
// the unknowns of a cell (AoS), i.e. coalesced.
//
// The rotation / mirroring onto the reference face (Section 4.1) is not
// materialised: each wave derives the physical strides of its face from the
// orientation and walks the reference-frame stencil through them.
#include <hip/hip_runtime.h>

#include "ft_internal.h"
#include "ft_kernels.h"

#include <algorithm>

namespace ft {

// Launch geometry for one call.
struct Geometry {
  int64_t n_faces;
  int anchors;  // expansion anchors per face, E * E
  int waves_per_block;
  int xcd_remap;  // 1: consecutive logical blocks land on one XCD
};

__device__ inline int64_t logical_block(int xcd_remap) {
  const int64_t b = blockIdx.x;
  if (!xcd_remap) return b;
  // Hardware dispatches block i to XCD i % 8.  Renumber so that each XCD
  // receives a contiguous range of logical blocks (neighbouring anchors of
  // one face then share that XCD's L2).
  const int64_t nb = gridDim.x;
  const int64_t per = nb / 8;
  const int64_t full = per * 8;
  if (b >= full) return b;
  return (b % 8) * per + b / 8;
}

// DIR 0: interpolation (src = coarse, dst = fine).  DIR 1: restriction
// (src = fine, dst = coarse).  R rows per anchor; EC anchors per axis (0 = read
// from the operator); COPY is the exact-copy row (its source is stencil entry
// 0 of every block) or -1.  T storage, A accumulator, W weight type.
template <int DIR, int R, int EC, int COPY, typename T, typename A, typename W>
__global__ __launch_bounds__(256) void apply_kernel(
    const DevOp op, const Geometry geo, const int8_t* __restrict__ orientation,
    const int8_t* __restrict__ subface, const int64_t* __restrict__ src_offset,
    const int64_t* __restrict__ dst_offset, const int U, const T* __restrict__ src,
    const int64_t src_elems, T* __restrict__ dst, const int64_t dst_elems,
    const W* __restrict__ weights, int* __restrict__ errors) {
  constexpr int kGroup = 4;  // stencil loads in flight per wave before their FMAs
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int E = EC > 0 ? EC : op.E;
  const int anchors = E * E;
  // Launches are split on the host so that items fit in 31 bits.
  const int item = (int)logical_block(geo.xcd_remap) * geo.waves_per_block + wave;
  const int face = item / anchors;
  if (face >= geo.n_faces) return;
  const int e = item - face * anchors;
  const int eb = e % E, ec = e / E;
  const int p = op.p, k = op.k;

  const int o = __builtin_amdgcn_readfirstlane((int)orientation[face]);
  const int s = __builtin_amdgcn_readfirstlane((int)subface[face]);
  const int64_t face_elems = (int64_t)(2 * k * p * p) * U;
  const int64_t so = src_offset[face];
  const int64_t dof = dst_offset[face];
  const bool bad = o < 0 || o > 5 || s < 0 || s > 8 || so < 0 || dof < 0 ||
                   so > src_elems - face_elems || dof > dst_elems - face_elems;
  if (bad) {
    if (e == 0 && lane == 0) atomicAdd(errors, 1);
    return;
  }
  const FaceStrides st = face_strides(o % 3, p, k);
  int nbase, nsign;
  normal_map(DIR, o, k, &nbase, &nsign);
  const int sb = s % 3, sc = s / 3;

  // Anchor column in the source buffer and the block that serves it.
  const int anc_b = DIR == 0 ? sb * E + eb : 3 * eb + 1;
  const int anc_c = DIR == 0 ? sc * E + ec : 3 * ec + 1;
  const int cls = axis_class(anc_b, p) * kAxisClasses + axis_class(anc_c, p);
  const int width = op.width[cls];
  const int start = op.start[cls];
  const int anchor_cell = anc_b * st.sb + anc_c * st.sc + nbase * st.sa;
  const int nstride = nsign * st.sa;
  // First destination cell of this anchor and the strides of its rows.
  const int dst_b = DIR == 0 ? 3 * eb : sb * E + eb;
  const int dst_c = DIR == 0 ? 3 * ec : sc * E + ec;
  const int dst_cell0 = nbase * st.sa + dst_b * st.sb + dst_c * st.sc;

  const T* __restrict__ sp = src + so;
  T* __restrict__ dp = dst + dof;
  const int* __restrict__ pts = op.stencil + start;
  const W* __restrict__ wts = weights + (int64_t)start * R;

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
        const int cell = anchor_cell + n * nstride + db * st.sb + dc * st.sc;
        x[j] = A(sp[(int64_t)cell * U + uu]);
      }
      if (COPY >= 0 && q == 0) copy_val = x[0];
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const W* __restrict__ w = wts + (q + j) * R;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (r != COPY) acc[r] = fma(A(w[r]), x[j], acc[r]);
      }
    }
    for (; q < width; ++q) {
      int n, db, dc;
      unpack_point(pts[q], &n, &db, &dc);
      const int cell = anchor_cell + n * nstride + db * st.sb + dc * st.sc;
      const A x = A(sp[(int64_t)cell * U + uu]);
      if (COPY >= 0 && q == 0) copy_val = x;
      const W* __restrict__ w = wts + q * R;
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r != COPY) acc[r] = fma(A(w[r]), x, acc[r]);
    }
    if (!act) continue;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int dcell;
      if (DIR == 0) {
        const int g = r / 9, tb = (r / 3) % 3, tc = r % 3;
        dcell = dst_cell0 + g * nstride + tb * st.sb + tc * st.sc;
      } else {
        dcell = dst_cell0 + r * nstride;
      }
      // Streaming (non-temporal) stores: the written halo is not re-read by
      // this launch, and keeping it out of L2 preserves the source
      // footprints that neighbouring anchors of the same face re-read.
      __builtin_nontemporal_store(T(r == COPY ? copy_val : acc[r]), &dp[(int64_t)dcell * U + u]);
    }
  }
}

template <int DIR, int R, int EC, int COPY, typename T, typename A, typename W>
static hipError_t launch_one(const DevOp& op, const Geometry& g0, const LaunchArgs& la,
                             const W* weights, hipStream_t stream) {
  const int anchors = op.E * op.E;
  // Split so that (faces in a launch) x anchors stays below 2^30.
  const int64_t chunk = ((int64_t)1 << 30) / anchors;
  for (int64_t f0 = 0; f0 < la.n_faces; f0 += chunk) {
    Geometry g = g0;
    g.n_faces = std::min<int64_t>(chunk, la.n_faces - f0);
    const int64_t items = g.n_faces * anchors;
    const int64_t blocks = (items + g.waves_per_block - 1) / g.waves_per_block;
    hipLaunchKernelGGL((apply_kernel<DIR, R, EC, COPY, T, A, W>), dim3((unsigned)blocks),
                       dim3(64 * g.waves_per_block), 0, stream, op, g, la.orientation + f0,
                       la.subface + f0, la.src_offset + f0, la.dst_offset + f0, la.U,
                       static_cast<const T*>(la.src), la.src_elems, static_cast<T*>(la.dst),
                       la.dst_elems, weights, la.errors);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Dispatch on the compile-time anchor count (p = 6, 9, 12) or the generic form.
template <int DIR, int R, int COPY, typename T, typename A, typename W>
static hipError_t launch_e(const DevOp& op, const Geometry& g, const LaunchArgs& la,
                           const W* weights, hipStream_t stream) {
  switch (op.E) {
    case 2: return launch_one<DIR, R, 2, COPY, T, A, W>(op, g, la, weights, stream);
    case 3: return launch_one<DIR, R, 3, COPY, T, A, W>(op, g, la, weights, stream);
    case 4: return launch_one<DIR, R, 4, COPY, T, A, W>(op, g, la, weights, stream);
    default: return launch_one<DIR, R, 0, COPY, T, A, W>(op, g, la, weights, stream);
  }
}

template <typename T, typename IA>
static hipError_t launch_typed(const ft_operator* op, const Geometry& g, const LaunchArgs& la,
                               hipStream_t stream) {
  const DevOp& d = op->dev;
  // Interpolation accumulates in the storage precision (IA) with weights of
  // that precision; restriction sums always run in float64.
  const IA* iw;
  if constexpr (sizeof(IA) == 8) iw = d.w64; else iw = d.w32;
  if (op->direction == FT_INTERPOLATE) {
    if (op->k == 2) return launch_e<0, 18, 13, T, IA, IA>(d, g, la, iw, stream);
    return launch_e<0, 27, 13, T, IA, IA>(d, g, la, iw, stream);
  }
  const bool inject = op->copy_row == 0;
  if (op->k == 2)
    return inject ? launch_e<1, 2, 0, T, double, double>(d, g, la, d.w64, stream)
                  : launch_e<1, 2, -1, T, double, double>(d, g, la, d.w64, stream);
  return inject ? launch_e<1, 3, 0, T, double, double>(d, g, la, d.w64, stream)
                : launch_e<1, 3, -1, T, double, double>(d, g, la, d.w64, stream);
}

hipError_t launch_apply(const ft_operator* op, const LaunchArgs& la, const LaunchConfig& cfg,
                        hipStream_t stream) {
  if (cfg.waves_per_block < 1 || cfg.waves_per_block > 4) return hipErrorInvalidValue;
  Geometry g;
  g.n_faces = la.n_faces;
  g.anchors = op->E * op->E;
  g.waves_per_block = cfg.waves_per_block;
  g.xcd_remap = cfg.xcd_remap;
  if (la.dtype == FT_F64) return launch_typed<double, double>(op, g, la, stream);
  // FT_F32 and (for restriction) the split-bfloat16 modes: float32 storage.
  return launch_typed<float, float>(op, g, la, stream);
}

}  // namespace ft
