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
// (src = fine, dst = coarse).  R rows per anchor.  T storage, A accumulator,
// W weight type.
template <int DIR, int R, typename T, typename A, typename W>
__global__ __launch_bounds__(1024) void apply_kernel(
    const DevOp op, const Geometry geo, const int8_t* __restrict__ orientation,
    const int8_t* __restrict__ subface, const int64_t* __restrict__ src_offset,
    const int64_t* __restrict__ dst_offset, const int U, const T* __restrict__ src,
    const int64_t src_elems, T* __restrict__ dst, const int64_t dst_elems,
    const W* __restrict__ weights, int* __restrict__ errors) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t item = logical_block(geo.xcd_remap) * geo.waves_per_block + wave;
  const int64_t face = item / geo.anchors;
  if (face >= geo.n_faces) return;
  const int e = (int)(item - face * geo.anchors);
  const int E = op.E;
  const int eb = e % E, ec = e / E;
  const int p = op.p, k = op.k;

  const int o = __builtin_amdgcn_readfirstlane((int)orientation[face]);
  const int s = __builtin_amdgcn_readfirstlane((int)subface[face]);
  const int64_t ncell = 2LL * k * p * p;
  const int64_t face_elems = ncell * U;
  const int64_t so = src_offset[face];
  const int64_t dof = dst_offset[face];
  const bool bad = o < 0 || o > 5 || s < 0 || s > 8 || so < 0 || dof < 0 ||
                   so + face_elems > src_elems || dof + face_elems > dst_elems;
  if (bad) {
    if (e == 0 && lane == 0) atomicAdd(errors, 1);
    return;
  }
  const int a = o % 3;
  const FaceStrides st = face_strides(a, p, k);
  int nbase, nsign;
  normal_map(DIR, o, k, &nbase, &nsign);
  const int sb = s % 3, sc = s / 3;

  // Anchor column in the source buffer and the block that serves it.
  int anc_b, anc_c;
  if (DIR == 0) {
    anc_b = sb * E + eb;  // containing coarse column
    anc_c = sc * E + ec;
  } else {
    anc_b = 3 * eb + 1;  // fine column coincident with the coarse centre
    anc_c = 3 * ec + 1;
  }
  const int cls = axis_class(anc_b, p) * kAxisClasses + axis_class(anc_c, p);
  const int width = op.width[cls];
  const int start = op.start[cls];
  const int anchor_cell = anc_b * st.sb + anc_c * st.sc;

  const T* __restrict__ sp = src + so;
  T* __restrict__ dp = dst + dof;

  for (int u0 = 0; u0 < U; u0 += 64) {
    const int u = u0 + lane;
    const bool act = u < U;
    const int uu = act ? u : U - 1;  // idle lanes re-read a valid element
    A acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = A(0);
    // Stencil points in groups of kGroup: all loads of a group are issued
    // before its multiply-adds, keeping several cache lines in flight per
    // wave.  The per-output summation order is the stencil order either way.
    constexpr int kGroup = 8;
    int q = 0;
    for (; q + kGroup <= width; q += kGroup) {
      A x[kGroup];
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        int n, db, dc;
        unpack_point(op.stencil[start + q + j], &n, &db, &dc);
        const int cell = anchor_cell + (nbase + nsign * n) * st.sa + db * st.sb + dc * st.sc;
        x[j] = A(sp[(int64_t)cell * U + uu]);
      }
#pragma unroll
      for (int j = 0; j < kGroup; ++j) {
        const W* __restrict__ w = weights + (int64_t)(start + q + j) * R;
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = fma(A(w[r]), x[j], acc[r]);
      }
    }
    for (; q < width; ++q) {
      int n, db, dc;
      unpack_point(op.stencil[start + q], &n, &db, &dc);
      const int cell = anchor_cell + (nbase + nsign * n) * st.sa + db * st.sb + dc * st.sc;
      const A x = A(sp[(int64_t)cell * U + uu]);
      const W* __restrict__ w = weights + (int64_t)(start + q) * R;
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = fma(A(w[r]), x, acc[r]);
    }
    if (!act) continue;
    // Exact copy row (coinciding centres): the source value itself.
    T copy_val = T(0);
    if (op.copy_row >= 0) {
      const int cell = anchor_cell + (nbase + nsign * op.copy_n) * st.sa;
      copy_val = sp[(int64_t)cell * U + u];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int dcell;
      if (DIR == 0) {
        const int g = r / 9, tb = (r / 3) % 3, tc = r % 3;
        dcell = (nbase + nsign * g) * st.sa + (3 * eb + tb) * st.sb + (3 * ec + tc) * st.sc;
      } else {
        dcell = (nbase + nsign * r) * st.sa + (sb * E + eb) * st.sb + (sc * E + ec) * st.sc;
      }
      const T val = (r == op.copy_row) ? copy_val : T(acc[r]);
      dp[(int64_t)dcell * U + u] = val;
    }
  }
}

template <int DIR, int R, typename T, typename A, typename W>
static hipError_t launch_one(const DevOp& op, const Geometry& g, const LaunchArgs& la,
                             const W* weights, hipStream_t stream) {
  const int64_t items = g.n_faces * g.anchors;
  const int64_t blocks = (items + g.waves_per_block - 1) / g.waves_per_block;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((apply_kernel<DIR, R, T, A, W>), dim3((unsigned)blocks),
                     dim3(64 * g.waves_per_block), 0, stream, op, g, la.orientation, la.subface,
                     la.src_offset, la.dst_offset, la.U, static_cast<const T*>(la.src),
                     la.src_elems, static_cast<T*>(la.dst), la.dst_elems, weights, la.errors);
  return hipGetLastError();
}

hipError_t launch_apply(const ft_operator* op, const LaunchArgs& la, const LaunchConfig& cfg,
                        hipStream_t stream) {
  Geometry g;
  g.n_faces = la.n_faces;
  g.anchors = op->E * op->E;
  g.waves_per_block = cfg.waves_per_block;
  g.xcd_remap = cfg.xcd_remap;
  const DevOp& d = op->dev;
  const bool f64 = la.dtype == FT_F64;
  if (op->direction == FT_INTERPOLATE) {
    if (op->k == 2)
      return f64 ? launch_one<0, 18, double, double, double>(d, g, la, d.w64, stream)
                 : launch_one<0, 18, float, float, float>(d, g, la, d.w32, stream);
    return f64 ? launch_one<0, 27, double, double, double>(d, g, la, d.w64, stream)
               : launch_one<0, 27, float, float, float>(d, g, la, d.w32, stream);
  }
  // Restriction sums stay in float64 for both storage types.
  if (op->k == 2)
    return f64 ? launch_one<1, 2, double, double, double>(d, g, la, d.w64, stream)
               : launch_one<1, 2, float, double, double>(d, g, la, d.w64, stream);
  return f64 ? launch_one<1, 3, double, double, double>(d, g, la, d.w64, stream)
             : launch_one<1, 3, float, double, double>(d, g, la, d.w64, stream);
}

}  // namespace ft
