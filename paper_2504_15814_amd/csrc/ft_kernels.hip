// gfx950 kernels applying one face-transfer operator to a batch of hanging
// faces: one wave per (face, expansion anchor), 1..4 waves per block.  The
// per-item work lives in ft_device.h.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ft_device.h"
#include "ft_internal.h"
#include "ft_kernels.h"

namespace ft {

// Launch geometry for one call.
struct Geometry {
  int64_t n_faces;
  int anchors;  // expansion anchors per face, E * E
  int waves_per_block;
  int xcd_remap;  // block numbering, see logical_block (0, 1 or 2)
  int layout;     // kFaceBuffers or kPatches
};

template <int DIR, int R, int EC, int COPY, typename T, typename A, typename W, int DIM, typename TD>
__global__ __launch_bounds__(256) void apply_kernel(
    const DevOp* __restrict__ op, const Geometry geo, const int8_t* __restrict__ orientation,
    const int8_t* __restrict__ subface, const int64_t* __restrict__ src_offset,
    const int64_t* __restrict__ dst_offset, const int U, const T* __restrict__ src,
    const int64_t src_elems, TD* __restrict__ dst, const int64_t dst_elems,
    const W* __restrict__ weights, int* __restrict__ errors) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int E = EC > 0 ? EC : op->E;
  const int anchors = DIM == 3 ? E * E : E;
  // Launches are split on the host so that items fit in 31 bits.
  const int item = (int)logical_block(geo.xcd_remap) * geo.waves_per_block + wave;
  const int face = item / anchors;
  if (face >= geo.n_faces) return;
  apply_item<DIR, R, EC, COPY, T, A, W, DIM, TD>(op, face, item - face * anchors, geo.layout, orientation,
                                        subface, src_offset, dst_offset, U, src, src_elems, dst,
                                        dst_elems, weights, errors);
}

template <int DIR, int R, int EC, int COPY, typename T, typename A, typename W, int DIM = 3,
          typename TD = T>
static hipError_t launch_one(const ft_operator* op, const Geometry& g0, const LaunchArgs& la,
                             const W* weights, hipStream_t stream) {
  const int anchors = DIM == 3 ? op->E * op->E : op->E;
  // Split so that (faces in a launch) x anchors stays below 2^30.
  const int64_t chunk = ((int64_t)1 << 30) / anchors;
  for (int64_t f0 = 0; f0 < la.n_faces; f0 += chunk) {
    Geometry g = g0;
    g.n_faces = std::min<int64_t>(chunk, la.n_faces - f0);
    const int64_t items = g.n_faces * anchors;
    const int64_t blocks = (items + g.waves_per_block - 1) / g.waves_per_block;
    hipLaunchKernelGGL((apply_kernel<DIR, R, EC, COPY, T, A, W, DIM, TD>), dim3((unsigned)blocks),
                       dim3(64 * g.waves_per_block), 0, stream, op->d_devop, g, la.orientation + f0,
                       la.subface + f0, la.src_offset + f0, la.dst_offset + f0, la.U,
                       static_cast<const T*>(la.src), la.src_elems, static_cast<TD*>(la.dst),
                       la.dst_elems, weights, la.errors);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Dispatch on the compile-time anchor count (p = 6, 9, 12) or the generic form.
template <int DIR, int R, int COPY, typename T, typename A, typename W, typename TD = T>
static hipError_t launch_e(const ft_operator* op, const Geometry& g, const LaunchArgs& la,
                           const W* weights, hipStream_t stream) {
  switch (op->E) {
    case 2: return launch_one<DIR, R, 2, COPY, T, A, W, 3, TD>(op, g, la, weights, stream);
    case 3: return launch_one<DIR, R, 3, COPY, T, A, W, 3, TD>(op, g, la, weights, stream);
    case 4: return launch_one<DIR, R, 4, COPY, T, A, W, 3, TD>(op, g, la, weights, stream);
    default: return launch_one<DIR, R, 0, COPY, T, A, W, 3, TD>(op, g, la, weights, stream);
  }
}

// Interpolation accumulates in the storage precision (IA) with weights of
// that precision.
template <typename T, typename IA>
static hipError_t launch_interp_typed(const ft_operator* op, const Geometry& g,
                                      const LaunchArgs& la, hipStream_t stream) {
  const DevOp& d = op->dev;  // host copy: device pointers of the weight tables
  const IA* iw;
  if constexpr (sizeof(IA) == 8) iw = d.w64; else iw = d.w32;
  if (op->dim == 2) {
    // Two-dimensional faces: 3k rows per interpolation anchor.
    if (op->k == 1) return launch_one<0, 3, 0, -1, T, IA, IA, 2>(op, g, la, iw, stream);
    if (op->k == 2) return launch_one<0, 6, 0, 4, T, IA, IA, 2>(op, g, la, iw, stream);
    return launch_one<0, 9, 0, 4, T, IA, IA, 2>(op, g, la, iw, stream);
  }
  if (op->k == 1) return launch_e<0, 9, -1, T, IA, IA>(op, g, la, iw, stream);
  if (op->k == 2) return launch_e<0, 18, 13, T, IA, IA>(op, g, la, iw, stream);
  return launch_e<0, 27, 13, T, IA, IA>(op, g, la, iw, stream);
}

// Restriction sums always run in float64; fine data of type T, coarse of TD.
template <typename T, typename TD>
static hipError_t launch_restrict_typed(const ft_operator* op, const Geometry& g,
                                        const LaunchArgs& la, hipStream_t stream) {
  const double* w = op->dev.w64;
  const bool inject = op->copy_row == 0;
  if (op->dim == 2) {
    // Two-dimensional faces: k rows per restriction anchor.
    if (op->k == 1) return launch_one<1, 1, 0, -1, T, double, double, 2, TD>(op, g, la, w, stream);
    if (op->k == 2)
      return inject ? launch_one<1, 2, 0, 0, T, double, double, 2, TD>(op, g, la, w, stream)
                    : launch_one<1, 2, 0, -1, T, double, double, 2, TD>(op, g, la, w, stream);
    return inject ? launch_one<1, 3, 0, 0, T, double, double, 2, TD>(op, g, la, w, stream)
                  : launch_one<1, 3, 0, -1, T, double, double, 2, TD>(op, g, la, w, stream);
  }
  // k = 1: d-linear only, no injection row
  if (op->k == 1) return launch_e<1, 1, -1, T, double, double, TD>(op, g, la, w, stream);
  if (op->k == 2)
    return inject ? launch_e<1, 2, 0, T, double, double, TD>(op, g, la, w, stream)
                  : launch_e<1, 2, -1, T, double, double, TD>(op, g, la, w, stream);
  return inject ? launch_e<1, 3, 0, T, double, double, TD>(op, g, la, w, stream)
                : launch_e<1, 3, -1, T, double, double, TD>(op, g, la, w, stream);
}

// Few unknowns per cell: small_item with a wave-private LDS slice of
// xs_stride values of A (the anchor's weight block and its source values).
template <int DIR, int R, int COPY, typename T, typename A, typename W, int DIM, typename TD>
__global__ __launch_bounds__(256) void small_kernel(
    const DevOp* __restrict__ op, const Geometry geo, const int8_t* __restrict__ orientation,
    const int8_t* __restrict__ subface, const int64_t* __restrict__ src_offset,
    const int64_t* __restrict__ dst_offset, const int U, const T* __restrict__ src,
    const int64_t src_elems, TD* __restrict__ dst, const int64_t dst_elems,
    const W* __restrict__ weights, int* __restrict__ errors, const int xs_stride) {
  extern __shared__ double lds_words[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int anchors = geo.anchors;
  const int item = (int)logical_block(geo.xcd_remap) * geo.waves_per_block + wave;
  const int face = item / anchors;
  if (face >= geo.n_faces) return;
  A* xs = reinterpret_cast<A*>(lds_words) + wave * xs_stride;
  small_item<DIR, R, COPY, T, A, W, DIM, TD>(op, face, item - face * anchors, geo.layout,
                                             orientation, subface, src_offset, dst_offset, U, src,
                                             src_elems, dst, dst_elems, weights, errors, xs);
}

template <int DIR, int R, int COPY, typename T, typename A, typename W, int DIM = 3,
          typename TD = T>
static hipError_t launch_small_one(const ft_operator* op, const Geometry& g0, const LaunchArgs& la,
                                   const W* weights, hipStream_t stream) {
  int widest = 0;
  for (int c = 0; c < kClasses; ++c) widest = std::max(widest, op->blocks[c].width);
  const int xs_stride = widest * (R + la.U);  // weight block, then source values
  const size_t lds = (size_t)g0.waves_per_block * xs_stride * sizeof(A);
  if (lds > 65536) return hipErrorInvalidValue;  // beyond one workgroup's LDS
  const int anchors = g0.anchors;
  const int64_t chunk = ((int64_t)1 << 30) / anchors;
  for (int64_t f0 = 0; f0 < la.n_faces; f0 += chunk) {
    Geometry g = g0;
    g.n_faces = std::min<int64_t>(chunk, la.n_faces - f0);
    const int64_t blocks = (g.n_faces * anchors + g.waves_per_block - 1) / g.waves_per_block;
    hipLaunchKernelGGL((small_kernel<DIR, R, COPY, T, A, W, DIM, TD>), dim3((unsigned)blocks),
                       dim3(64 * g.waves_per_block), lds, stream, op->d_devop, g,
                       la.orientation + f0, la.subface + f0, la.src_offset + f0, la.dst_offset + f0,
                       la.U, static_cast<const T*>(la.src), la.src_elems, static_cast<TD*>(la.dst),
                       la.dst_elems, weights, la.errors, xs_stride);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T, typename IA>
static hipError_t launch_small_interp(const ft_operator* op, const Geometry& g,
                                      const LaunchArgs& la, hipStream_t stream) {
  const DevOp& d = op->dev;
  const IA* iw;
  if constexpr (sizeof(IA) == 8) iw = d.w64; else iw = d.w32;
  if (op->dim == 2) {
    if (op->k == 1) return launch_small_one<0, 3, -1, T, IA, IA, 2>(op, g, la, iw, stream);
    if (op->k == 2) return launch_small_one<0, 6, 4, T, IA, IA, 2>(op, g, la, iw, stream);
    return launch_small_one<0, 9, 4, T, IA, IA, 2>(op, g, la, iw, stream);
  }
  if (op->k == 1) return launch_small_one<0, 9, -1, T, IA, IA>(op, g, la, iw, stream);
  if (op->k == 2) return launch_small_one<0, 18, 13, T, IA, IA>(op, g, la, iw, stream);
  return launch_small_one<0, 27, 13, T, IA, IA>(op, g, la, iw, stream);
}

template <typename T, typename TD>
static hipError_t launch_small_restrict(const ft_operator* op, const Geometry& g,
                                        const LaunchArgs& la, hipStream_t stream) {
  const double* w = op->dev.w64;
  const bool inject = op->copy_row == 0;
  if (op->dim == 2) {
    if (op->k == 1) return launch_small_one<1, 1, -1, T, double, double, 2, TD>(op, g, la, w, stream);
    if (op->k == 2)
      return inject ? launch_small_one<1, 2, 0, T, double, double, 2, TD>(op, g, la, w, stream)
                    : launch_small_one<1, 2, -1, T, double, double, 2, TD>(op, g, la, w, stream);
    return inject ? launch_small_one<1, 3, 0, T, double, double, 2, TD>(op, g, la, w, stream)
                  : launch_small_one<1, 3, -1, T, double, double, 2, TD>(op, g, la, w, stream);
  }
  if (op->k == 1) return launch_small_one<1, 1, -1, T, double, double, 3, TD>(op, g, la, w, stream);
  if (op->k == 2)
    return inject ? launch_small_one<1, 2, 0, T, double, double, 3, TD>(op, g, la, w, stream)
                  : launch_small_one<1, 2, -1, T, double, double, 3, TD>(op, g, la, w, stream);
  return inject ? launch_small_one<1, 3, 0, T, double, double, 3, TD>(op, g, la, w, stream)
                : launch_small_one<1, 3, -1, T, double, double, 3, TD>(op, g, la, w, stream);
}

hipError_t launch_apply(const ft_operator* op, const LaunchArgs& la, const LaunchConfig& cfg,
                        hipStream_t stream) {
  if (cfg.waves_per_block < 1 || cfg.waves_per_block > 4) return hipErrorInvalidValue;
  Geometry g;
  g.n_faces = la.n_faces;
  g.anchors = op->dim == 3 ? op->E * op->E : op->E;
  g.waves_per_block = cfg.waves_per_block;
  // XCD-contiguous numbering: restriction 2.5 % faster, float64
  // interpolation unchanged (half the L2 misses), float32 interpolation 3-5 %
  // slower; there runs of four blocks per XCD (mode 2) cut the HBM reads from
  // 2.3x to 1.4x of the algorithmic bytes at the same speed.
  g.xcd_remap = (op->direction == FT_INTERPOLATE && la.dtype != FT_F64) ? 2 : cfg.xcd_remap;
  g.layout = la.layout;
  const bool small = la.U <= cfg.small_unknowns[op->direction];
  if (small) g.xcd_remap = cfg.xcd_remap;
  if (op->direction == FT_INTERPOLATE) {
    // FT_F64_TO_F32 is rejected for interpolation before any launch.
    if (la.dtype == FT_F64_TO_F32) return hipErrorInvalidValue;
    if (la.dtype == FT_F64)
      return small ? launch_small_interp<double, double>(op, g, la, stream)
                   : launch_interp_typed<double, double>(op, g, la, stream);
    // FT_F32 (and the split-bfloat16 modes at few unknowns): float32 storage.
    return small ? launch_small_interp<float, float>(op, g, la, stream)
                 : launch_interp_typed<float, float>(op, g, la, stream);
  }
  if (la.dtype == FT_F64)
    return small ? launch_small_restrict<double, double>(op, g, la, stream)
                 : launch_restrict_typed<double, double>(op, g, la, stream);
  if (la.dtype == FT_F64_TO_F32)
    return small ? launch_small_restrict<double, float>(op, g, la, stream)
                 : launch_restrict_typed<double, float>(op, g, la, stream);
  // Every float32 mode restricts float32 data with float64 sums.
  return small ? launch_small_restrict<float, float>(op, g, la, stream)
               : launch_restrict_typed<float, float>(op, g, la, stream);
}

}  // namespace ft
