// Launch interface between the C ABI and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "ft_internal.h"

// Largest unknown count per cell that runs the small-U body: interpolation
// (27 rows per anchor; the body's two LDS reads per product bound it above
// this) and restriction (3 rows).
#ifndef FT_SMALL_UNKNOWNS_INTERP
#define FT_SMALL_UNKNOWNS_INTERP 8
#endif
#ifndef FT_SMALL_UNKNOWNS_RESTRICT
#define FT_SMALL_UNKNOWNS_RESTRICT 16
#endif

namespace ft {

struct LaunchArgs {
  int64_t n_faces;
  const int8_t* orientation;
  const int8_t* subface;
  const int64_t* src_offset;
  const int64_t* dst_offset;
  int U;
  int dtype;
  const void* src;
  int64_t src_elems;
  void* dst;
  int64_t dst_elems;
  int* errors;
  int layout = kFaceBuffers;  // kFaceBuffers or kPatches
};

// Tunable launch shape (schedules never change the per-output summation
// order, so every shape gives bitwise identical results).
struct LaunchConfig {
  int waves_per_block = 4;  // 1..4 (1 and 2 are 1-8 % slower)
  // Consecutive blocks on one XCD, so that the anchors of a face share one
  // L2: halves the float64 interpolation's L2 misses (Taylor-3: 1.49 -> 0.75
  // GB per 20,000 faces) and gives restriction ~2 %.  Float32 interpolation,
  // which it slows down, takes runs of four blocks per XCD instead (mode 2).
  int xcd_remap = 1;
  // Calls with at most this many unknowns per cell run the small-U body
  // (lanes over stencil points and rows instead of unknowns; every float32
  // mode then runs on the vector ALUs), per direction.  Plans, which mix
  // directions, use the interpolation limit.
  int small_unknowns[2] = {FT_SMALL_UNKNOWNS_INTERP, FT_SMALL_UNKNOWNS_RESTRICT};
};

hipError_t launch_apply(const ft_operator* op, const LaunchArgs& la, const LaunchConfig& cfg,
                        hipStream_t stream);

// Float32 interpolation on the matrix cores with 3 or 6 split-bfloat16 terms.
hipError_t launch_interp_mfma(const ft_operator* op, const LaunchArgs& la,
                              const LaunchConfig& cfg, int terms, hipStream_t stream);

// Copies of face views between patches and face buffers, and same-level halo
// pairs (see ft_patch.hip).
enum FaceCopyMode { kGatherFaces = 0, kScatterFaces = 1, kHaloPairs = 2 };
struct FaceCopyArgs {
  int mode;
  int p, k;
  int halves;  // FT_HALF_* (gather / scatter)
  int64_t n_items;
  const int8_t* sel;  // patch face (gather / scatter) or axis (halo pairs)
  const int64_t* off_a;
  const int64_t* off_b;
  int U;
  int elem_size;  // 4 or 8 bytes
  const void* src;
  int64_t src_elems;
  void* dst;
  int64_t dst_elems;
  int* errors;  // may be null
};
hipError_t launch_face_copy(const FaceCopyArgs& c, hipStream_t stream);

}  // namespace ft
