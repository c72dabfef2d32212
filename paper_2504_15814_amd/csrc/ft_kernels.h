// Launch interface between the C ABI and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "ft_internal.h"

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
};

// Tunable launch shape (schedules never change the per-output summation
// order, so every shape gives bitwise identical results).
struct LaunchConfig {
  int waves_per_block = 4;  // 1..4
  int xcd_remap = 0;
};

hipError_t launch_apply(const ft_operator* op, const LaunchArgs& la, const LaunchConfig& cfg,
                        hipStream_t stream);

// Float32 interpolation on the matrix cores with 3 or 6 split-bfloat16 terms.
hipError_t launch_interp_mfma(const ft_operator* op, const LaunchArgs& la,
                              const LaunchConfig& cfg, int terms, hipStream_t stream);

}  // namespace ft
