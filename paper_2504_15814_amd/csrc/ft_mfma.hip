// Float32 interpolation on the matrix cores for one operator and a batch of
// hanging faces (split-bfloat16 MFMA; the per-item work is mfma_item in
// ft_device.h).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ft_device.h"
#include "ft_internal.h"
#include "ft_kernels.h"

namespace ft {

// Six waves per SIMD: the accumulators then live in 80 VGPRs (the compiler's
// own choice, 58 VGPRs + 32 AGPRs, allows five; six-term Taylor-3
// interpolation 2-3 % faster, same-machine A/B).  The six-term form spills three
// registers under this hint; five waves per SIMD avoids that and is no faster.
template <int R, int EC, int TERMS, int DIM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void interp_mfma_kernel(
    const DevOp* __restrict__ op, const int64_t n_faces, const int waves_per_block,
    const int8_t* __restrict__ orientation, const int8_t* __restrict__ subface,
    const int64_t* __restrict__ src_offset, const int64_t* __restrict__ dst_offset, const int U,
    const float* __restrict__ src, const int64_t src_elems, float* __restrict__ dst,
    const int64_t dst_elems, int* __restrict__ errors, const int layout, const int xcd_remap) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int E = EC > 0 ? EC : op->E;
  const int anchors = DIM == 3 ? E * E : E;
  const int item = (int)logical_block(xcd_remap) * waves_per_block + wave;
  const int face = item / anchors;
  if (face >= n_faces) return;
  mfma_item<R, EC, TERMS, DIM>(op, face, item - face * anchors, layout, orientation, subface,
                               src_offset, dst_offset, U, src, src_elems, dst, dst_elems, errors);
}

template <int R, int EC, int TERMS, int DIM = 3>
static hipError_t launch_mfma_one(const ft_operator* op, const LaunchArgs& la,
                                  const LaunchConfig& cfg, hipStream_t stream) {
  const int anchors = DIM == 3 ? op->E * op->E : op->E;
  const int64_t chunk = ((int64_t)1 << 30) / anchors;
  for (int64_t f0 = 0; f0 < la.n_faces; f0 += chunk) {
    const int64_t nf = std::min<int64_t>(chunk, la.n_faces - f0);
    const int64_t blocks = (nf * anchors + cfg.waves_per_block - 1) / cfg.waves_per_block;
    hipLaunchKernelGGL((interp_mfma_kernel<R, EC, TERMS, DIM>), dim3((unsigned)blocks),
                       dim3(64 * cfg.waves_per_block), 0, stream, op->d_devop, nf,
                       cfg.waves_per_block, la.orientation + f0, la.subface + f0,
                       la.src_offset + f0, la.dst_offset + f0, la.U,
                       static_cast<const float*>(la.src), la.src_elems,
                       static_cast<float*>(la.dst), la.dst_elems, la.errors, la.layout,
                       2 /* runs of blocks per XCD (fully XCD-contiguous: 2-5 % slower) */);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int R, int TERMS>
static hipError_t launch_mfma_e(const ft_operator* op, const LaunchArgs& la,
                                const LaunchConfig& cfg, hipStream_t stream) {
  switch (op->E) {
    case 2: return launch_mfma_one<R, 2, TERMS>(op, la, cfg, stream);
    case 3: return launch_mfma_one<R, 3, TERMS>(op, la, cfg, stream);
    case 4: return launch_mfma_one<R, 4, TERMS>(op, la, cfg, stream);
    default: return launch_mfma_one<R, 0, TERMS>(op, la, cfg, stream);
  }
}

hipError_t launch_interp_mfma(const ft_operator* op, const LaunchArgs& la,
                              const LaunchConfig& cfg, int terms, hipStream_t stream) {
  if (cfg.waves_per_block < 1 || cfg.waves_per_block > 4) return hipErrorInvalidValue;
  if (op->dim == 2) {
    const bool six = terms == 6;
    if (op->k == 1)
      return six ? launch_mfma_one<3, 0, 6, 2>(op, la, cfg, stream)
                 : launch_mfma_one<3, 0, 3, 2>(op, la, cfg, stream);
    if (op->k == 2)
      return six ? launch_mfma_one<6, 0, 6, 2>(op, la, cfg, stream)
                 : launch_mfma_one<6, 0, 3, 2>(op, la, cfg, stream);
    return six ? launch_mfma_one<9, 0, 6, 2>(op, la, cfg, stream)
               : launch_mfma_one<9, 0, 3, 2>(op, la, cfg, stream);
  }
  if (op->k == 1)
    return terms == 6 ? launch_mfma_e<9, 6>(op, la, cfg, stream)
                      : launch_mfma_e<9, 3>(op, la, cfg, stream);
  if (op->k == 2)
    return terms == 6 ? launch_mfma_e<18, 6>(op, la, cfg, stream)
                      : launch_mfma_e<18, 3>(op, la, cfg, stream);
  return terms == 6 ? launch_mfma_e<27, 6>(op, la, cfg, stream)
                    : launch_mfma_e<27, 3>(op, la, cfg, stream);
}

}  // namespace ft
