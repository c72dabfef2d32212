// Copies between patches and face buffers, and the same-level halo exchange
// (Section 2: patches of p^3 cells with a halo of depth k on their faces; where
// neighbours share one resolution the halo is a copy of the neighbour's
// boundary layers).  Pure data movement, bound by HBM bandwidth.
//
// Every job copies a range of normal layers [n0, n0 + L) (face-buffer
// numbering) between two face views of one physical face.  Along axis 0 both
// views are contiguous (stride one cell in a face buffer and in a patch box),
// so a job is a set of rows of contiguous cells: p x p rows of L cells when
// the normal is axis 0, L x p rows of p cells otherwise.  One wave copies the
// p x L cells that share the outermost tangential index, lanes over the
// elements of a row (coalesced on both sides), four loads in flight.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ft_internal.h"
#include "ft_kernels.h"

namespace ft {

// Normal layers of the chosen halves of patch face `face` in face-buffer
// numbering: layers [0, k) lie on the - side of the face, which is inside the
// patch for an upper face (face >= 3) and in its halo for a lower face.
__device__ inline void half_range(int face, int k, int halves, int* n0, int* len) {
  if (halves == FT_HALF_BOTH) {
    *n0 = 0;
    *len = 2 * k;
    return;
  }
  const bool minus_is_inner = face >= 3;
  const bool want_minus = (halves == FT_HALF_INNER) == minus_is_inner;
  *n0 = want_minus ? 0 : k;
  *len = k;
}

template <typename E>
__device__ inline void copy_row(const E* src, E* dst, int64_t n, int lane) {
  constexpr int kInFlight = 4;
  for (int64_t i0 = 0; i0 < n; i0 += 64 * kInFlight) {
    E v[kInFlight];
#pragma unroll
    for (int j = 0; j < kInFlight; ++j) {
      const int64_t i = i0 + j * 64 + lane;
      if (i < n) v[j] = src[i];
    }
#pragma unroll
    for (int j = 0; j < kInFlight; ++j) {
      const int64_t i = i0 + j * 64 + lane;
      if (i < n) dst[i] = v[j];
    }
  }
}

// mode kGatherFaces: sel = patch face (0..5), off_a = patch, off_b = face
// buffer; src = patches, dst = face buffers.  kScatterFaces: the same
// descriptors, src = face buffers, dst = patches.  kHaloPairs: sel = axis,
// off_a = lower patch, off_b = upper patch, src = dst = the patch array; two
// jobs per pair.
template <typename E>
__global__ __launch_bounds__(256) void face_copy_kernel(
    const int mode, const int p, const int k, const int halves, const int64_t n_items,
    const int8_t* __restrict__ sel, const int64_t* __restrict__ off_a,
    const int64_t* __restrict__ off_b, const int U, const E* src, const int64_t src_elems,
    E* dst, const int64_t dst_elems, int* errors) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  const int jobs = mode == kHaloPairs ? 2 : 1;
  const int64_t jw = w / p;
  const int r2 = (int)(w - jw * p);
  const int64_t item = jw / jobs;
  const int job = (int)(jw - item * jobs);
  if (item >= n_items) return;

  const int P = p + 2 * k;
  const int64_t patch_elems = (int64_t)P * P * P * U;
  const int64_t face_elems = (int64_t)2 * k * p * p * U;
  const int s = sel[item];
  const int64_t oa = off_a[item], ob = off_b[item];
  const bool halo = mode == kHaloPairs;
  const bool gather = mode == kGatherFaces;
  // Patches: the pair's two patches, or the gathered / scattered patch.
  const int64_t pa_lim = (halo || gather ? src_elems : dst_elems) - patch_elems;
  const int64_t pb_lim = halo ? src_elems - patch_elems
                              : (gather ? dst_elems : src_elems) - face_elems;
  const bool bad = s < 0 || s > (halo ? 2 : 5) || oa < 0 || ob < 0 || oa > pa_lim || ob > pb_lim;
  if (bad) {
    if (errors && r2 == 0 && job == 0 && lane == 0) atomicAdd(errors, 1);
    return;
  }
  FaceView sv, dv;
  int64_t so, dof;
  int a, n0, len;
  if (halo) {
    a = s;
    const FaceView lower_patch_upper_face = patch_view(a + 3, p, k);
    const FaceView upper_patch_lower_face = patch_view(a, p, k);
    if (job == 0) {  // layers [k, 2k): the lower patch's halo from the upper patch
      sv = upper_patch_lower_face;
      so = ob;
      dv = lower_patch_upper_face;
      dof = oa;
      n0 = k;
    } else {  // layers [0, k): the upper patch's halo from the lower patch
      sv = lower_patch_upper_face;
      so = oa;
      dv = upper_patch_lower_face;
      dof = ob;
      n0 = 0;
    }
    len = k;
  } else {
    a = s % 3;
    half_range(s, k, halves, &n0, &len);
    const FaceView pv = patch_view(s, p, k);
    const FaceView bv = buffer_view(a, p, k);
    sv = gather ? pv : bv;
    dv = gather ? bv : pv;
    so = gather ? oa : ob;
    dof = gather ? ob : oa;
  }
  const E* sp = src + so;
  E* dp = dst + dof;
  if (a == 0) {
    // rows along the normal: L cells at (ib = r1, ic = r2)
    for (int r1 = 0; r1 < p; ++r1) {
      const int sc0 = sv.base + n0 * sv.sa + r1 * sv.sb + r2 * sv.sc;
      const int dc0 = dv.base + n0 * dv.sa + r1 * dv.sb + r2 * dv.sc;
      copy_row(sp + (int64_t)sc0 * U, dp + (int64_t)dc0 * U, (int64_t)len * U, lane);
    }
  } else {
    // rows along the first tangential axis (axis 0): p cells at (ia = n0 + r1, ic = r2)
    for (int r1 = 0; r1 < len; ++r1) {
      const int sc0 = sv.base + (n0 + r1) * sv.sa + r2 * sv.sc;
      const int dc0 = dv.base + (n0 + r1) * dv.sa + r2 * dv.sc;
      copy_row(sp + (int64_t)sc0 * U, dp + (int64_t)dc0 * U, (int64_t)p * U, lane);
    }
  }
}

template <typename E>
static hipError_t launch_copy_typed(const FaceCopyArgs& c, hipStream_t stream) {
  constexpr int kWaves = 4;
  const int jobs = c.mode == kHaloPairs ? 2 : 1;
  // Split so that waves per launch stay below 2^30.
  const int64_t chunk = ((int64_t)1 << 30) / ((int64_t)jobs * c.p);
  for (int64_t i0 = 0; i0 < c.n_items; i0 += chunk) {
    const int64_t n = std::min<int64_t>(chunk, c.n_items - i0);
    const int64_t waves = n * jobs * c.p;
    const int64_t blocks = (waves + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(face_copy_kernel<E>, dim3((unsigned)blocks), dim3(64 * kWaves), 0, stream,
                       c.mode, c.p, c.k, c.halves, n, c.sel + i0, c.off_a + i0, c.off_b + i0, c.U,
                       static_cast<const E*>(c.src), c.src_elems, static_cast<E*>(c.dst),
                       c.dst_elems, c.errors);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_face_copy(const FaceCopyArgs& c, hipStream_t stream) {
  if (c.elem_size == 8) return launch_copy_typed<uint64_t>(c, stream);
  return launch_copy_typed<uint32_t>(c, stream);
}

}  // namespace ft
