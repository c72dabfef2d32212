// Plans: uneven mixes of hanging faces (orientation, direction, scheme, patch
// size, halo depth) in one persistent launch, an autotuner over launch
// shapes, and HIP-graph capture of whole steps.
//
// Device side: a plan phase is a table of segments, one per batch, each a
// contiguous range of (face, anchor) work items.  A fixed grid of waves walks
// the items with a grid stride, segment by segment, and runs the same
// per-item bodies as the per-batch kernels (ft_device.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "facetransfer.h"
#include "ft_device.h"
#include "ft_internal.h"
#include "ft_kernels.h"

namespace ft {

enum PlanKind {
  kInterp18,
  kInterp27,
  kRestrict2Inject,
  kRestrict2Plain,
  kRestrict3Inject,
  kRestrict3Plain,
  kInterp9,        // k = 1
  kRestrict1Plain  // k = 1
};

struct PlanSeg {
  const DevOp* op;
  const int8_t* orientation;
  const int8_t* subface;
  const int64_t* coarse_offset;
  const int64_t* fine_offset;
  int* errors;
  int64_t item0;     // first work item of the segment
  int64_t item_end;  // one past its last work item
  int kind;
  int anchors;
  int layout;  // kFaceBuffers, or kPatches (FT_PLAN_PATCHES)
  int pad_;
};

// One work item of a plan segment, for one kind of operator.  T: coarse
// storage, TF: fine storage (float64 fine data restricted into float32 coarse
// faces, else T; interpolation only runs with TF = T).
template <typename T, int MODE, int KIND, typename TF>
__device__ __forceinline__ void plan_item(const PlanSeg* __restrict__ S, const int face_, const int e_,
                                       const int U, T* __restrict__ coarse,
                                       const int64_t coarse_elems, TF* __restrict__ fine,
                                       const int64_t fine_elems) {
  const int face = __builtin_amdgcn_readfirstlane(face_);
  const int e = __builtin_amdgcn_readfirstlane(e_);
  const DevOp* __restrict__ op = S->op;
  const FT_CONST DevOp* cop = cptr(op);
  if constexpr (KIND == kInterp9 || KIND == kInterp18 || KIND == kInterp27) {
    constexpr int R = KIND == kInterp9 ? 9 : (KIND == kInterp18 ? 18 : 27);
    constexpr int COPY = R >= 18 ? 13 : -1;
    if constexpr (!std::is_same_v<T, TF>)
      return;  // the host admits no interpolation batch into such a plan
    else if constexpr (MODE == 0)
      apply_item<0, R, 0, COPY, T, T, T>(
          op, face, e, S->layout, S->orientation, S->subface, S->coarse_offset,
          S->fine_offset, U, coarse, coarse_elems, fine, fine_elems,
          (const T*)(sizeof(T) == 8 ? (const void*)cop->w64 : (const void*)cop->w32), S->errors);
    else
      mfma_item<R, 0, MODE>(op, face, e, S->layout, S->orientation, S->subface,
                            S->coarse_offset, S->fine_offset, U, (const float*)coarse,
                            coarse_elems, (float*)fine, fine_elems, S->errors);
  } else {
    constexpr int R = KIND == kRestrict1Plain
                          ? 1
                          : ((KIND == kRestrict2Inject || KIND == kRestrict2Plain) ? 2 : 3);
    constexpr int COPY = (KIND == kRestrict2Inject || KIND == kRestrict3Inject) ? 0 : -1;
    apply_item<1, R, 0, COPY, TF, double, double, 3, T>(op, face, e, S->layout, S->orientation,
                                                        S->subface, S->fine_offset,
                                                        S->coarse_offset, U, fine, fine_elems,
                                                        coarse, coarse_elems, cop->w64, S->errors);
  }
}

// MODE 0: interpolation on the vector ALUs in precision T; MODE 3 / 6:
// float32 interpolation on the matrix cores with that many bfloat16 product
// terms.  Restriction always sums in float64.  Storage types as for plan_item.
template <typename T, int MODE, typename TF = T>
__global__ __launch_bounds__(256) void plan_kernel(const PlanSeg* __restrict__ segs,
                                                   const int nseg, const int wpb,
                                                   const int remap, const int U,
                                                   T* __restrict__ coarse, const int64_t coarse_elems,
                                                   TF* __restrict__ fine, const int64_t fine_elems) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t b = blockIdx.x;
  if (remap) {
    // Block i runs on XCD i % 8: give every XCD a contiguous range of
    // logical waves, so that neighbouring items share an L2.
    const int64_t nb = gridDim.x, per = nb / 8, full = per * 8;
    if (b < full) b = (b % 8) * per + b / 8;
  }
  const int64_t stride = (int64_t)gridDim.x * wpb;
  const int64_t w = b * wpb + wave;
  // Segments in order; inside a segment this wave takes every stride-th item
  // (continuing the grid-stride sequence across segments).  The kind switch
  // sits outside the item loop so each loop holds a single body.
  for (int sg = 0; sg < nseg; ++sg) {
    const PlanSeg* __restrict__ S = segs + sg;
    const int64_t item0 = S->item0, item_end = S->item_end;
    int64_t first = item0 + ((w - item0) % stride + stride) % stride;
    if (first >= item_end) continue;
    const int anchors = S->anchors;
    switch (S->kind) {
#define FT_PLAN_LOOP(KIND)                                                                     \
  for (int64_t it = first; it < item_end; it += stride) {                                      \
    const int local = (int)(it - item0); /* segments hold < 2^31 items */                      \
    const int face = local / anchors;                                                          \
    plan_item<T, MODE, KIND, TF>(S, face, local - face * anchors, U, coarse, coarse_elems,     \
                                 fine, fine_elems);                                            \
  }                                                                                            \
  break;
      case kInterp18: FT_PLAN_LOOP(kInterp18)
      case kInterp27: FT_PLAN_LOOP(kInterp27)
      case kRestrict2Inject: FT_PLAN_LOOP(kRestrict2Inject)
      case kRestrict2Plain: FT_PLAN_LOOP(kRestrict2Plain)
      case kRestrict3Inject: FT_PLAN_LOOP(kRestrict3Inject)
      case kInterp9: FT_PLAN_LOOP(kInterp9)
      case kRestrict1Plain: FT_PLAN_LOOP(kRestrict1Plain)
      default: FT_PLAN_LOOP(kRestrict3Plain)
#undef FT_PLAN_LOOP
    }
  }
}

// Non-persistent form of the same fused launch: the grid covers every work
// item once, and each wave finds its segment by binary search over the
// segment table (a handful of scalar loads).  Without the grid-stride loop
// the bodies keep their stand-alone register budget.
template <typename T, int MODE, typename TF = T>
__global__ __launch_bounds__(256) void plan_item_kernel(const PlanSeg* __restrict__ segs,
                                                        const int nseg, const int64_t total,
                                                        const int wpb, const int remap,
                                                        const int U, T* __restrict__ coarse,
                                                        const int64_t coarse_elems,
                                                        TF* __restrict__ fine,
                                                        const int64_t fine_elems) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t b = blockIdx.x;
  if (remap) {
    const int64_t nb = gridDim.x, per = nb / 8, full = per * 8;
    if (b < full) b = (b % 8) * per + b / 8;
  }
  const int64_t it = b * wpb + wave;
  if (it >= total) return;
  int lo = 0, hi = nseg - 1;  // first segment whose item_end exceeds it
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (it >= segs[mid].item_end) lo = mid + 1; else hi = mid;
  }
  // The search is wave-uniform; say so, so that the segment and the operator
  // it points to are read through the scalar cache.
  const PlanSeg* __restrict__ S = segs + __builtin_amdgcn_readfirstlane(lo);
  const int local = (int)(it - S->item0);
  const int anchors = S->anchors;
  const int face = local / anchors;
  const int e = local - face * anchors;
  switch (S->kind) {
    case kInterp18: plan_item<T, MODE, kInterp18, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems); break;
    case kInterp27: plan_item<T, MODE, kInterp27, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems); break;
    case kRestrict2Inject: plan_item<T, MODE, kRestrict2Inject, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems); break;
    case kRestrict2Plain: plan_item<T, MODE, kRestrict2Plain, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems); break;
    case kRestrict3Inject: plan_item<T, MODE, kRestrict3Inject, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems); break;
    case kInterp9: plan_item<T, MODE, kInterp9, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems); break;
    case kRestrict1Plain: plan_item<T, MODE, kRestrict1Plain, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems); break;
    default: plan_item<T, MODE, kRestrict3Plain, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems); break;
  }
}

// One work item of a plan segment with the small-U body (few unknowns per
// cell): every mode runs on the vector ALUs, as the per-batch calls do.
// Storage types as for plan_item.
template <typename T, int KIND, typename TF>
__device__ __forceinline__ void plan_small_item(const PlanSeg* __restrict__ S, const int face_,
                                                const int e_, const int U, T* __restrict__ coarse,
                                                const int64_t coarse_elems, TF* __restrict__ fine,
                                                const int64_t fine_elems, double* xs_words) {
  const int face = __builtin_amdgcn_readfirstlane(face_);
  const int e = __builtin_amdgcn_readfirstlane(e_);
  const DevOp* __restrict__ op = S->op;
  const FT_CONST DevOp* cop = cptr(op);
  if constexpr (KIND == kInterp9 || KIND == kInterp18 || KIND == kInterp27) {
    constexpr int R = KIND == kInterp9 ? 9 : (KIND == kInterp18 ? 18 : 27);
    constexpr int COPY = R >= 18 ? 13 : -1;
    if constexpr (!std::is_same_v<T, TF>)
      return;  // the host admits no interpolation batch into such a plan
    else
      small_item<0, R, COPY, T, T, T>(
          op, face, e, S->layout, S->orientation, S->subface, S->coarse_offset, S->fine_offset, U,
          coarse, coarse_elems, fine, fine_elems,
          (const T*)(sizeof(T) == 8 ? (const void*)cop->w64 : (const void*)cop->w32), S->errors,
          reinterpret_cast<T*>(xs_words));
  } else {
    constexpr int R = KIND == kRestrict1Plain
                          ? 1
                          : ((KIND == kRestrict2Inject || KIND == kRestrict2Plain) ? 2 : 3);
    constexpr int COPY = (KIND == kRestrict2Inject || KIND == kRestrict3Inject) ? 0 : -1;
    small_item<1, R, COPY, TF, double, double, 3, T>(op, face, e, S->layout, S->orientation,
                                                     S->subface, S->fine_offset, S->coarse_offset,
                                                     U, fine, fine_elems, coarse, coarse_elems,
                                                     cop->w64, S->errors, xs_words);
  }
}

// The non-persistent plan launch with the small-U body; each wave owns
// xs_stride words of the block's dynamic LDS.
template <typename T, typename TF = T>
__global__ __launch_bounds__(256) void plan_small_kernel(const PlanSeg* __restrict__ segs,
                                                         const int nseg, const int64_t total,
                                                         const int wpb, const int remap,
                                                         const int U, T* __restrict__ coarse,
                                                         const int64_t coarse_elems,
                                                         TF* __restrict__ fine,
                                                         const int64_t fine_elems,
                                                         const int xs_stride) {
  extern __shared__ double plan_lds[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int64_t b = blockIdx.x;
  if (remap) {
    const int64_t nb = gridDim.x, per = nb / 8, full = per * 8;
    if (b < full) b = (b % 8) * per + b / 8;
  }
  const int64_t it = b * wpb + wave;
  if (it >= total) return;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (it >= segs[mid].item_end) lo = mid + 1; else hi = mid;
  }
  const PlanSeg* __restrict__ S = segs + __builtin_amdgcn_readfirstlane(lo);
  const int local = (int)(it - S->item0);
  const int anchors = S->anchors;
  const int face = local / anchors;
  const int e = local - face * anchors;
  double* xs = plan_lds + wave * xs_stride;
  switch (S->kind) {
    case kInterp18: plan_small_item<T, kInterp18, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems, xs); break;
    case kInterp27: plan_small_item<T, kInterp27, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems, xs); break;
    case kRestrict2Inject: plan_small_item<T, kRestrict2Inject, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems, xs); break;
    case kRestrict2Plain: plan_small_item<T, kRestrict2Plain, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems, xs); break;
    case kRestrict3Inject: plan_small_item<T, kRestrict3Inject, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems, xs); break;
    case kInterp9: plan_small_item<T, kInterp9, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems, xs); break;
    case kRestrict1Plain: plan_small_item<T, kRestrict1Plain, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems, xs); break;
    default: plan_small_item<T, kRestrict3Plain, TF>(S, face, e, U, coarse, coarse_elems, fine, fine_elems, xs); break;
  }
}

// ---------------------------------------------------------------------------
// Allocation-free fused launch (run_transfer_batches): the segment tables of
// one call live in `scratch`, a fixed array of this library in device memory
// (every device holds its own copy), filled by a small kernel whose
// arguments carry the segments, then read by plan_item_kernel.
// ---------------------------------------------------------------------------
constexpr int kScratchSegs = 128;  // segments per phase
static __device__ __align__(256) PlanSeg scratch[2 * kScratchSegs];

constexpr int kFillSegs = 16;  // segments per fill launch (passed by value)
struct SegFill {
  PlanSeg seg[kFillSegs];
  int first;  // first table entry written
  int count;
};

__global__ __launch_bounds__(64) void fill_segments_kernel(PlanSeg* __restrict__ table,
                                                           const SegFill fill) {
  const int i = threadIdx.x;
  if (i < fill.count) table[fill.first + i] = fill.seg[i];
}

// Device segment tables of a plan: for each phase, the segments in batch
// order and in heavy-first order, uploaded once when the plan is built.  A
// schedule change only picks the other table, so a captured graph keeps
// valid kernel arguments; graphs share ownership of the tables, so they stay
// valid after the plan is destroyed as well.
struct PlanTables {
  int device = -1;
  PlanSeg* d_segs[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [phase][heavy first]
  ~PlanTables() {
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (device >= 0) (void)hipSetDevice(device);
    for (auto& ph : d_segs)
      for (PlanSeg*& t : ph)
        if (t) (void)hipFree(t);
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};
}  // namespace ft

struct ft_plan {
  std::vector<ft_plan_batch> batches;
  int U = 0, dtype = 0, flags = 0, device = -1, n_cu = 256;
  void* coarse = nullptr;
  void* fine = nullptr;
  int64_t coarse_elems = 0, fine_elems = 0;
  int64_t schedule = 0;
  std::shared_ptr<ft::PlanTables> tables;
  int nseg[2] = {0, 0};
  int64_t total[2] = {0, 0};
  bool interp[2] = {false, false};  // the phase holds interpolation segments
  int widest = 0;                   // widest weight block of any batch's operator
};

struct ft_graph {
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = -1;
  std::vector<std::shared_ptr<ft::PlanTables>> tables;  // read by the captured kernels
};

namespace {

int pfail(int code, const std::string& msg) {
  ft::set_last_error(msg);
  return code;
}

int phip(hipError_t e, const char* what) {
  return pfail(FT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int wpb_of(int64_t s) { return (int)(s & 0xff); }
int bpc_of(int64_t s) { return (int)((s >> 8) & 0xff); }
int remap_of(int64_t s) { return (int)((s >> 16) & 1); }
int heavy_of(int64_t s) { return (int)((s >> 17) & 1); }
int persistent_of(int64_t s) { return (int)((s >> 18) & 1); }

int plan_kind(const ft_operator* op) {
  if (op->direction == FT_INTERPOLATE)
    return op->k == 1 ? ft::kInterp9 : (op->k == 2 ? ft::kInterp18 : ft::kInterp27);
  if (op->k == 1) return ft::kRestrict1Plain;
  const bool inject = op->copy_row == 0;
  if (op->k == 2) return inject ? ft::kRestrict2Inject : ft::kRestrict2Plain;
  return inject ? ft::kRestrict3Inject : ft::kRestrict3Plain;
}

// Relative cost of one work item (rows x widest block), for heavy-first order.
double item_cost(const ft_operator* op) {
  int w = 0;
  for (int c = 0; c < ft::kClasses; ++c) w = std::max(w, op->blocks[c].width);
  return (double)op->R * w + 64.0 * op->R;  // FMAs + stores
}

// Host checks shared by plans and run_transfer_batches; on success *dev_out
// is the current device.
int check_batches(const ft_plan_batch* batches, int n_batches, int unknowns, int dtype,
                  const void* coarse, int64_t coarse_elems, const void* fine, int64_t fine_elems,
                  int flags, int* dev_out) {
  if (!batches || n_batches < 1) return pfail(FT_ERR_INVALID, "need at least one batch");
  if (unknowns < 1 || unknowns > 4096) return pfail(FT_ERR_UNSUPPORTED, "unknowns must be 1..4096");
  if (dtype < FT_F64 || dtype > FT_F64_TO_F32) return pfail(FT_ERR_UNSUPPORTED, "unsupported dtype");
  if (flags & ~(FT_PLAN_RESTRICT_FIRST | FT_PLAN_PATCHES))
    return pfail(FT_ERR_INVALID, "unknown flags");
  if (dtype == FT_F64_TO_F32 && (flags & FT_PLAN_PATCHES))
    return pfail(FT_ERR_UNSUPPORTED, "FT_F64_TO_F32 takes face buffers");
  // Face buffers: one array for coarse and fine would let a face overwrite
  // what it reads.  Patches: reads are face views, writes halos of other
  // faces, so one pool may hold both.
  if (!coarse || !fine || coarse_elems < 0 || fine_elems < 0 ||
      (coarse == fine && !(flags & FT_PLAN_PATCHES)))
    return pfail(FT_ERR_INVALID, "bad coarse / fine buffers");
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return phip(e, "hipGetDevice");
  for (int i = 0; i < n_batches; ++i) {
    const ft_plan_batch& b = batches[i];
    if (!b.op || b.n_faces < 0) return pfail(FT_ERR_INVALID, "batch with NULL op or n_faces < 0");
    if (!b.op->on_device || b.op->device != dev)
      return pfail(FT_ERR_INVALID, "batch operator is host-only or on another device");
    if (b.op->dim != 3) return pfail(FT_ERR_UNSUPPORTED, "plans take three-dimensional operators");
    if (b.n_faces > 0 && (!b.orientation || !b.subface || !b.coarse_offset || !b.fine_offset))
      return pfail(FT_ERR_INVALID, "batch with NULL descriptor arrays");
    if (b.n_faces * (int64_t)b.op->E * b.op->E >= ((int64_t)1 << 31))
      return pfail(FT_ERR_UNSUPPORTED, "batch too large (faces x anchors must stay below 2^31)");
    if (dtype == FT_F64_TO_F32 && b.op->direction == FT_INTERPOLATE)
      return pfail(FT_ERR_UNSUPPORTED, "FT_F64_TO_F32 is a restriction type (interpolation batch)");
    if ((dtype == FT_F32_BF16X3 || dtype == FT_F32_BF16X6) && b.op->direction == FT_INTERPOLATE &&
        !b.op->d_wbf16)
      return pfail(FT_ERR_UNSUPPORTED, "operator blocks too wide for the matrix-core path");
  }
  // Every array the kernels will dereference must be device memory of this
  // device, as large as stated.
  const int64_t coarse_size = dtype == FT_F64 ? 8 : 4;
  const int64_t fine_size = (dtype == FT_F64 || dtype == FT_F64_TO_F32) ? 8 : 4;
  std::string err = ft::device_range_error(coarse, coarse_size * coarse_elems, dev, "coarse buffer");
  if (err.empty()) err = ft::device_range_error(fine, fine_size * fine_elems, dev, "fine buffer");
  for (int i = 0; i < n_batches && err.empty(); ++i) {
    const ft_plan_batch& b = batches[i];
    if (b.n_faces == 0) continue;
    err = ft::device_range_error(b.orientation, b.n_faces, dev, "batch orientation");
    if (err.empty()) err = ft::device_range_error(b.subface, b.n_faces, dev, "batch subface");
    if (err.empty())
      err = ft::device_range_error(b.coarse_offset, 8 * b.n_faces, dev, "batch coarse offsets");
    if (err.empty())
      err = ft::device_range_error(b.fine_offset, 8 * b.n_faces, dev, "batch fine offsets");
  }
  if (!err.empty()) return pfail(FT_ERR_INVALID, err);
  *dev_out = dev;
  return FT_OK;
}

// Phase of a batch: restriction first with FT_PLAN_RESTRICT_FIRST.
int phase_of(const ft_plan_batch& b, int flags) {
  return (flags & FT_PLAN_RESTRICT_FIRST) ? (b.op->direction == FT_RESTRICT ? 0 : 1) : 0;
}

// Segment of one batch whose work items start at item0.
ft::PlanSeg make_segment(const ft_plan_batch& b, int flags, int64_t item0) {
  ft::PlanSeg sgm;
  sgm.op = b.op->d_devop;
  sgm.orientation = b.orientation;
  sgm.subface = b.subface;
  sgm.coarse_offset = b.coarse_offset;
  sgm.fine_offset = b.fine_offset;
  sgm.errors = b.op->d_errors;
  sgm.anchors = b.op->E * b.op->E;
  sgm.kind = plan_kind(b.op);
  sgm.layout = (flags & FT_PLAN_PATCHES) ? ft::kPatches : ft::kFaceBuffers;
  sgm.pad_ = 0;
  sgm.item0 = item0;
  sgm.item_end = item0 + b.n_faces * sgm.anchors;
  return sgm;
}

// Widest weight block over the batches' operators (LDS of the small-U body).
int widest_block(const ft_plan_batch* batches, int n_batches) {
  int w = 0;
  for (int i = 0; i < n_batches; ++i)
    for (int c = 0; c < ft::kClasses; ++c) w = std::max(w, batches[i].op->blocks[c].width);
  return w;
}

// Small-U launch of one phase: one wave per work item (the persistent form
// and the matrix-core bodies are not used for few unknowns).
template <typename T, typename TF = T>
hipError_t launch_small_items(const ft::PlanSeg* segs, int nseg, int64_t total, int wpb, int remap,
                              int U, int widest, void* coarse, int64_t coarse_elems, void* fine,
                              int64_t fine_elems, hipStream_t stream) {
  const int64_t blocks = (total + wpb - 1) / wpb;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  // one slice per wave: the weight block (at most 27 rows) and the source
  // values, counted in doubles (float slices use half of it)
  const int xs_stride = widest * (27 + U);
  const size_t lds = (size_t)wpb * xs_stride * sizeof(double);
  if (lds > 65536) return hipErrorInvalidValue;  // beyond one workgroup's LDS
  hipLaunchKernelGGL((ft::plan_small_kernel<T, TF>), dim3((unsigned)blocks), dim3(64 * wpb), lds,
                     stream, segs, nseg, total, wpb, remap, U, static_cast<T*>(coarse),
                     coarse_elems, static_cast<TF*>(fine), fine_elems, xs_stride);
  return hipGetLastError();
}

// The small-U launch for a plan's storage types.
hipError_t launch_small_typed(int dtype, const ft::PlanSeg* segs, int nseg, int64_t total,
                              int wpb, int remap, int U, int widest, void* coarse,
                              int64_t coarse_elems, void* fine, int64_t fine_elems,
                              hipStream_t stream) {
  if (dtype == FT_F64)
    return launch_small_items<double>(segs, nseg, total, wpb, remap, U, widest, coarse,
                                      coarse_elems, fine, fine_elems, stream);
  if (dtype == FT_F64_TO_F32)
    return launch_small_items<float, double>(segs, nseg, total, wpb, remap, U, widest, coarse,
                                             coarse_elems, fine, fine_elems, stream);
  return launch_small_items<float>(segs, nseg, total, wpb, remap, U, widest, coarse,
                                   coarse_elems, fine, fine_elems, stream);
}

// Build and upload the segment tables of both phases in both orders.
int upload_tables(ft_plan* plan) {
  auto tables = std::make_shared<ft::PlanTables>();
  tables->device = plan->device;
  for (int ph = 0; ph < 2; ++ph) {
    std::vector<int> idx;
    for (int i = 0; i < (int)plan->batches.size(); ++i) {
      const ft_plan_batch& b = plan->batches[i];
      if (b.n_faces > 0 && phase_of(b, plan->flags) == ph) idx.push_back(i);
    }
    plan->nseg[ph] = 0;
    plan->total[ph] = 0;
    plan->interp[ph] = false;
    if (idx.empty()) continue;
    for (int heavy = 0; heavy < 2; ++heavy) {
      if (heavy)
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) {
          return item_cost(plan->batches[a].op) > item_cost(plan->batches[c].op);
        });
      std::vector<ft::PlanSeg> segs;
      int64_t item = 0;
      for (int i : idx) {
        const ft_plan_batch& b = plan->batches[i];
        segs.push_back(make_segment(b, plan->flags, item));
        item = segs.back().item_end;
        if (b.op->direction == FT_INTERPOLATE) plan->interp[ph] = true;
      }
      ft::PlanSeg*& table = tables->d_segs[ph][heavy];
      hipError_t e = hipMalloc(&table, segs.size() * sizeof(ft::PlanSeg));
      if (e != hipSuccess) {
        table = nullptr;
        return e == hipErrorOutOfMemory ? pfail(FT_ERR_NOMEM, "plan table")
                                        : phip(e, "hipMalloc plan table");
      }
      e = hipMemcpy(table, segs.data(), segs.size() * sizeof(ft::PlanSeg), hipMemcpyHostToDevice);
      if (e != hipSuccess) return phip(e, "uploading the plan table");
      plan->nseg[ph] = (int)segs.size();
      plan->total[ph] = item;
    }
  }
  plan->tables = std::move(tables);
  return FT_OK;
}

template <typename T, int MODE, typename TF = T>
hipError_t launch_phase(const ft_plan* plan, int ph, hipStream_t stream) {
  const int wpb = wpb_of(plan->schedule);
  const int64_t want = (plan->total[ph] + wpb - 1) / wpb;
  if (!persistent_of(plan->schedule)) {
    if (want > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((ft::plan_item_kernel<T, MODE, TF>), dim3((unsigned)want), dim3(64 * wpb),
                       0, stream, plan->tables->d_segs[ph][heavy_of(plan->schedule)],
                       plan->nseg[ph], plan->total[ph], wpb,
                       remap_of(plan->schedule), plan->U, static_cast<T*>(plan->coarse),
                       plan->coarse_elems, static_cast<TF*>(plan->fine), plan->fine_elems);
    return hipGetLastError();
  }
  const int64_t blocks = std::min<int64_t>(want, (int64_t)plan->n_cu * bpc_of(plan->schedule));
  hipLaunchKernelGGL((ft::plan_kernel<T, MODE, TF>), dim3((unsigned)blocks), dim3(64 * wpb), 0,
                     stream, plan->tables->d_segs[ph][heavy_of(plan->schedule)], plan->nseg[ph],
                     wpb, remap_of(plan->schedule), plan->U,
                     static_cast<T*>(plan->coarse), plan->coarse_elems,
                     static_cast<TF*>(plan->fine), plan->fine_elems);
  return hipGetLastError();
}

int run_plan(const ft_plan* plan, hipStream_t stream) {
  for (int ph = 0; ph < 2; ++ph) {
    if (plan->total[ph] == 0) continue;
    // Restriction items run the same vector-ALU body in every float32 mode; a
    // phase without interpolation takes the kernel without matrix-core code
    // (fewer registers, more waves per SIMD).
    const int dtype = (plan->dtype != FT_F64 && plan->dtype != FT_F64_TO_F32 && !plan->interp[ph])
                          ? FT_F32
                          : plan->dtype;
    hipError_t e;
    if (plan->U <= ft::LaunchConfig().small_unknowns[0]) {
      e = launch_small_typed(plan->dtype, plan->tables->d_segs[ph][heavy_of(plan->schedule)],
                             plan->nseg[ph], plan->total[ph], wpb_of(plan->schedule),
                             remap_of(plan->schedule), plan->U, plan->widest, plan->coarse,
                             plan->coarse_elems, plan->fine, plan->fine_elems, stream);
      if (e != hipSuccess) return phip(e, "run_transfer_plan launch");
      continue;
    }
    switch (dtype) {
      case FT_F64: e = launch_phase<double, 0>(plan, ph, stream); break;
      case FT_F64_TO_F32: e = launch_phase<float, 0, double>(plan, ph, stream); break;
      case FT_F32: e = launch_phase<float, 0>(plan, ph, stream); break;
      case FT_F32_BF16X3: e = launch_phase<float, 3>(plan, ph, stream); break;
      default: e = launch_phase<float, 6>(plan, ph, stream); break;
    }
    if (e != hipSuccess) return phip(e, "run_transfer_plan launch");
  }
  return FT_OK;
}

// Device address of `scratch` on device `dev` (the current device), looked
// up once per device and kept: host code never passes the array's own name.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
ft::PlanSeg* g_scratch[kMaxDevices] = {};

int scratch_on(int dev, ft::PlanSeg** out) {
  if (dev < 0 || dev >= kMaxDevices) return pfail(FT_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(ft::scratch));
    if (e != hipSuccess) return phip(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return pfail(FT_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = static_cast<ft::PlanSeg*>(ptr);
  }
  *out = g_scratch[dev];
  return FT_OK;
}

// One wave per work item, four waves per block, over `nseg` segments at
// `segs` (the default plan schedule).
template <typename T, int MODE, typename TF = T>
hipError_t launch_items(const ft::PlanSeg* segs, int nseg, int64_t total, int U, void* coarse,
                        int64_t coarse_elems, void* fine, int64_t fine_elems, hipStream_t stream) {
  constexpr int wpb = 4;
  const int64_t blocks = (total + wpb - 1) / wpb;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((ft::plan_item_kernel<T, MODE, TF>), dim3((unsigned)blocks), dim3(64 * wpb),
                     0, stream, segs, nseg, total, wpb, 0, U, static_cast<T*>(coarse),
                     coarse_elems, static_cast<TF*>(fine), fine_elems);
  return hipGetLastError();
}

bool valid_schedule(int64_t s) {
  const int w = wpb_of(s), b = bpc_of(s);
  return (w == 1 || w == 2 || w == 4) && b >= 1 && b <= 64 && (s >> 19) == 0;
}

}  // namespace

extern "C" {

int build_transfer_plan(const ft_plan_batch* batches, int n_batches, int unknowns, int dtype,
                        void* coarse, int64_t coarse_elems, void* fine, int64_t fine_elems,
                        int flags, ft_plan** out) {
  if (!out) return pfail(FT_ERR_INVALID, "out is NULL");
  *out = nullptr;
  int dev = -1;
  const int rc0 = check_batches(batches, n_batches, unknowns, dtype, coarse, coarse_elems, fine,
                                fine_elems, flags, &dev);
  if (rc0 != FT_OK) return rc0;
  ft_plan* plan = new (std::nothrow) ft_plan();
  if (!plan) return pfail(FT_ERR_NOMEM, "host allocation failed");
  plan->batches.assign(batches, batches + n_batches);
  plan->U = unknowns;
  plan->dtype = dtype;
  plan->flags = flags;
  plan->device = dev;
  plan->coarse = coarse;
  plan->fine = fine;
  plan->coarse_elems = coarse_elems;
  plan->fine_elems = fine_elems;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    plan->n_cu = ncu;
  plan->schedule = 4 | (1 << 8);  // 4 waves per block, one wave per work item
  plan->widest = widest_block(batches, n_batches);
  const int rc = upload_tables(plan);
  if (rc != FT_OK) {
    delete plan;  // releases whatever tables were uploaded
    return rc;
  }
  *out = plan;
  ft::set_last_error("");
  return FT_OK;
}

int run_transfer_batches(const ft_plan_batch* batches, int n_batches, int unknowns, int dtype,
                         void* coarse, int64_t coarse_elems, void* fine, int64_t fine_elems,
                         int flags, void* stream) {
  int dev = -1;
  int rc = check_batches(batches, n_batches, unknowns, dtype, coarse, coarse_elems, fine,
                         fine_elems, flags, &dev);
  if (rc != FT_OK) return rc;
  int count[2] = {0, 0};
  for (int i = 0; i < n_batches; ++i)
    if (batches[i].n_faces > 0) ++count[phase_of(batches[i], flags)];
  if (count[0] > ft::kScratchSegs || count[1] > ft::kScratchSegs)
    return pfail(FT_ERR_UNSUPPORTED,
                 "run_transfer_batches takes at most 128 non-empty batches per phase");
  ft::PlanSeg* table = nullptr;
  if ((rc = scratch_on(dev, &table)) != FT_OK) return rc;
  const hipStream_t s = (hipStream_t)stream;
  for (int ph = 0; ph < 2; ++ph) {
    if (count[ph] == 0) continue;
    ft::PlanSeg* segs = table + ph * ft::kScratchSegs;
    ft::SegFill fill;
    fill.first = 0;
    fill.count = 0;
    int64_t item = 0;
    bool interp = false;
    hipError_t e = hipSuccess;
    for (int i = 0; i < n_batches && e == hipSuccess; ++i) {
      const ft_plan_batch& b = batches[i];
      if (b.n_faces == 0 || phase_of(b, flags) != ph) continue;
      fill.seg[fill.count] = make_segment(b, flags, item);
      item = fill.seg[fill.count].item_end;
      interp = interp || b.op->direction == FT_INTERPOLATE;
      if (++fill.count == ft::kFillSegs || fill.first + fill.count == count[ph]) {
        hipLaunchKernelGGL(ft::fill_segments_kernel, dim3(1), dim3(64), 0, s, segs, fill);
        e = hipGetLastError();
        fill.first += fill.count;
        fill.count = 0;
      }
    }
    if (e != hipSuccess) return phip(e, "run_transfer_batches table fill");
    if (unknowns <= ft::LaunchConfig().small_unknowns[0]) {
      e = launch_small_typed(dtype, segs, count[ph], item, 4, 0, unknowns,
                             widest_block(batches, n_batches), coarse, coarse_elems, fine,
                             fine_elems, s);
      if (e != hipSuccess) return phip(e, "run_transfer_batches launch");
      continue;
    }
    // As in plans: a phase without interpolation runs the vector-ALU kernel.
    const int mode = (dtype != FT_F64 && dtype != FT_F64_TO_F32 && !interp) ? FT_F32 : dtype;
    switch (mode) {
      case FT_F64: e = launch_items<double, 0>(segs, count[ph], item, unknowns, coarse, coarse_elems, fine, fine_elems, s); break;
      case FT_F64_TO_F32: e = launch_items<float, 0, double>(segs, count[ph], item, unknowns, coarse, coarse_elems, fine, fine_elems, s); break;
      case FT_F32: e = launch_items<float, 0>(segs, count[ph], item, unknowns, coarse, coarse_elems, fine, fine_elems, s); break;
      case FT_F32_BF16X3: e = launch_items<float, 3>(segs, count[ph], item, unknowns, coarse, coarse_elems, fine, fine_elems, s); break;
      default: e = launch_items<float, 6>(segs, count[ph], item, unknowns, coarse, coarse_elems, fine, fine_elems, s); break;
    }
    if (e != hipSuccess) return phip(e, "run_transfer_batches launch");
  }
  ft::set_last_error("");
  return FT_OK;
}

int run_transfer_plan(const ft_plan* plan, void* stream) {
  if (!plan) return pfail(FT_ERR_INVALID, "plan is NULL");
  const int rc = run_plan(plan, (hipStream_t)stream);
  if (rc == FT_OK) ft::set_last_error("");
  return rc;
}

int transfer_plan_set_schedule(ft_plan* plan, int64_t schedule) {
  if (!plan) return pfail(FT_ERR_INVALID, "plan is NULL");
  if (!valid_schedule(schedule)) return pfail(FT_ERR_INVALID, "invalid schedule");
  plan->schedule = schedule;  // both segment orders are uploaded already
  return FT_OK;
}

int transfer_plan_get_schedule(const ft_plan* plan, int64_t* schedule) {
  if (!plan || !schedule) return pfail(FT_ERR_INVALID, "NULL plan or schedule");
  *schedule = plan->schedule;
  return FT_OK;
}

int transfer_plan_autotune(ft_plan* plan, void* stream, int reps, int64_t* best_schedule,
                           double* best_ms) {
  if (!plan || reps < 1) return pfail(FT_ERR_INVALID, "NULL plan or reps < 1");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return pfail(FT_ERR_HIP, "hipEventCreate");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return pfail(FT_ERR_HIP, "hipEventCreate");
  }
  const int64_t orig = plan->schedule;
  int64_t best = orig;
  double best_t = INFINITY;
  int rc = FT_OK;
  // Candidates: one wave per work item, 2 or 4 waves per block, either block
  // numbering, either segment order.  The persistent grid-stride form is not
  // swept: it was 35-60 % slower on every measured mix, because a wave that
  // walks items must wait for its previous item's stores before the loads of
  // the next one count as returned (one in-order counter tracks a wave's
  // loads and stores), while a wave that ends after its stores leaves its slot
  // to a new wave whose loads start at once.
  std::vector<int64_t> cands;
  for (int heavy = 0; heavy < 2; ++heavy)
    for (int remap = 0; remap < 2; ++remap)
      for (int wpb : {2, 4})
        cands.push_back(wpb | (1LL << 8) | ((int64_t)remap << 16) | ((int64_t)heavy << 17));
  for (const int64_t sch : cands) {
    if ((rc = transfer_plan_set_schedule(plan, sch)) != FT_OK) break;
    if ((rc = run_plan(plan, s)) != FT_OK) break;  // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && rc == FT_OK; ++r) rc = run_plan(plan, s);
    (void)hipEventRecord(e1, s);
    if (rc != FT_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = pfail(FT_ERR_HIP, "autotune synchronisation");
      break;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double t = ms / reps;
    if (t < best_t) {
      best_t = t;
      best = sch;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != FT_OK) {
    (void)transfer_plan_set_schedule(plan, orig);
    return rc;
  }
  rc = transfer_plan_set_schedule(plan, best);
  if (rc != FT_OK) return rc;
  if (best_schedule) *best_schedule = best;
  if (best_ms) *best_ms = best_t;
  ft::set_last_error("");
  return FT_OK;
}

int destroy_transfer_plan(ft_plan* plan) {
  if (!plan) return FT_OK;
  delete plan;  // the tables go with the last graph that still uses them
  return FT_OK;
}

int transfer_plans_capture(const ft_plan* const* plans, int n_plans, int steps, ft_graph** out) {
  if (!out) return pfail(FT_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!plans || n_plans < 1 || steps < 1)
    return pfail(FT_ERR_INVALID, "NULL plans, n_plans < 1 or steps < 1");
  int dev = -1;
  const hipError_t de = hipGetDevice(&dev);
  if (de != hipSuccess) return phip(de, "hipGetDevice");
  for (int i = 0; i < n_plans; ++i) {
    if (!plans[i]) return pfail(FT_ERR_INVALID, "NULL plan");
    if (plans[i]->device != dev) return pfail(FT_ERR_INVALID, "plan belongs to another device");
  }
  ft_graph* g = new (std::nothrow) ft_graph();
  if (!g) return pfail(FT_ERR_NOMEM, "host allocation failed");
  g->device = dev;
  for (int i = 0; i < n_plans; ++i) g->tables.push_back(plans[i]->tables);
  hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete g;
    return phip(e, "hipStreamCreateWithFlags");
  }
  int rc = FT_OK;
  e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) rc = phip(e, "hipStreamBeginCapture");
  for (int i = 0; i < steps && rc == FT_OK; ++i)
    for (int j = 0; j < n_plans && rc == FT_OK; ++j) rc = run_plan(plans[j], g->stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(g->stream, &graph);
  if (rc == FT_OK && e != hipSuccess) rc = phip(e, "hipStreamEndCapture");
  g->graph = graph;
  if (rc == FT_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = phip(e, "hipGraphInstantiate");
  }
  if (rc != FT_OK) {
    destroy_transfer_graph(g);
    return rc;
  }
  *out = g;
  ft::set_last_error("");
  return FT_OK;
}

int transfer_plan_capture(const ft_plan* plan, int steps, ft_graph** out) {
  if (!plan) {
    if (out) *out = nullptr;
    return pfail(FT_ERR_INVALID, "NULL plan or steps < 1");
  }
  return transfer_plans_capture(&plan, 1, steps, out);
}

int transfer_graph_launch(const ft_graph* graph, void* stream) {
  if (!graph || !graph->exec) return pfail(FT_ERR_INVALID, "graph is NULL");
  const hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
  if (e != hipSuccess) return phip(e, "hipGraphLaunch");
  ft::set_last_error("");
  return FT_OK;
}

int destroy_transfer_graph(ft_graph* graph) {
  if (!graph) return FT_OK;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  if (graph->stream) (void)hipStreamDestroy(graph->stream);
  delete graph;
  return FT_OK;
}

}  // extern "C"
