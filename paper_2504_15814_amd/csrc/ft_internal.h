// Internal types shared by the host-side operator builder, the C ABI and the
// gfx950 kernels.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include "facetransfer.h"

#include <cstdint>
#include <string>
#include <vector>

namespace ft {

constexpr int kMaxP = 48;        // largest supported patch size
constexpr int kAxisClasses = 5;  // tangential classes per axis (see axis_class)
constexpr int kClasses = kAxisClasses * kAxisClasses;
constexpr int kMaxStencil = 64;  // widest weight block (a 3rd-order fit uses <= 33)

// Reference frame used by the builder and the kernels.
//  * Normal coordinate n: interpolation counts coarse layers from the face
//    into the coarse side (n >= 0 inside the coarse patch, n < 0 the coarse
//    face's fine-side half); restriction counts fine layers into the fine
//    side (n >= 0 the fine patch's inner half, n < 0 its halo).  Both
//    destinations use the same n-mapping as their source buffer.
//  * Tangential coordinates (b, c): cell index along the tangential axes b < c.
// A block of weights serves every expansion cell whose tangential anchor
// column lies in the same class along each axis.

// Class of an anchor column m in [0, p): how far it is from either face edge,
// saturated at two cells (all stencils reach at most two cells out).
__host__ __device__ inline int axis_class(int m, int p) {
  const int lo = m < 2 ? m : 2;
  const int hi = (p - 1 - m) < 2 ? (p - 1 - m) : 2;
  return lo < 2 ? lo : 4 - hi;
}

// Anchors along one tangential axis of fine subface digit sd (0..2); p need
// not be a multiple of 3.  Fine column j of the subface is global fine column
// J = sd*p + j, inside coarse column J / 3 at offset (J % 3 - 1) / 3.
// Interpolation: the anchors are the coarse columns m = interp_anchor0 + e
// that hold at least one fine column of the subface.
__host__ __device__ inline int interp_anchor0(int sd, int p) { return (sd * p) / 3; }
__host__ __device__ inline bool interp_anchor_valid(int m, int sd, int p) {
  return 3 * m <= sd * p + p - 1;
}
// Restriction: the coarse columns m = restrict_anchor0 + e whose centre lies
// on the subface; it coincides with the subface's fine column 3m + 1 - sd*p.
__host__ __device__ inline int restrict_anchor0(int sd, int p) { return (sd * p + 1) / 3; }
__host__ __device__ inline bool restrict_anchor_valid(int m, int sd, int p) {
  return 3 * m + 1 - sd * p <= p - 1;
}
// Largest number of anchors per axis over the three subface digits.
__host__ __device__ inline int anchors_per_axis(int direction, int p) {
  int best = 0;
  for (int sd = 0; sd < 3; ++sd) {
    const int n = direction == 0 ? (sd * p + p - 1) / 3 - interp_anchor0(sd, p) + 1
                                 : (sd * p + p - 2) / 3 - restrict_anchor0(sd, p) + 1;
    best = n > best ? n : best;
  }
  return best;
}

// Physical strides (in cells) of the normal and tangential axes of a face
// buffer with normal axis a: cell = i0 + e0 * (i1 + e1 * i2).
struct FaceStrides {
  int sa, sb, sc;
};
__host__ __device__ inline FaceStrides face_strides(int a, int p, int k) {
  FaceStrides s;
  if (a == 0) {
    s.sa = 1; s.sb = 2 * k; s.sc = 2 * k * p;
  } else if (a == 1) {
    s.sa = p; s.sb = 1; s.sc = 2 * k * p;
  } else {
    s.sa = p * p; s.sb = 1; s.sc = p;
  }
  return s;
}

// Where the 2k x p x p cells of one face live: cell (ia, ib, ic) of the face
// (normal index ia in face-buffer numbering, tangential ib, ic) is cell
// base + ia * sa + ib * sb + ic * sc of the array.
struct FaceView {
  int sa, sb, sc, base;
};
// The face buffer itself.
__host__ __device__ inline FaceView buffer_view(int a, int p, int k) {
  const FaceStrides s = face_strides(a, p, k);
  return FaceView{s.sa, s.sb, s.sc, 0};
}
// Face `face` (a + 3 * upper) of a patch box of (p + 2k)^3 cells, interior
// [k, k + p) per axis, axis 0 fastest: normal layers [0, 2k) for a lower face,
// [p, p + 2k) for an upper face, tangential cells [k, k + p).
__host__ __device__ inline FaceView patch_view(int face, int p, int k) {
  const int P = p + 2 * k;
  const int a = face % 3;
  const int b = a == 0 ? 1 : 0;
  const int c = a == 2 ? 1 : 2;
  const int S[3] = {1, P, P * P};
  FaceView v;
  v.sa = S[a];
  v.sb = S[b];
  v.sc = S[c];
  v.base = (face >= 3 ? p : 0) * v.sa + k * v.sb + k * v.sc;
  return v;
}

// A two-dimensional face buffer (normal axis a of two): 2k cells along a and
// p along the other axis, axis 0 fastest; the third stride is unused.
__host__ __device__ inline FaceView buffer_view2d(int a, int p, int k) {
  return a == 0 ? FaceView{1, 2 * k, 0, 0} : FaceView{p, 1, 0, 0};
}

// Layout of the arrays a transfer call reads and writes.
enum Layout { kFaceBuffers = 0, kPatches = 1 };

// Source and destination views of one hanging face of orientation o.  With
// patches the fine patch's face is o and the coarse patch's face (o + 3) % 6.
__host__ __device__ inline void transfer_views(int direction, int layout, int o, int p, int k,
                                               FaceView* src, FaceView* dst) {
  if (layout == kFaceBuffers) {
    *src = *dst = buffer_view(o % 3, p, k);
    return;
  }
  const FaceView coarse = patch_view((o + 3) % 6, p, k);
  const FaceView fine = patch_view(o, p, k);
  *src = direction == 0 ? coarse : fine;
  *dst = direction == 0 ? fine : coarse;
}

// Buffer index along the normal of reference coordinate n: base + sign * n.
// Interpolation: n counts into the coarse side, which is the - side (buffer
// indices k-1, k-2, ...) when the fine patch lies on the + side (o < 3).
// Restriction: n counts into the fine side.
__host__ __device__ inline void normal_map_side(int direction, bool fine_plus, int k, int* base,
                                                int* sign) {
  const bool count_minus = (direction == 0) ? fine_plus : !fine_plus;
  *base = count_minus ? k - 1 : k;
  *sign = count_minus ? -1 : 1;
}
// Three dimensions: the fine patch is on the + side for o < 3 (o < 2 in 2D).
__host__ __device__ inline void normal_map(int direction, int o, int k, int* base, int* sign) {
  normal_map_side(direction, o < 3, k, base, sign);
}

// Packed stencil entry: normal coordinate (absolute) and tangential offsets
// from the block's anchor column, each as a signed byte.
__host__ __device__ inline int pack_point(int n, int db, int dc) {
  return (n & 0xff) | ((db & 0xff) << 8) | ((dc & 0xff) << 16);
}
__host__ __device__ inline void unpack_point(int v, int* n, int* db, int* dc) {
  *n = (int)(int8_t)(v & 0xff);
  *db = (int)(int8_t)((v >> 8) & 0xff);
  *dc = (int)(int8_t)((v >> 16) & 0xff);
}

// Kernel-side view of an operator (passed by value as a kernel argument).
struct DevOp {
  int direction, scheme, p, k;
  int dim;        // 3, or 2 for two-dimensional faces
  int R;          // rows per expansion cell
  int E;          // anchors per axis and subface (p / 3 when 3 divides p)
  int copy_row;   // row that is an exact copy of a source cell, or -1
  int copy_n;     // normal coordinate of that source cell (tangential = anchor)
  int width[kClasses];  // stencil width per block (0 = class unused)
  int start[kClasses];  // first stencil entry of the block
  const int* stencil;   // packed points, [sum of widths]
  const double* w64;    // weights, [(start + q) * R + r]
  const float* w32;
  // Interpolation only: the weights split into three bfloat16 parts
  // (W = W0 + W1 + W2 to ~2^-27 relative), laid out as MFMA A operands:
  // [class][k-step][part][lane][8], see mfma_a_index().
  const uint16_t* wbf16;
};

// MFMA v_mfma_f32_32x32x16_bf16 operand layout (lane l of a wave):
//   A (32 x 16): lane l holds A[l % 32][8 * (l / 32) + i], i = 0..7
//   B (16 x 32): lane l holds B[8 * (l / 32) + i][l % 32]
//   D (32 x 32): register v of lane l holds D[8 * (v / 4) + 4 * (l / 32) + v % 4][l % 32]
constexpr int kMfmaK = 16;       // stencil points per MFMA k-step
constexpr int kMfmaSteps = 3;    // k-steps per block: stencils up to 48 points
constexpr int kBf16Parts = 3;
__host__ __device__ inline int64_t mfma_a_index(int cls, int step, int part, int lane) {
  return ((((int64_t)cls * kMfmaSteps + step) * kBf16Parts + part) * 64 + lane) * 8;
}

// Host-side operator: the weight tables plus their device copies.
struct HostBlock {
  int width = 0;
  std::vector<int> points;      // packed
  std::vector<double> weights;  // [q * R + r]
};

}  // namespace ft

struct ft_operator {
  int direction, scheme, p, k, R, E, copy_row, copy_n;
  int dim = 3;
  ft::HostBlock blocks[ft::kClasses];
  bool on_device = false;
  int device = -1;
  int* d_stencil = nullptr;
  double* d_w64 = nullptr;
  float* d_w32 = nullptr;
  uint16_t* d_wbf16 = nullptr;
  int* d_errors = nullptr;
  ft::DevOp* d_devop = nullptr;  // device copy of `dev` (kernels read it through a pointer)
  ft::DevOp dev{};
};

namespace ft {
// Message returned by transfer_last_error() on the calling thread.
void set_last_error(const std::string& msg);

// Empty if [ptr, ptr + bytes) lies inside one allocation of device memory of
// device `dev`; otherwise a message naming `what`.  Host pointers (pageable or
// pinned), other devices' memory and ranges running past the end of their
// allocation are refused before any kernel can dereference them.
std::string device_range_error(const void* ptr, int64_t bytes, int dev, const char* what);

// Builder (host): fills blocks[] of op for op->direction/scheme/p/k.
// Returns an empty string on success, else a message.
std::string build_tables(ft_operator* op);
}  // namespace ft
