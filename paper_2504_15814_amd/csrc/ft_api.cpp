// C ABI of the face-transfer library: argument checking, operator lifetime,
// device upload and error reporting.  No exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "facetransfer.h"
#include "ft_internal.h"
#include "ft_kernels.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int ok() {
  g_last_error.clear();
  return FT_OK;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(FT_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Round a float to bfloat16 (round to nearest even); NaN stays NaN.
uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// MFMA A-operand table of an interpolation operator: every weight split into
// three bfloat16 parts, zero for padding rows / stencil points and for the
// exact-copy row.  Empty if a block is wider than the MFMA path supports.
std::vector<uint16_t> bf16_table(const ft_operator* op) {
  std::vector<uint16_t> t;
  if (op->direction != FT_INTERPOLATE) return t;
  for (int c = 0; c < ft::kClasses; ++c)
    if (op->blocks[c].width > ft::kMfmaSteps * ft::kMfmaK) return t;
  t.assign((size_t)ft::mfma_a_index(ft::kClasses, 0, 0, 0), 0);
  for (int c = 0; c < ft::kClasses; ++c) {
    const ft::HostBlock& b = op->blocks[c];
    for (int st = 0; st < ft::kMfmaSteps; ++st)
      for (int lane = 0; lane < 64; ++lane) {
        const int m = lane % 32;
        for (int i = 0; i < 8; ++i) {
          const int q = ft::kMfmaK * st + 8 * (lane / 32) + i;
          if (m >= op->R || m == op->copy_row || q >= b.width) continue;
          const double w = b.weights[(size_t)q * op->R + m];
          const uint16_t w0 = bf16_rne((float)w);
          const double r1 = w - bf16_value(w0);
          const uint16_t w1 = bf16_rne((float)r1);
          const uint16_t w2 = bf16_rne((float)(r1 - bf16_value(w1)));
          const uint16_t parts[3] = {w0, w1, w2};
          for (int part = 0; part < ft::kBf16Parts; ++part)
            t[(size_t)ft::mfma_a_index(c, st, part, lane) + i] = parts[part];
        }
      }
  }
  return t;
}

void free_device(ft_operator* op) {
  if (!op->on_device) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(op->device);
  if (op->d_stencil) (void)hipFree(op->d_stencil);
  if (op->d_w64) (void)hipFree(op->d_w64);
  if (op->d_w32) (void)hipFree(op->d_w32);
  if (op->d_wbf16) (void)hipFree(op->d_wbf16);
  if (op->d_devop) (void)hipFree(op->d_devop);
  if (op->d_errors) (void)hipFree(op->d_errors);
  if (prev >= 0) (void)hipSetDevice(prev);
  op->d_stencil = nullptr;
  op->d_w64 = nullptr;
  op->d_w32 = nullptr;
  op->d_wbf16 = nullptr;
  op->d_devop = nullptr;
  op->d_errors = nullptr;
  op->on_device = false;
}

int upload(ft_operator* op) {
  std::vector<int> pts;
  std::vector<double> w64;
  std::vector<float> w32;
  ft::DevOp& d = op->dev;
  d.direction = op->direction;
  d.scheme = op->scheme;
  d.p = op->p;
  d.k = op->k;
  d.dim = op->dim;
  d.R = op->R;
  d.E = op->E;
  d.copy_row = op->copy_row;
  d.copy_n = op->copy_n;
  for (int c = 0; c < ft::kClasses; ++c) {
    const ft::HostBlock& b = op->blocks[c];
    d.width[c] = b.width;
    d.start[c] = (int)pts.size();
    pts.insert(pts.end(), b.points.begin(), b.points.end());
    w64.insert(w64.end(), b.weights.begin(), b.weights.end());
  }
  w32.resize(w64.size());
  for (size_t i = 0; i < w64.size(); ++i) w32[i] = (float)w64[i];
  const std::vector<uint16_t> wbf = bf16_table(op);
  if (pts.empty()) return fail(FT_ERR_INVALID, "operator has no weights");
  hipError_t e = hipGetDevice(&op->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  op->on_device = true;  // so that free_device releases partial allocations
  if ((e = hipMalloc(&op->d_stencil, pts.size() * sizeof(int))) != hipSuccess ||
      (e = hipMalloc(&op->d_w64, w64.size() * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&op->d_w32, w32.size() * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&op->d_errors, sizeof(int))) != hipSuccess ||
      (!wbf.empty() &&
       (e = hipMalloc(&op->d_wbf16, wbf.size() * sizeof(uint16_t))) != hipSuccess)) {
    free_device(op);
    return e == hipErrorOutOfMemory ? fail(FT_ERR_NOMEM, "device allocation failed")
                                    : hip_fail(e, "hipMalloc");
  }
  if ((e = hipMemcpy(op->d_stencil, pts.data(), pts.size() * sizeof(int), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(op->d_w64, w64.data(), w64.size() * sizeof(double), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(op->d_w32, w32.data(), w32.size() * sizeof(float), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemset(op->d_errors, 0, sizeof(int))) != hipSuccess ||
      (!wbf.empty() && (e = hipMemcpy(op->d_wbf16, wbf.data(), wbf.size() * sizeof(uint16_t),
                                      hipMemcpyHostToDevice)) != hipSuccess)) {
    free_device(op);
    return hip_fail(e, "uploading operator tables");
  }
  d.stencil = op->d_stencil;
  d.w64 = op->d_w64;
  d.w32 = op->d_w32;
  d.wbf16 = op->d_wbf16;
  if ((e = hipMalloc(&op->d_devop, sizeof(ft::DevOp))) != hipSuccess ||
      (e = hipMemcpy(op->d_devop, &d, sizeof(ft::DevOp), hipMemcpyHostToDevice)) != hipSuccess) {
    free_device(op);
    return hip_fail(e, "uploading the operator view");
  }
  return FT_OK;
}

int check_apply(const ft_operator* op, int direction, int64_t n_faces, const void* orientation,
                const void* subface, const void* so, const void* dof, int unknowns, int dtype,
                const void* src, int64_t src_elems, const void* dst, int64_t dst_elems,
                bool patches = false) {
  if (!op) return fail(FT_ERR_INVALID, "operator is NULL");
  if (op->direction != direction)
    return fail(FT_ERR_INVALID, direction == FT_INTERPOLATE
                                    ? "operator was built for restriction"
                                    : "operator was built for interpolation");
  if (!op->on_device) return fail(FT_ERR_INVALID, "operator was built host-only");
  if (n_faces < 0) return fail(FT_ERR_INVALID, "n_faces < 0");
  if (unknowns < 1 || unknowns > 4096) return fail(FT_ERR_UNSUPPORTED, "unknowns must be 1..4096");
  if (dtype < FT_F64 || dtype > FT_F64_TO_F32) return fail(FT_ERR_UNSUPPORTED, "unsupported dtype");
  if (dtype == FT_F64_TO_F32 && direction == FT_INTERPOLATE)
    return fail(FT_ERR_UNSUPPORTED, "FT_F64_TO_F32 is a restriction type");
  if (dtype == FT_F64_TO_F32 && patches)
    return fail(FT_ERR_UNSUPPORTED, "FT_F64_TO_F32 takes face buffers");
  if (direction == FT_INTERPOLATE && (dtype == FT_F32_BF16X3 || dtype == FT_F32_BF16X6) &&
      op->on_device && !op->d_wbf16)
    return fail(FT_ERR_UNSUPPORTED, "operator blocks too wide for the matrix-core path");
  if (src_elems < 0 || dst_elems < 0) return fail(FT_ERR_INVALID, "negative buffer size");
  if (n_faces == 0) return FT_OK;
  if (!orientation || !subface || !so || !dof || !src || !dst)
    return fail(FT_ERR_INVALID, "NULL descriptor or buffer pointer");
  // Face buffers: a face's source and destination are one cell box, so one
  // array for both would overwrite what is read.  Patches: a call reads face
  // views and writes halos of other faces, so one pool may hold both.
  if (src == dst && !patches) return fail(FT_ERR_INVALID, "source and destination alias");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != op->device) return fail(FT_ERR_INVALID, "operator belongs to another device");
  // FT_F64_TO_F32 (restriction only): float64 source, float32 destination.
  const int64_t src_size = (dtype == FT_F64 || dtype == FT_F64_TO_F32) ? 8 : 4;
  const int64_t dst_size = dtype == FT_F64 ? 8 : 4;
  const struct {
    const void* ptr;
    int64_t bytes;
    const char* what;
  } ranges[6] = {{orientation, n_faces, "orientation"},
                 {subface, n_faces, "subface"},
                 {so, 8 * n_faces, "source offsets"},
                 {dof, 8 * n_faces, "destination offsets"},
                 {src, src_size * src_elems, "source buffer"},
                 {dst, dst_size * dst_elems, "destination buffer"}};
  for (const auto& r : ranges) {
    const std::string err = ft::device_range_error(r.ptr, r.bytes, dev, r.what);
    if (!err.empty()) return fail(FT_ERR_INVALID, err);
  }
  return FT_OK;
}

// Host checks of the patch / face-buffer copies.  dst == nullptr: the
// same-level halo exchange, which reads and writes one array.
int check_copy(int p, int k, int64_t n, const void* sel, const void* off_a, const void* off_b,
               int halves, int unknowns, int dtype, const void* src, int64_t src_elems,
               const void* dst, int64_t dst_elems, const void* skipped) {
  if (p < 1 || p > 1024) return fail(FT_ERR_UNSUPPORTED, "p must be in 1..1024");
  if (k < 1 || k > p) return fail(FT_ERR_UNSUPPORTED, "k must be in 1..p");
  const int64_t P = p + 2 * k;
  if (P * P * P > ((int64_t)1 << 31) - 1) return fail(FT_ERR_UNSUPPORTED, "patch too large");
  if (n < 0) return fail(FT_ERR_INVALID, "negative item count");
  if (unknowns < 1 || unknowns > 4096) return fail(FT_ERR_UNSUPPORTED, "unknowns must be 1..4096");
  if (dtype < FT_F64 || dtype > FT_F32_BF16X6) return fail(FT_ERR_UNSUPPORTED, "unsupported dtype");
  if (halves < FT_HALF_INNER || halves > FT_HALF_BOTH)
    return fail(FT_ERR_INVALID, "halves must be FT_HALF_INNER, FT_HALF_OUTER or FT_HALF_BOTH");
  if (src_elems < 0 || dst_elems < 0) return fail(FT_ERR_INVALID, "negative buffer size");
  if (n == 0) return FT_OK;
  if (!sel || !off_a || !off_b || !src) return fail(FT_ERR_INVALID, "NULL descriptor or buffer");
  if (dst == src) return fail(FT_ERR_INVALID, "source and destination alias");
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const int64_t esz = dtype == FT_F64 ? 8 : 4;
  const struct {
    const void* ptr;
    int64_t bytes;
    const char* what;
  } ranges[6] = {{sel, n, "face / axis selectors"},
                 {off_a, 8 * n, "first offsets"},
                 {off_b, 8 * n, "second offsets"},
                 {src, esz * src_elems, "source buffer"},
                 {dst ? dst : src, esz * dst_elems, "destination buffer"},
                 {skipped, skipped ? 4 : 0, "skipped counter"}};
  for (const auto& r : ranges) {
    if (!r.ptr) continue;  // the optional counter
    const std::string err = ft::device_range_error(r.ptr, r.bytes, dev, r.what);
    if (!err.empty()) return fail(FT_ERR_INVALID, err);
  }
  return FT_OK;
}

// COO entries of the 1/9 (2D: 1/3) segment of `op` for one (orientation,
// subface), in the face buffer's physical cell numbering.
void segment_entries(const ft_operator* op, int orientation, int subface,
                     std::vector<int64_t>& rr, std::vector<int64_t>& cc, std::vector<double>& vv) {
  const bool d3 = op->dim == 3;
  const int p = op->p, k = op->k, E = op->E, R = op->R;
  const ft::FaceView st = d3 ? ft::buffer_view(orientation % 3, p, k)
                             : ft::buffer_view2d(orientation % 2, p, k);
  int nbase, nsign;
  ft::normal_map_side(op->direction, orientation < (d3 ? 3 : 2), k, &nbase, &nsign);
  const int sb = d3 ? subface % 3 : subface, sc = d3 ? subface / 3 : 0;
  for (int ec = 0; ec < (d3 ? E : 1); ++ec)
    for (int eb = 0; eb < E; ++eb) {
      // anchor columns in the source face (ab, ac) and the first destination
      // columns (db0, dc0); see the anchor helpers in ft_internal.h
      int ab, ac = 0, db0, dc0 = 0;
      if (op->direction == 0) {
        ab = ft::interp_anchor0(sb, p) + eb;
        if (!ft::interp_anchor_valid(ab, sb, p)) continue;
        db0 = 3 * ab - sb * p;
        if (d3) {
          ac = ft::interp_anchor0(sc, p) + ec;
          if (!ft::interp_anchor_valid(ac, sc, p)) continue;
          dc0 = 3 * ac - sc * p;
        }
      } else {
        db0 = ft::restrict_anchor0(sb, p) + eb;
        if (!ft::restrict_anchor_valid(db0, sb, p)) continue;
        ab = 3 * db0 + 1 - sb * p;
        if (d3) {
          dc0 = ft::restrict_anchor0(sc, p) + ec;
          if (!ft::restrict_anchor_valid(dc0, sc, p)) continue;
          ac = 3 * dc0 + 1 - sc * p;
        }
      }
      const auto& blk = op->blocks[ft::axis_class(ab, p) * ft::kAxisClasses +
                                   (d3 ? ft::axis_class(ac, p) : 0)];
      const int anchor = ab * st.sb + ac * st.sc;
      for (int r = 0; r < R; ++r) {
        int dcell;
        if (op->direction == 0) {
          const int g = d3 ? r / 9 : r / 3, tb = d3 ? (r / 3) % 3 : r % 3, tc = d3 ? r % 3 : 0;
          const int jb = db0 + tb, jc = dc0 + tc;
          if (jb < 0 || jb >= p || (d3 && (jc < 0 || jc >= p))) continue;  // other fine face
          dcell = (nbase + nsign * g) * st.sa + jb * st.sb + jc * st.sc;
        } else {
          dcell = (nbase + nsign * r) * st.sa + db0 * st.sb + dc0 * st.sc;
        }
        for (int q = 0; q < blk.width; ++q) {
          const double w = blk.weights[(size_t)q * R + r];
          if (w == 0.0) continue;
          int n, db, dc;
          ft::unpack_point(blk.points[q], &n, &db, &dc);
          rr.push_back(dcell);
          cc.push_back(anchor + (nbase + nsign * n) * st.sa + db * st.sb + dc * st.sc);
          vv.push_back(w);
        }
      }
    }
}

}  // namespace

void ft::set_last_error(const std::string& msg) { g_last_error = msg; }

std::string ft::device_range_error(const void* ptr, int64_t bytes, int dev, const char* what) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // do not leave the lookup's error for the next launch check
    return std::string(what) + " is not device memory";
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return std::string(what) + " is host memory, not device memory";
  if (attr.device != dev) return std::string(what) + " lives on another device";
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return std::string(what) + ": allocation range lookup failed";
  }
  const uintptr_t lo = (uintptr_t)base, hi = lo + size, p = (uintptr_t)ptr;
  if (bytes < 0 || p < lo || (uint64_t)bytes > (uint64_t)(hi - p))
    return std::string(what) + " extends past the end of its device allocation";
  return std::string();
}

extern "C" {

int build_transfer_operator(int direction, int scheme, int p, int k, int flags,
                            ft_operator** out) {
  if (!out) return fail(FT_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (direction != FT_INTERPOLATE && direction != FT_RESTRICT)
    return fail(FT_ERR_INVALID, "direction must be FT_INTERPOLATE or FT_RESTRICT");
  if (scheme != FT_DLINEAR && scheme != FT_TAYLOR2 && scheme != FT_TAYLOR3)
    return fail(FT_ERR_INVALID, "scheme must be FT_DLINEAR, FT_TAYLOR2 or FT_TAYLOR3");
  if (p < 6 || p > ft::kMaxP) return fail(FT_ERR_UNSUPPORTED, "p must be in [6, 48]");
  if (k < 1 || k > 3) return fail(FT_ERR_UNSUPPORTED, "k must be 1, 2 or 3");
  if (k == 1 && scheme != FT_DLINEAR)
    return fail(FT_ERR_UNSUPPORTED, "k = 1 is supported by FT_DLINEAR only");
  if (flags & ~(FT_BUILD_HOST_ONLY | FT_BUILD_2D)) return fail(FT_ERR_INVALID, "unknown flags");
  ft_operator* op = new (std::nothrow) ft_operator();
  if (!op) return fail(FT_ERR_NOMEM, "host allocation failed");
  op->dim = (flags & FT_BUILD_2D) ? 2 : 3;
  op->direction = direction;
  op->scheme = scheme;
  op->p = p;
  op->k = k;
  std::string err;
  try {
    err = ft::build_tables(op);
  } catch (const std::bad_alloc&) {
    delete op;
    return fail(FT_ERR_NOMEM, "host allocation failed");
  } catch (...) {
    delete op;
    return fail(FT_ERR_INVALID, "operator build failed");
  }
  if (!err.empty()) {
    delete op;
    return fail(FT_ERR_UNSUPPORTED, err);
  }
  if (!(flags & FT_BUILD_HOST_ONLY)) {
    const int rc = upload(op);
    if (rc != FT_OK) {
      delete op;
      return rc;
    }
  }
  *out = op;
  return ok();
}

int destroy_transfer_operator(ft_operator* op) {
  if (!op) return ok();
  free_device(op);
  delete op;
  return ok();
}

int interpolate_faces(const ft_operator* op, int64_t n_faces, const int8_t* orientation,
                      const int8_t* subface, const int64_t* coarse_offset,
                      const int64_t* fine_offset, int unknowns, int dtype, const void* coarse,
                      int64_t coarse_elems, void* fine, int64_t fine_elems, void* stream) {
  int rc = check_apply(op, FT_INTERPOLATE, n_faces, orientation, subface, coarse_offset,
                       fine_offset, unknowns, dtype, coarse, coarse_elems, fine, fine_elems);
  if (rc != FT_OK || n_faces == 0) return rc == FT_OK ? ok() : rc;
  ft::LaunchArgs la{n_faces, orientation, subface, coarse_offset, fine_offset, unknowns, dtype,
                    coarse, coarse_elems, fine, fine_elems, op->d_errors};
  hipError_t e;
  const ft::LaunchConfig cfg;
  if ((dtype == FT_F32_BF16X3 || dtype == FT_F32_BF16X6) && unknowns > cfg.small_unknowns[0])
    e = ft::launch_interp_mfma(op, la, cfg, dtype == FT_F32_BF16X6 ? 6 : 3, (hipStream_t)stream);
  else
    e = ft::launch_apply(op, la, cfg, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "interpolate_faces launch");
  return ok();
}

int restrict_faces(const ft_operator* op, int64_t n_faces, const int8_t* orientation,
                   const int8_t* subface, const int64_t* coarse_offset,
                   const int64_t* fine_offset, int unknowns, int dtype, const void* fine,
                   int64_t fine_elems, void* coarse, int64_t coarse_elems, void* stream) {
  int rc = check_apply(op, FT_RESTRICT, n_faces, orientation, subface, fine_offset,
                       coarse_offset, unknowns, dtype, fine, fine_elems, coarse, coarse_elems);
  if (rc != FT_OK || n_faces == 0) return rc == FT_OK ? ok() : rc;
  ft::LaunchArgs la{n_faces, orientation, subface, fine_offset, coarse_offset, unknowns, dtype,
                    fine, fine_elems, coarse, coarse_elems, op->d_errors};
  hipError_t e = ft::launch_apply(op, la, ft::LaunchConfig(), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "restrict_faces launch");
  return ok();
}

int interpolate_patches(const ft_operator* op, int64_t n_faces, const int8_t* orientation,
                        const int8_t* subface, const int64_t* coarse_offset,
                        const int64_t* fine_offset, int unknowns, int dtype, const void* coarse,
                        int64_t coarse_elems, void* fine, int64_t fine_elems, void* stream) {
  int rc = check_apply(op, FT_INTERPOLATE, n_faces, orientation, subface, coarse_offset,
                       fine_offset, unknowns, dtype, coarse, coarse_elems, fine, fine_elems, true);
  if (rc == FT_OK && op->dim != 3)
    rc = fail(FT_ERR_UNSUPPORTED, "patch calls take three-dimensional operators");
  if (rc != FT_OK || n_faces == 0) return rc == FT_OK ? ok() : rc;
  ft::LaunchArgs la{n_faces, orientation, subface, coarse_offset, fine_offset, unknowns, dtype,
                    coarse, coarse_elems, fine, fine_elems, op->d_errors, ft::kPatches};
  hipError_t e;
  const ft::LaunchConfig cfg;
  if ((dtype == FT_F32_BF16X3 || dtype == FT_F32_BF16X6) && unknowns > cfg.small_unknowns[0])
    e = ft::launch_interp_mfma(op, la, cfg, dtype == FT_F32_BF16X6 ? 6 : 3, (hipStream_t)stream);
  else
    e = ft::launch_apply(op, la, cfg, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "interpolate_patches launch");
  return ok();
}

int restrict_patches(const ft_operator* op, int64_t n_faces, const int8_t* orientation,
                     const int8_t* subface, const int64_t* coarse_offset,
                     const int64_t* fine_offset, int unknowns, int dtype, const void* fine,
                     int64_t fine_elems, void* coarse, int64_t coarse_elems, void* stream) {
  int rc = check_apply(op, FT_RESTRICT, n_faces, orientation, subface, fine_offset,
                       coarse_offset, unknowns, dtype, fine, fine_elems, coarse, coarse_elems,
                       true);
  if (rc == FT_OK && op->dim != 3)
    rc = fail(FT_ERR_UNSUPPORTED, "patch calls take three-dimensional operators");
  if (rc != FT_OK || n_faces == 0) return rc == FT_OK ? ok() : rc;
  ft::LaunchArgs la{n_faces, orientation, subface, fine_offset, coarse_offset, unknowns, dtype,
                    fine, fine_elems, coarse, coarse_elems, op->d_errors, ft::kPatches};
  hipError_t e = ft::launch_apply(op, la, ft::LaunchConfig(), (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "restrict_patches launch");
  return ok();
}

int gather_patch_faces(int p, int k, int64_t n, const int8_t* face, const int64_t* patch_offset,
                       const int64_t* face_offset, int halves, int unknowns, int dtype,
                       const void* patches, int64_t patch_elems, void* faces, int64_t face_elems,
                       int* skipped, void* stream) {
  const int rc = check_copy(p, k, n, face, patch_offset, face_offset, halves, unknowns, dtype,
                            patches, patch_elems, faces, face_elems, skipped);
  if (rc != FT_OK || n == 0) return rc == FT_OK ? ok() : rc;
  ft::FaceCopyArgs c{ft::kGatherFaces, p, k, halves, n, face, patch_offset, face_offset,
                     unknowns, dtype == FT_F64 ? 8 : 4, patches, patch_elems, faces,
                     face_elems, skipped};
  const hipError_t e = ft::launch_face_copy(c, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gather_patch_faces launch");
  return ok();
}

int scatter_patch_faces(int p, int k, int64_t n, const int8_t* face, const int64_t* patch_offset,
                        const int64_t* face_offset, int halves, int unknowns, int dtype,
                        const void* faces, int64_t face_elems, void* patches,
                        int64_t patch_elems, int* skipped, void* stream) {
  const int rc = check_copy(p, k, n, face, patch_offset, face_offset, halves, unknowns, dtype,
                            faces, face_elems, patches, patch_elems, skipped);
  if (rc != FT_OK || n == 0) return rc == FT_OK ? ok() : rc;
  ft::FaceCopyArgs c{ft::kScatterFaces, p, k, halves, n, face, patch_offset, face_offset,
                     unknowns, dtype == FT_F64 ? 8 : 4, faces, face_elems, patches,
                     patch_elems, skipped};
  const hipError_t e = ft::launch_face_copy(c, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "scatter_patch_faces launch");
  return ok();
}

int copy_patch_halos(int p, int k, int64_t n_pairs, const int8_t* axis,
                     const int64_t* lower_offset, const int64_t* upper_offset, int unknowns,
                     int dtype, void* patches, int64_t patch_elems, int* skipped, void* stream) {
  const int rc = check_copy(p, k, n_pairs, axis, lower_offset, upper_offset, FT_HALF_BOTH,
                            unknowns, dtype, patches, patch_elems, nullptr, patch_elems, skipped);
  if (rc != FT_OK || n_pairs == 0) return rc == FT_OK ? ok() : rc;
  ft::FaceCopyArgs c{ft::kHaloPairs, p, k, FT_HALF_BOTH, n_pairs, axis, lower_offset,
                     upper_offset, unknowns, dtype == FT_F64 ? 8 : 4, patches, patch_elems,
                     patches, patch_elems, skipped};
  const hipError_t e = ft::launch_face_copy(c, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "copy_patch_halos launch");
  return ok();
}

int transfer_operator_info(const ft_operator* op, int64_t* info, int n_info) {
  if (!op || !info || n_info < 1) return fail(FT_ERR_INVALID, "NULL op / info or n_info < 1");
  int64_t blocks = 0, widest = 0, wbytes = 0;
  for (int c = 0; c < ft::kClasses; ++c) {
    if (op->blocks[c].width == 0) continue;
    ++blocks;
    widest = std::max<int64_t>(widest, op->blocks[c].width);
    wbytes += (int64_t)op->blocks[c].weights.size() * 8;
  }
  const bool d3 = op->dim == 3;
  int64_t nnz = 0;
  {
    // Nonzero weights of the middle segment (orientation 0, subface 4; in 2D
    // subface 1).
    std::vector<int64_t> rr, cc;
    std::vector<double> vv;
    segment_entries(op, 0, d3 ? 4 : 1, rr, cc, vv);
    nnz = (int64_t)vv.size();
  }
  const int64_t vals[11] = {op->direction, op->scheme, op->p, op->k, op->R,
                            d3 ? (int64_t)op->E * op->E : (int64_t)op->E, blocks, widest, nnz,
                            wbytes, op->dim};
  for (int i = 0; i < n_info && i < 11; ++i) info[i] = vals[i];
  for (int i = 11; i < n_info; ++i) info[i] = 0;
  return ok();
}

int transfer_operator_segment(const ft_operator* op, int orientation, int subface,
                              int64_t capacity, int64_t* rows, int64_t* cols, double* vals,
                              int64_t* n_entries) {
  if (!op || !n_entries) return fail(FT_ERR_INVALID, "NULL op or n_entries");
  const bool d3 = op->dim == 3;
  if (orientation < 0 || orientation > (d3 ? 5 : 3) || subface < 0 || subface > (d3 ? 8 : 2))
    return fail(FT_ERR_INVALID, d3 ? "orientation must be 0..5 and subface 0..8"
                                   : "orientation must be 0..3 and subface 0..2 (2D)");
  std::vector<int64_t> rr, cc;
  std::vector<double> vv;
  segment_entries(op, orientation, subface, rr, cc, vv);
  *n_entries = (int64_t)rr.size();
  if (capacity < (int64_t)rr.size()) return fail(FT_ERR_INVALID, "capacity too small");
  if (!rows || !cols || !vals) return fail(FT_ERR_INVALID, "NULL output array");
  std::memcpy(rows, rr.data(), rr.size() * sizeof(int64_t));
  std::memcpy(cols, cc.data(), cc.size() * sizeof(int64_t));
  std::memcpy(vals, vv.data(), vv.size() * sizeof(double));
  return ok();
}

int transfer_operator_errors(const ft_operator* op, int64_t* n_skipped, int reset) {
  if (!op || !n_skipped) return fail(FT_ERR_INVALID, "NULL op or n_skipped");
  if (!op->on_device) return fail(FT_ERR_INVALID, "operator was built host-only");
  int prev = -1;
  (void)hipGetDevice(&prev);
  hipError_t e = hipSetDevice(op->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  int h = 0;
  if (e == hipSuccess) e = hipMemcpy(&h, op->d_errors, sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess && reset) e = hipMemset(op->d_errors, 0, sizeof(int));
  if (prev >= 0) (void)hipSetDevice(prev);
  if (e != hipSuccess) return hip_fail(e, "reading the error counter");
  *n_skipped = h;
  return ok();
}

const char* transfer_last_error(void) { return g_last_error.c_str(); }

int transfer_version(void) { return 200; }

}  // extern "C"
