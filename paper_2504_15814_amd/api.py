"""Python binding of the C ABI in include/facetransfer.h, same names.

Tensors are torch tensors on the GPU; the binding passes their data pointers
and element counts, the current HIP stream, and raises FTError on any
non-zero return code.  Every step of the transfer runs in the HIP library.
"""

import ctypes

import numpy as np
import torch

from . import _lib

FT_OK, FT_ERR_INVALID, FT_ERR_UNSUPPORTED, FT_ERR_HIP, FT_ERR_NOMEM = 0, 1, 2, 3, 4
FT_INTERPOLATE, FT_RESTRICT = 0, 1
FT_DLINEAR, FT_TAYLOR2, FT_TAYLOR3 = 1, 2, 3
FT_F64, FT_F32, FT_F32_BF16X3, FT_F32_BF16X6, FT_F64_TO_F32 = 0, 1, 2, 3, 4
FT_BUILD_HOST_ONLY = 1
FT_BUILD_2D = 2
FT_HALF_INNER, FT_HALF_OUTER, FT_HALF_BOTH = 1, 2, 3

_DTYPES = {torch.float64: FT_F64, torch.float32: FT_F32}


class FTError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.load().transfer_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with code {code}: {msg}")
        self.code = code


def _check(code, where):
    if code != FT_OK:
        raise FTError(code, where)


class TransferOperator:
    """Owns an ft_operator handle."""

    def __init__(self, handle, direction, scheme, p, k):
        self._h = handle
        self.direction, self.scheme, self.p, self.k = direction, scheme, p, k

    @property
    def handle(self):
        if not self._h:
            raise ValueError("operator already destroyed")
        return self._h

    def info(self):
        buf = (ctypes.c_int64 * 11)()
        _check(_lib.load().transfer_operator_info(self.handle, buf, 11), "transfer_operator_info")
        keys = ("direction", "scheme", "p", "k", "rows_per_anchor", "anchors", "blocks",
                "max_width", "nnz_segment", "weight_bytes", "dim")
        return dict(zip(keys, list(buf)))

    def segment(self, orientation, subface):
        """COO (rows, cols, vals) of the physical 1/9 segment."""
        lib = _lib.load()
        n = ctypes.c_int64(0)
        lib.transfer_operator_segment(self.handle, orientation, subface, 0, None, None, None, ctypes.byref(n))
        rows = np.zeros(n.value, dtype=np.int64)
        cols = np.zeros(n.value, dtype=np.int64)
        vals = np.zeros(n.value, dtype=np.float64)
        _check(
            lib.transfer_operator_segment(
                self.handle, orientation, subface, n.value,
                rows.ctypes.data_as(_lib.c_int64_p), cols.ctypes.data_as(_lib.c_int64_p),
                vals.ctypes.data_as(_lib.c_double_p), ctypes.byref(n)),
            "transfer_operator_segment",
        )
        return rows, cols, vals

    def errors(self, reset=True):
        n = ctypes.c_int64(0)
        _check(_lib.load().transfer_operator_errors(self.handle, ctypes.byref(n), int(reset)),
               "transfer_operator_errors")
        return n.value

    def destroy(self):
        if self._h:
            _lib.load().destroy_transfer_operator(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def build_transfer_operator(direction, scheme, p, k, flags=0):
    h = ctypes.c_void_p()
    _check(_lib.load().build_transfer_operator(direction, scheme, p, k, flags, ctypes.byref(h)),
           "build_transfer_operator")
    return TransferOperator(h.value, direction, scheme, p, k)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _on_device(name, t):
    """Every tensor handed to the library is a contiguous tensor on the
    current GPU: kernels dereference raw pointers with dense strides."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise TypeError(f"{name} must live on the GPU, not on {t.device}")
    if t.device.index != torch.cuda.current_device():
        raise TypeError(f"{name} lives on {t.device}, not on the current GPU "
                        f"(cuda:{torch.cuda.current_device()})")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return t


def _descriptors(orientation, subface, coarse_offset, fine_offset):
    for name, t, dt in (("orientation", orientation, torch.int8), ("subface", subface, torch.int8),
                        ("coarse_offset", coarse_offset, torch.int64), ("fine_offset", fine_offset, torch.int64)):
        if not isinstance(t, torch.Tensor) or t.dtype != dt:
            raise TypeError(f"{name} must be a {dt} tensor")
        _on_device(name, t)
    n = orientation.numel()
    if not (subface.numel() == coarse_offset.numel() == fine_offset.numel() == n):
        raise ValueError("descriptor arrays differ in length")
    return n


def _mode(coarse, fine, mode):
    """The C dtype code for the coarse and fine tensors: float64 -> FT_F64;
    float32 -> FT_F32 unless a split-bfloat16 mode is requested;
    FT_F64_TO_F32 (restriction) only on request, with float64 fine and
    float32 coarse data."""
    _on_device("coarse buffer", coarse)
    _on_device("fine buffer", fine)
    if mode == FT_F64_TO_F32:
        if fine.dtype != torch.float64 or coarse.dtype != torch.float32:
            raise TypeError("FT_F64_TO_F32 takes a float64 fine and a float32 coarse buffer")
        return mode
    if coarse.dtype != fine.dtype or coarse.dtype not in _DTYPES:
        raise TypeError("coarse and fine must share dtype float64 or float32")
    if mode is None:
        return _DTYPES[coarse.dtype]
    if coarse.dtype == torch.float64 and mode != FT_F64:
        raise TypeError("float64 buffers only support FT_F64")
    if coarse.dtype == torch.float32 and mode not in (FT_F32, FT_F32_BF16X3, FT_F32_BF16X6):
        raise TypeError("float32 buffers support FT_F32, FT_F32_BF16X3 and FT_F32_BF16X6")
    return mode


def interpolate_faces(op, orientation, subface, coarse_offset, fine_offset, unknowns, coarse, fine,
                      stream=None, mode=None):
    """Fill the halo half of every fine face buffer from its coarse face.
    `mode` selects the float32 application (FT_F32, FT_F32_BF16X3,
    FT_F32_BF16X6); by default it follows the tensors' dtype."""
    n = _descriptors(orientation, subface, coarse_offset, fine_offset)
    dt = _mode(coarse, fine, mode)
    _check(
        _lib.load().interpolate_faces(
            op.handle, n, _ptr(orientation), _ptr(subface), _ptr(coarse_offset), _ptr(fine_offset),
            unknowns, dt, _ptr(coarse), coarse.numel(), _ptr(fine), fine.numel(),
            _stream_ptr(stream)),
        "interpolate_faces",
    )


def restrict_faces(op, orientation, subface, coarse_offset, fine_offset, unknowns, fine, coarse,
                   stream=None, mode=None):
    """Fill each fine face's segment of its coarse face's fine-side half.
    mode=FT_F64_TO_F32 restricts float64 fine data into float32 coarse faces."""
    n = _descriptors(orientation, subface, coarse_offset, fine_offset)
    dt = _mode(coarse, fine, mode)
    _check(
        _lib.load().restrict_faces(
            op.handle, n, _ptr(orientation), _ptr(subface), _ptr(coarse_offset), _ptr(fine_offset),
            unknowns, dt, _ptr(fine), fine.numel(), _ptr(coarse), coarse.numel(),
            _stream_ptr(stream)),
        "restrict_faces",
    )


def interpolate_patches(op, orientation, subface, coarse_offset, fine_offset, unknowns, coarse, fine,
                        stream=None, mode=None):
    """Fill each fine patch's halo across its transition face straight from
    the coarse patch (offsets are patch offsets; coarse and fine may be the
    same tensor)."""
    n = _descriptors(orientation, subface, coarse_offset, fine_offset)
    dt = _mode(coarse, fine, mode)
    _check(
        _lib.load().interpolate_patches(
            op.handle, n, _ptr(orientation), _ptr(subface), _ptr(coarse_offset), _ptr(fine_offset),
            unknowns, dt, _ptr(coarse), coarse.numel(), _ptr(fine), fine.numel(),
            _stream_ptr(stream)),
        "interpolate_patches",
    )


def restrict_patches(op, orientation, subface, coarse_offset, fine_offset, unknowns, fine, coarse,
                     stream=None, mode=None):
    """Fill, in each coarse patch's halo, the segment under each fine patch."""
    n = _descriptors(orientation, subface, coarse_offset, fine_offset)
    dt = _mode(coarse, fine, mode)
    _check(
        _lib.load().restrict_patches(
            op.handle, n, _ptr(orientation), _ptr(subface), _ptr(coarse_offset), _ptr(fine_offset),
            unknowns, dt, _ptr(fine), fine.numel(), _ptr(coarse), coarse.numel(),
            _stream_ptr(stream)),
        "restrict_patches",
    )


def _copy_descriptors(sel, off_a, off_b):
    for name, t, dt in (("selector", sel, torch.int8), ("offset", off_a, torch.int64),
                        ("offset", off_b, torch.int64)):
        if not isinstance(t, torch.Tensor) or t.dtype != dt:
            raise TypeError(f"{name} must be a {dt} tensor")
        _on_device(name, t)
    n = sel.numel()
    if not (off_a.numel() == off_b.numel() == n):
        raise ValueError("descriptor arrays differ in length")
    return n


def _counter(skipped):
    """The optional int32 device counter of skipped items."""
    if skipped is None:
        return None
    if not isinstance(skipped, torch.Tensor) or skipped.dtype != torch.int32 or skipped.numel() < 1:
        raise TypeError("skipped must be an int32 tensor with at least one element")
    return _on_device("skipped", skipped)


def _elem_mode(*tensors):
    for t in tensors:
        _on_device("buffer", t)
    dts = {t.dtype for t in tensors}
    if len(dts) != 1 or tensors[0].dtype not in _DTYPES:
        raise TypeError("buffers must share dtype float64 or float32")
    return _DTYPES[tensors[0].dtype]


def gather_patch_faces(p, k, face, patch_offset, face_offset, halves, unknowns, patches, faces,
                       skipped=None, stream=None):
    """Copy the chosen halves of face view face[i] of each patch into its
    face buffer.  skipped: optional int32 device tensor counting bad items."""
    n = _copy_descriptors(face, patch_offset, face_offset)
    _check(
        _lib.load().gather_patch_faces(
            p, k, n, _ptr(face), _ptr(patch_offset), _ptr(face_offset), halves, unknowns,
            _elem_mode(patches, faces), _ptr(patches), patches.numel(), _ptr(faces), faces.numel(),
            _ptr(_counter(skipped)), _stream_ptr(stream)),
        "gather_patch_faces",
    )


def scatter_patch_faces(p, k, face, patch_offset, face_offset, halves, unknowns, faces, patches,
                        skipped=None, stream=None):
    """Write the chosen halves of each face buffer into face view face[i] of
    its patch."""
    n = _copy_descriptors(face, patch_offset, face_offset)
    _check(
        _lib.load().scatter_patch_faces(
            p, k, n, _ptr(face), _ptr(patch_offset), _ptr(face_offset), halves, unknowns,
            _elem_mode(patches, faces), _ptr(faces), faces.numel(), _ptr(patches), patches.numel(),
            _ptr(_counter(skipped)), _stream_ptr(stream)),
        "scatter_patch_faces",
    )


def copy_patch_halos(p, k, axis, lower_offset, upper_offset, unknowns, patches, skipped=None,
                     stream=None):
    """Same-level halo exchange across the upper face (along axis[i]) of the
    patch at lower_offset[i]."""
    n = _copy_descriptors(axis, lower_offset, upper_offset)
    _check(
        _lib.load().copy_patch_halos(
            p, k, n, _ptr(axis), _ptr(lower_offset), _ptr(upper_offset), unknowns,
            _elem_mode(patches), _ptr(patches), patches.numel(), _ptr(_counter(skipped)),
            _stream_ptr(stream)),
        "copy_patch_halos",
    )


def transfer_last_error():
    return _lib.load().transfer_last_error().decode(errors="replace")


def transfer_version():
    return _lib.load().transfer_version()


# ---------------------------------------------------------------------------
# Plans and graphs
# ---------------------------------------------------------------------------
FT_PLAN_RESTRICT_FIRST = 1
FT_PLAN_PATCHES = 2


def pack_schedule(waves_per_block=4, blocks_per_cu=8, xcd_remap=0, heavy_first=0, persistent=1):
    return (waves_per_block | (blocks_per_cu << 8) | (xcd_remap << 16) | (heavy_first << 17)
            | (persistent << 18))


def unpack_schedule(s):
    return {"waves_per_block": s & 0xFF, "blocks_per_cu": (s >> 8) & 0xFF,
            "xcd_remap": (s >> 16) & 1, "heavy_first": (s >> 17) & 1, "persistent": (s >> 18) & 1}


class TransferPlan:
    """Owns an ft_plan.  batches: list of (operator, orientation, subface,
    coarse_offset, fine_offset) with device descriptor tensors; the tensors
    and buffers are kept alive by the plan."""

    def __init__(self, handle, keepalive):
        self._h = handle
        self._keep = keepalive

    @property
    def handle(self):
        if not self._h:
            raise ValueError("plan already destroyed")
        return self._h

    def run(self, stream=None):
        run_transfer_plan(self, stream)

    @property
    def schedule(self):
        v = ctypes.c_int64()
        _check(_lib.load().transfer_plan_get_schedule(self.handle, ctypes.byref(v)), "transfer_plan_get_schedule")
        return v.value

    @schedule.setter
    def schedule(self, value):
        _check(_lib.load().transfer_plan_set_schedule(self.handle, int(value)), "transfer_plan_set_schedule")

    def autotune(self, reps=3, stream=None):
        return transfer_plan_autotune(self, reps, stream)

    def capture(self, steps=1):
        return transfer_plan_capture(self, steps)

    def destroy(self):
        if self._h:
            _lib.load().destroy_transfer_plan(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class TransferGraph:
    def __init__(self, handle, plan):
        self._h = handle
        self._plan = plan

    def launch(self, stream=None):
        transfer_graph_launch(self, stream)

    def destroy(self):
        if self._h:
            _lib.load().destroy_transfer_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _plan_batches(batches):
    arr = (_lib.PlanBatch * len(batches))()
    keep = []
    for i, (op, o, s, co, fo) in enumerate(batches):
        n = _descriptors(o, s, co, fo)
        arr[i] = _lib.PlanBatch(op.handle, n, o.data_ptr(), s.data_ptr(), co.data_ptr(), fo.data_ptr())
        keep.extend([op, o, s, co, fo])
    return arr, keep


def build_transfer_plan(batches, unknowns, coarse, fine, mode=None, flags=0):
    """A plan over batches of (operator, orientation, subface,
    coarse_offset, fine_offset); `coarse` and `fine` are the pools every
    batch addresses (mode FT_F64_TO_F32: restriction batches only, float64
    fine and float32 coarse pools)."""
    dt = _mode(coarse, fine, mode)
    arr, keep = _plan_batches(batches)
    keep.extend([coarse, fine])
    h = ctypes.c_void_p()
    _check(_lib.load().build_transfer_plan(arr, len(batches), unknowns, dt, _ptr(coarse), coarse.numel(),
                                           _ptr(fine), fine.numel(), flags, ctypes.byref(h)),
           "build_transfer_plan")
    return TransferPlan(h.value, keep)


def run_transfer_batches(batches, unknowns, coarse, fine, mode=None, flags=0, stream=None):
    """One fused launch over the batches without a plan object; the library
    allocates nothing (its segment table sits in a fixed device workspace).
    Calls on one GPU that overlap in time race on that workspace."""
    dt = _mode(coarse, fine, mode)
    arr, _ = _plan_batches(batches)
    _check(_lib.load().run_transfer_batches(arr, len(batches), unknowns, dt, _ptr(coarse), coarse.numel(),
                                            _ptr(fine), fine.numel(), flags, _stream_ptr(stream)),
           "run_transfer_batches")


def run_transfer_plan(plan, stream=None):
    _check(_lib.load().run_transfer_plan(plan.handle, _stream_ptr(stream)), "run_transfer_plan")


def transfer_plan_autotune(plan, reps=3, stream=None):
    best = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(_lib.load().transfer_plan_autotune(plan.handle, _stream_ptr(stream), reps, ctypes.byref(best),
                                              ctypes.byref(ms)), "transfer_plan_autotune")
    return best.value, ms.value


def transfer_plan_capture(plan, steps=1):
    h = ctypes.c_void_p()
    _check(_lib.load().transfer_plan_capture(plan.handle, steps, ctypes.byref(h)), "transfer_plan_capture")
    return TransferGraph(h.value, plan)


def transfer_plans_capture(plans, steps=1):
    """One graph of `steps` steps, each running the plans in order."""
    arr = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
    h = ctypes.c_void_p()
    _check(_lib.load().transfer_plans_capture(arr, len(plans), steps, ctypes.byref(h)),
           "transfer_plans_capture")
    return TransferGraph(h.value, list(plans))


def transfer_graph_launch(graph, stream=None):
    _check(_lib.load().transfer_graph_launch(graph._h, _stream_ptr(stream)), "transfer_graph_launch")
