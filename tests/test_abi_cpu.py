"""C-ABI checks that need no GPU: the library loads and exports every
declared symbol, host-side argument checks return the documented codes, and
the host-built weight tables with their orientation maps equal the oracle's
operators (maps bit-exact, weights to 1e-13 of the row's 1-norm)."""

import ctypes
import os
import re
from itertools import product

import numpy as np
import pytest

import oracle
from paper_2504_15814_amd import _lib, api
from paper_2504_15814_amd.build import lib_path

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "facetransfer.h")

pytestmark = pytest.mark.skipif(not os.path.exists(lib_path()), reason="library not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_functions()
    assert "interpolate_faces" in names and "restrict_faces" in names and "build_transfer_operator" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES)


def test_binding_constants_match_the_header():
    defines = dict(re.findall(r"^#define (FT_\w+) (\d+)", open(HEADER).read(), flags=re.M))
    assert "FT_F64_TO_F32" in defines and "FT_PLAN_PATCHES" in defines
    for name, value in defines.items():
        assert getattr(api, name) == int(value), name


def test_version_and_empty_error():
    assert api.transfer_version() == 200
    assert isinstance(api.transfer_last_error(), str)


@pytest.mark.parametrize(
    "args,code",
    [
        ((2, 2, 9, 3), api.FT_ERR_INVALID),   # bad direction
        ((0, 4, 9, 3), api.FT_ERR_INVALID),   # bad scheme
        ((0, 2, 3, 3), api.FT_ERR_UNSUPPORTED),   # p too small
        ((0, 2, 51, 3), api.FT_ERR_UNSUPPORTED),  # p too large
        ((0, 2, 9, 1), api.FT_ERR_UNSUPPORTED),   # k = 1
        ((0, 2, 9, 4), api.FT_ERR_UNSUPPORTED),   # k = 4
    ],
)
def test_build_rejects_bad_arguments(args, code):
    lib = _lib.load()
    h = ctypes.c_void_p(123)
    rc = lib.build_transfer_operator(*args, api.FT_BUILD_HOST_ONLY, ctypes.byref(h))
    assert rc == code
    assert h.value is None
    assert api.transfer_last_error() != ""


def test_build_rejects_null_out_and_bad_flags():
    lib = _lib.load()
    assert lib.build_transfer_operator(0, 2, 9, 3, 1, None) == api.FT_ERR_INVALID
    h = ctypes.c_void_p()
    assert lib.build_transfer_operator(0, 2, 9, 3, 8, ctypes.byref(h)) == api.FT_ERR_INVALID


def test_apply_checks_happen_on_host():
    """Every rejection below happens before any HIP call."""
    lib = _lib.load()
    op = api.build_transfer_operator(0, 2, 9, 3, api.FT_BUILD_HOST_ONLY)
    rop = api.build_transfer_operator(1, 2, 9, 3, api.FT_BUILD_HOST_ONLY)
    p = ctypes.c_void_p(16)
    args = (1, p, p, p, p, 59, 0, p, 10**6, ctypes.c_void_p(32), 10**6, None)
    assert lib.interpolate_faces(None, *args) == api.FT_ERR_INVALID
    assert lib.interpolate_faces(rop.handle, *args) == api.FT_ERR_INVALID  # wrong direction
    assert lib.restrict_faces(op.handle, *args) == api.FT_ERR_INVALID
    assert lib.interpolate_faces(op.handle, *args) == api.FT_ERR_INVALID  # host-only operator
    assert "host-only" in api.transfer_last_error()
    n = ctypes.c_int64()
    assert lib.transfer_operator_errors(op.handle, ctypes.byref(n), 0) == api.FT_ERR_INVALID
    assert lib.transfer_operator_info(None, None, 0) == api.FT_ERR_INVALID
    assert lib.transfer_operator_segment(op.handle, 6, 0, 0, None, None, None, ctypes.byref(n)) == api.FT_ERR_INVALID
    assert lib.transfer_operator_segment(op.handle, 0, 9, 0, None, None, None, ctypes.byref(n)) == api.FT_ERR_INVALID
    assert lib.destroy_transfer_operator(None) == api.FT_OK
    op.destroy()
    rop.destroy()


def test_info_counts():
    op = api.build_transfer_operator(0, 3, 9, 3, api.FT_BUILD_HOST_ONLY)
    info = op.info()
    assert info["rows_per_anchor"] == 27 and info["anchors"] == 9
    assert info["blocks"] == 25 and 30 <= info["max_width"] <= 33
    rop = api.build_transfer_operator(1, 3, 9, 3, api.FT_BUILD_HOST_ONLY)
    assert rop.info()["rows_per_anchor"] == 3 and rop.info()["blocks"] == 9


def _dense(op, o, s, p, k):
    rows, cols, vals = op.segment(o, s)
    ncell = 2 * k * p * p
    D = np.zeros((ncell, ncell))
    np.add.at(D, (rows, cols), vals)
    return set(rows.tolist()), D


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2, 3])
@pytest.mark.parametrize("p,k", [(6, 2), (6, 3), (9, 2), (9, 3), (12, 2), (12, 3)])
def test_library_segments_equal_oracle(direction, scheme, p, k):
    op = api.build_transfer_operator(direction, scheme, p, k, api.FT_BUILD_HOST_ONLY)
    subfaces = range(9)
    for o, s in product(range(6), subfaces):
        rows_lib, D = _dense(op, o, s, p, k)
        rows, W = oracle.transfer_operator(direction, scheme, p, k, o, s)
        assert rows_lib == set(rows.tolist())  # destination map, exact
        got = D[rows]
        scale = np.abs(W).sum(axis=1)
        err = (np.abs(got - W).max(axis=1) / scale).max()
        assert err < 1e-13, (o, s, err)
        # source map: every oracle weight above rounding level is present
        big = np.abs(W) > 1e-12 * scale[:, None]
        assert np.all(got[big] != 0.0)


def test_copy_rows_are_unit_weights():
    """Rows whose centres coincide hold a single weight of exactly 1."""
    for direction, scheme in ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3)):
        op = api.build_transfer_operator(direction, scheme, 9, 3, api.FT_BUILD_HOST_ONLY)
        rows, cols, vals = op.segment(1, 4)
        ones = np.flatnonzero(vals == 1.0)
        per_row = np.bincount(rows, minlength=rows.max() + 1)
        singles = [r for r in np.unique(rows) if per_row[r] == 1]
        assert len(singles) == 9
        assert set(rows[ones]) >= set(singles)


def test_apply_without_gpu_fails_cleanly():
    """Building for the device on a machine without a GPU reports FT_ERR_HIP."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib.load()
    h = ctypes.c_void_p()
    rc = lib.build_transfer_operator(0, 2, 9, 3, 0, ctypes.byref(h))
    assert rc == api.FT_ERR_HIP
    assert h.value is None


def test_plan_checks_happen_on_host():
    lib = _lib.load()
    h = ctypes.c_void_p()
    p = ctypes.c_void_p(64)
    assert lib.build_transfer_plan(None, 1, 59, 0, p, 100, ctypes.c_void_p(128), 100, 0, ctypes.byref(h)) == api.FT_ERR_INVALID
    op = api.build_transfer_operator(0, 2, 9, 3, api.FT_BUILD_HOST_ONLY)
    arr = (_lib.PlanBatch * 1)()
    arr[0] = _lib.PlanBatch(op.handle, 1, 8, 8, 8, 8)
    rc = lib.build_transfer_plan(arr, 1, 59, 0, p, 100, ctypes.c_void_p(128), 100, 0, ctypes.byref(h))
    assert rc in (api.FT_ERR_INVALID, api.FT_ERR_HIP)  # host-only operator (or no device at all)
    assert lib.build_transfer_plan(arr, 0, 59, 0, p, 100, ctypes.c_void_p(128), 100, 0, ctypes.byref(h)) == api.FT_ERR_INVALID
    assert lib.build_transfer_plan(arr, 1, 0, 0, p, 100, ctypes.c_void_p(128), 100, 0, ctypes.byref(h)) == api.FT_ERR_UNSUPPORTED
    assert lib.build_transfer_plan(arr, 1, 59, 9, p, 100, ctypes.c_void_p(128), 100, 0, ctypes.byref(h)) == api.FT_ERR_UNSUPPORTED
    assert lib.build_transfer_plan(arr, 1, 59, 0, p, 100, p, 100, 0, ctypes.byref(h)) == api.FT_ERR_INVALID
    assert lib.run_transfer_plan(None, None) == api.FT_ERR_INVALID
    assert lib.transfer_plan_set_schedule(None, 4) == api.FT_ERR_INVALID
    assert lib.transfer_plan_capture(None, 1, ctypes.byref(h)) == api.FT_ERR_INVALID
    assert lib.transfer_plans_capture(None, 1, 1, ctypes.byref(h)) == api.FT_ERR_INVALID
    plans = (ctypes.c_void_p * 1)(None)
    assert lib.transfer_plans_capture(plans, 0, 1, ctypes.byref(h)) == api.FT_ERR_INVALID
    assert lib.transfer_plans_capture(plans, 1, 0, ctypes.byref(h)) == api.FT_ERR_INVALID
    # float64 fine into float32 coarse data: face buffers only, checked first
    assert lib.build_transfer_plan(arr, 1, 59, api.FT_F64_TO_F32, p, 100, ctypes.c_void_p(128), 100,
                                   api.FT_PLAN_PATCHES, ctypes.byref(h)) == api.FT_ERR_UNSUPPORTED
    assert lib.build_transfer_plan(arr, 1, 59, api.FT_F64_TO_F32 + 1, p, 100, ctypes.c_void_p(128), 100, 0,
                                   ctypes.byref(h)) == api.FT_ERR_UNSUPPORTED
    assert lib.transfer_graph_launch(None, None) == api.FT_ERR_INVALID
    assert lib.destroy_transfer_plan(None) == api.FT_OK
    assert lib.destroy_transfer_graph(None) == api.FT_OK


def test_schedule_packing_roundtrip():
    s = api.pack_schedule(2, 16, 1, 1, 0)
    assert api.unpack_schedule(s) == {"waves_per_block": 2, "blocks_per_cu": 16, "xcd_remap": 1, "heavy_first": 1,
                                      "persistent": 0}


def test_patch_copy_checks_happen_on_host():
    """Host-side rejections of the patch / face-buffer copies (nothing is
    launched: every case fails before a HIP call)."""
    lib = _lib.load()
    q = ctypes.c_void_p(16)
    r = ctypes.c_void_p(32)

    def gather(p=9, k=3, n=1, sel=q, halves=api.FT_HALF_BOTH, U=59, dtype=0, src=q, dst=r):
        return lib.gather_patch_faces(p, k, n, sel, q, q, halves, U, dtype, src, 10**6, dst, 10**6, None, None)

    assert gather(p=0) == api.FT_ERR_UNSUPPORTED
    assert gather(k=0) == api.FT_ERR_UNSUPPORTED
    assert gather(p=2, k=3) == api.FT_ERR_UNSUPPORTED  # k > p
    assert gather(U=0) == api.FT_ERR_UNSUPPORTED
    assert gather(dtype=7) == api.FT_ERR_UNSUPPORTED
    assert gather(halves=0) == api.FT_ERR_INVALID
    assert gather(halves=4) == api.FT_ERR_INVALID
    assert gather(n=-1) == api.FT_ERR_INVALID
    assert gather(sel=None) == api.FT_ERR_INVALID
    assert gather(src=r) == api.FT_ERR_INVALID  # alias
    assert gather(n=0, sel=None) == api.FT_OK  # empty call is a no-op
    assert lib.scatter_patch_faces(9, 3, 1, q, q, q, 3, 59, 0, q, 10**6, q, 10**6, None, None) == api.FT_ERR_INVALID
    assert lib.copy_patch_halos(9, 3, 1, None, q, q, 59, 0, q, 10**6, None, None) == api.FT_ERR_INVALID
    assert lib.copy_patch_halos(9, 0, 1, q, q, q, 59, 0, q, 10**6, None, None) == api.FT_ERR_UNSUPPORTED
    assert lib.copy_patch_halos(9, 3, 0, None, None, None, 59, 0, q, 10**6, None, None) == api.FT_OK


def test_patch_transfer_needs_device_operator():
    lib = _lib.load()
    op = api.build_transfer_operator(0, 3, 9, 3, api.FT_BUILD_HOST_ONLY)
    rop = api.build_transfer_operator(1, 3, 9, 3, api.FT_BUILD_HOST_ONLY)
    p = ctypes.c_void_p(16)
    args = (1, p, p, p, p, 59, 0, p, 10**6, p, 10**6, None)
    assert lib.interpolate_patches(op.handle, *args) == api.FT_ERR_INVALID  # host-only operator
    assert lib.interpolate_patches(rop.handle, *args) == api.FT_ERR_INVALID  # wrong direction
    assert lib.restrict_patches(op.handle, *args) == api.FT_ERR_INVALID
    assert lib.interpolate_patches(None, *args) == api.FT_ERR_INVALID


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("p", [6, 9, 12])
def test_library_segments_equal_oracle_k1(direction, p):
    """Halo depth 1 (finite volumes), d-linear: maps exact, weights equal."""
    test_library_segments_equal_oracle(direction, 1, p, 1)


def test_k1_only_for_dlinear():
    lib = _lib.load()
    h = ctypes.c_void_p()
    for scheme in (2, 3):
        assert lib.build_transfer_operator(0, scheme, 9, 1, api.FT_BUILD_HOST_ONLY, ctypes.byref(h)) == api.FT_ERR_UNSUPPORTED
    op = api.build_transfer_operator(0, 1, 9, 1, api.FT_BUILD_HOST_ONLY)
    info = op.info()
    assert info["rows_per_anchor"] == 9 and info["k"] == 1
    rop = api.build_transfer_operator(1, 1, 9, 1, api.FT_BUILD_HOST_ONLY)
    assert rop.info()["rows_per_anchor"] == 1


# Two-dimensional operators (FT_BUILD_2D) against the two-dimensional oracle.


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme,p,k", [(s, p, k) for s in (1, 2, 3) for p in (6, 9, 12) for k in (2, 3)]
                         + [(1, p, 1) for p in (6, 9, 12)])
def test_library_2d_segments_equal_oracle(direction, scheme, p, k):
    op = api.build_transfer_operator(direction, scheme, p, k, api.FT_BUILD_HOST_ONLY | api.FT_BUILD_2D)
    ncell = 2 * k * p
    for o, s in product(range(4), range(3)):
        rows_l, cols_l, vals_l = op.segment(o, s)
        D = np.zeros((ncell, ncell))
        np.add.at(D, (rows_l, cols_l), vals_l)
        rows, W = oracle.transfer2d.transfer_operator(direction, scheme, p, k, o, s)
        assert set(rows_l.tolist()) == set(rows.tolist())
        got = D[rows]
        scale = np.abs(W).sum(axis=1)
        assert (np.abs(got - W).max(axis=1) / scale).max() < 1e-13, (o, s)
        big = np.abs(W) > 1e-12 * scale[:, None]
        assert np.all(got[big] != 0.0)


def test_2d_info_and_ranges():
    op = api.build_transfer_operator(0, 3, 9, 3, api.FT_BUILD_HOST_ONLY | api.FT_BUILD_2D)
    info = op.info()
    assert info["dim"] == 2 and info["rows_per_anchor"] == 9 and info["anchors"] == 3
    assert info["blocks"] == 5
    assert api.build_transfer_operator(0, 3, 9, 3, api.FT_BUILD_HOST_ONLY).info()["dim"] == 3
    lib = _lib.load()
    n = ctypes.c_int64()
    assert lib.transfer_operator_segment(op.handle, 4, 0, 0, None, None, None, ctypes.byref(n)) == api.FT_ERR_INVALID
    assert lib.transfer_operator_segment(op.handle, 0, 3, 0, None, None, None, ctypes.byref(n)) == api.FT_ERR_INVALID
    h = ctypes.c_void_p()
    assert lib.build_transfer_operator(0, 2, 9, 1, api.FT_BUILD_HOST_ONLY | api.FT_BUILD_2D, ctypes.byref(h)) == api.FT_ERR_UNSUPPORTED


# Patch sizes that are not multiples of 3.


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2, 3])
@pytest.mark.parametrize("p,k", [(7, 2), (8, 3), (10, 2), (11, 3)])
def test_library_segments_equal_oracle_general_p(direction, scheme, p, k):
    test_library_segments_equal_oracle(direction, scheme, p, k)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("p", [7, 8, 10])
def test_library_segments_equal_oracle_general_p_k1_and_2d(direction, p):
    test_library_segments_equal_oracle(direction, 1, p, 1)
    for scheme, k in ((1, 1), (2, 2), (3, 3)):
        test_library_2d_segments_equal_oracle(direction, scheme, p, k)


def test_general_p_anchor_counts():
    """Anchors per axis: p / 3 for multiples of 3; otherwise the largest
    number of coarse columns a subface touches (interpolation) or holds the
    centres of (restriction)."""
    for p, ei, er in ((6, 2, 2), (9, 3, 3), (7, 3, 3), (8, 4, 3), (10, 4, 4), (11, 5, 4)):
        assert api.build_transfer_operator(0, 2, p, 2, api.FT_BUILD_HOST_ONLY).info()["anchors"] == ei * ei
        assert api.build_transfer_operator(1, 2, p, 2, api.FT_BUILD_HOST_ONLY).info()["anchors"] == er * er


def test_binding_rejects_host_tensors_before_any_call():
    """The binding hands the library only contiguous tensors on the current
    GPU: host tensors are refused in Python, before the C ABI is reached."""
    import torch

    op = api.build_transfer_operator(0, 2, 9, 3, api.FT_BUILD_HOST_ONLY)
    o = torch.zeros(2, dtype=torch.int8)
    off = torch.zeros(2, dtype=torch.int64)
    buf = torch.zeros(2 * 6 * 81 * 3, dtype=torch.float64)
    for fn in (api.interpolate_faces, api.restrict_faces, api.interpolate_patches, api.restrict_patches):
        with pytest.raises(TypeError, match="GPU"):
            fn(op, o, o, off, off, 3, buf, buf.clone())
    with pytest.raises(TypeError, match="GPU"):
        api.gather_patch_faces(9, 3, o, off, off, api.FT_HALF_BOTH, 3, buf, buf.clone())
    with pytest.raises(TypeError):
        api.interpolate_faces(op, o.numpy(), o, off, off, 3, buf, buf.clone())
    with pytest.raises(TypeError):
        api.gather_patch_faces(9, 3, o, off, off, api.FT_HALF_BOTH, 3, buf, buf.clone(),
                               skipped=torch.zeros(1, dtype=torch.int64))
