"""Two-dimensional faces (FT_BUILD_2D) on the GPU against the
two-dimensional oracle, through the C ABI: float64 to 1e-12 per unknown,
exact-copy rows and unwritten cells bit for bit, the float32 modes within
their per-element rounding bounds, bad descriptors skipped and counted."""

import numpy as np
import pytest
import torch

from oracle import transfer2d as o2
from paper_2504_15814_amd import api
from paper_2504_15814_amd.workloads import faces_2d
from tests.gpu_helpers import SENTINEL, require_gpu

pytestmark = pytest.mark.gpu

# per-element bounds of the float32 modes, times sum |w x| (as for 3D faces)
C = {api.FT_F32: 35 * 2.0**-24, api.FT_F32_BF16X3: 3 * 2.0**-16 + 9 * 2.0**-24, api.FT_F32_BF16X6: 21 * 2.0**-24}


def run(direction, scheme, b, dtype, mode=None):
    op = api.build_transfer_operator(direction, scheme, b.p, b.k, api.FT_BUILD_2D)
    src = (b.coarse if direction == 0 else b.fine).to(dtype)
    dst = torch.full_like((b.fine if direction == 0 else b.coarse).to(dtype), SENTINEL)
    before = dst.double().cpu().numpy()
    args = (op, b.orientation, b.subface, b.coarse_offset, b.fine_offset, b.U)
    if direction == 0:
        api.interpolate_faces(*args, src, dst, mode=mode)
    else:
        api.restrict_faces(*args, src, dst, mode=mode)
    torch.cuda.synchronize()
    assert op.errors() == 0
    return dst.double().cpu().numpy(), src.double().cpu().numpy(), before


def oracle_out(direction, scheme, b, src, before, absolute=False):
    o, s = b.orientation.cpu().numpy(), b.subface.cpu().numpy()
    co, fo = b.coarse_offset.cpu().numpy(), b.fine_offset.cpu().numpy()
    out = np.array(before, copy=True)
    mask = np.zeros(len(before), dtype=bool)
    copy = np.zeros(len(before), dtype=bool)
    ncell, U = 2 * b.k * b.p, b.U
    for f in range(len(o)):
        rows, W = o2.transfer_operator(direction, scheme, b.p, b.k, int(o[f]), int(s[f]))
        so, do = (co[f], fo[f]) if direction == 0 else (fo[f], co[f])
        x = src[so : so + ncell * U].reshape(ncell, U)
        y = out[do : do + ncell * U].reshape(ncell, U)
        y[rows] = (np.abs(W) @ np.abs(x)) if absolute else (W @ x)
        idx = do + rows[:, None] * U + np.arange(U)[None, :]
        mask[idx.ravel()] = True
        single = (np.count_nonzero(W, axis=1) == 1) & (W.max(axis=1) == 1.0)
        copy[(do + rows[single][:, None] * U + np.arange(U)[None, :]).ravel()] = True
    return out, mask, copy


CASES = [(s, p, k) for s in (1, 2, 3) for p, k in ((6, 2), (9, 3), (12, 3), (8, 3), (10, 2))] + \
    [(1, 9, 1), (1, 12, 1), (1, 7, 1)]


@pytest.mark.parametrize("scheme,p,k", CASES)
@pytest.mark.parametrize("U", [1, 59, 70])
def test_2d_parity_f64(scheme, p, k, U):
    dev = require_gpu()
    b = faces_2d(60, p, k, U, seed=10 * p + k + U + scheme, device=dev)
    for direction in (0, 1):
        got, src, before = run(direction, scheme, b, torch.float64)
        want, mask, copy = oracle_out(direction, scheme, b, src, before)
        assert np.array_equal(got[~mask], before[~mask])
        assert np.array_equal(got[copy], want[copy])
        d = np.abs(got[mask] - want[mask]).reshape(-1, U).max(axis=0)
        assert (d / np.abs(want[mask]).reshape(-1, U).max(axis=0)).max() <= 1e-12


@pytest.mark.parametrize("mode", [api.FT_F32, api.FT_F32_BF16X3, api.FT_F32_BF16X6])
@pytest.mark.parametrize("scheme,p,k", [(1, 9, 3), (2, 9, 3), (3, 9, 3), (3, 6, 2), (1, 9, 1), (3, 8, 3)])
def test_2d_float32_modes(mode, scheme, p, k):
    dev = require_gpu()
    U = 59
    b = faces_2d(40, p, k, U, seed=500 + mode + p + k, device=dev)
    got, src, before = run(0, scheme, b, torch.float32, mode=mode)
    want, mask, copy = oracle_out(0, scheme, b, src, before)
    scale, _, _ = oracle_out(0, scheme, b, src, before, absolute=True)
    bound = C[mode] * scale + 2.0**-24 * np.abs(want)
    err = np.abs(got - want)
    assert np.all(err[mask] <= bound[mask])
    assert np.array_equal(got[copy], want[copy])
    assert np.array_equal(got[~mask], before[~mask])
    # restriction in float32 storage sums in float64: one rounding
    got, src, before = run(1, scheme, b, torch.float32, mode=mode)
    want, mask, _ = oracle_out(1, scheme, b, src, before)
    assert np.all(np.abs(got[mask] - want[mask]) <= 2.0**-24 * np.abs(want[mask]) + 1e-12 * np.abs(want[mask]).max())


def test_2d_bad_descriptors_and_scope():
    dev = require_gpu()
    p, k, U = 9, 3, 5
    b = faces_2d(4, p, k, U, seed=3, device=dev)
    op = api.build_transfer_operator(0, 3, p, k, api.FT_BUILD_2D)
    o = b.orientation.clone()
    s = b.subface.clone()
    o[1] = 4  # out of range in 2D
    s[2] = 3
    dst = torch.full_like(b.fine, SENTINEL)
    api.interpolate_faces(op, o, s, b.coarse_offset, b.fine_offset, U, b.coarse, dst)
    torch.cuda.synchronize()
    assert op.errors() == 2
    fe = 2 * k * p * U
    got = dst.cpu().numpy()
    assert np.all(got[fe : 3 * fe] == SENTINEL)
    # plans and patch calls take three-dimensional operators only
    with pytest.raises(api.FTError):
        api.build_transfer_plan([(op, b.orientation, b.subface, b.coarse_offset, b.fine_offset)], U,
                                b.coarse.clone(), b.fine.clone())
    with pytest.raises(api.FTError):
        api.interpolate_patches(op, b.orientation, b.subface, b.coarse_offset, b.fine_offset, U, b.coarse, dst)
