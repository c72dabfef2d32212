"""Shared helpers for GPU parity tests: run the HIP path through the C ABI and
the oracle on the same inputs, and compare."""

import numpy as np
import torch

import oracle
from paper_2504_15814_amd import api

SENTINEL = -7.25e11


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch.device("cuda:0")


def written_mask(direction, scheme, p, k, U, orientation, subface, dst_offset, dst_len):
    """Boolean mask of the destination elements a transfer writes, and the
    positions of exact-copy rows, from the oracle's operators."""
    mask = np.zeros(dst_len, dtype=bool)
    copy = np.zeros(dst_len, dtype=bool)
    u = np.arange(U)
    for f in range(len(orientation)):
        rows, W = oracle.transfer_operator(direction, scheme, p, k, int(orientation[f]), int(subface[f]))
        base = int(dst_offset[f])
        idx = base + rows[:, None] * U + u[None, :]
        mask[idx.ravel()] = True
        single = (np.count_nonzero(W, axis=1) == 1) & (W.max(axis=1) == 1.0)
        copy[(base + rows[single][:, None] * U + u[None, :]).ravel()] = True
    return mask, copy


def run_gpu(direction, scheme, batch, dtype=torch.float64, op=None, mode=None):
    """Apply the HIP path; returns (destination after the call as float64
    numpy, source as float64 numpy, destination before the call)."""
    dev = batch.coarse.device
    coarse = batch.coarse.to(dtype)
    fine = batch.fine.to(dtype)
    if op is None:
        op = api.build_transfer_operator(direction, scheme, batch.p, batch.k)
    if direction == 0:
        dst = torch.full_like(fine, SENTINEL)
        before = dst.clone()
        api.interpolate_faces(op, batch.orientation, batch.subface, batch.coarse_offset,
                              batch.fine_offset, batch.U, coarse, dst, mode=mode)
        src = coarse
    else:
        dst = torch.full_like(coarse, SENTINEL)
        before = dst.clone()
        api.restrict_faces(op, batch.orientation, batch.subface, batch.coarse_offset,
                           batch.fine_offset, batch.U, fine, dst, mode=mode)
        src = fine
    torch.cuda.synchronize(dev)
    assert op.errors() == 0
    return (dst.double().cpu().numpy(), src.double().cpu().numpy(), before.double().cpu().numpy())


def run_oracle(direction, scheme, batch, src, before, faces=None):
    """Oracle output for the given faces (default all) on the same source."""
    o = batch.orientation.cpu().numpy()
    s = batch.subface.cpu().numpy()
    co = batch.coarse_offset.cpu().numpy()
    fo = batch.fine_offset.cpu().numpy()
    if faces is not None:
        o, s, co, fo = o[faces], s[faces], co[faces], fo[faces]
    if direction == 0:
        return oracle.interpolate_faces(scheme, batch.p, batch.k, o, s, co, fo, batch.U, src, before), (o, s, fo)
    return oracle.restrict_faces(scheme, batch.p, batch.k, o, s, co, fo, batch.U, src, before), (o, s, co)


def rel_errors(got, want, mask, U):
    """Per-unknown max and RMS error relative to the largest / RMS expected
    value over the written elements."""
    g = got[mask].reshape(-1, U)
    w = want[mask].reshape(-1, U)
    d = np.abs(g - w)
    emax = d.max(axis=0) / np.maximum(np.abs(w).max(axis=0), 1e-300)
    erms = np.sqrt((d**2).mean(axis=0)) / np.maximum(np.sqrt((w**2).mean(axis=0)), 1e-300)
    return emax, erms


def check_parity(direction, scheme, batch, dtype=torch.float64, tol=1e-12, faces=None, op=None):
    got, src, before = run_gpu(direction, scheme, batch, dtype, op=op)
    want, (o, s, doff) = run_oracle(direction, scheme, batch, src, before, faces)
    mask, copy = written_mask(direction, scheme, batch.p, batch.k, batch.U, o, s, doff, len(got))
    if faces is None:
        # everything not written keeps its sentinel, bit for bit
        assert np.array_equal(got[~mask], before[~mask])
    emax, erms = rel_errors(got, want, mask, batch.U)
    assert emax.max() <= tol, (emax.max(), erms.max())
    # exact-copy rows are bit-exact
    assert np.array_equal(got[copy], want[copy])
    return emax, erms


def abs_weighted_sums(direction, scheme, batch, src, dst_len, faces=None):
    """Per destination element, sum_q |w_q x_q| from the oracle's operators
    (the scale of the rounding error of any evaluation order)."""
    out = np.zeros(dst_len)
    o = batch.orientation.cpu().numpy()
    s = batch.subface.cpu().numpy()
    so = (batch.coarse_offset if direction == 0 else batch.fine_offset).cpu().numpy()
    do = (batch.fine_offset if direction == 0 else batch.coarse_offset).cpu().numpy()
    U = batch.U
    ncell = 2 * batch.k * batch.p * batch.p
    for f in (range(len(o)) if faces is None else faces):
        rows, W = oracle.transfer_operator(direction, scheme, batch.p, batch.k, int(o[f]), int(s[f]))
        x = np.abs(src[int(so[f]): int(so[f]) + ncell * U].reshape(ncell, U))
        y = out[int(do[f]): int(do[f]) + ncell * U].reshape(ncell, U)
        y[rows] = np.abs(W) @ x
    return out
