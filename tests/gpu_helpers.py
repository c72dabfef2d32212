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


# ---------------------------------------------------------------------------
# Full-size checks: every face on the device, a sample against the oracle
# ---------------------------------------------------------------------------
def local_written(direction, scheme, p, k, U, o, s, dim=3):
    """Element indices, relative to a face's destination offset, that one
    face of orientation o and subface s writes (the oracle's operator rows)."""
    if dim == 3:
        rows, _ = oracle.transfer_operator(direction, scheme, p, k, int(o), int(s))
    else:
        rows, _ = oracle.transfer2d.transfer_operator(direction, scheme, p, k, int(o), int(s))
    return (np.asarray(rows)[:, None] * U + np.arange(U)[None, :]).ravel()


def device_written_mask(direction, scheme, p, k, U, orientation, subface, dst_offset, dst_len,
                        device, dim=3, chunk=2048):
    """Boolean device tensor over the destination array: True where some face
    of the batch writes.  Built per (orientation, subface) group from the
    oracle's rows, in chunks of faces."""
    o = orientation.cpu().numpy().astype(np.int64)
    s = subface.cpu().numpy().astype(np.int64)
    offs = dst_offset.to(device)
    mask = torch.zeros(dst_len, dtype=torch.bool, device=device)
    key = o * 16 + s
    for kv in np.unique(key):
        faces = torch.from_numpy(np.flatnonzero(key == kv)).to(device)
        loc = torch.from_numpy(local_written(direction, scheme, p, k, U, kv // 16, kv % 16, dim)).to(device)
        for c0 in range(0, faces.numel(), chunk):
            idx = offs[faces[c0:c0 + chunk]][:, None] + loc[None, :]
            mask[idx.reshape(-1)] = True
    return mask


def _bits(t):
    return t.view(torch.int64) if t.dtype == torch.float64 else t.view(torch.int32)


def check_written_region(dst, before, mask, chunk=1 << 28):
    """On the device, over the whole destination: every element in `mask`
    differs from `before` (a sentinel fill, so every written element was
    written) and every element outside it is bit-identical to `before`."""
    d, b = _bits(dst), _bits(before)
    for c0 in range(0, d.numel(), chunk):
        dd, bb, mm = d[c0:c0 + chunk], b[c0:c0 + chunk], mask[c0:c0 + chunk]
        same = dd == bb
        assert not bool((same & mm).any()), "an element of a written half kept its sentinel"
        assert not bool((~same & ~mm).any()), "an element outside the written halves changed"


def compact_faces(t, offsets, faces, elems):
    """Host float64 copy of `elems` elements at offsets[f] for the sampled
    faces, back to back (face i at i * elems)."""
    offs = offsets.cpu().numpy()
    return np.concatenate([t[int(offs[f]):int(offs[f]) + elems].double().cpu().numpy() for f in faces])


def compact_batch(batch, faces, coarse=None, fine=None):
    """A host FaceBatch holding the sampled faces' coarse and fine buffers
    (or the given tensors instead), each face at i * face_elems."""
    from paper_2504_15814_amd import workloads as wl

    E = batch.face_elems
    offs = torch.arange(len(faces), dtype=torch.int64) * E
    c = compact_faces(batch.coarse if coarse is None else coarse, batch.coarse_offset, faces, E)
    f = compact_faces(batch.fine if fine is None else fine, batch.fine_offset, faces, E)
    sel = torch.from_numpy(np.asarray(faces, dtype=np.int64))
    return wl.FaceBatch(batch.p, batch.k, batch.U, batch.orientation.cpu()[sel].contiguous(),
                        batch.subface.cpu()[sel].contiguous(), offs, offs.clone(),
                        torch.from_numpy(c), torch.from_numpy(f))


def run_gpu_device(direction, scheme, batch, dtype=torch.float64, op=None, mode=None):
    """Apply the HIP path into a sentinel-filled destination; returns
    (destination, source, sentinel copy) as device tensors."""
    coarse = batch.coarse.to(dtype)
    fine = batch.fine.to(dtype)
    if op is None:
        op = api.build_transfer_operator(direction, scheme, batch.p, batch.k)
    src = coarse if direction == 0 else fine
    dst = torch.full_like(fine if direction == 0 else coarse, SENTINEL)
    if direction == 0:
        api.interpolate_faces(op, batch.orientation, batch.subface, batch.coarse_offset,
                              batch.fine_offset, batch.U, coarse, dst, mode=mode)
    else:
        api.restrict_faces(op, batch.orientation, batch.subface, batch.coarse_offset,
                           batch.fine_offset, batch.U, fine, dst, mode=mode)
    torch.cuda.synchronize(dst.device)
    assert op.errors() == 0
    return dst, src, torch.full_like(dst, SENTINEL)


def check_full_size(direction, scheme, batch, dst, before, faces, tol=1e-12, src=None):
    """Whole-batch region check on the device plus an oracle comparison of
    the sampled faces (their buffers copied out compactly)."""
    dst_off = batch.fine_offset if direction == 0 else batch.coarse_offset
    mask = device_written_mask(direction, scheme, batch.p, batch.k, batch.U, batch.orientation,
                               batch.subface, dst_off, dst.numel(), dst.device)
    check_written_region(dst, before, mask)
    del mask
    if direction == 0:
        cb = compact_batch(batch, faces, coarse=src)
    else:
        cb = compact_batch(batch, faces, fine=src)
    got = compact_faces(dst, dst_off, faces, batch.face_elems)
    src_np = (cb.coarse if direction == 0 else cb.fine).numpy()
    before_np = compact_faces(before, dst_off, faces, batch.face_elems)
    want, (o, s, doff) = run_oracle(direction, scheme, cb, src_np, before_np)
    m, copy = written_mask(direction, scheme, cb.p, cb.k, cb.U, o, s, doff, len(got))
    assert np.array_equal(got[~m], before_np[~m])
    emax, erms = rel_errors(got, want, m, cb.U)
    assert emax.max() <= tol, (emax.max(), erms.max())
    assert np.array_equal(got[copy], want[copy])
    return emax
