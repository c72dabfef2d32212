"""Seeded random configurations against the oracle: patch size, halo depth,
scheme, direction, unknown count, face count and the (orientation, subface)
mix drawn from a fixed generator, so that combinations no hand-written case
names are covered too.  FP64 at 1e-12 relative; float32 storage on the
vector ALUs at 1e-5; float64 fine data restricted into float32 coarse faces
within one float32 rounding."""

import numpy as np
import pytest
import torch

from paper_2504_15814_amd import api
from paper_2504_15814_amd import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu


def _cases(n, seed=2504):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        scheme = int(rng.integers(1, 4))
        k = int(rng.integers(1, 4)) if scheme == 1 else int(rng.integers(2, 4))
        p = int(rng.integers(6, 15))
        U = int(rng.choice([1, 2, 7, 33, 59, 64, 65, 100, 130]))
        n_faces = int(rng.integers(1, 7))
        direction = int(rng.integers(0, 2))
        out.append((i, scheme, p, k, U, n_faces, direction))
    return out


CASES = _cases(24)


@pytest.fixture(scope="module")
def dev():
    return gh.require_gpu()


@pytest.mark.parametrize("case", CASES, ids=[f"c{c[0]}-s{c[1]}-p{c[2]}-k{c[3]}-U{c[4]}-n{c[5]}-d{c[6]}"
                                            for c in CASES])
def test_random_configuration_f64(dev, case):
    i, scheme, p, k, U, n_faces, direction = case
    batch = wl.uniform_faces(n_faces, p, k, U, seed=9000 + i, device=dev)
    gh.check_parity(direction, scheme, batch)


@pytest.mark.parametrize("case", CASES[:12], ids=[f"c{c[0]}" for c in CASES[:12]])
def test_random_configuration_f32(dev, case):
    i, scheme, p, k, U, n_faces, direction = case
    batch = wl.uniform_faces(n_faces, p, k, U, seed=9000 + i, device=dev)
    got, src, before = gh.run_gpu(direction, scheme, batch, torch.float32, mode=api.FT_F32)
    want, (o, s, doff) = gh.run_oracle(direction, scheme, batch, src, before)
    mask, copy = gh.written_mask(direction, scheme, p, k, U, o, s, doff, len(got))
    assert np.array_equal(got[~mask], before[~mask])
    assert np.array_equal(got[copy], want[copy])
    emax, _ = gh.rel_errors(got, want, mask, U)
    assert emax.max() < 1e-5


@pytest.mark.parametrize("case", [c for c in CASES if c[6] == 1],
                         ids=[f"c{c[0]}" for c in CASES if c[6] == 1])
def test_random_restriction_f64_to_f32(dev, case):
    """FT_F64_TO_F32 restriction of the float64 data: bitwise the FP64
    result rounded to float32, within 2^-24 |y| + 2e-12 max|y| of the oracle,
    injected values exact, untouched cells kept."""
    i, scheme, p, k, U, n_faces, _ = case
    batch = wl.uniform_faces(n_faces, p, k, U, seed=9000 + i, device=dev)
    op = api.build_transfer_operator(api.FT_RESTRICT, scheme, p, k)
    d = (batch.orientation, batch.subface, batch.coarse_offset, batch.fine_offset)
    got = torch.full(batch.coarse.shape, gh.SENTINEL, dtype=torch.float32, device=dev)
    ref = torch.full_like(batch.coarse, gh.SENTINEL)
    api.restrict_faces(op, *d, U, batch.fine, got, mode=api.FT_F64_TO_F32)
    api.restrict_faces(op, *d, U, batch.fine, ref)
    torch.cuda.synchronize()
    assert op.errors() == 0
    before = np.full(got.numel(), np.float32(gh.SENTINEL), dtype=np.float64)
    want, (o, s, co) = gh.run_oracle(1, scheme, batch, batch.fine.cpu().numpy(), before)
    mask, copy = gh.written_mask(1, scheme, p, k, U, o, s, co, len(want))
    g = got.double().cpu().numpy()
    assert np.array_equal(g[~mask], before[~mask])
    assert np.array_equal(g, ref.cpu().numpy().astype(np.float32).astype(np.float64))
    w = want[mask].reshape(-1, U)
    bound = 2.0**-24 * np.abs(w) + 2e-12 * np.abs(w).max(axis=0)
    assert (np.abs(g[mask].reshape(-1, U) - w) <= bound).all()
    assert np.array_equal(g[copy], want[copy].astype(np.float32).astype(np.float64))


def _patch_cases(n, seed=1581):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        scheme = int(rng.integers(1, 4))
        k = int(rng.integers(1, 4)) if scheme == 1 else int(rng.integers(2, 4))
        p = int(rng.integers(6, 14))
        U = int(rng.choice([1, 5, 31, 59, 66]))
        out.append((i, scheme, p, k, U))
    return out


PATCH_CASES = _patch_cases(10)


@pytest.mark.parametrize("case", PATCH_CASES, ids=[f"c{c[0]}-s{c[1]}-p{c[2]}-k{c[3]}-U{c[4]}"
                                                  for c in PATCH_CASES])
def test_random_patch_transfer_f64(dev, case):
    """Nine fine patches per coarse face, both directions, in place in the
    patch boxes, against the oracle's patch functions."""
    from oracle import patches as opt
    from tests.test_gpu_patches import npy, written_halo_mask

    i, scheme, p, k, U = case
    b = wl.patch_transitions(18, p, k, U, seed=7000 + i, device=dev, faces_per_coarse=9)
    o, s = b.orientation.cpu().numpy(), b.subface.cpu().numpy()
    co, fo = b.coarse_offset.cpu().numpy(), b.fine_offset.cpu().numpy()
    iop = api.build_transfer_operator(0, scheme, p, k)
    rop = api.build_transfer_operator(1, scheme, p, k)
    fine, coarse = b.fine.clone(), b.coarse.clone()
    api.interpolate_patches(iop, b.orientation, b.subface, b.coarse_offset, b.fine_offset, U, b.coarse, fine)
    api.restrict_patches(rop, b.orientation, b.subface, b.coarse_offset, b.fine_offset, U, b.fine, coarse)
    torch.cuda.synchronize()
    assert iop.errors() == 0 and rop.errors() == 0
    want_f = opt.interpolate_patches(scheme, p, k, o, s, co, fo, U, npy(b.coarse), npy(b.fine))
    want_c = opt.restrict_patches(scheme, p, k, o, s, co, fo, U, npy(b.fine), npy(b.coarse))
    mask_f = written_halo_mask(p, k, U, o, fo, b.fine.numel())
    mask_c = written_halo_mask(p, k, U, ((o.astype(np.int64) + 3) % 6)[::9], co[::9], b.coarse.numel())
    for got, want, before, mask in ((npy(fine), want_f, npy(b.fine), mask_f),
                                    (npy(coarse), want_c, npy(b.coarse), mask_c)):
        assert np.array_equal(got[~mask], before[~mask])
        d = np.abs(got[mask] - want[mask]).reshape(-1, U).max(axis=0)
        scale = np.abs(want[mask]).reshape(-1, U).max(axis=0)
        assert (d / scale).max() <= 1e-12
