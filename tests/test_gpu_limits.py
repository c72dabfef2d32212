"""The largest supported sizes on the GPU against the oracle: p = 48 (16 x 16
anchors per subface, the generic anchor-count path) and U = 4096 (64 chunks of
64 unknowns per wave), in float64 and in the float32 modes, plus a patch of
the largest size."""

import numpy as np
import pytest
import torch

import oracle
from oracle import patches as opt
from paper_2504_15814_amd import api
from paper_2504_15814_amd import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def small_oracle_cache():
    # one p = 48 segment is a dense 6912 x 13824 matrix: drop them after use
    oracle.clear_operator_cache()
    yield
    oracle.clear_operator_cache()


@pytest.mark.parametrize("scheme", [1, 3])
@pytest.mark.parametrize("direction", [0, 1])
def test_largest_patch_size(scheme, direction):
    dev = gh.require_gpu()
    batch = wl.uniform_faces(2, 48, 3, 3, seed=48 + scheme + direction, device=dev)
    gh.check_parity(direction, scheme, batch)


@pytest.mark.parametrize("mode", [None, api.FT_F32, api.FT_F32_BF16X6])
def test_largest_unknown_count(mode):
    dev = gh.require_gpu()
    U = 4096
    batch = wl.uniform_faces(3, 6, 2, U, seed=4096, device=dev)
    for direction in (0, 1):
        if mode is None:
            gh.check_parity(direction, 3, batch)
            continue
        got, src, before = gh.run_gpu(direction, 3, batch, torch.float32, mode=mode)
        want, (o, s, doff) = gh.run_oracle(direction, 3, batch, src, before)
        mask, copy = gh.written_mask(direction, 3, batch.p, batch.k, U, o, s, doff, len(got))
        assert np.array_equal(got[~mask], before[~mask])
        assert np.array_equal(got[copy], want[copy])
        err = np.abs(got[mask] - want[mask]).reshape(-1, U).max(axis=0)
        assert (err / np.abs(want[mask]).reshape(-1, U).max(axis=0)).max() < 1e-5


def test_largest_patch_box():
    """Fused interpolation and restriction on p = 48 patches (54^3 cells)."""
    dev = gh.require_gpu()
    p, k, U = 48, 3, 2
    b = wl.patch_transitions(2, p, k, U, seed=54, device=dev)
    iop = api.build_transfer_operator(0, oracle.DLINEAR, p, k)
    rop = api.build_transfer_operator(1, oracle.DLINEAR, p, k)
    o, s = b.orientation.cpu().numpy(), b.subface.cpu().numpy()
    co, fo = b.coarse_offset.cpu().numpy(), b.fine_offset.cpu().numpy()
    fine, coarse = b.fine.clone(), b.coarse.clone()
    api.interpolate_patches(iop, b.orientation, b.subface, b.coarse_offset, b.fine_offset, U, b.coarse, fine)
    api.restrict_patches(rop, b.orientation, b.subface, b.coarse_offset, b.fine_offset, U, b.fine, coarse)
    torch.cuda.synchronize()
    assert iop.errors() == 0 and rop.errors() == 0
    want_f = opt.interpolate_patches(1, p, k, o, s, co, fo, U, b.coarse.cpu().numpy(), b.fine.cpu().numpy())
    want_c = opt.restrict_patches(1, p, k, o, s, co, fo, U, b.fine.cpu().numpy(), b.coarse.cpu().numpy())
    for got, want in ((fine.cpu().numpy(), want_f), (coarse.cpu().numpy(), want_c)):
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
