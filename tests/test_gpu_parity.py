"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: float64 storage 1e-12 relative per unknown (max error over the
written cells divided by the largest expected magnitude); float32 storage
1e-5 against the oracle fed the same rounded inputs.  Exact-copy rows
(coinciding centres) and every cell a call must not write are compared bit
for bit.
"""

import numpy as np
import pytest
import torch

from paper_2504_15814_amd import api
from paper_2504_15814_amd import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

SCHEMES = [1, 2, 3]
DIRS = [0, 1]


@pytest.fixture(scope="module")
def dev():
    return gh.require_gpu()


@pytest.fixture(scope="module")
def w1(dev):
    return wl.workload1(device=dev)


@pytest.fixture(scope="module")
def small59(dev):
    return wl.uniform_faces(150, 9, 3, 59, seed=42, device=dev)


@pytest.mark.parametrize("direction", DIRS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_workload1_single_unknown(w1, direction, scheme):
    """64 faces, every (orientation, subface) pair, U = 1."""
    gh.check_parity(direction, scheme, w1)


@pytest.mark.parametrize("direction", DIRS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_ccz4_sized_state_f64(small59, direction, scheme):
    gh.check_parity(direction, scheme, small59)


@pytest.mark.parametrize("direction", DIRS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_ccz4_sized_state_f32(small59, direction, scheme):
    gh.check_parity(direction, scheme, small59, dtype=torch.float32, tol=1e-5)


@pytest.mark.parametrize("p,k", [(6, 2), (6, 3), (12, 2), (12, 3), (9, 2)])
@pytest.mark.parametrize("U", [1, 7, 64, 70, 130])
def test_shapes_and_ragged_unknowns(dev, p, k, U):
    """Patch sizes, halo depths and unknown counts that span several 64-lane
    chunks with a ragged tail."""
    batch = wl.uniform_faces(24, p, k, U, seed=1000 + 10 * p + k + U, device=dev)
    for direction in DIRS:
        for scheme in SCHEMES:
            gh.check_parity(direction, scheme, batch)


@pytest.mark.parametrize("p", [6, 9, 12])
@pytest.mark.parametrize("U", [1, 59, 70])
def test_halo_depth_one_dlinear(dev, p, U):
    """k = 1 (finite volumes): the d-linear scheme, both directions, float64
    and float32 storage."""
    batch = wl.uniform_faces(30, p, 1, U, seed=2000 + p + U, device=dev)
    for direction in DIRS:
        gh.check_parity(direction, 1, batch)
        gh.check_parity(direction, 1, batch, dtype=torch.float32, tol=1e-5)


@pytest.mark.parametrize("p,k", [(7, 2), (8, 3), (10, 3), (11, 2)])
def test_patch_sizes_not_multiples_of_three(dev, p, k):
    """Fine and coarse cells do not align at the subface boundaries: partial
    anchors, rows of the neighbouring fine face skipped, restriction columns
    chosen by their centres."""
    batch = wl.uniform_faces(40, p, k, 59, seed=3000 + 10 * p + k, device=dev)
    for direction in DIRS:
        for scheme in SCHEMES:
            gh.check_parity(direction, scheme, batch)
        gh.check_parity(direction, 3, batch, dtype=torch.float32, tol=1e-5)
    k1 = wl.uniform_faces(20, p, 1, 7, seed=3100 + p, device=dev)
    for direction in DIRS:
        gh.check_parity(direction, 1, k1)


def test_empty_batch_is_a_noop(dev):
    batch = wl.uniform_faces(3, 9, 3, 5, seed=3, device=dev)
    for direction in DIRS:
        op = api.build_transfer_operator(direction, 2, 9, 3)
        empty8 = torch.zeros(0, dtype=torch.int8, device=dev)
        empty64 = torch.zeros(0, dtype=torch.int64, device=dev)
        dst = torch.full_like(batch.fine, gh.SENTINEL)
        if direction == 0:
            api.interpolate_faces(op, empty8, empty8, empty64, empty64, 5, batch.coarse, dst)
        else:
            api.restrict_faces(op, empty8, empty8, empty64, empty64, 5, batch.fine, dst)
        torch.cuda.synchronize()
        assert torch.all(dst == gh.SENTINEL)


def test_nine_subfaces_share_one_coarse_face(dev):
    """Restriction: the nine fine faces of one coarse face write disjoint
    segments of it in one call; interpolation: they all read it."""
    p, k, U = 9, 3, 11
    base = wl.uniform_faces(9, p, k, U, seed=77, device=dev)
    E = base.face_elems
    sub = torch.arange(9, dtype=torch.int8, device=dev)
    orient = torch.full((9,), 4, dtype=torch.int8, device=dev)
    shared = wl.FaceBatch(p, k, U, orient, sub,
                          torch.zeros(9, dtype=torch.int64, device=dev),
                          torch.arange(9, dtype=torch.int64, device=dev) * E,
                          base.coarse[:E].clone(), base.fine.clone())
    for scheme in SCHEMES:
        gh.check_parity(0, scheme, shared)
        gh.check_parity(1, scheme, shared)


def test_permuted_and_gapped_offsets(dev):
    """Faces stored out of order and with gaps between buffers."""
    p, k, U = 9, 3, 13
    base = wl.uniform_faces(20, p, k, U, seed=5, device=dev)
    E = base.face_elems
    perm = torch.randperm(20, generator=torch.Generator().manual_seed(9))
    slots = (perm * 2 + 1).to(torch.int64)  # every other slot, shuffled
    coarse = torch.zeros(41 * E, dtype=torch.float64, device=dev)
    fine = torch.zeros(41 * E, dtype=torch.float64, device=dev)
    for f in range(20):
        sl = int(slots[f])
        coarse[sl * E:(sl + 1) * E] = base.coarse[f * E:(f + 1) * E]
        fine[sl * E:(sl + 1) * E] = base.fine[f * E:(f + 1) * E]
    offs = (slots * E).to(dev)
    gapped = wl.FaceBatch(p, k, U, base.orientation, base.subface, offs, offs.clone(), coarse, fine)
    for scheme in SCHEMES:
        for direction in DIRS:
            gh.check_parity(direction, scheme, gapped)


def test_bad_descriptors_are_skipped_and_counted(dev):
    """Out-of-range orientation, subface or offsets: the kernel's own checks
    skip the face (nothing written) and count it."""
    p, k, U = 9, 3, 4
    batch = wl.uniform_faces(6, p, k, U, seed=8, device=dev)
    E = batch.face_elems
    orient = batch.orientation.clone()
    sub = batch.subface.clone()
    coff = batch.coarse_offset.clone()
    foff = batch.fine_offset.clone()
    orient[1] = 6
    sub[2] = 9
    coff[3] = 5 * E + 1  # runs past the end of the buffer
    foff[4] = -E
    for direction in DIRS:
        op = api.build_transfer_operator(direction, 2, p, k)
        dst = torch.full_like(batch.fine, gh.SENTINEL)
        if direction == 0:
            api.interpolate_faces(op, orient, sub, coff, foff, U, batch.coarse, dst)
        else:
            api.restrict_faces(op, orient, sub, coff, foff, U, batch.fine, dst)
        torch.cuda.synchronize()
        assert op.errors() == 4
        d = dst.view(6, E)
        for f in (1, 2, 3):
            assert torch.all(d[f] == gh.SENTINEL)
        assert not torch.all(d[0] == gh.SENTINEL) and not torch.all(d[5] == gh.SENTINEL)


def test_host_side_rejections_on_device(dev):
    op = api.build_transfer_operator(0, 2, 9, 3)
    b = wl.uniform_faces(2, 9, 3, 3, seed=2, device=dev)
    with pytest.raises(api.FTError):
        api.interpolate_faces(op, b.orientation, b.subface, b.coarse_offset, b.fine_offset, 0, b.coarse, b.fine)
    with pytest.raises(api.FTError):
        api.interpolate_faces(op, b.orientation, b.subface, b.coarse_offset, b.fine_offset, 3, b.coarse, b.coarse)
    with pytest.raises(api.FTError):
        api.restrict_faces(op, b.orientation, b.subface, b.coarse_offset, b.fine_offset, 3, b.fine, b.coarse)


@pytest.fixture(scope="module")
def full2(dev):
    return wl.workload2(device=dev)


@pytest.mark.parametrize("direction", DIRS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_full_size_workload2_sampled(full2, direction, scheme):
    """20,000 faces x 59 unknowns in the benchmark's launch configuration.
    On the device, for all faces: every element of every written half was
    written and every other element kept its sentinel bit for bit.  A seeded
    sample of 150 faces is recomputed by the oracle."""
    rng = np.random.default_rng(scheme + 10 * direction)
    faces = np.sort(rng.choice(full2.n, size=150, replace=False))
    dst, src, before = gh.run_gpu_device(direction, scheme, full2)
    gh.check_full_size(direction, scheme, full2, dst, before, faces, src=src)
