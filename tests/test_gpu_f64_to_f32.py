"""Restriction of float64 fine data into float32 coarse faces (FT_F64_TO_F32),
through the C ABI.

Every output of this type is the float64 restriction rounded once to
float32, so a call must equal the FT_F64 call followed by a cast, bit for
bit; against the oracle each value lies within 2^-24 of itself plus the
float64 tolerance, injected values are the float32 rounding of the fine
value, and every cell a call must not write keeps its sentinel.  Plans, the
allocation-free fused launch and graphs of several plans per step run the
same bodies and must equal the per-batch calls bit for bit.  Last, the
restrict-then-interpolate step with float64 fine data and float32 coarse
faces and fine halos stays within 1e-6 of the float64 step.
"""

import numpy as np
import pytest
import torch

from paper_2504_15814_amd import api
from paper_2504_15814_amd import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu

MIXED = api.FT_F64_TO_F32


@pytest.fixture(scope="module")
def dev():
    return gh.require_gpu()


def restrict_both(op, b, fine=None):
    """FT_F64_TO_F32 and FT_F64 restriction of the batch's float64 fine data
    into sentinel-filled coarse arrays: (float32 result, its sentinel copy,
    float64 result)."""
    fine = b.fine if fine is None else fine
    d = (b.orientation, b.subface, b.coarse_offset, b.fine_offset)
    got = torch.full(b.coarse.shape, gh.SENTINEL, dtype=torch.float32, device=b.coarse.device)
    before = got.clone()
    ref = torch.full_like(b.coarse, gh.SENTINEL)
    api.restrict_faces(op, *d, b.U, fine, got, mode=MIXED)
    api.restrict_faces(op, *d, b.U, fine, ref)
    torch.cuda.synchronize()
    assert op.errors() == 0
    return got, before, ref


@pytest.mark.parametrize("scheme,p,k,U", [
    (1, 9, 1, 59), (1, 9, 3, 59), (2, 9, 2, 59), (3, 9, 3, 59), (3, 7, 3, 59), (2, 10, 2, 59),
    (3, 12, 3, 130), (3, 9, 3, 17),
    (3, 9, 3, 1), (2, 9, 3, 3), (3, 9, 2, 16),  # the small-U body (at most 16 unknowns)
])
def test_rounded_float64_result_and_oracle(dev, scheme, p, k, U):
    """Every (orientation, subface) pair (60 faces): bitwise the FP64 result
    rounded to float32, within 2^-24 |y| + 2e-12 max|y| of the oracle per
    unknown, injected values exact, untouched cells kept."""
    b = wl.pair_faces(60, p, k, U, seed=700 + 10 * scheme + p + k, device=dev)
    op = api.build_transfer_operator(api.FT_RESTRICT, scheme, p, k)
    got, before, ref = restrict_both(op, b)
    mask = gh.device_written_mask(1, scheme, p, k, U, b.orientation, b.subface, b.coarse_offset,
                                  got.numel(), dev)
    gh.check_written_region(got, before, mask)
    assert torch.equal(got[mask], ref[mask].float())

    want, (o, s, co) = gh.run_oracle(1, scheme, b, b.fine.cpu().numpy(), before.double().cpu().numpy())
    m, copy = gh.written_mask(1, scheme, p, k, U, o, s, co, len(want))
    g = got.double().cpu().numpy()
    w, gm = want[m].reshape(-1, U), g[m].reshape(-1, U)
    bound = 2.0**-24 * np.abs(w) + 2e-12 * np.abs(w).max(axis=0)
    assert (np.abs(gm - w) <= bound).all(), float((np.abs(gm - w) / np.maximum(bound, 1e-300)).max())
    assert np.array_equal(g[copy], want[copy].astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("scheme,p,k", [(1, 9, 1), (2, 9, 2), (3, 9, 3), (3, 12, 3)])
@pytest.mark.parametrize("U", [4, 59])
def test_two_dimensional_faces(dev, scheme, p, k, U):
    """FT_BUILD_2D restriction: bitwise the FP64 result rounded to float32,
    untouched cells kept (the FP64 two-dimensional path is checked against
    the two-dimensional oracle elsewhere)."""
    b = wl.faces_2d(40, p, k, U, seed=800 + p + k, device=dev)
    op = api.build_transfer_operator(api.FT_RESTRICT, scheme, p, k, api.FT_BUILD_2D)
    got, before, ref = restrict_both(op, b)
    mask = gh.device_written_mask(1, scheme, p, k, U, b.orientation, b.subface, b.coarse_offset,
                                  got.numel(), dev, dim=2)
    gh.check_written_region(got, before, mask)
    assert torch.equal(got[mask], ref[mask].float())


def test_type_is_rejected_where_it_does_not_apply(dev):
    b = wl.pair_faces(12, 9, 3, 4, seed=901, device=dev)
    d = (b.orientation, b.subface, b.coarse_offset, b.fine_offset)
    c32 = b.coarse.float()
    iop = api.build_transfer_operator(api.FT_INTERPOLATE, 3, 9, 3)
    rop = api.build_transfer_operator(api.FT_RESTRICT, 3, 9, 3)
    with pytest.raises(api.FTError) as e:
        api.interpolate_faces(iop, *d, b.U, c32, b.fine, mode=MIXED)
    assert e.value.code == api.FT_ERR_UNSUPPORTED
    with pytest.raises(api.FTError) as e:
        api.restrict_patches(rop, *d, b.U, b.fine, c32, mode=MIXED)
    assert e.value.code == api.FT_ERR_UNSUPPORTED
    with pytest.raises(api.FTError) as e:
        api.build_transfer_plan([(rop, *d), (iop, *d)], b.U, c32, b.fine, mode=MIXED)
    assert e.value.code == api.FT_ERR_UNSUPPORTED
    with pytest.raises(api.FTError) as e:
        api.build_transfer_plan([(rop, *d)], b.U, c32, b.fine, mode=MIXED, flags=api.FT_PLAN_PATCHES)
    assert e.value.code == api.FT_ERR_UNSUPPORTED
    with pytest.raises(TypeError):  # the binding wants float64 fine, float32 coarse
        api.restrict_faces(rop, *d, b.U, b.fine.float(), c32, mode=MIXED)
    # faces whose coarse buffer lies past the end of a shorter float32 array
    # are skipped and counted; the others are written
    half = torch.full((c32.numel() // 2,), gh.SENTINEL, dtype=torch.float32, device=dev)
    api.restrict_faces(rop, *d, b.U, b.fine, half, mode=MIXED)
    torch.cuda.synchronize()
    E = b.face_elems
    assert rop.errors() == int((b.coarse_offset + E > half.numel()).sum()) > 0
    assert iop.errors() == 0


def restriction_mix(dev, U, seed):
    """The restriction faces of an uneven mix (p in {6, 9, 12}, k in
    {1, 2, 3}, three schemes) with float64 fine data."""
    mb = wl.workload4(n_faces=1200, device=dev, dtype=torch.float64, U=U, seed=seed, k_values=(1, 2, 3))
    groups = {key: idx for key, idx in mb.groups().items() if key[0] == 1}
    ops = {key: api.build_transfer_operator(1, key[1], key[2], key[3]) for key in groups}
    batches = [(ops[key], *mb.subset(idx)) for key, idx in groups.items()]
    return mb, ops, batches


@pytest.mark.parametrize("U", [59, 12, 3])
def test_plan_schedules_and_fused_launch_equal_per_batch_calls(dev, U):
    """A restriction-only plan over the mix: bitwise equal to the per-batch
    calls under every schedule (persistent ones included) and equal to the
    allocation-free fused launch.  At U = 12 the per-batch calls run the
    few-unknowns body and the plan the one-lane-per-unknown body."""
    mb, ops, batches = restriction_mix(dev, U, seed=902 + U)
    assert len(batches) >= 10
    ref = torch.full(mb.coarse.shape, gh.SENTINEL, dtype=torch.float32, device=dev)
    for op, o, s, co, fo in batches:
        api.restrict_faces(op, o, s, co, fo, U, mb.fine, ref, mode=MIXED)
    coarse = torch.full_like(ref, gh.SENTINEL)
    plan = api.build_transfer_plan(batches, U, coarse, mb.fine, mode=MIXED)
    schedules = [None, api.pack_schedule(2, 1, 1, 1, 0), api.pack_schedule(4, 1, 0, 0, 0)]
    if U > 8:  # the small-U plan body has no persistent form
        schedules += [api.pack_schedule(4, 8, 1, 1, 1), api.pack_schedule(2, 2, 0, 0, 1)]
    for sch in schedules:
        coarse.fill_(gh.SENTINEL)
        if sch is not None:
            plan.schedule = sch
        plan.run()
        torch.cuda.synchronize()
        assert torch.equal(coarse, ref), sch
    best, _ = plan.autotune(reps=1)
    assert api.unpack_schedule(best)["persistent"] == 0
    fused = torch.full_like(ref, gh.SENTINEL)
    api.run_transfer_batches(batches, U, fused, mb.fine, mode=MIXED)
    torch.cuda.synchronize()
    assert torch.equal(fused, ref)
    for op in ops.values():
        assert op.errors() == 0


@pytest.fixture(scope="module")
def mesh(dev):
    return wl.workload5(n_meshes=1, U=8, device=dev)


def test_mixed_storage_mesh_step(mesh):
    """The AMR-mesh step with float64 fine data, float32 coarse faces and
    float32 fine halo buffers: an FT_F64_TO_F32 restriction plan, then a
    six-term float32 interpolation plan.  Three steps captured in one graph
    of both plans equal three eager steps bit for bit (replayed twice, with
    eager work between the replays), and one step stays within 1e-6 of the
    float64 step relative to the largest value."""
    mf = mesh
    U = mf.U
    d = (mf.orientation, mf.subface, mf.coarse_offset, mf.fine_offset)
    rop = api.build_transfer_operator(api.FT_RESTRICT, 3, mf.p, mf.k)
    iop = api.build_transfer_operator(api.FT_INTERPOLATE, 3, mf.p, mf.k)
    c64, f64 = mf.coarse.clone(), mf.fine.clone()
    api.restrict_faces(rop, *d, U, f64, c64)
    api.interpolate_faces(iop, *d, U, c64, f64)

    def eager(c32, h32, steps):
        for _ in range(steps):
            api.restrict_faces(rop, *d, U, mf.fine, c32, mode=MIXED)
            api.interpolate_faces(iop, *d, U, c32, h32, mode=api.FT_F32_BF16X6)

    c32, h32 = mf.coarse.float(), mf.fine.float()
    eager(c32, h32, 1)
    torch.cuda.synchronize()
    for got, ref in ((c32, c64), (h32, f64)):
        err = float((got.double() - ref).abs().max() / ref.abs().max())
        assert err <= 1e-6, err

    ec, eh = mf.coarse.float(), mf.fine.float()
    eager(ec, eh, 3)
    pc, ph = mf.coarse.float(), mf.fine.float()
    rplan = api.build_transfer_plan([(rop, *d)], U, pc, mf.fine, mode=MIXED)
    iplan = api.build_transfer_plan([(iop, *d)], U, pc, ph, mode=api.FT_F32_BF16X6)
    graph = api.transfer_plans_capture([rplan, iplan], steps=3)
    for rep in range(2):
        pc.copy_(mf.coarse)
        ph.copy_(mf.fine)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(pc, ec) and torch.equal(ph, eh), rep
        eager(c32, h32, 1)  # eager work between replays
        torch.cuda.synchronize()
    assert rop.errors() == 0 and iop.errors() == 0


@pytest.fixture(scope="module")
def w3_full(dev):
    return wl.workload3(device=dev)


@pytest.mark.parametrize("scheme", [1, 3])
def test_full_size_precision_workload(w3_full, scheme):
    """20,000 faces x 59 unknowns scaled 1e-6 .. 1e3, in the benchmark's
    launch configuration: on the device, for all faces, every written element
    is written, nothing else changes and every value is the FP64 result
    rounded to float32; a seeded sample of 150 faces against the oracle."""
    b = w3_full
    op = api.build_transfer_operator(api.FT_RESTRICT, scheme, b.p, b.k)
    got, before, ref = restrict_both(op, b)
    mask = gh.device_written_mask(1, scheme, b.p, b.k, b.U, b.orientation, b.subface, b.coarse_offset,
                                  got.numel(), got.device)
    gh.check_written_region(got, before, mask)
    assert torch.equal(got[mask], ref[mask].float())
    del mask, ref
    rng = np.random.default_rng(400 + scheme)
    faces = np.sort(rng.choice(b.n, size=150, replace=False))
    cb = gh.compact_batch(b, faces)
    g = gh.compact_faces(got, b.coarse_offset, faces, b.face_elems)
    before_np = gh.compact_faces(before, b.coarse_offset, faces, b.face_elems)
    want, (o, s, co) = gh.run_oracle(1, scheme, cb, cb.fine.numpy(), before_np)
    m, copy = gh.written_mask(1, scheme, b.p, b.k, b.U, o, s, co, len(want))
    w, gm = want[m].reshape(-1, b.U), g[m].reshape(-1, b.U)
    bound = 2.0**-24 * np.abs(w) + 2e-12 * np.abs(w).max(axis=0)
    assert (np.abs(gm - w) <= bound).all(), float((np.abs(gm - w) / np.maximum(bound, 1e-300)).max())
    assert np.array_equal(g[copy], want[copy].astype(np.float32).astype(np.float64))
    assert np.array_equal(g[~m], before_np[~m])
