"""Plans (one fused launch over an uneven mix), schedules, the autotuner
and HIP-graph capture, all through the C ABI.

A plan runs the same per-item code as the per-batch kernels, so its output
must equal the per-batch calls bit for bit under every schedule; graph
replays must equal eager runs bit for bit.  A sample is also checked against
the FP64 oracle.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2504_15814_amd import api
from paper_2504_15814_amd import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gh.require_gpu()


@pytest.fixture(scope="module")
def mixed32(dev):
    return wl.workload4(n_faces=1500, device=dev, dtype=torch.float32)


@pytest.fixture(scope="module")
def mixed64(dev):
    return wl.workload4(n_faces=600, device=dev, dtype=torch.float64, seed=99)


def build_ops(mb):
    return {key: api.build_transfer_operator(key[0], key[1], key[2], key[3]) for key in mb.groups()}


def batches_of(mb, ops):
    return [(ops[key], *mb.subset(idx)) for key, idx in mb.groups().items()]


def per_batch_reference(mb, ops, mode):
    coarse, fine = mb.coarse.clone(), mb.fine.clone()
    for key, idx in mb.groups().items():
        o, s, co, fo = mb.subset(idx)
        if key[0] == 0:
            api.interpolate_faces(ops[key], o, s, co, fo, mb.U, mb.coarse, fine, mode=mode)
        else:
            api.restrict_faces(ops[key], o, s, co, fo, mb.U, mb.fine, coarse, mode=mode)
    torch.cuda.synchronize()
    return coarse, fine


def run_plan(mb, ops, mode, schedule=None):
    coarse, fine = mb.coarse.clone(), mb.fine.clone()
    # The plan reads and writes the same pools: interpolated faces read coarse
    # and write fine, restricted faces read fine and write coarse; faces are
    # independent, so one launch is race-free.
    plan = api.build_transfer_plan(batches_of(mb, ops), mb.U, coarse, fine, mode=mode)
    if schedule is not None:
        plan.schedule = schedule
    plan.run()
    torch.cuda.synchronize()
    return plan, coarse, fine


@pytest.mark.parametrize("mode", [api.FT_F32, api.FT_F32_BF16X3, api.FT_F32_BF16X6])
def test_plan_equals_per_batch_calls_f32(mixed32, mode):
    ops = build_ops(mixed32)
    rc, rf = per_batch_reference(mixed32, ops, mode)
    _, pc, pf = run_plan(mixed32, ops, mode)
    assert torch.equal(pc, rc) and torch.equal(pf, rf)
    for op in ops.values():
        assert op.errors() == 0


def test_plan_equals_per_batch_calls_f64_and_oracle(mixed64):
    ops = build_ops(mixed64)
    rc, rf = per_batch_reference(mixed64, ops, None)
    _, pc, pf = run_plan(mixed64, ops, None)
    assert torch.equal(pc, rc) and torch.equal(pf, rf)
    # oracle on up to 4 faces of every (direction, scheme, p, k) group
    coarse_in = mixed64.coarse.cpu().numpy()
    fine_in = mixed64.fine.cpu().numpy()
    pc_np, pf_np = pc.cpu().numpy(), pf.cpu().numpy()
    co = mixed64.coarse_offset.cpu().numpy()
    fo = mixed64.fine_offset.cpu().numpy()
    orient = mixed64.orientation.cpu().numpy()
    sub = mixed64.subface.cpu().numpy()
    U = mixed64.U
    for (d, sch, p, k), idx in mixed64.groups().items():
        for f in idx[:4].tolist():
            rows, W = oracle.transfer_operator(d, sch, p, k, int(orient[f]), int(sub[f]))
            ncell = 2 * k * p * p
            if d == 0:
                x = coarse_in[co[f]:co[f] + ncell * U].reshape(ncell, U)
                got = pf_np[fo[f]:fo[f] + ncell * U].reshape(ncell, U)[rows]
            else:
                x = fine_in[fo[f]:fo[f] + ncell * U].reshape(ncell, U)
                got = pc_np[co[f]:co[f] + ncell * U].reshape(ncell, U)[rows]
            want = W @ x
            assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_every_schedule_gives_identical_bits(mixed32):
    ops = build_ops(mixed32)
    _, c0, f0 = run_plan(mixed32, ops, api.FT_F32_BF16X6)
    for sch in (api.pack_schedule(1, 1), api.pack_schedule(2, 3, 1, 0), api.pack_schedule(4, 16, 1, 1),
                api.pack_schedule(4, 64, 0, 1), api.pack_schedule(2, 1, 0, 0, 0), api.pack_schedule(4, 1, 1, 1, 0)):
        _, c, f = run_plan(mixed32, ops, api.FT_F32_BF16X6, sch)
        assert torch.equal(c, c0) and torch.equal(f, f0)


def test_autotune_picks_a_valid_schedule(mixed32):
    ops = build_ops(mixed32)
    coarse, fine = mixed32.coarse.clone(), mixed32.fine.clone()
    plan = api.build_transfer_plan(batches_of(mixed32, ops), mixed32.U, coarse, fine, mode=api.FT_F32)
    best, ms = plan.autotune(reps=2)
    sch = api.unpack_schedule(best)
    assert sch["waves_per_block"] in (2, 4) and sch["blocks_per_cu"] == 1 and sch["persistent"] == 0
    assert plan.schedule == best and ms > 0
    rc, rf = per_batch_reference(mixed32, ops, api.FT_F32)
    plan.run()
    torch.cuda.synchronize()
    assert torch.equal(coarse, rc) and torch.equal(fine, rf)


def test_graph_replays_equal_eager_runs(mixed32):
    ops = build_ops(mixed32)
    coarse, fine = mixed32.coarse.clone(), mixed32.fine.clone()
    plan = api.build_transfer_plan(batches_of(mixed32, ops), mixed32.U, coarse, fine, mode=api.FT_F32_BF16X3)
    plan.run()
    torch.cuda.synchronize()
    eager_c, eager_f = coarse.clone(), fine.clone()
    graph = plan.capture(steps=1)
    for rep in range(4):
        coarse.copy_(mixed32.coarse)  # eager work between replays
        fine.copy_(mixed32.fine)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(coarse, eager_c) and torch.equal(fine, eager_f), rep


def _shared_face_setup(dev, dtype):
    """Nine fine faces of one coarse face (so interpolation reads what
    restriction writes), three copies side by side."""
    p, k, U = 9, 3, 17
    base = wl.uniform_faces(27, p, k, U, seed=31, device=dev, dtype=dtype)
    E = base.face_elems
    sub = (torch.arange(27) % 9).to(torch.int8).to(dev)
    orient = torch.tensor([1] * 9 + [3] * 9 + [5] * 9, dtype=torch.int8, device=dev)
    coff = ((torch.arange(27) // 9) * E).to(torch.int64).to(dev)
    foff = (torch.arange(27) * E).to(torch.int64).to(dev)
    coarse = base.coarse[: 3 * E].clone()
    return p, k, U, orient, sub, coff, foff, coarse, base.fine.clone()


@pytest.mark.parametrize("dtype,mode", [(torch.float64, None), (torch.float32, api.FT_F32),
                                        (torch.float32, api.FT_F32_BF16X3), (torch.float32, api.FT_F32_BF16X6)])
def test_restrict_first_plan_and_multi_step_graph(dev, dtype, mode):
    """Restriction phase then interpolation phase (in the float32 modes the
    restriction-only phase runs the vector-ALU plan kernel): bitwise equal to
    eager per-call steps in the same mode."""
    p, k, U, orient, sub, coff, foff, coarse0, fine0 = _shared_face_setup(dev, dtype)
    rop = api.build_transfer_operator(1, 3, p, k)
    iop = api.build_transfer_operator(0, 3, p, k)
    # eager reference: restrict then interpolate, three steps
    rc, rf = coarse0.clone(), fine0.clone()
    for _ in range(3):
        api.restrict_faces(rop, orient, sub, coff, foff, U, rf, rc, mode=mode)
        api.interpolate_faces(iop, orient, sub, coff, foff, U, rc, rf, mode=mode)
    torch.cuda.synchronize()
    coarse, fine = coarse0.clone(), fine0.clone()
    plan = api.build_transfer_plan([(iop, orient, sub, coff, foff), (rop, orient, sub, coff, foff)], U, coarse, fine,
                                   mode=mode, flags=api.FT_PLAN_RESTRICT_FIRST)
    graph = plan.capture(steps=3)
    for rep in range(3):
        coarse.copy_(coarse0)
        fine.copy_(fine0)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(coarse, rc) and torch.equal(fine, rf), rep
    # and the plan run eagerly three times
    coarse.copy_(coarse0)
    fine.copy_(fine0)
    for _ in range(3):
        plan.run()
    torch.cuda.synchronize()
    assert torch.equal(coarse, rc) and torch.equal(fine, rf)


def test_plan_with_halo_depth_one(dev):
    """A mix with k in {1, 2, 3} (k = 1 faces are d-linear): the plan equals
    the per-batch calls bit for bit in every float32 mode and in float64."""
    for dtype, modes in ((torch.float32, (api.FT_F32, api.FT_F32_BF16X6)), (torch.float64, (None,))):
        mb = wl.workload4(n_faces=900, device=dev, dtype=dtype, seed=123, k_values=(1, 2, 3))
        assert any(key[3] == 1 for key in mb.groups())
        ops = build_ops(mb)
        for mode in modes:
            rc, rf = per_batch_reference(mb, ops, mode)
            _, pc, pf = run_plan(mb, ops, mode)
            assert torch.equal(pc, rc) and torch.equal(pf, rf)
        for op in ops.values():
            assert op.errors() == 0


def test_plan_with_patch_sizes_not_multiples_of_three(dev):
    """A mix of p = 7, 8, 10 (partial anchors in every segment): the plan
    equals the per-batch calls bit for bit, and they equal the oracle on a
    sample (float64)."""
    mb = wl.workload4(n_faces=600, device=dev, dtype=torch.float64, seed=321, p_values=(7, 8, 10))
    ops = build_ops(mb)
    rc, rf = per_batch_reference(mb, ops, None)
    _, pc, pf = run_plan(mb, ops, None)
    assert torch.equal(pc, rc) and torch.equal(pf, rf)
    for op in ops.values():
        assert op.errors() == 0
    coarse_in, fine_in = mb.coarse.cpu().numpy(), mb.fine.cpu().numpy()
    pc_np, pf_np = pc.cpu().numpy(), pf.cpu().numpy()
    co, fo = mb.coarse_offset.cpu().numpy(), mb.fine_offset.cpu().numpy()
    orient, sub = mb.orientation.cpu().numpy(), mb.subface.cpu().numpy()
    U = mb.U
    for (d, sch, p, k), idx in mb.groups().items():
        for f in idx[:2].tolist():
            rows, W = oracle.transfer_operator(d, sch, p, k, int(orient[f]), int(sub[f]))
            ncell = 2 * k * p * p
            if d == 0:
                x = coarse_in[co[f]:co[f] + ncell * U].reshape(ncell, U)
                got = pf_np[fo[f]:fo[f] + ncell * U].reshape(ncell, U)[rows]
            else:
                x = fine_in[fo[f]:fo[f] + ncell * U].reshape(ncell, U)
                got = pc_np[co[f]:co[f] + ncell * U].reshape(ncell, U)[rows]
            want = W @ x
            assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_full_size_uneven_mix_sampled(dev):
    """50,000 faces of the uneven mix in one float32 plan launch (split
    bfloat16, six terms) as the benchmark runs it: bitwise equal to the
    per-batch calls, and two faces of every (direction, scheme, p, k) group
    within the float32 bound of the oracle on the same inputs."""
    mb = wl.workload4(n_faces=50000, device=dev, dtype=torch.float32)
    ops = build_ops(mb)
    rc, rf = per_batch_reference(mb, ops, api.FT_F32_BF16X6)
    plan, pc, pf = run_plan(mb, ops, api.FT_F32_BF16X6)
    plan.autotune(reps=1)
    pc.copy_(mb.coarse)
    pf.copy_(mb.fine)
    plan.run()
    torch.cuda.synchronize()
    assert torch.equal(pc, rc) and torch.equal(pf, rf)
    del rc, rf
    # All 50,000 faces on the device: the halves the plan writes (fine ghost
    # halves of interpolated faces, coarse segments of restricted faces) are
    # never read by the launch, so they start as sentinels; afterwards each
    # of their elements was written and nothing else changed.
    U = mb.U
    fmask = torch.zeros(mb.fine.numel(), dtype=torch.bool, device=dev)
    cmask = torch.zeros(mb.coarse.numel(), dtype=torch.bool, device=dev)
    for (d, sch, p, k), idx in mb.groups().items():
        o, s_, co_, fo_ = mb.subset(idx)
        if d == 0:
            fmask |= gh.device_written_mask(0, sch, p, k, U, o, s_, fo_, fmask.numel(), dev)
        else:
            cmask |= gh.device_written_mask(1, sch, p, k, U, o, s_, co_, cmask.numel(), dev)
    fs, cs = mb.fine.clone(), mb.coarse.clone()
    fs[fmask] = gh.SENTINEL
    cs[cmask] = gh.SENTINEL
    fb, cb = fs.clone(), cs.clone()
    plan2 = api.build_transfer_plan(batches_of(mb, ops), U, cs, fs, mode=api.FT_F32_BF16X6)
    plan2.schedule = plan.schedule
    plan2.run()
    torch.cuda.synchronize()
    assert torch.equal(cs, pc) and torch.equal(fs, pf)
    gh.check_written_region(fs, fb, fmask)
    gh.check_written_region(cs, cb, cmask)
    del fmask, cmask, fs, cs, fb, cb, plan2
    coarse_in = mb.coarse.double().cpu().numpy()
    fine_in = mb.fine.double().cpu().numpy()
    pc_np, pf_np = pc.double().cpu().numpy(), pf.double().cpu().numpy()
    co, fo = mb.coarse_offset.cpu().numpy(), mb.fine_offset.cpu().numpy()
    orient, sub = mb.orientation.cpu().numpy(), mb.subface.cpu().numpy()
    for (d, sch, p, k), idx in mb.groups().items():
        for f in idx[:2].tolist():
            rows, W = oracle.transfer_operator(d, sch, p, k, int(orient[f]), int(sub[f]))
            ncell = 2 * k * p * p
            if d == 0:
                x = coarse_in[co[f]:co[f] + ncell * U].reshape(ncell, U)
                got = pf_np[fo[f]:fo[f] + ncell * U].reshape(ncell, U)[rows]
            else:
                x = fine_in[fo[f]:fo[f] + ncell * U].reshape(ncell, U)
                got = pc_np[co[f]:co[f] + ncell * U].reshape(ncell, U)[rows]
            want = W @ x
            bound = 21 * 2.0**-24 * (np.abs(W) @ np.abs(x)) + 2.0**-24 * np.abs(want)
            assert np.all(np.abs(got - want) <= bound)


@pytest.mark.parametrize("U,mode", [(3, None), (3, api.FT_F32_BF16X6), (8, api.FT_F32), (12, None),
                                    (12, api.FT_F32_BF16X3)])
def test_plan_at_few_unknowns(dev, U, mode):
    """Uneven mixes at few unknowns per cell: up to U = 8 the plan runs the
    small-U body for every item (so does every per-batch call); at U = 12 the
    plan keeps lanes over unknowns while per-batch restriction takes the
    small-U body.  Either way the plan equals the per-batch calls bit for
    bit, and two faces per group match the oracle (float64: 1e-12; float32:
    the vector-ALU bound up to U = 8, the mode's bound above)."""
    dtype = torch.float64 if mode is None else torch.float32
    mb = wl.workload4(n_faces=700, device=dev, dtype=dtype, seed=400 + U, U=U, k_values=(1, 2, 3),
                      p_values=(6, 8, 12))
    ops = build_ops(mb)
    rc, rf = per_batch_reference(mb, ops, mode)
    _, pc, pf = run_plan(mb, ops, mode)
    assert torch.equal(pc, rc) and torch.equal(pf, rf)
    for op in ops.values():
        assert op.errors() == 0
    coarse_in, fine_in = mb.coarse.double().cpu().numpy(), mb.fine.double().cpu().numpy()
    pc_np, pf_np = pc.double().cpu().numpy(), pf.double().cpu().numpy()
    co, fo = mb.coarse_offset.cpu().numpy(), mb.fine_offset.cpu().numpy()
    orient, sub = mb.orientation.cpu().numpy(), mb.subface.cpu().numpy()
    c_interp = {None: 0.0, api.FT_F32: 35 * 2.0**-24, api.FT_F32_BF16X6: 35 * 2.0**-24,
                api.FT_F32_BF16X3: 3 * 2.0**-16 + 9 * 2.0**-24}[mode]
    for (d, sch, p, k), idx in mb.groups().items():
        for f in idx[:2].tolist():
            rows, W = oracle.transfer_operator(d, sch, p, k, int(orient[f]), int(sub[f]))
            ncell = 2 * k * p * p
            if d == 0:
                x = coarse_in[co[f]:co[f] + ncell * U].reshape(ncell, U)
                got = pf_np[fo[f]:fo[f] + ncell * U].reshape(ncell, U)[rows]
            else:
                x = fine_in[fo[f]:fo[f] + ncell * U].reshape(ncell, U)
                got = pc_np[co[f]:co[f] + ncell * U].reshape(ncell, U)[rows]
            want = W @ x
            if mode is None:
                assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
            else:
                c = c_interp if d == 0 else 0.0  # restriction sums in float64
                bound = (c + 1e-13) * (np.abs(W) @ np.abs(x)) + 1.001 * 2.0**-24 * np.abs(want)
                assert np.all(np.abs(got - want) <= bound)
