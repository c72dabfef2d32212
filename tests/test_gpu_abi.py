"""C-ABI argument checks that need a device, and the lifetime of captured
graphs: every pointer a kernel would dereference is checked on the host
(device memory of the current device, as large as stated) and refused with
FT_ERR_INVALID before any launch; a graph captured from a plan stays valid
after the plan's schedule changes and after the plan is destroyed."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2504_15814_amd import _lib, api
from paper_2504_15814_amd import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gh.require_gpu()


def _raw_interpolate(op, n, o, s, co, fo, U, dtype, src, src_elems, dst, dst_elems):
    return _lib.load().interpolate_faces(op.handle, n, o, s, co, fo, U, dtype, src, src_elems, dst,
                                         dst_elems, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_host_pointers_and_overstated_sizes_are_refused(dev):
    U = 3
    b = wl.uniform_faces(4, 9, 3, U, seed=5, device=dev)
    op = api.build_transfer_operator(0, 2, 9, 3)
    dst = torch.full_like(b.fine, gh.SENTINEL)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    good = [P(b.orientation), P(b.subface), P(b.coarse_offset), P(b.fine_offset)]
    n = b.n
    # the valid call works
    assert _raw_interpolate(op, n, *good, U, 0, P(b.coarse), b.coarse.numel(), P(dst), dst.numel()) == 0
    torch.cuda.synchronize()
    # pageable host descriptor arrays
    host_o = np.zeros(n, dtype=np.int8)
    args = list(good)
    args[0] = ctypes.c_void_p(host_o.ctypes.data)
    rc = _raw_interpolate(op, n, *args, U, 0, P(b.coarse), b.coarse.numel(), P(dst), dst.numel())
    assert rc == api.FT_ERR_INVALID and "orientation" in api.transfer_last_error()
    # pinned host memory is host memory too
    pinned = torch.zeros(b.fine.numel(), dtype=torch.float64, pin_memory=True)
    rc = _raw_interpolate(op, n, *good, U, 0, P(b.coarse), b.coarse.numel(), P(pinned), pinned.numel())
    assert rc == api.FT_ERR_INVALID and "destination" in api.transfer_last_error()
    # a buffer claimed larger than its allocation
    small = torch.zeros(1 << 20, dtype=torch.float64, device=dev)
    rc = _raw_interpolate(op, n, *good, U, 0, P(small), small.numel() + (1 << 30), P(dst), dst.numel())
    assert rc == api.FT_ERR_INVALID and "past the end" in api.transfer_last_error()
    # descriptor arrays shorter than n_faces claims (allocations are rounded,
    # so claim far more than was allocated)
    rc = _raw_interpolate(op, 1 << 40, *good, U, 0, P(b.coarse), b.coarse.numel(), P(dst), dst.numel())
    assert rc == api.FT_ERR_INVALID
    # nothing above launched: the destination still holds the first result
    before = dst.clone()
    torch.cuda.synchronize()
    assert torch.equal(before, dst) and op.errors() == 0
    # the next launch after a refused pointer check is unaffected
    dst2 = torch.full_like(b.fine, gh.SENTINEL)
    api.interpolate_faces(op, b.orientation, b.subface, b.coarse_offset, b.fine_offset, U, b.coarse, dst2)
    torch.cuda.synchronize()
    assert torch.equal(dst2, dst)


def test_copy_and_plan_pointer_checks(dev):
    U = 2
    b = wl.uniform_faces(3, 9, 3, U, seed=6, device=dev)
    lib = _lib.load()
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    host_off = np.zeros(b.n, dtype=np.int64)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.gather_patch_faces(9, 3, b.n, P(b.orientation), ctypes.c_void_p(host_off.ctypes.data),
                                P(b.fine_offset), api.FT_HALF_BOTH, U, 0, P(b.fine), b.fine.numel(),
                                P(b.coarse), b.coarse.numel(), None, stream)
    assert rc == api.FT_ERR_INVALID
    host_counter = np.zeros(1, dtype=np.int32)
    rc = lib.copy_patch_halos(9, 3, b.n, P(b.orientation), P(b.coarse_offset), P(b.fine_offset), U, 0,
                              P(b.fine), b.fine.numel(), ctypes.c_void_p(host_counter.ctypes.data), stream)
    assert rc == api.FT_ERR_INVALID and "counter" in api.transfer_last_error()
    op = api.build_transfer_operator(0, 1, 9, 3)
    arr = (_lib.PlanBatch * 1)()
    arr[0] = _lib.PlanBatch(op.handle, b.n, host_off.ctypes.data, b.subface.data_ptr(),
                            b.coarse_offset.data_ptr(), b.fine_offset.data_ptr())
    h = ctypes.c_void_p()
    rc = lib.build_transfer_plan(arr, 1, U, 0, P(b.coarse), b.coarse.numel(), P(b.fine), b.fine.numel(), 0,
                                 ctypes.byref(h))
    assert rc == api.FT_ERR_INVALID and not h.value


def _mix(dev):
    mb = wl.workload4(n_faces=400, device=dev, dtype=torch.float32, seed=31)
    ops = {key: api.build_transfer_operator(*key) for key in mb.groups()}
    batches = [(ops[key], *mb.subset(idx)) for key, idx in mb.groups().items()]
    return mb, ops, batches


def test_graph_survives_schedule_change_and_plan_destruction(dev):
    mb, ops, batches = _mix(dev)
    c_ref, f_ref = mb.coarse.clone(), mb.fine.clone()
    ref_plan = api.build_transfer_plan(batches, mb.U, c_ref, f_ref, mode=api.FT_F32_BF16X6)
    ref_plan.run()
    torch.cuda.synchronize()
    c, f = mb.coarse.clone(), mb.fine.clone()
    plan = api.build_transfer_plan(batches, mb.U, c, f, mode=api.FT_F32_BF16X6)
    plan.schedule = api.pack_schedule(waves_per_block=4, blocks_per_cu=1, heavy_first=0, persistent=0)
    graph = plan.capture(steps=1)
    # reorder the segments (the other table) after capture, then run both
    for sched in (api.pack_schedule(4, 1, 0, 1, 0), api.pack_schedule(2, 4, 1, 1, 1)):
        plan.schedule = sched
        for runner in (plan.run, graph.launch):
            c.copy_(mb.coarse)
            f.copy_(mb.fine)
            torch.cuda.synchronize()
            runner()
            torch.cuda.synchronize()
            assert torch.equal(c, c_ref) and torch.equal(f, f_ref)
    # the graph outlives its plan
    plan.destroy()
    for _ in range(3):
        c.copy_(mb.coarse)
        f.copy_(mb.fine)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(c, c_ref) and torch.equal(f, f_ref)
    graph.destroy()


def test_graph_of_several_plans_outlives_them(dev):
    """transfer_plans_capture: the mix's restriction batches and its
    interpolation batches as two plans in one graph equal the single plan
    over all batches bit for bit (the faces are independent), also after
    both plans are destroyed; bad arguments are refused."""
    mb, ops, batches = _mix(dev)
    c_ref, f_ref = mb.coarse.clone(), mb.fine.clone()
    api.build_transfer_plan(batches, mb.U, c_ref, f_ref, mode=api.FT_F32_BF16X6).run()
    torch.cuda.synchronize()
    c, f = mb.coarse.clone(), mb.fine.clone()
    plans = [api.build_transfer_plan([b for b in batches if b[0].direction == d], mb.U, c, f,
                                     mode=api.FT_F32_BF16X6) for d in (1, 0)]
    graph = api.transfer_plans_capture(plans, steps=1)
    lib = _lib.load()
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 2)(plans[0].handle, None)
    assert lib.transfer_plans_capture(arr, 2, 1, ctypes.byref(h)) == api.FT_ERR_INVALID
    arr = (ctypes.c_void_p * 2)(plans[0].handle, plans[1].handle)
    assert lib.transfer_plans_capture(arr, 0, 1, ctypes.byref(h)) == api.FT_ERR_INVALID
    assert lib.transfer_plans_capture(arr, 2, 0, ctypes.byref(h)) == api.FT_ERR_INVALID
    assert h.value is None
    for p in plans:
        p.destroy()
    for _ in range(3):
        c.copy_(mb.coarse)
        f.copy_(mb.fine)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(c, c_ref) and torch.equal(f, f_ref)
    graph.destroy()
    for op in ops.values():
        assert op.errors() == 0
