"""run_transfer_batches, the allocation-free fused launch, through the C ABI:
its outputs equal those of a plan (build_transfer_plan + run_transfer_plan,
the entry point it is a variant of) bit for bit, on two calls in a row, the
second with a smaller input; more batches than its workspace holds are
refused with a clear error."""

import pytest
import torch

from paper_2504_15814_amd import api
from paper_2504_15814_amd import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return gh.require_gpu()


def _groups(mb, limit_groups=None, limit_faces=None):
    ops, batches = {}, []
    for i, (key, idx) in enumerate(mb.groups().items()):
        if limit_groups is not None and i >= limit_groups:
            break
        if limit_faces is not None:
            idx = idx[:limit_faces]
        ops[key] = api.build_transfer_operator(*key)
        batches.append((ops[key], *mb.subset(idx)))
    return ops, batches


def _via_plan(batches, U, coarse, fine, mode, flags):
    c, f = coarse.clone(), fine.clone()
    plan = api.build_transfer_plan(batches, U, c, f, mode=mode, flags=flags)
    plan.run()
    torch.cuda.synchronize()
    plan.destroy()
    return c, f


def _via_batches(batches, U, coarse, fine, mode, flags):
    c, f = coarse.clone(), fine.clone()
    api.run_transfer_batches(batches, U, c, f, mode=mode, flags=flags)
    torch.cuda.synchronize()
    return c, f


@pytest.mark.parametrize("dtype,mode", [(torch.float32, api.FT_F32_BF16X6), (torch.float64, None)])
def test_uneven_mix_equals_plan_on_two_calls(dev, dtype, mode):
    mb = wl.workload4(n_faces=1500, device=dev, dtype=dtype, seed=57)
    U = mb.U
    # first call: every group of the mix; second call: fewer groups, fewer faces
    for limit_groups, limit_faces in ((None, None), (7, 40)):
        ops, batches = _groups(mb, limit_groups, limit_faces)
        want_c, want_f = _via_plan(batches, U, mb.coarse, mb.fine, mode, 0)
        got_c, got_f = _via_batches(batches, U, mb.coarse, mb.fine, mode, 0)
        assert torch.equal(got_c, want_c) and torch.equal(got_f, want_f)
        assert not torch.equal(got_f, mb.fine) or not torch.equal(got_c, mb.coarse)
        for op in ops.values():
            assert op.errors() == 0


def test_restrict_first_mesh_step_equals_plan(dev):
    """Both phases (restriction into shared coarse faces, then interpolation
    from them), FP64, then the mixed form, then the FP64 step again on a
    smaller mesh."""
    for n_meshes, U, base, mode in ((1, 3, 3, None), (1, 3, 3, api.FT_F32_BF16X6), (1, 2, 2, None)):
        mf = wl.workload5(n_meshes=n_meshes, U=U, device=dev, base_level=base,
                          dtype=torch.float64 if mode is None else torch.float32)
        rop = api.build_transfer_operator(1, 3, mf.p, mf.k)
        iop = api.build_transfer_operator(0, 3, mf.p, mf.k)
        d = (mf.orientation, mf.subface, mf.coarse_offset, mf.fine_offset)
        batches = [(rop, *d), (iop, *d)]
        flags = api.FT_PLAN_RESTRICT_FIRST
        want_c, want_f = _via_plan(batches, U, mf.coarse, mf.fine, mode, flags)
        got_c, got_f = _via_batches(batches, U, mf.coarse, mf.fine, mode, flags)
        assert torch.equal(got_c, want_c) and torch.equal(got_f, want_f)
        assert rop.errors() == 0 and iop.errors() == 0


def test_too_many_batches_are_refused(dev):
    b = wl.uniform_faces(129, 9, 3, 2, seed=3, device=dev)
    op = api.build_transfer_operator(0, 1, 9, 3)
    batches = [(op, b.orientation[i:i + 1], b.subface[i:i + 1], b.coarse_offset[i:i + 1],
                b.fine_offset[i:i + 1]) for i in range(129)]
    fine = b.fine.clone()
    with pytest.raises(api.FTError, match="128") as exc:
        api.run_transfer_batches(batches, 2, b.coarse, fine)
    assert exc.value.code == api.FT_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert torch.equal(fine, b.fine)
    # 128 batches fit, and equal the plan
    want_c, want_f = _via_plan(batches[:128], 2, b.coarse, b.fine, None, 0)
    got_c, got_f = _via_batches(batches[:128], 2, b.coarse, b.fine, None, 0)
    assert torch.equal(got_f, want_f) and torch.equal(got_c, want_c)
