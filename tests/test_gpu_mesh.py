"""One time step on the hanging faces of a synthetic 3-level AMR mesh:
restriction into the shared coarse faces, then interpolation from them, as a
restrict-first plan and as captured multi-step graphs, against eager calls
and against the FP64 oracle (restriction of all nine subfaces of a coarse
face followed by interpolation from the updated coarse face)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2504_15814_amd import api
from paper_2504_15814_amd import workloads as wl
from tests import gpu_helpers as gh

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mesh(dev):
    return wl.workload5(n_meshes=1, U=5, device=dev)


@pytest.fixture(scope="module")
def dev():
    return gh.require_gpu()


def step_eager(mf, rop, iop, coarse, fine, mode=None):
    api.restrict_faces(rop, mf.orientation, mf.subface, mf.coarse_offset, mf.fine_offset, mf.U, fine, coarse, mode=mode)
    api.interpolate_faces(iop, mf.orientation, mf.subface, mf.coarse_offset, mf.fine_offset, mf.U, coarse, fine,
                          mode=mode)


def make_plan(mf, rop, iop, coarse, fine, mode=None):
    descr = (mf.orientation, mf.subface, mf.coarse_offset, mf.fine_offset)
    return api.build_transfer_plan([(rop, *descr), (iop, *descr)], mf.U, coarse, fine, mode=mode,
                                   flags=api.FT_PLAN_RESTRICT_FIRST)


@pytest.mark.parametrize("scheme", [1, 3])
def test_mesh_step_plan_graph_and_oracle(mesh, scheme):
    mf = mesh
    rop = api.build_transfer_operator(1, scheme, mf.p, mf.k)
    iop = api.build_transfer_operator(0, scheme, mf.p, mf.k)
    ec, ef = mf.coarse.clone(), mf.fine.clone()
    step_eager(mf, rop, iop, ec, ef)
    torch.cuda.synchronize()
    pc, pf = mf.coarse.clone(), mf.fine.clone()
    plan = make_plan(mf, rop, iop, pc, pf)
    plan.run()
    torch.cuda.synchronize()
    assert torch.equal(pc, ec) and torch.equal(pf, ef)
    assert rop.errors() == 0 and iop.errors() == 0

    # oracle: all nine subfaces of 12 coarse faces, restriction then interpolation
    o = mf.orientation.cpu().numpy()
    s = mf.subface.cpu().numpy()
    co = mf.coarse_offset.cpu().numpy()
    fo = mf.fine_offset.cpu().numpy()
    coarse0, fine0 = mf.coarse.cpu().numpy(), mf.fine.cpu().numpy()
    picks = np.unique(co)[:: max(1, mf.n_coarse // 12)][:12]
    faces = np.flatnonzero(np.isin(co, picks))
    assert len(faces) == 9 * len(picks)
    c1 = oracle.restrict_faces(scheme, mf.p, mf.k, o[faces], s[faces], co[faces], fo[faces], mf.U, fine0, coarse0)
    f1 = oracle.interpolate_faces(scheme, mf.p, mf.k, o[faces], s[faces], co[faces], fo[faces], mf.U, c1, fine0)
    E = mf.face_elems
    got_c, got_f = pc.cpu().numpy(), pf.cpu().numpy()
    for cidx in picks:
        a, b = got_c[cidx:cidx + E], c1[cidx:cidx + E]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    for f in faces:
        a, b = got_f[fo[f]:fo[f] + E], f1[fo[f]:fo[f] + E]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()

    # five captured steps equal five eager steps, replayed twice
    for _ in range(4):
        step_eager(mf, rop, iop, ec, ef)
    torch.cuda.synchronize()
    graph = plan.capture(steps=5)
    for rep in range(2):
        pc.copy_(mf.coarse)
        pf.copy_(mf.fine)
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(pc, ec) and torch.equal(pf, ef), rep


def test_mesh_step_mixed_precision_plan(mesh):
    """Float32 storage: the Taylor-3 restriction at k = 3 extrapolates with
    row 1-norms up to ~406, which amplifies the 2^-24 rounding of the stored
    inputs to ~2.4e-5 of max|x|; interpolation then reads those values."""
    mf = mesh
    rop = api.build_transfer_operator(1, 3, mf.p, mf.k)
    iop = api.build_transfer_operator(0, 3, mf.p, mf.k)
    ec, ef = mf.coarse.clone(), mf.fine.clone()
    step_eager(mf, rop, iop, ec, ef)
    pc, pf = mf.coarse.float(), mf.fine.float()
    plan = make_plan(mf, rop, iop, pc, pf, mode=api.FT_F32_BF16X6)
    plan.run()
    torch.cuda.synchronize()
    for got, ref in ((pc, ec), (pf, ef)):
        err = (got.double() - ref).abs().max() / ref.abs().max()
        assert err < 5e-5


@pytest.fixture(scope="module")
def mesh_full(dev):
    return wl.workload5(n_meshes=3, device=dev)


def test_full_size_mesh_step(mesh_full):
    """The AMR-mesh workload at full size (three meshes, U = 59, Taylor-3) as
    the benchmark runs it: the FP64 plan equals the eager step bit for bit and
    matches the oracle on all nine subfaces of 12 coarse faces; the float32
    six-term plan stays within 1e-6 (relative to the largest value) of the
    FP64 step run on the same float32-rounded inputs."""
    mf = mesh_full
    U, E = mf.U, mf.face_elems
    rop = api.build_transfer_operator(1, 3, mf.p, mf.k)
    iop = api.build_transfer_operator(0, 3, mf.p, mf.k)
    ec, ef = mf.coarse.clone(), mf.fine.clone()
    step_eager(mf, rop, iop, ec, ef)
    pc, pf = mf.coarse.clone(), mf.fine.clone()
    make_plan(mf, rop, iop, pc, pf).run()
    torch.cuda.synchronize()
    assert torch.equal(pc, ec) and torch.equal(pf, ef)
    assert rop.errors() == 0 and iop.errors() == 0
    del pc, pf

    # Every face on the device, one direction at a time: restriction into the
    # shared coarse faces (whose written segments start as sentinels) and
    # interpolation into the fine halos (likewise) write every element of
    # their regions and nothing else.
    d = (mf.orientation, mf.subface, mf.coarse_offset, mf.fine_offset)
    dev = mf.coarse.device
    cmask = gh.device_written_mask(1, 3, mf.p, mf.k, U, mf.orientation, mf.subface, mf.coarse_offset,
                                   mf.coarse.numel(), dev)
    cs = mf.coarse.clone()
    cs[cmask] = gh.SENTINEL
    cb = cs.clone()
    api.restrict_faces(rop, *d, U, mf.fine, cs)
    torch.cuda.synchronize()
    gh.check_written_region(cs, cb, cmask)
    del cmask, cs, cb
    fmask = gh.device_written_mask(0, 3, mf.p, mf.k, U, mf.orientation, mf.subface, mf.fine_offset,
                                   mf.fine.numel(), dev)
    fs = mf.fine.clone()
    fs[fmask] = gh.SENTINEL
    fb = fs.clone()
    api.interpolate_faces(iop, *d, U, mf.coarse, fs)
    torch.cuda.synchronize()
    gh.check_written_region(fs, fb, fmask)
    del fmask, fs, fb

    # oracle on compact copies of 12 coarse faces and their nine fine faces
    o, s = mf.orientation.cpu().numpy(), mf.subface.cpu().numpy()
    co, fo = mf.coarse_offset.cpu().numpy(), mf.fine_offset.cpu().numpy()
    picks = np.unique(co)[:: max(1, mf.n_coarse // 12)][:12]
    faces = np.flatnonzero(np.isin(co, picks))
    assert len(faces) == 9 * len(picks)
    slot = {int(c): i for i, c in enumerate(picks)}
    co_c = np.array([slot[int(co[f])] * E for f in faces], dtype=np.int64)
    fo_c = np.arange(len(faces), dtype=np.int64) * E
    coarse_c = np.concatenate([mf.coarse[int(c):int(c) + E].cpu().numpy() for c in picks])
    fine_c = np.concatenate([mf.fine[int(fo[f]):int(fo[f]) + E].cpu().numpy() for f in faces])
    c1 = oracle.restrict_faces(3, mf.p, mf.k, o[faces], s[faces], co_c, fo_c, U, fine_c, coarse_c)
    f1 = oracle.interpolate_faces(3, mf.p, mf.k, o[faces], s[faces], co_c, fo_c, U, c1, fine_c)
    for i, c in enumerate(picks):
        got, want = ec[int(c):int(c) + E].cpu().numpy(), c1[i * E:(i + 1) * E]
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    for j, f in enumerate(faces):
        got, want = ef[int(fo[f]):int(fo[f]) + E].cpu().numpy(), f1[j * E:(j + 1) * E]
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    del ec, ef

    # float32 six-term plan against the FP64 step on the rounded inputs
    c32, f32 = mf.coarse.float(), mf.fine.float()
    rc, rf = c32.double(), f32.double()
    make_plan(mf, rop, iop, c32, f32, mode=api.FT_F32_BF16X6).run()
    step_eager(mf, rop, iop, rc, rf)
    torch.cuda.synchronize()
    for got, ref in ((c32, rc), (f32, rf)):
        diff, scale = 0.0, float(ref.abs().max())
        for c0 in range(0, ref.numel(), 1 << 27):
            diff = max(diff, float((got[c0:c0 + (1 << 27)].double() - ref[c0:c0 + (1 << 27)]).abs().max()))
        assert diff / scale < 1e-6, diff / scale


def test_full_size_mixed_storage_step(mesh_full):
    """The benchmark's AMR-mesh step with float64 fine data: restriction of
    the float64 fine faces into float32 coarse faces, then six-term float32
    interpolation into float32 fine halo buffers, as two plans captured in
    one graph.  It equals the per-call step bit for bit and stays within
    1e-6 (relative to the largest value) of the FP64 step end to end."""
    mf = mesh_full
    U = mf.U
    d = (mf.orientation, mf.subface, mf.coarse_offset, mf.fine_offset)
    rop = api.build_transfer_operator(1, 3, mf.p, mf.k)
    iop = api.build_transfer_operator(0, 3, mf.p, mf.k)
    cs, hs = mf.coarse.float(), mf.fine.float()
    rplan = api.build_transfer_plan([(rop, *d)], U, cs, mf.fine, mode=api.FT_F64_TO_F32)
    iplan = api.build_transfer_plan([(iop, *d)], U, cs, hs, mode=api.FT_F32_BF16X6)
    graph = api.transfer_plans_capture([rplan, iplan], steps=1)
    graph.launch()
    pc, ph = mf.coarse.float(), mf.fine.float()
    api.restrict_faces(rop, *d, U, mf.fine, pc, mode=api.FT_F64_TO_F32)
    api.interpolate_faces(iop, *d, U, pc, ph, mode=api.FT_F32_BF16X6)
    torch.cuda.synchronize()
    assert torch.equal(cs, pc) and torch.equal(hs, ph)
    del pc, ph
    ec, ef = mf.coarse.clone(), mf.fine.clone()
    step_eager(mf, rop, iop, ec, ef)
    torch.cuda.synchronize()
    assert rop.errors() == 0 and iop.errors() == 0
    for got, ref in ((cs, ec), (hs, ef)):
        diff, scale = 0.0, float(ref.abs().max())
        for c0 in range(0, ref.numel(), 1 << 27):
            diff = max(diff, float((got[c0:c0 + (1 << 27)].double() - ref[c0:c0 + (1 << 27)]).abs().max()))
        assert diff / scale <= 1e-6, diff / scale
