#!/usr/bin/env python3
"""Throughput of the AMR face transfer on one MI355X.

One step = the whole transfer on one batch: for each scheme (d-linear,
Taylor-2, Taylor-3), restrict every hanging face into its coarse face and
interpolate every fine halo from its coarse face.  Workload: 20,000
independent hanging faces, patches of 9^3 cells, halo depth 3, 59 unknowns
per cell (a CCZ4-sized state), float64, seeded synthetic smooth fields
(Gaussian bumps plus 1e-3 noise).  Inputs are resident in HBM before timing.

Reported value: ghost-cell-unknowns written per second (interpolated fine
halo values plus restricted coarse values) over the timed steps.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "interpolated+restricted ghost-cell-unknowns/sec and % HBM peak; mixed vs FP64"
HBM_PEAK_GBS = 8000.0
SCHEME_NAMES = {1: "dlinear", 2: "taylor2", 3: "taylor3"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="timed steps (the paper times each method over 100 runs)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--faces", type=int, default=20000)
    ap.add_argument("--cpu-faces", type=int, default=8000,
                    help="faces in the oracle's CPU-baseline sample (0 disables it)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--batched-faces", type=int, default=50000,
                    help="faces of the uneven-mix workload run as one plan (0 disables it)")
    ap.add_argument("--mesh-meshes", type=int, default=3,
                    help="independently seeded 3-level AMR meshes in the per-step leg (0 disables it)")
    ap.add_argument("--mesh-steps", type=int, default=100)
    ap.add_argument("--patch-faces", type=int, default=6003,
                    help="fine patches in the fused patch-halo leg, rounded up to a multiple "
                         "of 9 (0 disables it)")
    ap.add_argument("--mesh-patch-meshes", type=int, default=1,
                    help="meshes whose transition zone runs as patches (0 disables the leg)")
    ap.add_argument("--faces-2d", type=int, default=200000,
                    help="two-dimensional faces in the 2D leg (0 disables it)")
    ap.add_argument("--small-u-reps", type=int, default=200,
                    help="calls per latency sample in the 64-face U=1 leg (0 disables it)")
    ap.add_argument("--detail", default=os.path.join(ROOT, "gpurun_out", "bench_detail.json"),
                    help="file that receives every leg's full record (the headline is the "
                         "last stdout line)")
    ap.add_argument("--no-reports", action="store_true",
                    help="skip the convergence and operator-build reports")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def calibrate_copy(torch):
    """A plain 2 GiB float64 device-to-device copy, five times: the bytes the
    HBM counters report for it give their scale factor."""
    n = 1 << 28
    src = torch.arange(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read": n * 8, "bytes_written": n * 8, "reps": 5}))


def algorithmic_bytes(op, orientation, subface, U, elem_bytes):
    """Per-face (distinct source cells with a nonzero weight + destination
    cells) x U x element size, summed over the batch's (orientation, subface)
    mix."""
    import numpy as np

    per = {}
    for o in range(6):
        for s in range(9):
            rows, cols, vals = op.segment(o, s)
            per[(o, s)] = (len(np.unique(cols[vals != 0])) + len(np.unique(rows))) * U * elem_bytes
    counts = np.zeros((6, 9), dtype=np.int64)
    np.add.at(counts, (orientation, subface), 1)
    return int(sum(per[(o, s)] * counts[o, s] for o in range(6) for s in range(9)))


KERNEL_SOURCES = ("ft_device.h", "ft_kernels.hip", "ft_mfma.hip", "ft_kernels.h")


def kernel_source_hash():
    """sha256 prefix of the kernel sources with comments and blank space
    removed (a comment edit does not invalidate recorded counters)."""
    import hashlib
    import re

    csrc = os.path.join(ROOT, "paper_2504_15814_amd", "csrc")
    code = []
    for f in KERNEL_SOURCES:
        text = open(os.path.join(csrc, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code.append("\n".join(line.strip() for line in text.splitlines() if line.strip()))
    return hashlib.sha256("\n".join(code).encode()).hexdigest()[:16]


def recorded_traffic(kernel_name, mode="f64"):
    """HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated) recorded for this kernel
    in profiles/, or None if the kernel sources changed since they were taken."""
    prof = os.path.join(ROOT, "profiles", "transfer_kernels_workload2.md")
    try:
        text = open(prof).read()
        rec = json.loads(text.split("```json")[1].split("```")[0])
        cur = kernel_source_hash()
        if rec.get("kernel_source_sha256_16") != cur:
            return None
        k = rec["kernels"][f"{mode}/{kernel_name}"]
        return int(k["read_bytes"] + k["write_bytes"])
    except (OSError, IndexError, KeyError, ValueError):
        return None


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_steps(launches, steps, warmup, torch):
    """Time `steps` passes over `launches` (list of (name, fn)); per-launch
    durations come from events recorded on the launch stream."""
    for _ in range(warmup):
        for _, fn in launches:
            fn()
    torch.cuda.synchronize()
    events = {name: [] for name, _ in launches}
    t0 = time.perf_counter()
    for _ in range(steps):
        for name, fn in launches:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            events[name].append((a, b))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms = {name: sum(a.elapsed_time(b) for a, b in ev) / len(ev) for name, ev in events.items()}
    return (t1 - t0) * 1e3 / steps, kern_ms


def batched_leg(args, torch, api, wl):
    """Uneven mix (50,000 faces: p 6/9/12, k 2/3, three schemes, both
    directions interleaved, U = 59): FP64 per-batch launches versus one
    float32 plan launch (split-bfloat16 matrix-core interpolation with
    compensation, autotuned, replayed from a captured graph)."""
    mb = wl.workload4(n_faces=args.batched_faces, device="cuda:0", dtype=torch.float32)
    groups = mb.groups()
    U = mb.U
    produced = 0
    for (d, _sch, p, k), idx in groups.items():
        produced += idx.numel() * (k * p * p if d == 0 else k * (p // 3) ** 2) * U
    ops = {key: api.build_transfer_operator(key[0], key[1], key[2], key[3]) for key in groups}
    descr = {key: mb.subset(idx) for key, idx in groups.items()}
    # FP64 reference path: one launch per (direction, scheme, p, k) group.
    c64, f64 = mb.coarse.double(), mb.fine.double()
    oc64, of64 = c64.clone(), f64.clone()

    def step64():
        for key, (o, s_, co, fo) in descr.items():
            if key[0] == 0:
                api.interpolate_faces(ops[key], o, s_, co, fo, U, c64, of64)
            else:
                api.restrict_faces(ops[key], o, s_, co, fo, U, f64, oc64)

    ms64, _ = run_steps([("f64_per_batch", step64)], args.steps, args.warmup, torch)
    batches = [(ops[key], *descr[key]) for key in groups]
    # the FP64 mix as one autotuned plan launch replayed from a graph as well
    p64c, p64f = c64.clone(), f64.clone()
    plan64 = api.build_transfer_plan(batches, U, p64c, p64f)
    plan64.autotune(reps=3)
    graph64 = plan64.capture(steps=1)
    ms64_graph, _ = run_steps([("graph", graph64.launch)], args.steps, args.warmup, torch)
    del graph64, plan64, p64c, p64f
    out = {"workload": "uneven mix: p 6/9/12 at 30/50/20%, k 2/3, dlinear/taylor2/taylor3, "
                       "restrict+interpolate interleaved, U=59",
           "faces": mb.n, "groups": len(groups), "ghost_cell_unknowns_per_step": produced,
           "f64_per_batch_ms": ms64, "f64_plan_graph_ms": ms64_graph}
    for label, mode in (("bf16x6", api.FT_F32_BF16X6), ("f32", api.FT_F32)):
        pc, pf = mb.coarse.clone(), mb.fine.clone()
        # interpolated faces read coarse and write fine; restricted faces read
        # fine and write coarse: run on copies so inputs stay unchanged
        plan = api.build_transfer_plan(batches, U, pc, pf, mode=mode)
        best, tuned_ms = plan.autotune(reps=3)
        ms_plan, _ = run_steps([("plan", plan.run)], args.steps, args.warmup, torch)
        graph = plan.capture(steps=1)
        ms_graph, _ = run_steps([("graph", graph.launch)], args.steps, args.warmup, torch)
        # error of the float32 plan against the FP64 per-batch outputs, over
        # the cells each direction writes (taken where FP64 changed them)
        errs = []
        for got, ref, before in ((pf, of64, f64), (pc, oc64, c64)):
            written = ref != before
            d = (got.double() - ref).abs()[written]
            errs.append(float(d.max() / ref.abs()[written].max()))
        out[label] = {"plan_ms": ms_plan, "graph_ms": ms_graph, "autotune_ms": tuned_ms,
                      "schedule": api.unpack_schedule(best),
                      "value": produced / (ms_graph * 1e-3),
                      "speedup_vs_f64_per_batch": ms64 / ms_graph,
                      "speedup_vs_f64_plan_graph": ms64_graph / ms_graph,
                      "max_rel_err_vs_f64": max(errs)}
        del graph, plan, pc, pf
    return out


def mesh_leg(args, torch, api, wl):
    """Full per-step transfer on synthetic 3-level AMR meshes (Taylor-3,
    p=9, k=3, U=59): every step restricts all hanging faces into their shared
    coarse faces and then interpolates all fine halos from them.  Plain FP64
    (two launches per step, eager) versus the mixed form (float32 plan,
    split-bfloat16 matrix-core interpolation with compensation) with all
    steps captured in one HIP graph, and the mixed-storage form (float64
    fine data restricted into float32 coarse faces, six-term interpolation
    into float32 fine halos; two plans per step in one graph)."""
    mf = wl.workload5(n_meshes=args.mesh_meshes, device="cuda:0", dtype=torch.float64)
    U, steps = mf.U, args.mesh_steps
    rop = api.build_transfer_operator(api.FT_RESTRICT, 3, mf.p, mf.k)
    iop = api.build_transfer_operator(api.FT_INTERPOLATE, 3, mf.p, mf.k)
    d = (mf.orientation, mf.subface, mf.coarse_offset, mf.fine_offset)
    produced = mf.n * (9 * mf.k + mf.k) * (mf.p // 3) ** 2 * U

    c64, f64 = mf.coarse.clone(), mf.fine.clone()

    def step64():
        api.restrict_faces(rop, *d, U, f64, c64)
        api.interpolate_faces(iop, *d, U, c64, f64)

    step64()
    torch.cuda.synchronize()
    ref1_c, ref1_f = c64.clone(), f64.clone()
    ms64, _ = run_steps([("f64_step", step64)], steps, args.warmup, torch)

    c32, f32 = mf.coarse.float(), mf.fine.float()
    # FP64 step on the float32-rounded inputs: the error of the mixed
    # arithmetic alone (the end-to-end error also carries the rounding of the
    # stored inputs, amplified by the restriction's extrapolation rows)
    rc_c, rc_f = c32.double(), f32.double()
    api.restrict_faces(rop, *d, U, rc_f, rc_c)
    api.interpolate_faces(iop, *d, U, rc_c, rc_f)
    plan = api.build_transfer_plan([(rop, *d), (iop, *d)], U, c32, f32, mode=api.FT_F32_BF16X6,
                                   flags=api.FT_PLAN_RESTRICT_FIRST)
    plan.run()
    torch.cuda.synchronize()
    err = max(float((c32.double() - ref1_c).abs().max() / ref1_c.abs().max()),
              float((f32.double() - ref1_f).abs().max() / ref1_f.abs().max()))
    kerr = max(float((c32.double() - rc_c).abs().max() / rc_c.abs().max()),
               float((f32.double() - rc_f).abs().max() / rc_f.abs().max()))
    del rc_c, rc_f

    def graph_ms(p):
        best, _ = p.autotune(reps=3)
        g = p.capture(steps=steps)
        g.launch()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        g.launch()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps, best

    ms_mixed, best = graph_ms(plan)
    del plan, c32, f32
    # Mixed storage: restriction reads the float64 fine data and writes
    # float32 coarse faces (one rounding of the FP64 result), interpolation
    # runs in six split terms into float32 fine halo buffers: two plans per
    # step, all steps in one graph.
    cs, hs = mf.coarse.float(), mf.fine.float()
    rplan = api.build_transfer_plan([(rop, *d)], U, cs, mf.fine, mode=api.FT_F64_TO_F32)
    iplan = api.build_transfer_plan([(iop, *d)], U, cs, hs, mode=api.FT_F32_BF16X6)
    rplan.run()
    iplan.run()
    # FP64 step on the same stored inputs (float64 fine, float32-rounded coarse)
    sc_c = mf.coarse.float().double()
    sc_f = mf.fine.clone()
    api.restrict_faces(rop, *d, U, sc_f, sc_c)
    api.interpolate_faces(iop, *d, U, sc_c, sc_f)
    torch.cuda.synchronize()
    serr = max(float((cs.double() - ref1_c).abs().max() / ref1_c.abs().max()),
               float((hs.double() - ref1_f).abs().max() / ref1_f.abs().max()))
    skerr = max(float((cs.double() - sc_c).abs().max() / sc_c.abs().max()),
                float((hs.double() - sc_f).abs().max() / sc_f.abs().max()))
    del sc_c, sc_f
    rbest, _ = rplan.autotune(reps=3)
    ibest, _ = iplan.autotune(reps=3)
    sg = api.transfer_plans_capture([rplan, iplan], steps=steps)
    sg.launch()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    z = torch.cuda.Event(enable_timing=True)
    a.record()
    sg.launch()
    z.record()
    torch.cuda.synchronize()
    ms_storage = a.elapsed_time(z) / steps
    del sg, rplan, iplan, cs, hs
    # the FP64 step as a plan with all steps in one graph as well
    plan64 = api.build_transfer_plan([(rop, *d), (iop, *d)], U, c64, f64, flags=api.FT_PLAN_RESTRICT_FIRST)
    ms64_graph, _ = graph_ms(plan64)
    del plan64
    return {"workload": f"{args.mesh_meshes} seeded 3-level AMR meshes (27^3 base patches, refinement "
                        "radii 0.3 / 0.1), Taylor-3, p=9, k=3, U=59, restrict then interpolate",
            "hanging_faces": mf.n, "coarse_faces": mf.n_coarse,
            "faces_per_fine_level": {str(kk): v for kk, v in sorted(mf.transitions.items())},
            "steps": steps, "ghost_cell_unknowns_per_step": produced,
            "f64_ms_per_step": ms64, "f64_plan_graph_ms_per_step": ms64_graph,
            "mixed_graph_ms_per_step": ms_mixed, "speedup_vs_f64_plan_graph": ms64_graph / ms_mixed,
            "mixed_value": produced / (ms_mixed * 1e-3), "f64_value": produced / (ms64 * 1e-3),
            "speedup": ms64 / ms_mixed, "mixed_max_rel_err_one_step": err,
            "mixed_kernel_max_rel_err_one_step": kerr,
            "schedule": api.unpack_schedule(best),
            "f64_restrict_graph_ms_per_step": ms_storage,
            "f64_restrict_speedup_vs_f64_plan_graph": ms64_graph / ms_storage,
            "f64_restrict_max_rel_err_one_step": serr,
            "f64_restrict_kernel_max_rel_err_one_step": skerr,
            "f64_restrict_schedules": [api.unpack_schedule(rbest), api.unpack_schedule(ibest)]}


def patches_leg(args, torch, api, wl):
    """The transfer fused with the patch halos (Taylor-3, p=9, k=3, U=59,
    FP64): fine patches of 9^3 cells, nine per coarse face.  A step restricts
    every fine patch into its coarse patch's halo and then interpolates every
    fine halo from its coarse patch.  Unfused: gather the face views into face
    buffers, apply the face-buffer transfer, scatter the halo halves back.
    Fused: the transfer reads and writes the patches in place."""
    import numpy as np

    p, k, U = 9, 3, 59
    # every coarse face carries all nine of its fine faces
    b = wl.patch_transitions(-(-args.patch_faces // 9) * 9, p, k, U, seed=wl.SEED_BASE + 6,
                             device="cuda:0", faces_per_coarse=9)
    n = b.n
    groups = -(-n // 9)
    fe = 2 * k * p * p * U
    dev = b.coarse.device
    rop = api.build_transfer_operator(api.FT_RESTRICT, 3, p, k)
    iop = api.build_transfer_operator(api.FT_INTERPOLATE, 3, p, k)
    d = (b.orientation, b.subface, b.coarse_offset, b.fine_offset)
    # unfused: one face buffer per fine face, one per coarse face
    offs = torch.arange(n, dtype=torch.int64, device=dev) * fe
    goffs = torch.arange(n, dtype=torch.int64, device=dev) // 9 * fe
    first = torch.arange(0, n, 9, device=dev)
    cface = ((b.orientation.to(torch.int64) + 3) % 6).to(torch.int8)
    gface, gpatch, gbuf = cface[first].contiguous(), b.coarse_offset[first].contiguous(), goffs[first].contiguous()
    fbuf = torch.zeros(n * fe, dtype=torch.float64, device=dev)
    cbuf = torch.zeros(groups * fe, dtype=torch.float64, device=dev)
    uc, uf = b.coarse.clone(), b.fine.clone()
    fc, ff = b.coarse.clone(), b.fine.clone()
    BOTH, OUTER = api.FT_HALF_BOTH, api.FT_HALF_OUTER
    unfused = [
        ("gather_fine_faces", lambda: api.gather_patch_faces(p, k, b.orientation, b.fine_offset, offs, BOTH, U, uf, fbuf)),
        ("restrict_faces", lambda: api.restrict_faces(rop, b.orientation, b.subface, goffs, offs, U, fbuf, cbuf)),
        ("scatter_coarse_halos", lambda: api.scatter_patch_faces(p, k, gface, gpatch, gbuf, OUTER, U, cbuf, uc)),
        ("gather_coarse_faces", lambda: api.gather_patch_faces(p, k, gface, gpatch, gbuf, BOTH, U, uc, cbuf)),
        ("interpolate_faces", lambda: api.interpolate_faces(iop, b.orientation, b.subface, goffs, offs, U, cbuf, fbuf)),
        ("scatter_fine_halos", lambda: api.scatter_patch_faces(p, k, b.orientation, b.fine_offset, offs, OUTER, U, fbuf, uf)),
    ]
    fused = [
        ("restrict_patches", lambda: api.restrict_patches(rop, *d, U, ff, fc)),
        ("interpolate_patches", lambda: api.interpolate_patches(iop, *d, U, fc, ff)),
    ]
    for _, fn in unfused + fused:
        fn()
    torch.cuda.synchronize()
    same = bool(torch.equal(uc, fc) and torch.equal(uf, ff))
    ms_u, kern_u = run_steps(unfused, args.steps, args.warmup, torch)
    ms_f, kern_f = run_steps(fused, args.steps, args.warmup, torch)
    produced = n * (9 * k + k) * (p // 3) ** 2 * U
    # algorithmic bytes: restriction reads each fine face's stencil cells and
    # writes its segment; interpolation reads the union of the nine subfaces'
    # stencil cells of each coarse face and writes every fine halo
    o_np = b.orientation.cpu().numpy()
    s_np = b.subface.cpu().numpy()
    rbytes = algorithmic_bytes(rop, o_np, s_np, U, 8)
    union = {}
    rows_per_face = 0
    for o in range(6):
        cols_o = set()
        for s_ in range(9):
            rows, cols, vals = iop.segment(o, s_)
            cols_o.update(np.unique(cols[vals != 0]).tolist())
            rows_per_face = len(np.unique(rows))
        union[o] = len(cols_o)
    ibytes = (sum(union[int(o)] for o in o_np[::9]) + n * rows_per_face) * U * 8
    return {"workload": f"{n} fine patches of 9^3 cells with halo depth 3, nine per coarse face "
                        f"({groups} coarse patches), Taylor-3, U=59, FP64, restrict then interpolate",
            "ghost_cell_unknowns_per_step": produced,
            "unfused_ms_per_step": ms_u, "fused_ms_per_step": ms_f, "speedup": ms_u / ms_f,
            "fused_value": produced / (ms_f * 1e-3),
            "fused_equals_unfused_bitwise": same,
            "kernels_ms": {**{f"unfused/{kk}": round(v, 4) for kk, v in kern_u.items()},
                           **{f"fused/{kk}": round(v, 4) for kk, v in kern_f.items()}},
            "fused_GB/s": {"restrict_patches": round(rbytes / (kern_f["restrict_patches"] * 1e-3) / 1e9, 1),
                           "interpolate_patches": round(ibytes / (kern_f["interpolate_patches"] * 1e-3) / 1e9, 1)},
            "alg_bytes": {"restrict_patches": rbytes, "interpolate_patches": ibytes}}


def mesh_patches_leg(args, torch, api, wl):
    """The transition zone of a synthetic AMR mesh as patches (workload 8,
    Taylor-3, p=9, k=3, U=59): a step restricts every fine leaf into its
    coarse leaf's halo and then interpolates every fine halo, in place in one
    pool of patches.  FP64 per-call (two launches per step, eager), FP64 plan
    over patches with all steps in one captured graph, and the float32
    split-bfloat16 plan in a graph; error of one mixed step vs one FP64
    step."""
    mp = wl.mesh_patches(n_meshes=args.mesh_patch_meshes, device="cuda:0", dtype=torch.float64)
    U, steps = mp.U, args.mesh_steps
    rop = api.build_transfer_operator(api.FT_RESTRICT, 3, mp.p, mp.k)
    iop = api.build_transfer_operator(api.FT_INTERPOLATE, 3, mp.p, mp.k)
    d = (mp.orientation, mp.subface, mp.coarse_offset, mp.fine_offset)
    produced = mp.n * (9 * mp.k + mp.k) * (mp.p // 3) ** 2 * U
    pool64 = mp.pool
    pool32 = pool64.float()
    rounded = pool32.double()  # FP64 step on the float32-rounded inputs (kernel error)

    def step64():
        api.restrict_patches(rop, *d, U, pool64, pool64)
        api.interpolate_patches(iop, *d, U, pool64, pool64)

    flags = api.FT_PLAN_RESTRICT_FIRST | api.FT_PLAN_PATCHES
    plan32 = api.build_transfer_plan([(rop, *d), (iop, *d)], U, pool32, pool32, mode=api.FT_F32_BF16X6,
                                     flags=flags)
    step64()
    api.restrict_patches(rop, *d, U, rounded, rounded)
    api.interpolate_patches(iop, *d, U, rounded, rounded)
    plan32.run()
    torch.cuda.synchronize()
    err, kerr, scale = 0.0, 0.0, float(pool64.abs().max())
    for c0 in range(0, pool64.numel(), 1 << 28):
        a = pool64[c0:c0 + (1 << 28)]
        r = rounded[c0:c0 + (1 << 28)]
        b = pool32[c0:c0 + (1 << 28)].double()
        err = max(err, float((a - b).abs().max()))
        kerr = max(kerr, float((r - b).abs().max()))
    del rounded
    ms64, _ = run_steps([("f64_step", step64)], args.steps, args.warmup, torch)
    plan64 = api.build_transfer_plan([(rop, *d), (iop, *d)], U, pool64, pool64, flags=flags)
    out = {"workload": f"transition zone of {args.mesh_patch_meshes} seeded 3-level AMR mesh(es) as patches "
                       f"({mp.n_patches} patches of 9^3 cells with halo depth 3, one pool), Taylor-3, U=59, "
                       "restrict then interpolate in place",
           "hanging_faces": mp.n, "patches": mp.n_patches, "steps": steps,
           "ghost_cell_unknowns_per_step": produced, "f64_eager_ms_per_step": ms64,
           "mixed_max_rel_err_one_step": err / scale, "mixed_kernel_max_rel_err_one_step": kerr / scale}
    for label, plan in (("f64_plan_graph", plan64), ("bf16x6_plan_graph", plan32)):
        best, _ = plan.autotune(reps=3)
        graph = plan.capture(steps=steps)
        graph.launch()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        graph.launch()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        out[label] = {"ms_per_step": ms, "value": produced / (ms * 1e-3), "speedup_vs_f64_eager": ms64 / ms,
                      "schedule": api.unpack_schedule(best)}
        del graph
    return out


def faces_2d_leg(args, torch, api, wl):
    """Two-dimensional faces (p=9, k=3, U=59, FP64): the headline step's
    launches (three schemes, restrict then interpolate) on 2D face buffers."""
    import numpy as np

    p, k, U = 9, 3, 59
    b = wl.faces_2d(args.faces_2d, p, k, U, seed=wl.SEED_BASE + 7, device="cuda:0")
    n = b.n
    c_out, f_out = b.coarse.clone(), b.fine.clone()
    d = (b.orientation, b.subface, b.coarse_offset, b.fine_offset)
    launches, ops = [], {}
    for scheme in (1, 2, 3):
        rop = api.build_transfer_operator(api.FT_RESTRICT, scheme, p, k, api.FT_BUILD_2D)
        iop = api.build_transfer_operator(api.FT_INTERPOLATE, scheme, p, k, api.FT_BUILD_2D)
        ops[("restrict", scheme)], ops[("interpolate", scheme)] = rop, iop
        launches.append((f"restrict_{SCHEME_NAMES[scheme]}",
                         lambda rop=rop: api.restrict_faces(rop, *d, U, b.fine, c_out)))
        launches.append((f"interpolate_{SCHEME_NAMES[scheme]}",
                         lambda iop=iop: api.interpolate_faces(iop, *d, U, b.coarse, f_out)))
    ms, kern = run_steps(launches, args.steps, args.warmup, torch)
    o_np, s_np = b.orientation.cpu().numpy(), b.subface.cpu().numpy()
    kernels = {}
    for (direction, scheme), op in ops.items():
        name = f"{direction}_{SCHEME_NAMES[scheme]}"
        per = {}
        for o in range(4):
            for s_ in range(3):
                rows, cols, vals = op.segment(o, s_)
                per[(o, s_)] = (len(np.unique(cols[vals != 0])) + len(np.unique(rows))) * U * 8
        counts = np.zeros((4, 3), dtype=np.int64)
        np.add.at(counts, (o_np, s_np), 1)
        nbytes = int(sum(per[(o, s_)] * counts[o, s_] for o in range(4) for s_ in range(3)))
        kernels[name] = {"ms": round(kern[name], 4), "alg_bytes": nbytes,
                         "GB/s": round(nbytes / (kern[name] * 1e-3) / 1e9, 1)}
    produced = 3 * n * (3 * k * (p // 3) + k * (p // 3)) * U
    # the same step in float32 storage with the six-term matrix-core form
    c32, f32 = b.coarse.float(), b.fine.float()
    c32_out, f32_out = c32.clone(), f32.clone()
    launches32 = []
    for scheme in (1, 2, 3):
        rop, iop = ops[("restrict", scheme)], ops[("interpolate", scheme)]
        launches32.append((f"restrict_{SCHEME_NAMES[scheme]}",
                           lambda rop=rop: api.restrict_faces(rop, *d, U, f32, c32_out, mode=api.FT_F32_BF16X6)))
        launches32.append((f"interpolate_{SCHEME_NAMES[scheme]}",
                           lambda iop=iop: api.interpolate_faces(iop, *d, U, c32, f32_out,
                                                                 mode=api.FT_F32_BF16X6)))
    ms32, kern32 = run_steps(launches32, args.steps, args.warmup, torch)
    errs = {}
    for nm, got, ref in (("interpolate_taylor3", f32_out, f_out), ("restrict_taylor3", c32_out, c_out)):
        g, rr = got.view(-1, U).double(), ref.view(-1, U)
        errs[nm] = float(((g - rr).abs().amax(dim=0) / rr.abs().amax(dim=0)).max())
    return {"workload": f"{n} two-dimensional hanging faces, p=9, k=3, U=59, FP64; "
                        "dlinear+taylor2+taylor3; restrict+interpolate",
            "ms_per_step": ms, "value": produced / (ms * 1e-3), "kernels": kernels,
            "bf16x6": {"ms_per_step": ms32, "value": produced / (ms32 * 1e-3), "speedup_vs_f64": ms / ms32,
                       "kernels_ms": {kk: round(v, 4) for kk, v in kern32.items()},
                       "max_rel_err_vs_f64": errs}}


def small_u_leg(args, torch, api, wl):
    """Latency of one call on a cache-resident batch: 64 hanging faces, p=9,
    k=3, one unknown per cell (every orientation/subface pair present),
    d-linear and Taylor-2, FP64, both directions.  `call_us`: mean GPU time
    per call between events recorded around each call; `stream_us`: mean
    time per call of `reps` calls issued back to back (host launch cost
    included); `host_us`: host time to issue one call; `graph_us`: mean time
    per call of `reps` calls replayed from one captured graph."""
    b = wl.workload1(device="cuda:0")
    d = (b.orientation, b.subface, b.coarse_offset, b.fine_offset)
    reps = args.small_u_reps
    out = {"workload": "64 faces, p=9, k=3, U=1, FP64 (cubic + sine field)", "reps": reps}
    for scheme in (1, 2):
        for direction in (api.FT_INTERPOLATE, api.FT_RESTRICT):
            op = api.build_transfer_operator(direction, scheme, 9, 3)
            c, f = b.coarse.clone(), b.fine.clone()
            if direction == api.FT_INTERPOLATE:
                fn = lambda op=op, c=c, f=f: api.interpolate_faces(op, *d, 1, b.coarse, f)
            else:
                fn = lambda op=op, c=c, f=f: api.restrict_faces(op, *d, 1, b.fine, c)
            for _ in range(20):
                fn()
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            for a, z in ev:
                a.record()
                fn()
                z.record()
            torch.cuda.synchronize()
            call_us = 1e3 * sum(a.elapsed_time(z) for a, z in ev) / reps
            a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            t1 = time.perf_counter()
            z.record()
            torch.cuda.synchronize()
            name = ("interpolate_" if direction == api.FT_INTERPOLATE else "restrict_") + SCHEME_NAMES[scheme]
            out[name] = {"call_us": round(call_us, 2), "stream_us": round(1e3 * a.elapsed_time(z) / reps, 2),
                         "host_us": round(1e6 * (t1 - t0) / reps, 2)}
            # the same calls replayed from a captured graph: GPU time per call
            # without the host's launch cost
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, capture_error_mode="relaxed"):
                for _ in range(reps):
                    fn()
            g.replay()
            torch.cuda.synchronize()
            a.record()
            g.replay()
            z.record()
            torch.cuda.synchronize()
            out[name]["graph_us"] = round(1e3 * a.elapsed_time(z) / reps, 2)
            del g
    return out


def cpu_baseline(batch, n_faces, torch):
    """The FP64 oracle on the host, on the first n_faces faces of the same
    batch; operators are built before timing (the paper times repeated calls
    without reallocation) and their build is timed separately.  Median of
    three runs with the host BLAS threads, plus the median of three
    single-thread runs on a tenth of the sample."""
    import statistics

    import threadpoolctl

    import oracle

    U, p, k = batch.U, batch.p, batch.k
    E = batch.face_elems
    coarse = batch.coarse[: n_faces * E].cpu().numpy()
    fine = batch.fine[: n_faces * E].cpu().numpy()
    o = batch.orientation[:n_faces].cpu().numpy()
    s = batch.subface[:n_faces].cpu().numpy()
    co = batch.coarse_offset[:n_faces].cpu().numpy()
    fo = batch.fine_offset[:n_faces].cpu().numpy()
    oracle.clear_operator_cache()
    t0 = time.perf_counter()
    for scheme in (1, 2, 3):
        for oo in range(6):
            for ss in range(9):
                oracle.interpolation_operator(scheme, p, k, oo, ss)
                oracle.restriction_operator(scheme, p, k, oo, ss)
    build_s = time.perf_counter() - t0
    threads = max((i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()), default=1)

    def run(n):
        t = time.perf_counter()
        for scheme in (1, 2, 3):
            oracle.restrict_faces(scheme, p, k, o[:n], s[:n], co[:n], fo[:n], U, fine, coarse)
            oracle.interpolate_faces(scheme, p, k, o[:n], s[:n], co[:n], fo[:n], U, coarse, fine)
        return time.perf_counter() - t

    per_face = 3 * (9 * k * (p // 3) ** 2 + k * (p // 3) ** 2) * U
    dt = statistics.median(run(n_faces) for _ in range(3))
    n1 = max(1, n_faces // 10)
    with threadpoolctl.threadpool_limits(1):
        dt1 = statistics.median(run(n1) for _ in range(3))
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": per_face * n_faces / dt,
        "unit": "ghost-cell-unknowns/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"first {n_faces} of {batch.n} faces, all 3 schemes x restrict+interpolate, "
                  f"median of 3 runs {dt:.1f} s wall with {threads} BLAS threads",
        "single_thread_value": per_face * n1 / dt1,
        "single_thread_sample": f"first {n1} faces, median of 3 runs {dt1:.1f} s wall",
        "operator_build_s": build_s,
        "host": {"cpu": cpu_model, "nproc": os.cpu_count()},
    }


def _sig(x, digits=4):
    """x rounded to `digits` significant digits (JSON-friendly)."""
    return float(f"{x:.{digits}g}") if isinstance(x, (int, float)) and x is not None else x


def headline(result, detail_path):
    """The one-line record: the FP64 step of the benchmark workload with its
    roofline and CPU baseline, plus a short summary of every other leg (the
    full records are in the detail file)."""
    keys = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
            "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "hbm_frac_step")
    h = {k_: result[k_] for k_ in keys if k_ in result}
    h["kernels_ms_GBs"] = {k_: [v["ms"], v["GB/s"]] for k_, v in result["kernels"].items()}
    if "cpu_baseline" in result:
        cb = result["cpu_baseline"]
        h["cpu_baseline"] = {k_: cb[k_] for k_ in ("value", "unit", "cores", "kind", "sample")}
        h["cpu_baseline"]["single_thread_value"] = _sig(cb["single_thread_value"])
    if "mixed" in result:
        m = {"workload": "same faces, unknowns scaled 1e-6..1e3, float32 storage; err = worst "
                         "per-unknown max relative error of Taylor-3 outputs vs the FP64 GPU path "
                         "(e2e: on FP64 inputs; arith: on the float32-rounded inputs)"}
        for label, v in result["mixed"].items():
            if not isinstance(v, dict):
                continue
            e, ka = v["err_vs_f64_gpu"], v["err_vs_f64_gpu_on_rounded_inputs"]
            m[label] = {"ms": _sig(v["ms_per_step"]), "speedup": _sig(v["speedup_vs_f64"], 3),
                        "interp_err_e2e": _sig(e["interpolate_taylor3"]["max_rel"], 2),
                        "restrict_err_e2e": _sig(e["restrict_taylor3"]["max_rel"], 2),
                        "interp_err_arith": _sig(ka["interpolate_taylor3"]["max_rel"], 2),
                        "restrict_err_arith": _sig(ka["restrict_taylor3"]["max_rel"], 2)}
            if "interp_ms" in v:
                m[label]["interp_t3_ms"] = v["interp_ms"]
        h["mixed"] = m
    if "small_u" in result:
        h["small_u_latency_us"] = {k_: [v["call_us"], v["graph_us"]] for k_, v in result["small_u"].items()
                                   if isinstance(v, dict)}
    if "batched" in result:
        b = result["batched"]
        h["batched"] = {"faces": b["faces"], "f64_per_batch_ms": _sig(b["f64_per_batch_ms"]),
                        "f64_plan_graph_ms": _sig(b["f64_plan_graph_ms"])}
        for label in ("bf16x6", "f32"):
            if label in b:
                h["batched"][label] = {"graph_ms": _sig(b[label]["graph_ms"]),
                                       "speedup_vs_f64_plan_graph": _sig(b[label]["speedup_vs_f64_plan_graph"], 3),
                                       "err": _sig(b[label]["max_rel_err_vs_f64"], 2)}
    if "mesh" in result:
        me = result["mesh"]
        h["mesh"] = {"faces": me["hanging_faces"], "f64_ms": _sig(me["f64_ms_per_step"]),
                     "f64_plan_graph_ms": _sig(me["f64_plan_graph_ms_per_step"]),
                     "mixed_graph_ms": _sig(me["mixed_graph_ms_per_step"]),
                     "speedup_vs_f64_plan_graph": _sig(me["speedup_vs_f64_plan_graph"], 3),
                     "err_e2e": _sig(me["mixed_max_rel_err_one_step"], 2),
                     "err_arith": _sig(me["mixed_kernel_max_rel_err_one_step"], 2)}
        if "f64_restrict_graph_ms_per_step" in me:
            h["mesh"]["f64_restrict_mixed_graph_ms"] = _sig(me["f64_restrict_graph_ms_per_step"])
            h["mesh"]["f64_restrict_speedup"] = _sig(me["f64_restrict_speedup_vs_f64_plan_graph"], 3)
            h["mesh"]["f64_restrict_err_e2e"] = _sig(me["f64_restrict_max_rel_err_one_step"], 2)
            h["mesh"]["f64_restrict_err_arith"] = _sig(me["f64_restrict_kernel_max_rel_err_one_step"], 2)
    if "mesh_patches" in result:
        mp = result["mesh_patches"]
        h["mesh_patches"] = {"f64_plan_graph_ms": _sig(mp["f64_plan_graph"]["ms_per_step"]),
                             "bf16x6_plan_graph_ms": _sig(mp["bf16x6_plan_graph"]["ms_per_step"])}
    if "patches" in result:
        pa = result["patches"]
        h["patches"] = {"unfused_ms": _sig(pa["unfused_ms_per_step"]), "fused_ms": _sig(pa["fused_ms_per_step"]),
                        "bitwise_equal": pa["fused_equals_unfused_bitwise"]}
    if "faces_2d" in result:
        f2 = result["faces_2d"]
        h["faces_2d"] = {"ms": _sig(f2["ms_per_step"]), "bf16x6_ms": _sig(f2["bf16x6"]["ms_per_step"])}
    if "convergence" in result:
        h["reports"] = ["convergence", "operator_build", "runtime_vs_p"]
    h["detail"] = os.path.relpath(detail_path, ROOT) if detail_path else None
    return h


def write_detail(path, result):
    """Write the full record of every leg; returns the path, or None."""
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        with open(path, "w") as fh:
            json.dump(result, fh, indent=1)
        return path
    except OSError as exc:
        progress(f"could not write {path}: {exc}")
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus above 1 is not supported "
                                   "(faces would shard across GPUs by fine-patch owner)"}))
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy:
        calibrate_copy(torch)
        return

    from paper_2504_15814_amd import api
    from paper_2504_15814_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    batch = wl.workload2(n_faces=args.faces, device=dev)
    U, p, k, n = batch.U, batch.p, batch.k, batch.n
    orient_np = batch.orientation.cpu().numpy()
    sub_np = batch.subface.cpu().numpy()

    def make_launches(dtype, mode=None, batch=batch, restrict_mode=None):
        # restrict_mode FT_F64_TO_F32: restriction reads the float64 fine data
        # and writes float32 coarse faces; the rest is stored in `dtype`.
        coarse_in = batch.coarse.to(dtype)
        fine_in = batch.fine if restrict_mode == api.FT_F64_TO_F32 else batch.fine.to(dtype)
        coarse_out = coarse_in.clone()
        fine_out = batch.fine.to(dtype).clone()
        launches, ops = [], {}
        for scheme in (1, 2, 3):
            rop = api.build_transfer_operator(api.FT_RESTRICT, scheme, p, k)
            iop = api.build_transfer_operator(api.FT_INTERPOLATE, scheme, p, k)
            ops[("restrict", scheme)] = rop
            ops[("interpolate", scheme)] = iop

            def r(rop=rop):
                api.restrict_faces(rop, batch.orientation, batch.subface, batch.coarse_offset,
                                   batch.fine_offset, U, fine_in, coarse_out,
                                   mode=mode if restrict_mode is None else restrict_mode)

            def i(iop=iop):
                api.interpolate_faces(iop, batch.orientation, batch.subface, batch.coarse_offset,
                                      batch.fine_offset, U, coarse_in, fine_out, mode=mode)

            launches.append((f"restrict_{SCHEME_NAMES[scheme]}", r))
            launches.append((f"interpolate_{SCHEME_NAMES[scheme]}", i))
        return launches, ops, (coarse_out, fine_out)

    launches, ops, outs64 = make_launches(torch.float64)
    ms, kern_ms = run_steps(launches, args.steps, args.warmup, torch)
    progress(f"float64 step: {ms:.3f} ms")
    produced = 3 * n * (9 * k * (p // 3) ** 2 + k * (p // 3) ** 2) * U
    value = produced / (ms * 1e-3)

    kernels = {}
    for (direction, scheme), op in ops.items():
        name = f"{direction}_{SCHEME_NAMES[scheme]}"
        nbytes = algorithmic_bytes(op, orient_np, sub_np, U, 8)
        t = kern_ms[name]
        kernels[name] = {"ms": round(t, 4), "alg_bytes": nbytes, "GB/s": round(nbytes / (t * 1e-3) / 1e9, 1)}
    dom = max(kernels, key=lambda kk: kernels[kk]["ms"])
    ach = kernels[dom]["GB/s"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(dom)}
    total_bytes = sum(v["alg_bytes"] for v in kernels.values())

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "ghost-cell-unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "hanging faces p=9 k=3 U=59 FP64; dlinear+taylor2+taylor3; restrict+interpolate",
                   "faces": n, "p": p, "k": k, "unknowns": U},
        "hbm_frac_step": round(total_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "kernels": kernels,
    }

    if not args.no_mixed:
        del launches, outs64
        # Precision workload: the same faces with unknown u scaled by
        # 10^(-6 + 9u/58).  FP64 Taylor-3 references on the float64 inputs and
        # on the float32-rounded inputs: the difference to the second is the
        # error of the float32 arithmetic alone (the restriction's
        # extrapolation rows amplify the input rounding).
        b3 = wl.workload3(n_faces=args.faces, device=dev)
        d3 = (b3.orientation, b3.subface, b3.coarse_offset, b3.fine_offset)
        rop3 = api.build_transfer_operator(api.FT_RESTRICT, 3, p, k)
        iop3 = api.build_transfer_operator(api.FT_INTERPOLATE, 3, p, k)
        ref_c, ref_f = b3.coarse.clone(), b3.fine.clone()
        api.restrict_faces(rop3, *d3, U, b3.fine, ref_c)
        api.interpolate_faces(iop3, *d3, U, b3.coarse, ref_f)
        rin_c, rin_f = b3.coarse.float().double(), b3.fine.float().double()
        rref_c, rref_f = rin_c.clone(), rin_f.clone()
        api.restrict_faces(rop3, *d3, U, rin_f, rref_c)
        api.interpolate_faces(iop3, *d3, U, rin_c, rref_f)
        torch.cuda.synchronize()
        del rin_c, rin_f, rop3, iop3

        def rel_errors(got, ref):
            g = got.view(-1, U).double()
            rr = ref.view(-1, U)
            emax = (g - rr).abs().amax(dim=0) / rr.abs().amax(dim=0)
            erms = (g - rr).pow(2).mean(dim=0).sqrt() / rr.pow(2).mean(dim=0).sqrt()
            return {"max_rel": float(emax.max()), "rms_rel": float(erms.max()),
                    "max_rel_per_unknown": [float(f"{v:.2e}") for v in emax.tolist()]}

        result["mixed"] = {"workload": "hanging faces p=9 k=3 U=59, unknown u scaled by 10^(-6+9u/58); "
                                       "float32 storage, same step as the FP64 headline; errors of "
                                       "Taylor-3 outputs per unknown"}
        # f64_restrict_bf16x6: float64 fine data read by restriction, which
        # writes float32 coarse faces (one rounding of the FP64 result);
        # interpolation in six split terms into float32 fine halos.
        for label, mode, rmode in (("f32", api.FT_F32, None), ("bf16x3", api.FT_F32_BF16X3, None),
                                   ("bf16x6", api.FT_F32_BF16X6, None),
                                   ("f64_restrict_bf16x6", api.FT_F32_BF16X6, api.FT_F64_TO_F32)):
            mlaunches, mops, mouts = make_launches(torch.float32, mode, b3, restrict_mode=rmode)
            mms, mkern = run_steps(mlaunches, args.steps, args.warmup, torch)
            errs, kerrs = {}, {}
            for nm, got, ref, rref in (("interpolate_taylor3", mouts[1], ref_f, rref_f),
                                       ("restrict_taylor3", mouts[0], ref_c,
                                        ref_c if rmode is not None else rref_c)):
                errs[nm] = rel_errors(got, ref)
                kerrs[nm] = rel_errors(got, rref)
            progress(f"float32 {label} step: {mms:.3f} ms")
            result["mixed"][label] = {
                "value": produced / (mms * 1e-3),
                "ms_per_step": mms,
                "speedup_vs_f64": ms / mms,
                "kernels_ms": {kk: round(v, 4) for kk, v in mkern.items()},
                "err_vs_f64_gpu": errs,
                "err_vs_f64_gpu_on_rounded_inputs": kerrs,
            }
            del mlaunches, mops, mouts
        del b3, ref_c, ref_f, rref_c, rref_f

    if args.batched_faces > 0:
        result["batched"] = batched_leg(args, torch, api, wl)
        progress("batched leg done")

    if args.mesh_meshes > 0:
        result["mesh"] = mesh_leg(args, torch, api, wl)
        progress("mesh leg done")

    if args.mesh_patch_meshes > 0:
        result["mesh_patches"] = mesh_patches_leg(args, torch, api, wl)
        progress("mesh patch leg done")

    if args.faces_2d > 0:
        result["faces_2d"] = faces_2d_leg(args, torch, api, wl)
        progress("2D leg done")

    if args.patch_faces > 0:
        result["patches"] = patches_leg(args, torch, api, wl)
        progress("patch leg done")

    if args.small_u_reps > 0:
        result["small_u"] = small_u_leg(args, torch, api, wl)
        progress("small-U leg done: " + json.dumps({k_: v for k_, v in result["small_u"].items()
                                                     if isinstance(v, dict)}))

    if args.cpu_faces > 0:
        result["cpu_baseline"] = cpu_baseline(batch, min(args.cpu_faces, n), torch)
        progress("cpu baseline done")

    if not args.no_reports:
        from paper_2504_15814_amd import experiments

        del batch  # free the benchmark buffers before the reports allocate theirs
        torch.cuda.empty_cache()
        result["convergence"] = experiments.convergence(device=dev)
        result["operator_build"] = experiments.operator_build(device=dev)
        result["runtime_vs_p"] = experiments.runtime_vs_p(device=dev)
        progress("reports done")

    path = write_detail(args.detail, result)
    print(json.dumps(headline(result, path), separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
