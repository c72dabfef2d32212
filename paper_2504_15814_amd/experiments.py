"""The paper's accuracy and construction experiments, run through the library
on the GPU.

convergence()       Section 5.1: interpolate and restrict a smooth field
                    (a plane sine wave) at shrinking mesh widths and fit the
                    order of the maximum error, for every scheme and both
                    directions.  Taylor expansions of degree D give order
                    D + 1 at points; the d-linear scheme gives order 2.
operator_build()    Section 5.3: the paper builds the fit matrices on every
                    call and notes that precomputing them would pay; this
                    times one operator build (host fit + upload) against one
                    batched application, i.e. what a per-call construction
                    would add.
runtime_vs_p()      Section 5.3: runtime of every scheme as the patch size p
                    grows (halo depth 3, repeated calls without
                    reallocation), per face and as algorithmic GB/s, both
                    directions, including sizes that are not multiples of 3.

Run as ``python -m paper_2504_15814_amd.experiments`` (one JSON object).
"""

import json
import math
import time

import numpy as np
import torch

from . import api
from .workloads import coarse_centres, fine_centres

SCHEMES = {1: "dlinear", 2: "taylor2", 3: "taylor3"}
KAPPA = (2.1, 1.3, 1.7)
PHASE = 0.4
ORIGIN = (0.31, 0.27, 0.43)


def _sine(pos):
    return torch.sin(pos[..., 0] * KAPPA[0] + pos[..., 1] * KAPPA[1] + pos[..., 2] * KAPPA[2] + PHASE)


def _faces(p, k, h_c, device):
    """All 54 (orientation, subface) pairs as one batch of U = 1 faces, both
    buffers sampled from the sine wave at coarse width h_c.  Returns the
    descriptors, the buffers, and the exact values at every centre."""
    pairs = [(o, s) for o in range(6) for s in range(9)]
    n = len(pairs)
    ncell = 2 * k * p * p
    h_f = h_c / 3.0
    origin = torch.tensor(ORIGIN, dtype=torch.float64, device=device)
    coarse = torch.stack([coarse_centres(o, p, k, device) for o, _ in pairs]) * h_f + origin
    fine = torch.stack([fine_centres(o, p, k, s, device) for o, s in pairs]) * h_f + origin
    vc = _sine(coarse).reshape(-1).contiguous()
    vf = _sine(fine).reshape(-1).contiguous()
    o = torch.tensor([o for o, _ in pairs], dtype=torch.int8, device=device)
    s = torch.tensor([s for _, s in pairs], dtype=torch.int8, device=device)
    off = torch.arange(n, dtype=torch.int64, device=device) * ncell
    return o, s, off, vc, vf


def convergence(device="cuda:0", p=9, k=3, widths=(9, 27, 81, 243, 729)):
    """Maximum error of every scheme and direction at coarse widths 1/w, and
    the order fitted over the finest three widths (least squares on
    log error against log width)."""
    out = {}
    sentinel = -7.25e11
    for scheme, name in SCHEMES.items():
        ops = {d: api.build_transfer_operator(d, scheme, p, k) for d in (0, 1)}
        res = {}
        for d, dname in ((0, "interpolate"), (1, "restrict")):
            errs = []
            for w in widths:
                o, s, off, vc, vf = _faces(p, k, 1.0 / w, device)
                if d == 0:
                    dst = torch.full_like(vf, sentinel)
                    api.interpolate_faces(ops[0], o, s, off, off, 1, vc, dst)
                    exact = vf
                else:
                    dst = torch.full_like(vc, sentinel)
                    api.restrict_faces(ops[1], o, s, off, off, 1, vf, dst)
                    exact = vc
                torch.cuda.synchronize()
                written = dst != sentinel
                errs.append(float((dst[written] - exact[written]).abs().max()))
            x = np.log([1.0 / w for w in widths[-3:]])
            y = np.log(np.maximum(errs[-3:], 1e-300))
            slope = float(np.polyfit(x, y, 1)[0])
            res[dname] = {"h_coarse": [1.0 / w for w in widths], "max_err": errs, "order": slope}
        out[name] = res
    return out


def operator_build(device="cuda:0", p=9, k=3, n_faces=20000, U=59, reps=3):
    """Per (direction, scheme): median host build time, median build + upload
    time, and the time of one FP64 application to n_faces faces."""
    out = {}
    ncell = 2 * k * p * p
    gen = torch.Generator(device=device).manual_seed(7)
    src = torch.randn(n_faces * ncell * U, generator=gen, dtype=torch.float64, device=device)
    dst = torch.zeros_like(src)
    cg = torch.Generator().manual_seed(8)
    o = torch.randint(0, 6, (n_faces,), generator=cg).to(torch.int8).to(device)
    s = torch.randint(0, 9, (n_faces,), generator=cg).to(torch.int8).to(device)
    off = torch.arange(n_faces, dtype=torch.int64, device=device) * ncell * U
    for scheme, name in SCHEMES.items():
        for d, dname in ((0, "interpolate"), (1, "restrict")):
            host, full = [], []
            for _ in range(reps):
                t0 = time.perf_counter()
                h = api.build_transfer_operator(d, scheme, p, k, api.FT_BUILD_HOST_ONLY)
                host.append(time.perf_counter() - t0)
                h.destroy()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                op = api.build_transfer_operator(d, scheme, p, k)
                torch.cuda.synchronize()
                full.append(time.perf_counter() - t0)
            fn = (lambda: api.interpolate_faces(op, o, s, off, off, U, src, dst)) if d == 0 else \
                 (lambda: api.restrict_faces(op, o, s, off, off, U, src, dst))
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(5):
                fn()
            b.record()
            torch.cuda.synchronize()
            apply_ms = a.elapsed_time(b) / 5
            build_ms = 1e3 * float(np.median(host))
            out[f"{dname}_{name}"] = {
                "host_build_ms": build_ms,
                "build_and_upload_ms": 1e3 * float(np.median(full)),
                "apply_ms": apply_ms,
                "apply_us_per_face": 1e3 * apply_ms / n_faces,
                # one build per face call (what constructing the operator on
                # every call costs) against the precomputed operator
                "per_call_build_slowdown": (build_ms + apply_ms / n_faces) / (apply_ms / n_faces),
            }
            op.destroy()
    return {"p": p, "k": k, "unknowns": U, "faces": n_faces, "operators": out}


def runtime_vs_p(device="cuda:0", sizes=(6, 7, 8, 9, 12, 15, 18, 21, 24, 27), k=3, U=59, reps=10,
                 cells=20000 * 81):
    """Mean time of one batched FP64 application per scheme, direction and
    patch size; the batch holds about `cells` / p^2 faces (the same data
    volume at every p), and the report gives microseconds per face and
    algorithmic GB/s (distinct source cells with a nonzero weight plus
    destination cells, per (orientation, subface), times U x 8 bytes)."""
    out = {}
    cg = torch.Generator().manual_seed(11)
    for p in sizes:
        n = max(64, cells // (p * p))
        ncell = 2 * k * p * p
        gen = torch.Generator(device=device).manual_seed(p)
        src = torch.randn(n * ncell * U, generator=gen, dtype=torch.float64, device=device)
        dst = torch.zeros_like(src)
        o = torch.randint(0, 6, (n,), generator=cg).to(torch.int8)
        s = torch.randint(0, 9, (n,), generator=cg).to(torch.int8)
        counts = np.zeros((6, 9), dtype=np.int64)
        np.add.at(counts, (o.numpy(), s.numpy()), 1)
        o, s = o.to(device), s.to(device)
        off = torch.arange(n, dtype=torch.int64, device=device) * ncell * U
        row = {}
        for scheme, name in SCHEMES.items():
            for d, dname in ((0, "interpolate"), (1, "restrict")):
                op = api.build_transfer_operator(d, scheme, p, k)
                nbytes = 0
                for oo in range(6):
                    for ss in range(9):
                        if counts[oo, ss]:
                            r, c, v = op.segment(oo, ss)
                            nbytes += int(counts[oo, ss]) * (len(np.unique(c[v != 0])) + len(np.unique(r))) * U * 8
                fn = (lambda: api.interpolate_faces(op, o, s, off, off, U, src, dst)) if d == 0 else \
                     (lambda: api.restrict_faces(op, o, s, off, off, U, src, dst))
                fn()
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    fn()
                b.record()
                torch.cuda.synchronize()
                ms = a.elapsed_time(b) / reps
                row[f"{dname}_{name}"] = {"ms": ms, "us_per_face": 1e3 * ms / n,
                                          "alg_GB_per_s": nbytes / (ms * 1e-3) / 1e9}
                op.destroy()
        out[str(p)] = {"faces": n, **row}
        del src, dst
    return {"k": k, "unknowns": U, "sizes": out}


def main():
    torch.cuda.set_device(0)
    print(json.dumps({"convergence": convergence(), "operator_build": operator_build(),
                      "runtime_vs_p": runtime_vs_p()}))


if __name__ == "__main__":
    main()
