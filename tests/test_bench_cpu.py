"""bench.py's host-side contract (no GPU): one GPU only, and a compact
headline record for the last stdout line."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_headline_is_compact_and_complete():
    kernels = {f"{d}_{s}": {"ms": 0.5, "alg_bytes": 2.5e9, "GB/s": 5000.0}
               for d in ("restrict", "interpolate") for s in ("dlinear", "taylor2", "taylor3")}
    err = {"max_rel": 1e-7, "rms_rel": 1e-8, "max_rel_per_unknown": [1e-7] * 59}
    mixed = {"workload": "w"}
    for label in ("f32", "bf16x3", "bf16x6", "f64_restrict_bf16x6"):
        mixed[label] = {"ms_per_step": 2.0, "speedup_vs_f64": 1.9,
                        "err_vs_f64_gpu": {"interpolate_taylor3": err, "restrict_taylor3": err},
                        "err_vs_f64_gpu_on_rounded_inputs": {"interpolate_taylor3": err, "restrict_taylor3": err}}
    result = {"metric": bench.METRIC, "value": 2.5e11, "unit": "ghost-cell-unknowns/s", "n_gpus": 1,
              "steps": 100, "warmup": 3, "ms_per_step": 3.85, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f64", "data": "synthetic",
              "config": {"workload": "w", "faces": 20000, "p": 9, "k": 3, "unknowns": 59},
              "roofline": {"bound": "hbm", "kernel": "interpolate_taylor3", "achieved": 3900.0, "peak": 8000.0,
                           "unit": "GB/s", "frac": 0.49, "traffic": 3.1e9},
              "hbm_frac_step": 0.53, "kernels": kernels, "mixed": mixed,
              "cpu_baseline": {"value": 1.4e8, "unit": "ghost-cell-unknowns/s", "cores": 16, "kind": "oracle",
                               "sample": "s", "single_thread_value": 2.7e7}}
    h = bench.headline(result, None)
    line = json.dumps(h)
    assert len(line) < 4096
    for key in ("metric", "value", "unit", "n_gpus", "steps", "ms_per_step", "dtype", "config", "roofline",
                "cpu_baseline"):
        assert key in h, key
    assert set(h["mixed"]) >= {"f32", "bf16x3", "bf16x6", "f64_restrict_bf16x6"}
    assert h["cpu_baseline"]["kind"] == "oracle"
