"""Section 5.1's accuracy experiment on the GPU path: interpolating and
restricting a plane sine wave at coarse widths 1/9 ... 1/729 gives maximum
errors of order 2 (d-linear), 3 (Taylor-2) and 4 (Taylor-3) in both
directions, and the same errors as the oracle on the same samples.

The construction experiment (Section 5.3) is a timing report; its test only
checks that it runs and that a precomputed operator beats one built per call.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2504_15814_amd import experiments as ex
from tests.gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu

ORDERS = {"dlinear": 2.0, "taylor2": 3.0, "taylor3": 4.0}
WIDTHS = (9, 27, 81, 243, 729)


def oracle_errors(scheme, direction, p=9, k=3):
    errs = []
    for w in WIDTHS:
        o, s, off, vc, vf = ex._faces(p, k, 1.0 / w, "cpu")
        o, s, off = o.numpy(), s.numpy(), off.numpy()
        sent = -7.25e11
        if direction == 0:
            out = oracle.interpolate_faces(scheme, p, k, o, s, off, off, 1, vc.numpy(), np.full(vf.numel(), sent))
            exact = vf.numpy()
        else:
            out = oracle.restrict_faces(scheme, p, k, o, s, off, off, 1, vf.numpy(), np.full(vc.numel(), sent))
            exact = vc.numpy()
        m = out != sent
        errs.append(float(np.abs(out[m] - exact[m]).max()))
    return errs


def test_convergence_orders_match_the_oracle():
    dev = require_gpu()
    res = ex.convergence(device=dev, widths=WIDTHS)
    for scheme, name in ex.SCHEMES.items():
        for direction, dname in ((0, "interpolate"), (1, "restrict")):
            r = res[name][dname]
            assert abs(r["order"] - ORDERS[name]) < 0.3, (name, dname, r["order"])
            want = oracle_errors(scheme, direction)
            got = r["max_err"]
            for g, w in zip(got, want):
                # the same samples and operators: the errors differ by rounding only
                assert abs(g - w) <= 1e-3 * w + 1e-13, (name, dname, got, want)


def test_operator_build_report():
    dev = require_gpu()
    rep = ex.operator_build(device=dev, n_faces=2000, U=59, reps=1)
    assert set(rep["operators"]) == {f"{d}_{s}" for d in ("interpolate", "restrict") for s in ex.SCHEMES.values()}
    for v in rep["operators"].values():
        assert v["host_build_ms"] > 0 and v["apply_ms"] > 0
        assert v["per_call_build_slowdown"] > 1
