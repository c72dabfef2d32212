"""Pins of the two-dimensional oracle (oracle/transfer2d.py).

Positions are computed here from the conventions (never from the oracle),
and the oracle is checked against what the mathematics fixes: polynomial
reproduction (bilinear / quadratic / cubic fields, both directions, every
orientation and subface), its sharpness, unit row sums, bit-exact copies at
coinciding centres, exact-rational least squares, a hand-derived closed form
of the interior second-order fit, orientation equivariance, convergence
orders 2 / 3 / 4, and the d-linear scheme as the z-independent special case
of the three-dimensional one.
"""

from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import oracle
from oracle import transfer2d as o2
from tests import oracle_checks as chk

SHAPES = [(6, 2), (6, 3), (9, 3)]


def grid(o, p, k):
    a = o % 2
    ext = [p, p]
    ext[a] = 2 * k
    g1, g0 = np.indices((ext[1], ext[0]))
    return a, ext, np.stack([g0.ravel(), g1.ravel()], axis=1)


def coarse_centres(o, p, k):
    a, _, idx = grid(o, p, k)
    pos = 3.0 * idx + 1.5
    pos[:, a] = 3.0 * (idx[:, a] - k) + 1.5
    return pos


def fine_centres(o, p, k, s):
    a, _, idx = grid(o, p, k)
    pos = idx + 0.5
    pos[:, a] = idx[:, a] - k + 0.5
    pos[:, 1 - a] += s * p
    return pos


def exps(scheme):
    if scheme == 1:
        return [(0, 0), (1, 0), (0, 1), (1, 1)]
    return [e for e in product(range(scheme + 1), repeat=2) if sum(e) <= scheme]


def poly(pos, coeffs, ex, scale):
    x = pos / scale
    return sum(c * x[:, 0] ** e[0] * x[:, 1] ** e[1] for c, e in zip(coeffs, ex))


def reproduction_error(scheme, p, k, o, s, rng, direction, ex=None):
    ex = ex or exps(scheme)
    coeffs = rng.normal(size=len(ex))
    cv = poly(coarse_centres(o, p, k), coeffs, ex, 3.0 * p)
    fv = poly(fine_centres(o, p, k, s), coeffs, ex, 3.0 * p)
    rows, W = o2.transfer_operator(direction, scheme, p, k, o, s)
    got, want = (W @ cv, fv[rows]) if direction == 0 else (W @ fv, cv[rows])
    return np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)


@pytest.mark.parametrize("scheme", [1, 2, 3])
@pytest.mark.parametrize("p,k", SHAPES)
@pytest.mark.parametrize("direction", [0, 1])
def test_polynomial_reproduction(scheme, p, k, direction):
    rng = np.random.default_rng(100 * scheme + p + k + direction)
    worst = max(reproduction_error(scheme, p, k, o, s, rng, direction) for o in range(4) for s in range(3))
    assert worst < 1e-12, worst


@pytest.mark.parametrize("direction", [0, 1])
def test_dlinear_k1_reproduction(direction):
    rng = np.random.default_rng(5 + direction)
    worst = max(reproduction_error(1, 9, 1, o, s, rng, direction) for o in range(4) for s in range(3))
    assert worst < 1e-12


def test_reproduction_is_sharp():
    rng = np.random.default_rng(1)
    assert reproduction_error(2, 9, 3, 0, 1, rng, 0, ex=[(3, 0)]) > 1e-6
    assert reproduction_error(3, 9, 3, 0, 1, rng, 0, ex=[(2, 2)]) > 1e-6
    assert reproduction_error(1, 9, 3, 0, 1, rng, 0, ex=[(2, 0)]) > 1e-6


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_rows_sum_to_one_and_segments_tile(direction, scheme):
    for (p, k), o in product(SHAPES, range(4)):
        seen = []
        for s in range(3):
            rows, W = o2.transfer_operator(direction, scheme, p, k, o, s)
            err = np.abs(W.sum(axis=1) - 1.0) / np.abs(W).sum(axis=1)
            assert err.max() < 1e-14
            seen.extend(rows.tolist())
        want = k * p * (3 if direction == 0 else 1)
        # interpolation: each subface writes the whole fine ghost half of its own buffer
        assert len(set(seen)) == (k * p if direction == 0 else want)
        if direction == 1:
            assert len(seen) == want
        # the written half: the coarse side (interpolation) or the fine side
        # (restriction); the fine patch lies on the + side for o < 2
        a, ext, idx = grid(o, p, k)
        minus = {j for j in range(len(idx)) if idx[j, a] < k}
        coarse_side = minus if o < 2 else set(range(len(idx))) - minus
        assert set(seen) <= (coarse_side if direction == 0 else set(range(len(idx))) - coarse_side)


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_coincident_centres_are_copies(scheme):
    p, k = 9, 3
    for o, s in product(range(4), range(3)):
        rows, W = o2.interpolation_operator(scheme, p, k, o, s)
        fpos, cpos = fine_centres(o, p, k, s)[rows], coarse_centres(o, p, k)
        hits = 0
        for r in range(len(rows)):
            hit = np.flatnonzero(np.all(cpos == fpos[r], axis=1))
            if len(hit):
                want = np.zeros(W.shape[1])
                want[hit[0]] = 1.0
                assert np.array_equal(W[r], want)
                hits += 1
        assert hits == p // 3  # one per coarse column, in the middle ghost layer
        if scheme > 1:
            rows, W = o2.restriction_operator(scheme, p, k, o, s)
            fpos, cpos = fine_centres(o, p, k, s), coarse_centres(o, p, k)[rows]
            for r in range(len(rows)):
                hit = np.flatnonzero(np.all(fpos == cpos[r], axis=1))
                if len(hit):
                    want = np.zeros(W.shape[1])
                    want[hit[0]] = 1.0
                    assert np.array_equal(W[r], want)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("k", [2, 3])
def test_whole_operator_exact_rational(direction, scheme, k):
    p = 6
    for o, s in ((0, 0), (3, 2), (1, 1)):
        rows, W = o2.transfer_operator(direction, scheme, p, k, o, s)
        a, ext, idx = grid(o, p, k)
        src = coarse_centres(o, p, k) if direction == 0 else fine_centres(o, p, k, s)
        dst = fine_centres(o, p, k, s) if direction == 0 else coarse_centres(o, p, k)
        unit = 3.0 if direction == 0 else 1.0
        for r, d in enumerate(rows):
            X = dst[d]
            if direction == 0:
                home = int(np.flatnonzero(np.abs(src - X).max(axis=1) < 1.5)[0])
            else:
                home = int(np.argmin(((src - X) ** 2).sum(axis=1)))
            stencil = oracle.taylor_stencil(tuple(idx[home]), ext, scheme)
            cols = [int(np.flatnonzero(np.all(idx == np.array(q), axis=1))[0]) for q in stencil]
            offs = [tuple(int(round((src[c][i] - src[home][i]) / unit)) for i in range(2)) for c in cols]
            tgt = tuple(Fraction(int(round(X[i] - src[home][i])), int(unit)) for i in range(2))
            exact = chk.exact_pinned_fit(offs, cols.index(home), tgt, scheme)
            want = np.zeros(W.shape[1])
            for c, v in zip(cols, exact):
                want[c] += float(v)
            assert np.abs(W[r] - want).max() < 1e-14 * np.abs(want).sum()


def interior_taylor2_weights_2d(t):
    """Hand-derived interior second-order fit on the 3 x 3 box (pinned centre,
    unweighted least squares over the 8 neighbours).  First derivatives:
    sum of q_i dQ / 6; mixed: sum of q_0 q_1 dQ / 4; pure second
    derivatives: [[3/2, 1], [1, 3/2]]^-1 = [[6/5, -4/5], [-4/5, 6/5]]
    applied to the sums of (q_i^2 / 2) dQ."""
    tx, ty = t
    w = {}
    for q in product((-1, 0, 1), repeat=2):
        if q == (0, 0):
            continue
        qx, qy = q
        ex, ey = Fraction(qx * qx, 2), Fraction(qy * qy, 2)
        axx = Fraction(6, 5) * ex - Fraction(4, 5) * ey
        ayy = -Fraction(4, 5) * ex + Fraction(6, 5) * ey
        w[q] = (qx * tx + qy * ty) / 6 + axx * tx * tx / 2 + ayy * ty * ty / 2 + Fraction(qx * qy, 4) * tx * ty
    w[(0, 0)] = 1 - sum(w.values())
    return w


def test_interior_taylor2_closed_form():
    p, k, o, s = 9, 3, 1, 1
    rows, W = o2.interpolation_operator(2, p, k, o, s)
    fpos, cpos = fine_centres(o, p, k, s)[rows], coarse_centres(o, p, k)
    a = o % 2
    b = 1 - a
    checked = 0
    for r in range(len(rows)):
        home = np.floor(fpos[r] / 3.0) * 3.0 + 1.5
        # interior along the face: tangential box inside; normal box at coarse layers -1..1 exists (k = 3)
        if not (3.0 < home[b] < 3.0 * (p - 1)):
            continue
        t = tuple(Fraction(int(round(2 * (fpos[r][i] - home[i]))), 6) for i in range(2))
        want = interior_taylor2_weights_2d(t)
        for q, wq in want.items():
            col = np.flatnonzero(np.all(cpos == home + 3.0 * np.array(q), axis=1))[0]
            assert W[r, col] == pytest.approx(float(wq), abs=1e-14)
        checked += 1
    assert checked == 27  # 3 coarse columns x 3 fine columns x 3 ghost layers


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_orientation_equivariance(direction, scheme):
    p, k = 6, 3
    for s in range(3):
        ref = None
        for o in range(4):
            rows, W = o2.transfer_operator(direction, scheme, p, k, o, s)
            a, ext, idx = grid(o, p, k)
            depth = idx[:, a] - k if o < 2 else k - 1 - idx[:, a]
            key = [(int(depth[i]), int(idx[i, 1 - a])) for i in range(len(idx))]
            M = W[np.ix_(sorted(range(len(rows)), key=lambda r: key[rows[r]]),
                         sorted(range(W.shape[1]), key=lambda j: key[j]))]
            if ref is None:
                ref = M
            else:
                assert (np.abs(M - ref) / np.abs(ref).sum(axis=1, keepdims=True)).max() < 1e-14


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme,order", [(1, 2), (2, 3), (3, 4)])
def test_convergence_order(direction, scheme, order):
    kappa = np.array([0.9, -0.8])
    p, k, o, s = 9, 3, 2, 1
    hs = [2.0**-e for e in range(4, 9)]
    errs = []
    for h in hs:
        cv = np.sin(h * coarse_centres(o, p, k) @ kappa + 0.4)
        fv = np.sin(h * fine_centres(o, p, k, s) @ kappa + 0.4)
        rows, W = o2.transfer_operator(direction, scheme, p, k, o, s)
        errs.append(np.abs(W @ cv - fv[rows]).max() if direction == 0 else np.abs(W @ fv - cv[rows]).max())
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert abs(slope - order) < 0.3, (slope, errs)


@pytest.mark.parametrize("direction", [0, 1])
def test_dlinear_is_the_z_independent_3d_case(direction):
    """The tensor-product scheme of a field that does not depend on the third
    axis: every 3D row summed over that axis equals the 2D row."""
    p, k = 6, 3
    for o2d, s2d in product(range(4), range(3)):
        a2 = o2d % 2
        o3 = a2 + (0 if o2d < 2 else 3)  # same normal axis and side; third axis 2 is tangential
        s3 = s2d + 3 * 1  # middle subface along axis 2
        rows3, W3 = oracle.transfer_operator(direction, 1, p, k, o3, s3)
        rows2, W2 = o2.transfer_operator(direction, 1, p, k, o2d, s2d)
        ext3 = oracle.face_extents(o3, p, k)
        cells3 = oracle.storage_cells(ext3)
        _, ext2, idx2 = grid(o2d, p, k)
        col2 = {(int(i0), int(i1)): j for j, (i0, i1) in enumerate(idx2)}
        W3_2 = np.zeros((len(rows3), W2.shape[1]))
        for j, c in enumerate(cells3):
            W3_2[:, col2[(c[0], c[1])]] += W3[:, j]
        for r, dst in enumerate(rows3):
            c = cells3[dst]
            r2 = list(rows2).index(col2[(c[0], c[1])])
            assert np.abs(W3_2[r] - W2[r2]).max() < 1e-15


# Planted mistakes (on the CPU): each must make one of the pins above fail.


def _fails(fn, *args):
    o2.clear_operator_cache()
    try:
        fn(*args)
    except AssertionError:
        return True
    finally:
        o2.clear_operator_cache()
    return False


def test_shifted_subface_is_caught(monkeypatch):
    real = o2.fine_position
    monkeypatch.setattr(o2, "fine_position", lambda o, p, k, s, idx: real(o, p, k, s, idx) + np.array([0.0, 1.0]) * (s == 1))
    assert _fails(test_polynomial_reproduction, 2, 6, 2, 0)


def test_unpinned_fit_is_caught(monkeypatch):
    def free(offsets, centre_pos, target, degree):
        ex = [e for e in product(range(degree + 1), repeat=2) if sum(e) <= degree]
        A = np.array([[np.prod([o_ ** e_ for o_, e_ in zip(off, e)]) for e in ex] for off in offsets])
        t = np.array([np.prod([tt ** e_ for tt, e_ in zip(target, e)]) for e in ex])
        return t @ np.linalg.pinv(A)

    monkeypatch.setattr(o2, "pinned_fit_weights", free)
    assert _fails(test_coincident_centres_are_copies, 2)


def test_swapped_normal_side_is_caught(monkeypatch):
    monkeypatch.setattr(o2, "fine_on_plus_side", lambda o: int(o) >= 2)
    assert _fails(test_rows_sum_to_one_and_segments_tile, 0, 1)
    assert _fails(test_rows_sum_to_one_and_segments_tile, 1, 2)


@pytest.mark.parametrize("scheme", [1, 2, 3])
@pytest.mark.parametrize("direction", [0, 1])
def test_general_p_2d(scheme, direction):
    """p not a multiple of 3: reproduction, row sums, and restriction columns
    that tile the coarse halo (the same reading as in 3D)."""
    rng = np.random.default_rng(40 + scheme + direction)
    for p, k in ((7, 2), (8, 3), (10, 2)):
        worst = max(reproduction_error(scheme, p, k, o, s, rng, direction) for o in range(4) for s in range(3))
        assert worst < 1e-12
        for o in range(4):
            seen = []
            for s in range(3):
                rows, W = o2.transfer_operator(direction, scheme, p, k, o, s)
                assert np.allclose(W.sum(axis=1), 1.0, atol=1e-13)
                seen.extend(rows.tolist())
            if direction == 1:
                assert len(seen) == len(set(seen)) == k * p
