"""Plant plausible mistakes in the oracle (on the CPU) and check that at least
one of the pins fails for each: the pins are strong enough to notice a
dropped term, a wrong sign or index, an unpinned or weighted fit, a stencil
that is not shifted at the face edges, and a wrong extrapolation rule."""

from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import oracle
import oracle.fit as ofit
import oracle.geometry as ogeo
import oracle.transfer as otr
from tests import oracle_checks as chk


def _clear():
    otr.clear_operator_cache()
    ofit._derivative_operator.cache_clear()


@pytest.fixture(autouse=True)
def fresh_caches():
    _clear()
    yield
    _clear()


def _reproduction_fails(p=6, k=3, schemes=(1, 2, 3)):
    rng = np.random.default_rng(3)
    for scheme, direction, o, s in product(schemes, (0, 1), range(6), (0, 1, 4, 5, 8)):
        try:
            err = chk.reproduction_error(oracle, scheme, p, k, o, s, rng, direction)
        except Exception:
            return True
        if not err < 1e-12:
            return True
    return False


def _injection_fails(p=6, k=3):
    for scheme, o, s in product((2, 3), range(6), (0, 4)):
        try:
            rows, W = oracle.interpolation_operator(scheme, p, k, o, s)
        except Exception:
            return True
        fpos = chk.fine_centres(o, p, k, s)[rows]
        cpos = chk.coarse_centres(o, p, k)
        for r in range(len(rows)):
            hit = np.flatnonzero(np.all(cpos == fpos[r], axis=1))
            if len(hit):
                want = np.zeros(W.shape[1])
                want[hit[0]] = 1.0
                if not np.array_equal(W[r], want):
                    return True
    return False


def _exact_fit_fails():
    rng = np.random.default_rng(11)
    for ext, centre, degree, _ in chk.load_stencil_fixture():
        stencil = ofit.taylor_stencil(centre, ext, degree)
        offsets = [tuple(q[i] - centre[i] for i in range(3)) for q in stencil]
        target = tuple(Fraction(int(v), 3) for v in rng.integers(-6, 7, size=3))
        try:
            exact = chk.exact_pinned_fit(offsets, stencil.index(centre), target, degree)
            got = ofit.pinned_fit_weights(offsets, stencil.index(centre), [float(t) for t in target], degree)
        except Exception:
            return True
        scale = sum(abs(float(v)) for v in exact)
        if np.abs(got - np.array([float(v) for v in exact])).max() > 1e-14 * scale:
            return True
    return False


def _stencil_fixture_fails():
    for ext, centre, degree, want in chk.load_stencil_fixture():
        try:
            if set(ofit.taylor_stencil(centre, ext, degree)) != want:
                return True
        except Exception:
            return True
    return False


def _dlinear_restriction_fixture_fails():
    import os

    cases = []
    with open(os.path.join(chk.GOLDEN, "dlinear_restriction.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, l, *pairs = line.split()
                cases.append((int(k), int(l), {int(a): float(Fraction(b)) for a, b in (x.split(":") for x in pairs)}))
    p, o, s = 6, 0, 0
    for k, l, want in cases:
        rows, W = oracle.restriction_operator(1, p, k, o, s)
        a, ext, idx = chk.buffer_grid(o, p, k)
        # target: coarse layer l (buffer index k + l for o = 0), first column
        r = [i for i, cell in enumerate(rows) if tuple(idx[cell]) == (k + l, 0, 0)][0]
        for eta, w in want.items():
            cols = [j for j in range(len(idx)) if idx[j, 0] == k + eta and idx[j, 1] < 3 and idx[j, 2] < 3]
            if not np.allclose(W[r, cols], w / 9.0, atol=1e-15, rtol=0):
                return True
    return False


def test_unmutated_oracle_passes_the_quick_pins():
    assert not _reproduction_fails()
    assert not _injection_fails()
    assert not _exact_fit_fails()
    assert not _stencil_fixture_fails()
    assert not _dlinear_restriction_fixture_fails()


def test_dropped_mixed_term_is_caught(monkeypatch):
    real = ofit.taylor_exponents
    monkeypatch.setattr(ofit, "taylor_exponents", lambda d: [e for e in real(d) if e != (1, 1, 0)])
    assert _reproduction_fails(schemes=(2, 3))


def test_target_sign_flip_is_caught(monkeypatch):
    real = otr.pinned_fit_weights
    monkeypatch.setattr(otr, "pinned_fit_weights", lambda off, c, t, d: real(off, c, -np.asarray(t), d))
    assert _reproduction_fails(schemes=(2, 3))


def test_unpinned_constant_is_caught(monkeypatch):
    def free_constant_fit(offsets, centre_pos, target, degree):
        exps = [(0, 0, 0)] + ofit.taylor_exponents(degree)
        A = np.array([[ofit.taylor_term(q, e) for e in exps] for q in offsets])
        t = np.array([ofit.taylor_term(target, e) for e in exps])
        return t @ np.linalg.pinv(A)

    monkeypatch.setattr(otr, "pinned_fit_weights", free_constant_fit)
    monkeypatch.setattr(ofit, "pinned_fit_weights", free_constant_fit)
    assert _injection_fails() or _exact_fit_fails()


def test_distance_weighted_fit_is_caught(monkeypatch):
    def weighted(offsets, centre_pos, target, degree):
        offsets = np.asarray(offsets, dtype=float)
        exps = ofit.taylor_exponents(degree)
        others = [q for q in range(len(offsets)) if q != centre_pos]
        wts = np.array([1.0 / (1.0 + np.abs(offsets[q]).sum()) for q in others])
        A = np.array([[ofit.taylor_term(offsets[q], e) for e in exps] for q in others]) * wts[:, None]
        t = np.array([ofit.taylor_term(target, e) for e in exps])
        w_o = (t @ np.linalg.pinv(A)) * wts
        w = np.zeros(len(offsets))
        w[others] = w_o
        w[centre_pos] = 1 - w_o.sum()
        return w

    monkeypatch.setattr(ofit, "pinned_fit_weights", weighted)
    assert _exact_fit_fails()


def test_unshifted_edge_stencil_is_caught(monkeypatch):
    real = ofit.taylor_stencil

    def unshifted(centre, ext, degree):
        pts = [tuple(c + d for c, d in zip(centre, dd)) for dd in product((-1, 0, 1), repeat=3)]
        if degree >= 3:
            pts += [tuple(c + (st if ax == i else 0) for i, c in enumerate(centre))
                    for ax in range(3) for st in (-2, 2)]
        return pts

    monkeypatch.setattr(ofit, "taylor_stencil", unshifted)
    monkeypatch.setattr(otr, "taylor_stencil", unshifted)
    assert _stencil_fixture_fails() and _reproduction_fails(schemes=(2, 3))


def test_missing_third_order_axial_points_is_caught(monkeypatch):
    real = ofit.taylor_stencil
    monkeypatch.setattr(otr, "taylor_stencil", lambda c, e, d: real(c, e, 2))
    monkeypatch.setattr(ofit, "taylor_stencil", lambda c, e, d: real(c, e, 2))
    assert _reproduction_fails(schemes=(3,)) or _stencil_fixture_fails()


def test_swapped_subface_digits_are_caught(monkeypatch):
    real = ogeo.fine_position
    monkeypatch.setattr(ogeo, "fine_position", lambda o, p, k, s, idx: real(o, p, k, 3 * (s % 3) + s // 3, idx))
    assert _reproduction_fails()


def test_half_cell_shift_is_caught(monkeypatch):
    real = ogeo.coarse_position
    monkeypatch.setattr(ogeo, "coarse_position", lambda o, p, k, idx: real(o, p, k, idx) + np.array([0.0, 0.5, 0.0]))
    assert _reproduction_fails()


def test_constant_extrapolation_is_caught(monkeypatch):
    real = ofit.linear_weights_1d
    monkeypatch.setattr(otr, "linear_weights_1d", lambda x, n: real(min(max(Fraction(x), 0), n - 1), n))
    assert _reproduction_fails(schemes=(1,))


def test_wrong_averaging_extrapolation_pair_is_caught(monkeypatch):
    """Extrapolating from the two layers nearest the face is exact on linear
    data too; only the hand-written fixture notices it."""
    real = otr._dlinear_restriction_row

    def nearest_pair(o, p, k, s, XT, fine_pos, ext):
        row = real(o, p, k, s, XT, fine_pos, ext)
        a = o % 3
        side = 1.0 if o < 3 else -1.0
        depth = side * XT[a]
        if depth < 3.0 or k != 3:
            return row
        # redo the normal part through layers 0 and 1
        inner = sorted([i for i in range(ext[a]) if side * fine_pos[a][i] > 0], key=lambda i: side * fine_pos[a][i])
        i1, i2 = inner[0], inner[1]
        t = depth - side * fine_pos[a][i1]
        out = np.zeros_like(row)
        b, c = [ax for ax in range(3) if ax != a]
        for ia, wa in ((i1, 1 - t), (i2, t)):
            for ib in range(ext[b]):
                for ic in range(ext[c]):
                    if abs(fine_pos[b][ib] - XT[b]) < 1.5 and abs(fine_pos[c][ic] - XT[c]) < 1.5:
                        idx = [0, 0, 0]
                        idx[a], idx[b], idx[c] = ia, ib, ic
                        out[ogeo.cell_index(ext, idx)] += wa / 9.0
        return out

    monkeypatch.setattr(otr, "_dlinear_restriction_row", nearest_pair)
    assert not _reproduction_fails(schemes=(1,))
    assert _dlinear_restriction_fixture_fails()
