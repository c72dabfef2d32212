"""Pins of the FP64 oracle against what the paper and the mathematics fix.

* polynomial reproduction: d-linear is exact on trilinear fields, the second-
  and third-order Taylor schemes on all quadratics / cubics (Section 3: the
  fits are Taylor polynomials of that degree; Section 5.1: convergence orders)
* constants: every row sums to one
* coincident centres are copies, bit for bit (Section 3: coinciding fine and
  coarse centres; restriction with k > 1 reduces to injection)
* exact rational brute force of the least-squares fits on small faces
* closed forms: the interior second-order fit and the 1D linear weights
* stencil shapes (Appendix C reading) and convergence slopes 2 / 3 / 4
* orientation equivariance (Section 4.1: the six configurations are rotations
  and mirrors of one reference face)
"""

from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import oracle
from oracle import geometry as ogeo
from tests import oracle_checks as chk

SHAPES = [(6, 2), (6, 3), (9, 2), (9, 3)]


@pytest.mark.parametrize("scheme", [1, 2, 3])
@pytest.mark.parametrize("p,k", SHAPES)
@pytest.mark.parametrize("direction", [0, 1])
def test_polynomial_reproduction(scheme, p, k, direction):
    rng = np.random.default_rng(1000 * scheme + 10 * p + k + direction)
    worst = 0.0
    for o in range(6):
        for s in range(9):
            worst = max(worst, chk.reproduction_error(oracle, scheme, p, k, o, s, rng, direction))
    assert worst < 1e-12, worst


def test_reproduction_is_sharp():
    """The Taylor-2 operator is not exact on a cubic and Taylor-3 is not exact
    on a quartic (the orders are exactly the stated ones)."""
    p, k, o, s = 9, 3, 0, 4
    pos_c, pos_f = chk.coarse_centres(o, p, k), chk.fine_centres(o, p, k, s)
    for scheme, e in ((2, (3, 0, 0)), (3, (2, 2, 0))):
        cv = chk.poly_eval(pos_c, [1.0], [e], 27.0)
        fv = chk.poly_eval(pos_f, [1.0], [e], 27.0)
        rows, W = oracle.interpolation_operator(scheme, p, k, o, s)
        assert np.abs(W @ cv - fv[rows]).max() > 1e-6


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_rows_sum_to_one(direction, scheme):
    for (p, k), o, s in product(SHAPES, range(6), (0, 4, 8)):
        rows, W = oracle.transfer_operator(direction, scheme, p, k, o, s)
        err = np.abs(W.sum(axis=1) - 1.0) / np.abs(W).sum(axis=1)
        assert err.max() < 1e-14


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_coincident_interpolation_rows_are_copies(scheme):
    """Fine ghost centres that sit on a coarse centre (middle layer, middle
    column of each 3x3 group) copy that coarse value exactly."""
    for (p, k), o, s in product(SHAPES, range(6), range(9)):
        rows, W = oracle.interpolation_operator(scheme, p, k, o, s)
        fpos = chk.fine_centres(o, p, k, s)[rows]
        cpos = chk.coarse_centres(o, p, k)
        n_copy = 0
        for r in range(len(rows)):
            hit = np.flatnonzero(np.all(cpos == fpos[r], axis=1))
            if len(hit):
                n_copy += 1
                want = np.zeros(W.shape[1])
                want[hit[0]] = 1.0
                assert np.array_equal(W[r], want)
        assert n_copy == (p // 3) ** 2  # one per coarse column, layer g = 1


@pytest.mark.parametrize("scheme", [2, 3])
def test_restriction_layer0_is_injection(scheme):
    """Section 3: for k > 1 the fine cell nearest to the first coarse layer's
    centre coincides with it, so the restriction is an injection."""
    for (p, k), o, s in product(SHAPES, range(6), range(9)):
        rows, W = oracle.restriction_operator(scheme, p, k, o, s)
        cpos = chk.coarse_centres(o, p, k)[rows]
        fpos = chk.fine_centres(o, p, k, s)
        depth = np.abs(cpos[:, o % 3])
        layer0 = np.flatnonzero(depth == 1.5)
        assert len(layer0) == (p // 3) ** 2
        for r in layer0:
            hit = np.flatnonzero(np.all(fpos == cpos[r], axis=1))
            want = np.zeros(W.shape[1])
            want[hit[0]] = 1.0
            assert np.array_equal(W[r], want)


def test_restriction_segments_tile_the_fine_side_half():
    """The nine subfaces restrict into disjoint segments that together cover
    the coarse face's fine-side half exactly (so one launch has no races)."""
    for (p, k), o in product(SHAPES, range(6)):
        seen = []
        for s in range(9):
            rows, _ = oracle.restriction_operator(2, p, k, o, s)
            seen.extend(rows.tolist())
        assert len(seen) == len(set(seen)) == k * p * p
        cells = ogeo.storage_cells(ogeo.face_extents(o, p, k))
        half = {ogeo.cell_index(ogeo.face_extents(o, p, k), c) for c in cells
                if ogeo.coarse_fine_side_half(o, k, c)}
        assert set(seen) == half


def test_stencil_shapes_fixture():
    for ext, centre, degree, want in chk.load_stencil_fixture():
        got = oracle.taylor_stencil(centre, ext, degree)
        assert len(got) == len(set(got))
        assert set(got) == want, (ext, centre, degree)


def test_dlinear_1d_fixture():
    for x, n, want in chk.load_dlinear_fixture():
        got = oracle.linear_weights_1d(x, n)
        assert set(got) == set(want)
        for i, w in want.items():
            assert got[i] == pytest.approx(float(w), abs=1e-15)


def test_dlinear_interpolation_is_tensor_product_of_fixture_weights():
    """A d-linear interpolation row equals the product of the three 1D weight
    sets (Section 2, P = Px Py Pz); the largest row 1-norm is 25/9."""
    p, k = 9, 3
    big = 0.0
    for o, s in product(range(6), range(9)):
        rows, W = oracle.interpolation_operator(1, p, k, o, s)
        big = max(big, np.abs(W).sum(axis=1).max())
        assert np.all(np.count_nonzero(W, axis=1) <= 8)
    assert big == pytest.approx(25.0 / 9.0, abs=1e-14)


def test_interior_taylor2_closed_form():
    p, k, o, s = 9, 3, 0, 4  # interior subface of an x-normal face
    rows, W = oracle.interpolation_operator(2, p, k, o, s)
    fpos = chk.fine_centres(o, p, k, s)[rows]
    cpos = chk.coarse_centres(o, p, k)
    checked = 0
    for r in range(len(rows)):
        home = np.floor(fpos[r] / 3.0) * 3.0 + 1.5
        # interior expansion cells only: the whole box lies inside the face
        if not (3.0 * 1 < home[1] < 3.0 * (p - 1) and 3.0 * 1 < home[2] < 3.0 * (p - 1)):
            continue
        target = tuple(Fraction(float(v)).limit_denominator(6) / 3 for v in fpos[r] - home)
        want = chk.interior_taylor2_weights(target)
        for q, wq in want.items():
            qpos = home + 3.0 * np.array(q)
            col = np.flatnonzero(np.all(cpos == qpos, axis=1))[0]
            assert W[r, col] == pytest.approx(float(wq), abs=1e-14)
        assert abs(np.abs(W[r]).sum() - sum(abs(float(v)) for v in want.values())) < 1e-13
        checked += 1
    assert checked == 243  # the middle subface has only interior expansion cells


@pytest.mark.parametrize("scheme", [2, 3])
def test_fit_matches_exact_rational_least_squares(scheme):
    """The QR-based pinned fit equals the exact normal-equation solution."""
    rng = np.random.default_rng(scheme)
    for ext, centre, degree, pts in chk.load_stencil_fixture():
        if degree != scheme:
            continue
        stencil = oracle.taylor_stencil(centre, ext, degree)
        offsets = [tuple(q[i] - centre[i] for i in range(3)) for q in stencil]
        for _ in range(3):
            target = tuple(Fraction(int(v), 3) for v in rng.integers(-6, 7, size=3))
            exact = chk.exact_pinned_fit(offsets, stencil.index(centre), target, degree)
            got = oracle.pinned_fit_weights(offsets, stencil.index(centre), [float(t) for t in target], degree)
            scale = sum(abs(float(v)) for v in exact)
            assert np.abs(got - np.array([float(v) for v in exact])).max() < 1e-14 * scale


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("k", [2, 3])
def test_whole_operator_exact_rational(direction, scheme, k):
    """Brute force on a small face: every Taylor row from exact arithmetic,
    with the expansion cell chosen by distance (Section 3)."""
    p = 6
    for o, s in ((0, 0), (4, 8), (2, 5)):
        rows, W = oracle.transfer_operator(direction, scheme, p, k, o, s)
        a, ext, idx = chk.buffer_grid(o, p, k)
        src_pos = chk.coarse_centres(o, p, k) if direction == 0 else chk.fine_centres(o, p, k, s)
        dst_pos = chk.fine_centres(o, p, k, s) if direction == 0 else chk.coarse_centres(o, p, k)
        unit = 3.0 if direction == 0 else 1.0
        for r, dst in enumerate(rows):
            X = dst_pos[dst]
            if direction == 0:
                d = np.abs(src_pos - X).max(axis=1)
                home = int(np.flatnonzero(d < 1.5)[0])  # containing coarse cell
            else:
                d2 = ((src_pos - X) ** 2).sum(axis=1)
                home = int(np.argmin(d2))
            stencil = oracle.taylor_stencil(tuple(idx[home]), ext, scheme)
            cols = [int(np.flatnonzero(np.all(idx == np.array(q), axis=1))[0]) for q in stencil]
            offs = [tuple(int(round((src_pos[c][i] - src_pos[home][i]) / unit)) for i in range(3)) for c in cols]
            tgt = tuple(Fraction(int(round(X[i] - src_pos[home][i])), int(unit)) for i in range(3))
            exact = chk.exact_pinned_fit(offs, cols.index(home), tgt, scheme)
            want = np.zeros(W.shape[1])
            for c, v in zip(cols, exact):
                want[c] += float(v)
            scale = np.abs(want).sum()
            assert np.abs(W[r] - want).max() < 1e-14 * scale


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_orientation_equivariance(direction, scheme):
    """All six orientations give the same operator once rows and columns are
    written in reference coordinates (depth into the fine side, b, c)."""
    p, k = 6, 3
    for s in (0, 4, 7):
        ref = None
        for o in range(6):
            rows, W = oracle.transfer_operator(direction, scheme, p, k, o, s)
            a, ext, idx = chk.buffer_grid(o, p, k)
            depth = chk.depth_into_fine_side(o, p, k)
            b, c = [ax for ax in range(3) if ax != a]
            key = [(int(depth[i]), int(idx[i, b]), int(idx[i, c])) for i in range(len(idx))]
            order_r = sorted(range(len(rows)), key=lambda r: key[rows[r]])
            order_c = sorted(range(W.shape[1]), key=lambda j: key[j])
            M = W[np.ix_(order_r, order_c)]
            if ref is None:
                ref = M
            else:
                scale = np.abs(ref).sum(axis=1, keepdims=True)
                assert (np.abs(M - ref) / scale).max() < 1e-14


def _convergence_slope(scheme, direction):
    rng = np.random.default_rng(7)
    kappa = rng.normal(size=3)
    kappa *= 1.3 / np.linalg.norm(kappa)
    phase = 0.4
    p, k, o, s = 9, 3, 1, 3
    hs = [2.0**-e for e in range(4, 9)]
    errs = []
    for h in hs:
        cv = np.sin(h * chk.coarse_centres(o, p, k) @ kappa + phase)
        fv = np.sin(h * chk.fine_centres(o, p, k, s) @ kappa + phase)
        if direction == 0:
            rows, W = oracle.interpolation_operator(scheme, p, k, o, s)
            errs.append(np.abs(W @ cv - fv[rows]).max())
        else:
            rows, W = oracle.restriction_operator(scheme, p, k, o, s)
            errs.append(np.abs(W @ fv - cv[rows]).max())
    return np.polyfit(np.log(hs), np.log(errs), 1)[0], errs


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme,order", [(1, 2), (2, 3), (3, 4)])
def test_convergence_order(direction, scheme, order):
    """Section 5.1: d-linear converges as h^2, the Taylor schemes one order
    above their degree; no floor near 1e-8 appears with cell-unit fits."""
    slope, errs = _convergence_slope(scheme, direction)
    assert abs(slope - order) < 0.25, (slope, errs)
    assert errs[-1] < errs[0]


# k = 1 (finite volumes, Section 2): the d-linear scheme only.


@pytest.mark.parametrize("p", [6, 9])
@pytest.mark.parametrize("direction", [0, 1])
def test_dlinear_k1_reproduces_trilinear_fields(p, direction):
    rng = np.random.default_rng(77 + p + direction)
    worst = 0.0
    for o in range(6):
        for s in range(9):
            worst = max(worst, chk.reproduction_error(oracle, 1, p, 1, o, s, rng, direction))
    assert worst < 1e-12, worst


def test_dlinear_k1_rows_and_normal_weights():
    """Interpolation: the one fine ghost layer lies 1/6 coarse width into the
    coarse side, between coarse layer 0 (1/2 width in) and the coarse face's
    fine-side layer (1/2 width out): weights 2/3 and 1/3.  Restriction:
    the coarse centre 3/2 fine widths in, extrapolated through fine layer 0
    and the halo layer: 2 and -1 (fixture)."""
    p, k, o = 6, 1, 0
    for s in range(9):
        for direction in (0, 1):
            rows, W = oracle.transfer_operator(direction, 1, p, k, o, s)
            assert np.allclose(W.sum(axis=1), 1.0, atol=1e-15)
    rows, W = oracle.interpolation_operator(1, p, k, o, 4)
    a, ext, idx = chk.buffer_grid(o, p, k)
    for r in range(len(rows)):
        # o = 0: coarse side is buffer layer 0 (coarse layer 0), layer 1 is the fine-side half
        w_by_layer = {lay: W[r, idx[:, 0] == lay].sum() for lay in (0, 1)}
        assert w_by_layer[0] == pytest.approx(2.0 / 3.0, abs=1e-15)
        assert w_by_layer[1] == pytest.approx(1.0 / 3.0, abs=1e-15)
    for scheme in (2, 3):
        with pytest.raises(ValueError):
            oracle.transfer_operator(0, scheme, p, k, o, 0)


def test_restriction_segments_tile_k1():
    for p, o in product((6, 9), range(6)):
        seen = []
        for s in range(9):
            rows, _ = oracle.restriction_operator(1, p, 1, o, s)
            seen.extend(rows.tolist())
        assert len(seen) == len(set(seen)) == p * p


# Patch sizes that are not multiples of 3 (Section 5.3 times them; fine and
# coarse cells do not align at the subface boundaries).

GENERAL_P = [(7, 2), (8, 3), (10, 2), (10, 3)]


@pytest.mark.parametrize("scheme", [1, 2, 3])
@pytest.mark.parametrize("p,k", GENERAL_P)
@pytest.mark.parametrize("direction", [0, 1])
def test_general_p_reproduction(scheme, p, k, direction):
    rng = np.random.default_rng(3000 + 100 * scheme + 10 * p + k + direction)
    worst = 0.0
    for o in range(6):
        for s in (0, 1, 2, 4, 5, 8):
            worst = max(worst, chk.reproduction_error(oracle, scheme, p, k, o, s, rng, direction))
    assert worst < 1e-12, worst


@pytest.mark.parametrize("p", [7, 8, 10])
def test_general_p_rows_copies_and_tiling(p):
    for k in (1, 2, 3):
        schemes = (1,) if k == 1 else (1, 2, 3)
        for scheme, o in product(schemes, (0, 4)):
            seen = []
            for s in range(9):
                rows, W = oracle.restriction_operator(scheme, p, k, o, s)
                assert np.allclose(W.sum(axis=1), 1.0, atol=1e-13)
                seen.extend(rows.tolist())
                irows, IW = oracle.interpolation_operator(scheme, p, k, o, s)
                assert len(irows) == k * p * p and np.allclose(IW.sum(axis=1), 1.0, atol=1e-13)
                # coinciding centres are copies, bit for bit
                fpos = chk.fine_centres(o, p, k, s)[irows]
                cpos = chk.coarse_centres(o, p, k)
                for r in range(len(irows)):
                    hit = np.flatnonzero(np.all(cpos == fpos[r], axis=1))
                    if len(hit):
                        want = np.zeros(IW.shape[1])
                        want[hit[0]] = 1.0
                        assert np.array_equal(IW[r], want)
            # the nine fine faces restrict into disjoint columns covering the half
            assert len(seen) == len(set(seen)) == k * p * p


def test_general_p_restriction_columns_fixture():
    cases = []
    with open(chk.os.path.join(chk.GOLDEN, "general_p_columns.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                p, sb, m, *pairs = line.split()
                w = {int(a): float(Fraction(b)) for a, b in (x.split(":") for x in pairs)}
                cases.append((int(p), int(sb), int(m), w))
    assert len(cases) == 15
    k, o = 2, 0  # x-normal face: b = axis 1, c = axis 2; fine on the + side
    for p, sb, m, want in cases:
        mc = {7: 3, 8: 3}[p]  # a coarse column of the middle row sc = 1 with three fine columns
        rows, W = oracle.restriction_operator(1, p, k, o, sb + 3)
        a, ext, idx = chk.buffer_grid(o, p, k)
        r = [i for i, cell in enumerate(rows) if tuple(idx[cell]) == (k, m, mc)]
        assert len(r) == 1, (p, sb, m)
        wb = np.zeros(p)
        np.add.at(wb, idx[:, 1], W[r[0]])
        got = {j: wb[j] for j in range(p) if wb[j] != 0.0}
        assert set(got) == set(want), (p, sb, m, got)
        for j, v in want.items():
            assert got[j] == pytest.approx(v, abs=1e-15)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("scheme", [2, 3])
def test_general_p_exact_rational(direction, scheme):
    """Brute force on p = 7 faces: every Taylor row from exact arithmetic."""
    p, k = 7, 2
    for o, s in ((0, 1), (5, 7)):
        rows, W = oracle.transfer_operator(direction, scheme, p, k, o, s)
        a, ext, idx = chk.buffer_grid(o, p, k)
        src_pos = chk.coarse_centres(o, p, k) if direction == 0 else chk.fine_centres(o, p, k, s)
        dst_pos = chk.fine_centres(o, p, k, s) if direction == 0 else chk.coarse_centres(o, p, k)
        unit = 3.0 if direction == 0 else 1.0
        for r, dst in enumerate(rows):
            X = dst_pos[dst]
            if direction == 0:
                home = int(np.flatnonzero(np.abs(src_pos - X).max(axis=1) < 1.5)[0])
            else:
                home = int(np.argmin(((src_pos - X) ** 2).sum(axis=1)))
            stencil = oracle.taylor_stencil(tuple(idx[home]), ext, scheme)
            cols = [int(np.flatnonzero(np.all(idx == np.array(q), axis=1))[0]) for q in stencil]
            offs = [tuple(int(round((src_pos[c][i] - src_pos[home][i]) / unit)) for i in range(3)) for c in cols]
            tgt = tuple(Fraction(int(round(X[i] - src_pos[home][i])), int(unit)) for i in range(3))
            exact = chk.exact_pinned_fit(offs, cols.index(home), tgt, scheme)
            want = np.zeros(W.shape[1])
            for c, v in zip(cols, exact):
                want[c] += float(v)
            assert np.abs(W[r] - want).max() < 1e-14 * np.abs(want).sum()
