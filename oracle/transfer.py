"""Dense per-subface transfer operators and their application (oracle; test
infrastructure).

Section 2 writes the transfer as Q^f = P Q^c and Q^c = R Q^f, one sparse matrix
per face arrangement, of which one call applies the 1/9 segment belonging to
one fine face; every unknown is transferred independently by the same matrix.
Section 4.1 reduces the six arrangements to one reference face by rotation and
mirroring.  This oracle does NOT use that reduction: it builds each segment
directly from the physical cell-centre positions of the given orientation, so
that agreement with a reference-frame implementation also checks its index
maps.

Interpolation (Section 3): every fine ghost cell takes the coarse cell that
contains it as expansion cell, and the Taylor polynomial fitted there is
evaluated at the fine centre.
Restriction (Section 3): every coarse target takes the fine cell nearest to
its centre as expansion cell; the fit lives on the fine grid; a coincident
centre gives an injection, the others are extrapolations.
d-linear baseline (Section 2, tensor product P = Px Py Pz): 1D linear weights
per axis, multiplied; its restriction averages the covering fine cells.

Patch sizes that are not multiples of 3 (Section 5.3 times them): fine and
coarse cells do not align at the subface boundaries.  Every fine centre
still lies inside one coarse cell, at offset -1/3, 0 or 1/3 of a coarse width
from its centre, and every coarse centre lies on exactly one fine face, on a
fine centre; a fine face restricts into the coarse columns whose centres it
holds.  Where such a column straddles two fine faces, the averaging
restriction takes the fine column through its centre instead of the mean of
three.

Operators are dense float64 matrices W (rows = destination cells, columns = all
2k p^2 cells of the source face buffer) with the destination cell numbers.
"""

from fractions import Fraction
from functools import lru_cache

import numpy as np

from . import geometry as geo
from .fit import linear_weights_1d, pinned_fit_weights, taylor_stencil

DLINEAR, TAYLOR2, TAYLOR3 = 1, 2, 3
INTERPOLATE, RESTRICT = 0, 1


def _check(scheme, p, k, o, s):
    if scheme not in (DLINEAR, TAYLOR2, TAYLOR3):
        raise ValueError(f"unknown scheme {scheme}")
    if p < 6:
        raise ValueError(f"p must be >= 6, got {p}")
    if k not in (1, 2, 3):
        raise ValueError(f"k must be 1, 2 or 3, got {k}")
    if k == 1 and scheme != DLINEAR:
        # a 3-point Taylor stencil along the normal needs 2k >= 3 layers
        raise ValueError("k = 1 (finite volumes) is supported by the d-linear scheme only")
    if not (0 <= o < 6 and 0 <= s < 9):
        raise ValueError("orientation in 0..5 and subface in 0..8 required")


def _half_index(pos_fine_units, normal, k):
    """Fraction coordinate of a position (fine units) in coarse centre-index
    units of a coarse face buffer: coarse cell i is centred at coordinate i."""
    x = Fraction(float(pos_fine_units))  # half-integers: exact
    if normal:
        return (x - Fraction(3, 2)) / 3 + k
    return (x - Fraction(3, 2)) / 3


@lru_cache(maxsize=None)
def interpolation_operator(scheme, p, k, o, s):
    """(rows, W): fine ghost-half cells of subface s, and their weights over
    every cell of the coarse face buffer."""
    _check(scheme, p, k, o, s)
    a, _, _ = geo.face_axes(o)
    ext = geo.face_extents(o, p, k)
    cells = geo.storage_cells(ext)
    ncell = len(cells)
    coarse_pos = {c: geo.coarse_position(o, p, k, c) for c in cells}
    rows, W = [], []
    for fc in cells:
        if not geo.fine_ghost_half(o, k, fc):
            continue
        X = geo.fine_position(o, p, k, s, fc)
        # The coarse cell containing the fine centre (three-partitioning).
        home = tuple(
            int(np.floor(X[ax] / 3.0)) + (k if ax == a else 0) for ax in range(3)
        )
        if geo.coarse_fine_side_half(o, k, home):
            raise AssertionError("fine ghost centre must lie inside the coarse patch")
        row = np.zeros(ncell)
        if scheme == DLINEAR:
            per_axis = [
                linear_weights_1d(_half_index(X[ax], ax == a, k), ext[ax]) for ax in range(3)
            ]
            for i0, w0 in per_axis[0].items():
                for i1, w1 in per_axis[1].items():
                    for i2, w2 in per_axis[2].items():
                        row[geo.cell_index(ext, (i0, i1, i2))] += w0 * w1 * w2
        else:
            stencil = taylor_stencil(home, ext, scheme)
            # Offsets in coarse cell widths (the grid the stencil lives on).
            offsets = [(coarse_pos[q] - coarse_pos[home]) / 3.0 for q in stencil]
            target = (X - coarse_pos[home]) / 3.0
            w = pinned_fit_weights(offsets, stencil.index(home), target, scheme)
            for q, wq in zip(stencil, w):
                row[geo.cell_index(ext, q)] += wq
        rows.append(geo.cell_index(ext, fc))
        W.append(row)
    return np.array(rows, dtype=np.int64), np.array(W)


def _dlinear_restriction_row(o, p, k, s, target_pos, fine_pos, ext):
    """Averaging restriction (the tensor-product baseline's counterpart):
    mean over the fine columns under the target per tangential axis; along
    the normal the mean of the fine inner layers inside the target when all
    three exist, else linear extrapolation through the two fine layers
    deepest into the fine side (the last two inner layers; with k = 1 the
    single inner layer and the halo layer next to it)."""
    a, b, c = geo.face_axes(o)
    side = 1.0 if geo.fine_on_plus_side(o) else -1.0
    depth_T = side * target_pos[a]  # distance of the target centre into the fine side
    tang = {}
    for ax in (b, c):
        lo = target_pos[ax] - 1.5
        under = [i for i in range(ext[ax]) if lo < fine_pos[ax][i] < lo + 3.0]
        if len(under) == 3:
            tang[ax] = {i: 1.0 / 3.0 for i in under}
        else:
            # p not a multiple of 3: the coarse column straddles two fine
            # faces; this face holds the fine column through its centre
            hit = [i for i in under if fine_pos[ax][i] == target_pos[ax]]
            assert len(hit) == 1
            tang[ax] = {hit[0]: 1.0}
    layers = sorted(range(ext[a]), key=lambda i: side * fine_pos[a][i])
    inner = [i for i in layers if side * fine_pos[a][i] > 0]
    covered = [i for i in inner if abs(side * fine_pos[a][i] - depth_T) < 1.5]
    if len(covered) == 3:
        normal = {i: 1.0 / 3.0 for i in covered}
    else:
        i1, i2 = layers[-2], layers[-1]
        d1, d2 = side * fine_pos[a][i1], side * fine_pos[a][i2]
        t = (depth_T - d1) / (d2 - d1)
        normal = {i1: 1.0 - t, i2: t}
    row = np.zeros(geo.cell_count(p, k))
    for ia, wa in normal.items():
        for ib, wb in tang[b].items():
            for ic, wc in tang[c].items():
                idx = [0, 0, 0]
                idx[a], idx[b], idx[c] = ia, ib, ic
                row[geo.cell_index(ext, idx)] += wa * wb * wc
    return row


@lru_cache(maxsize=None)
def restriction_operator(scheme, p, k, o, s):
    """(rows, W): coarse fine-side-half cells under subface s, and their
    weights over every cell of the fine face buffer."""
    _check(scheme, p, k, o, s)
    a, b, c = geo.face_axes(o)
    ext = geo.face_extents(o, p, k)
    cells = geo.storage_cells(ext)
    ncell = len(cells)
    fpos = np.array([geo.fine_position(o, p, k, s, fc) for fc in cells])
    per_axis_pos = {
        ax: [geo.fine_position(o, p, k, s, tuple(i if d == ax else 0 for d in range(3)))[ax]
             for i in range(ext[ax])]
        for ax in range(3)
    }
    sb, sc = s % 3, s // 3
    rows, W = [], []
    for tc in cells:
        if not geo.coarse_fine_side_half(o, k, tc):
            continue
        XT = geo.coarse_position(o, p, k, tc)
        # the coarse columns whose centre lies on this fine face (with p not a
        # multiple of 3 a coarse column straddles two fine faces; its centre
        # never lies on their boundary)
        if not (sb * p <= XT[b] < (sb + 1) * p and sc * p <= XT[c] < (sc + 1) * p):
            continue
        if scheme == DLINEAR:
            row = _dlinear_restriction_row(o, p, k, s, XT, per_axis_pos, ext)
        else:
            # The fine cell closest to the coarse centre (must be unique).
            d2 = ((fpos - XT) ** 2).sum(axis=1)
            best = np.flatnonzero(d2 == d2.min())
            if len(best) != 1:
                raise AssertionError("nearest fine cell is not unique")
            home = cells[int(best[0])]
            stencil = taylor_stencil(home, ext, scheme)
            offsets = [fpos[geo.cell_index(ext, q)] - fpos[int(best[0])] for q in stencil]
            target = XT - fpos[int(best[0])]
            w = pinned_fit_weights(offsets, stencil.index(home), target, scheme)
            row = np.zeros(ncell)
            for q, wq in zip(stencil, w):
                row[geo.cell_index(ext, q)] += wq
        rows.append(geo.cell_index(ext, tc))
        W.append(row)
    return np.array(rows, dtype=np.int64), np.array(W)


def transfer_operator(direction, scheme, p, k, o, s):
    if direction == INTERPOLATE:
        return interpolation_operator(scheme, p, k, o, s)
    if direction == RESTRICT:
        return restriction_operator(scheme, p, k, o, s)
    raise ValueError(f"unknown direction {direction}")


def clear_operator_cache():
    interpolation_operator.cache_clear()
    restriction_operator.cache_clear()


def _apply(direction, scheme, p, k, orientation, subface, src_offset, dst_offset, U, src, dst):
    """dst (a copy) with every face's destination rows replaced by W @ source."""
    src = np.asarray(src, dtype=np.float64)
    out = np.array(dst, dtype=np.float64, copy=True)
    ncell = geo.cell_count(p, k)
    for f in range(len(orientation)):
        rows, W = transfer_operator(direction, scheme, p, k, int(orientation[f]), int(subface[f]))
        s0, d0 = int(src_offset[f]), int(dst_offset[f])
        x = src[s0 : s0 + ncell * U].reshape(ncell, U)
        y = out[d0 : d0 + ncell * U].reshape(ncell, U)
        y[rows] = W @ x
    return out


def interpolate_faces(scheme, p, k, orientation, subface, coarse_offset, fine_offset, U, coarse, fine):
    """Fill the ghost half of every fine face from its coarse face.

    orientation, subface : per-face ints; coarse_offset / fine_offset: element
    offsets of each face's buffers inside the flat `coarse` / `fine` arrays.
    Returns a float64 copy of `fine` with the ghost halves written.
    """
    return _apply(INTERPOLATE, scheme, p, k, orientation, subface, coarse_offset, fine_offset, U, coarse, fine)


def restrict_faces(scheme, p, k, orientation, subface, coarse_offset, fine_offset, U, fine, coarse):
    """Fill each fine face's segment of its coarse face's fine-side half.
    Returns a float64 copy of `coarse` with those segments written."""
    return _apply(RESTRICT, scheme, p, k, orientation, subface, fine_offset, coarse_offset, U, fine, coarse)
