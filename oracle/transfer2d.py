"""The face transfer in two dimensions (oracle; test infrastructure).

Sections 2 and 3 state the method for any dimension d: patches of p^d cells
with halos of depth k, three-partitioning, P and R as one matrix per face, the
d-linear tensor-product baseline and Taylor fits of degree 2 and 3 about the
containing coarse cell (interpolation) or the nearest fine cell
(restriction); the experiments are three-dimensional.  This module is the
d = 2 instance, written like the three-dimensional one: every 1/3 segment is
built as a dense matrix from the physical cell-centre positions of the given
orientation.

Conventions (the two-dimensional counterparts of the geometry module):

* Orientation o in 0..3; normal axis a = o mod 2, tangential axis b = 1 - a;
  the fine patch lies on the + side for o < 2.
* A face buffer has 2k cells along a and p along b; cell (i0, i1) is cell
  number i1 * e0 + i0 (axis 0 fastest) and unknown u of it is element
  cell * U + u.  Normal index [0, k) is the - side of the face.
* Fine subface s in 0..2 covers fine columns [s p, (s + 1) p) of the coarse
  face, measured in fine cells from its lower edge.
* Stencils (Appendix C reading of the fit module): the 3 x 3 box around the
  expansion cell with its centre clamped into [1, e - 2] per axis, plus, for
  degree 3, the points two cells away along each axis where inside the data.
* p need not be a multiple of 3: as in three dimensions, a fine face
  restricts into the coarse columns whose centres it holds, and the
  averaging restriction of a coarse column that straddles two fine faces
  takes the fine column through its centre.
"""

from fractions import Fraction
from functools import lru_cache

import numpy as np

from .fit import linear_weights_1d, pinned_fit_weights, taylor_stencil

DLINEAR, TAYLOR2, TAYLOR3 = 1, 2, 3
INTERPOLATE, RESTRICT = 0, 1


def face_axes(o):
    if not (0 <= int(o) < 4):
        raise ValueError(f"orientation must be in 0..3, got {o}")
    a = int(o) % 2
    return a, 1 - a


def face_extents(o, p, k):
    a, _ = face_axes(o)
    ext = [p, p]
    ext[a] = 2 * k
    return tuple(ext)


def cell_count(p, k):
    return 2 * k * p


def cell_index(ext, idx):
    return idx[1] * ext[0] + idx[0]


def storage_cells(ext):
    return [(i0, i1) for i1 in range(ext[1]) for i0 in range(ext[0])]


def coarse_position(o, p, k, idx):
    """Centre of coarse-face cell idx in fine-mesh units (face plane at normal
    coordinate 0, lower edge of the coarse face at 0)."""
    a, _ = face_axes(o)
    return np.array([3.0 * (idx[ax] - k) + 1.5 if ax == a else 3.0 * idx[ax] + 1.5 for ax in range(2)])


def fine_position(o, p, k, s, idx):
    a, b = face_axes(o)
    pos = [0.0, 0.0]
    pos[a] = (idx[a] - k) + 0.5
    pos[b] = s * p + idx[b] + 0.5
    return np.array(pos)


def fine_on_plus_side(o):
    return int(o) < 2


def coarse_fine_side_half(o, k, idx):
    a, _ = face_axes(o)
    return (idx[a] >= k) if fine_on_plus_side(o) else (idx[a] < k)


def fine_ghost_half(o, k, idx):
    a, _ = face_axes(o)
    return (idx[a] < k) if fine_on_plus_side(o) else (idx[a] >= k)


def _check(scheme, p, k, o, s):
    if scheme not in (DLINEAR, TAYLOR2, TAYLOR3):
        raise ValueError(f"unknown scheme {scheme}")
    if p < 6:
        raise ValueError(f"p must be >= 6, got {p}")
    if k not in (1, 2, 3) or (k == 1 and scheme != DLINEAR):
        raise ValueError("k must be 2 or 3 (or 1 for the d-linear scheme)")
    if not (0 <= o < 4 and 0 <= s < 3):
        raise ValueError("orientation in 0..3 and subface in 0..2 required")


def _half_index(pos_fine_units, normal, k):
    """Coordinate of a position (fine units) in coarse centre-index units of a
    coarse face buffer (coarse cell i centred at coordinate i)."""
    x = Fraction(float(pos_fine_units))
    if normal:
        return (x - Fraction(3, 2)) / 3 + k
    return (x - Fraction(3, 2)) / 3


@lru_cache(maxsize=None)
def interpolation_operator(scheme, p, k, o, s):
    """(rows, W): fine ghost-half cells of subface s and their weights over all
    2kp cells of the coarse face buffer."""
    _check(scheme, p, k, o, s)
    a, _ = face_axes(o)
    ext = face_extents(o, p, k)
    cells = storage_cells(ext)
    coarse_pos = {c: coarse_position(o, p, k, c) for c in cells}
    rows, W = [], []
    for fc in cells:
        if not fine_ghost_half(o, k, fc):
            continue
        X = fine_position(o, p, k, s, fc)
        home = tuple(int(np.floor(X[ax] / 3.0)) + (k if ax == a else 0) for ax in range(2))
        if coarse_fine_side_half(o, k, home):
            raise AssertionError("fine ghost centre must lie inside the coarse patch")
        row = np.zeros(len(cells))
        if scheme == DLINEAR:
            per_axis = [linear_weights_1d(_half_index(X[ax], ax == a, k), ext[ax]) for ax in range(2)]
            for i0, w0 in per_axis[0].items():
                for i1, w1 in per_axis[1].items():
                    row[cell_index(ext, (i0, i1))] += w0 * w1
        else:
            stencil = taylor_stencil(home, ext, scheme)
            offsets = [(coarse_pos[q] - coarse_pos[home]) / 3.0 for q in stencil]
            target = (X - coarse_pos[home]) / 3.0
            w = pinned_fit_weights(offsets, stencil.index(home), target, scheme)
            for q, wq in zip(stencil, w):
                row[cell_index(ext, q)] += wq
        rows.append(cell_index(ext, fc))
        W.append(row)
    return np.array(rows, dtype=np.int64), np.array(W)


def _dlinear_restriction_row(o, p, k, target_pos, fine_pos, ext):
    """Mean over the three fine columns under the target; along the normal the
    mean of the three covering inner layers, else the line through the two
    fine layers deepest into the fine side."""
    a, b = face_axes(o)
    side = 1.0 if fine_on_plus_side(o) else -1.0
    depth_T = side * target_pos[a]
    lo = target_pos[b] - 1.5
    under = [i for i in range(ext[b]) if lo < fine_pos[b][i] < lo + 3.0]
    if len(under) == 3:
        tang = {i: 1.0 / 3.0 for i in under}
    else:
        # p not a multiple of 3: the fine column through the coarse centre
        tang = {i: 1.0 for i in under if fine_pos[b][i] == target_pos[b]}
        assert len(tang) == 1
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
    row = np.zeros(cell_count(p, k))
    for ia, wa in normal.items():
        for ib, wb in tang.items():
            idx = [0, 0]
            idx[a], idx[b] = ia, ib
            row[cell_index(ext, idx)] += wa * wb
    return row


@lru_cache(maxsize=None)
def restriction_operator(scheme, p, k, o, s):
    """(rows, W): coarse fine-side-half cells under subface s and their weights
    over all 2kp cells of the fine face buffer."""
    _check(scheme, p, k, o, s)
    a, b = face_axes(o)
    ext = face_extents(o, p, k)
    cells = storage_cells(ext)
    fpos = np.array([fine_position(o, p, k, s, fc) for fc in cells])
    per_axis_pos = {
        ax: [fine_position(o, p, k, s, tuple(i if d == ax else 0 for d in range(2)))[ax] for i in range(ext[ax])]
        for ax in range(2)
    }
    rows, W = [], []
    for tc in cells:
        if not coarse_fine_side_half(o, k, tc):
            continue
        XT = coarse_position(o, p, k, tc)
        if not (s * p <= XT[b] < (s + 1) * p):  # coarse centres on this fine face
            continue
        if scheme == DLINEAR:
            row = _dlinear_restriction_row(o, p, k, XT, per_axis_pos, ext)
        else:
            d2 = ((fpos - XT) ** 2).sum(axis=1)
            best = np.flatnonzero(d2 == d2.min())
            if len(best) != 1:
                raise AssertionError("nearest fine cell is not unique")
            home = cells[int(best[0])]
            stencil = taylor_stencil(home, ext, scheme)
            offsets = [fpos[cell_index(ext, q)] - fpos[int(best[0])] for q in stencil]
            target = XT - fpos[int(best[0])]
            w = pinned_fit_weights(offsets, stencil.index(home), target, scheme)
            row = np.zeros(len(cells))
            for q, wq in zip(stencil, w):
                row[cell_index(ext, q)] += wq
        rows.append(cell_index(ext, tc))
        W.append(row)
    return np.array(rows, dtype=np.int64), np.array(W)


def transfer_operator(direction, scheme, p, k, o, s):
    if direction == INTERPOLATE:
        return interpolation_operator(scheme, p, k, o, s)
    if direction == RESTRICT:
        return restriction_operator(scheme, p, k, o, s)
    raise ValueError(f"unknown direction {direction}")


def _apply(direction, scheme, p, k, orientation, subface, src_offset, dst_offset, U, src, dst):
    src = np.asarray(src, dtype=np.float64)
    out = np.array(dst, dtype=np.float64, copy=True)
    ncell = cell_count(p, k)
    for f in range(len(orientation)):
        rows, W = transfer_operator(direction, scheme, p, k, int(orientation[f]), int(subface[f]))
        s0, d0 = int(src_offset[f]), int(dst_offset[f])
        x = src[s0 : s0 + ncell * U].reshape(ncell, U)
        y = out[d0 : d0 + ncell * U].reshape(ncell, U)
        y[rows] = W @ x
    return out


def interpolate_faces(scheme, p, k, orientation, subface, coarse_offset, fine_offset, U, coarse, fine):
    """Two-dimensional faces: fill the ghost half of every fine face buffer."""
    return _apply(INTERPOLATE, scheme, p, k, orientation, subface, coarse_offset, fine_offset, U, coarse, fine)


def restrict_faces(scheme, p, k, orientation, subface, coarse_offset, fine_offset, U, fine, coarse):
    """Two-dimensional faces: fill each fine face's segment of its coarse
    face's fine-side half."""
    return _apply(RESTRICT, scheme, p, k, orientation, subface, fine_offset, coarse_offset, U, fine, coarse)


def clear_operator_cache():
    interpolation_operator.cache_clear()
    restriction_operator.cache_clear()
