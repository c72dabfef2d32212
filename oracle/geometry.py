"""Face-buffer layout and cell-centre positions (oracle; test infrastructure).

The paper fixes the physical picture and leaves the bookkeeping open:

* Section 2: patches carry p cells per axis and a halo of depth k on their
  faces only; at a resolution transition the face data hold 2k layers along
  the normal (k on either side of the face) and p x p cells tangentially, and
  the unknowns of a cell are stored together ("AoS", lexicographic order).
* Section 2: three-partitioning, so a coarse face is covered by 3 x 3 fine
  faces and every fine cell is one third of a coarse cell per axis.
* Section 4.1: six face configurations, all rotations / mirrors of one.

Conventions used here (the library documents the same contract in its header):

* Orientation o in 0..5; normal axis a = o mod 3; the two tangential axes are
  the remaining ones in increasing order (b < c), never mirrored.
* For o < 3 the fine patch lies on the + side of the face, otherwise on the
  - side.
* A face buffer has extent 2k along a and p along b and c.  Cell (i0, i1, i2)
  (indices along physical axes 0, 1, 2) is stored at cell number
  (i2 * e1 + i1) * e0 + i0, i.e. axis 0 fastest, and unknown u of that cell at
  element cell * U + u.
* Normal index i_a in [0, k) is the - side of the face, [k, 2k) the + side.
* Fine subface (sb, sc) in {0,1,2}^2, numbered s = sb + 3 * sc, covers the
  tangential range [sb * p, (sb + 1) * p) x [sc * p, (sc + 1) * p) measured in
  fine cells from the coarse face's lower edge.

All positions below are in units of the fine mesh width, with the face plane
at normal coordinate 0 and the coarse face's lower tangential corner at 0.
Every centre is then a half-integer, so positions are exact in binary.
"""

import numpy as np


def face_axes(o):
    """Normal axis a and tangential axes b < c of orientation o."""
    if not (0 <= int(o) < 6):
        raise ValueError(f"orientation must be in 0..5, got {o}")
    a = int(o) % 3
    b, c = [ax for ax in range(3) if ax != a]
    return a, b, c


def fine_on_plus_side(o):
    return int(o) < 3


def face_extents(o, p, k):
    """Cell extents (e0, e1, e2) of a face buffer along the physical axes."""
    a, _, _ = face_axes(o)
    ext = [p, p, p]
    ext[a] = 2 * k
    return tuple(ext)


def cell_count(p, k):
    return 2 * k * p * p


def cell_index(ext, idx):
    """Storage number of cell idx = (i0, i1, i2) in a buffer of extents ext."""
    i0, i1, i2 = idx
    return (i2 * ext[1] + i1) * ext[0] + i0


def storage_cells(ext):
    """All cell index triples of a buffer, in storage order."""
    out = []
    for i2 in range(ext[2]):
        for i1 in range(ext[1]):
            for i0 in range(ext[0]):
                out.append((i0, i1, i2))
    return out


def coarse_position(o, p, k, idx):
    """Centre of coarse-face cell idx, in fine-mesh units (coarse width 3)."""
    a, _, _ = face_axes(o)
    pos = [0.0, 0.0, 0.0]
    for ax in range(3):
        if ax == a:
            pos[ax] = 3.0 * (idx[ax] - k) + 1.5
        else:
            pos[ax] = 3.0 * idx[ax] + 1.5
    return np.array(pos)


def fine_position(o, p, k, s, idx):
    """Centre of cell idx of the fine face that is subface s of the coarse face."""
    a, b, c = face_axes(o)
    shift = {b: (s % 3) * p, c: (s // 3) * p}
    pos = [0.0, 0.0, 0.0]
    for ax in range(3):
        if ax == a:
            pos[ax] = (idx[ax] - k) + 0.5
        else:
            pos[ax] = shift[ax] + idx[ax] + 0.5
    return np.array(pos)


def coarse_fine_side_half(o, k, idx):
    """True if coarse-face cell idx lies on the fine side (the restricted half)."""
    a, _, _ = face_axes(o)
    return (idx[a] >= k) if fine_on_plus_side(o) else (idx[a] < k)


def fine_ghost_half(o, k, idx):
    """True if fine-face cell idx lies on the coarse side (the interpolated halo)."""
    a, _, _ = face_axes(o)
    return (idx[a] < k) if fine_on_plus_side(o) else (idx[a] >= k)
