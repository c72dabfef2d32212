"""Patches with face halos, and the transfer written straight into them
(oracle; test infrastructure).

Section 2: every leaf of the spacetree is a patch of p^3 cells; each patch has
a halo of depth k on its six faces only (no edge or corner halos), which is
refilled at the start of a time step from the face-connected neighbours.
Between two patches of one level the halo is a plain copy of the neighbour's
boundary layers; at a resolution transition the fine halo is interpolated
from the coarse patch and the coarse halo is restricted from the fine
patches.  The face data used by the transfer (2k layers across the face,
p x p cells along it) are exactly the boundary layers of one patch and the
halo layers that face them.

Storage convention (stated here; the library documents the same one): a
patch is a box of P = p + 2k cells per axis whose interior is [k, k + p) on
every axis.  Cell (i0, i1, i2) is cell number (i2 * P + i1) * P + i0 (axis 0
fastest) and unknown u of it is element cell * U + u.  Cells outside the
interior on more than one axis (edges, corners) exist in storage but belong
to no halo.

Patch faces are numbered f = a + 3 * upper: f < 3 is the face at the lower
boundary along axis a, f >= 3 the one at the upper boundary.  The face view of
face f is the 2k x p x p box of cells around that face: normal range [0, 2k)
(f < 3) or [p, p + 2k) (f >= 3), tangential ranges [k, k + p).  Since it is
taken from the patch box with axis 0 still fastest, its cells in storage order
are the cells of a face buffer of that face (the face-buffer layout of the
geometry module): buffer layer 0 is the layer on the - side of the face.  The
half of the view inside the patch is its "inner" half, the other its "outer"
(halo) half.

At a transition face of orientation o (geometry module: normal a = o mod 3,
fine patch on the + side when o < 3) the fine patch's face is f = o and the
coarse patch's face is f = (o + 3) mod 6.  The fine ghost half of the fine face
buffer is then the fine patch's outer half, and the coarse face's fine-side
half is the coarse patch's outer half.

Every function here is the plain composition of slices with the face-buffer
transfer of the transfer module.
"""

import numpy as np

from . import transfer as tr

INNER, OUTER, BOTH = 1, 2, 3


def patch_extent(p, k):
    return p + 2 * k


def patch_cells(p, k):
    return patch_extent(p, k) ** 3


def _check(p, k):
    if p < 1 or k < 1:
        raise ValueError("p and k must be positive")


def _box(flat, offset, P, U):
    """The patch at `offset` of a flat array, as a writable [i2, i1, i0, u] view."""
    return flat[offset : offset + P**3 * U].reshape(P, P, P, U)


def _normal_range(face, p, k, halves):
    """Normal index range (in patch coordinates) of the chosen halves of the
    face view of `face`."""
    upper = face >= 3
    lo = p if upper else 0  # first normal index of the 2k-layer view
    # view layers [0, k) are on the - side of the face: inside the patch for an
    # upper face, in the halo for a lower face
    minus_is_inner = upper
    if halves == BOTH:
        return lo, lo + 2 * k
    want_minus = (halves == INNER) == minus_is_inner
    return (lo, lo + k) if want_minus else (lo + k, lo + 2 * k)


def _view_slices(face, p, k, halves):
    """numpy slices [i2, i1, i0] of the chosen halves of the face view."""
    if not (0 <= face < 6) or halves not in (INNER, OUTER, BOTH):
        raise ValueError("face in 0..5 and halves in {1, 2, 3} required")
    a = face % 3
    n0, n1 = _normal_range(face, p, k, halves)
    per_axis = [slice(k, k + p)] * 3
    per_axis[a] = slice(n0, n1)
    return per_axis[2], per_axis[1], per_axis[0]


def _buffer_slices(face, p, k, halves):
    """numpy slices [i2, i1, i0] of the same halves inside a face buffer."""
    a = face % 3
    n0, _ = _normal_range(face, p, k, BOTH)
    m0, m1 = _normal_range(face, p, k, halves)
    per_axis = [slice(0, p)] * 3
    per_axis[a] = slice(m0 - n0, m1 - n0)
    return per_axis[2], per_axis[1], per_axis[0]


def face_buffer_shape(face, p, k, U):
    ext = [p, p, p]
    ext[face % 3] = 2 * k
    return ext[2], ext[1], ext[0], U


def gather_patch_faces(p, k, face, patch_offset, face_offset, U, halves, patches, faces):
    """Copy the chosen halves of face view face[i] of the patch at
    patch_offset[i] into the face buffer at face_offset[i].  Returns a float64
    copy of `faces` with those cells written."""
    _check(p, k)
    P = patch_extent(p, k)
    src = np.asarray(patches, dtype=np.float64)
    out = np.array(faces, dtype=np.float64, copy=True)
    nbuf = 2 * k * p * p * U
    for i in range(len(face)):
        f = int(face[i])
        box = _box(src, int(patch_offset[i]), P, U)
        fo = int(face_offset[i])
        buf = out[fo : fo + nbuf].reshape(face_buffer_shape(f, p, k, U))
        buf[_buffer_slices(f, p, k, halves)] = box[_view_slices(f, p, k, halves)]
    return out


def scatter_patch_faces(p, k, face, patch_offset, face_offset, U, halves, faces, patches):
    """Copy the chosen halves of each face buffer back into face view face[i]
    of its patch.  Returns a float64 copy of `patches`."""
    _check(p, k)
    P = patch_extent(p, k)
    src = np.asarray(faces, dtype=np.float64)
    out = np.array(patches, dtype=np.float64, copy=True)
    nbuf = 2 * k * p * p * U
    for i in range(len(face)):
        f = int(face[i])
        fo = int(face_offset[i])
        buf = src[fo : fo + nbuf].reshape(face_buffer_shape(f, p, k, U))
        box = _box(out, int(patch_offset[i]), P, U)
        box[_view_slices(f, p, k, halves)] = buf[_buffer_slices(f, p, k, halves)]
    return out


def copy_patch_halos(p, k, axis, minus_offset, plus_offset, U, patches):
    """Same-level halo exchange (Section 2: a plain copy where both patches
    have one resolution).  For pair i the patch at minus_offset[i] touches the
    patch at plus_offset[i] across its upper face along axis[i]: the upper
    halo of the first receives the second's lowest k interior layers, and the
    lower halo of the second receives the first's highest k interior layers.
    Returns a float64 copy of `patches`."""
    _check(p, k)
    P = patch_extent(p, k)
    out = np.array(patches, dtype=np.float64, copy=True)
    for i in range(len(axis)):
        a = int(axis[i])
        if not (0 <= a < 3):
            raise ValueError("axis in 0..2 required")
        lo = _box(out, int(minus_offset[i]), P, U)
        hi = _box(out, int(plus_offset[i]), P, U)
        lo_halo = _view_slices(a + 3, p, k, OUTER)
        hi_inner = _view_slices(a, p, k, INNER)
        hi_halo = _view_slices(a, p, k, OUTER)
        lo_inner = _view_slices(a + 3, p, k, INNER)
        # both reads precede both writes (they touch disjoint cells anyway)
        a_vals = hi[hi_inner].copy()
        b_vals = lo[lo_inner].copy()
        lo[lo_halo] = a_vals
        hi[hi_halo] = b_vals
    return out


def interpolate_patches(scheme, p, k, orientation, subface, coarse_offset, fine_offset, U, coarse, fine):
    """Fill the halo of each fine patch across its transition face from the
    coarse patch: gather the coarse patch's face view (both halves), apply the
    face-buffer interpolation, and write the result's ghost half into the fine
    patch's outer half.  Returns a float64 copy of `fine`."""
    _check(p, k)
    src = np.asarray(coarse, dtype=np.float64)
    out = np.array(fine, dtype=np.float64, copy=True)
    nbuf = 2 * k * p * p * U
    zero = np.zeros(1, dtype=np.int64)
    for i in range(len(orientation)):
        o, s = int(orientation[i]), int(subface[i])
        cf, ff = (o + 3) % 6, o
        cbuf = gather_patch_faces(p, k, [cf], [int(coarse_offset[i])], zero, U, BOTH, src, np.zeros(nbuf))
        fbuf = gather_patch_faces(p, k, [ff], [int(fine_offset[i])], zero, U, BOTH, out, np.zeros(nbuf))
        fbuf = tr.interpolate_faces(scheme, p, k, [o], [s], zero, zero, U, cbuf, fbuf)
        out = scatter_patch_faces(p, k, [ff], [int(fine_offset[i])], zero, U, OUTER, fbuf, out)
    return out


def restrict_patches(scheme, p, k, orientation, subface, coarse_offset, fine_offset, U, fine, coarse):
    """Fill, in the halo of each coarse patch, the segment under each fine
    patch: gather both face views, apply the face-buffer restriction, and
    write the coarse face's fine-side half back into the coarse patch's outer
    half (cells outside the segment are written back unchanged).  Returns a
    float64 copy of `coarse`."""
    _check(p, k)
    src = np.asarray(fine, dtype=np.float64)
    out = np.array(coarse, dtype=np.float64, copy=True)
    nbuf = 2 * k * p * p * U
    zero = np.zeros(1, dtype=np.int64)
    for i in range(len(orientation)):
        o, s = int(orientation[i]), int(subface[i])
        cf, ff = (o + 3) % 6, o
        fbuf = gather_patch_faces(p, k, [ff], [int(fine_offset[i])], zero, U, BOTH, src, np.zeros(nbuf))
        cbuf = gather_patch_faces(p, k, [cf], [int(coarse_offset[i])], zero, U, BOTH, out, np.zeros(nbuf))
        cbuf = tr.restrict_faces(scheme, p, k, [o], [s], zero, zero, U, fbuf, cbuf)
        out = scatter_patch_faces(p, k, [cf], [int(coarse_offset[i])], zero, U, OUTER, cbuf, out)
    return out
