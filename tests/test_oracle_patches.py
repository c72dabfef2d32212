"""Pins of the oracle's patch functions (oracle/patches.py) against positions.

The oracle extracts face views with index slices; these tests never use those
slices.  They place patches in one physical frame, sample a field at every
cell centre, and check each result cell by cell against the field at the
centre the storage conventions assign to it: a face-buffer cell from the
face-buffer layout (normal layer i centred (i - k + 1/2) widths from the face
plane, tangential cell j centred (j + 1/2) widths from the face's lower
corner), a patch cell from the patch layout (cell i centred (i - k + 1/2)
widths from the interior's lower corner).  For the transfer composed with
patches, polynomial reproduction (Section 5.1) fixes the answer: a cubic field
comes out exact from the third-order schemes, a trilinear one from the
d-linear scheme.  A slice on the wrong side, a swapped half or face, or a
misplaced subface breaks these equalities.
"""

import itertools

import numpy as np
import pytest

from oracle import patches as pt
from oracle import DLINEAR, TAYLOR2, TAYLOR3

SENT = -7.25e11


def cubic_field(U, seed, degree=3):
    """Field with U components, each a random polynomial of the given degree."""
    rng = np.random.default_rng(seed)
    exps = [e for e in itertools.product(range(degree + 1), repeat=3) if sum(e) <= degree]
    coef = rng.normal(size=(U, len(exps)))

    def f(x):
        x = np.asarray(x, dtype=np.float64) / 40.0
        t = np.array([x[0] ** e[0] * x[1] ** e[1] * x[2] ** e[2] for e in exps])
        return coef @ t

    return f


def patch_centre(corner, h, p, k, idx):
    """Centre of patch cell idx (patch layout)."""
    return np.array([corner[ax] + (idx[ax] - k + 0.5) * h for ax in range(3)])


def sample_patch(field, corner, h, p, k, U, interior_only=False):
    P = p + 2 * k
    out = np.full((P, P, P, U), SENT)
    for i2, i1, i0 in itertools.product(range(P), repeat=3):
        idx = (i0, i1, i2)
        inside = [k <= v < k + p for v in idx]
        if interior_only and not all(inside):
            continue
        if sum(not v for v in inside) > 1:
            continue  # edge / corner cells belong to no halo
        out[i2, i1, i0] = field(patch_centre(corner, h, p, k, idx))
    return out.reshape(-1)


def face_cell_centre(face, corner, h, p, k, idx):
    """Centre of face-buffer cell idx of patch face `face` (face-buffer layout)."""
    a = face % 3
    plane = corner[a] + (p * h if face >= 3 else 0.0)
    pos = []
    for ax in range(3):
        if ax == a:
            pos.append(plane + (idx[ax] - k + 0.5) * h)
        else:
            pos.append(corner[ax] + (idx[ax] + 0.5) * h)
    return np.array(pos)


def in_patch(face, k, idx):
    """True if face-buffer layer idx[a] lies on the patch's own side."""
    a = face % 3
    minus = idx[a] < k
    return minus if face >= 3 else not minus


def buffer_cells(face, p, k):
    ext = [p, p, p]
    ext[face % 3] = 2 * k
    return [(i0, i1, i2) for i2 in range(ext[2]) for i1 in range(ext[1]) for i0 in range(ext[0])]


@pytest.mark.parametrize("p,k", [(6, 2), (6, 3)])
@pytest.mark.parametrize("halves", [pt.INNER, pt.OUTER, pt.BOTH])
def test_gather_by_position(p, k, halves):
    U = 2
    field = cubic_field(U, 1)
    corner = (3.0, -5.0, 7.0)
    patch = sample_patch(field, corner, 1.0, p, k, U)
    nbuf = 2 * k * p * p * U
    for face in range(6):
        out = pt.gather_patch_faces(p, k, [face], [0], [nbuf], U, halves, patch, np.full(3 * nbuf, SENT))
        assert np.all(out[:nbuf] == SENT) and np.all(out[2 * nbuf :] == SENT)
        buf = out[nbuf : 2 * nbuf].reshape(-1, U)
        for n, idx in enumerate(buffer_cells(face, p, k)):
            inside = in_patch(face, k, idx)
            chosen = halves == pt.BOTH or (halves == pt.INNER) == inside
            if chosen:
                assert np.array_equal(buf[n], field(face_cell_centre(face, corner, 1.0, p, k, idx))), (face, idx)
            else:
                assert np.all(buf[n] == SENT)


@pytest.mark.parametrize("p,k", [(6, 2), (9, 3)])
@pytest.mark.parametrize("halves", [pt.INNER, pt.OUTER])
def test_scatter_by_position(p, k, halves):
    U = 2
    field = cubic_field(U, 2)
    corner = (0.0, 9.0, -3.0)
    P = p + 2 * k
    for face in range(6):
        buf = np.concatenate([field(face_cell_centre(face, corner, 1.0, p, k, idx)) for idx in buffer_cells(face, p, k)])
        out = pt.scatter_patch_faces(p, k, [face], [P**3 * U], [0], U, halves, buf, np.full(2 * P**3 * U, SENT))
        assert np.all(out[: P**3 * U] == SENT)
        box = out[P**3 * U :].reshape(P, P, P, U)
        written = 0
        for i2, i1, i0 in itertools.product(range(P), repeat=3):
            v = box[i2, i1, i0]
            if np.all(v == SENT):
                continue
            written += 1
            assert np.array_equal(v, field(patch_centre(corner, 1.0, p, k, (i0, i1, i2))))
        assert written == k * p * p


@pytest.mark.parametrize("p,k", [(6, 2), (9, 3)])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_halo_copy_by_position(p, k, axis):
    """Two neighbours of one level, interiors sampled from one field: after the
    exchange both facing halos hold the field at their centres and nothing
    else changed."""
    U = 2
    field = cubic_field(U, 3)
    P = p + 2 * k
    c0 = np.array([2.0, -4.0, 1.0])
    c1 = c0.copy()
    c1[axis] += p
    a = sample_patch(field, c0, 1.0, p, k, U, interior_only=True)
    b = sample_patch(field, c1, 1.0, p, k, U, interior_only=True)
    n = P**3 * U
    flat = np.concatenate([np.full(n, SENT), b, a])  # plus patch at n, minus patch at 2n
    out = pt.copy_patch_halos(p, k, [axis], [2 * n], [n], U, flat)
    assert np.all(out[:n] == SENT)
    for patch, corner, off, upper in ((b, c1, n, False), (a, c0, 2 * n, True)):
        box_in = patch.reshape(P, P, P, U)
        box = out[off : off + n].reshape(P, P, P, U)
        changed = 0
        for i2, i1, i0 in itertools.product(range(P), repeat=3):
            idx = (i0, i1, i2)
            if np.array_equal(box[i2, i1, i0], box_in[i2, i1, i0]):
                continue
            changed += 1
            tang = all(k <= idx[ax] < k + p for ax in range(3) if ax != axis)
            na = idx[axis]
            assert tang and ((na >= p + k) if upper else (na < k)), idx
            assert np.array_equal(box[i2, i1, i0], field(patch_centre(corner, 1.0, p, k, idx)))
        assert changed == k * p * p


def transition(o, s, p):
    """Lower interior corners of a coarse patch (width 3) and of the fine patch
    (width 1) that is subface s across face orientation o of it."""
    a = o % 3
    b, c = [ax for ax in range(3) if ax != a]
    cc = np.array([-27.0, 9.0, 18.0])
    fc = cc.copy()
    fc[a] = cc[a] + 3 * p if o < 3 else cc[a] - p
    fc[b] = cc[b] + (s % 3) * p
    fc[c] = cc[c] + (s // 3) * p
    return cc, fc


CASES = [(DLINEAR, 1), (TAYLOR2, 2), (TAYLOR3, 3)]


@pytest.mark.parametrize("p,k", [(6, 2), (6, 3)])
@pytest.mark.parametrize("scheme,degree", CASES)
def test_interpolate_patches_reproduces(p, k, scheme, degree):
    U = 2
    P = p + 2 * k
    n = P**3 * U
    for o in range(6):
        for s in (0, 5, 7):
            field = cubic_field(U, 10 * o + s, degree=degree) if degree != 1 else trilinear(U, o + s)
            cc, fc = transition(o, s, p)
            coarse = sample_patch(field, cc, 3.0, p, k, U)
            fine = sample_patch(field, fc, 1.0, p, k, U, interior_only=True)
            out = pt.interpolate_patches(scheme, p, k, [o], [s], [0], [n], U, coarse, np.concatenate([fine, fine]))
            assert np.array_equal(out[:n], fine)
            box_in = fine.reshape(P, P, P, U)
            box = out[n:].reshape(P, P, P, U)
            changed = 0
            for i2, i1, i0 in itertools.product(range(P), repeat=3):
                idx = (i0, i1, i2)
                if np.array_equal(box[i2, i1, i0], box_in[i2, i1, i0]):
                    continue
                changed += 1
                want = field(patch_centre(fc, 1.0, p, k, idx))
                assert np.allclose(box[i2, i1, i0], want, rtol=0, atol=1e-11 * (1 + np.abs(want).max())), (o, s, idx)
            assert changed == k * p * p, (o, s)


def trilinear(U, seed):
    rng = np.random.default_rng(seed)
    coef = rng.normal(size=(U, 8))

    def f(x):
        x = np.asarray(x, dtype=np.float64) / 40.0
        t = np.array([x[0] ** e[0] * x[1] ** e[1] * x[2] ** e[2] for e in itertools.product((0, 1), repeat=3)])
        return coef @ t

    return f


@pytest.mark.parametrize("p,k", [(6, 2), (6, 3)])
@pytest.mark.parametrize("scheme,degree", CASES)
def test_restrict_patches_reproduces(p, k, scheme, degree):
    """The coarse halo segment under the fine patch receives the field; the
    rest of the coarse patch is unchanged."""
    U = 2
    P = p + 2 * k
    n = P**3 * U
    E = p // 3
    for o in range(6):
        for s in (1, 4, 8):
            field = cubic_field(U, 7 * o + s, degree=degree) if degree != 1 else trilinear(U, o + 2 * s)
            cc, fc = transition(o, s, p)
            fine = sample_patch(field, fc, 1.0, p, k, U)
            coarse = sample_patch(field, cc, 3.0, p, k, U, interior_only=True)
            out = pt.restrict_patches(scheme, p, k, [o], [s], [0], [0], U, fine, coarse)
            box_in = coarse.reshape(P, P, P, U)
            box = out.reshape(P, P, P, U)
            a = o % 3
            b, c = [ax for ax in range(3) if ax != a]
            changed = 0
            for i2, i1, i0 in itertools.product(range(P), repeat=3):
                idx = (i0, i1, i2)
                if np.array_equal(box[i2, i1, i0], box_in[i2, i1, i0]):
                    continue
                changed += 1
                na = idx[a]
                assert (na >= p + k) if o < 3 else (na < k), (o, s, idx)
                assert k + (s % 3) * E <= idx[b] < k + (s % 3 + 1) * E
                assert k + (s // 3) * E <= idx[c] < k + (s // 3 + 1) * E
                want = field(patch_centre(cc, 3.0, p, k, idx))
                tol = 1e-9 * (1 + np.abs(want).max())
                assert np.allclose(box[i2, i1, i0], want, rtol=0, atol=tol), (o, s, idx)
            assert changed == k * E * E, (o, s)


def test_restrict_patches_nine_subfaces_fill_halo():
    """All nine fine patches of one coarse face together fill its whole halo
    half, each writing only its own segment."""
    p, k, U = 6, 2, 1
    P = p + 2 * k
    n = P**3 * U
    field = cubic_field(U, 99)
    o = 4
    fines = []
    for s in range(9):
        cc, fc = transition(o, s, p)
        fines.append(sample_patch(field, fc, 1.0, p, k, U))
    cc, _ = transition(o, 0, p)
    coarse = sample_patch(field, cc, 3.0, p, k, U, interior_only=True)
    out = pt.restrict_patches(TAYLOR3, p, k, [o] * 9, list(range(9)), [0] * 9, [i * n for i in range(9)], U, np.concatenate(fines), coarse)
    box = out.reshape(P, P, P, U)
    a = o % 3
    for i2, i1, i0 in itertools.product(range(P), repeat=3):
        idx = (i0, i1, i2)
        face_halo = idx[a] < k and all(k <= idx[ax] < k + p for ax in range(3) if ax != a)
        if face_halo:
            want = field(patch_centre(cc, 3.0, p, k, idx))
            assert np.allclose(box[i2, i1, i0], want, atol=1e-9 * (1 + abs(want).max()))
        else:
            assert np.array_equal(box[i2, i1, i0], coarse.reshape(P, P, P, U)[i2, i1, i0])


# Planted mistakes (on the CPU): each must make one of the pins above fail.


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_swapped_halves_are_caught(monkeypatch):
    real = pt._normal_range

    def swapped(face, p, k, halves):
        h = {pt.INNER: pt.OUTER, pt.OUTER: pt.INNER}.get(halves, halves)
        return real(face, p, k, h)

    monkeypatch.setattr(pt, "_normal_range", swapped)
    assert _fails(test_gather_by_position, 6, 2, pt.INNER)
    assert _fails(test_halo_copy_by_position, 6, 2, 1)


def test_untrimmed_tangential_range_is_caught(monkeypatch):
    real = pt._view_slices

    def shifted(face, p, k, halves):
        sl = list(real(face, p, k, halves))
        return tuple(slice(s.start - 1, s.stop - 1) if s.stop - s.start == p else s for s in sl)

    monkeypatch.setattr(pt, "_view_slices", shifted)
    assert _fails(test_gather_by_position, 6, 2, pt.BOTH)
    assert _fails(test_interpolate_patches_reproduces, 6, 2, TAYLOR2, 2)


def test_wrong_coarse_face_is_caught(monkeypatch):
    """Gathering the coarse patch's face on the wrong side of the patch."""
    real = pt.gather_patch_faces

    def wrong(p, k, face, *rest):
        return real(p, k, [(int(f) + 3) % 6 for f in face], *rest)

    monkeypatch.setattr(pt, "gather_patch_faces", wrong)
    assert _fails(test_interpolate_patches_reproduces, 6, 3, TAYLOR3, 3)
    assert _fails(test_restrict_patches_reproduces, 6, 3, TAYLOR3, 3)
