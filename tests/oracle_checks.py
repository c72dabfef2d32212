"""Independent checks that pin the oracle to what the paper and mathematics fix.

Nothing here calls the oracle's geometry helpers: cell positions are rebuilt
with numpy index grids from the documented buffer convention, and exact
least-squares solutions are recomputed with rational arithmetic.  Each check
returns the worst deviation it saw so that the mutation tests can assert that
a planted mistake in the oracle is caught.
"""

import os
from fractions import Fraction
from itertools import product

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# --------------------------------------------------------------------------
# Geometry, restated with index grids (axis 0 fastest, fine-mesh units, face
# plane at normal coordinate 0, coarse face's lower tangential corner at 0).
# --------------------------------------------------------------------------
def buffer_grid(o, p, k):
    a = o % 3
    ext = [p, p, p]
    ext[a] = 2 * k
    g2, g1, g0 = np.indices((ext[2], ext[1], ext[0]))
    return a, ext, np.stack([g0.ravel(), g1.ravel(), g2.ravel()], axis=1)


def coarse_centres(o, p, k):
    a, _, idx = buffer_grid(o, p, k)
    pos = 3.0 * idx + 1.5
    pos[:, a] = 3.0 * (idx[:, a] - k) + 1.5
    return pos


def fine_centres(o, p, k, s):
    a, _, idx = buffer_grid(o, p, k)
    tang = [ax for ax in range(3) if ax != a]
    pos = idx + 0.5
    pos[:, a] = idx[:, a] - k + 0.5
    pos[:, tang[0]] += (s % 3) * p
    pos[:, tang[1]] += (s // 3) * p
    return pos


def depth_into_fine_side(o, p, k):
    """Reference normal index per buffer cell: 0 is the first layer on the fine
    side, -1 the first on the coarse side (mirror of the o >= 3 faces)."""
    a, _, idx = buffer_grid(o, p, k)
    return idx[:, a] - k if o < 3 else k - 1 - idx[:, a]


# --------------------------------------------------------------------------
# Polynomial fields
# --------------------------------------------------------------------------
def exponent_set(scheme):
    if scheme == 1:  # d-linear reproduces the trilinear space
        return [e for e in product((0, 1), repeat=3)]
    return [e for e in product(range(scheme + 1), repeat=3) if sum(e) <= scheme]


def poly_eval(pos, coeffs, exps, scale):
    x = pos / scale
    out = np.zeros(len(pos))
    for cf, e in zip(coeffs, exps):
        out += cf * x[:, 0] ** e[0] * x[:, 1] ** e[1] * x[:, 2] ** e[2]
    return out


def reproduction_error(oracle, scheme, p, k, o, s, rng, direction):
    """Max |oracle - exact| / max|exact| on a random polynomial of the
    scheme's reproduction space."""
    exps = exponent_set(scheme)
    coeffs = rng.normal(size=len(exps))
    scale = 3.0 * p
    cv = poly_eval(coarse_centres(o, p, k), coeffs, exps, scale)
    fv = poly_eval(fine_centres(o, p, k, s), coeffs, exps, scale)
    if direction == 0:
        rows, W = oracle.interpolation_operator(scheme, p, k, o, s)
        got, want = W @ cv, fv[rows]
    else:
        rows, W = oracle.restriction_operator(scheme, p, k, o, s)
        got, want = W @ fv, cv[rows]
    return np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)


# --------------------------------------------------------------------------
# Exact rational least squares (brute force)
# --------------------------------------------------------------------------
def exact_pinned_fit(offsets, centre_pos, target, degree):
    """Unweighted least squares with the constant pinned, solved exactly via
    the normal equations over plain monomials (not the Taylor basis)."""
    dim = len(offsets[0])
    exps = [e for e in product(range(degree + 1), repeat=dim) if 1 <= sum(e) <= degree]
    others = [q for q in range(len(offsets)) if q != centre_pos]

    def mono(d, e):
        v = Fraction(1)
        for di, ei in zip(d, e):
            v *= Fraction(di) ** ei
        return v

    A = [[mono(offsets[q], e) for e in exps] for q in others]
    n = len(exps)
    M = [[sum(A[r][i] * A[r][j] for r in range(len(A))) for j in range(n)] for i in range(n)]
    t = [mono(target, e) for e in exps]
    # Solve M^T z = t (M symmetric) by Gauss-Jordan, then w_others = A z.
    aug = [M[i][:] + [t[i]] for i in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        pv = aug[col][col]
        aug[col] = [v / pv for v in aug[col]]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [vr - f * vc for vr, vc in zip(aug[r], aug[col])]
    z = [aug[i][n] for i in range(n)]
    w_others = [sum(A[r][i] * z[i] for i in range(n)) for r in range(len(A))]
    w = [Fraction(0)] * len(offsets)
    for r, q in enumerate(others):
        w[q] = w_others[r]
    w[centre_pos] = 1 - sum(w_others)
    return w


# --------------------------------------------------------------------------
# Golden fixtures
# --------------------------------------------------------------------------
def load_stencil_fixture():
    cases = []
    with open(os.path.join(GOLDEN, "stencils.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            ext, centre, degree, box, extra = [f.strip() for f in line.split("|")]
            ext = tuple(int(v) for v in ext.split(","))
            centre = tuple(int(v) for v in centre.split(","))
            ranges = [tuple(int(v) for v in r.split("..")) for r in box.split(",")]
            pts = set(product(*[range(lo, hi + 1) for lo, hi in ranges]))
            for tok in extra.split():
                pts.add(tuple(int(v) for v in tok.split(",")))
            cases.append((ext, centre, int(degree), pts))
    return cases


def load_dlinear_fixture():
    cases = []
    with open(os.path.join(GOLDEN, "dlinear_1d.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            x, n, *pairs = line.split()
            want = {}
            for pr in pairs:
                i, w = pr.split(":")
                want[int(i)] = Fraction(w)
            cases.append((Fraction(x), int(n), want))
    return cases


def load_interior_taylor2():
    tab = {}
    with open(os.path.join(GOLDEN, "interior_taylor2.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, cls, w = line.split()
            tab[(kind, cls)] = Fraction(w)
    return tab


def interior_taylor2_weights(target):
    """Closed-form weights of the interior second-order fit at `target` (a
    3-tuple of Fractions), over offsets q in {-1,0,1}^3 (dict q -> Fraction)."""
    tab = load_interior_taylor2()
    out = {}
    for q in product((-1, 0, 1), repeat=3):
        w = Fraction(0)
        nz = sum(1 for v in q if v)
        if q == (0, 0, 0):
            w += 1  # pinned constant
            for i in range(3):
                w += tab[("pure", "centre")] * target[i] ** 2
        else:
            for i in range(3):
                if q[i]:
                    w += tab[("linear", "qx=+1" if q[i] > 0 else "qx=-1")] * target[i]
            for i in range(3):
                w += tab[("pure", f"({q[i] * q[i]},{nz})")] * target[i] ** 2
            for i in range(3):
                for j in range(i + 1, 3):
                    if q[i] and q[j]:
                        key = "qx*qy=+1" if q[i] * q[j] > 0 else "qx*qy=-1"
                        w += tab[("mixed", key)] * target[i] * target[j]
        out[q] = w
    return out
