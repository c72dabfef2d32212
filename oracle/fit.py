"""Taylor fits and 1D linear weights (oracle; test infrastructure).

Section 3 ("Operator construction"): per expansion cell, the derivatives up to
order D (in 3D, D = 2: n = 1 + 3 + 6 = 10 terms, D = 3: n = 20; in 2D 6 and 10)
are fitted from the
values at a stencil of cell centres, giving an s x n system A x = Q that is
solved with a QR decomposition ("standard matrix inversion"), and the fitted
Taylor polynomial is evaluated at the target centres.

Readings where the paper is silent (each listed in the design notes):

* The constant term is pinned to the expansion cell's own value and the other
  n - 1 derivatives are the unweighted least-squares solution over the
  remaining stencil points.  Without the pin a least-squares fit would not
  reproduce the centre value, and Section 3's coincident-centre injection
  would not hold.
* Appendix C: stencils are central inside the face data and are shifted
  toward the face interior near its edges and vertices (no diagonal data
  exists).  Second order: the 3x3x3 box around the expansion cell, with each
  axis' box centre clamped into [1, e - 2].  Third order (the cited
  Colella-McCorquodale stencil is not printed): that box plus the points two
  cells away from the clamped box centre along each axis, where inside the
  data.  Both rules are mirror- and permutation-symmetric.
* d-linear: per axis linear interpolation between the two bracketing centres,
  linear extrapolation from the two end centres beyond the data, and a pure
  copy where the target coincides with a centre.
"""

import math
from fractions import Fraction
from functools import lru_cache
from itertools import product
from math import factorial

import numpy as np
from scipy.linalg import solve_triangular


def taylor_exponents(degree, dim=3):
    """Multi-indices alpha (dim components) with 1 <= |alpha| <= degree (the
    non-constant terms)."""
    out = []
    for total in range(1, degree + 1):
        for alpha in product(range(total + 1), repeat=dim):
            if sum(alpha) == total:
                out.append(alpha)
    return out


def taylor_term(offset, alpha):
    """Taylor basis term offset^alpha / alpha! for an offset vector."""
    val = 1.0
    for d, e in zip(offset, alpha):
        val *= d**e / factorial(e)
    return val


def taylor_stencil(centre, ext, degree):
    """Stencil (list of index triples) for an expansion cell at `centre` inside a
    buffer of extents `ext` (Appendix C, reading above)."""
    dim = len(centre)
    shifted = [min(max(int(ci), 1), int(e) - 2) for ci, e in zip(centre, ext)]
    pts = []
    for d in product((-1, 0, 1), repeat=dim):
        pts.append(tuple(shifted[ax] + d[ax] for ax in range(dim)))
    if degree >= 3:
        for ax in range(dim):
            for step in (-2, 2):
                q = list(shifted)
                q[ax] += step
                if 0 <= q[ax] < ext[ax]:
                    pts.append(tuple(q))
    if tuple(int(c) for c in centre) not in pts:
        raise AssertionError("expansion cell must lie in its own stencil")
    return pts


@lru_cache(maxsize=None)
def _derivative_operator(offsets, centre_pos, degree):
    """QR solve of the pinned fit for one stencil: the matrix that maps the
    stencil values minus the centre value to the derivatives."""
    s = len(offsets)
    exps = taylor_exponents(degree, len(offsets[0]))
    others = [q for q in range(s) if q != centre_pos]
    # A: rows = stencil points other than the centre, columns = derivatives.
    A = np.array([[taylor_term(offsets[q], al) for al in exps] for q in others])
    if np.linalg.matrix_rank(A) < len(exps):
        raise AssertionError("stencil does not determine all derivatives")
    Qm, Rm = np.linalg.qr(A, mode="reduced")
    # derivatives = R^{-1} Q^T (Q_others - Q_centre): one column per stencil value.
    return solve_triangular(Rm, Qm.T), tuple(others)


def pinned_fit_weights(offsets, centre_pos, target, degree):
    """Weights w over the stencil such that sum_q w_q Q_q is the Taylor
    polynomial of degree `degree`, fitted with its constant pinned to the
    centre value, evaluated at `target`.

    offsets    : (s, d) stencil offsets from the expansion centre (d = 2 or 3)
    centre_pos : position of the expansion cell inside the stencil list
    target     : (d,) offset of the evaluation point from the centre
    """
    key = tuple(tuple(float(v) for v in row) for row in offsets)
    deriv_op, others = _derivative_operator(key, int(centre_pos), int(degree))
    t = np.array([taylor_term(target, al) for al in taylor_exponents(degree, len(key[0]))])
    w_others = t @ deriv_op
    w = np.zeros(len(key))
    w[list(others)] = w_others
    w[centre_pos] = 1.0 - w_others.sum()
    return w


def linear_weights_1d(x, n):
    """{centre index: weight} for 1D linear interpolation at coordinate x
    (a Fraction, in units where centre i sits at i) on centres 0..n-1, with
    linear extrapolation from the end pair outside [0, n-1]."""
    x = Fraction(x)
    if x.denominator == 1 and 0 <= x <= n - 1:
        return {int(x): 1.0}
    a = min(max(math.floor(x), 0), n - 2)
    t = x - a
    return {a: float(1 - t), a + 1: float(t)}
