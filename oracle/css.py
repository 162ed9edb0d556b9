"""Column subset selection and leverage scores of the selected columns, plain
FP64.  Test infrastructure: only the tests, the smoke check and the bench's
CPU baseline use this module; the library never does.

Paper passages followed (arXiv 2203.02798, section 4.1 and 4.3):

* Algorithm ``cgrrqr``: B = G S A (Algorithm ``countgauss_multiply``), a
  pivoted QR of B gives a permutation P, and its first k columns name the
  selected columns of A.
* Algorithm ``ls_hrn_exact``: select k columns K that way, then the
  leverage scores of A[:, K] by Algorithm ``ls_direct`` (exact leverage
  scores of the column subset).

Readings: the pivoted QR is the column-pivoted Householder QR of Businger and
Golub (1965), the one LAPACK's geqp3 computes: at step j the remaining column
with the largest norm of its rows j .. m-1 is brought to position j and a
Householder reflector zeroes its rows below j.  Ties go to the lowest column
index; a step whose chosen column has zero norm applies no reflector.  The
residual norms are recomputed exactly at every step (no norm downdating).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .leverage import leverage_exact
from .sketch import sketch_gcs


def qrcp_pivots(b, k=None):
    """First k pivots (column indices, in order) of the Businger-Golub
    column-pivoted Householder QR of b (m x d, m >= d), and the residual
    norm of each chosen column at the step it was chosen (|R[j, j]|)."""
    w = np.array(b, dtype=np.float64, copy=True)
    m, d = w.shape
    k = d if k is None else k
    live = np.ones(d, dtype=bool)
    piv = np.empty(k, dtype=np.int64)
    rdiag = np.empty(k)
    for j in range(k):
        norms2 = np.where(live, np.sum(w[j:, :] ** 2, axis=0), -1.0)
        p = int(np.argmax(norms2))          # first index of the maximum
        piv[j] = p
        live[p] = False
        x = w[j:, p].copy()
        nx = np.sqrt(norms2[p])
        rdiag[j] = nx
        if nx == 0.0:
            continue
        alpha = x[0]
        beta = -nx if alpha >= 0 else nx
        v = x
        v[0] = alpha - beta
        vtv = 2.0 * beta * (beta - alpha)
        cols = np.flatnonzero(live)
        proj = v @ w[j:, cols]
        w[j:, cols] -= np.outer(v, 2.0 * proj / vtv)
    return piv, rdiag


def qrcp_replay(b, piv):
    """The pivoted QR of b forced to take the columns piv in order: for each
    step, (squared residual norm of the column taken, largest squared
    residual norm among the remaining columns).  A pivot sequence is a valid
    outcome of the selection when the two agree at every step up to rounding."""
    w = np.array(b, dtype=np.float64, copy=True)
    m, d = w.shape
    live = np.ones(d, dtype=bool)
    took = np.empty(len(piv))
    best = np.empty(len(piv))
    for j, p in enumerate(piv):
        norms2 = np.sum(w[j:, :] ** 2, axis=0)
        took[j] = norms2[p]
        best[j] = norms2[live].max()
        live[p] = False
        nx = np.sqrt(norms2[p])
        if nx == 0.0:
            continue
        x = w[j:, p].copy()
        alpha = x[0]
        beta = -nx if alpha >= 0 else nx
        x[0] = alpha - beta
        vtv = 2.0 * beta * (beta - alpha)
        cols = np.flatnonzero(live)
        w[j:, cols] -= np.outer(x, 2.0 * (x @ w[j:, cols]) / vtv)
    return took, best


def qrcp_pivots_by_projection(b, k=None):
    """The same selection by its definition, for tiny inputs: at each step
    the column of b farthest from the span of the columns already chosen
    (residual of a least-squares projection), lowest index on ties."""
    b = np.asarray(b, dtype=np.float64)
    m, d = b.shape
    k = d if k is None else k
    chosen = []
    for _ in range(k):
        best, bestval = -1, -1.0
        for c in range(d):
            if c in chosen:
                continue
            if chosen:
                q = b[:, chosen]
                coef, *_ = np.linalg.lstsq(q, b[:, c], rcond=None)
                res = b[:, c] - q @ coef
            else:
                res = b[:, c]
            val = float(res @ res)
            if val > bestval:
                best, bestval = c, val
        chosen.append(best)
    return np.array(chosen, dtype=np.int64)


def css_select(a, m, r, k, seed):
    """Algorithm cgrrqr: the first k pivots of the pivoted QR of G S A
    (S A alone when m = 0)."""
    piv, _ = qrcp_pivots(sketch_gcs(a, m, r, seed), k)
    return piv


def leverage_css(a, m, r, k, seed):
    """Algorithm ls_hrn_exact: exact leverage scores of A[:, K] for the k
    columns K that css_select picks; returns (theta, K)."""
    cols = css_select(a, m, r, k, seed)
    sub = a[:, cols]
    if sp.issparse(sub):
        sub = sub.toarray()
    return leverage_exact(sub), cols
