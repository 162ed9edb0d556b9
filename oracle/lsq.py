"""Least squares min ||A x - b||, plain FP64.

Paper passages followed (arXiv 2203.02798): Algorithm
``least_squares_precondition`` (sketch-and-precondition): B = G S A, factor B,
N = the inverse factor, solve min_y ||A N y - b|| with a preconditioned
iterative method, return x = N y.  Algorithm ``least_squares_approx``
(sketch-and-solve): [A~ b~] = G S [A b], x = the least-squares solution of
A~ x = b~ (the SVD route, here LAPACK's least-squares solver).  Algorithm
``least_squares_gram`` computes the same x* as ``lstsq`` (from the Gram
matrix), so ``lstsq`` is its oracle.

Readings: the factor is the R of a QR of the sketch (N = R^{-1}); the
iterative method, which the paper leaves open, is LSQR (Paige & Saunders,
ACM TOMS 8(1), 1982), here SciPy's; one refinement pass solves the same
preconditioned problem for the residual and adds the correction.
Ground truth is LAPACK's least-squares solver.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.linalg import LinearOperator, lsqr

from .leverage import qr_r
from .sketch import sketch_gcs


def lstsq(a, b):
    """x* = argmin ||A x - b|| by LAPACK (dense copy for sparse A)."""
    if sp.issparse(a):
        a = a.toarray()
    x, *_ = np.linalg.lstsq(np.asarray(a, dtype=np.float64),
                            np.asarray(b, dtype=np.float64), rcond=None)
    return x


def lsq_sketch_solve(a, b, m, r, seed):
    """Sketch-and-solve (Algorithm ``least_squares_approx``): the sketch of A
    and the sketch of b with the same S and G (the same seed), then the
    least-squares solution of the small m x d problem."""
    c = sketch_gcs(a, m, r, seed)
    cb = sketch_gcs(np.asarray(b, dtype=np.float64)[:, None], m, r, seed)[:, 0]
    return lstsq(c, cb)


def _precond_op(a, rr):
    n, d = a.shape

    def mv(y):
        return a @ sla.solve_triangular(rr, y, lower=False)

    def rmv(u):
        return sla.solve_triangular(rr, a.T @ u, trans="T", lower=False)

    return LinearOperator((n, d), matvec=mv, rmatvec=rmv, dtype=np.float64)


def lsq_sketch_precond(a, b, m, r, seed, atol=1e-14, btol=1e-14,
                       iter_lim=300, refine=1):
    """Sketch-and-precondition least squares.  Returns (x, info) where info
    holds the LSQR iteration counts and the final residual norm."""
    if sp.issparse(a):
        a = sp.csr_matrix(a, dtype=np.float64)
    else:
        a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    rr = qr_r(sketch_gcs(a, m, r, seed))
    op = _precond_op(a, rr)
    y, istop, itn, *_ = lsqr(op, b, atol=atol, btol=btol, iter_lim=iter_lim)
    x = sla.solve_triangular(rr, y, lower=False)
    its = [int(itn)]
    for _ in range(refine):
        res = b - a @ x
        dy, _, itn2, *_ = lsqr(op, res, atol=atol, btol=btol, iter_lim=iter_lim)
        x = x + sla.solve_triangular(rr, dy, lower=False)
        its.append(int(itn2))
    res = b - a @ x
    return x, dict(iters=its, resid=float(np.linalg.norm(res)),
                   istop=int(istop), cond_precond=float(np.linalg.cond(rr)))


def lsq_quality(a, b, x):
    """(||r||, ||A^T r|| / (||A||_F ||r||)) for a candidate solution."""
    if sp.issparse(a):
        a = sp.csr_matrix(a, dtype=np.float64)
        fro = sp.linalg.norm(a)
    else:
        a = np.asarray(a, dtype=np.float64)
        fro = np.linalg.norm(a)
    res = np.asarray(b, dtype=np.float64) - a @ x
    rn = float(np.linalg.norm(res))
    return rn, float(np.linalg.norm(a.T @ res) / (fro * max(rn, 1e-300)))
