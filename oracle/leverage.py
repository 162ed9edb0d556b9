"""QR of a sketch, its triangular inverse, and leverage scores, plain FP64.

Paper passages followed (arXiv 2203.02798):

* Algorithm ``ls_approximate_drineas``: sketch A, factor the sketch, and take
  squared row norms of A times the inverse factor (Algorithm
  ``squared_row_norms``).  The paper factors with an SVD (V Sigma^{-1}); here
  the factor is the R of a QR of the sketch, which spans the same
  orthogonaliser: A R^{-1} and A V Sigma^{-1} differ by an orthogonal d x d
  matrix, so the row norms agree.
* Algorithm ``ls_approximate_drineas`` with its Johnson-Lindenstrauss step:
  X = R^{-1} Pi for a d x t Gaussian Pi scaled to variance 1/t, and
  theta~_i = ||e_i^T A X||^2, which preserves each row norm of A R^{-1} up to
  a factor 1 +- eps when t = O(log n / eps^2).  The sketch is S A alone in
  the algorithm (m = 0 here) or G S A (m > 0).
* Algorithm ``ls_direct``: exact leverage scores theta_i = ||e_i^T U||^2 for an
  orthonormal basis U of range(A) (computed here from a thin QR of A).
* The perturbation of a sketch, delta = ||(C^ - C) R^{-1}||_2 for a sketch C^
  that stands in for C = G S A (a reduced-precision one, say) and R from a QR
  of C.  It measures C^ in the metric in which C is orthonormal, the one of
  Definition 2's embedding bound: with C^ R^{-1} = Q + F, ||F||_2 = delta,
  the singular values of R^ R^{-1} lie in [1 - delta, 1 + delta], so the scores
  of Algorithm ``ls_approximate_drineas`` from C^ and from C satisfy
  (1 + delta)^-2 <= theta^_i / theta~_i <= (1 - delta)^-2 (delta < 1), and
  the preconditioner of Algorithm ``least_squares_precondition`` built from
  C^ keeps cond(A R^^{-1}) within a factor (1 + delta) / (1 - delta) of the
  one built from C.

Readings: full column rank is assumed (the paper's "truncate if needed" is
not applied); R is normalised to a non-negative diagonal.  Pi is drawn by the
generator of G (``oracle.sketch``) on stream 2: Pi[b, j] = Z[j, b] / sqrt(t)
with Z the normals of a t-row Gaussian whose columns are indexed by
b = 0 .. d-1, so Pi^T is that t x d Gaussian.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .gram import rownorms_sq
from .sketch import gaussian_normals, sketch_gcs


def qr_r(c):
    """Upper-triangular R of C = Q R (LAPACK Householder QR), rows scaled so
    that diag(R) >= 0."""
    c = np.asarray(c, dtype=np.float64)
    r = np.linalg.qr(c, mode="r")
    r = np.triu(r[: c.shape[1], :])
    sgn = np.where(np.diag(r) < 0, -1.0, 1.0)
    return r * sgn[:, None]


def tri_inv(r):
    """R^{-1} for an upper-triangular R (triangular solve against I)."""
    d = r.shape[0]
    return sla.solve_triangular(r, np.eye(d), lower=False)


def leverage_sketched(a, m, r, seed):
    """theta~_i = ||e_i^T A R^{-1}||^2 with R from QR(G S A)."""
    c = sketch_gcs(a, m, r, seed)
    rr = qr_r(c)
    return rownorms_sq(1.0, a, tri_inv(rr)), rr


def jl_matrix(d, t, seed):
    """Pi (d x t): the scaled Gaussian of the JL step, entries of variance 1/t."""
    return gaussian_normals(t, 0, d, seed, stream=2).T / np.sqrt(t)


def leverage_from_sketch(a, c, t, seed):
    """theta~_i = ||e_i^T A X||^2 with X = R^{-1} (t = 0) or X = R^{-1} Pi
    (t > 0), R from QR(c) for the sketch c of A."""
    x = tri_inv(qr_r(c))
    if t > 0:
        x = x @ jl_matrix(x.shape[0], t, seed)
    return rownorms_sq(1.0, a, x)


def leverage_sketched_jl(a, m, r, t, seed):
    """Algorithm ``ls_approximate_drineas`` with the JL step: sketch
    (S A for m = 0, else G S A), factor, X = R^{-1} Pi, row norms of A X."""
    return leverage_from_sketch(a, sketch_gcs(a, m, r, seed), t, seed)


def leverage_sketched_svd(a, m, r, seed):
    """Same quantity by the paper's SVD route: ||e_i^T A V Sigma^{-1}||^2."""
    c = sketch_gcs(a, m, r, seed)
    _, s, vt = np.linalg.svd(c, full_matrices=False)
    return rownorms_sq(1.0, a, vt.T / s[None, :])


def leverage_exact(a):
    """Exact leverage scores from a thin QR of A (dense copy for sparse A)."""
    if sp.issparse(a):
        a = a.toarray()
    q, _ = np.linalg.qr(np.asarray(a, dtype=np.float64), mode="reduced")
    return np.einsum("ij,ij->i", q, q)


def sketch_perturbation(c_hat, c):
    """delta = ||(C^ - C) R^{-1}||_2 with R from QR(C) (both m x d, C of full
    column rank): the relative perturbation of the sketch C^ against C in
    the metric in which C is orthonormal.  Computed exactly: the triangular
    solve F^T = R^{-T} (C^ - C)^T, then the largest singular value of F."""
    c_hat = np.asarray(c_hat, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    r = qr_r(c)
    f = sla.solve_triangular(r, (c_hat - c).T, trans="T", lower=False).T
    return float(np.linalg.norm(f, 2))


def leverage_ratio_bound(delta):
    """Largest |theta^_i / theta~_i - 1| a sketch perturbation delta < 1 allows:
    (1 - delta)^-2 - 1 (the upper edge; the lower one, 1 - (1 + delta)^-2, is
    smaller)."""
    return (1.0 - delta) ** -2 - 1.0


def sketch_distortion(a, m, r, seed):
    """Singular values of G S U for an orthonormal basis U of range(A); the
    subspace-embedding distortion is max |sigma - 1|."""
    if sp.issparse(a):
        a = a.toarray()
    q, _ = np.linalg.qr(np.asarray(a, dtype=np.float64), mode="reduced")
    return np.linalg.svd(sketch_gcs(q, m, r, seed), compute_uv=False)
