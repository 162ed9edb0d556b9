"""Gram matrix and squared row norms of a product, plain FP64.

Paper passages followed (arXiv 2203.02798):

* ``csrrk`` (section "Software") and Algorithm ``gram``:
  B <- alpha * A^T A + beta * B, B a dense row-major d x d array (both
  triangles are written).
* Algorithm ``gram_serial``: the outer-product loop over the non-zeros of each
  CSR row, B[J_k, J_j] += V_k * V_j.
* ``csrsqn``/``rmsqn`` and Algorithm ``squared_row_norms``:
  x <- alpha * q + beta * x with q_i = ||e_i^T A B||^2; the CSR form first
  builds Bt = B B^T and then, per row, sums V_k * V_j * Bt[J_j, J_k] over all
  pairs of non-zeros of that row.

Reading: when beta == 0 the previous contents of B (or x) are ignored rather
than multiplied (so NaN in uninitialised output does not propagate), the
usual BLAS convention; the paper does not say.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _f64(a):
    if sp.issparse(a):
        return sp.csr_matrix(a, dtype=np.float64)
    return np.asarray(a, dtype=np.float64)


def gram(alpha, a, beta=0.0, c=None):
    """alpha * A^T A + beta * C (dense d x d result)."""
    a = _f64(a)
    g = a.T @ a
    if sp.issparse(g):
        g = g.toarray()
    out = alpha * np.asarray(g)
    if beta != 0.0:
        out = out + beta * np.asarray(c, dtype=np.float64)
    return out


def gram_csr_literal(a):
    """A^T A by the serial outer-product loop of Algorithm ``gram_serial``
    (tiny inputs only)."""
    a = sp.csr_matrix(a, dtype=np.float64)
    d = a.shape[1]
    b = np.zeros((d, d))
    for i in range(a.shape[0]):
        lo, hi = a.indptr[i], a.indptr[i + 1]
        for k in range(lo, hi):
            for j in range(lo, hi):
                b[a.indices[k], a.indices[j]] += a.data[k] * a.data[j]
    return b


def rownorms_sq(alpha, a, bmat, beta=0.0, x=None):
    """alpha * ||e_i^T A B||^2 + beta * x_i for every row i of A."""
    a = _f64(a)
    bmat = np.asarray(bmat, dtype=np.float64)
    ab = a @ bmat
    if sp.issparse(ab):
        ab = ab.toarray()
    q = np.einsum("ij,ij->i", ab, ab)
    out = alpha * q
    if beta != 0.0:
        out = out + beta * np.asarray(x, dtype=np.float64)
    return out


def rownorms_sq_csr_literal(alpha, a, bmat):
    """The per-row pair loop of Algorithm ``squared_row_norms`` with
    Bt = B B^T (tiny inputs only); beta = 0."""
    a = sp.csr_matrix(a, dtype=np.float64)
    bmat = np.asarray(bmat, dtype=np.float64)
    bt = bmat @ bmat.T
    n = a.shape[0]
    x = np.zeros(n)
    for i in range(n):
        lo, hi = a.indptr[i], a.indptr[i + 1]
        acc = 0.0
        for k in range(lo, hi):
            gamma = alpha * a.data[k]
            for j in range(lo, hi):
                acc += gamma * a.data[j] * bt[a.indices[j], a.indices[k]]
        x[i] = acc
    return x


def rownorm_bound_terms(a, bmat):
    """z_i = sum_j (sum_k |a_ik| |B_kj|)^2: the magnitude a forward-error
    bound of the row norms scales with."""
    a = _f64(a)
    aa = abs(a)
    ab = aa @ np.abs(np.asarray(bmat, dtype=np.float64))
    if sp.issparse(ab):
        ab = ab.toarray()
    return np.einsum("ij,ij->i", ab, ab)
