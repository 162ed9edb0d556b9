"""OSNAP sketches with s > 1 non-zeros per column, plain FP64.

TEST INFRASTRUCTURE: only tests/, the smoke check and the benchmark's CPU
baseline use this module; the library never does.

Paper passages followed (arXiv 2203.02798):

* Section 2's introduction and the related-work footnote: CountSketch is the
  OSNAP of Nelson and Nguyen with s = 1 non-zero per column, and the paper's
  data structures and products carry over to any OSNAP.
* Definition 3 (CountSketch) for the s = 1 case; Algorithm ``bcs_multiply``
  for S*A and Algorithm ``countgauss_multiply`` for G*(S*A), unchanged but
  for the sketch S.

Reading (the paper fixes no OSNAP construction): the block construction of
the OSNAP distribution.  The r rows are split into s blocks of r/s
consecutive rows (s must divide r); column i of S has exactly one non-zero
in each block, so its s non-zeros sit in s distinct rows, each equal to
sigma / sqrt(s) with an independent sign.  The k-th non-zero of column i
(k = 0 .. s-1) is drawn like the CountSketch hash with the non-zero's index
in counter word 2:
    x = Philox4x32-10(counter=(i mod 2^32, i div 2^32, k, 0), key as the hash),
    row = k * (r/s) + floor((x1*2^32 + x0) * (r/s) / 2^64),
    sign = +1 if x2 is even, else -1.
For s = 1 this is the CountSketch hash of ``oracle.sketch`` exactly.
Every column of S has unit norm, so E[S^T S] = I and E||S x||^2 = ||x||^2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .philox import philox4x32, seed_key
from .sketch import gaussian_block


def _check(r, s):
    if s < 1 or r < 1 or r % s != 0:
        raise ValueError("OSNAP needs s >= 1 dividing r")
    if r >= 2 ** 32:
        raise ValueError("r must be < 2^32")


def osnap_hash(n, r, s, seed, row0=0):
    """Rows h[i, k] and signs sigma[i, k] of the s non-zeros of columns
    row0 .. row0+n-1.  Returns (h int64 (n, s), sigma int8 (n, s))."""
    _check(r, s)
    rb = np.uint64(r // s)
    i = np.arange(row0, row0 + n, dtype=np.uint64)
    h = np.empty((n, s), dtype=np.int64)
    sg = np.empty((n, s), dtype=np.int8)
    for k in range(s):
        ctr = np.zeros((n, 4), dtype=np.uint64)
        ctr[:, 0] = i & np.uint64(0xFFFFFFFF)
        ctr[:, 1] = i >> np.uint64(32)
        ctr[:, 2] = k
        x = philox4x32(ctr, seed_key(seed)).astype(np.uint64)
        # floor((x1*2^32 + x0) * rb / 2^64), all partial terms below 2^64
        off = (x[:, 1] * rb + ((x[:, 0] * rb) >> np.uint64(32))) >> np.uint64(32)
        h[:, k] = k * (r // s) + off.astype(np.int64)
        sg[:, k] = np.where((x[:, 2] & np.uint64(1)) == 0, 1, -1)
    return h, sg


def osnap_hash_bigint(i, r, s, seed):
    """The same rows and signs of column i with Python integers (exact
    128-bit products), for spot checks."""
    _check(r, s)
    rb = r // s
    out = []
    for k in range(s):
        ctr = np.array([[i & 0xFFFFFFFF, i >> 32, k, 0]], dtype=np.uint64)
        x = [int(v) for v in philox4x32(ctr, seed_key(seed))[0]]
        out.append((k * rb + (((x[1] << 32 | x[0]) * rb) >> 64), 1 if x[2] % 2 == 0 else -1))
    return out


def osnap_sparse(n, r, s, seed):
    """S as a SciPy CSR matrix (r x n, exactly n*s non-zeros of +-1/sqrt(s))."""
    h, sg = osnap_hash(n, r, s, seed)
    cols = np.repeat(np.arange(n), s)
    vals = sg.ravel().astype(np.float64) / np.sqrt(s)
    return sp.csr_matrix((vals, (h.ravel(), cols)), shape=(r, n))


def osnap_dense(n, r, s, seed):
    """Explicit dense S (r x n), written entry by entry; tiny inputs only."""
    h, sg = osnap_hash(n, r, s, seed)
    out = np.zeros((r, n))
    for i in range(n):
        for k in range(s):
            out[h[i, k], i] = sg[i, k] / np.sqrt(s)
    return out


def sketch_osnap(a, r, s, seed):
    """S*A in FP64 for the OSNAP S (Algorithm ``bcs_multiply`` with this S);
    dense r x d result."""
    a = sp.csr_matrix(a, dtype=np.float64) if sp.issparse(a) else np.asarray(a, np.float64)
    out = osnap_sparse(a.shape[0], r, s, seed) @ a
    if sp.issparse(out):
        out = out.toarray()
    return np.ascontiguousarray(out)


def sketch_gosnap(a, m, r, s, seed, batch=4096):
    """C = G*(S*A) with the OSNAP S (Algorithm ``countgauss_multiply``): S*A
    once, then C over bucket batches with the same G as the CountSketch
    form (G depends only on m, r and the seed).  m = 0 returns S*A."""
    sa = sketch_osnap(a, r, s, seed)
    if m == 0:
        return sa
    c = np.zeros((m, sa.shape[1]))
    for b0 in range(0, r, batch):
        b1 = min(r, b0 + batch)
        c += gaussian_block(m, b0, b1, seed) @ sa[b0:b1]
    return c
