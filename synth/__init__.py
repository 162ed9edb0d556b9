"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws matrices and vectors; it holds none of the sketching,
Gram, row-norm or least-squares arithmetic.  Every generator is a pure
function of its arguments (NumPy ``default_rng(seed)``), so the CPU oracle and
the device path see byte-identical inputs.

CSR matrices are returned as ``scipy.sparse.csr_matrix`` with ``int64``
``indptr`` and ``int32`` ``indices`` (the layout the device library takes).

Workload recipes (the paper's own test matrices are random with unstated
distributions, Table ``tab:matrices``; these stand in for them):

* ``dense_gaussian``       -- iid N(0,1) entries.
* ``csr_uniform``          -- exactly round(density*n*d) distinct positions,
                              uniform over the n*d grid, values N(0,1).
* ``dense_coherent``       -- A = D U diag(s) V^T, geometric singular values,
                              a fraction of rows scaled up (high coherence).
* ``csr_zipf``             -- Zipf-distributed row lengths on a random subset
                              of rows (load imbalance), values N(0,1).
* ``lsq_problem``          -- A = X diag(s) V^T with a chosen condition
                              number, b = A x + noise.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = [
    "dense_gaussian",
    "dense_integer",
    "csr_uniform",
    "csr_integer",
    "csr_zipf",
    "dense_coherent",
    "lsq_problem",
    "serving_trace",
    "csr_from_parts",
]


def _rng(seed):
    return np.random.default_rng(seed)


def dense_gaussian(n, d, seed=0, dtype=np.float64):
    """n x d row-major matrix with iid N(0,1) entries."""
    return np.ascontiguousarray(_rng(seed).standard_normal((n, d)).astype(dtype))


def dense_integer(n, d, seed=0, lo=-8, hi=8, dtype=np.float64):
    """Integer-valued n x d matrix (exact in any float format)."""
    a = _rng(seed).integers(lo, hi + 1, size=(n, d)).astype(dtype)
    return np.ascontiguousarray(a)


def csr_from_parts(n, d, rows, cols, vals, dtype=np.float64):
    """Build a CSR matrix (int64 indptr, int32 indices) from COO triplets,
    keeping the given order of entries inside each row."""
    rows = np.asarray(rows, dtype=np.int64)
    order = np.argsort(rows, kind="stable")
    rows = rows[order]
    cols = np.asarray(cols, dtype=np.int32)[order]
    vals = np.asarray(vals)[order].astype(dtype)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    np.cumsum(indptr, out=indptr)
    m = sp.csr_matrix((vals, cols, indptr), shape=(n, d))
    m.indptr = indptr
    m.indices = cols
    return m


def csr_uniform(n, d, density, seed=0, dtype=np.float64):
    """Exactly ``round(density*n*d)`` distinct positions drawn uniformly from
    the n*d grid; values N(0,1).  Row lengths are then ~Poisson(density*d)."""
    rng = _rng(seed)
    total = n * d
    k = int(round(density * total))
    k = min(k, total)
    if k == 0:
        return csr_from_parts(n, d, [], [], [], dtype)
    if k > total // 4:
        pos = rng.choice(total, size=k, replace=False)
    else:
        pos = np.unique(rng.integers(0, total, size=int(k * 1.05) + 16))
        while pos.size < k:
            extra = rng.integers(0, total, size=k - pos.size + 16)
            pos = np.unique(np.concatenate([pos, extra]))
        pos = rng.permutation(pos)[:k]
    pos = np.sort(pos)
    rows = pos // d
    cols = pos % d
    vals = rng.standard_normal(k)
    return csr_from_parts(n, d, rows, cols, vals, dtype)


def csr_integer(n, d, density, seed=0, lo=-8, hi=8, dtype=np.float64,
                shuffle_within_rows=True):
    """Integer-valued CSR matrix; column order inside each row is shuffled
    (unsorted CSR is allowed by the library)."""
    base = csr_uniform(n, d, density, seed=seed, dtype=np.float64)
    rng = _rng(seed + 7919)
    vals = rng.integers(lo, hi + 1, size=base.nnz)
    vals[vals == 0] = 1
    cols = base.indices.copy()
    if shuffle_within_rows:
        for i in range(n):
            a, b = base.indptr[i], base.indptr[i + 1]
            if b - a > 1:
                cols[a:b] = cols[a:b][rng.permutation(b - a)]
    m = sp.csr_matrix((vals.astype(dtype), cols, base.indptr.copy()),
                      shape=(n, d))
    m.indptr = base.indptr.astype(np.int64)
    m.indices = cols.astype(np.int32)
    return m


def csr_zipf(n, d, density, zipf_a=1.5, seed=0, dtype=np.float32):
    """Zipf(``zipf_a``) row lengths truncated to [1, d] (values above d are
    redrawn), assigned to a uniformly random subset of rows until the total
    reaches ``round(density*n*d)`` (the last row is clipped); all other rows
    are empty.  Columns are distinct and uniform within a row; values N(0,1)."""
    rng = _rng(seed)
    target = int(round(density * n * d))
    lengths = []
    total = 0
    while total < target:
        batch = rng.zipf(zipf_a, size=max(1024, (target - total) // 8))
        bad = batch > d
        while bad.any():
            batch[bad] = rng.zipf(zipf_a, size=int(bad.sum()))
            bad = batch > d
        for L in batch:
            L = int(min(L, target - total))
            lengths.append(L)
            total += L
            if total >= target:
                break
    lengths = np.asarray(lengths, dtype=np.int64)
    if lengths.size > n:
        raise ValueError("csr_zipf: more non-empty rows than n")
    rows_sel = np.sort(rng.choice(n, size=lengths.size, replace=False))
    perm_len = rng.permutation(lengths)
    counts = np.zeros(n, dtype=np.int64)
    counts[rows_sel] = perm_len
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    nnz = int(indptr[-1])
    cols = np.empty(nnz, dtype=np.int32)
    pos = 0
    for L in perm_len:
        L = int(L)
        if L * 4 < d:
            c = np.unique(rng.integers(0, d, size=L + 8))
            while c.size < L:
                c = np.unique(np.concatenate([c, rng.integers(0, d, size=L)]))
            c = rng.permutation(c)[:L]
        else:
            c = rng.choice(d, size=L, replace=False)
        cols[pos:pos + L] = np.sort(c)
        pos += L
    vals = rng.standard_normal(nnz).astype(dtype)
    m = sp.csr_matrix((vals, cols, indptr), shape=(n, d))
    m.indptr = indptr
    m.indices = cols
    return m


def dense_coherent(n, d, seed=0, smin=1e-6, frac_scaled=0.05, scale=100.0,
                   dtype=np.float32, block=1 << 18):
    """A = D U diag(s) V^T: U the Q factor of an n x d Gaussian matrix, V the
    Q factor of a d x d Gaussian matrix, s geometric from 1 to ``smin``, D
    scaling ``floor(frac_scaled*n)`` uniformly chosen rows by ``scale``.

    U is formed as G R_g^{-1} with R_g from a Cholesky factor of G^T G
    accumulated over row blocks, so memory stays O(block*d + d^2) beyond A."""
    rng = _rng(seed)
    s = np.geomspace(1.0, smin, d)
    v, _ = np.linalg.qr(rng.standard_normal((d, d)))
    g_seed = int(rng.integers(0, 2**62))
    # pass 1: Gram of the Gaussian factor
    gram = np.zeros((d, d))
    for r0 in range(0, n, block):
        gb = np.random.default_rng([g_seed, r0]).standard_normal(
            (min(block, n - r0), d))
        gram += gb.T @ gb
    # two Cholesky-QR steps for an orthonormal U to working accuracy
    rg = np.linalg.cholesky(gram).T
    rg_inv = np.linalg.inv(rg)
    gram2 = np.zeros((d, d))
    for r0 in range(0, n, block):
        gb = np.random.default_rng([g_seed, r0]).standard_normal(
            (min(block, n - r0), d)) @ rg_inv
        gram2 += gb.T @ gb
    rg2_inv = np.linalg.inv(np.linalg.cholesky(gram2).T)
    core = rg_inv @ rg2_inv @ np.diag(s) @ v.T
    out = np.empty((n, d), dtype=dtype)
    for r0 in range(0, n, block):
        gb = np.random.default_rng([g_seed, r0]).standard_normal(
            (min(block, n - r0), d))
        out[r0:r0 + gb.shape[0]] = (gb @ core).astype(dtype)
    k = int(np.floor(frac_scaled * n))
    rows = rng.choice(n, size=k, replace=False)
    out[rows] *= dtype(scale) if isinstance(dtype, type) else scale
    return out


def lsq_problem(n, d, cond, seed=0, noise=1e-3, dtype=np.float64):
    """A = X diag(s) V^T with X = N(0,1)/sqrt(n) (n x d), V orthogonal,
    s geometric from 1 to 1/cond; x_true ~ N(0, I); b = A x_true + noise*N(0,I).
    Returns (A, b, x_true)."""
    rng = _rng(seed)
    x = rng.standard_normal((n, d)) / np.sqrt(n)
    v, _ = np.linalg.qr(rng.standard_normal((d, d)))
    s = np.geomspace(1.0, 1.0 / cond, d)
    a = np.ascontiguousarray((x * s) @ v.T).astype(dtype)
    x_true = rng.standard_normal(d)
    b = a.astype(np.float64) @ x_true + noise * rng.standard_normal(n)
    return a, b, x_true


def serving_trace(num, seed=0, n_lo=1e4, n_hi=1e6, dims=(32, 64, 128, 256),
                  cond_hi=1e8, rate=None):
    """Request descriptors for a least-squares serving trace: n log-uniform in
    [n_lo, n_hi], d uniform over ``dims``, condition number log-uniform in
    [1, cond_hi], Poisson arrivals at ``rate`` requests/s (None: all at t=0).
    Request k's matrix is drawn with seed ``seed*100003 + k``."""
    rng = _rng(seed)
    n = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=num)).astype(np.int64)
    d = rng.choice(np.asarray(dims), size=num)
    cond = np.exp(rng.uniform(0.0, np.log(cond_hi), size=num))
    if rate is None:
        t = np.zeros(num)
    else:
        t = np.cumsum(rng.exponential(1.0 / rate, size=num))
    return [dict(id=k, n=int(n[k]), d=int(d[k]), cond=float(cond[k]),
                 t_arrive=float(t[k]), seed=seed * 100003 + k)
            for k in range(num)]


def dense_coherent_torch(n, d, seed=0, smin=1e-6, frac_scaled=0.05, scale=100.0,
                         device="cuda:0"):
    """The coherent dense structure drawn on the device (torch), FP32:
    A = D Z diag(s) V^T with Z an n x d N(0, 1) matrix (not orthogonalised:
    its condition number is 1 + O(sqrt(d/n))), V the Q factor of a d x d
    Gaussian, s geometric from 1 to ``smin``, and D scaling
    ``floor(frac_scaled*n)`` uniformly chosen rows by ``scale``.  For the
    large configurations whose host generation would take minutes."""
    import torch
    g = torch.Generator(device=device).manual_seed(seed)
    v, _ = torch.linalg.qr(torch.randn(d, d, generator=g, device=device, dtype=torch.float64))
    sv = torch.logspace(0.0, float(np.log10(smin)), d, dtype=torch.float64, device=device)
    w = (sv[:, None] * v.T).to(torch.float32)
    a = torch.randn(n, d, generator=g, device=device, dtype=torch.float32) @ w
    hot = torch.randperm(n, generator=g, device=device)[: int(np.floor(frac_scaled * n))]
    a[hot] *= scale
    return a


def lsq_trace_torch(num, seed, n_lo, n_hi, d_choices=(32, 64, 128, 256), cond_hi=1e8,
                    noise=1e-3, device="cuda:0"):
    """Least-squares requests drawn on the device: n log-uniform in [n_lo,
    n_hi], d uniform over d_choices, condition number log-uniform in
    [1, cond_hi]; A = X diag(s) V^T with X ~ N(0,1)/sqrt(n), V the Q factor of
    a Gaussian, s geometric from 1 to 1/cond; b = A x + noise * e.  Request
    k is seeded by (seed, k)."""
    import torch
    rng = _rng(seed)
    reqs = []
    for k in range(num):
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        d = int(rng.choice(list(d_choices)))
        cond = float(np.exp(rng.uniform(0.0, np.log(cond_hi))))
        g = torch.Generator(device=device)
        g.manual_seed(seed * 100003 + k)
        x = torch.randn(n, d, generator=g, device=device, dtype=torch.float64) / n ** 0.5
        v, _ = torch.linalg.qr(torch.randn(d, d, generator=g, device=device,
                                           dtype=torch.float64))
        sv = torch.logspace(0.0, -np.log10(cond), d, device=device, dtype=torch.float64)
        a = ((x * sv) @ v.T).contiguous()
        del x
        xt = torch.randn(d, generator=g, device=device, dtype=torch.float64)
        b = a @ xt + noise * torch.randn(n, generator=g, device=device, dtype=torch.float64)
        reqs.append(dict(a=a, b=b, n=n, d=d, cond=cond, seed=k))
    return reqs
