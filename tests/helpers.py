"""Shared helpers of the GPU parity tests: device placement of synthetic
inputs and the error bounds the comparisons use."""
import numpy as np
import scipy.sparse as sp

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def gamma(k, u):
    """gamma_k = k u / (1 - k u) (Higham's constant for k roundings)."""
    ku = k * u
    return ku / (1.0 - ku)


def to_device(a, dtype=None):
    """NumPy dense or SciPy CSR -> torch device tensor / CsrMatrix."""
    import torch
    from paper_2203_02798_amd.api import CsrMatrix
    if sp.issparse(a):
        return CsrMatrix.from_scipy(a, device="cuda")
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return t if dtype is None else t.to(dtype)


def abs_of(a):
    return abs(a) if sp.issparse(a) else np.abs(a)


def sketch_abs_bound(a, r, seed, u):
    """Componentwise bound gamma_k (|S| |A|) of the rounding error of S*A,
    k = the largest bucket occupancy (terms summed per output entry)."""
    from oracle import sketch as osk
    n = a.shape[0]
    h, _ = osk.cs_hash(n, r, seed)
    k = int(np.bincount(h, minlength=r).max())
    s_abs = sp.csr_matrix((np.ones(n), (h, np.arange(n))), shape=(r, n))
    mag = s_abs @ abs_of(sp.csr_matrix(a, dtype=np.float64) if sp.issparse(a)
                         else np.asarray(a, dtype=np.float64))
    if sp.issparse(mag):
        mag = mag.toarray()
    return gamma(max(k, 1), u) * np.asarray(mag)


def rel_fro(x, ref):
    den = np.linalg.norm(ref)
    return np.linalg.norm(x - ref) / (den if den > 0 else 1.0)
