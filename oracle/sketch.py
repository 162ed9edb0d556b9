"""CountSketch, Gaussian and combined (CountGauss) sketches in plain FP64.

Paper passages followed (arXiv 2203.02798):

* Definition 3 (CountSketch): S in R^{r x n} has, for every column i, the
  single non-zero S[h(i), i] = sigma_i; h and sigma are treated as fully
  independent and uniform.
* Figure ``countsketch_vector_example``: the signed vector representation,
  v_k = +-|row|, with S[|v_k|, k] = sign(v_k) (1-based rows).
* Algorithm ``bcs_multiply``: S*A stored as a dense row-major r x d array.
* Algorithm ``countgauss_multiply``: G*S*A computed in batches of buckets; a
  batch forms B = S_i*A, draws a fresh Gaussian block G_i and accumulates
  C += G_i*B.  ``csrcgs``/``rmcgs`` (section "Software") scale G by 1/sqrt(m)
  and return S*A when m = 0.
* Algorithm ``gaussian_sketch`` (section "Gaussian sketching"; ``csrjlt``):
  C = G*A for an m x n Gaussian G, each row k of A scaled by its own fresh
  column of normals and added into C.

Readings where the paper leaves the choice open (it uses per-thread STL
engines, so its streams are not reproducible across thread counts):

* hash: x = Philox4x32-10(counter=(i mod 2^32, i div 2^32, 0, 0),
  key=(seed mod 2^32, seed div 2^32)); h(i) = floor((x1*2^32 + x0) * r / 2^64)
  (a 64-bit multiply-high range reduction, bias at most r/2^64);
  sigma_i = +1 if x2 is even, else -1.
* Gaussian: for bucket column b (for G*A: row b of A) and row a of G,
  q = b div 4 and
  x = Philox4x32-10(counter=(q mod 2^32, q div 2^32, a, 1), key as above);
  u_k = (x_k + 1/2) * 2^-32 lies in (0, 1); Box-Muller gives
  z0, z1 = sqrt(-2 ln u0) * (cos, sin)(2 pi u1) and
  z2, z3 = sqrt(-2 ln u2) * (cos, sin)(2 pi u3);  G[a, b] = z_{b mod 4} / sqrt(m)
  (variance 1/m, i.e. N(0, 1/sqrt(m)) in the paper's (mean, std) notation).
  Counter word 3 names the stream: 0 for the hash, 1 for G, 2 for the JL
  matrix of the leverage-score estimate (see ``oracle.leverage``).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .philox import philox4x32, seed_key

TWO_M32 = 2.0 ** -32


# ----------------------------------------------------------------------------
# CountSketch hash (Definition 3)
# ----------------------------------------------------------------------------
def cs_hash(n, r, seed, row0=0):
    """Bucket h[i] in [0, r) and sign sigma[i] in {+1, -1} for rows
    row0 .. row0+n-1.  Returns (h int64, sigma int8)."""
    if r < 1 or r >= 2 ** 32:
        raise ValueError("r must be in [1, 2^32)")
    i = np.arange(row0, row0 + n, dtype=np.uint64)
    ctr = np.zeros((n, 4), dtype=np.uint64)
    ctr[:, 0] = i & np.uint64(0xFFFFFFFF)
    ctr[:, 1] = i >> np.uint64(32)
    x = philox4x32(ctr, seed_key(seed)).astype(np.uint64)
    # floor((x1*2^32 + x0) * r / 2^64) without 128-bit integers:
    # = (x1*r + floor(x0*r / 2^32)) div 2^32, all terms below 2^64 for r < 2^32.
    rr = np.uint64(r)
    h = (x[:, 1] * rr + ((x[:, 0] * rr) >> np.uint64(32))) >> np.uint64(32)
    sigma = np.where((x[:, 2] & np.uint64(1)) == 0, 1, -1).astype(np.int8)
    return h.astype(np.int64), sigma


def cs_hash_bigint(i, r, seed):
    """Same hash for one row with Python integers (exact 128-bit product)."""
    ctr = np.array([[i & 0xFFFFFFFF, i >> 32, 0, 0]], dtype=np.uint64)
    x = [int(v) for v in philox4x32(ctr, seed_key(seed))[0]]
    h = ((x[1] << 32 | x[0]) * r) >> 64
    return h, (1 if x[2] % 2 == 0 else -1)


def vector_representation(h, sigma):
    """Signed 1-based vector v with S[|v_k|-1, k] = sign(v_k)."""
    return (np.asarray(h, dtype=np.int64) + 1) * np.asarray(sigma, np.int64)


def dense_from_vector(v, r):
    """Explicit r x n CountSketch from its vector representation."""
    v = np.asarray(v, dtype=np.int64)
    s = np.zeros((r, v.size))
    for k, vk in enumerate(v):
        s[abs(vk) - 1, k] = 1.0 if vk > 0 else -1.0
    return s


def countsketch_dense(n, r, seed):
    """Explicit dense S (r x n); for tiny inputs only."""
    h, sg = cs_hash(n, r, seed)
    s = np.zeros((r, n))
    s[h, np.arange(n)] = sg
    return s


def countsketch_sparse(n, r, seed):
    """S as a SciPy CSR matrix (r x n, exactly n non-zeros)."""
    h, sg = cs_hash(n, r, seed)
    return sp.csr_matrix((sg.astype(np.float64), (h, np.arange(n))),
                         shape=(r, n))


def _as_f64(a):
    if sp.issparse(a):
        return sp.csr_matrix(a, dtype=np.float64)
    return np.asarray(a, dtype=np.float64)


def sketch_cs(a, r, seed):
    """S*A in FP64 (Algorithm ``bcs_multiply``); dense r x d result."""
    a = _as_f64(a)
    n = a.shape[0]
    s = countsketch_sparse(n, r, seed)
    out = s @ a
    if sp.issparse(out):
        out = out.toarray()
    return np.ascontiguousarray(out)


def bucket_occupancy(n, r, seed):
    """Rows per bucket (the length of each bucket's row list)."""
    h, _ = cs_hash(n, r, seed)
    return np.bincount(h, minlength=r)


# ----------------------------------------------------------------------------
# Gaussian matrix (generated in column blocks, never whole)
# ----------------------------------------------------------------------------
def gaussian_normals(m, b0, b1, seed, stream=1, a0=0):
    """Unscaled standard normals Z[a, b] for rows a0 <= a < a0 + m, buckets
    b0 <= b < b1 (counter word 3 = stream)."""
    if b1 <= b0 or m == 0:
        return np.zeros((m, max(b1 - b0, 0)))
    q0, q1 = b0 // 4, (b1 + 3) // 4
    q = np.arange(q0, q1, dtype=np.uint64)
    a = np.arange(a0, a0 + m, dtype=np.uint64)
    ctr = np.zeros((m, q.size, 4), dtype=np.uint64)
    ctr[:, :, 0] = (q & np.uint64(0xFFFFFFFF))[None, :]
    ctr[:, :, 1] = (q >> np.uint64(32))[None, :]
    ctr[:, :, 2] = a[:, None]
    ctr[:, :, 3] = stream
    x = philox4x32(ctr, seed_key(seed)).astype(np.float64)
    u = (x + 0.5) * TWO_M32
    rho0 = np.sqrt(-2.0 * np.log(u[..., 0]))
    rho2 = np.sqrt(-2.0 * np.log(u[..., 2]))
    z = np.empty((m, q.size, 4))
    z[..., 0] = rho0 * np.cos(2.0 * np.pi * u[..., 1])
    z[..., 1] = rho0 * np.sin(2.0 * np.pi * u[..., 1])
    z[..., 2] = rho2 * np.cos(2.0 * np.pi * u[..., 3])
    z[..., 3] = rho2 * np.sin(2.0 * np.pi * u[..., 3])
    z = z.reshape(m, q.size * 4)
    return z[:, b0 - 4 * q0: b1 - 4 * q0]


def gaussian_block(m, b0, b1, seed):
    """Scaled Gaussian block G[:, b0:b1] = Z / sqrt(m)."""
    return gaussian_normals(m, b0, b1, seed) / np.sqrt(m)


def sketch_g(a, m, seed, batch=4096):
    """C = G*A, G the m x n Gaussian with entries of variance 1/m (Algorithm
    ``gaussian_sketch``): column i of G, the normals drawn for row i of A,
    is the one the combined sketch draws for bucket i, so G*A is the
    combined sketch with S the identity.  Rows of A in batches."""
    a = _as_f64(a)
    n, d = a.shape
    c = np.zeros((m, d))
    for b0 in range(0, n, batch):
        b1 = min(n, b0 + batch)
        blk = a[b0:b1]
        if sp.issparse(blk):
            c += np.asarray((blk.T @ gaussian_block(m, b0, b1, seed).T).T)
        else:
            c += gaussian_block(m, b0, b1, seed) @ blk
    return c


def sketch_g_literal(a, m, seed):
    """Algorithm ``gaussian_sketch`` as written, for tiny CSR inputs: for each
    row k draw its m normals g, then for each stored entry (k, j, v) add
    g * v to column j of C (one processor, so the block of rows of G is all
    of it).  Duplicated entries of a row are added one after another."""
    a = sp.csr_matrix(a, dtype=np.float64)
    n, d = a.shape
    c = np.zeros((m, d))
    for k in range(n):
        g = gaussian_normals(m, k, k + 1, seed)[:, 0] / np.sqrt(m)
        for h in range(a.indptr[k], a.indptr[k + 1]):
            j = a.indices[h]
            for i in range(m):
                c[i, j] += g[i] * a.data[h]
    return c


def sketch_gcs(a, m, r, seed, batch=4096):
    """C = G*(S*A) (Algorithm ``countgauss_multiply``): S*A formed once, then
    C accumulated over bucket batches with a fresh block of G each.
    m = 0 returns S*A."""
    sa = sketch_cs(a, r, seed)
    if m == 0:
        return sa
    c = np.zeros((m, sa.shape[1]))
    for b0 in range(0, r, batch):
        b1 = min(r, b0 + batch)
        c += gaussian_block(m, b0, b1, seed) @ sa[b0:b1]
    return c


# ----------------------------------------------------------------------------
# Reduced-precision operand formats (for the BF16 / FP8 Gaussian GEMM)
# ----------------------------------------------------------------------------
def round_to_bits(x, mant_bits, emin, emax_val=None):
    """Round-to-nearest-even of FP64 values onto a binary format with
    ``mant_bits`` fraction bits and minimum normal exponent ``emin``
    (subnormals below it).  Values beyond ``emax_val`` saturate to it."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    # exact binary exponent: ax = f * 2^fe with f in [1/2, 1)
    _, fe = np.frexp(ax)
    e = np.where(ax > 0, fe - 1, 0).astype(np.float64)
    e = np.maximum(e, emin)
    quantum = np.ldexp(1.0, (e - mant_bits).astype(np.int64))
    y = np.round(x / quantum) * quantum  # np.round: half to even
    if emax_val is not None:
        y = np.clip(y, -emax_val, emax_val)
    return y


def to_bf16(x):
    """Round FP64 to bfloat16 (8-bit exponent, 7 fraction bits), RNE."""
    return round_to_bits(x, 7, -126)


def to_e4m3(x):
    """Round FP64 to OCP FP8 e4m3fn (bias 7, 3 fraction bits, max 448),
    RNE with saturation."""
    return round_to_bits(x, 3, -6, 448.0)


def bf16_limbs(x, nlimbs=2):
    """Split x into ``nlimbs`` bfloat16 limbs: l0 = bf16(x),
    l1 = bf16(x - l0), ...  (Ozaki-style error-free splitting up to the last
    limb's rounding)."""
    x = np.asarray(x, dtype=np.float64)
    limbs = []
    rest = x.copy()
    for _ in range(nlimbs):
        l = to_bf16(rest)
        limbs.append(l)
        rest = rest - l
    return limbs


def gauss_product_bf16_reference(b, m, seed, nlimbs=2, batch=4096):
    """G*B with G's unscaled normals rounded to bfloat16 and B (r x d, the
    operand: S*A or A) as its bfloat16 limbs, the product exact in FP64,
    then scaled by 1/sqrt(m)."""
    b = np.asarray(b, dtype=np.float64)
    r = b.shape[0]
    bq = np.sum(bf16_limbs(b, nlimbs), axis=0)
    c = np.zeros((m, b.shape[1]))
    for b0 in range(0, r, batch):
        b1 = min(r, b0 + batch)
        zq = to_bf16(gaussian_normals(m, b0, b1, seed))
        c += zq @ bq[b0:b1]
    return c / np.sqrt(m)


def sketch_gcs_bf16_reference(a, m, r, seed, nlimbs=2, batch=4096):
    """Quantisation-aware reference of the BF16 Gaussian GEMM: the exact (FP64)
    product of the BF16-rounded unscaled normals with the BF16 limb
    decomposition of S*A, then scaled by 1/sqrt(m).  Comparing the device
    result with this isolates the kernel's arithmetic from the format loss."""
    return gauss_product_bf16_reference(sketch_cs(a, r, seed), m, seed, nlimbs, batch)


def sketch_g_bf16_reference(a, m, seed, nlimbs=2, batch=4096):
    """The same for G*A (the operand is A itself)."""
    a = _as_f64(a)
    return gauss_product_bf16_reference(a.toarray() if sp.issparse(a) else a, m, seed,
                                        nlimbs, batch)


# ----------------------------------------------------------------------------
# FP8 e4m3 with power-of-two block scales (reading of the per-128 scales)
# ----------------------------------------------------------------------------
E4M3_MAX = 448.0


def e8m0_exponent(amax):
    """Exponent e of the power-of-two scale 2^e of a block whose largest
    magnitude is amax: the smallest integer with 448 * 2^e >= amax, i.e.
    ceil(log2(amax / 448)), taken exactly from the binary exponent of amax
    (amax = f 2^x, f in [1/2, 1); 448 = 0.875 2^9).  0 for an all-zero block."""
    amax = np.asarray(amax, dtype=np.float64)
    f, x = np.frexp(amax)
    e = np.where(f <= 0.875, x - 9, x - 8)
    return np.where(amax > 0, e, 0).astype(np.int64)


def quantize_e4m3_blocks(x, block=128, axis=0):
    """Blocks of `block` consecutive entries along `axis` (starting at index
    0; the last may be shorter) share one scale 2^e with e = e8m0_exponent of
    the block's largest magnitude; each entry becomes 2^e * e4m3(x / 2^e)
    (RNE, |x / 2^e| <= 448 by construction).  Returns (dequantised x, e)
    with e of shape (blocks, other axis)."""
    x = np.asarray(x, dtype=np.float64)
    xt = np.moveaxis(x, axis, 0)
    n = xt.shape[0]
    nb = (n + block - 1) // block
    out = np.empty_like(xt)
    exps = np.empty((nb,) + xt.shape[1:], dtype=np.int64)
    for b in range(nb):
        sl = xt[b * block:(b + 1) * block]
        e = e8m0_exponent(np.max(np.abs(sl), axis=0))
        s = np.ldexp(1.0, e)
        out[b * block:(b + 1) * block] = to_e4m3(sl / s) * s
        exps[b] = e
    return np.moveaxis(out, 0, axis), exps


# The unscaled normals of this generator are bounded: u >= 2^-33 gives
# |z| <= sqrt(-2 ln 2^-33) = sqrt(66 ln 2) < 6.77, so the power-of-two scale
# 2^G_FP8_EXP with 448 * 2^G_FP8_EXP >= 6.77 covers every block of G; with
# it the e4m3 rounding of G never saturates, and for every value in the
# normal e4m3 range (|z| >= 2^-12) it equals the rounding under the block's
# own amax scale (a power-of-two scale does not move the significand).
G_FP8_EXP = -6


def quantize_gaussian_e4m3(z):
    """The FP8 operand of G: 2^G_FP8_EXP * e4m3(z / 2^G_FP8_EXP), one fixed
    E8M0 scale for every 128-bucket block of every row."""
    s = np.ldexp(1.0, G_FP8_EXP)
    return to_e4m3(np.asarray(z, dtype=np.float64) / s) * s


def gauss_product_fp8_reference(b, m, seed, block=128, batch=4096):
    """G*B with B (r x d: S*A or A) quantised per column in blocks of `block`
    rows (scale from each block's amax), the unscaled normals quantised with
    G's fixed scale (quantize_gaussian_e4m3), their exact (FP64) product
    scaled by 1/sqrt(m)."""
    assert batch % block == 0
    b = np.asarray(b, dtype=np.float64)
    r = b.shape[0]
    bq, _ = quantize_e4m3_blocks(b, block, axis=0)
    c = np.zeros((m, b.shape[1]))
    for b0 in range(0, r, batch):
        b1 = min(r, b0 + batch)
        zq = quantize_gaussian_e4m3(gaussian_normals(m, b0, b1, seed))
        c += zq @ bq[b0:b1]
    return c / np.sqrt(m)


def sketch_gcs_fp8_reference(a, m, r, seed, block=128, batch=4096):
    """Quantisation-aware reference of the FP8 Gaussian GEMM: S*A quantised
    per column in blocks of `block` buckets, the unscaled normals quantised
    with G's fixed scale, their exact (FP64) product scaled by 1/sqrt(m)."""
    return gauss_product_fp8_reference(sketch_cs(a, r, seed), m, seed, block, batch)


def sketch_g_fp8_reference(a, m, seed, block=128, batch=4096):
    """The same for G*A (blocks of `block` rows of A)."""
    a = _as_f64(a)
    return gauss_product_fp8_reference(a.toarray() if sp.issparse(a) else a, m, seed,
                                       block, batch)
