"""Pins of the oracle's CountSketch, Gaussian and CountGauss sketches:
the paper's worked example, structural invariants of Definition 3, the
workload moments of Lemma 1, associativity, m = 0 semantics, Gaussian
moments, and the reduced-precision rounding against PyTorch's CPU casts."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import sketch as osk


def _example(golden_dir):
    vec, mat = None, []
    with open(os.path.join(golden_dir, "countsketch_example.txt")) as f:
        lines = [l for l in f if not l.startswith("#") and l.strip()]
    for l in lines:
        if l.startswith("vector:"):
            vec = [int(t) for t in l.split(":")[1].split()]
        elif l.startswith("matrix:"):
            continue
        else:
            mat.append([int(t) for t in l.split()])
    return np.array(vec), np.array(mat, dtype=float)


def test_worked_example_vector_to_matrix(golden_dir):
    v, s_fig = _example(golden_dir)
    s = osk.dense_from_vector(v, 6)
    assert s.shape == (6, 12)
    # exactly one +-1 per column (Definition 3) and nnz(S) = n
    assert np.all((s != 0).sum(axis=0) == 1)
    assert np.count_nonzero(s) == 12
    # 11 of 12 columns agree with the printed matrix; column 5 (1-based) is the
    # printed sign typo recorded with the fixture
    diff = np.nonzero(np.any(s != s_fig, axis=0))[0]
    assert list(diff) == [4]
    assert s[0, 4] == 1.0 and s_fig[0, 4] == -1.0


def test_vector_representation_round_trip():
    h, sg = osk.cs_hash(50, 7, seed=3)
    v = osk.vector_representation(h, sg)
    s = osk.dense_from_vector(v, 7)
    np.testing.assert_array_equal(s, osk.countsketch_dense(50, 7, seed=3))


def test_countsketch_structure():
    s = osk.countsketch_dense(300, 40, seed=11)
    assert np.all((s != 0).sum(axis=0) == 1)
    assert set(np.unique(s[s != 0])) <= {-1.0, 1.0}
    assert np.count_nonzero(s) == 300


@pytest.mark.parametrize("sparse", [False, True])
def test_sketch_cs_sum_identity_integer(sparse):
    """1^T (S A) = sigma^T A holds exactly for integer A (every column of S has
    one entry, so summing the rows of S A re-adds every signed row of A)."""
    n, d, r = 500, 9, 37
    a = (synth.csr_integer(n, d, 0.3, seed=1) if sparse
         else synth.dense_integer(n, d, seed=1))
    sa = osk.sketch_cs(a, r, seed=8)
    _, sg = osk.cs_hash(n, r, seed=8)
    ad = a.toarray() if sparse else a
    np.testing.assert_array_equal(sa.sum(axis=0), sg.astype(float) @ ad)


def test_sketch_cs_row_lists_brute_force():
    """Each row of S A is the signed sum of the rows of A hashed to it."""
    n, d, r = 200, 5, 13
    a = synth.dense_integer(n, d, seed=4)
    sa = osk.sketch_cs(a, r, seed=21)
    for b in range(r):
        acc = np.zeros(d)
        for i in range(n):
            hb, sb = osk.cs_hash_bigint(i, r, 21)
            if hb == b:
                acc += sb * a[i]
        np.testing.assert_array_equal(sa[b], acc)


def test_sketch_norm_preserved_in_expectation():
    """E ||S A||_F^2 = ||A||_F^2 (cross terms vanish in expectation)."""
    n, d, r = 60, 4, 10
    a = synth.dense_gaussian(n, d, seed=2)
    vals = [np.linalg.norm(osk.sketch_cs(a, r, seed=s)) ** 2 for s in range(600)]
    ref = np.linalg.norm(a) ** 2
    se = np.std(vals) / np.sqrt(len(vals))
    assert abs(np.mean(vals) - ref) < 5 * se


def test_lemma1_bucket_set_workload_moments():
    """Lemma 1: for a fixed set of B of the r buckets, the work
    Y = sum_i eps_i w_i has mean q nnz(A) and variance q(1-q) nnz_2(A), q=B/r."""
    n, r, B = 3000, 64, 16
    w = synth.csr_zipf(n, 200, 0.02, seed=3).getnnz(axis=1).astype(float)
    nnz, nnz2 = w.sum(), (w ** 2).sum()
    q = B / r
    ys = []
    for s in range(400):
        h, _ = osk.cs_hash(n, r, seed=1000 + s)
        ys.append(w[h < B].sum())
    ys = np.array(ys)
    mu, var = q * nnz, q * (1 - q) * nnz2
    assert abs(ys.mean() - mu) < 5 * np.sqrt(var / ys.size)
    # sample variance within 25% (400 samples: relative s.e. ~ 7-15%)
    assert abs(ys.var(ddof=1) / var - 1) < 0.3


def test_gaussian_moments_and_normality():
    from scipy import stats
    m, r = 64, 4000
    z = osk.gaussian_normals(m, 0, r, seed=9).ravel()
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    g = osk.gaussian_block(m, 0, r, seed=9)
    np.testing.assert_allclose(g, z.reshape(m, r) / 8.0, rtol=0, atol=0)


def test_gaussian_column_blocks_consistent():
    """Any bucket range gives the same columns (blocks are only batching)."""
    full = osk.gaussian_normals(11, 0, 103, seed=4)
    for b0, b1 in [(0, 1), (1, 5), (3, 4), (5, 103), (50, 77)]:
        np.testing.assert_array_equal(osk.gaussian_normals(11, b0, b1, seed=4),
                                      full[:, b0:b1])
    # and any row range: row a is drawn from counter word 2 = a alone
    for a0, cnt in [(0, 3), (4, 7), (10, 1)]:
        np.testing.assert_array_equal(osk.gaussian_normals(cnt, 0, 103, seed=4, a0=a0),
                                      full[a0:a0 + cnt])


def test_gaussian_embedding_isotropic():
    """E[(G S)^T (G S)] = I: G with variance 1/m, S with +-1 entries."""
    n, m, r = 6, 8, 16
    acc = np.zeros((n, n))
    T = 1500
    for s in range(T):
        gs = osk.gaussian_block(m, 0, r, seed=s) @ osk.countsketch_dense(n, r, s)
        acc += gs.T @ gs
    np.testing.assert_allclose(acc / T, np.eye(n), atol=0.12)


@pytest.mark.parametrize("sparse", [False, True])
def test_countgauss_associativity_and_batching(sparse):
    n, d, m, r = 300, 7, 12, 50
    a = (synth.csr_uniform(n, d, 0.4, seed=5) if sparse
         else synth.dense_gaussian(n, d, seed=5))
    c = osk.sketch_gcs(a, m, r, seed=77)
    s = osk.countsketch_dense(n, r, 77)
    g = osk.gaussian_block(m, 0, r, seed=77)
    ad = a.toarray() if sparse else a
    np.testing.assert_allclose(c, (g @ s) @ ad, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(osk.sketch_gcs(a, m, r, 77, batch=7), c,
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(osk.sketch_gcs(a, 0, r, 77),
                                  osk.sketch_cs(a, r, 77))


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, 1.0, -1.0, 1.00390625, 1.01171875, 3e38, 1e-40]])
    x32 = x.astype(np.float32)
    want = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(osk.to_bf16(x32.astype(np.float64)), want)


def test_e4m3_rounding_matches_torch_in_range():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = rng.uniform(-440, 440, 20000) * 10.0 ** rng.integers(-4, 1, 20000)
    x = np.concatenate([x, [0.0, 448.0, -448.0, 2 ** -9, 2 ** -10, 3 * 2 ** -10, 0.5 + 2 ** -5]])
    x32 = x.astype(np.float32)
    want = torch.from_numpy(x32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(osk.to_e4m3(x32.astype(np.float64)), want)
    # saturation beyond the largest finite e4m3 value
    assert osk.to_e4m3(np.array([1e6, -500.0])).tolist() == [448.0, -448.0]


def test_bf16_limbs_refine():
    x = np.random.default_rng(2).standard_normal(1000)
    l = osk.bf16_limbs(x, 2)
    e1 = np.abs(x - l[0]).max() / np.abs(x).max()
    e2 = np.abs(x - l[0] - l[1]).max() / np.abs(x).max()
    assert e1 < 2 ** -8 and e2 < 2 ** -15


def test_bf16_of_doubles_is_nearest_even():
    # FP64 inputs that are not FP32 values: the result must be the nearest
    # bfloat16 neighbour (ties to the even significand), checked against the
    # two neighbours enumerated from the bfloat16 bit patterns.
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(5000) * 10.0 ** rng.integers(-20, 20, 5000)
    # exact ties between neighbours, and values one FP64 ulp off a tie
    base = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    ulp = np.ldexp(1.0, np.frexp(np.abs(base))[1] - 8)
    ties = base + 0.5 * ulp
    x = np.concatenate([x, ties, np.nextafter(ties, np.inf), np.nextafter(ties, -np.inf)])
    y = osk.to_bf16(x)
    bits = torch.from_numpy(np.abs(x).astype(np.float32)).to(torch.bfloat16).view(torch.int16)
    bits = bits.numpy().astype(np.int64)
    cands = []
    for db in (-1, 0, 1):
        c = torch.from_numpy((bits + db).astype(np.int16)).view(torch.bfloat16)
        cands.append(c.to(torch.float64).numpy())
    cands = np.stack(cands) * np.sign(x)[None, :]
    dist = np.abs(cands - x[None, :])
    best = dist.min(axis=0)
    assert np.all(np.abs(y - x) == best)
    # among equidistant candidates the chosen one has an even last bit
    yb = torch.from_numpy(np.abs(y).astype(np.float32)).to(torch.bfloat16).view(torch.int16)
    tie = (dist == best[None, :]).sum(axis=0) > 1
    assert np.all((yb.numpy()[tie] & 1) == 0)


def test_bf16_reference_within_rounding_bound():
    # |bf16(z) - z| <= 2^-8 |z| and |hi + lo - sa| <= 2^-16 |sa| (RNE with 8
    # significant bits), so the quantised product differs from the FP64 one
    # by at most (2^-8 + 2^-16 + 2^-24) (|Z| |SA|) / sqrt(m) per entry.
    a = synth.dense_gaussian(3000, 20, seed=4)
    m, r, seed = 40, 500, 6
    cq = osk.sketch_gcs_bf16_reference(a, m, r, seed)
    c = osk.sketch_gcs(a, m, r, seed)
    mag = np.abs(osk.gaussian_normals(m, 0, r, seed)) @ np.abs(osk.sketch_cs(a, r, seed))
    bound = mag * (2.0 ** -8 + 2.0 ** -16 + 2.0 ** -24 + 1e-13) / np.sqrt(m)
    assert np.all(np.abs(cq - c) <= bound)
    rel = np.linalg.norm(cq - c) / np.linalg.norm(c)
    assert 1e-4 < rel < 1e-2


def test_e8m0_exponent_is_smallest_covering_power():
    rng = np.random.default_rng(11)
    amax = np.concatenate([np.abs(rng.standard_normal(2000)) * 10.0 ** rng.integers(-8, 8, 2000),
                           448.0 * 2.0 ** np.arange(-12, 12),          # exact boundaries
                           np.nextafter(448.0 * 2.0 ** np.arange(-12, 12), np.inf),
                           np.nextafter(448.0 * 2.0 ** np.arange(-12, 12), 0.0)])
    e = osk.e8m0_exponent(amax)
    # brute force: smallest integer e with 448 * 2^e >= amax
    for v, ev in zip(amax, e):
        assert np.ldexp(448.0, int(ev)) >= v
        assert np.ldexp(448.0, int(ev) - 1) < v
    assert osk.e8m0_exponent(0.0) == 0


def test_block_quantisation_bounds():
    rng = np.random.default_rng(12)
    x = rng.standard_normal((300, 7)) * 10.0 ** rng.integers(-3, 3, (300, 7))
    q, e = osk.quantize_e4m3_blocks(x, 128, axis=0)
    assert e.shape == (3, 7)
    for b in range(3):
        blk, qb = x[128 * b:128 * (b + 1)], q[128 * b:128 * (b + 1)]
        s = np.ldexp(1.0, e[b])
        amax = np.abs(blk).max(axis=0)
        # the block maximum lands in (224, 448] after scaling
        assert np.all(amax / s <= 448.0) and np.all(amax / s > 224.0)
        # RNE with 3 fraction bits: relative error <= 2^-4 for normal values,
        # absolute <= 2^-10 s in the subnormal range
        err = np.abs(qb - blk)
        assert np.all(err <= np.maximum(2.0 ** -4 * np.abs(blk), 2.0 ** -10 * s) * (1 + 1e-15))
    # along the other axis as well
    q2, e2 = osk.quantize_e4m3_blocks(x.T, 128, axis=1)
    np.testing.assert_array_equal(q2, q.T)
    np.testing.assert_array_equal(e2, e)


def test_fp8_reference_within_rounding_bound():
    a = synth.dense_gaussian(3000, 20, seed=4)
    m, r, seed = 40, 500, 6
    cq = osk.sketch_gcs_fp8_reference(a, m, r, seed)
    c = osk.sketch_gcs(a, m, r, seed)
    z = osk.gaussian_normals(m, 0, r, seed)
    sa = osk.sketch_cs(a, r, seed)
    zq = osk.quantize_gaussian_e4m3(z)
    saq, es = osk.quantize_e4m3_blocks(sa, 128, axis=0)
    # elementwise rounding bounds of the two operands (see above); G's scale
    # is the fixed 2^G_FP8_EXP
    sz = np.full(z.shape, np.ldexp(1.0, osk.G_FP8_EXP))
    ss = np.repeat(np.ldexp(1.0, es), 128, axis=0)[:r]
    dz = np.maximum(2.0 ** -4 * np.abs(z), 2.0 ** -10 * sz)
    ds = np.maximum(2.0 ** -4 * np.abs(sa), 2.0 ** -10 * ss)
    assert np.all(np.abs(zq - z) <= dz * (1 + 1e-15))
    bound = (dz @ np.abs(sa) + np.abs(z) @ ds + dz @ ds) / np.sqrt(m)
    assert np.all(np.abs(cq - c) <= bound * (1 + 1e-12) + 1e-13 * np.abs(c).max())
    rel = np.linalg.norm(cq - c) / np.linalg.norm(c)
    assert 5e-3 < rel < 1e-1


# ---------------------------------------------------------------------------
# G*A (Algorithm gaussian_sketch, csrjlt)
# ---------------------------------------------------------------------------
def _csr_with_duplicates():
    """Tiny CSR with empty rows, unsorted columns and a duplicated entry."""
    indptr = np.array([0, 2, 2, 5, 6, 6, 8])
    indices = np.array([3, 0, 1, 4, 1, 2, 4, 0])
    data = np.array([1.5, -2.0, 0.5, 3.0, -1.0, 2.5, 1.0, -0.75])
    return sp.csr_matrix((data, indices, indptr), shape=(6, 5))


def test_sketch_g_matches_algorithm_loops():
    """The batched matrix form equals Algorithm gaussian_sketch's loops (a
    fresh column of normals per row of A, entries added one by one)."""
    a = _csr_with_duplicates()
    c = osk.sketch_g(a, 7, seed=3)
    np.testing.assert_allclose(c, osk.sketch_g_literal(a, 7, seed=3), rtol=1e-14, atol=1e-15)
    b = synth.csr_uniform(200, 9, 0.3, seed=2)
    np.testing.assert_allclose(osk.sketch_g(b, 5, seed=8, batch=17),
                               osk.sketch_g_literal(b, 5, seed=8), rtol=1e-12, atol=1e-13)
    # dense input, different batch size: same matrix
    np.testing.assert_allclose(osk.sketch_g(b.toarray(), 5, seed=8, batch=64),
                               osk.sketch_g(b, 5, seed=8), rtol=1e-12, atol=1e-13)


def test_sketch_g_is_the_combined_sketch_with_identity():
    """G*(S*A) through sketch_g on the r-row matrix S*A is the combined sketch:
    both draw column b of G for bucket (row) b."""
    a = synth.dense_gaussian(400, 6, seed=1)
    r, m = 90, 11
    np.testing.assert_allclose(osk.sketch_g(osk.sketch_cs(a, r, 4), m, 4),
                               osk.sketch_gcs(a, m, r, 4), rtol=1e-12, atol=1e-12)


def test_sketch_g_embedding_in_expectation():
    """E[C^T C] = A^T A for C = G*A, G with variance 1/m (Monte Carlo)."""
    a = synth.dense_gaussian(30, 3, seed=6)
    m, T = 8, 800
    acc = np.zeros((3, 3))
    for s in range(T):
        c = osk.sketch_g(a, m, seed=s)
        acc += c.T @ c
    ata = a.T @ a
    # the entries' standard error is about sqrt(2/(m T)) of the diagonal scale
    assert np.abs(acc / T - ata).max() <= 6 * np.sqrt(2.0 / (m * T)) * np.abs(np.diag(ata)).max()


def test_sketch_g_quantised_references_within_bounds():
    a = synth.csr_uniform(900, 10, 0.2, seed=3)
    ad = a.toarray()
    m, seed = 16, 5
    c = osk.sketch_g(a, m, seed)
    z = osk.gaussian_normals(m, 0, 900, seed)
    mag = np.abs(z) @ np.abs(ad) / np.sqrt(m)
    cb = osk.sketch_g_bf16_reference(a, m, seed)
    assert np.all(np.abs(cb - c) <= mag * (2.0 ** -8 + 2.0 ** -16 + 2.0 ** -24 + 1e-13))
    c8 = osk.sketch_g_fp8_reference(a, m, seed)
    zq = osk.quantize_gaussian_e4m3(z)
    aq, ea = osk.quantize_e4m3_blocks(ad, 128, axis=0)
    np.testing.assert_allclose(c8, zq @ aq / np.sqrt(m), rtol=1e-12, atol=1e-14)
    # 900 = 7 * 128 + 4: the last block holds rows 896 .. 899, and its scale
    # is taken over those rows only
    np.testing.assert_array_equal(ea[-1], osk.e8m0_exponent(np.abs(ad[896:]).max(axis=0)))


def test_gaussian_fp8_scale_covers_every_normal():
    """G's fixed FP8 scale: the largest radius the generator can produce
    (smallest uniform, u = 2^-33) maps below 448, so no value of G
    saturates; on the normal e4m3 range the fixed scale rounds exactly as the
    block-amax scale does (power-of-two scaling keeps the significand), and
    below it the rounding error stays under half a subnormal quantum."""
    rmax = np.sqrt(-2.0 * np.log(2.0 ** -33))
    assert rmax * 2.0 ** -osk.G_FP8_EXP < 448.0
    assert 448.0 * 2.0 ** (osk.G_FP8_EXP - 1) < rmax  # and 2^-7 would not cover it
    z = osk.gaussian_normals(64, 0, 4096, 3)
    zq = osk.quantize_gaussian_e4m3(z)
    zb, _ = osk.quantize_e4m3_blocks(z, 128, axis=1)
    big = np.abs(z) >= 2.0 ** (osk.G_FP8_EXP - 6)
    np.testing.assert_array_equal(zq[big], zb[big])
    quantum = 2.0 ** (osk.G_FP8_EXP - 9)  # e4m3 subnormal step at this scale
    assert np.all(np.abs(zq - z)[~big] <= quantum / 2)
    # the largest normal the generator gives (u0 = 2^-33, u1 -> 0) quantises
    # to a finite e4m3 value within the relative rounding bound
    zr = osk.quantize_gaussian_e4m3(np.array([rmax, -rmax]))
    np.testing.assert_array_equal(zr, osk.to_e4m3(np.array([rmax, -rmax]) * 64.0) / 64.0)
    assert np.all(np.abs(np.abs(zr) - rmax) <= rmax * 2.0 ** -4)
