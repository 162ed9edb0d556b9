"""Pins of the OSNAP oracle (oracle/osnap.py) against what the definition and
the mathematics fix: the exact hash with Python integers, s = 1 equal to the
CountSketch of Definition 3 bit for bit, the structure of S (s distinct rows
per column, one per block, +-1/sqrt(s)), unit column norms and E[S^T S] = I,
uniform rows and balanced signs, the subspace-embedding distortion of an
incoherent basis at the Marchenko-Pastur edges, and the coherent basis that
CountSketch cannot embed at r < d^2 while OSNAP with s = 8 can."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy import stats

from oracle import osnap as oo
from oracle import sketch as osk


@pytest.mark.parametrize("r,s", [(8, 2), (4096, 4), (65536, 8), (3 * 5 * 7, 7)])
def test_hash_matches_bigint(r, s):
    rng = np.random.default_rng(r + s)
    for i in list(rng.integers(0, 2 ** 40, 40)) + [0, 1, 2 ** 32 - 1, 2 ** 32]:
        i = int(i)
        h, sg = oo.osnap_hash(1, r, s, seed=77, row0=i)
        want = oo.osnap_hash_bigint(i, r, s, seed=77)
        assert [(int(a), int(b)) for a, b in zip(h[0], sg[0])] == want


def test_s1_is_countsketch():
    h, sg = oo.osnap_hash(5000, 777, 1, seed=3)
    ho, so = osk.cs_hash(5000, 777, seed=3)
    np.testing.assert_array_equal(h[:, 0], ho)
    np.testing.assert_array_equal(sg[:, 0], so)
    a = np.random.default_rng(0).standard_normal((3000, 9))
    np.testing.assert_array_equal(oo.sketch_osnap(a, 200, 1, 5), osk.sketch_cs(a, 200, 5))
    np.testing.assert_array_equal(oo.sketch_gosnap(a, 17, 200, 1, 5),
                                  osk.sketch_gcs(a, 17, 200, 5))


@pytest.mark.parametrize("r,s", [(48, 2), (48, 3), (48, 4), (48, 6), (48, 48)])
def test_structure_of_s(r, s):
    n = 300
    S = oo.osnap_dense(n, r, s, seed=11)
    np.testing.assert_array_equal(S, oo.osnap_sparse(n, r, s, seed=11).toarray())
    rb = r // s
    for i in range(n):
        nz = np.flatnonzero(S[:, i])
        assert len(nz) == s                                   # s non-zeros ...
        assert np.array_equal(nz // rb, np.arange(s))         # ... one per block
        np.testing.assert_array_equal(np.abs(S[nz, i]), 1 / np.sqrt(s))


def test_unit_columns_and_isotropy():
    """||S e_i|| = 1 for every column; E[S^T S] = I and E||S A||_F^2 =
    ||A||_F^2 by Monte Carlo over seeds."""
    n, r, s = 40, 64, 4
    S = oo.osnap_dense(n, r, s, seed=0)
    np.testing.assert_allclose(np.linalg.norm(S, axis=0), 1.0, rtol=1e-15)
    T = 2000
    acc = np.zeros((n, n))
    for t in range(T):
        S = oo.osnap_sparse(n, r, s, seed=t)
        acc += (S.T @ S).toarray()
    mean = acc / T
    np.testing.assert_allclose(np.diag(mean), 1.0, rtol=1e-14)
    off = mean[~np.eye(n, dtype=bool)]
    # each off-diagonal entry is a mean of T terms of variance
    # s * (1/(r/s)) / s^2 = 1/r: |mean| < 5 / sqrt(r T) for all of them
    assert np.abs(off).max() < 5.0 / np.sqrt(r * T)
    a = np.random.default_rng(1).standard_normal((500, 6))
    ratios = np.array([np.linalg.norm(oo.sketch_osnap(a, 96, 3, seed=t)) ** 2
                       for t in range(400)]) / np.linalg.norm(a) ** 2
    assert abs(ratios.mean() - 1.0) < 4 * ratios.std() / np.sqrt(len(ratios))


def test_uniform_rows_and_balanced_signs():
    n, r, s = 200_000, 512, 8
    h, sg = oo.osnap_hash(n, r, s, seed=9)
    rb = r // s
    for k in range(s):
        counts = np.bincount(h[:, k] - k * rb, minlength=rb)
        assert counts.size == rb
        assert stats.chisquare(counts).pvalue > 1e-4
        assert stats.binomtest(int((sg[:, k] > 0).sum()), n).pvalue > 1e-4


def test_incoherent_distortion_at_marchenko_pastur_edges():
    """An orthonormal Gaussian basis U (n x d): the singular values of S U
    spread to the Marchenko-Pastur edges 1 +- sqrt(d / r) of a Gaussian
    embedding, for every s."""
    rng = np.random.default_rng(0)
    n, d, r = 20000, 32, 1024
    u, _ = np.linalg.qr(rng.standard_normal((n, d)))
    edge = np.sqrt(d / r)
    for s in (2, 4, 8):
        for seed in range(3):
            sv = np.linalg.svd(oo.sketch_osnap(u, r, s, seed), compute_uv=False)
            assert sv.max() - 1 <= edge + 0.05 and 1 - sv.min() <= edge + 0.05
            assert abs((sv ** 2).sum() / d - 1) < 0.1   # ||S U||_F^2 ~ d


def test_coherent_basis_needs_s_above_one():
    """U = the first d columns of the identity (d rows of leverage 1) with
    r = 8 d < d^2: CountSketch puts two of those rows in one bucket for most
    seeds (S U then loses rank), OSNAP with s = 8 keeps S U well conditioned
    (two columns would have to meet in all 8 blocks)."""
    n, d, r = 1000, 32, 256
    u = np.zeros((n, d))
    u[np.arange(d), np.arange(d)] = 1.0
    lost, worst8 = 0, 0.0
    for seed in range(20):
        sv1 = np.linalg.svd(oo.sketch_osnap(u, r, 1, seed), compute_uv=False)
        lost += sv1.min() < 1e-12
        sv8 = np.linalg.svd(oo.sketch_osnap(u, r, 8, seed), compute_uv=False)
        worst8 = max(worst8, abs(sv8 - 1).max())
    assert lost >= 14           # collision probability 1 - e^{-2} ~ 0.86
    assert worst8 < 0.75


def test_products_brute_force():
    """S*A and G*S*A against the explicit dense S and the whole G."""
    rng = np.random.default_rng(4)
    n, d, r, s, m = 150, 7, 30, 3, 11
    a = rng.standard_normal((n, d))
    S = oo.osnap_dense(n, r, s, seed=2)
    np.testing.assert_allclose(oo.sketch_osnap(a, r, s, 2), S @ a, rtol=1e-13, atol=1e-13)
    ac = sp.random(n, d, density=0.2, random_state=1, format="csr")
    np.testing.assert_allclose(oo.sketch_osnap(ac, r, s, 2), S @ ac.toarray(), rtol=1e-13,
                               atol=1e-13)
    G = osk.gaussian_normals(m, 0, r, seed=2) / np.sqrt(m)
    np.testing.assert_allclose(oo.sketch_gosnap(a, m, r, s, 2), G @ (S @ a), rtol=1e-12,
                               atol=1e-12)
    np.testing.assert_array_equal(oo.sketch_gosnap(a, 0, r, s, 2), oo.sketch_osnap(a, r, s, 2))


def test_rejects_s_not_dividing_r():
    with pytest.raises(ValueError):
        oo.osnap_hash(10, 30, 4, seed=0)
    with pytest.raises(ValueError):
        oo.osnap_hash(10, 30, 0, seed=0)
