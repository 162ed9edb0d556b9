"""Pins of the oracle's Gram matrix, squared row norms, QR / leverage scores and
least-squares solvers: the paper's literal CSR loops on tiny inputs, closed
forms (trace, B = I, exact leverage), the leverage-score invariants of a
sketched basis, and LAPACK least squares."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import gram as og
from oracle import leverage as olev
from oracle import lsq as olsq
from oracle import sketch as osk


def test_gram_literal_loop_equals_blas():
    a = synth.csr_integer(40, 9, 0.35, seed=3)
    np.testing.assert_array_equal(og.gram_csr_literal(a), og.gram(1.0, a))
    np.testing.assert_array_equal(og.gram(1.0, a), og.gram(1.0, a.toarray()))


def test_gram_closed_forms_and_alpha_beta():
    a = synth.dense_gaussian(100, 6, seed=1)
    g = og.gram(1.0, a)
    assert np.allclose(g, g.T, rtol=0, atol=0)
    assert abs(np.trace(g) - np.linalg.norm(a) ** 2) < 1e-12 * np.trace(g)
    c = synth.dense_gaussian(6, 6, seed=2)
    np.testing.assert_allclose(og.gram(2.5, a, -0.5, c), 2.5 * g - 0.5 * c,
                               rtol=1e-14, atol=1e-12)
    nan = np.full((6, 6), np.nan)
    assert np.all(np.isfinite(og.gram(1.0, a, 0.0, nan)))
    # Gram of an orthonormal basis is the identity
    q, _ = np.linalg.qr(a)
    np.testing.assert_allclose(og.gram(1.0, q), np.eye(6), atol=1e-14)


def test_rownorms_identity_and_literal():
    a = synth.csr_integer(50, 8, 0.4, seed=4)
    ad = a.toarray()
    np.testing.assert_array_equal(og.rownorms_sq(1.0, a, np.eye(8)),
                                  (ad ** 2).sum(axis=1))
    b = synth.dense_integer(8, 5, seed=5)
    np.testing.assert_array_equal(og.rownorms_sq_csr_literal(1.0, a, b),
                                  og.rownorms_sq(1.0, ad, b))
    x = np.arange(50.0)
    np.testing.assert_array_equal(og.rownorms_sq(2.0, ad, b, 3.0, x),
                                  2.0 * og.rownorms_sq(1.0, ad, b) + 3.0 * x)


def test_rownorms_exact_leverage_via_exact_r():
    a = synth.dense_gaussian(300, 7, seed=6)
    r = np.linalg.qr(a, mode="r")
    theta = og.rownorms_sq(1.0, a, np.linalg.inv(r))
    np.testing.assert_allclose(theta, olev.leverage_exact(a), rtol=1e-11, atol=1e-14)


def test_exact_leverage_sum_is_rank_and_bounded():
    a = synth.dense_gaussian(400, 11, seed=7)
    th = olev.leverage_exact(a)
    assert th.min() >= 0 and th.max() <= 1 + 1e-12
    assert abs(th.sum() - 11) < 1e-10
    # a row orthogonal to the others (coherent) has leverage 1
    b = np.zeros((50, 3)); b[:, :2] = synth.dense_gaussian(50, 2, seed=1)
    b[17, 2] = 5.0
    assert abs(olev.leverage_exact(b)[17] - 1.0) < 1e-12


@pytest.mark.parametrize("sparse", [False, True])
def test_sketched_leverage_invariants(sparse):
    """With U an orthonormal basis of range(A) and sigma_j the singular values
    of G S U: theta_i / sigma_max^2 <= theta~_i <= theta_i / sigma_min^2 and
    sum_i theta~_i = sum_j sigma_j^{-2} (A R^{-1} = U (R_U)^{-1} with R_U the
    triangular factor of G S U)."""
    n, d, m, r = 2000, 6, 40, 300
    a = synth.csr_uniform(n, d, 0.5, seed=8) if sparse else synth.dense_gaussian(n, d, seed=8)
    th = olev.leverage_exact(a)
    tt, _ = olev.leverage_sketched(a, m, r, seed=5)
    sv = olev.sketch_distortion(a, m, r, seed=5)
    assert np.all(tt >= th / sv.max() ** 2 * (1 - 1e-9))
    assert np.all(tt <= th / sv.min() ** 2 * (1 + 1e-9))
    assert abs(tt.sum() - (sv ** -2).sum()) < 1e-9 * tt.sum()
    # QR route equals the paper's SVD route
    np.testing.assert_allclose(olev.leverage_sketched_svd(a, m, r, seed=5), tt,
                               rtol=1e-9, atol=1e-15)


def test_countsketch_only_leverage_invariants():
    """Algorithm ls_approximate_drineas sketches with S alone (m = 0): the
    bracket by the singular values of S U holds for that sketch too."""
    n, d, r = 3000, 5, 400
    a = synth.dense_gaussian(n, d, seed=2)
    th = olev.leverage_exact(a)
    tt, _ = olev.leverage_sketched(a, 0, r, seed=6)
    sv = olev.sketch_distortion(a, 0, r, seed=6)
    assert np.all(tt >= th / sv.max() ** 2 * (1 - 1e-9))
    assert np.all(tt <= th / sv.min() ** 2 * (1 + 1e-9))
    assert abs(tt.sum() - (sv ** -2).sum()) < 1e-9 * tt.sum()


def test_jl_matrix_distribution_and_stream():
    """Pi (d x t) has independent entries of mean 0 and variance 1/t, so
    E[Pi Pi^T] = I, and its normals are not those of G at the same counters
    (stream 2 against stream 1)."""
    d, t = 64, 4096
    pi = olev.jl_matrix(d, t, seed=3)
    assert pi.shape == (d, t)
    z = pi * np.sqrt(t)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    g = osk.gaussian_normals(t, 0, d, 3)  # stream 1, same (row, column) counters
    assert abs((z * g.T).mean()) < 5 / np.sqrt(z.size)
    pp = pi @ pi.T
    assert np.abs(np.diag(pp) - 1).max() < 6 * np.sqrt(2 / t)
    assert np.abs(pp - np.diag(np.diag(pp))).max() < 6 / np.sqrt(t)
    # the first columns of Pi do not depend on t beyond the 1/sqrt(t) scale
    np.testing.assert_allclose(olev.jl_matrix(d, 100, seed=3)[:, :40] * 10,
                               z[:, :40], rtol=1e-15, atol=0)


def test_jl_leverage_t0_is_the_unreduced_estimate():
    a = synth.csr_uniform(800, 7, 0.4, seed=3)
    tt, _ = olev.leverage_sketched(a, 30, 200, seed=8)
    np.testing.assert_array_equal(olev.leverage_sketched_jl(a, 30, 200, 0, seed=8), tt)


def test_jl_leverage_unbiased_over_pi():
    """For a fixed sketch, theta~_i / theta_i (JL step) is chi^2_t / t: mean 1,
    variance 2/t.  The mean over K draws of Pi stays within 6 standard
    deviations of 1 on every row."""
    n, d, t, K = 200, 6, 8, 400
    a = synth.dense_gaussian(n, d, seed=4)
    c = osk.sketch_gcs(a, 24, 120, seed=1)
    t0 = olev.leverage_from_sketch(a, c, 0, seed=1)
    acc = np.zeros(n)
    for s in range(K):
        acc += olev.leverage_from_sketch(a, c, t, seed=1000 + s)
    ratio = acc / K / t0
    assert np.abs(ratio - 1).max() < 6 * np.sqrt(2 / t / K)
    # and one draw alone is spread as chi^2_t / t
    one = olev.leverage_from_sketch(a, c, t, seed=7) / t0
    assert 0.5 < one.var() / (2 / t) < 2.0


@pytest.mark.parametrize("m", [0, 60])
def test_jl_leverage_within_jl_bound(m):
    """With t = 3000 every row norm of A R^{-1} is kept to within
    1 +- 6 sqrt(2/t) (about 0.155): the JL property the step relies on."""
    n, d, r, t = 3000, 10, 500, 3000
    a = synth.dense_gaussian(n, d, seed=11)
    t0 = olev.leverage_sketched_jl(a, m, r, 0, seed=4)
    tj = olev.leverage_sketched_jl(a, m, r, t, seed=4)
    assert np.abs(tj / t0 - 1).max() < 6 * np.sqrt(2 / t)
    assert abs(tj.sum() / t0.sum() - 1) < 6 * np.sqrt(2 / t / d)


def test_distortion_within_marchenko_pastur_edges():
    n, d, m, r = 20000, 8, 400, 4000
    a = synth.dense_gaussian(n, d, seed=9)
    sv = olev.sketch_distortion(a, m, r, seed=3)
    # Gaussian stage edges 1 +- sqrt(d/m) widened for the CountSketch stage
    e = np.sqrt(d / m)
    assert sv.max() < 1 + 3 * e and sv.min() > 1 - 3 * e


def test_qr_r_and_tri_inv():
    c = synth.dense_gaussian(30, 5, seed=1)
    r = olev.qr_r(c)
    assert np.all(np.diag(r) >= 0) and np.allclose(np.tril(r, -1), 0)
    np.testing.assert_allclose(r.T @ r, c.T @ c, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(olev.tri_inv(r) @ r, np.eye(5), atol=1e-13)


def test_lsq_noise_free_recovers_solution():
    a, b, xt = synth.lsq_problem(3000, 10, cond=1e4, seed=1, noise=0.0)
    x, info = olsq.lsq_sketch_precond(a, b, m=40, r=100, seed=2)
    assert np.linalg.norm(x - xt) / np.linalg.norm(xt) < 1e4 * 1e-12
    assert info["cond_precond"] > 1e3  # the preconditioner carries kappa(A)


@pytest.mark.parametrize("cond", [1e2, 1e6])
def test_lsq_matches_lapack(cond):
    a, b, _ = synth.lsq_problem(5000, 16, cond=cond, seed=3)
    xs = olsq.lstsq(a, b)
    x, info = olsq.lsq_sketch_precond(a, b, m=64, r=256, seed=4)
    rs, _ = olsq.lsq_quality(a, b, xs)
    rn, ne = olsq.lsq_quality(a, b, x)
    assert (rn - rs) / rs < 1e-10
    assert ne < 1e-10
    # a preconditioned LSQR converges in few iterations regardless of cond
    assert info["iters"][0] < 80


# ---------------------------------------------------------------------------
# sketch-and-solve (Algorithm least_squares_approx)
# ---------------------------------------------------------------------------
def test_sketch_solve_recovers_consistent_solution():
    """b in range(A): the sketched system is consistent too, so the sketched
    least-squares solution is the exact one."""
    a, b, xt = synth.lsq_problem(3000, 8, cond=1e3, seed=5, noise=0.0)
    x = olsq.lsq_sketch_solve(a, b, m=40, r=200, seed=3)
    assert np.linalg.norm(x - xt) / np.linalg.norm(xt) < 1e3 * 1e-12


def test_sketch_solve_residual_near_optimal():
    """||A x~ - b|| >= ||A x* - b|| always (x* minimises it), and for a
    Gaussian embedding the squared ratio averages about 1 + d / (m - d - 1)
    (Monte Carlo over seeds, loose bounds)."""
    a, b, _ = synth.lsq_problem(4000, 6, cond=10.0, seed=6, noise=1.0)
    xs = olsq.lstsq(a, b)
    rs = np.linalg.norm(a @ xs - b)
    m, r = 30, 600
    ratios = []
    for s in range(60):
        x = olsq.lsq_sketch_solve(a, b, m, r, seed=s)
        ratios.append((np.linalg.norm(a @ x - b) / rs) ** 2)
    ratios = np.array(ratios)
    assert np.all(ratios >= 1.0 - 1e-12)
    expect = 1.0 + 6 / (m - 6 - 1)
    assert 1.0 + 0.5 * (expect - 1.0) < ratios.mean() < 1.0 + 2.0 * (expect - 1.0)
