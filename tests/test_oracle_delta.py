"""Pins of the sketch perturbation delta = ||(C^ - C) R^{-1}||_2
(oracle.leverage.sketch_perturbation) and of the leverage-score bracket it
implies for Algorithm ls_approximate_drineas:
(1 + delta)^-2 <= theta^_i / theta~_i <= (1 - delta)^-2."""
import numpy as np
import pytest

import synth
from oracle import leverage as olev
from oracle import sketch as osk


def _orthonormal(m, d, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((m, d)))
    return q


def test_delta_zero_for_identical_sketch():
    c = np.random.default_rng(0).standard_normal((80, 12))
    assert olev.sketch_perturbation(c, c) == 0.0


@pytest.mark.parametrize("j,k,t", [(0, 0, 1e-3), (7, 3, -0.25), (59, 11, 2.0)])
def test_delta_rank_one_closed_form(j, k, t):
    """C = Q diag(s) has R = diag(s); E = t u e_k^T gives E R^{-1} =
    (t / s_k) u e_k^T, so delta = |t| ||u|| / s_k exactly.  A transposed
    operand, R in place of R^{-1}, or the wrong column scale all miss it."""
    m, d = 60, 12
    q = _orthonormal(m, d, 1)
    s = np.logspace(0, -4, d)
    c = q * s[None, :]
    u = np.random.default_rng(j).standard_normal(m)
    e = t * np.outer(u, np.eye(d)[k])
    delta = olev.sketch_perturbation(c + e, c)
    assert delta == pytest.approx(abs(t) * np.linalg.norm(u) / s[k], rel=1e-10)


def test_delta_of_a_scaled_sketch():
    """C^ = (1 + x) C gives E R^{-1} = x Q, so delta = |x|; the scores of C^
    are theta~ / (1 + x)^2 exactly, the lower edge of the bracket."""
    a = synth.dense_gaussian(4000, 10, seed=2)
    c = osk.sketch_gcs(a, 60, 500, 3)
    for x in (0.1, -0.3):
        delta = olev.sketch_perturbation((1 + x) * c, c)
        assert delta == pytest.approx(abs(x), rel=1e-12)
    th = olev.leverage_from_sketch(a, c, 0, 3)
    th_hat = olev.leverage_from_sketch(a, 1.1 * c, 0, 3)
    np.testing.assert_allclose(th_hat / th, 1.1 ** -2, rtol=1e-12)


def test_delta_norm_inequalities_and_invariances():
    """||E|| / ||R|| <= delta <= ||E|| ||R^{-1}||; delta is unchanged by a left
    orthogonal factor (U C^, U C) and by a right upper-triangular one (C^ M,
    C M), under which R becomes U-free and R M."""
    rng = np.random.default_rng(4)
    m, d = 70, 9
    c = rng.standard_normal((m, d)) @ np.diag(np.logspace(0, -3, d))
    e = 1e-3 * rng.standard_normal((m, d))
    delta = olev.sketch_perturbation(c + e, c)
    r = olev.qr_r(c)
    ne = np.linalg.norm(e, 2)
    assert ne / np.linalg.norm(r, 2) <= delta * (1 + 1e-12)
    assert delta <= ne * np.linalg.norm(olev.tri_inv(r), 2) * (1 + 1e-12)
    u = _orthonormal(m, m, 5)
    assert olev.sketch_perturbation(u @ (c + e), u @ c) == pytest.approx(delta, rel=1e-9)
    mm = np.triu(rng.standard_normal((d, d))) + 3 * np.eye(d)
    assert olev.sketch_perturbation((c + e) @ mm, c @ mm) == pytest.approx(delta, rel=1e-8)


@pytest.mark.parametrize("scale", [1e-3, 3e-2, 0.2])
def test_leverage_bracket_holds(scale):
    """Random perturbations of a sketch: every row's score ratio lies inside
    [(1 + delta)^-2, (1 - delta)^-2], and the bracket is not slack by orders
    of magnitude (the extreme ratio reaches a fair part of it)."""
    a = synth.dense_coherent(3000, 16, seed=6, smin=1e-4)
    c = osk.sketch_gcs(a, 96, 800, 7)
    rng = np.random.default_rng(8)
    # a perturbation of size ~scale in the metric of C (E = N R, N Gaussian)
    e = scale * rng.standard_normal(c.shape) / np.sqrt(c.shape[0]) @ olev.qr_r(c)
    delta = olev.sketch_perturbation(c + e, c)
    assert 0 < delta < 1
    th = olev.leverage_from_sketch(a, c, 0, 7)
    ratio = olev.leverage_from_sketch(a, c + e, 0, 7) / th
    assert np.all(ratio <= (1 - delta) ** -2 * (1 + 1e-12))
    assert np.all(ratio >= (1 + delta) ** -2 * (1 - 1e-12))
    assert np.abs(ratio - 1).max() >= 0.05 * olev.leverage_ratio_bound(delta)


def test_delta_of_quantised_sketches_is_small():
    """The BF16 and FP8 operand formats perturb the sketch of a well-conditioned
    A by roughly their unit roundoff (BF16 2^-9 on G; FP8 e4m3 2^-4)."""
    a = synth.dense_gaussian(20000, 50, seed=0)
    c = osk.sketch_gcs(a, 200, 2500, 0)
    d16 = olev.sketch_perturbation(osk.sketch_gcs_bf16_reference(a, 200, 2500, 0), c)
    d8 = olev.sketch_perturbation(osk.sketch_gcs_fp8_reference(a, 200, 2500, 0), c)
    assert 1e-4 < d16 < 2e-2
    assert 1e-3 < d8 < 0.3
    assert d8 > 4 * d16
