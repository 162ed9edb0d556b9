"""Pins of the oracle's column subset selection (Algorithm cgrrqr) and the
leverage scores of the selected columns (Algorithm ls_hrn_exact): LAPACK's
column-pivoted QR (geqp3), the selection's definition by projections on tiny
inputs, rank-revealing and zero-column cases, and the exact leverage scores
when k = rank(A)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import css as ocss
from oracle import leverage as olev


def _scaled(m, d, seed, spread=1e3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, d)) * np.logspace(0, -np.log10(spread), d)[
        rng.permutation(d)]


@pytest.mark.parametrize("m,d,seed", [(40, 12, 1), (300, 100, 2), (64, 64, 3)])
def test_qrcp_matches_lapack_geqp3(m, d, seed):
    b = _scaled(m, d, seed)
    piv, rdiag = ocss.qrcp_pivots(b)
    r, pl = sla.qr(b, pivoting=True, mode="r")
    np.testing.assert_array_equal(piv, pl)
    np.testing.assert_allclose(rdiag, np.abs(np.diag(r)), rtol=1e-10)


def test_qrcp_matches_selection_by_projection():
    for seed in range(6):
        b = np.random.default_rng(seed).standard_normal((9, 6)) * [1, 3, 0.5, 2, 1.5, 0.7]
        np.testing.assert_array_equal(ocss.qrcp_pivots(b)[0],
                                      ocss.qrcp_pivots_by_projection(b))
    b = _scaled(20, 8, 9)
    np.testing.assert_array_equal(ocss.qrcp_pivots(b, 5)[0],
                                  ocss.qrcp_pivots_by_projection(b, 5))


def test_qrcp_replay_accepts_its_own_pivots_and_flags_others():
    b = _scaled(60, 15, 7)
    piv, rdiag = ocss.qrcp_pivots(b)
    took, best = ocss.qrcp_replay(b, piv)
    np.testing.assert_allclose(took, best, rtol=1e-13)
    np.testing.assert_allclose(np.sqrt(took), rdiag, rtol=1e-13)
    bad = piv.copy()
    bad[[2, 3]] = bad[[3, 2]]
    took, best = ocss.qrcp_replay(b, bad)
    assert took[2] < best[2] * (1 - 1e-6)


def test_qrcp_reveals_rank_and_orders_the_diagonal():
    rng = np.random.default_rng(4)
    base = rng.standard_normal((50, 5))
    b = np.hstack([base, base @ rng.standard_normal((5, 7))])  # rank 5, d = 12
    piv, rdiag = ocss.qrcp_pivots(b)
    assert np.all(np.diff(rdiag) <= 1e-12 * rdiag[0])
    assert rdiag[4] > 1e-3 * rdiag[0] and rdiag[5] < 1e-12 * rdiag[0]
    assert np.linalg.matrix_rank(b[:, piv[:5]]) == 5


def test_qrcp_zero_columns_come_last_in_index_order():
    b = np.random.default_rng(5).standard_normal((30, 8))
    b[:, [1, 4, 6]] = 0.0
    piv, rdiag = ocss.qrcp_pivots(b)
    np.testing.assert_array_equal(piv[5:], [1, 4, 6])
    assert np.all(rdiag[5:] == 0.0)
    # the first pivot is the column of largest norm
    assert piv[0] == int(np.argmax(np.linalg.norm(b, axis=0)))


def test_css_picks_the_dominant_columns():
    a = synth.dense_gaussian(5000, 30, seed=6)
    heavy = [3, 11, 17, 25]
    a[:, heavy] *= 100.0
    cols = ocss.css_select(a, 60, 900, 4, seed=2)
    assert sorted(cols.tolist()) == heavy


@pytest.mark.parametrize("sparse", [False, True])
def test_leverage_css_full_rank_is_exact(sparse):
    a = synth.csr_uniform(3000, 10, 0.4, seed=7) if sparse else \
        synth.dense_gaussian(3000, 10, seed=7)
    th, cols = ocss.leverage_css(a, 20, 100, 10, seed=1)
    assert sorted(cols.tolist()) == list(range(10))
    np.testing.assert_allclose(th, olev.leverage_exact(a), rtol=1e-10, atol=1e-15)


def test_leverage_css_subset_scores():
    a = synth.dense_gaussian(2000, 16, seed=8)
    th, cols = ocss.leverage_css(a, 32, 256, 6, seed=3)
    assert len(set(cols.tolist())) == 6
    assert th.min() >= 0 and th.max() <= 1 + 1e-12
    assert abs(th.sum() - 6) < 1e-10
    # the scores of A[:, K] are those of its orthonormal basis, not of A
    q, _ = np.linalg.qr(a[:, cols])
    np.testing.assert_allclose(th, (q ** 2).sum(axis=1), rtol=1e-12, atol=1e-16)
