"""Pins of the oracle's pivoted Cholesky and preconditioner."""
import numpy as np

from oracle import kernel as ok
from oracle.pivchol import Preconditioner, pivoted_cholesky


def _setup(n=80, d=3, seed=0, noise=1e-2):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    th = ok.Theta(rng.uniform(1.0, 3.0, d), 1.2, noise)
    return X, th


def test_first_pivot_is_row_zero_and_pivots_distinct():
    X, th = _setup()
    L, piv, _ = pivoted_cholesky(X, th, 12)
    assert piv[0] == 0
    assert len(set(piv)) == len(piv) == 12


def test_factor_is_nystrom_on_its_pivots():
    # L L^T = K[:, pi] K[pi, pi]^{-1} K[pi, :], an exact identity of the greedy factor.
    X, th = _setup()
    L, piv, _ = pivoted_cholesky(X, th, 10)
    K = ok.kernel(X, X, th)
    ny = K[:, piv] @ np.linalg.solve(K[np.ix_(piv, piv)], K[piv, :])
    np.testing.assert_allclose(L @ L.T, ny, atol=1e-10)


def test_residual_diagonal_and_monotone_trace():
    X, th = _setup()
    K = ok.kernel(X, X, th)
    prev = np.inf
    for k in range(0, 16, 3):
        L, piv, delta = pivoted_cholesky(X, th, k) if k else (np.zeros((80, 0)), [], np.full(80, th.sf))
        np.testing.assert_allclose(delta, np.diag(K - L @ L.T), atol=1e-12)
        assert delta.sum() <= prev + 1e-12
        prev = delta.sum()


def test_full_rank_reproduces_kernel():
    X, th = _setup(n=12)
    L, piv, _ = pivoted_cholesky(X, th, 12)
    np.testing.assert_allclose(L @ L.T, ok.kernel(X, X, th), atol=1e-10)


def test_breakdown_on_duplicate_rows_returns_lower_rank():
    X, th = _setup(n=10)
    Xd = np.vstack([X[:4], X[:4]])  # 4 distinct points, each twice
    L, piv, _ = pivoted_cholesky(Xd, th, 8)
    assert L.shape[1] == 4


def test_woodbury_solve_and_determinant_lemma():
    X, th = _setup(n=60)
    L, piv, _ = pivoted_cholesky(X, th, 9)
    P = Preconditioner(L, th.noise)
    dense = L @ L.T + th.noise * np.eye(60)
    R = np.random.default_rng(1).standard_normal((60, 4))
    np.testing.assert_allclose(P.solve(R), np.linalg.solve(dense, R), rtol=1e-9, atol=1e-9)
    sign, ld = np.linalg.slogdet(dense)
    assert sign > 0 and abs(P.logdet - ld) < 1e-9 * abs(ld)


def test_rank_zero_is_identity():
    P = Preconditioner(np.zeros((5, 0)), 0.1)
    R = np.arange(10.0).reshape(5, 2)
    np.testing.assert_array_equal(P.solve(R), R)
    assert P.logdet == 0.0


def test_forced_pivot_order_is_consistent():
    X, th = _setup()
    L, piv, _ = pivoted_cholesky(X, th, 7)
    L2, piv2, _ = pivoted_cholesky(X, th, 7, pivots=piv)
    assert piv2 == piv
    np.testing.assert_array_equal(L, L2)
