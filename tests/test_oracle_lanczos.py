"""Pins of the Lanczos variance cache: one-sided bound, exactness at full rank, orthogonality."""
import numpy as np

from oracle import exact, kernel as ok
from oracle.lanczos import cached_variance, lanczos, variance_cache


def _setup(n=60, d=3, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    th = ok.Theta(rng.uniform(1.0, 3.0, d), 1.0, 1e-2)
    y = rng.standard_normal(n)
    Xq = rng.standard_normal((25, d))
    return X, y, th, Xq


def test_basis_orthonormal_and_tridiagonal():
    X, y, th, _ = _setup()
    Q, a, b = lanczos(lambda v: ok.khat_matmul(X, th, v), y, 20)
    np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-12)
    T = Q.T @ ok.khat(X, th) @ Q
    ref = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    np.testing.assert_allclose(T, ref, atol=1e-10)


def test_cached_variance_upper_bounds_exact_and_is_exact_at_full_rank():
    X, y, th, Xq = _setup()
    mm = lambda v: ok.khat_matmul(X, th, v)
    _, var_ex = exact.predict(X, y, Xq, th)
    R = variance_cache(mm, y, 15)
    v15 = cached_variance(Xq, X, th, R)
    assert np.all(v15 >= var_ex - 1e-10)
    R_full = variance_cache(mm, y, X.shape[0])
    np.testing.assert_allclose(cached_variance(Xq, X, th, R_full), var_ex, atol=1e-8)
