"""Oracle: Lanczos variance cache for predictive variances.  Test infrastructure only.

Predictive variances need K(x', X) K_hat^{-1} K(X, x') (paper Eq. 1).  A rank-k
Lanczos decomposition K_hat Q ~ Q T (Q orthonormal, T tridiagonal), started
from y / ||y||, gives K_hat^{-1} ~ Q T^{-1} Q^T on the Krylov space; with the
Cholesky factor T = L_T L_T^T the cache R = Q L_T^{-T} satisfies
R R^T = Q T^{-1} Q^T, so

    var(x') ~ k(x', x') - || K(x', X) R ||^2

(Pleiss et al., "Constant-time predictive distributions for Gaussian
processes", 2018).  Since Q T^{-1} Q^T <= K_hat^{-1} in the Loewner order,
the cached variance is never below the exact one, and equals it when the
Krylov space is the whole space.  Lanczos here keeps Q orthonormal with
full re-orthogonalisation against all previous vectors (twice).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import cholesky, solve_triangular

from .kernel import Theta, cross_matmul


def lanczos(matmul, q0: np.ndarray, k: int):
    """k steps of Lanczos with full re-orthogonalisation; returns (Q, diag, off)."""
    n = q0.shape[0]
    k = min(k, n)
    Q = np.zeros((n, k))
    a = np.zeros(k)
    b = np.zeros(k)
    q = q0 / np.linalg.norm(q0)
    m = 0
    for j in range(k):
        Q[:, j] = q
        w = matmul(q)
        a[j] = q @ w
        for _ in range(2):
            w = w - Q[:, :j + 1] @ (Q[:, :j + 1].T @ w)
        m = j + 1
        bj = np.linalg.norm(w)
        if j + 1 < k:
            if bj <= 1e-12 * abs(a[j]):
                break
            b[j] = bj
            q = w / bj
    return Q[:, :m], a[:m], b[:m - 1]


def variance_cache(matmul, y: np.ndarray, k: int) -> np.ndarray:
    """R = Q L_T^{-T} (n x k)."""
    Q, a, b = lanczos(matmul, y, k)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    LT = cholesky(T, lower=True)
    return solve_triangular(LT, Q.T, lower=True).T


def cached_variance(Xq, X, th: Theta, R: np.ndarray, add_noise: bool = False) -> np.ndarray:
    KR = cross_matmul(Xq, X, th, R)
    var = th.sf - np.sum(KR * KR, axis=1)
    return var + th.noise if add_noise else var
