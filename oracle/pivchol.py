"""Oracle: pivoted-Cholesky preconditioner.  Test infrastructure only.

BBMM preconditions CG with a partial pivoted Cholesky factor of the kernel
matrix (paper Sec. 3.2, citing Bach 2013 and Harbrecht et al. 2012).  The
greedy rank-k factor L of K (the noise-free kernel) is built one column at a
time:

    delta = diag(K)                       (= s_f for a stationary kernel)
    for m = 0..k-1:
        i = argmax delta over the unpivoted rows (ties: lowest index)
        stop if delta_i <= 1e-12 s_f      (numerical rank reached)
        L[:, m] = (K[:, i] - L[:, :m] L[i, :m]^T) / sqrt(delta_i)
        delta -= L[:, m]^2 ;  delta_i = 0

The preconditioner is P = L L^T + sigma^2 I.  With C = sigma^2 I_k + L^T L,
    P^{-1} R = sigma^{-2} (R - L C^{-1} L^T R)            (Woodbury)
    log|P|   = (N - k) log sigma^2 + log|C|               (determinant lemma)
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .kernel import Theta, kernel

BREAKDOWN_REL = 1e-12


def pivoted_cholesky(X, th: Theta, k: int, pivots=None):
    """Rank-<=k factor of K(X, X).  Returns (L (n x rank), pivots, final delta).

    ``pivots`` forces the pivot order (used when two equally valid orders exist
    because of near-ties in delta); the factor is then the one of that order.
    """
    X = np.asarray(X)
    n = X.shape[0]
    k = min(int(k), n)
    delta = np.full(n, th.sf, dtype=np.float64)
    L = np.zeros((n, k))
    piv = []
    for m in range(k):
        if pivots is not None:
            if m >= len(pivots):
                break
            i = int(pivots[m])
        else:
            cand = delta.copy()
            cand[piv] = -np.inf
            i = int(np.argmax(cand))  # first maximum = lowest index
            if cand[i] <= BREAKDOWN_REL * th.sf:
                break
        col = kernel(X, X[i:i + 1], th)[:, 0]
        l = (col - L[:, :m] @ L[i, :m]) / math.sqrt(delta[i])
        L[:, m] = l
        delta -= l * l
        delta[i] = 0.0
        piv.append(i)
    return L[:, :len(piv)], piv, delta


class Preconditioner:
    """P = L L^T + sigma^2 I (or P = I when the rank is 0)."""

    def __init__(self, L: np.ndarray, noise: float):
        self.L = np.asarray(L)
        self.noise = float(noise)
        n, k = self.L.shape
        self.n, self.k = n, k
        if k == 0:
            self.logdet = 0.0
            self.C = None
            return
        C = noise * np.eye(k) + self.L.T @ self.L
        self.C = cho_factor(C, lower=True)
        self.logdet = (n - k) * math.log(noise) + 2.0 * float(np.sum(np.log(np.diag(self.C[0]))))

    def solve(self, R: np.ndarray) -> np.ndarray:
        if self.k == 0:
            return np.array(R, dtype=np.float64, copy=True)
        return (R - self.L @ cho_solve(self.C, self.L.T @ R)) / self.noise

    def dense(self) -> np.ndarray:
        if self.k == 0:
            return np.eye(self.n)
        return self.L @ self.L.T + self.noise * np.eye(self.n)
