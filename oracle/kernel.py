"""Oracle: the ARD kernel, K_hat = K(X, X) + sigma^2 I, and matrix-free K_hat V.

Test infrastructure only (see the package docstring).

Kernel (paper Sec. 4 names the Matern-5/2 kernel; Sec. 2.2 defines
K_hat = K(X, X) + sigma^2 I below Eq. 1):

    r_ab^2 = sum_j ((x_aj - x_bj) / l_j)^2           (direct differences)
    Matern-5/2:  k(r) = s_f (1 + sqrt5 r + 5 r^2 / 3) exp(-sqrt5 r)
    RBF:         k(r) = s_f exp(-r^2 / 2)

Distances are taken by direct differences (``scipy.spatial.distance.cdist``),
never by the norm expansion ||a||^2 + ||b||^2 - 2 a.b, so that any error in
an expansion elsewhere shows up against this module.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial.distance import cdist

MATERN52 = 0
RBF = 1
SQRT5 = math.sqrt(5.0)


@dataclasses.dataclass(frozen=True)
class Theta:
    """Hyperparameters: ARD lengthscales, outputscale s_f, total noise sigma^2."""

    ell: np.ndarray
    sf: float
    noise: float
    kind: int = MATERN52

    @property
    def d(self) -> int:
        return int(np.asarray(self.ell).shape[0])

    def log_vector(self) -> np.ndarray:
        """(log l_1..log l_d, log s_f, log sigma^2)."""
        return np.concatenate([np.log(self.ell), [math.log(self.sf), math.log(self.noise)]])

    @staticmethod
    def from_log(v, kind=MATERN52) -> "Theta":
        v = np.asarray(v, dtype=np.float64)
        return Theta(np.exp(v[:-2]), float(math.exp(v[-2])), float(math.exp(v[-1])), kind)


def sqdist(Xa: np.ndarray, Xb: np.ndarray, ell) -> np.ndarray:
    """r^2 between rows of Xa and Xb after dividing each feature by its lengthscale."""
    ell = np.asarray(ell, dtype=np.float64)
    return cdist(np.asarray(Xa) / ell, np.asarray(Xb) / ell, "sqeuclidean")


def matern52_profile(r: np.ndarray) -> np.ndarray:
    """m(r) = (1 + sqrt5 r + 5 r^2/3) exp(-sqrt5 r); m(0) = 1."""
    s = SQRT5 * r
    return (1.0 + s + s * s / 3.0) * np.exp(-s)


def profile_of_r2(r2: np.ndarray, kind: int) -> np.ndarray:
    if kind == MATERN52:
        return matern52_profile(np.sqrt(np.maximum(r2, 0.0)))
    if kind == RBF:
        return np.exp(-0.5 * r2)
    raise ValueError(f"unknown kernel kind {kind}")


def kernel(Xa, Xb, th: Theta) -> np.ndarray:
    """K(Xa, Xb) = s_f m(r)."""
    return th.sf * profile_of_r2(sqdist(Xa, Xb, th.ell), th.kind)


def khat(X, th: Theta) -> np.ndarray:
    """Dense K_hat = K(X, X) + sigma^2 I."""
    K = kernel(X, X, th)
    K[np.diag_indices_from(K)] += th.noise
    return K


def khat_matmul(X, th: Theta, V: np.ndarray, rows=None, block: int = 1024) -> np.ndarray:
    """(K_hat V)[rows], never forming K_hat.  V is (n, t); returns (len(rows), t).

    Each block of output rows forms its kernel slab K(X[rows_blk], X) and
    multiplies it by V; rows of the identity part add sigma^2 V[row].
    """
    X = np.asarray(X)
    V = np.asarray(V, dtype=np.float64)
    squeeze = V.ndim == 1
    if squeeze:
        V = V[:, None]
    n = X.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.empty((rows.shape[0], V.shape[1]))
    for s in range(0, rows.shape[0], block):
        r = rows[s:s + block]
        out[s:s + block] = kernel(X[r], X, th) @ V + th.noise * V[r]
    return out[:, 0] if squeeze else out


def cross_matmul(Xq, X, th: Theta, V: np.ndarray, block: int = 1024) -> np.ndarray:
    """K(Xq, X) V without noise (the cross-covariance of the predictive equations)."""
    V = np.asarray(V, dtype=np.float64)
    squeeze = V.ndim == 1
    if squeeze:
        V = V[:, None]
    out = np.empty((Xq.shape[0], V.shape[1]))
    for s in range(0, Xq.shape[0], block):
        out[s:s + block] = kernel(Xq[s:s + block], X, th) @ V
    return out[:, 0] if squeeze else out


def dkernel_dlogell(Xa, Xb, th: Theta, j: int) -> np.ndarray:
    """d K(Xa, Xb) / d log l_j = psi(r) * ((x_aj - x_bj) / l_j)^2.

    Matern-5/2: psi(r) = (5/3) s_f (1 + sqrt5 r) exp(-sqrt5 r)  (from
    dm/dr = -(5/3) r (1 + sqrt5 r) exp(-sqrt5 r) and dr^2/dlog l_j = -2 (dx/l)^2);
    RBF: psi = k.
    """
    r2 = sqdist(Xa, Xb, th.ell)
    diff = (np.asarray(Xa)[:, j][:, None] - np.asarray(Xb)[:, j][None, :]) / th.ell[j]
    return psi_of_r2(r2, th) * diff * diff


def psi_of_r2(r2: np.ndarray, th: Theta) -> np.ndarray:
    if th.kind == MATERN52:
        r = np.sqrt(np.maximum(r2, 0.0))
        return (5.0 / 3.0) * th.sf * (1.0 + SQRT5 * r) * np.exp(-SQRT5 * r)
    return th.sf * np.exp(-0.5 * r2)
