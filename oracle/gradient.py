"""Oracle: bilinear forms of the kernel-matrix derivatives.  Test infrastructure only.

For hyperparameters theta = (l_1..l_d, s_f, sigma^2), taken in logs,

    g_j = sum_c w_c  u_c^T (dK_hat / dlog theta_j) v_c

with
    dK_ab/dlog l_j   = psi(r_ab) ((x_aj - x_bj)/l_j)^2
    dK_hat/dlog s_f  = K                 (diagonal entries s_f included)
    dK_hat/dlog sig2 = sigma^2 I.

The gradient of the log marginal likelihood (Eq. 2) is one such form:
    U = [u_0, u_1..u_t],  V = [u_0, z0_1..z0_t],  w = [1/2, -1/(2t), ..]
where u_0 = K_hat^{-1} y and the other columns are the probe solves and
preconditioned probes of mBCG.  Differences are direct, block by block.
"""
from __future__ import annotations

import numpy as np

from .kernel import Theta, profile_of_r2, psi_of_r2, sqdist


def bilinear_forms(X, th: Theta, U: np.ndarray, V: np.ndarray, w, block: int = 128, rows=None) -> np.ndarray:
    """The d + 2 forms; ``rows = (start, stop)`` restricts the outer sum to rows a in that range
    (the forms over a partition of the rows add up to the whole)."""
    X = np.asarray(X)
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, d = X.shape
    r0, r1 = (0, n) if rows is None else (int(rows[0]), int(rows[1]))
    Xs = X / th.ell
    g = np.zeros(d + 2)
    for s in range(r0, r1, block):
        a = slice(s, min(s + block, r1))
        r2 = sqdist(X[a], X, th.ell)
        C = (U[a] * w) @ V.T  # C_ab = sum_c w_c U_ac V_bc
        K = th.sf * profile_of_r2(r2, th.kind)
        M = psi_of_r2(r2, th) * C
        diff = Xs[a][:, None, :] - Xs[None, :, :]
        g[:d] += np.einsum("ab,abj->j", M, diff * diff)
        g[d] += float(np.sum(K * C))
    g[d + 1] = th.noise * float(np.sum(w * np.sum(U[r0:r1] * V[r0:r1], axis=0)))
    return g


def mll_gradient_forms(U: np.ndarray, Z0: np.ndarray, t: int):
    """The (U, V, w) triple whose bilinear forms are the stochastic mll gradient."""
    V = np.concatenate([U[:, :1], Z0[:, 1:t + 1]], axis=1)
    w = np.concatenate([[0.5], np.full(t, -0.5 / t)])
    return U[:, :t + 1], V, w
