"""Oracle: textbook modified batched preconditioned CG (mBCG) and SLQ.

Test infrastructure only.

mBCG (paper Sec. 3.2, after Gardner et al. 2018) runs s independent
preconditioned CG recurrences in lock-step on the block B = [y | b_1..b_t];
each column has its own step sizes, unlike block CG (the footnote of
Sec. 3.2 stresses the difference).  Per column c, from U = 0, R = B,
Z = P^{-1} R, D = Z, gamma = r.z:

    W     = K_hat D
    alpha = gamma / (d . w)
    U    += alpha D ;   R -= alpha W
    freeze c once ||r_c|| <= tol ||b_c||   (alpha_c = 0 afterwards)
    Z     = P^{-1} R ;  gamma' = r.z ;  beta = gamma' / gamma
    D     = Z + beta D ;  gamma = gamma'

Each column's coefficients define the Lanczos tridiagonal of the
preconditioned operator A = P^{-1/2} K_hat P^{-1/2} started from
P^{-1/2} b_c / ||P^{-1/2} b_c|| (the CG-Lanczos correspondence):

    T_00 = 1/alpha_0
    T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}
    T_j,j-1 = T_j-1,j = sqrt(beta_{j-1}) / alpha_{j-1}

Stochastic Lanczos quadrature then gives
    log|K_hat| ~ log|P| + (1/t) sum_c gamma0_c sum_m V_0m^2 log theta_m
with (theta, V) the eigenpairs of T_c and gamma0_c = b_c^T P^{-1} b_c, and the
trace term of the gradient is
    tr(K_hat^{-1} dK_hat) ~ (1/t) sum_c u_c^T dK_hat z0_c,  z0_c = P^{-1} b_c.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import eigh_tridiagonal


def mbcg(matmul, B: np.ndarray, precond, max_iter: int, tol: float) -> dict:
    """Run mBCG on the (n, s) block B.  ``matmul(D)`` returns K_hat D; ``precond(R)`` P^{-1} R."""
    B = np.asarray(B, dtype=np.float64)
    n, s = B.shape
    U = np.zeros((n, s))
    R = B.copy()
    Z = precond(R)
    Z0 = Z.copy()
    D = Z.copy()
    gamma = np.sum(R * Z, axis=0)
    gamma0 = gamma.copy()
    bnorm = np.linalg.norm(B, axis=0)
    active = bnorm > 0
    iters = np.zeros(s, dtype=np.int64)
    alphas, betas, hist = [], [], []
    relres = np.where(bnorm > 0, 1.0, 0.0)
    for j in range(max_iter):
        if not active.any():
            break
        W = matmul(D)
        delta = np.sum(D * W, axis=0)
        a = np.where(active, gamma / np.where(active, delta, 1.0), 0.0)
        U += D * a
        R -= W * a
        iters[active] = j + 1
        rn = np.linalg.norm(R, axis=0)
        relres = np.where(active, rn / np.where(bnorm > 0, bnorm, 1.0), relres)
        hist.append(relres.copy())
        alphas.append(a)
        active = active & ~(rn <= tol * bnorm)
        Z = precond(R)
        gnew = np.sum(R * Z, axis=0)
        b = np.where(active, gnew / gamma, 0.0)
        D = Z + D * b
        gamma = np.where(active, gnew, gamma)
        betas.append(b)
    J = len(alphas)
    return {
        "U": U,
        "Z0": Z0,
        "alpha": np.array(alphas).reshape(J, s),
        "beta": np.array(betas).reshape(J, s),
        "iters": iters,
        "relres": relres,
        "gamma0": gamma0,
        "relres_hist": np.array(hist).reshape(J, s),  # residual after each iteration (recording only)
    }


def tridiagonal(alpha: np.ndarray, beta: np.ndarray, J: int):
    """Diagonal and off-diagonal of T from one column's CG coefficients."""
    a = np.asarray(alpha[:J], dtype=np.float64)
    b = np.asarray(beta[:max(J - 1, 0)], dtype=np.float64)
    diag = 1.0 / a
    diag[1:] += b / a[:-1]
    off = np.sqrt(b) / a[:-1]
    return diag, off


def quadrature_log(alpha, beta, J: int) -> float:
    """e_1^T log(T) e_1 for one column."""
    diag, off = tridiagonal(alpha, beta, J)
    if J == 1:
        return math.log(diag[0])
    w, V = eigh_tridiagonal(diag, off)
    return float(np.sum(V[0, :] ** 2 * np.log(w)))


def slq_logdet(res: dict, logdet_p: float, cols) -> float:
    """log|K_hat| ~ log|P| + mean over probe columns of gamma0 e1^T log(T) e1."""
    vals = [res["gamma0"][c] * quadrature_log(res["alpha"][:, c], res["beta"][:, c], int(res["iters"][c]))
            for c in cols]
    return logdet_p + float(np.mean(vals))


def mll_from_solve(y: np.ndarray, u0: np.ndarray, logdet: float) -> float:
    n = y.shape[0]
    return -0.5 * float(y @ u0) - 0.5 * logdet - 0.5 * n * math.log(2.0 * math.pi)
