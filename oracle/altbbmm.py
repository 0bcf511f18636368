"""Oracle: AltBBMM, block CG with the symmetric Nystrom preconditioner, and block preconditioned CG.

Test infrastructure only.

Block conjugate gradients (Sec. 3.1) solve K_hat W = B for the s columns of
B = [y | y_1 .. y_{s-1}] at once (y_i ~ N(0, I)); after k iterations column i
is optimal over the block Krylov space span{K_hat^j y_l : l < s, j < k}, which
contains the single-vector space CG searches.  AltBBMM (Sec. 3.2) runs block
CG in FP64 on the symmetrically preconditioned system

    P^{-1/2} K_hat P^{-1/2} Z = P^{-1/2} B,     W = P^{-1/2} Z,

with the Nystrom preconditioner over r landmark rows M (Sec. 3.2, Sec. 4):

    P = K_XM K_MM^{-1} K_MX + sigma^2 I,

and stops when all s relative residuals are below the tolerance (1e-6 in
Sec. 4).  The inverse square root here is the plain definition: the
eigendecomposition of the dense P.

Block CG (O'Leary), from X = 0, R = B, D = R:
    Q     = A D
    alpha = (D^T Q)^{-1} (R^T R)          (s x s)
    X    += D alpha ;   R_new = R - Q alpha
    stop when ||R_new[:, c]|| <= tol ||B[:, c]|| for every c
    beta  = (R^T R)^{-1} (R_new^T R_new)  (s x s)
    D     = R_new + D beta ;   R = R_new
"""
from __future__ import annotations

import numpy as np

from .kernel import Theta, kernel, khat


def nystrom_matrix(X, th: Theta, landmarks, rcond: float = 0.0) -> np.ndarray:
    """Dense P = K_XM K_MM^{-1} K_MX + sigma^2 I for the landmark row indices M.  With rcond > 0 the
    inverse is the pseudo-inverse over the eigenvalues of K_MM above rcond * lambda_max (nearly
    repeated landmarks make K_MM numerically singular)."""
    M = np.asarray(landmarks, dtype=np.int64)
    KXM = kernel(X, X[M], th)
    KMM = KXM[M]
    if rcond > 0.0:
        lam, U = np.linalg.eigh(0.5 * (KMM + KMM.T))
        keep = lam > rcond * lam.max()
        C = U[:, keep] / np.sqrt(lam[keep])
        F = KXM @ C
        Q = F @ F.T
    else:
        Q = KXM @ np.linalg.solve(KMM, KXM.T)
    Q = 0.5 * (Q + Q.T)
    return Q + th.noise * np.eye(X.shape[0])


def inv_sqrt(P: np.ndarray) -> np.ndarray:
    """P^{-1/2} of a symmetric positive definite matrix from its eigendecomposition."""
    w, V = np.linalg.eigh(P)
    return (V / np.sqrt(w)) @ V.T


def block_cg(matmul, B: np.ndarray, tol: float, max_iter: int) -> dict:
    """Block CG on the SPD operator ``matmul`` for the (n, s) block B."""
    B = np.asarray(B, dtype=np.float64)
    n, s = B.shape
    X = np.zeros((n, s))
    R = B.copy()
    D = R.copy()
    RtR = R.T @ R
    bnorm = np.linalg.norm(B, axis=0)
    alphas, betas, hist = [], [], []
    relres = np.ones(s)
    iters = 0
    for k in range(max_iter):
        Q = matmul(D)
        alpha = np.linalg.solve(D.T @ Q, RtR)
        X = X + D @ alpha
        Rn = R - Q @ alpha
        iters = k + 1
        alphas.append(alpha)
        relres = np.linalg.norm(Rn, axis=0) / bnorm
        hist.append(relres.copy())
        if np.all(relres <= tol):
            R = Rn
            break
        RtRn = Rn.T @ Rn
        beta = np.linalg.solve(RtR, RtRn)
        betas.append(beta)
        D = Rn + D @ beta
        R, RtR = Rn, RtRn
    return {"X": X, "iters": iters, "relres": relres, "relres_hist": hist, "alphas": alphas, "betas": betas}


def nystrom_matrix_jitter(X, th: Theta, landmarks, jitter_rel: float = 1e-10) -> np.ndarray:
    """Dense P = K_XM (K_MM + delta I)^{-1} K_MX + sigma^2 I with delta = jitter_rel * r * s_f: the
    Nystrom approximation with the landmark Gram matrix regularised, as the large-rank
    preconditioner defines it (a shift of K_MM keeps its inverse bounded when landmark rows nearly
    repeat)."""
    M = np.asarray(landmarks, dtype=np.int64)
    KXM = kernel(X, X[M], th)
    KMM = KXM[M]
    delta = jitter_rel * M.shape[0] * th.sf
    Q = KXM @ np.linalg.solve(KMM + delta * np.eye(M.shape[0]), KXM.T)
    Q = 0.5 * (Q + Q.T)
    return Q + th.noise * np.eye(X.shape[0])


def block_pcg(matmul, B: np.ndarray, precond, tol: float, max_iter: int) -> dict:
    """Block preconditioned CG (O'Leary) on the SPD operator ``matmul`` with ``precond(R)`` = P^{-1} R,
    from W = 0, R = B, Z = P^{-1} R, D = Z:
        Q = A D;  alpha = (D^T Q)^{-1} (R^T Z);  W += D alpha;  R_new = R - Q alpha
        stop when sqrt(r_c^T P^{-1} r_c) <= tol sqrt(b_c^T P^{-1} b_c) for every column c
        Z_new = P^{-1} R_new;  beta = (R^T Z)^{-1} (R_new^T Z_new);  D = Z_new + D beta."""
    B = np.asarray(B, dtype=np.float64)
    n, s = B.shape
    W = np.zeros((n, s))
    R = B.copy()
    Z = precond(R)
    D = Z.copy()
    RtZ = R.T @ Z
    bnorm = np.sqrt(np.diag(RtZ))
    alphas, betas, hist = [], [], []
    relres = np.ones(s)
    iters = 0
    for k in range(max_iter):
        Q = matmul(D)
        alpha = np.linalg.solve(D.T @ Q, RtZ)
        W = W + D @ alpha
        Rn = R - Q @ alpha
        Zn = precond(Rn)
        RtZn = Rn.T @ Zn
        iters = k + 1
        alphas.append(alpha)
        relres = np.sqrt(np.maximum(np.diag(RtZn), 0.0)) / bnorm
        hist.append(relres.copy())
        if np.all(relres <= tol):
            break
        beta = np.linalg.solve(RtZ, RtZn)
        betas.append(beta)
        D = Zn + D @ beta
        R, Z, RtZ = Rn, Zn, RtZn
    return {"W": W, "iters": iters, "relres": relres, "relres_hist": hist, "alphas": alphas, "betas": betas}


def altbbmm_solve(X, th: Theta, B: np.ndarray, landmarks, tol: float, max_iter: int, rcond: float = 0.0) -> dict:
    """Block CG on P^{-1/2} K_hat P^{-1/2} (P Nystrom over ``landmarks``, or the identity when None)."""
    Kh = khat(X, th)
    S = np.eye(X.shape[0]) if landmarks is None else inv_sqrt(nystrom_matrix(X, th, landmarks, rcond))
    A = S @ Kh @ S
    res = block_cg(lambda D: A @ D, S @ B, tol, max_iter)
    res["W"] = S @ res["X"]
    res["Pinvsqrt"] = S
    return res
