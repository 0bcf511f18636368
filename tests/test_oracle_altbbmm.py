"""Pins of the AltBBMM oracle (block CG, symmetric Nystrom preconditioner)."""
import numpy as np
import pytest

import oracle.kernel as ok
from oracle import altbbmm as ab
from oracle import mbcg as om


def _problem(n=160, d=4, seed=0, noise=1e-2):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)) * 1.5
    th = ok.Theta(rng.uniform(0.8, 2.0, d), 1.0, noise)
    return X, th, rng


def _spd(n, rng, cond=1e3):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T


def test_block_cg_reaches_the_dense_solve():
    rng = np.random.default_rng(1)
    A = _spd(80, rng)
    B = rng.standard_normal((80, 6))
    r = ab.block_cg(lambda D: A @ D, B, 1e-12, 200)
    ref = np.linalg.solve(A, B)
    assert np.all(r["relres"] <= 1e-12)
    np.testing.assert_allclose(r["X"], ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_block_cg_with_one_column_is_cg():
    """s = 1: block CG's alpha and beta are CG's step sizes (the unpreconditioned mBCG column)."""
    rng = np.random.default_rng(2)
    A = _spd(60, rng, 1e2)
    b = rng.standard_normal((60, 1))
    r = ab.block_cg(lambda D: A @ D, b, 1e-10, 100)
    c = om.mbcg(lambda D: A @ D, b, lambda R: R, 100, 1e-10)
    # the same scalars in a different rounding order: equal while the Krylov basis is still orthogonal
    got = np.array([a[0, 0] for a in r["alphas"][:10]])
    np.testing.assert_allclose(got, c["alpha"][:10, 0], rtol=1e-9)
    np.testing.assert_allclose(r["X"][:, 0], c["U"][:, 0], rtol=0, atol=1e-8 * np.abs(c["U"]).max())


def test_block_krylov_error_never_exceeds_cg():
    """Column 0 of block CG minimises the A-norm error over a space that contains CG's Krylov space."""
    rng = np.random.default_rng(3)
    A = _spd(120, rng, 1e4)
    B = rng.standard_normal((120, 5))
    x = np.linalg.solve(A, B[:, 0])

    def anorm(e):
        return float(np.sqrt(e @ A @ e))

    for k in range(1, 12):
        blk = ab.block_cg(lambda D: A @ D, B, 0.0, k)
        cg = ab.block_cg(lambda D: A @ D, B[:, :1], 0.0, k)
        assert anorm(blk["X"][:, 0] - x) <= anorm(cg["X"][:, 0] - x) * (1 + 1e-8) + 1e-12


def test_nystrom_interpolates_the_landmark_rows_and_bounds_k_from_below():
    X, th, rng = _problem()
    M = rng.choice(X.shape[0], 25, replace=False)
    P = ab.nystrom_matrix(X, th, M)
    K = ok.kernel(X, X, th)
    Q = P - th.noise * np.eye(X.shape[0])
    np.testing.assert_allclose(Q[M], K[M], rtol=0, atol=1e-10)  # K_XM K_MM^-1 K_MX reproduces rows M
    assert np.linalg.eigvalsh(K - Q).min() >= -1e-10             # Schur complement: K - Q is PSD


def test_symmetric_preconditioned_spectrum():
    """P^{-1/2} P P^{-1/2} = I; P^{-1/2} K_hat P^{-1/2} = I + P^{-1/2}(K - Q)P^{-1/2} has every eigenvalue >= 1
    and the eigenvalue 1 with multiplicity at least r."""
    X, th, rng = _problem(seed=4)
    r = 30
    M = rng.choice(X.shape[0], r, replace=False)
    P = ab.nystrom_matrix(X, th, M)
    S = ab.inv_sqrt(P)
    np.testing.assert_allclose(S @ P @ S, np.eye(X.shape[0]), rtol=0, atol=1e-9)
    ev = np.linalg.eigvalsh(S @ ok.khat(X, th) @ S)
    assert ev.min() >= 1 - 1e-9
    assert np.sum(np.abs(ev - 1) < 1e-7) >= r


def test_altbbmm_solution_and_iteration_bound():
    """The unpreconditioned solution equals the dense solve; with r landmarks the preconditioned operator has
    at most n - r + 1 distinct eigenvalues, so block CG ends within ceil((n - r + 1) / s) iterations in exact
    arithmetic (allow two more for rounding)."""
    X, th, rng = _problem(n=120, seed=5, noise=1e-3)
    s = 6
    B = np.column_stack([rng.standard_normal(120), rng.standard_normal((120, s - 1))])
    ref = np.linalg.solve(ok.khat(X, th), B)
    plain = ab.altbbmm_solve(X, th, B, None, 1e-11, 500)
    np.testing.assert_allclose(plain["W"], ref, rtol=0, atol=1e-7 * np.abs(ref).max())
    r = 60
    M = rng.choice(120, r, replace=False)
    pre = ab.altbbmm_solve(X, th, B, M, 1e-11, 500)
    np.testing.assert_allclose(pre["W"], ref, rtol=0, atol=1e-7 * np.abs(ref).max())
    assert pre["iters"] <= -(-(120 - r + 1) // s) + 2
    assert pre["iters"] < plain["iters"]


def test_truncated_nystrom_keeps_the_bounds_and_matches_when_nothing_is_dropped():
    """The pseudo-inverse form drops only directions of K_MM below rcond * lambda_max: it equals the
    exact form on a well-conditioned K_MM, and with a nearly repeated landmark it stays a lower bound
    of K (K - Q PSD), so the preconditioned spectrum stays >= 1."""
    X, th, rng = _problem(seed=6)
    M = rng.choice(X.shape[0], 20, replace=False)
    np.testing.assert_allclose(ab.nystrom_matrix(X, th, M, 1e-7), ab.nystrom_matrix(X, th, M), rtol=0, atol=1e-9)
    X2 = np.vstack([X, X[M[:3]] + 1e-7])  # three landmarks repeated to 1e-7
    M2 = np.concatenate([M, X.shape[0] + np.arange(3)])
    P = ab.nystrom_matrix(X2, th, M2, 1e-7)
    Q = P - th.noise * np.eye(X2.shape[0])
    K = ok.kernel(X2, X2, th)
    assert np.linalg.eigvalsh(K - Q).min() >= -1e-9
    S = ab.inv_sqrt(P)
    assert np.linalg.eigvalsh(S @ ok.khat(X2, th) @ S).min() >= 1 - 1e-7


def test_block_pcg_without_preconditioner_is_block_cg():
    rng = np.random.default_rng(11)
    A = _spd(70, rng, 1e2)
    B = rng.standard_normal((70, 5))
    a = ab.block_cg(lambda D: A @ D, B, 1e-10, 200)
    b = ab.block_pcg(lambda D: A @ D, B, lambda R: R.copy(), 1e-10, 200)
    assert a["iters"] == b["iters"]
    np.testing.assert_allclose(b["W"], a["X"], rtol=0, atol=1e-10 * np.abs(a["X"]).max())
    np.testing.assert_allclose(b["relres_hist"][:5], a["relres_hist"][:5], rtol=1e-8)


def test_block_pcg_is_block_cg_on_the_symmetric_system():
    """Left preconditioning with P^{-1} and block CG on P^{-1/2} A P^{-1/2} give the same iterates
    (W = P^{-1/2} X) and the same residual norms sqrt(r^T P^{-1} r) = ||P^{-1/2} r||."""
    rng = np.random.default_rng(12)
    n, s = 90, 4
    A = _spd(n, rng, 1e4)
    P = _spd(n, rng, 1e2)
    B = rng.standard_normal((n, s))
    S = ab.inv_sqrt(P)
    sym = ab.block_cg(lambda D: S @ (A @ (S @ D)), S @ B, 1e-9, 300)
    left = ab.block_pcg(lambda D: A @ D, B, lambda R: np.linalg.solve(P, R), 1e-9, 300)
    # equal in exact arithmetic; rounding separates the two Krylov bases only late in the run
    k = 6
    np.testing.assert_allclose(left["relres_hist"][:k], sym["relres_hist"][:k], rtol=1e-7)
    for j in range(k):
        np.testing.assert_allclose(left["alphas"][j], sym["alphas"][j], rtol=1e-6, atol=1e-9)
    assert abs(left["iters"] - sym["iters"]) <= 0.1 * sym["iters"]
    ref = np.linalg.solve(A, B)
    for W in (left["W"], S @ sym["X"]):
        assert np.max(np.abs(W - ref)) <= 1e-9 * np.linalg.cond(A) * np.abs(ref).max()


def test_block_pcg_reaches_the_dense_solve():
    X, th, rng = _problem(n=220, d=3, noise=1e-3)
    th = ok.Theta(th.ell * 3.0, th.sf, th.noise)  # correlated: an ill-conditioned K_hat
    Kh = ok.khat(X, th)
    B = rng.standard_normal((220, 6))
    M = np.sort(rng.choice(220, 40, replace=False))
    P = ab.nystrom_matrix_jitter(X, th, M)
    plain = ab.block_pcg(lambda D: Kh @ D, B, lambda R: R.copy(), 1e-10, 500)
    pre = ab.block_pcg(lambda D: Kh @ D, B, lambda R: np.linalg.solve(P, R), 1e-10, 500)
    ref = np.linalg.solve(Kh, B)
    kappa = np.linalg.cond(Kh)
    for r in (plain, pre):
        assert np.all(r["relres"] <= 1e-10)
        assert np.max(np.abs(r["W"] - ref)) <= 1e-9 * kappa * np.abs(ref).max()
    assert pre["iters"] < plain["iters"]


def test_jittered_nystrom_bounds_and_limits():
    """delta -> 0 recovers the plain Nystrom matrix; with delta > 0 the approximation stays below K
    (K_hat - P positive semidefinite) and above sigma^2 I; the large-rank factor identity
    P^{-1} = sigma^{-2} (I - E E^T), E = F L_G^{-T}, F = K_XM L_M^{-T}, holds."""
    X, th, rng = _problem(n=150, d=4, noise=1e-2)
    M = np.sort(rng.choice(150, 30, replace=False))
    P0 = ab.nystrom_matrix(X, th, M)
    np.testing.assert_allclose(ab.nystrom_matrix_jitter(X, th, M, 0.0), P0, rtol=0, atol=1e-10)
    P = ab.nystrom_matrix_jitter(X, th, M, 1e-4)
    Kh = ok.khat(X, th)
    assert np.linalg.eigvalsh(Kh - P).min() >= -1e-10
    assert np.linalg.eigvalsh(P).min() >= th.noise * (1 - 1e-10)
    assert np.linalg.eigvalsh(P0 - P).min() >= -1e-10  # a larger shift gives a smaller approximation
    # the factor form of the inverse
    KXM = ok.kernel(X, X[M], th)
    delta = 1e-4 * M.shape[0] * th.sf
    LM = np.linalg.cholesky(KXM[M] + delta * np.eye(M.shape[0]))
    F = np.linalg.solve(LM, KXM.T).T
    LG = np.linalg.cholesky(F.T @ F + th.noise * np.eye(M.shape[0]))
    E = np.linalg.solve(LG, F.T).T
    Pinv = (np.eye(150) - E @ E.T) / th.noise
    np.testing.assert_allclose(Pinv @ P, np.eye(150), rtol=0, atol=1e-9)
    assert np.linalg.eigvalsh(E.T @ E).max() < 1.0
