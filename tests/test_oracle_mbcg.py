"""Pins of the textbook mBCG / SLQ oracle: solves, exact quadrature, spectra, unbiasedness."""
import itertools
import math

import numpy as np
import pytest
from scipy.linalg import eigh

from oracle import exact, kernel as ok
from oracle.bbmm import mll_and_grad_estimate
from oracle.gradient import bilinear_forms
from oracle.mbcg import mbcg, quadrature_log, slq_logdet, tridiagonal
from oracle.pivchol import Preconditioner, pivoted_cholesky
from oracle.probes import probe_block


def _setup(n, d=3, seed=0, noise=1e-2, scale=2.0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    th = ok.Theta(scale * rng.uniform(0.5, 2.0, d), 1.0, noise)
    y = rng.standard_normal(n)
    return X, y, th


def _sym_funcs(K, P):
    """A = P^{-1/2} K P^{-1/2} and P^{-1/2} through eigen-decompositions."""
    w, V = eigh(P)
    Pmh = V @ np.diag(w ** -0.5) @ V.T
    A = Pmh @ K @ Pmh
    return A, Pmh


@pytest.mark.parametrize("k", [0, 6])
def test_solution_column_matches_cholesky(k):
    X, y, th = _setup(150)
    L, _, _ = pivoted_cholesky(X, th, k) if k else (np.zeros((150, 0)), None, None)
    P = Preconditioner(L, th.noise)
    B = probe_block(3, y, 4, L, th.noise)
    res = mbcg(lambda D: ok.khat_matmul(X, th, D), B, P.solve, 400, 1e-13)
    K = ok.khat(X, th)
    np.testing.assert_allclose(res["U"], np.linalg.solve(K, B), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(res["gamma0"], np.sum(B * np.linalg.solve(P.dense(), B), axis=0), rtol=1e-12)


def test_columns_are_independent_recurrences():
    # well conditioned, so that BLAS rounding differences between a 1-column and a
    # 4-column product stay at rounding level through the iterations
    X, y, th = _setup(90, seed=1, noise=0.2)
    L, _, _ = pivoted_cholesky(X, th, 5)
    P = Preconditioner(L, th.noise)
    B = probe_block(5, y, 3, L, th.noise)
    mm = lambda D: ok.khat_matmul(X, th, D)
    full = mbcg(mm, B, P.solve, 12, 0.0)
    for c in range(4):
        one = mbcg(mm, B[:, c:c + 1], P.solve, 12, 0.0)
        np.testing.assert_allclose(full["alpha"][:, c], one["alpha"][:, 0], rtol=1e-9)
        np.testing.assert_allclose(full["beta"][:, c], one["beta"][:, 0], rtol=1e-9)
        np.testing.assert_allclose(full["U"][:, c], one["U"][:, 0], rtol=0,
                                   atol=1e-9 * np.abs(one["U"]).max())


@pytest.mark.parametrize("k", [0, 3])
def test_quadrature_is_exact_at_full_krylov_dimension(k):
    # Gauss quadrature of log is exact once the Krylov space is complete.  With a
    # rank-k pivoted-Cholesky preconditioner, A - I = P^{-1/2} (K - L L^T) P^{-1/2} has
    # rank N - k (the Nystrom residual vanishes on the pivots), so A has the eigenvalue 1
    # k times and N - k + 1 distinct eigenvalues: that is the Krylov dimension.
    n = 10
    X, y, th = _setup(n, seed=2, noise=0.05, scale=1.0)
    L, _, _ = pivoted_cholesky(X, th, k) if k else (np.zeros((n, 0)), None, None)
    P = Preconditioner(L, th.noise)
    J = n - k + 1 if k else n
    B = probe_block(11, y, 5, L, th.noise)
    res = mbcg(lambda D: ok.khat_matmul(X, th, D), B, P.solve, J, 0.0)
    K = ok.khat(X, th)
    A, Pmh = _sym_funcs(K, P.dense())
    wA, VA = eigh(A)
    logA = VA @ np.diag(np.log(wA)) @ VA.T
    distinct = np.unique(np.round(wA, 9))
    assert distinct.shape[0] == J
    for c in range(6):
        assert res["iters"][c] == J
        z = Pmh @ B[:, c]
        exact_q = z @ logA @ z
        est = res["gamma0"][c] * quadrature_log(res["alpha"][:, c], res["beta"][:, c], J)
        assert abs(est - exact_q) < 1e-8 * max(1.0, abs(exact_q)), (c, est, exact_q)
        # the Ritz values of the complete tridiagonal are the distinct eigenvalues of A
        dg, off = tridiagonal(res["alpha"][:, c], res["beta"][:, c], J)
        T = np.diag(dg) + np.diag(off, 1) + np.diag(off, -1)
        np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(T)), distinct, rtol=1e-7)


def test_ritz_values_inside_spectrum():
    n = 120
    X, y, th = _setup(n, seed=3)
    L, _, _ = pivoted_cholesky(X, th, 8)
    P = Preconditioner(L, th.noise)
    B = probe_block(2, y, 4, L, th.noise)
    res = mbcg(lambda D: ok.khat_matmul(X, th, D), B, P.solve, 15, 0.0)
    A, _ = _sym_funcs(ok.khat(X, th), P.dense())
    lo, hi = np.linalg.eigvalsh(A)[[0, -1]]
    for c in range(5):
        dg, off = tridiagonal(res["alpha"][:, c], res["beta"][:, c], int(res["iters"][c]))
        T = np.diag(dg) + np.diag(off, 1) + np.diag(off, -1)
        ev = np.linalg.eigvalsh(T)
        assert ev.min() >= lo * (1 - 1e-9) and ev.max() <= hi * (1 + 1e-9)


def test_estimators_unbiased_by_enumeration():
    # Average the log-det and trace estimates over every sign pattern of (eps1, eps2):
    # the means equal log|K_hat| and tr(K_hat^{-1} dK_hat) exactly.
    n, k = 7, 2
    X, y, th = _setup(n, seed=4, noise=0.1, scale=1.0)
    L, _, _ = pivoted_cholesky(X, th, k)
    P = Preconditioner(L, th.noise)
    pats = np.array(list(itertools.product((-1.0, 1.0), repeat=n + k)))
    Bp = (L @ pats[:, :k].T) + math.sqrt(th.noise) * pats[:, k:].T  # (n, 2^(n+k))
    B = np.concatenate([y[:, None], Bp], axis=1)
    res = mbcg(lambda D: ok.khat_matmul(X, th, D), B, P.solve, n, 0.0)
    t = Bp.shape[1]
    ld = slq_logdet(res, P.logdet, range(1, t + 1))
    assert abs(ld - np.linalg.slogdet(ok.khat(X, th))[1]) < 1e-8
    K = ok.khat(X, th)
    Kinv = np.linalg.inv(K)
    for j, Dj in exact.dkhat_all(X, th):
        tr_est = np.mean(np.sum(res["U"][:, 1:] * (Dj @ res["Z0"][:, 1:]), axis=0))
        assert abs(tr_est - np.trace(Kinv @ Dj)) < 1e-8 * max(1.0, abs(np.trace(Kinv @ Dj)))


def test_bilinear_forms_match_finite_differences():
    X, y, th = _setup(70, d=4, seed=5)
    rng = np.random.default_rng(0)
    U = rng.standard_normal((70, 3))
    V = rng.standard_normal((70, 3))
    w = np.array([0.5, -0.25, 0.7])
    g = bilinear_forms(X, th, U, V, w, block=32)
    v = th.log_vector()
    h = 1e-5

    def F(vec):
        t2 = ok.Theta.from_log(vec, th.kind)
        return float(np.sum(w * np.sum(U * ok.khat_matmul(X, t2, V), axis=0)))

    for j in range(v.shape[0]):
        vp = v.copy(); vp[j] += h
        vm = v.copy(); vm[j] -= h
        fd = (F(vp) - F(vm)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 * max(abs(g[j]), 1e-3 * np.abs(g).max()), (j, fd, g[j])


def test_pipeline_estimate_close_to_exact_with_many_probes():
    n = 200
    X, y, th = _setup(n, d=3, seed=6, noise=0.02)
    t = 400
    est = mll_and_grad_estimate(X, y, th, t=t, k=10, seed=17, max_iter=300, tol=1e-12)
    ex = exact.cholesky_gp(X, y, th)
    assert abs(est["quad"] - ex["quad"]) < 1e-8 * abs(ex["quad"])
    res = est["res"]
    per = np.array([res["gamma0"][c] * quadrature_log(res["alpha"][:, c], res["beta"][:, c], int(res["iters"][c]))
                    for c in range(1, t + 1)])
    se = per.std(ddof=1) / math.sqrt(t)
    assert abs(est["logdet"] - ex["logdet"]) < 5 * se + 1e-9
    g_ex = exact.mll_grad(X, y, th)
    # stochastic gradient: loose statistical agreement on the dominant entries
    assert np.linalg.norm(est["grad"] - g_ex) < 0.1 * np.linalg.norm(g_ex)
