"""Pins of the dense oracle: library routines, brute force, closed forms, finite differences."""
import math

import numpy as np
import pytest

from oracle import exact, kernel as ok


def _problem(n, d, seed, kind=ok.MATERN52, noise=1e-2, scale=1.0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    th = ok.Theta(scale * rng.uniform(0.5, 2.0, d), 1.1, noise, kind)
    y = rng.standard_normal(n)
    return X, y, th


def test_solve_brute_force_inverse():
    X, y, th = _problem(8, 3, 0)
    res = exact.cholesky_gp(X, y, th)
    K = ok.khat(X, th)
    np.testing.assert_allclose(res["omega"], np.linalg.inv(K) @ y, rtol=1e-10)
    np.testing.assert_allclose(res["omega"], np.linalg.solve(K, y), rtol=1e-12)


def test_logdet_three_ways():
    X, y, th = _problem(60, 4, 1)
    res = exact.cholesky_gp(X, y, th)
    K = ok.khat(X, th)
    sign, ld = np.linalg.slogdet(K)
    assert sign > 0
    assert abs(res["logdet"] - ld) < 1e-10 * abs(ld) + 1e-10
    assert abs(res["logdet"] - np.sum(np.log(np.linalg.eigvalsh(K)))) < 1e-9


def test_mll_closed_form_when_kernel_is_scaled_identity():
    rng = np.random.default_rng(2)
    n = 40
    X = rng.standard_normal((n, 3)) * 100.0
    th = ok.Theta(np.full(3, 1e-3), 0.8, 0.3)
    y = rng.standard_normal(n)
    res = exact.cholesky_gp(X, y, th)
    s = th.sf + th.noise
    ref = -0.5 * (y @ y) / s - 0.5 * n * math.log(s) - 0.5 * n * math.log(2 * math.pi)
    assert abs(res["mll"] - ref) < 1e-12 * abs(ref)
    # d/dlog sigma^2 of the same closed form: sigma^2 (1/2 |y|^2 / s^2 - n / (2 s))
    g = exact.mll_grad(X, y, th)
    ref_g = th.noise * (0.5 * (y @ y) / s ** 2 - 0.5 * n / s)
    assert abs(g[-1] - ref_g) < 1e-11 * abs(ref_g)
    ref_gs = th.sf * (0.5 * (y @ y) / s ** 2 - 0.5 * n / s)
    assert abs(g[-2] - ref_gs) < 1e-11 * abs(ref_gs)
    np.testing.assert_allclose(g[:-2], 0.0, atol=1e-300)


@pytest.mark.parametrize("kind", [ok.MATERN52, ok.RBF])
def test_gradient_matches_central_differences(kind):
    X, y, th = _problem(48, 4, 3, kind=kind, scale=2.0)
    g = exact.mll_grad(X, y, th)
    v = th.log_vector()
    h = 1e-4
    for j in range(v.shape[0]):
        vp = v.copy(); vp[j] += h
        vm = v.copy(); vm[j] -= h
        fp = exact.cholesky_gp(X, y, ok.Theta.from_log(vp, kind))["mll"]
        fm = exact.cholesky_gp(X, y, ok.Theta.from_log(vm, kind))["mll"]
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(abs(g[j]), 1e-3 * np.abs(g).max()), (j, fd, g[j])


def test_predictive_variance_from_joint_precision():
    # For one query point, var = 1 / (Sigma_joint^{-1})_qq where Sigma_joint is the
    # prior covariance of (f(x'), y): a different route than the Schur complement.
    X, y, th = _problem(30, 3, 4, scale=1.5)
    rng = np.random.default_rng(5)
    Xq = rng.standard_normal((5, 3))
    mean, var = exact.predict(X, y, Xq, th)
    for q in range(5):
        Z = np.vstack([Xq[q:q + 1], X])
        S = ok.kernel(Z, Z, th)
        S[1:, 1:] += th.noise * np.eye(30)
        prec = np.linalg.inv(S)
        assert abs(var[q] - 1.0 / prec[0, 0]) < 1e-9
        # conditional mean from the precision: -prec_qy y / prec_qq
        assert abs(mean[q] - (-(prec[0, 1:] @ y) / prec[0, 0])) < 1e-8
    assert np.all(var >= -1e-12)


def test_prediction_at_training_points_small_noise():
    X, y, th = _problem(20, 3, 6, noise=1e-8)
    mean, var = exact.predict(X, y, X, th)
    np.testing.assert_allclose(mean, y, atol=1e-5)
    assert np.all(var < 1e-6)
