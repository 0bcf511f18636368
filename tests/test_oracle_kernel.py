"""Pins of the oracle's kernel against independent library routines and closed forms."""
import math

import numpy as np
import pytest
from scipy.special import gamma as gamma_fn
from scipy.special import kv

from oracle import kernel as ok

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _theta(d, rng, kind=ok.MATERN52, sf=1.3, noise=1e-2):
    return ok.Theta(rng.uniform(0.5, 2.0, d), sf, noise, kind)


def test_matern_matches_sklearn():
    from sklearn.gaussian_process.kernels import Matern
    rng = np.random.default_rng(0)
    X = rng.standard_normal((40, 5))
    Z = rng.standard_normal((30, 5))
    th = _theta(5, rng, sf=1.0)
    ref = Matern(length_scale=th.ell, nu=2.5)(X, Z)
    np.testing.assert_allclose(ok.kernel(X, Z, th), ref, rtol=1e-13, atol=1e-15)


def test_rbf_matches_sklearn():
    from sklearn.gaussian_process.kernels import RBF
    rng = np.random.default_rng(1)
    X = rng.standard_normal((40, 5))
    th = _theta(5, rng, kind=ok.RBF, sf=1.0)
    ref = RBF(length_scale=th.ell)(X, X)
    np.testing.assert_allclose(ok.kernel(X, X, th), ref, rtol=1e-13, atol=1e-15)


def test_matern_matches_bessel_form():
    # General Matern: 2^(1-nu)/Gamma(nu) (sqrt(2 nu) r)^nu K_nu(sqrt(2 nu) r), nu = 5/2.
    nu = 2.5
    r = np.linspace(1e-3, 12.0, 257)
    z = math.sqrt(2 * nu) * r
    bessel = 2 ** (1 - nu) / gamma_fn(nu) * z ** nu * kv(nu, z)
    np.testing.assert_allclose(ok.matern52_profile(r), bessel, rtol=1e-11, atol=1e-300)
    assert ok.matern52_profile(np.array([0.0]))[0] == 1.0


def test_direct_differences_brute_force():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((6, 4))
    Z = rng.standard_normal((5, 4))
    ell = rng.uniform(0.5, 2, 4)
    got = ok.sqdist(X, Z, ell)
    for a in range(6):
        for b in range(5):
            s = 0.0
            for j in range(4):
                s += ((X[a, j] - Z[b, j]) / ell[j]) ** 2
            assert abs(got[a, b] - s) <= 1e-13 * max(1.0, s)


def test_khat_symmetric_psd_and_diagonal():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((120, 6))
    th = _theta(6, rng)
    K = ok.khat(X, th)
    assert np.array_equal(K, K.T)
    assert np.all(np.diag(K) == th.sf + th.noise)
    assert np.linalg.eigvalsh(K).min() >= th.noise - 1e-10


def test_matrix_free_product_equals_dense():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((300, 7))
    th = _theta(7, rng)
    V = rng.standard_normal((300, 3))
    dense = ok.khat(X, th) @ V
    np.testing.assert_allclose(ok.khat_matmul(X, th, V, block=64), dense, rtol=1e-12, atol=1e-12)
    rows = np.array([0, 5, 299, 17])
    np.testing.assert_allclose(ok.khat_matmul(X, th, V, rows=rows), dense[rows], rtol=1e-12, atol=1e-12)


def test_far_apart_points_reduce_to_scaled_identity():
    # Tiny lengthscales: every off-diagonal entry underflows, K_hat = (s_f + sigma^2) I.
    rng = np.random.default_rng(5)
    X = rng.standard_normal((50, 3))
    th = ok.Theta(np.full(3, 1e-4), 0.7, 0.05)
    np.testing.assert_array_equal(ok.khat(X, th), (0.7 + 0.05) * np.eye(50))


def test_derivative_against_finite_differences():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((20, 4))
    for kind in (ok.MATERN52, ok.RBF):
        th = _theta(4, rng, kind=kind)
        for j in range(4):
            h = 1e-5
            lp = th.ell.copy(); lp[j] *= math.exp(h)
            lm = th.ell.copy(); lm[j] *= math.exp(-h)
            fd = (ok.kernel(X, X, ok.Theta(lp, th.sf, th.noise, kind))
                  - ok.kernel(X, X, ok.Theta(lm, th.sf, th.noise, kind))) / (2 * h)
            np.testing.assert_allclose(ok.dkernel_dlogell(X, X, th, j), fd, rtol=1e-7, atol=1e-10)
