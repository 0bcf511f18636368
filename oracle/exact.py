"""Oracle: exact (dense Cholesky) GP quantities.  Test infrastructure only.

* omega = K_hat^{-1} y and the log marginal likelihood
      L = -1/2 y^T K_hat^{-1} y - 1/2 log|K_hat| - N/2 log 2 pi     (paper Eq. 2)
  through the Cholesky factorisation K_hat = L_c L_c^T (the O(N^3) route that
  the paper describes as limiting exact GPs to ~50k points, Sec. 2.2).
* The gradient in log-hyperparameters,
      dL/dtheta = 1/2 omega^T (dK_hat/dtheta) omega - 1/2 tr(K_hat^{-1} dK_hat/dtheta),
  the standard GP identity (the paper states that mBCG estimates the marginal
  likelihood "and its derivatives", Sec. 3.2).
* Predictive mean and variance (Eq. 1).  The printed variance omits the prior
  term; the latent-f marginal variance used here is
      var(x') = k(x', x') - K(x', X) K_hat^{-1} K(X, x').
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from .kernel import Theta, dkernel_dlogell, kernel, khat


def cholesky_gp(X, y, th: Theta) -> dict:
    Kh = khat(X, th)
    c = cho_factor(Kh, lower=True)
    omega = cho_solve(c, y)
    logdet = 2.0 * float(np.sum(np.log(np.diag(c[0]))))
    quad = float(y @ omega)
    n = X.shape[0]
    mll = -0.5 * quad - 0.5 * logdet - 0.5 * n * math.log(2.0 * math.pi)
    return {"omega": omega, "logdet": logdet, "quad": quad, "mll": mll, "chol": c}


def dkhat_all(X, th: Theta):
    """Yield (index, dK_hat/dlog theta_index) for theta = (l_1..l_d, s_f, sigma^2)."""
    for j in range(th.d):
        yield j, dkernel_dlogell(X, X, th, j)
    yield th.d, kernel(X, X, th)
    yield th.d + 1, th.noise * np.eye(X.shape[0])


def mll_grad(X, y, th: Theta) -> np.ndarray:
    """Exact gradient of Eq. 2 with respect to (log l_1..log l_d, log s_f, log sigma^2)."""
    res = cholesky_gp(X, y, th)
    n = X.shape[0]
    Kinv = cho_solve(res["chol"], np.eye(n))
    om = res["omega"]
    g = np.empty(th.d + 2)
    for j, Dj in dkhat_all(X, th):
        g[j] = 0.5 * om @ (Dj @ om) - 0.5 * float(np.sum(Kinv * Dj))
    return g


def predict(X, y, Xq, th: Theta, add_noise: bool = False):
    """Predictive mean and marginal variance at the query rows Xq (Eq. 1)."""
    Kh = khat(X, th)
    c = cho_factor(Kh, lower=True)
    Kq = kernel(Xq, X, th)
    mean = Kq @ cho_solve(c, y)
    var = th.sf - np.sum(Kq * cho_solve(c, Kq.T).T, axis=1)
    if add_noise:
        var = var + th.noise
    return mean, var
