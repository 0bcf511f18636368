"""Oracle: the whole BBMM training step, composed from the other oracle modules.

Test infrastructure only.  One log-marginal-likelihood evaluation (Eq. 2) and
its gradient by the BBMM recipe of Sec. 3.2: pivoted-Cholesky preconditioner,
probe block [y | b_1..b_t], mBCG, stochastic Lanczos quadrature for the
log-determinant and stochastic trace estimates for the gradient.
"""
from __future__ import annotations

import numpy as np

from .gradient import bilinear_forms, mll_gradient_forms
from .kernel import Theta, khat_matmul
from .mbcg import mbcg, mll_from_solve, slq_logdet
from .pivchol import Preconditioner, pivoted_cholesky
from .probes import probe_block


def mll_and_grad_estimate(X, y, th: Theta, t: int, k: int, seed: int, max_iter: int, tol: float,
                          pivots=None, with_grad: bool = True) -> dict:
    L, piv, _ = pivoted_cholesky(X, th, k, pivots=pivots) if k > 0 else (np.zeros((X.shape[0], 0)), [], None)
    P = Preconditioner(L, th.noise)
    B = probe_block(seed, y, t, L, th.noise)
    res = mbcg(lambda D: khat_matmul(X, th, D), B, P.solve, max_iter, tol)
    logdet = slq_logdet(res, P.logdet, range(1, t + 1))
    mll = mll_from_solve(y, res["U"][:, 0], logdet)
    out = {"mll": mll, "logdet": logdet, "quad": float(y @ res["U"][:, 0]), "logdet_p": P.logdet,
           "res": res, "pivots": piv, "L": L, "B": B}
    if with_grad:
        U, V, w = mll_gradient_forms(res["U"], res["Z0"], t)
        out["grad"] = bilinear_forms(X, th, U, V, w)
    return out
