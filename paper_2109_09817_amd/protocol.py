"""The AltBBMM training protocol (Sec. 3.2, Sec. 4).

1. Hyperparameters from an exact GP on a random subset of the training
   molecules (the paper: 50 molecules), by Adam on the exact log marginal
   likelihood (``autograd.fit_exact``; dense FP64 Cholesky on the device).
2. The noise regularisation sigma^2_add (the paper: 1e-5) added to the
   optimised sigma^2.
3. One block-CG solve on the full training set with the symmetric Nystrom
   preconditioner (``gp.nystrom_precond``, ``gp.bcg``): B = [y | N(0, I)
   columns] (block size s, the paper: 50), every column's relative residual
   below tol (the paper: 1e-6); omega = K_hat^{-1} y is the first column.

The subset rows, landmark rows and random right-hand sides are inputs.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Optional

import numpy as np
import torch

from . import autograd, gp


@dataclasses.dataclass
class ProtocolResult:
    log_theta: np.ndarray       # hyperparameters from the subset (log l_1..log l_d, log s_f, log sigma^2)
    kernel: gp.Kernel           # the full-set kernel: sigma^2 = exp(log sigma^2) + sigma^2_add
    fit: autograd.FitResult     # the subset trajectory
    omega: torch.Tensor         # (n,) K_hat^{-1} y on the full set
    W: torch.Tensor             # (s, n) the whole block solve
    iters: int
    relres: np.ndarray
    status: int
    kept: int                   # Nystrom directions kept
    seconds: dict


def altbbmm_train(X: torch.Tensor, y: torch.Tensor, subset, log_theta0, landmarks, B_extra: np.ndarray,
                  steps: int = 50, lr: float = 0.05, noise_add: float = 1e-5, tol: float = 1e-6,
                  max_iter: int = 1000, precision: str = "fp64", kind: str = "matern52",
                  callback=None) -> ProtocolResult:
    """Subset hyperparameters, then the full-set AltBBMM solve.  ``subset``: row indices of the exact-GP
    subset; ``landmarks``: Nystrom landmark rows (None: no preconditioner); ``B_extra``: (s - 1, n) random
    right-hand sides appended to y."""
    n = X.shape[0]
    sub = torch.as_tensor(np.asarray(subset, dtype=np.int64), device=X.device)
    Xs = X.index_select(0, sub).contiguous()
    ys = y.index_select(0, sub).contiguous()
    torch.cuda.synchronize(X.device)
    t0 = time.perf_counter()
    fr = autograd.fit_exact(Xs, ys, log_theta0, steps=steps, lr=lr, kind=kind, callback=callback)
    t1 = time.perf_counter()
    k = autograd.kernel_from_log(fr.log_theta, kind)
    kern = gp.Kernel(k.lengthscale, k.outputscale, k.noise + noise_add, kind)
    Bx = np.asarray(B_extra, dtype=np.float64)
    if Bx.ndim != 2 or Bx.shape[1] != n:
        raise ValueError("B_extra must be (s - 1, n)")
    B = torch.empty((1 + Bx.shape[0], n), dtype=torch.float64, device=X.device)
    B[0] = y
    B[1:] = torch.from_numpy(np.ascontiguousarray(Bx)).to(X.device)
    pc = None if landmarks is None else gp.nystrom_precond(kern, X, landmarks)
    torch.cuda.synchronize(X.device)
    t2 = time.perf_counter()
    r = gp.bcg(kern, X, B, max_iter, tol, pc=pc, precision=precision)
    torch.cuda.synchronize(X.device)
    t3 = time.perf_counter()
    return ProtocolResult(fr.log_theta, kern, fr, r.W[0], r.W, r.iters, r.relres, r.status,
                          0 if pc is None else pc.kept,
                          {"subset_fit": t1 - t0, "precond": t2 - t1, "solve": t3 - t2})
