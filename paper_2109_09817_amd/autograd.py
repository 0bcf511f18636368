"""Differentiable entry points over the C ABI, and hyperparameter training.

Hyperparameters travel as one float64 tensor ``log_theta`` of length d + 2:
(log l_1 .. log l_d, log s_f, log sigma^2), the parametrisation of the
gradient entries that ``gp_kmm_grad`` and ``gp_mll_and_grad`` return.

* ``KhatV``: W = K_hat(theta) V.  Backward: dL/dV = K_hat G (K_hat is
  symmetric) and dL/dlog theta_j = sum_c G_c^T (dK_hat/dlog theta_j) V_c, the
  bilinear forms of the gradient sweep (with unit column weights); the kernel
  tiles are recomputed, never stored.  X is data: no gradient flows to it.
* ``MLL``: the BBMM estimate of the log marginal likelihood (Eq. 2, Sec. 3.2).
  Its forward runs preconditioner, probes, mBCG, stochastic Lanczos quadrature
  and the gradient sweep in one library call; backward scales the gradient
  estimate that call returned.
* ``ExactMLL``: the exact log marginal likelihood of a dense Cholesky GP (the
  AltBBMM protocol's subset model, Sec. 3.2, Sec. 4) and its exact gradient.
* ``fit``: Adam on log theta against -L / n (BBMM estimates); ``fit_exact``:
  the same on the exact GP.

All arithmetic runs in libgpkmm's kernels; these classes only marshal.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np
import torch

from . import gp


def kernel_from_log(log_theta, kind: str = "matern52") -> gp.Kernel:
    """gp.Kernel from (log l_1..log l_d, log s_f, log sigma^2)."""
    v = np.asarray(log_theta.detach().cpu().numpy() if isinstance(log_theta, torch.Tensor) else log_theta,
                   dtype=np.float64)
    if v.ndim != 1 or v.shape[0] < 3:
        raise ValueError("log_theta must hold d lengthscales, the outputscale and the noise (d + 2 >= 3 entries)")
    if not np.all(np.isfinite(v)):
        raise ValueError("log_theta must be finite")
    e = np.exp(v)
    return gp.Kernel(e[:-2], float(e[-2]), float(e[-1]), kind)


def _like(a, ref: torch.Tensor) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a, dtype=np.float64), dtype=ref.dtype, device=ref.device)


class KhatV(torch.autograd.Function):
    """W = (K(X, X) + sigma^2 I) V with V, W of shape (t, n); t <= 64 for the backward."""

    @staticmethod
    def forward(ctx, log_theta: torch.Tensor, X: torch.Tensor, V: torch.Tensor, kind: str = "matern52",
                precision: str = "bf16x3") -> torch.Tensor:
        kern = kernel_from_log(log_theta, kind)
        V = V.detach().contiguous()
        W = gp.kmm(kern, X.detach(), V, precision=precision)
        ctx.save_for_backward(log_theta.detach(), X.detach(), V)
        ctx.kind = kind
        ctx.precision = precision
        return W

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        log_theta, X, V = ctx.saved_tensors
        if ctx.needs_input_grad[1]:
            raise NotImplementedError("KhatV: no gradient with respect to the inputs X")
        kern = kernel_from_log(log_theta, ctx.kind)
        G = G.detach().contiguous()
        g_theta = g_v = None
        if ctx.needs_input_grad[0]:
            g = gp.kmm_grad(kern, X, G, V, np.ones(V.shape[0]), precision=ctx.precision)
            g_theta = _like(g, log_theta)
        if ctx.needs_input_grad[2]:
            g_v = gp.kmm(kern, X, G, precision=ctx.precision)
        return g_theta, None, g_v, None, None


class MLL(torch.autograd.Function):
    """BBMM estimate of the log marginal likelihood L(theta) as a scalar tensor."""

    @staticmethod
    def forward(ctx, log_theta: torch.Tensor, X: torch.Tensor, y: torch.Tensor, probes: int = 15, rank: int = 100,
                max_iter: int = 100, tol: float = 1e-6, seed: int = 0, kind: str = "matern52",
                precision: str = "bf16x3") -> torch.Tensor:
        kern = kernel_from_log(log_theta, kind)
        r = gp.mll_and_grad(kern, X.detach(), y.detach(), probes, rank, max_iter, tol, seed, precision,
                            with_grad=True)
        ctx.save_for_backward(_like(r.grad, log_theta))
        ctx.info = r.info
        ctx.status = r.status
        return _like(r.mll, log_theta)

    @staticmethod
    def backward(ctx, go: torch.Tensor):
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            raise NotImplementedError("MLL: gradients flow to the hyperparameters only")
        (g,) = ctx.saved_tensors
        return (go * g,) + (None,) * 9


class ExactMLL(torch.autograd.Function):
    """Exact log marginal likelihood L(theta) of the dense GP on (X, y) as a scalar tensor."""

    @staticmethod
    def forward(ctx, log_theta: torch.Tensor, X: torch.Tensor, y: torch.Tensor, kind: str = "matern52") -> torch.Tensor:
        kern = kernel_from_log(log_theta, kind)
        r = gp.exact_mll_and_grad(kern, X.detach(), y.detach(), with_grad=True)
        ctx.save_for_backward(_like(r.grad, log_theta))
        return _like(r.mll, log_theta)

    @staticmethod
    def backward(ctx, go: torch.Tensor):
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            raise NotImplementedError("ExactMLL: gradients flow to the hyperparameters only")
        (g,) = ctx.saved_tensors
        return go * g, None, None, None


@dataclasses.dataclass
class FitResult:
    log_theta: np.ndarray                 # final (d + 2)
    trajectory: List[np.ndarray]          # log theta before each step
    mll: List[float]                      # estimate at each step
    iters: List[int]                      # mBCG iterations per step
    seconds: List[float]                  # wall time per step


def fit(X: torch.Tensor, y: torch.Tensor, log_theta0, steps: int = 50, lr: float = 0.05, probes: int = 15,
        rank: int = 100, max_iter: int = 100, tol: float = 1e-6, seed: int = 0, kind: str = "matern52",
        precision: str = "bf16x3", callback=None) -> FitResult:
    """Adam on log theta minimising -L/n; fresh probes every step (seed + step)."""
    n = X.shape[0]
    p = torch.tensor(np.asarray(log_theta0, dtype=np.float64), requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr)
    out = FitResult(np.empty(0), [], [], [], [])
    for s in range(steps):
        t0 = time.perf_counter()
        opt.zero_grad()
        out.trajectory.append(p.detach().numpy().copy())
        mll = MLL.apply(p, X, y, probes, rank, max_iter, tol, seed + s, kind, precision)
        loss = -mll / n
        loss.backward()
        opt.step()
        out.mll.append(float(mll.detach()))
        out.iters.append(_mll_iters(mll))
        out.seconds.append(time.perf_counter() - t0)
        if callback is not None:
            callback(s, out)
    out.log_theta = p.detach().numpy().copy()
    return out


def fit_exact(X: torch.Tensor, y: torch.Tensor, log_theta0, steps: int = 50, lr: float = 0.05,
              kind: str = "matern52", callback=None) -> FitResult:
    """Adam on log theta minimising -L/n of the exact GP (deterministic: no probes)."""
    n = X.shape[0]
    p = torch.tensor(np.asarray(log_theta0, dtype=np.float64), requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr)
    out = FitResult(np.empty(0), [], [], [], [])
    for s in range(steps):
        t0 = time.perf_counter()
        opt.zero_grad()
        out.trajectory.append(p.detach().numpy().copy())
        mll = ExactMLL.apply(p, X, y, kind)
        (-mll / n).backward()
        opt.step()
        out.mll.append(float(mll.detach()))
        out.iters.append(0)
        out.seconds.append(time.perf_counter() - t0)
        if callback is not None:
            callback(s, out)
    out.log_theta = p.detach().numpy().copy()
    return out


def _mll_iters(mll: torch.Tensor) -> int:
    """mBCG iterations of the MLL evaluation that produced `mll` (0 if unknown)."""
    fn = mll.grad_fn
    info = getattr(fn, "info", None) if fn is not None else None
    return int(info["iters"]) if info else 0
