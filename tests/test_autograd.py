"""Wiring of the autograd layer (KhatV, MLL, fit), checked on the CPU.

The library calls are replaced, inside these tests only, by the FP64 oracle,
so that torch.autograd.gradcheck can compare each backward formula with
central differences of its forward in exact arithmetic.  The GPU versions are
checked against the oracle in test_gpu_autograd.py.
"""
import numpy as np
import pytest
import torch

import oracle.kernel as ok
from oracle import exact
from paper_2109_09817_amd import autograd as ag
from paper_2109_09817_amd import gp

KIND = {"matern52": ok.MATERN52, "rbf": ok.RBF}


def _theta(kern):
    return ok.Theta(np.asarray(kern.lengthscale, dtype=np.float64), kern.outputscale, kern.noise, KIND[kern.kind])


class OracleGp:
    """The four gp entry points the autograd layer calls, on CPU tensors, from the oracle."""

    Kernel = gp.Kernel

    def kmm(self, kern, X, V, precision="bf16x3"):
        K = ok.khat(X.numpy(), _theta(kern))
        return torch.from_numpy(np.ascontiguousarray((K @ V.numpy().T).T))

    def kmm_grad(self, kern, X, U, W, colw, precision="fp32"):
        th = _theta(kern)
        Un, Wn = U.numpy(), W.numpy()
        g = np.zeros(th.d + 2)
        for j, D in exact.dkhat_all(X.numpy(), th):
            g[j] = sum(colw[c] * Un[c] @ (D @ Wn[c]) for c in range(Un.shape[0]))
        return g

    def mll_and_grad(self, kern, X, y, probes, rank, max_iter, tol, seed, precision="bf16x3", with_grad=True):
        th = _theta(kern)
        r = exact.cholesky_gp(X.numpy(), y.numpy(), th)
        return gp.MllResult(r["mll"], exact.mll_grad(X.numpy(), y.numpy(), th), {"iters": 0}, 0)


@pytest.fixture
def oracle_backend(monkeypatch):
    monkeypatch.setattr(ag, "gp", OracleGp())


def _data(n, d, seed=0):
    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.standard_normal((n, d)))
    lt = torch.tensor(np.concatenate([np.log(rng.uniform(0.8, 2.0, d)), [np.log(1.3), np.log(0.05)]]))
    return X, lt, rng


@pytest.mark.parametrize("kind", ["matern52", "rbf"])
def test_khatv_gradcheck(oracle_backend, kind):
    X, lt, rng = _data(24, 3)
    V = torch.from_numpy(rng.standard_normal((3, 24)))
    lt.requires_grad_(True)
    V.requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: ag.KhatV.apply(a, X, b, kind, "fp32"), (lt, V),
                                    eps=1e-6, atol=1e-7, rtol=1e-6)


def test_khatv_refuses_gradient_to_x(oracle_backend):
    X, lt, rng = _data(10, 2)
    X.requires_grad_(True)
    V = torch.from_numpy(rng.standard_normal((2, 10)))
    W = ag.KhatV.apply(lt, X, V, "matern52", "fp32")
    with pytest.raises(NotImplementedError):
        W.sum().backward()


@pytest.mark.parametrize("kind", ["matern52", "rbf"])
def test_mll_gradcheck(oracle_backend, kind):
    X, lt, rng = _data(30, 3, seed=1)
    y = torch.from_numpy(rng.standard_normal(30))
    lt.requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a: ag.MLL.apply(a, X, y, 8, 10, 50, 0.0, 0, kind, "fp32"), (lt,),
                                    eps=1e-6, atol=1e-6, rtol=1e-6)


def test_fit_increases_exact_mll(oracle_backend):
    X, lt, rng = _data(60, 2, seed=2)
    th_true = ok.Theta(np.array([0.7, 1.5]), 1.0, 0.05)
    y = rng.multivariate_normal(np.zeros(60), ok.khat(X.numpy(), th_true))
    y = torch.from_numpy(y)
    start = np.zeros(4)
    start[-1] = np.log(1e-2)
    res = ag.fit(X, y, start, steps=40, lr=0.05)
    assert len(res.trajectory) == 40 and len(res.mll) == 40
    mll0 = exact.cholesky_gp(X.numpy(), y.numpy(), ok.Theta.from_log(start))["mll"]
    mll1 = exact.cholesky_gp(X.numpy(), y.numpy(), ok.Theta.from_log(res.log_theta))["mll"]
    assert mll1 > mll0
    # Adam with a small step: the exact objective improves over the run, and the first step moves every
    # coordinate against the sign of -dL
    g0 = exact.mll_grad(X.numpy(), y.numpy(), ok.Theta.from_log(start))
    step = res.trajectory[1] - res.trajectory[0]
    assert np.all(np.sign(step[np.abs(g0) > 1e-9]) == np.sign(g0[np.abs(g0) > 1e-9]))


def test_kernel_from_log_rejects_bad_vectors():
    with pytest.raises(ValueError):
        ag.kernel_from_log(np.array([0.0, 0.0]))
    with pytest.raises(ValueError):
        ag.kernel_from_log(np.array([0.0, np.nan, 0.0]))
    k = ag.kernel_from_log(np.log(np.array([2.0, 3.0, 0.5, 0.01])))
    np.testing.assert_allclose(k.lengthscale, [2.0, 3.0])
    assert abs(k.outputscale - 0.5) < 1e-15 and abs(k.noise - 0.01) < 1e-15
