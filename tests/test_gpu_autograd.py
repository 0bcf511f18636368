"""The autograd layer on the GPU: KhatV's backward against the oracle and against
central differences of its own forward, and MLL / fit on a subsample of the
gradient configuration (N = 4096, d = 48, 48 lengthscales + s_f + sigma^2)."""
import sys

import numpy as np
import pytest

import oracle.kernel as ok
import synth
from oracle import exact
from _helpers import dev, host

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _forms(X, th, G, V):
    """sum_c G_c^T (dK_hat/dlog theta_j) V_c for every j (oracle), and the same on |G|, |V|."""
    g = np.zeros(th.d + 2)
    s = np.zeros(th.d + 2)
    for j, D in exact.dkhat_all(X, th):
        g[j] = sum(G[c] @ (D @ V[c]) for c in range(G.shape[0]))
        s[j] = sum(np.abs(G[c]) @ (np.abs(D) @ np.abs(V[c])) for c in range(G.shape[0]))
    return g, s


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-4)])
@pytest.mark.parametrize("kind", ["matern52", "rbf"])
def test_khatv_backward_matches_oracle(prec, tol, kind):
    import torch
    from paper_2109_09817_amd import autograd as ag
    p = synth.make_problem("c4", n=700, cond_variant=True)
    X = p.X
    rng = np.random.default_rng(11)
    V = rng.standard_normal((5, X.shape[0]))
    G = rng.standard_normal((5, X.shape[0]))
    th = ok.Theta(p.ell, 1.2, 3e-3, ok.MATERN52 if kind == "matern52" else ok.RBF)
    lt = torch.tensor(th.log_vector(), requires_grad=True)
    Vd = dev(V).requires_grad_(True)
    W = ag.KhatV.apply(lt, dev(X), Vd, kind, prec)
    (W * dev(G)).sum().backward()
    K = ok.khat(X, th)
    w_err = np.abs(host(W) - V @ K).max() / np.abs(V @ np.abs(K)).max()
    gv_err = np.abs(host(Vd.grad) - G @ K).max() / np.abs(G @ np.abs(K)).max()
    ref, scale = _forms(X, th, G, V)
    gt_err = np.max(np.abs(lt.grad.numpy() - ref) / scale)
    log(f"KhatV {prec} {kind}: W err {w_err:.1e}, dV err {gv_err:.1e}, dtheta err/term scale {gt_err:.1e}")
    assert w_err <= tol and gv_err <= tol and gt_err <= tol


def test_khatv_backward_matches_central_differences():
    """FP32 form: d/dlog theta of f = sum G . K_hat V by central differences of the forward (h = 1e-3)."""
    import torch
    from paper_2109_09817_amd import autograd as ag
    p = synth.make_problem("c4", n=1000, cond_variant=True)
    X = dev(p.X)
    rng = np.random.default_rng(12)
    V = dev(rng.standard_normal((3, p.X.shape[0])))
    G = dev(rng.standard_normal((3, p.X.shape[0])))
    th = ok.Theta(p.ell, 1.0, 1e-2)
    v = th.log_vector()
    lt = torch.tensor(v, requires_grad=True)
    (ag.KhatV.apply(lt, X, V, "matern52", "fp32") * G).sum().backward()
    g = lt.grad.numpy()
    h = 1e-3
    idx = [0, 7, 23, 47, 48, 49]
    fd = []
    for j in idx:
        vp, vm = v.copy(), v.copy()
        vp[j] += h
        vm[j] -= h
        with torch.no_grad():
            fp = float((ag.KhatV.apply(torch.tensor(vp), X, V, "matern52", "fp32") * G).sum())
            fm = float((ag.KhatV.apply(torch.tensor(vm), X, V, "matern52", "fp32") * G).sum())
        fd.append((fp - fm) / (2 * h))
    fd = np.array(fd)
    scale = np.abs(g).max()
    err = np.abs(fd - g[idx]) / scale
    log(f"KhatV central differences: max |fd - grad| / max|grad| = {err.max():.1e}")
    assert err.max() <= 1e-3


def test_mll_function_and_fit_on_gradient_config_subsample():
    """MLL.backward returns the library's gradient estimate; 8 Adam steps from the stated start
    (l = 1, s_f = 1, sigma^2 = 1e-2) raise the exact mll on the N = 4096 subsample."""
    import torch
    from paper_2109_09817_amd import autograd as ag
    from paper_2109_09817_amd import gp
    p = synth.make_problem("c4", n=4096)
    X, y = dev(p.X), dev(p.y)
    d = p.X.shape[1]
    start = np.concatenate([np.zeros(d), [0.0, np.log(1e-2)]])
    lt = torch.tensor(start, requires_grad=True)
    mll = ag.MLL.apply(lt, X, y, 32, 100, 100, 1e-6, 5, "matern52", "bf16x3")
    mll.backward()
    r = gp.mll_and_grad(ag.kernel_from_log(start), X, y, 32, 100, 100, 1e-6, 5, "bf16x3")
    np.testing.assert_array_equal(lt.grad.numpy(), r.grad)
    assert float(mll.detach()) == r.mll
    res = ag.fit(X, y, start, steps=8, lr=0.05, probes=32, rank=100, max_iter=100, tol=1e-6, seed=1)
    m0 = exact.cholesky_gp(p.X, p.y, ok.Theta.from_log(start))["mll"]
    m1 = exact.cholesky_gp(p.X, p.y, ok.Theta.from_log(res.log_theta))["mll"]
    log(f"fit: exact mll {m0:.3f} -> {m1:.3f}; estimates {res.mll[0]:.3f} .. {res.mll[-1]:.3f}; "
        f"iters {res.iters}; s/step {np.mean(res.seconds):.3f}")
    assert m1 > m0
    assert all(i > 0 for i in res.iters)
