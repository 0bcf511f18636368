"""The exact GP of the AltBBMM protocol (gp_exact_mll_and_grad, ExactMLL, fit_exact, altbbmm_train)
against the dense oracle."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle.kernel as ok
import synth
from oracle import exact
from _helpers import dev, host

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _gk(th):
    from paper_2109_09817_amd import gp
    return gp.Kernel(th.ell, th.sf, th.noise, "matern52" if th.kind == ok.MATERN52 else "rbf")


def _case(n, d, seed, kind, cond):
    if d == 48 or d == 32:
        p = synth.make_problem("c2" if d == 48 else "c1", n=n, cond_variant=cond, seed=seed)
        return p.X, p.y, ok.Theta(p.ell, 1.0, p.noise, kind)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    ell = rng.uniform(0.5, 2.0, d) * (math.sqrt(2 * d) if cond else 1.0)
    return X, rng.standard_normal(n), ok.Theta(ell, 1.3, 1e-2, kind)


def _grad_scale(X, th, om, Kinv):
    """Per entry: 1/2 |omega|^T |D_j| |omega| + 1/2 sum |K_hat^{-1}| |D_j| (the size of the two terms)."""
    s = np.empty(th.d + 2)
    for j, D in exact.dkhat_all(X, th):
        s[j] = 0.5 * np.abs(om) @ (np.abs(D) @ np.abs(om)) + 0.5 * float(np.sum(np.abs(Kinv) * np.abs(D)))
    return s


CASES = [(1, 3, False), (2, 3, False), (63, 5, False), (64, 7, False), (65, 7, True), (130, 48, True),
         (700, 48, True), (1000, 64, False), (2100, 32, True)]


@pytest.mark.parametrize("kind", [ok.MATERN52, ok.RBF])
@pytest.mark.parametrize("n,d,cond", CASES)
def test_exact_gp_matches_the_dense_oracle(n, d, cond, kind):
    from paper_2109_09817_amd import gp
    X, y, th = _case(n, d, 11 + n, kind, cond)
    r = gp.exact_mll_and_grad(_gk(th), dev(X), dev(y), with_grad=True, with_omega=True)
    o = exact.cholesky_gp(X, y, th)
    Kh = ok.khat(X, th)
    Kinv = np.linalg.inv(Kh)
    ev = np.linalg.eigvalsh(Kh)
    kappa = ev[-1] / ev[0]
    tol = max(1e-10, 1e-14 * kappa)
    mll_scale = abs(o["quad"]) + abs(o["logdet"]) + 0.5 * n * math.log(2 * math.pi)
    e_mll = abs(r.mll - o["mll"]) / mll_scale
    om = host(r.omega)
    e_om = np.linalg.norm(om - o["omega"]) / np.linalg.norm(o["omega"])
    g_ref = exact.mll_grad(X, y, th)
    scale = _grad_scale(X, th, o["omega"], Kinv)
    diff = np.abs(r.grad - g_ref)
    e_g = float(np.max(np.where(scale > 0, diff / np.where(scale > 0, scale, 1.0), diff)))  # n = 1: no pairs
    log(f"exact n={n} d={d} kind={kind} cond={cond} (kappa {kappa:.1e}): mll err {e_mll:.1e}, "
        f"omega err {e_om:.1e}, grad err / term scale {e_g:.1e}")
    assert e_mll <= tol
    assert e_om <= max(1e-10, 1e-13 * kappa)
    assert e_g <= tol


def test_exact_gp_reports_a_singular_kernel():
    from paper_2109_09817_amd import _lib, gp
    X, y, th = _case(70, 4, 3, ok.MATERN52, False)
    X[:] = X[3]  # identical rows and no noise: K_hat = s_f 1 1^T, whose second pivot is exactly 0
    th0 = ok.Theta(th.ell, 1.0, 0.0, th.kind)
    with pytest.raises(_lib.GpError) as e:
        gp.exact_mll_and_grad(_gk(th0), dev(X), dev(y))
    assert e.value.code == _lib.GP_ENOTPD


def test_exact_fit_follows_the_oracle_trajectory():
    """Adam on -L/n with the library's exact gradient against the same Adam on the oracle's gradient."""
    from paper_2109_09817_amd import autograd as ag
    X, y, th = _case(300, 48, 5, ok.MATERN52, True)
    d = X.shape[1]
    start = np.concatenate([np.log(th.ell) - 0.3, [0.2, math.log(1e-2)]])
    steps = 8
    res = ag.fit_exact(dev(X), dev(y), start, steps=steps, lr=0.05)
    p = torch.tensor(start, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.05)
    traj = []
    for _ in range(steps):
        traj.append(p.detach().numpy().copy())
        v = p.detach().numpy()
        tho = ok.Theta(np.exp(v[:d]), math.exp(v[d]), math.exp(v[d + 1]), ok.MATERN52)
        opt.zero_grad()
        p.grad = torch.from_numpy(-exact.mll_grad(X, y, tho) / X.shape[0])
        opt.step()
    err = max(np.abs(a - b).max() for a, b in zip(res.trajectory, traj))
    err = max(err, np.abs(res.log_theta - p.detach().numpy()).max())
    log(f"fit_exact: {steps} Adam steps, max |log theta - oracle| {err:.1e}, mll {res.mll[0]:.4f} -> {res.mll[-1]:.4f}")
    assert err <= 1e-9
    assert res.mll[-1] > res.mll[0]


def test_altbbmm_protocol_end_to_end():
    """Subset hyperparameters (5 molecules), sigma^2_add = 1e-5, then the full-set Nystrom block CG in FP64:
    omega against the dense solve at the protocol's final kernel."""
    from paper_2109_09817_amd import protocol
    p = synth.make_problem("c2", n=2500, cond_variant=True, seed=9)
    n, d = p.X.shape
    sub = synth.molecule_subset(p.mol, 5, 3)
    start = np.concatenate([np.log(p.ell), [0.0, math.log(1e-2)]])
    M = np.sort(np.random.default_rng(4).choice(n, 250, replace=False))
    Bx = synth.random_block(n, 7, 21)
    res = protocol.altbbmm_train(dev(p.X), dev(p.y), sub, start, M, Bx, steps=10, lr=0.05, noise_add=1e-5,
                                 tol=1e-8, max_iter=2000, precision="fp64")
    k = res.kernel
    th = ok.Theta(np.asarray(k.lengthscale), k.outputscale, k.noise, ok.MATERN52)
    Kh = ok.khat(p.X, th)
    om_ref = np.linalg.solve(Kh, p.y)
    om = host(res.omega)
    ev = np.linalg.eigvalsh(Kh)
    kappa = ev[-1] / ev[0]
    e = np.linalg.norm(om - om_ref) / np.linalg.norm(om_ref)
    true = np.linalg.norm(Kh @ om - p.y) / np.linalg.norm(p.y)
    log(f"protocol: subset {sub.size} rows, noise {k.noise:.2e}, kept {res.kept}, bcg {res.iters} it "
        f"(status {res.status}), omega err {e:.1e} (kappa {kappa:.1e}), true residual {true:.1e}, "
        f"seconds {res.seconds}")
    assert res.status == 0
    assert abs(k.noise - (math.exp(res.log_theta[-1]) + 1e-5)) <= 1e-15
    assert true <= 1e-7
    assert e <= 10 * kappa * 1e-8
