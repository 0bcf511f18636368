"""AltBBMM on the GPU (gp_nystrom_precond, gp_nystrom_apply, gp_bcg) against the oracle."""
import math
import sys

import numpy as np
import pytest

import oracle.kernel as ok
import synth
from oracle import altbbmm as ab
from _helpers import dev, host

pytestmark = pytest.mark.gpu

EPS_PRODUCT = {"bf16x3": 3e-5, "fp32": 2e-6}
RCOND = 1e-7  # the library's eigenvalue cut of K_MM (nearly repeated landmarks)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _gk(th):
    from paper_2109_09817_amd import gp
    return gp.Kernel(th.ell, th.sf, th.noise, "matern52" if th.kind == ok.MATERN52 else "rbf")


def _problem(n, noise=1e-3, seed=0, kind=ok.MATERN52):
    p = synth.make_problem("c2", n=n, cond_variant=True, seed=seed)
    th = ok.Theta(p.ell, 1.0, noise, kind)
    return p.X, p.y, th


def _landmarks(n, r, seed):
    return np.sort(np.random.default_rng(seed).choice(n, r, replace=False))


@pytest.mark.parametrize("kind", [ok.MATERN52, ok.RBF])
@pytest.mark.parametrize("r", [1, 37, 300])
def test_nystrom_matches_oracle(kind, r):
    from paper_2109_09817_amd import gp
    n = 1500
    X, y, th = _problem(n, kind=kind)
    M = _landmarks(n, r, 7)
    pc = gp.nystrom_precond(_gk(th), dev(X), M)
    KXM_ref = ok.kernel(X, X[M], th)
    kmm_cond = np.linalg.cond(KXM_ref[M])
    lam = np.linalg.eigvalsh(KXM_ref[M])
    P_ref = ab.nystrom_matrix(X, th, M, RCOND)
    Q_ref = P_ref - th.noise * np.eye(n)
    # the factor: Z^T Z is the Nystrom approximation; rows beyond the kept rank are zero
    Z, g = host(pc.Z), host(pc.g)
    k = pc.kept
    assert k == int((lam > RCOND * lam.max()).sum())
    assert np.all(g[k:] == 0) and np.all(Z[k:] == 0) and np.all(g[:k] < 0)
    e_q = np.abs(Z.T @ Z - Q_ref).max() / np.abs(Q_ref).max()
    # g_m from the factor's own row norms S_m = |Z_m|^2
    sig = math.sqrt(th.noise)
    q = np.sqrt((Z[:k] ** 2).sum(axis=1) + th.noise)
    np.testing.assert_allclose(g[:k], -1 / (sig * q * (sig + q)), rtol=1e-9)
    S_ref = ab.inv_sqrt(P_ref)
    V = np.random.default_rng(3).standard_normal((5, n))
    got = host(gp.nystrom_apply(pc, dev(V)))
    ref = V @ S_ref  # S symmetric: rows of (S V^T)^T
    e_a = np.abs(got - ref).max() / (np.abs(V) @ np.abs(S_ref)).max()
    log(f"nystrom kind={kind} r={r}: kept {k}, Z^T Z err {e_q:.1e}, P^-1/2 V err {e_a:.1e} (cond K_MM {kmm_cond:.1e})")
    assert e_q <= max(1e-12, 1e-16 * kmm_cond)
    assert e_a <= max(1e-10, 1e-15 * kmm_cond)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("r", [0, 120])
def test_bcg_matches_oracle(prec, r):
    from paper_2109_09817_amd import gp
    n, s = 1200, 8
    X, y, th = _problem(n, seed=1)
    rng = np.random.default_rng(5)
    B = np.column_stack([y, rng.standard_normal((n, s - 1))])
    M = _landmarks(n, r, 9) if r else None
    Kh = ok.khat(X, th)
    ref = np.linalg.solve(Kh, B)
    o = ab.altbbmm_solve(X, th, B, M, 1e-6, 400, RCOND)
    pc = gp.nystrom_precond(_gk(th), dev(X), M) if r else None
    res = gp.bcg(_gk(th), dev(X), dev(B.T), 400, 1e-6, pc=pc, precision=prec)
    W = host(res.W).T
    ev = np.linalg.eigvalsh(Kh)
    kappa = ev[-1] / ev[0]
    err = np.linalg.norm(W - ref, axis=0) / np.linalg.norm(ref, axis=0)
    bound = max(1e-5, 10 * kappa * max(1e-6, EPS_PRODUCT[prec]))
    true_res = np.linalg.norm(Kh @ W - B, axis=0) / np.linalg.norm(B, axis=0)
    log(f"bcg {prec} r={r}: iters gpu {res.iters} oracle {o['iters']}, relres max {res.relres.max():.1e}, "
        f"true residual max {true_res.max():.1e}, solution err max {err.max():.1e} (kappa {kappa:.1e}, bound {bound:.1e})")
    assert res.status == 0
    assert np.all(res.relres <= 1e-6)
    assert err.max() <= bound
    # inexact products (kappa * eps ~ 7e-3 FP32, ~0.1 BF16x3 here) delay the block Krylov process
    # against the exact-arithmetic oracle; allow twice its count
    assert res.iters <= 2 * o["iters"] + 5
    assert true_res.max() <= 10 * (1e-6 + EPS_PRODUCT[prec]) * math.sqrt(kappa)
    if r:
        plain = gp.bcg(_gk(th), dev(X), dev(B.T), 400, 1e-6, precision=prec)
        log(f"bcg {prec}: unpreconditioned {plain.iters} iterations, Nystrom r={r} {res.iters}")
        assert o["iters"] < ab.altbbmm_solve(X, th, B, None, 1e-6, 400)["iters"]
        assert res.iters < plain.iters


def test_bcg_one_column_is_cg_on_the_gpu():
    """s = 1: block CG is CG; it reaches the same solve as mBCG's first column."""
    from paper_2109_09817_amd import gp
    n = 900
    X, y, th = _problem(n, seed=2)
    r1 = gp.bcg(_gk(th), dev(X), dev(y[None, :]), 300, 1e-8, precision="fp32")
    ref = np.linalg.solve(ok.khat(X, th), y)
    e = np.linalg.norm(host(r1.W)[0] - ref) / np.linalg.norm(ref)
    log(f"bcg s=1: iters {r1.iters}, err {e:.1e}")
    assert r1.status == 0 and e <= 1e-4


def test_bcg_reports_no_convergence():
    from paper_2109_09817_amd import _lib, gp
    n = 600
    X, y, th = _problem(n, seed=3)
    B = np.column_stack([y, np.random.default_rng(1).standard_normal((n, 3))])
    res = gp.bcg(_gk(th), dev(X), dev(B.T), 2, 1e-12, precision="fp32")
    assert res.status == _lib.GP_WNOCONV and res.iters == 2


# ---------------------------------------------------------------- large rank (Cholesky factor form)

@pytest.mark.parametrize("kind", [ok.MATERN52, ok.RBF])
@pytest.mark.parametrize("n,r", [(1500, 37), (1500, 300), (4000, 2048)])
def test_nystrom_chol_matches_oracle(kind, n, r):
    """E of the large-rank preconditioner: sigma^{-2} (V - E E^T V) against the oracle's dense
    P^{-1} V, P = K_XM (K_MM + delta I)^{-1} K_MX + sigma^2 I (r = 2048 is beyond the spectral
    form's limit of 1024)."""
    from paper_2109_09817_amd import gp
    X, y, th = _problem(n, kind=kind)
    M = _landmarks(n, r, 17)
    pc = gp.nystrom_chol_precond(_gk(th), dev(X), M)
    E = host(pc.E).T  # n x r
    P_ref = ab.nystrom_matrix_jitter(X, th, M)
    V = np.random.default_rng(4).standard_normal((n, 5))
    got = (V - E @ (E.T @ V)) / th.noise
    ref = np.linalg.solve(P_ref, V)
    condP = np.linalg.cond(P_ref)
    e = np.abs(got - ref).max() / np.abs(ref).max()
    ee = np.linalg.eigvalsh(E.T @ E)
    log(f"nystrom chol kind={kind} n={n} r={r}: P^-1 V err {e:.1e} (cond P {condP:.1e}); "
        f"eig(E^T E) in [{ee.min():.2e}, {ee.max():.6f}]")
    assert ee.max() < 1.0  # P^{-1} as applied is positive definite
    assert e <= max(1e-10, 1e-14 * condP)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
@pytest.mark.parametrize("r", [0, 120])
def test_bpcg_matches_oracle(prec, r):
    from paper_2109_09817_amd import gp
    n, s = 1200, 8
    X, y, th = _problem(n, seed=1)
    rng = np.random.default_rng(5)
    B = np.column_stack([y, rng.standard_normal((n, s - 1))])
    M = _landmarks(n, r, 9) if r else None
    Kh = ok.khat(X, th)
    ref = np.linalg.solve(Kh, B)
    if r:
        P_ref = ab.nystrom_matrix_jitter(X, th, M)
        o = ab.block_pcg(lambda D: Kh @ D, B, lambda R: np.linalg.solve(P_ref, R), 1e-6, 400)
    else:
        o = ab.block_pcg(lambda D: Kh @ D, B, lambda R: R.copy(), 1e-6, 400)
    pc = gp.nystrom_chol_precond(_gk(th), dev(X), M) if r else None
    res = gp.bpcg(_gk(th), dev(X), dev(B.T), 400, 1e-6, pc=pc, precision=prec)
    W = host(res.W).T
    ev = np.linalg.eigvalsh(Kh)
    kappa = ev[-1] / ev[0]
    eps = {"fp32": 2e-6, "bf16x3": 3e-5, "fp64": 1e-15}[prec]
    err = np.linalg.norm(W - ref, axis=0) / np.linalg.norm(ref, axis=0)
    bound = max(1e-5, 10 * kappa * max(1e-6, eps))
    true_res = np.linalg.norm(Kh @ W - B, axis=0) / np.linalg.norm(B, axis=0)
    log(f"bpcg {prec} r={r}: iters gpu {res.iters} oracle {o['iters']}, relres max {res.relres.max():.1e}, "
        f"true residual max {true_res.max():.1e}, solution err max {err.max():.1e} (kappa {kappa:.1e})")
    assert res.status == 0
    assert np.all(res.relres <= 1e-6)
    assert err.max() <= bound
    assert res.iters <= 2 * o["iters"] + 5
    if prec == "fp64":
        # FP64 products: the same recurrence as the oracle's, iteration for iteration
        assert abs(res.iters - o["iters"]) <= 1
        assert true_res.max() <= 1e-5
    if r:
        plain = ab.block_pcg(lambda D: Kh @ D, B, lambda R: R.copy(), 1e-6, 400)
        assert o["iters"] < plain["iters"]


def test_bpcg_at_rank_beyond_the_spectral_form():
    """r = 2048 landmarks on n = 4000 rows of the ill-conditioned variant, FP64 products: the
    preconditioner captures most of the spectrum, and the solve matches the dense one."""
    from paper_2109_09817_amd import gp
    n, s, r = 4000, 6, 2048
    X, y, th = _problem(n, seed=6)
    rng = np.random.default_rng(8)
    B = np.column_stack([y, rng.standard_normal((n, s - 1))])
    M = _landmarks(n, r, 19)
    pc = gp.nystrom_chol_precond(_gk(th), dev(X), M)
    res = gp.bpcg(_gk(th), dev(X), dev(B.T), 300, 1e-8, pc=pc, precision="fp64")
    plain = gp.bpcg(_gk(th), dev(X), dev(B.T), 300, 1e-8, precision="fp64")
    Kh = ok.khat(X, th)
    ref = np.linalg.solve(Kh, B)
    W = host(res.W).T
    err = np.linalg.norm(W - ref, axis=0) / np.linalg.norm(ref, axis=0)
    ev = np.linalg.eigvalsh(Kh)
    kappa = ev[-1] / ev[0]
    log(f"bpcg r={r} n={n}: {res.iters} iterations (unpreconditioned {plain.iters}), solution err {err.max():.1e} "
        f"(kappa {kappa:.1e})")
    assert res.status == 0 and plain.status == 0
    assert res.iters < plain.iters
    assert err.max() <= max(1e-6, 1e-8 * kappa * 10)


def test_bpcg_reports_no_convergence():
    from paper_2109_09817_amd import _lib, gp
    n = 600
    X, y, th = _problem(n, seed=3)
    B = np.column_stack([y, np.random.default_rng(1).standard_normal((n, 3))])
    res = gp.bpcg(_gk(th), dev(X), dev(B.T), 2, 1e-12, precision="fp32")
    assert res.status == _lib.GP_WNOCONV and res.iters == 2
