"""The low-noise regime (sigma^2 down to 1e-8; the paper's failure mode is rounding beyond the
noise, Sec. 3.2): mBCG and block CG with FP64 products reach the dense solve where it is well
defined, at a noise level where the BF16x3 products cannot resolve K_hat."""
import sys

import numpy as np
import pytest

import oracle.kernel as ok
import synth
from _helpers import dev, host

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _gk(th):
    from paper_2109_09817_amd import gp
    return gp.Kernel(th.ell, th.sf, th.noise, "matern52")


@pytest.mark.parametrize("noise", [1e-5, 1e-7])
def test_fp64_solves_reach_the_dense_solution_at_low_noise(noise):
    """mBCG with FP64 products reaches the FP64 limit (true residual ~ kappa * eps) at kappa ~ 1e7; the
    BF16x3 products stall orders of magnitude above it."""
    from paper_2109_09817_amd import gp
    n = 1536
    X, y, ell = synth.near_duplicate_pairs(n, 4)
    th = ok.Theta(ell, 1.0, noise)
    Kh = ok.khat(X, th)
    ev = np.linalg.eigvalsh(Kh)
    kappa = ev[-1] / ev[0]
    B = np.column_stack([y, np.random.default_rng(2).standard_normal((n, 5))])
    from paper_2109_09817_amd import _lib
    res = {}
    for prec in ("fp64", "bf16x3"):
        try:
            r = gp.mbcg(_gk(th), dev(X), dev(B.T), 4000, 1e-10, precision=prec)
        except _lib.GpError as e:
            # the product's rounding (~eps |K|) exceeds lambda_min: the operator it applies is
            # indefinite and CG breaks down (d^T K d <= 0), reported as GP_ENOTPD
            assert prec == "bf16x3" and e.code == _lib.GP_ENOTPD, e
            res[prec] = (None, np.inf, e.code)
            log(f"noise {noise:.0e} (kappa {kappa:.1e}) mbcg {prec}: breakdown ({e})")
            continue
        W = host(r.U).T
        true_res = np.linalg.norm(Kh @ W - B, axis=0) / np.linalg.norm(B, axis=0)
        res[prec] = (int(r.iters.max()), float(true_res.max()), r.status)
        log(f"noise {noise:.0e} (kappa {kappa:.1e}) mbcg {prec}: iters {r.iters.max()}, status {r.status}, "
            f"true residual {true_res.max():.1e}")
    it, tr, st = res["fp64"]
    assert tr <= max(1e-8, 100 * kappa * 2.2e-16)
    assert tr <= 1e-2 * res["bf16x3"][1]


def test_fp64_block_cg_at_low_noise():
    """Block CG with FP64 products and half the rows as Nystrom landmarks at sigma^2 = 1e-6: the random
    landmarks include both rows of some nearly repeated pairs (cond K_MM ~ 1e7), which the
    rank-revealing inverse of K_MM keeps from spoiling P^{-1/2}."""
    from paper_2109_09817_amd import gp
    n, s = 1200, 8
    X, y, ell = synth.near_duplicate_pairs(n, 5)
    th = ok.Theta(ell, 1.0, 1e-6)
    Kh = ok.khat(X, th)
    B = np.column_stack([y, np.random.default_rng(3).standard_normal((n, s - 1))])
    M = np.sort(np.random.default_rng(4).choice(n, 600, replace=False))
    pc = gp.nystrom_precond(_gk(th), dev(X), M)
    r = gp.bcg(_gk(th), dev(X), dev(B.T), 3000, 1e-9, pc=pc, precision="fp64")
    W = host(r.W).T
    true_res = np.linalg.norm(Kh @ W - B, axis=0) / np.linalg.norm(B, axis=0)
    log(f"bcg fp64 noise 1e-6: iters {r.iters}, status {r.status}, true residual {true_res.max():.1e}")
    assert true_res.max() <= 1e-6
