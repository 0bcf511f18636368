"""Write the stored oracle results of the N = 65,536 and N = 131,072 models.

Runs on the CPU and calls only ``oracle/`` (plus the seeded inputs of ``synth``): the
pivoted-Cholesky preconditioner, the probe block, textbook mBCG, stochastic Lanczos
quadrature, the mll (Eq. 2) and its estimated gradient (Sec. 3.2) for one BBMM
evaluation of each model, with the probe seed and solver settings of the workload.
The K_hat products and the gradient forms are summed over row slices in a process
pool (each slice is an ordinary oracle call; the slices partition the rows).

    python tests/golden/make_config_goldens.py [c2] [c3d]     (minutes to an hour)

Writes tests/golden/config_<name>.json.
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import kernel as ok  # noqa: E402
from oracle.gradient import bilinear_forms, mll_gradient_forms  # noqa: E402
from oracle.mbcg import mbcg, mll_from_solve, slq_logdet  # noqa: E402
from oracle.pivchol import Preconditioner, pivoted_cholesky  # noqa: E402
from oracle.probes import probe_block  # noqa: E402

PROBE_SEED = 17     # probe seed of the stored evaluation
SAMPLED_ROWS = 64   # rows of the solve block that are stored
ALPHA_ITERS = 6     # CG coefficients stored per column

_G = {}


def _init(X, th, U=None, V=None, w=None):
    _G.update(X=X, th=th, U=U, V=V, w=w)


def _kmm_slice(args):
    rows, D = args
    return ok.khat_matmul(_G["X"], _G["th"], D, rows=rows)


def _forms_slice(r):
    return bilinear_forms(_G["X"], _G["th"], _G["U"], _G["V"], _G["w"], block=16, rows=r)


def _slices(n, parts):
    edges = np.linspace(0, n, parts + 1).astype(np.int64)
    return [(int(edges[i]), int(edges[i + 1])) for i in range(parts)]


def run(name: str, workers: int) -> dict:
    cfg = synth.CONFIGS[name]
    p = synth.make_problem(name)
    X, y = p.X, p.y
    n = X.shape[0]
    th = ok.Theta(p.ell, p.sf, p.noise)
    t0 = time.time()
    L, piv, _ = pivoted_cholesky(X, th, cfg.rank)
    P = Preconditioner(L, th.noise)
    B = probe_block(PROBE_SEED, y, cfg.probes, L, th.noise)
    print(f"{name}: n={n} preconditioner and probes {time.time() - t0:.1f} s", flush=True)
    with mp.get_context("fork").Pool(workers, initializer=_init, initargs=(X, th)) as pool:
        parts = _slices(n, 4 * workers)

        def matmul(D):
            t1 = time.time()
            out = np.vstack(pool.map(_kmm_slice, [(np.arange(a, b), D) for a, b in parts]))
            print(f"  K_hat V ({D.shape[1]} columns) {time.time() - t1:.1f} s", flush=True)
            return out

        res = mbcg(matmul, B, P.solve, cfg.max_iter, cfg.tol)
    logdet = slq_logdet(res, P.logdet, range(1, cfg.probes + 1))
    mll = mll_from_solve(y, res["U"][:, 0], logdet)
    U, V, w = mll_gradient_forms(res["U"], res["Z0"], cfg.probes)
    t1 = time.time()
    with mp.get_context("fork").Pool(workers, initializer=_init, initargs=(X, th, U, V, w)) as pool:
        grad = np.sum(pool.map(_forms_slice, _slices(n, 64 * workers)), axis=0)
    print(f"  gradient forms {time.time() - t1:.1f} s", flush=True)
    rows = np.sort(np.random.default_rng(np.random.SeedSequence([cfg.seed, 31])).choice(n, SAMPLED_ROWS,
                                                                                         replace=False))
    J = min(ALPHA_ITERS, res["alpha"].shape[0])
    return {
        "config": name,
        "n": n,
        "d": int(X.shape[1]),
        "y_sum": float(np.sum(y)),
        "seed": PROBE_SEED,
        "probes": cfg.probes,
        "rank": cfg.rank,
        "tol": cfg.tol,
        "max_iter": cfg.max_iter,
        "pivots": [int(i) for i in piv],
        "logdet_p": float(P.logdet),
        "gamma0": [float(v) for v in res["gamma0"]],
        "iters": [int(v) for v in res["iters"]],
        "alpha": res["alpha"][:J].tolist(),
        "beta": res["beta"][:J].tolist(),
        "rows": [int(r) for r in rows],
        "U_rows": res["U"][rows, :].T.tolist(),  # (t + 1, rows): column c of the solve block
        "quad": float(y @ res["U"][:, 0]),
        "logdet": float(logdet),
        "mll": float(mll),
        "grad": [float(v) for v in grad],
        "oracle_seconds": round(time.time() - t0, 1),
    }


def main(argv):
    names = [a for a in argv if not a.startswith("-")] or ["c2", "c3d"]
    workers = min(8, os.cpu_count() or 1)
    for name in names:
        out = run(name, workers)
        path = os.path.join(HERE, f"config_{name}.json")
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print(f"wrote {path} ({out['oracle_seconds']} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
