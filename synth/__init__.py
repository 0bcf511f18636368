"""Seeded synthetic inputs shaped like MOB-ML pair-feature data.

This module only draws random inputs: feature matrices, lengthscales,
regression targets, probe seeds and request streams.  It holds none of the
Gaussian-process arithmetic of the method (no kernel matrix, no solve, no
Krylov iteration), so both the FP64 oracle and the GPU path may consume its
arrays without sharing any computation.

The real training data of the paper (QM7b-T / GDB-13-T pair energies, Sec. 4)
is not available; these generators stand in for it with the same shapes:

* feature vectors come in "molecules" of 10..300 rows (the paper trains on
  about 177 off-diagonal and 19 diagonal pairs per molecule, Tables 1-2), each
  molecule drawn around one of 64 cluster means (means ~ N(0, 4 I), unit
  variance inside a cluster);
* lengthscales are U(0.5, 2) per feature, outputscale 1;
* targets are a random-Fourier-feature sample of the Matern-5/2 (or RBF) prior
  plus Gaussian noise, so the GP model is well specified.

Every stream is derived from one master seed through
``numpy.random.SeedSequence`` and named child streams, so that any array can be
regenerated exactly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

MATERN52 = 0
RBF = 1

_STREAMS = ("means", "assign", "rows", "ell", "rff", "ynoise", "probes", "arrivals")


def streams(seed: int, model: int = 0) -> Dict[str, np.random.Generator]:
    """Named, independent generators spawned from one master seed."""
    ss = np.random.SeedSequence([int(seed), int(model)])
    kids = ss.spawn(len(_STREAMS))
    return {name: np.random.default_rng(k) for name, k in zip(_STREAMS, kids)}


@dataclasses.dataclass(frozen=True)
class Config:
    """One workload: sizes and solver knobs (the arithmetic lives elsewhere)."""

    name: str
    n: int
    d: int
    layout: str  # "mixture" (row-wise components) or "clustered" (molecules)
    ncomp: int
    noise: float
    probes: int  # Rademacher probe columns t (the block adds y as column 0)
    rank: int  # pivoted-Cholesky preconditioner rank k
    max_iter: int
    tol: float
    seed: int
    model: int = 0
    kind: int = MATERN52


CONFIGS: Dict[str, Config] = {
    # exact GP small enough for a dense FP64 Cholesky in seconds
    "c1": Config("c1", 2048, 32, "mixture", 8, 1e-2, 8, 20, 30, 0.0, 1),
    # plain method at N = 65,536, tolerance 1e-3
    "c2": Config("c2", 65536, 48, "clustered", 64, 1e-3, 15, 100, 100, 1e-3, 2),
    # the two independent models of the N = 1,048,576 run
    "c3o": Config("c3o", 917504, 48, "clustered", 64, 1e-3, 15, 100, 100, 1e-6, 3, 0),
    "c3d": Config("c3d", 131072, 48, "clustered", 64, 1e-3, 15, 100, 100, 1e-6, 3, 1),
    # hyperparameter-gradient workload
    "c4": Config("c4", 262144, 48, "clustered", 64, 1e-3, 32, 100, 100, 1e-6, 4),
    # serving model (same shape as c4)
    "c5": Config("c5", 262144, 48, "clustered", 64, 1e-3, 32, 100, 100, 1e-6, 5),
}


def component_means(rs, ncomp: int, d: int) -> np.ndarray:
    return 2.0 * rs["means"].standard_normal((ncomp, d))


def mixture_rows(n: int, d: int, ncomp: int, rs) -> np.ndarray:
    """Each row independently picks one of ``ncomp`` unit-variance components."""
    mu = component_means(rs, ncomp, d)
    c = rs["assign"].integers(0, ncomp, size=n)
    return mu[c] + rs["rows"].standard_normal((n, d))


def molecule_sizes(n: int, rng: np.random.Generator, lo: int = 10, hi: int = 300) -> np.ndarray:
    """Sizes U{lo..hi} drawn until they cover n rows; the last one is truncated."""
    sizes = []
    total = 0
    while total < n:
        m = int(rng.integers(lo, hi + 1))
        m = min(m, n - total)
        sizes.append(m)
        total += m
    return np.asarray(sizes, dtype=np.int64)


def clustered_rows(n: int, d: int, ncomp: int, rs):
    """Molecules of 10..300 contiguous rows, each molecule around one cluster mean."""
    mu = component_means(rs, ncomp, d)
    sizes = molecule_sizes(n, rs["assign"])
    comp = rs["assign"].integers(0, ncomp, size=len(sizes))
    mol = np.repeat(np.arange(len(sizes)), sizes)
    X = mu[comp[mol]] + rs["rows"].standard_normal((n, d))
    return X, mol


def lengthscales(d: int, rng: np.random.Generator, lo: float = 0.5, hi: float = 2.0) -> np.ndarray:
    return rng.uniform(lo, hi, size=d)


class RandomFeatures:
    """A random-Fourier-feature sample path of a stationary ARD prior.

    f(x) = sqrt(2 s_f / D) * sum_m w_m cos(omega_m . x + b_m).  The frequencies
    follow the kernel's spectral density: Gaussian for RBF, a multivariate
    Student-t with 5 degrees of freedom for Matern-5/2 (Rahimi & Recht 2007).
    """

    def __init__(self, d, ell, sf, kind, rng, D=512):
        g = rng.standard_normal((D, d))
        if kind == MATERN52:
            u = rng.chisquare(5.0, size=D)
            scale = np.sqrt(5.0 / u)[:, None]
        else:
            scale = np.ones((D, 1))
        self.omega = (g / np.asarray(ell)[None, :]) * scale
        self.b = rng.uniform(0.0, 2.0 * math.pi, size=D)
        self.w = rng.standard_normal(D)
        self.amp = math.sqrt(2.0 * sf / D)

    def __call__(self, X: np.ndarray, chunk: int = 65536) -> np.ndarray:
        out = np.empty(X.shape[0])
        for s in range(0, X.shape[0], chunk):
            ph = X[s:s + chunk] @ self.omega.T + self.b
            out[s:s + chunk] = self.amp * (np.cos(ph) @ self.w)
        return out


@dataclasses.dataclass
class Problem:
    X: np.ndarray  # (n, d) FP64, row-major
    y: np.ndarray  # (n,)
    ell: np.ndarray  # (d,) generating lengthscales
    sf: float
    noise: float
    kind: int
    mol: Optional[np.ndarray]
    cfg: Config
    cond_variant: bool


def make_problem(name: str, n: Optional[int] = None, cond_variant: bool = False,
                 kind: Optional[int] = None, seed: Optional[int] = None) -> Problem:
    """Draw the inputs of one workload.

    ``n`` overrides the row count (for test-sized versions of a workload).
    ``cond_variant`` multiplies every lengthscale by sqrt(2d): with unit
    variance clusters in d = 32..48 dimensions the literal workloads give a
    nearly diagonal kernel matrix; the variant gives an ill-conditioned one.
    """
    cfg = CONFIGS[name]
    n = cfg.n if n is None else int(n)
    kind = cfg.kind if kind is None else int(kind)
    rs = streams(cfg.seed if seed is None else seed, cfg.model)
    if cfg.layout == "mixture":
        X = mixture_rows(n, cfg.d, cfg.ncomp, rs)
        mol = None
    else:
        X, mol = clustered_rows(n, cfg.d, cfg.ncomp, rs)
    ell = lengthscales(cfg.d, rs["ell"])
    if cond_variant:
        ell = ell * math.sqrt(2.0 * cfg.d)
    sf = 1.0
    f = RandomFeatures(cfg.d, ell, sf, kind, rs["rff"])
    y = f(X) + math.sqrt(cfg.noise) * rs["ynoise"].standard_normal(n)
    return Problem(np.ascontiguousarray(X), y, ell, sf, cfg.noise, kind, mol, cfg, cond_variant)


def near_duplicate_pairs(n: int, seed: int, jitter: float = 1e-3):
    """The ill-conditioned variant of the n = 65,536 workload's layout at n // 2 rows, each row paired
    with a copy moved by ``jitter`` of a lengthscale per feature (N(0, 1) directions).  Like the nearly
    repeated pair features of molecular data, the pairs make K nearly singular (lambda_min ~ 1e-5 at
    jitter 1e-3), so that the noise level decides the conditioning.  Returns (X, y, ell); the targets
    of a pair are equal."""
    p = make_problem("c2", n=n // 2, cond_variant=True, seed=seed)
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 100]))
    X = np.vstack([p.X, p.X + jitter * p.ell * rng.standard_normal(p.X.shape)])
    return np.ascontiguousarray(X), np.concatenate([p.y, p.y]), p.ell


def molecule_subset(mol: np.ndarray, count: int, seed: int) -> np.ndarray:
    """Sorted row indices of ``count`` molecules drawn uniformly without replacement (the molecule ids
    ``mol`` of a clustered layout)."""
    ids = np.unique(mol)
    if count > ids.size:
        raise ValueError(f"{count} molecules requested, {ids.size} available")
    pick = np.random.default_rng(np.random.SeedSequence([int(seed), 13])).choice(ids, count, replace=False)
    return np.flatnonzero(np.isin(mol, pick))


def random_block(n: int, t: int, seed: int) -> np.ndarray:
    """A dense (t, n) block of N(0,1) right-hand sides (column c is row c)."""
    return np.random.default_rng(np.random.SeedSequence([int(seed), 7])).standard_normal((t, n))


def query_molecule(cfg_name: str, rows: int, seed: int) -> np.ndarray:
    """One request: a new molecule of ``rows`` feature vectors from the same mixture."""
    cfg = CONFIGS[cfg_name]
    rs = streams(cfg.seed, cfg.model)
    mu = component_means(rs, cfg.ncomp, cfg.d)
    r = np.random.default_rng(np.random.SeedSequence([int(seed), 11]))
    c = int(r.integers(0, cfg.ncomp))
    return mu[c] + r.standard_normal((rows, cfg.d))


def request_stream(rate: float, duration: float, seed: int, lo: int = 10, hi: int = 300, count=None):
    """Poisson arrivals: (arrival_time_s, rows, request_seed) tuples, those before `duration`
    seconds, or exactly `count` of them when a count is given (duration then unused)."""
    r = np.random.default_rng(np.random.SeedSequence([int(seed), 13]))
    t = 0.0
    out = []
    i = 0
    while True:
        t += r.exponential(1.0 / rate)
        if (count is None and t >= duration) or (count is not None and i >= count):
            break
        out.append((t, int(r.integers(lo, hi + 1)), int(seed) * 1_000_003 + i))
        i += 1
    return out
