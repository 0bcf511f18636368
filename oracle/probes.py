"""Oracle: Rademacher probe vectors from a counter-based hash.  Test infrastructure only.

The block right-hand side of the solver is B = [y | b_1 .. b_t] (paper Sec. 3.1
sets y_0 = y and random y_i for i > 0).  Probes are Rademacher rather than
Gaussian, and with a preconditioner P = L L^T + sigma^2 I they are drawn as

    b_i = L eps1_i + sigma eps2_i,   eps1_i in {+-1}^k,  eps2_i in {+-1}^N,

so that E[b b^T] = L L^T + sigma^2 I = P; then z = P^{-1/2} b has identity
covariance and both the stochastic log-determinant and the trace estimates are
unbiased.  Without a preconditioner (P = I) b_i = eps2_i.

Signs come from SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014): one generator step from state x is

    z = x + 0x9E3779B97F4A7C15
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    out = z ^ (z >> 31)                         (all mod 2^64)

The key of a seed is one step from the seed; the sign of (stream, row) is the
top bit of one step from key ^ ((stream << 40) | row): bit 0 gives +1, bit 1
gives -1.  Probe column c (1..t) uses stream c for eps2 and stream c + 65536
for eps1.
"""
from __future__ import annotations

import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
EPS1_STREAM_OFFSET = 65536


def splitmix64(x) -> np.ndarray:
    """One SplitMix64 output for each uint64 state in x (vectorised, wraps mod 2^64)."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = z + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def seed_key(seed: int) -> np.uint64:
    return splitmix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]


def rademacher(seed: int, stream: int, nrows: int) -> np.ndarray:
    """Signs (+1.0 / -1.0) of rows 0..nrows-1 of one stream."""
    key = seed_key(seed)
    rows = np.arange(nrows, dtype=np.uint64)
    ctr = key ^ ((np.uint64(stream) << np.uint64(40)) | rows)
    top = splitmix64(ctr) >> np.uint64(63)
    return 1.0 - 2.0 * top.astype(np.float64)


def probe_block(seed: int, y: np.ndarray, t: int, L: np.ndarray, noise: float) -> np.ndarray:
    """B = [y | b_1..b_t] as an (n, t+1) array; L is the (n, k) factor (k may be 0)."""
    n = y.shape[0]
    k = 0 if L is None else L.shape[1]
    B = np.empty((n, t + 1))
    B[:, 0] = y
    for c in range(1, t + 1):
        e2 = rademacher(seed, c, n)
        if k == 0:
            B[:, c] = e2
        else:
            e1 = rademacher(seed, c + EPS1_STREAM_OFFSET, k)
            B[:, c] = L @ e1 + math.sqrt(noise) * e2
    return B
