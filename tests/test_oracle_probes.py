"""Pins of the probe generator: the published reference outputs, integer arithmetic, sign statistics,
covariance by enumeration."""
import itertools
import math
import os

import numpy as np

from oracle import probes

MASK = (1 << 64) - 1


def _splitmix_int(x: int) -> int:
    # the same generator step evaluated with Python's unbounded integers
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "splitmix64_reference.txt")


def test_splitmix64_matches_published_reference_outputs():
    # The reference generator's k-th output from seed s is one oracle step applied to the state
    # s + (k - 1) * 0x9E3779B97F4A7C15 (the step adds the increment once more before mixing).
    rows = [line.split() for line in open(GOLDEN) if line.strip() and not line.startswith("#")]
    assert len(rows) == 10
    for seed, k, hexval in rows:
        state = (int(seed) + (int(k) - 1) * 0x9E3779B97F4A7C15) & MASK
        got = int(probes.splitmix64(np.array([state], dtype=np.uint64))[0])
        assert got == int(hexval, 16), (seed, k)


def test_vectorised_uint64_matches_big_integer_arithmetic():
    xs = [0, 1, 2, 12345, MASK, MASK - 7, 1 << 63, 0x0123456789ABCDEF]
    got = probes.splitmix64(np.array(xs, dtype=np.uint64))
    assert [int(g) for g in got] == [_splitmix_int(x) for x in xs]


def test_signs_from_big_integer_reference():
    seed, stream, n = 42, 3, 257
    key = _splitmix_int(seed)
    ref = [1.0 if (_splitmix_int(key ^ ((stream << 40) | r)) >> 63) == 0 else -1.0 for r in range(n)]
    np.testing.assert_array_equal(probes.rademacher(seed, stream, n), ref)


def test_sign_statistics():
    n = 1 << 16
    a = probes.rademacher(7, 1, n)
    b = probes.rademacher(7, 2, n)
    c = probes.rademacher(8, 1, n)
    assert set(np.unique(a)) == {-1.0, 1.0}
    for v in (a, b, c):
        assert abs(v.mean()) < 5 / math.sqrt(n)
    for u, v in ((a, b), (a, c), (b, c)):
        assert abs(np.mean(u * v)) < 5 / math.sqrt(n)
    assert abs(np.mean(a[1:] * a[:-1])) < 5 / math.sqrt(n)


def test_probe_covariance_equals_preconditioner_by_enumeration():
    # b = L e1 + sigma e2 with all 2^(k+n) sign patterns: mean of b b^T is exactly L L^T + sigma^2 I.
    rng = np.random.default_rng(0)
    n, k, noise = 6, 3, 0.3
    L = rng.standard_normal((n, k))
    acc = np.zeros((n, n))
    count = 0
    for s in itertools.product((-1.0, 1.0), repeat=n + k):
        e = np.array(s)
        b = L @ e[:k] + math.sqrt(noise) * e[k:]
        acc += np.outer(b, b)
        count += 1
    np.testing.assert_allclose(acc / count, L @ L.T + noise * np.eye(n), atol=1e-12)


def test_probe_block_layout():
    rng = np.random.default_rng(1)
    n, k, t = 40, 5, 4
    L = rng.standard_normal((n, k))
    y = rng.standard_normal(n)
    B = probes.probe_block(9, y, t, L, 0.25)
    np.testing.assert_array_equal(B[:, 0], y)
    for c in range(1, t + 1):
        e1 = probes.rademacher(9, c + probes.EPS1_STREAM_OFFSET, k)
        e2 = probes.rademacher(9, c, n)
        np.testing.assert_allclose(B[:, c], L @ e1 + 0.5 * e2, rtol=0, atol=1e-14)
    B0 = probes.probe_block(9, y, t, np.zeros((n, 0)), 0.25)
    np.testing.assert_array_equal(B0[:, 2], probes.rademacher(9, 2, n))
