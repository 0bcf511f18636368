"""gp_kmm_noalloc (the product of gp_kmm with the library's fixed device scratch) against
gp_kmm with a caller workspace, on consecutive calls that shrink, through the C ABI."""
import sys

import numpy as np
import pytest

import synth
from _helpers import dev, host

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _case(n, t, seed, d=48):
    p = synth.make_problem("c2", n=n, cond_variant=True, seed=seed)
    V = synth.random_block(n, t, seed)
    return np.ascontiguousarray(p.X[:, :d]), V, p.ell[:d], p.noise


# consecutive calls, each smaller than the one before: the scratch keeps the previous call's
# contents, which the next call must never read
CALLS = [
    ("square bf16x3", 5000, 16, None, "bf16x3"),
    ("square bf16x3, smaller, ragged", 3001, 9, None, "bf16x3"),
    ("cross fp32", 2500, 5, 333, "fp32"),
    ("square fp64", 700, 3, None, "fp64"),
]


def test_noalloc_matches_workspace_entry_point():
    import torch
    from paper_2109_09817_amd import gp
    for i, (what, n, t, m, prec) in enumerate(CALLS):
        X, V, ell, noise = _case(n, t, 40 + i)
        k = gp.Kernel(ell, 1.1, noise)
        Xd, Vd = dev(X), dev(V)
        Zd = dev(synth.query_molecule("c2", m, seed=9)[:, :X.shape[1]]) if m else None
        rows = n if m is None else m
        ref = gp.kmm(k, Xd, Vd, Z=Zd, precision=prec)
        out = torch.full((t, rows), float("nan"), dtype=torch.float64, device=Xd.device)
        gp.kmm_noalloc(k, Xd, Vd, out, Z=Zd, precision=prec)
        torch.cuda.synchronize()
        got, want = host(out), host(ref)
        log(f"noalloc call {i} ({what}, n={n}, t={t}): max |diff| {np.max(np.abs(got - want)):.1e}")
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got, want)  # the same kernels on the same plan: bitwise


def test_noalloc_rejects_oversize_product():
    from paper_2109_09817_amd import _lib, gp
    n, t = 40000, 16
    X, V, ell, noise = _case(n, t, 7)
    out = dev(np.zeros((t, n)))
    with pytest.raises(_lib.GpError) as e:
        gp.kmm_noalloc(gp.Kernel(ell, 1.0, noise), dev(X), dev(V), out, precision="bf16x3")
    assert e.value.code == _lib.GP_EWORKSPACE
    assert np.all(host(out) == 0.0)  # rejected before any GPU work
