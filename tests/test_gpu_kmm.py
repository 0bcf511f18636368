"""Parity of gp_kmm (the fused K_hat V / K(Z, X) V kernels) with the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

import synth
from _helpers import col_rel_err, dev, host
from oracle import kernel as ok

pytestmark = pytest.mark.gpu

# Relative error per vector ||got - ref|| / ||ref|| (the 1e-4 target; FP32 is held tighter).
TOL = {"fp32": 2e-6, "bf16x3": 1e-4}
# The bound on the off-diagonal part s_f M V alone (K_hat V minus its exact diagonal): the mixed
# form's FP16 halves of distance, kernel values and V measure <= 2.2e-5 (the n = 917,504 model as
# configured, where the distance's rounding dominates), so it is held to half the target.
TOL_OFF = {"fp32": 2e-5, "bf16x3": 5e-5}


def _run(kern_np, X, V, prec, Z=None):
    import torch
    from paper_2109_09817_amd import gp
    k = gp.Kernel(kern_np.ell, kern_np.sf, kern_np.noise, "matern52" if kern_np.kind == 0 else "rbf")
    out = gp.kmm(k, dev(X), dev(V), None if Z is None else dev(Z), precision=prec)
    torch.cuda.synchronize()
    return host(out)


def _case(n, d, t, cond, seed, kind=ok.MATERN52):
    p = synth.make_problem("c2", n=n, cond_variant=cond, kind=kind, seed=seed)
    X = p.X[:, :d].copy()
    ell = p.ell[:d]
    if d > X.shape[1]:  # beyond the workload's 48 features: more features of the same kind
        extra = d - X.shape[1]
        rng = np.random.default_rng(seed + 77)
        X = np.hstack([X, X[:, np.arange(extra) % X.shape[1]] + rng.standard_normal((n, extra))])
        ell = np.concatenate([ell, rng.uniform(0.5, 2.0, extra) * (math.sqrt(2 * p.cfg.d) if cond else 1.0)])
    ell = ell * (math.sqrt(d / 48.0) if cond else 1.0)
    th = ok.Theta(ell, 1.3, 1e-3, kind)
    V = synth.random_block(n, t, seed)
    return X, th, V


CASES = [
    # n, d, t, cond-variant lengthscales
    (2048, 32, 9, True),     # the N = 2048 workload's shape (8 probes + y)
    (2048, 32, 9, False),
    (4096 + 17, 48, 16, True),  # several row blocks and a ragged tail
    (333, 7, 3, True),       # smaller than one workgroup
    (1000, 48, 33, True),    # three 16-column blocks
    (1500, 48, 50, True),    # four column blocks, padded (the AltBBMM block size s = 50)
    (700, 20, 64, True),     # four full column blocks
    (900, 64, 16, True),     # the widest features (224 BF16x3 K)
    (600, 48, 100, True),    # two column groups of four blocks
    (1, 5, 1, True),         # degenerate: one point
]


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
@pytest.mark.parametrize("kind", [ok.MATERN52, ok.RBF])
@pytest.mark.parametrize("case", CASES)
def test_square_product_matches_oracle(case, kind, prec):
    n, d, t, cond = case
    print(f"case n={n} d={d} t={t} cond={cond} kind={kind} prec={prec}", file=sys.stderr, flush=True)
    X, th, V = _case(n, d, t, cond, seed=n + t, kind=kind)
    got = _run(th, X, V, prec)
    ref = ok.khat_matmul(X, th, V.T).T
    err = col_rel_err(got, ref)
    diag = (th.sf + th.noise) * V
    err_off = col_rel_err(got - diag, ref - diag) if n > 1 else 0.0
    print(f"  err={err:.3e} err_offdiag={err_off:.3e}", file=sys.stderr, flush=True)
    assert err <= TOL[prec]
    if cond and n > 1:
        assert err_off <= TOL_OFF[prec]
    if n == 1:
        np.testing.assert_allclose(got, (th.sf + th.noise) * V, rtol=1e-15)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
@pytest.mark.parametrize("m", [1, 155, 1000 + 3])
def test_cross_product_matches_oracle(m, prec):
    n, d, t = 3000, 48, 20
    X, th, V = _case(n, d, t, True, seed=5)
    Z = synth.query_molecule("c2", m, seed=m)[:, :d]
    got = _run(th, X, V, prec, Z=Z)
    ref = ok.cross_matmul(Z, X, th, V.T).T
    # over the whole block: with m = 1 a single entry per vector can be a cancelled sum
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"cross m={m} prec={prec} err={err:.3e}", file=sys.stderr, flush=True)
    assert err <= TOL_OFF[prec]


@pytest.mark.parametrize("d", [7, 32, 64])
def test_cross_product_every_feature_width(d):
    # The row-independent cross sweep is instantiated per K step count: d = 7, 32
    # and 64 take 32, 128 and 224 BF16x3 K (48 and 16 are covered above).
    n, t, m = 2500, 40, 99
    X, th, V = _case(n, d, t, True, seed=13)
    Z = synth.query_molecule("c2", m, seed=21)[:, :d]
    if Z.shape[1] < d:  # widen the queries like the training rows
        Z = np.hstack([Z, np.random.default_rng(3).standard_normal((m, d - Z.shape[1]))])
    got = _run(th, X, V, "bf16x3", Z=Z)
    ref = ok.cross_matmul(Z, X, th, V.T).T
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"cross d={d} err={err:.3e}", file=sys.stderr, flush=True)
    assert err <= TOL_OFF["bf16x3"]


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
@pytest.mark.parametrize("d", [80, 128])
def test_products_beyond_the_workload_features(d, prec):
    # Up to the ABI's 128 features: the square product and a cross product.
    n, t, m = 1200, 9, 70
    X, th, V = _case(n, d, t, True, seed=17)
    got = _run(th, X, V, prec)
    ref = ok.khat_matmul(X, th, V.T).T
    err = col_rel_err(got, ref)
    Z = X[:m] + np.random.default_rng(5).standard_normal((m, d)) * 0.1
    gotc = _run(th, X, V, prec, Z=Z)
    refc = ok.cross_matmul(Z, X, th, V.T).T
    errc = float(np.linalg.norm(gotc - refc) / np.linalg.norm(refc))
    print(f"d={d} {prec}: square err {err:.3e} cross err {errc:.3e}", file=sys.stderr, flush=True)
    assert err <= TOL[prec]
    assert errc <= TOL_OFF[prec]


def test_cross_rows_are_independent_of_the_batch():
    # Each query row's result is bitwise the same alone and inside a larger batch.
    n, d, t = 5000, 48, 17
    X, th, V = _case(n, d, t, True, seed=9)
    Z = synth.query_molecule("c2", 300, seed=3)[:, :d]
    full = _run(th, X, V, "bf16x3", Z=Z)
    part = _run(th, X, V, "bf16x3", Z=Z[100:137])
    np.testing.assert_array_equal(full[:, 100:137], part)


@pytest.mark.parametrize("n,d,t,m,kind", [
    (150_000, 48, 257, 150, ok.MATERN52),  # the prediction shape: 1 + 256 columns, 3 row groups (ragged)
    (140_001, 16, 33, 70, ok.RBF),          # 3 column blocks, 2 row groups
    (300_007, 16, 33, 70, ok.MATERN52),     # 37 chunks per split: two FP32 windows into FP64 partials
])
def test_long_split_cross_product_matches_oracle(n, d, t, m, kind):
    # Long chunk splits: up to 32 chunks a split is one FP32 window stored as
    # FP32; beyond n = 262,144 a split spans several windows added into FP64
    # partials.  Also the widest column set and the batch independence at size.
    X, th, V = _case(n, d, t, True, seed=11, kind=kind)
    Z = synth.query_molecule("c2", m, seed=7)[:, :d]
    got = _run(th, X, V, "bf16x3", Z=Z)
    ref = ok.cross_matmul(Z, X, th, V.T).T
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"cross n={n} t={t} m={m} err={err:.3e}", file=sys.stderr, flush=True)
    assert err <= TOL_OFF["bf16x3"]
    part = _run(th, X, V, "bf16x3", Z=Z[64:80])
    np.testing.assert_array_equal(got[:, 64:80], part)


def test_repeat_runs_are_bitwise_identical():
    n, d, t = 4096, 48, 16
    X, th, V = _case(n, d, t, True, seed=2)
    a = _run(th, X, V, "bf16x3")
    b = _run(th, X, V, "bf16x3")
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("name,nrows,cond", [("c2", 65536, True), ("c3d", 131072, True), ("c3o", 917504, True),
                                             ("c3o", 917504, False)])
def test_full_size_sampled_rows(name, nrows, cond):
    # Full-size products (the launch configuration the benchmark times), checked on sampled rows; the
    # N = 917,504 model also as configured (the data the benchmark runs).
    import torch
    from paper_2109_09817_amd import gp
    p = synth.make_problem(name, n=nrows, cond_variant=cond)
    th = ok.Theta(p.ell, p.sf, p.noise)
    t = 16
    V = synth.random_block(nrows, t, 1)
    k = gp.Kernel(p.ell, p.sf, p.noise)
    Xg, Vg = dev(p.X), dev(V)
    rows = np.random.default_rng(0).choice(nrows, 96, replace=False)
    rows = np.concatenate([rows, [0, nrows - 1]])
    for prec in ("bf16x3", "fp32"):
        out = gp.kmm(k, Xg, Vg, precision=prec)
        torch.cuda.synchronize()
        got = host(out)[:, rows]
        ref = ok.khat_matmul(p.X, th, V.T, rows=rows).T
        err = col_rel_err(got, ref)
        diag = (th.sf + th.noise) * V[:, rows]
        err_off = col_rel_err(got - diag, ref - diag)
        print(f"{name} n={nrows} cond={cond} {prec}: err={err:.3e} off={err_off:.3e}", file=sys.stderr, flush=True)
        assert err <= TOL[prec]
        assert err_off <= TOL_OFF[prec]
        del out


FP64_CASES = [
    (333, 7, 3, True),
    (2048 + 17, 48, 16, True),   # ragged last chunk
    (1000, 64, 20, True),        # widest features of the form, two column groups
    (1, 5, 1, True),
    (2048, 32, 9, False),
    (1500 + 3, 48, 50, True),    # block CG width: four column groups, one per wave
    (777, 32, 40, True),         # three column groups (one wave idle in the product)
    (500, 64, 64, False),        # the widest single pass
    (300 + 1, 16, 70, True),     # two passes over the columns
]


@pytest.mark.parametrize("kind", [ok.MATERN52, ok.RBF])
@pytest.mark.parametrize("case", FP64_CASES)
def test_fp64_square_product_matches_oracle(case, kind):
    """The FP64 form (low-noise regime): agreement to FP64 rounding of the sums."""
    n, d, t, cond = case
    X, th, V = _case(n, d, t, cond, seed=n + t + 1, kind=kind)
    got = _run(th, X, V, "fp64")
    ref = ok.khat_matmul(X, th, V.T).T
    # error against the same sum of magnitudes: rounding is relative to |K| |V|, not to the result
    scale = ok.khat_matmul(X, ok.Theta(th.ell, th.sf, th.noise, th.kind), np.abs(V).T).T
    err = np.max(np.abs(got - ref) / scale)
    print(f"fp64 case n={n} d={d} t={t} kind={kind}: err / |K||V| = {err:.2e}", file=sys.stderr, flush=True)
    assert err <= 1e-13


@pytest.mark.parametrize("m", [1, 155])
def test_fp64_cross_product_matches_oracle(m):
    n, d, t = 3000, 48, 20
    X, th, V = _case(n, d, t, True, seed=6)
    Z = synth.query_molecule("c2", m, seed=m)[:, :d]
    got = _run(th, X, V, "fp64", Z=Z)
    ref = ok.cross_matmul(Z, X, th, V.T).T
    scale = ok.cross_matmul(Z, X, th, np.abs(V).T).T
    err = np.max(np.abs(got - ref) / scale)
    assert err <= 1e-13


MID_CASES = [
    # n, d, t, kind: mid-size square products, ragged tails, every instantiated K-step class
    (32768, 48, 16, ok.MATERN52),
    (40000 + 37, 48, 9, ok.MATERN52),   # ragged last chunk and last 256-row workgroup
    (40000 + 37, 32, 1, ok.RBF),        # a single column, the other kernel, 4 K steps
    (50001, 7, 16, ok.MATERN52),        # 2 K steps
]


@pytest.mark.parametrize("n,d,t,kind", MID_CASES)
def test_mid_size_square_products_match_oracle(n, d, t, kind):
    """Rows at every 768th boundary, the first and last rows and random rows against the oracle; two
    runs bitwise identical."""
    X, th, V = _case(n, d, t, True, seed=5, kind=kind)
    band = 768
    edges = [r for b in range(band, n, band) for r in (b - 1, b, b + 1)]
    rows = np.unique(np.concatenate([np.random.default_rng(1).choice(n, 64, replace=False), edges[:60],
                                     [0, 1, 255, 256, n - 2, n - 1]]))
    rows = rows[rows < n]
    got = _run(th, X, V, "bf16x3")
    ref = ok.khat_matmul(X, th, V.T, rows=rows).T
    err = col_rel_err(got[:, rows], ref)
    diag = (th.sf + th.noise) * V[:, rows]
    err_off = col_rel_err(got[:, rows] - diag, ref - diag)
    again = _run(th, X, V, "bf16x3")
    print(f"square n={n} d={d} t={t} kind={kind}: err={err:.3e} off={err_off:.3e} rows={rows.size}",
          file=sys.stderr, flush=True)
    assert err <= TOL["bf16x3"]
    assert err_off <= TOL_OFF["bf16x3"]
    np.testing.assert_array_equal(got, again)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_products_do_not_depend_on_an_offset_of_the_data(prec):
    """The kernel depends on differences only.  The mixed form centres its FP16 coordinates on the
    training points' column means, so shifting every point (training and query) by 10^4 lengthscales leaves
    its results at the unshifted accuracy; the FP32 form's norms are not centred and are checked
    only at a small offset."""
    n, d, t, m = 3000, 48, 9, 155
    X, th, V = _case(n, d, t, True, seed=19)
    Z = synth.query_molecule("c2", m, seed=4)[:, :d]
    shift = (1e4 if prec == "bf16x3" else 1.0) * th.ell * np.random.default_rng(2).choice([-1.0, 1.0], d)
    ref = ok.khat_matmul(X, th, V.T).T
    refc = ok.cross_matmul(Z, X, th, V.T).T
    got = _run(th, X + shift, V, prec)
    gotc = _run(th, X + shift, V, prec, Z=Z + shift)
    diag = (th.sf + th.noise) * V
    err_off = col_rel_err(got - diag, ref - diag)
    errc = float(np.linalg.norm(gotc - refc) / np.linalg.norm(refc))
    print(f"offset {prec}: square off-diagonal err {err_off:.3e}, cross err {errc:.3e}", file=sys.stderr, flush=True)
    assert err_off <= TOL_OFF[prec] and errc <= TOL_OFF[prec]


def test_mixed_form_columns_of_any_magnitude():
    """The mixed form scales each column of V by a power of two before its FP16 split, so columns
    of very different magnitudes (1e-300 to 1e300, a zero column, a column below FP32's range)
    keep the accuracy of a unit column, and a non-finite entry stays in its own column.  (Arrays
    here hold one column per row, as the other tests' do.)"""
    n, d, t, m = 2500, 48, 9, 97
    X, th, V = _case(n, d, t, True, seed=41)
    V = V.copy()
    mags = [1.0, 1e-300, 1e300, 0.0, 1e-45, 3.7e5, 1e-12, 1.0, 1.0]
    for c, s in enumerate(mags):
        V[c] *= s
    Z = synth.query_molecule("c2", m, seed=8)[:, :d]
    ref = ok.khat_matmul(X, th, V.T).T
    refc = ok.cross_matmul(Z, X, th, V.T).T
    got = _run(th, X, V, "bf16x3")
    gotc = _run(th, X, V, "bf16x3", Z=Z)
    diag = (th.sf + th.noise) * V
    for c, s in enumerate(mags):
        if s == 0.0:
            assert not np.any(got[c]) and not np.any(gotc[c])
            continue
        # norms of the columns divided by their magnitude (squares of 1e-300 or 1e300 leave FP64)
        g_off, r_off = (got - diag)[c] / s, (ref - diag)[c] / s
        e_off = float(np.linalg.norm(g_off - r_off) / np.linalg.norm(r_off))
        e_c = float(np.linalg.norm(gotc[c] / s - refc[c] / s) / np.linalg.norm(refc[c] / s))
        print(f"column scale {s:.1e}: off-diagonal err {e_off:.3e}, cross err {e_c:.3e}", file=sys.stderr, flush=True)
        assert e_off <= TOL_OFF["bf16x3"] and e_c <= TOL_OFF["bf16x3"]
    V[8, 7] = np.nan
    got = _run(th, X, V, "bf16x3")
    assert np.all(np.isnan(got[8])) and np.all(np.isfinite(got[:8]))


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_products_with_an_outlying_first_point(prec):
    """The first training point moved 100 lengthscales away from the rest: the mixed form's centre is
    the column mean, not a data point, so the other points' coordinates stay small and their distances
    keep their accuracy."""
    n, d, t, m = 3000, 48, 9, 155
    X, th, V = _case(n, d, t, True, seed=29)
    X = X.copy()
    X[0] += 100.0 * th.ell
    Z = synth.query_molecule("c2", m, seed=6)[:, :d]
    ref = ok.khat_matmul(X, th, V.T).T
    refc = ok.cross_matmul(Z, X, th, V.T).T
    got = _run(th, X, V, prec)
    gotc = _run(th, X, V, prec, Z=Z)
    diag = (th.sf + th.noise) * V
    err_off = col_rel_err(got - diag, ref - diag)
    errc = float(np.linalg.norm(gotc - refc) / np.linalg.norm(refc))
    print(f"outlying first point {prec}: square off-diagonal err {err_off:.3e}, cross err {errc:.3e}",
          file=sys.stderr, flush=True)
    assert err_off <= TOL_OFF[prec] and errc <= TOL_OFF[prec]


def test_mixed_form_out_of_range_coordinates_give_nan():
    """A training point whose scaled coordinate lies beyond the FP16 range of the mixed form's distance
    (about 10^4 lengthscales from the training points' column means) makes the product NaN rather than silently wrong;
    the FP32 form still computes it."""
    n, d, t = 700, 16, 3
    X, th, V = _case(n, d, t, True, seed=23)
    X = X.copy()
    X[n // 2, 3] += 1e5 * th.ell[3]
    got = _run(th, X, V, "bf16x3")
    assert np.all(np.isnan(got))
    ref = ok.khat_matmul(X, th, V.T).T
    assert col_rel_err(_run(th, X, V, "fp32"), ref) <= TOL["fp32"]
    # a solve on such data stops with a non-finite error instead of running to max_iter
    from paper_2109_09817_amd import _lib, gp
    k = gp.Kernel(th.ell, th.sf, th.noise)
    with pytest.raises(_lib.GpError) as e:
        gp.mbcg(k, dev(X), dev(V), 50, 1e-6, precision="bf16x3")
    assert e.value.code == _lib.GP_ENONFINITE
