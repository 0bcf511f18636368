"""The C ABI on the CPU: the library loads, exports every declared symbol, and rejects
bad arguments before any GPU work (no compute call is made here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from _helpers import ROOT, ensure_built

HEADER = os.path.join(ROOT, "include", "gpkmm.h")


@pytest.fixture(scope="module")
def lib():
    ensure_built()
    from paper_2109_09817_amd import _lib
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "gp_kmm" in names and "gp_mbcg" in names and len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    from paper_2109_09817_amd import _lib
    assert set(names) == set(_lib.PROTOTYPES), "binding and header disagree"


def test_version_and_error_strings(lib):
    assert b"gfx950" in lib.gp_version()


def _kernel(d=4, ell=1.0, sf=1.0, noise=1e-2, kind=0):
    from paper_2109_09817_amd import _lib
    return _lib.kernel_struct(kind, np.full(d, ell), sf, noise)


BAD = [
    dict(kind=7),
    dict(ell=0.0),
    dict(ell=-1.0),
    dict(ell=float("nan")),
    dict(sf=0.0),
    dict(noise=-1e-3),
    dict(d=0),
    dict(d=129),
]


@pytest.mark.parametrize("bad", BAD)
def test_kmm_rejects_bad_kernel(lib, bad):
    from paper_2109_09817_amd import _lib
    kw = dict(d=4)
    kw.update(bad)
    d = kw["d"]
    ell = np.full(max(d, 1), kw.get("ell", 1.0))
    k = _lib.GpKernel(kw.get("kind", 0), d, ell.ctypes.data_as(C.POINTER(C.c_double)), kw.get("sf", 1.0),
                      kw.get("noise", 1e-2))
    fake = 4096  # never dereferenced: validation fails first
    rc = lib.gp_kmm(C.byref(k), 1, fake, 10, None, 0, fake, 10, 2, fake + 8, 10, None, 0, None)
    assert rc == _lib.GP_EINVAL
    assert lib.gp_last_error()


def test_kmm_rejects_bad_shapes_and_workspace(lib):
    from paper_2109_09817_amd import _lib
    k, keep = _kernel()
    fake = 4096
    assert lib.gp_kmm(C.byref(k), 1, None, 10, None, 0, fake, 10, 2, fake, 10, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_kmm(C.byref(k), 1, fake, 0, None, 0, fake, 10, 2, fake * 2, 10, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_kmm(C.byref(k), 9, fake, 10, None, 0, fake, 10, 2, fake * 2, 10, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_kmm(C.byref(k), 1, fake, 10, None, 0, fake, 5, 2, fake * 2, 10, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_kmm(C.byref(k), 1, fake, 10, None, 0, fake, 10, 0, fake * 2, 10, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_kmm(C.byref(k), 1, fake, 10, None, 0, fake, 10, 2, fake, 10, None, 0, None) == _lib.GP_EINVAL
    # workspace missing / too small / misaligned
    assert lib.gp_kmm(C.byref(k), 1, fake, 10, None, 0, fake, 10, 2, fake * 2, 10, None, 0, None) == _lib.GP_EWORKSPACE
    assert lib.gp_kmm(C.byref(k), 1, fake, 10, None, 0, fake, 10, 2, fake * 2, 10, fake * 4, 16, None) == _lib.GP_EWORKSPACE
    assert lib.gp_kmm(C.byref(k), 1, fake, 10, None, 0, fake, 10, 2, fake * 2, 10, fake + 3, 1 << 30, None) == _lib.GP_EWORKSPACE
    assert b"workspace" in lib.gp_last_error()


def test_kmm_noalloc_rejects_on_the_host(lib):
    """gp_kmm_noalloc checks its arguments as gp_kmm does and refuses products whose scratch exceeds
    the library's fixed array, both before any GPU work."""
    from paper_2109_09817_amd import _lib
    k, keep = _kernel(d=48)
    fake = 4096  # never dereferenced: validation fails first
    n = 40000
    assert lib.gp_workspace_bytes(_lib.GP_OP_KMM, n, 0, 48, 16, 0, 1) > _lib.GP_KMM_NOALLOC_MAX_BYTES
    assert lib.gp_kmm_noalloc(C.byref(k), 1, fake, n, None, 0, fake, n, 16, fake * 2, n, None) == _lib.GP_EWORKSPACE
    assert b"scratch" in lib.gp_last_error()
    assert lib.gp_kmm_noalloc(C.byref(k), 1, None, n, None, 0, fake, n, 16, fake * 2, n, None) == _lib.GP_EINVAL
    assert lib.gp_kmm_noalloc(C.byref(k), 1, fake, n, None, 0, fake, n, 16, fake, n, None) == _lib.GP_EINVAL
    assert lib.gp_kmm_noalloc(C.byref(k), 9, fake, 10, None, 0, fake, 10, 2, fake * 2, 10, None) == _lib.GP_EINVAL
    for n_ok in (1, 333, 2048, 5500):
        assert lib.gp_workspace_bytes(_lib.GP_OP_KMM, n_ok, 0, 48, 16, 0, 1) <= _lib.GP_KMM_NOALLOC_MAX_BYTES
        assert lib.gp_workspace_bytes(_lib.GP_OP_KMM, n_ok, 0, 48, 16, 0, 0) <= _lib.GP_KMM_NOALLOC_MAX_BYTES


def test_workspace_sizes_are_sane(lib):
    from paper_2109_09817_amd import _lib
    small = lib.gp_workspace_bytes(_lib.GP_OP_KMM, 1000, 0, 48, 16, 0, 1)
    big = lib.gp_workspace_bytes(_lib.GP_OP_KMM, 917504, 0, 48, 16, 0, 1)
    assert 0 < small < big < 2 * 1024 ** 3
    # per training point: fragments of both sides + V fragments + FP64 partials, a few hundred bytes
    assert big / 917504 < 1024
    assert lib.gp_workspace_bytes(_lib.GP_OP_KMM, 1000, 0, 500, 16, 0, 1) == 0


def test_altbbmm_entry_points_validate_on_the_host(lib):
    from paper_2109_09817_amd import _lib
    k, keep = _kernel()
    fake = 4096  # never dereferenced: validation fails first
    M = np.array([0, 3, 3], dtype=np.int64)
    Mp = M.ctypes.data_as(C.POINTER(C.c_int64))
    # repeated landmark, r > n, landmark out of range, NULL output
    assert lib.gp_nystrom_precond(C.byref(k), fake, 10, Mp, 3, fake, fake, None, 0, None) == _lib.GP_EINVAL
    assert b"repeated" in lib.gp_last_error()
    M2 = np.array([0, 1, 2], dtype=np.int64)
    M2p = M2.ctypes.data_as(C.POINTER(C.c_int64))
    assert lib.gp_nystrom_precond(C.byref(k), fake, 2, M2p, 3, fake, fake, None, 0, None) == _lib.GP_EINVAL
    M3 = np.array([0, 10], dtype=np.int64)
    assert lib.gp_nystrom_precond(C.byref(k), fake, 10, M3.ctypes.data_as(C.POINTER(C.c_int64)), 2, fake, fake,
                                  None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_nystrom_precond(C.byref(k), fake, 10, M2p, 3, None, fake, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_nystrom_precond(C.byref(k), fake, 10, M2p, 3, fake, fake, None, 0, None) == _lib.GP_EWORKSPACE
    k0, keep0 = _kernel(noise=0.0)
    assert lib.gp_nystrom_precond(C.byref(k0), fake, 10, M2p, 3, fake, fake, None, 0, None) == _lib.GP_EINVAL
    # apply: s outside [1, 64], zero noise
    assert lib.gp_nystrom_apply(fake, fake, 10, 3, 1e-2, fake, 65, fake, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_nystrom_apply(fake, fake, 10, 3, 0.0, fake, 2, fake, None, 0, None) == _lib.GP_EINVAL
    # block CG: s, ld, max_iter, tol, missing preconditioner, workspace
    it = C.c_int32(0)
    rr = np.zeros(64)
    rrp = rr.ctypes.data_as(C.POINTER(C.c_double))
    base = dict(prec=1, n=10, z=None, g=None, r=0, ldb=10, s=2, mi=5, tol=1e-6, ldw=10)

    def call(**kw):
        a = dict(base)
        a.update(kw)
        return lib.gp_bcg(C.byref(k), a["prec"], fake, a["n"], a["z"], a["g"], a["r"], fake, a["ldb"], a["s"],
                          a["mi"], a["tol"], fake, a["ldw"], C.byref(it), rrp, None, 0, None)

    assert call(s=0) == _lib.GP_EINVAL and call(s=65) == _lib.GP_EINVAL
    assert call(ldb=9) == _lib.GP_EINVAL and call(ldw=9) == _lib.GP_EINVAL
    assert call(mi=0) == _lib.GP_EINVAL and call(tol=-1.0) == _lib.GP_EINVAL
    assert call(r=3) == _lib.GP_EINVAL  # r > 0 without Z, g
    assert call(prec=5) == _lib.GP_EINVAL
    assert call() == _lib.GP_EWORKSPACE
    assert lib.gp_workspace_bytes(_lib.GP_OP_BCG, 917504, 0, 48, 50, 512, 1) > 0
    assert lib.gp_workspace_bytes(_lib.GP_OP_BCG, 1000, 0, 48, 65, 0, 1) == 0
    assert lib.gp_workspace_bytes(_lib.GP_OP_NYSTROM, 1000, 0, 48, 0, 1025, 1) == 0


def test_large_rank_altbbmm_entry_points_validate_on_the_host(lib):
    from paper_2109_09817_amd import _lib
    k, keep = _kernel()
    fake = 4096  # never dereferenced: validation fails first
    M = np.array([0, 3, 3], dtype=np.int64)
    Mp = M.ctypes.data_as(C.POINTER(C.c_int64))
    assert lib.gp_nystrom_chol_precond(C.byref(k), fake, 10, Mp, 3, fake, None, 0, None) == _lib.GP_EINVAL
    assert b"repeated" in lib.gp_last_error()
    M2 = np.array([0, 1, 2], dtype=np.int64)
    M2p = M2.ctypes.data_as(C.POINTER(C.c_int64))
    assert lib.gp_nystrom_chol_precond(C.byref(k), fake, 10, M2p, 3, None, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_nystrom_chol_precond(C.byref(k), fake, 10, M2p, 3, fake, None, 0, None) == _lib.GP_EWORKSPACE
    k0, keep0 = _kernel(noise=0.0)
    assert lib.gp_nystrom_chol_precond(C.byref(k0), fake, 10, M2p, 3, fake, None, 0, None) == _lib.GP_EINVAL
    it = C.c_int32(0)
    rr = np.zeros(64)
    rrp = rr.ctypes.data_as(C.POINTER(C.c_double))

    def call(prec=1, E=None, r=0, s=2, ldb=10, mi=5, tol=1e-6):
        return lib.gp_bpcg(C.byref(k), prec, fake, 10, E, r, fake, ldb, s, mi, tol, fake, 10, C.byref(it), rrp,
                           None, 0, None)

    assert call(s=0) == _lib.GP_EINVAL and call(s=65) == _lib.GP_EINVAL
    assert call(ldb=9) == _lib.GP_EINVAL and call(mi=0) == _lib.GP_EINVAL and call(tol=-1.0) == _lib.GP_EINVAL
    assert call(r=3) == _lib.GP_EINVAL  # r > 0 without E
    assert call(prec=5) == _lib.GP_EINVAL
    assert call() == _lib.GP_EWORKSPACE
    assert lib.gp_workspace_bytes(_lib.GP_OP_NYSTROM_CHOL, 131072, 0, 48, 0, 10000, 1) > 131072 * 10000 * 8
    assert lib.gp_workspace_bytes(_lib.GP_OP_NYSTROM_CHOL, 1000, 0, 48, 0, 16385, 1) == 0
    assert lib.gp_workspace_bytes(_lib.GP_OP_BPCG, 131072, 0, 48, 50, 10000, 2) > 0
    assert lib.gp_workspace_bytes(_lib.GP_OP_BPCG, 1000, 0, 48, 65, 0, 1) == 0


def test_fp64_products_are_limited_to_the_solves(lib):
    from paper_2109_09817_amd import _lib
    k, keep = _kernel()
    fake = 4096
    g = np.zeros(6)
    w = np.ones(2)
    rc = lib.gp_kmm_grad(C.byref(k), _lib.GP_PREC_FP64, fake, 10, fake, 10, fake, 10, 2,
                         w.ctypes.data_as(C.POINTER(C.c_double)), g.ctypes.data_as(C.POINTER(C.c_double)),
                         None, 0, None)
    assert rc == _lib.GP_EINVAL and b"FP64" in lib.gp_last_error()
    assert lib.gp_workspace_bytes(_lib.GP_OP_KMM, 1000, 0, 48, 16, 0, _lib.GP_PREC_FP64) > 0
    assert lib.gp_workspace_bytes(_lib.GP_OP_MBCG, 1000, 0, 48, 16, 0, _lib.GP_PREC_FP64) > 0
    assert lib.gp_workspace_bytes(_lib.GP_OP_KMM_GRAD, 1000, 0, 48, 16, 0, _lib.GP_PREC_FP64) == 0
    assert lib.gp_workspace_bytes(_lib.GP_OP_MLL, 1000, 0, 48, 16, 10, _lib.GP_PREC_FP64) == 0
    assert lib.gp_workspace_bytes(_lib.GP_OP_KMM, 1000, 0, 65, 16, 0, _lib.GP_PREC_FP64) == 0  # d <= 64
    assert lib.gp_predict_model_bytes(C.byref(k), _lib.GP_PREC_FP64, 100, 0) == 0


def test_exact_gp_entry_point_validates_on_the_host(lib):
    from paper_2109_09817_amd import _lib
    k, keep = _kernel()
    fake = 4096  # never dereferenced: validation fails first
    mll = C.c_double(0.0)
    g = np.zeros(6)
    gp_ = g.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.gp_exact_mll_and_grad(C.byref(k), None, fake, 10, C.byref(mll), gp_, None, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_exact_mll_and_grad(C.byref(k), fake, fake, 0, C.byref(mll), gp_, None, None, 0, None) == _lib.GP_EINVAL
    assert lib.gp_exact_mll_and_grad(C.byref(k), fake, fake, 65537, C.byref(mll), gp_, None, None, 0,
                                     None) == _lib.GP_EINVAL
    k65, keep65 = _kernel(d=65)
    assert lib.gp_exact_mll_and_grad(C.byref(k65), fake, fake, 10, C.byref(mll), None, None, None, 0,
                                     None) == _lib.GP_EINVAL
    assert lib.gp_exact_mll_and_grad(C.byref(k), fake, fake, 10, C.byref(mll), gp_, None, None, 0,
                                     None) == _lib.GP_EWORKSPACE
    # two n x n FP64 matrices dominate the workspace
    b = lib.gp_workspace_bytes(_lib.GP_OP_EXACT, 8192, 0, 48, 0, 0, _lib.GP_PREC_FP64)
    assert 2 * 8192 * 8192 * 8 <= b < 1.1 * 2 * 8192 * 8192 * 8
    assert lib.gp_workspace_bytes(_lib.GP_OP_EXACT, 65537, 0, 48, 0, 0, 1) == 0
    assert lib.gp_workspace_bytes(_lib.GP_OP_EXACT, 100, 0, 65, 0, 0, 1) == 0


def test_bbmm_and_prediction_entry_points_validate_on_the_host(lib):
    """Every argument error of the BBMM and prediction entry points is reported before any GPU work;
    each call below either fails its argument checks or, with valid arguments, finds no workspace."""
    from paper_2109_09817_amd import _lib
    EINVAL, EWS = _lib.GP_EINVAL, _lib.GP_EWORKSPACE
    k, keep = _kernel()
    k0, keep0 = _kernel(noise=0.0)
    k65, keep65 = _kernel(d=65)
    fake = 4096  # never dereferenced: validation fails first
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731

    # gp_kmm_grad: t in [1, 64], d <= 64, ld = n, finite column weights (read on the host)
    g = np.zeros(6)
    w = np.ones(64)

    def grad(kern=k, prec=1, X=fake, n=10, ldu=10, ldw=10, t=2, colw=w):
        return lib.gp_kmm_grad(C.byref(kern), prec, X, n, fake, ldu, fake, ldw, t, dp(colw), dp(g), None, 0, None)

    assert grad(prec=7) == EINVAL and grad(X=None) == EINVAL and grad(n=0) == EINVAL
    assert grad(t=0) == EINVAL and grad(t=65) == EINVAL and grad(kern=k65) == EINVAL
    assert grad(ldu=9) == EINVAL and grad(ldw=11) == EINVAL
    w_nan = np.ones(2)
    w_nan[1] = np.nan
    assert grad(colw=w_nan) == EINVAL and b"colw" in lib.gp_last_error()
    assert grad() == EWS and grad(t=64) == EWS

    # gp_pivchol_precond: k in [1, min(n, 1024)], noise > 0, outputs present
    rank = C.c_int32(0)
    ldp = C.c_double(0.0)

    def piv(kern=k, n=10, kk=3, L=fake):
        return lib.gp_pivchol_precond(C.byref(kern), fake, n, kk, L, fake, None, C.byref(rank), C.byref(ldp),
                                      None, 0, None)

    assert piv(kk=0) == EINVAL and piv(kk=11) == EINVAL and piv(n=2000, kk=1025) == EINVAL
    assert piv(kern=k0) == EINVAL and piv(L=None) == EINVAL and piv(n=0) == EINVAL
    assert piv() == EWS

    # gp_probe_block has no workspace: only rejected calls are made
    def probes(y=fake, n=10, t=3, L=fake, kk=2, noise=1e-2, B=fake):
        return lib.gp_probe_block(y, n, t, L, kk, noise, 7, B, None)

    assert probes(y=None) == EINVAL and probes(B=None) == EINVAL and probes(n=0) == EINVAL
    assert probes(t=-1) == EINVAL and probes(t=256) == EINVAL
    assert probes(kk=-1) == EINVAL and probes(kk=1025) == EINVAL and probes(L=None) == EINVAL
    assert probes(noise=-1e-3) == EINVAL and probes(noise=float("nan")) == EINVAL

    # gp_mbcg: s in [1, 256], max_iter >= 1, tol finite and >= 0, a consistent preconditioner
    def mbcg(kern=k, prec=1, n=10, pc=None, B=fake, s=2, mi=5, tol=1e-6):
        return lib.gp_mbcg(C.byref(kern), prec, fake, n, C.byref(pc) if pc is not None else None, B, s, mi, tol,
                           fake, None, None, None, 0, None)

    assert mbcg(prec=7) == EINVAL and mbcg(n=0) == EINVAL and mbcg(B=None) == EINVAL
    assert mbcg(s=0) == EINVAL and mbcg(s=257) == EINVAL and mbcg(mi=0) == EINVAL
    assert mbcg(tol=-1.0) == EINVAL and mbcg(tol=float("inf")) == EINVAL
    assert mbcg(pc=_lib.GpPrecond(11, fake, fake)) == EINVAL  # rank > n
    assert mbcg(pc=_lib.GpPrecond(3, None, fake)) == EINVAL
    assert mbcg(kern=k0, pc=_lib.GpPrecond(3, fake, fake)) == EINVAL  # preconditioner without noise
    assert mbcg() == EWS and mbcg(prec=_lib.GP_PREC_FP64) == EWS and mbcg(pc=_lib.GpPrecond(3, fake, fake)) == EWS

    # gp_mll_and_grad: probes in [1, 255], rank in [0, min(n, 1024)], noise > 0
    mll = C.c_double(0.0)

    def mllg(kern=k, probes=4, rank=3, mi=20, prec=1, tol=1e-6, n=10, y=fake, opts=True):
        o = _lib.GpMllOpts(probes, rank, mi, prec, tol, 1)
        return lib.gp_mll_and_grad(C.byref(kern), C.byref(o) if opts else None, fake, y, n, C.byref(mll), dp(g),
                                   None, None, 0, None)

    assert mllg(opts=False) == EINVAL and mllg(prec=_lib.GP_PREC_FP64) == EINVAL
    assert mllg(probes=0) == EINVAL and mllg(probes=256) == EINVAL
    assert mllg(rank=-1) == EINVAL and mllg(rank=11) == EINVAL and mllg(mi=0) == EINVAL
    assert mllg(tol=float("nan")) == EINVAL and mllg(kern=k0) == EINVAL and mllg(y=None) == EINVAL
    assert mllg() == EWS and mllg(rank=0) == EWS

    # gp_lanczos_cache: kc in [1, min(n, 4095)]
    kco = C.c_int32(0)

    def lanczos(n=10, kc=4, R=fake, prec=1):
        return lib.gp_lanczos_cache(C.byref(k), prec, fake, fake, n, kc, R, C.byref(kco), None, 0, None)

    assert lanczos(kc=0) == EINVAL and lanczos(kc=11) == EINVAL and lanczos(n=5000, kc=4096) == EINVAL
    assert lanczos(R=None) == EINVAL and lanczos(prec=_lib.GP_PREC_FP64) == EINVAL
    assert lanczos() == EWS

    # prediction: model size, prepare, run and the one-call form
    assert lib.gp_predict_model_bytes(C.byref(k), 1, 100, 16) > 0
    assert lib.gp_predict_model_bytes(C.byref(k), 1, 100, -1) == 0
    assert lib.gp_predict_model_bytes(C.byref(k), 1, 100, 4096) == 0
    assert lib.gp_predict_model_bytes(C.byref(k65), 7, 100, 0) == 0
    assert lib.gp_predict_prepare(C.byref(k), 1, fake, 10, fake, None, 4, fake, 1 << 30, None) == EINVAL  # kc, no R
    assert lib.gp_predict_prepare(C.byref(k), 1, fake, 10, None, fake, 4, fake, 1 << 30, None) == EINVAL
    assert lib.gp_predict_prepare(C.byref(k), 1, fake, 10, fake, fake, 4096, fake, 1 << 30, None) == EINVAL
    assert lib.gp_predict_prepare(C.byref(k), 1, fake, 10, fake, fake, 4, None, 0, None) == EWS

    def run(model=fake, kc=4, Z=fake, m=3, mean=fake, var=fake):
        return lib.gp_predict_run(C.byref(k), 1, model, 10, kc, Z, m, mean, var, None, 0, None)

    assert run(model=None) == EINVAL and run(Z=None) == EINVAL and run(mean=None) == EINVAL
    assert run(m=0) == EINVAL and run(kc=0) == EINVAL  # a variance needs a cache
    assert run() == EWS and run(kc=0, var=None) == EWS

    def predict(R=fake, kc=4, Z=fake, m=3, mean=fake, var=fake):
        return lib.gp_predict(C.byref(k), 1, fake, 10, fake, R, kc, Z, m, mean, var, None, 0, None)

    assert predict(m=0) == EINVAL and predict(Z=None) == EINVAL and predict(mean=None) == EINVAL
    assert predict(R=None) == EINVAL and b"variance" in lib.gp_last_error()  # var without a cache
    assert predict() == EWS and predict(R=None, var=None) == EWS
