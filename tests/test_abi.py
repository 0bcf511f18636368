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


def test_workspace_sizes_are_sane(lib):
    from paper_2109_09817_amd import _lib
    small = lib.gp_workspace_bytes(_lib.GP_OP_KMM, 1000, 0, 48, 16, 0, 1)
    big = lib.gp_workspace_bytes(_lib.GP_OP_KMM, 917504, 0, 48, 16, 0, 1)
    assert 0 < small < big < 2 * 1024 ** 3
    # per training point: fragments of both sides + V fragments + FP64 partials, a few hundred bytes
    assert big / 917504 < 1024
    assert lib.gp_workspace_bytes(_lib.GP_OP_KMM, 1000, 0, 500, 16, 0, 1) == 0
