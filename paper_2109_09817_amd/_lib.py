"""ctypes binding of libgpkmm.so (include/gpkmm.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgpkmm.so")

GP_OK = 0
GP_WNOCONV = 1
GP_EINVAL = -1
GP_EWORKSPACE = -2
GP_EHIP = -3
GP_ENOTPD = -4
GP_ENONFINITE = -5

GP_MATERN52 = 0
GP_RBF = 1
GP_PREC_FP32 = 0
GP_PREC_BF16X3 = 1
GP_PREC_FP64 = 2
GP_MAX_D = 128
GP_KMM_NOALLOC_MAX_BYTES = 64 << 20

GP_OP_KMM = 1
GP_OP_KMM_GRAD = 2
GP_OP_PIVCHOL = 3
GP_OP_MBCG = 4
GP_OP_MLL = 5
GP_OP_PREDICT = 6
GP_OP_LANCZOS = 7
GP_OP_PREDICT_RUN = 8
GP_OP_NYSTROM = 9
GP_OP_NYSTROM_APPLY = 10
GP_OP_BCG = 11
GP_OP_EXACT = 12
GP_OP_NYSTROM_CHOL = 13
GP_OP_BPCG = 14


class GpKernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("d", C.c_int32), ("lengthscale", C.POINTER(C.c_double)),
                ("outputscale", C.c_double), ("noise", C.c_double)]


class GpPrecond(C.Structure):
    _fields_ = [("rank", C.c_int32), ("L", C.c_void_p), ("Cchol", C.c_void_p)]


class GpMbcgOut(C.Structure):
    _fields_ = [("alpha", C.POINTER(C.c_double)), ("beta", C.POINTER(C.c_double)),
                ("iters", C.POINTER(C.c_int32)), ("relres", C.POINTER(C.c_double)),
                ("gamma0", C.POINTER(C.c_double)), ("total_iters", C.c_int32)]


class GpMllOpts(C.Structure):
    _fields_ = [("probes", C.c_int32), ("rank", C.c_int32), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("tol", C.c_double), ("seed", C.c_uint64)]


class GpMllInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rank", C.c_int32), ("logdet", C.c_double),
                ("logdet_p", C.c_double), ("quad", C.c_double), ("max_relres", C.c_double),
                ("ms_precond", C.c_double), ("ms_mbcg", C.c_double), ("ms_grad", C.c_double)]


_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_D = C.c_double
_SZ = C.c_size_t

PROTOTYPES = {
    "gp_kmm": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _I64, _P, _I64, _P, _I64, _I32, _P, _I64, _P, _SZ, _P]),
    "gp_kmm_noalloc": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _I64, _P, _I64, _P, _I64, _I32, _P, _I64, _P]),
    "gp_kmm_grad": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _I64, _P, _I64, _P, _I64, _I32,
                              C.POINTER(_D), C.POINTER(_D), _P, _SZ, _P]),
    "gp_pivchol_precond": (C.c_int, [C.POINTER(GpKernel), _P, _I64, _I32, _P, _P, C.POINTER(C.c_int64),
                                     C.POINTER(_I32), C.POINTER(_D), _P, _SZ, _P]),
    "gp_mbcg": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _I64, C.POINTER(GpPrecond), _P, _I32, _I32, _D,
                          _P, _P, C.POINTER(GpMbcgOut), _P, _SZ, _P]),
    "gp_probe_block": (C.c_int, [_P, _I64, _I32, _P, _I32, _D, C.c_uint64, _P, _P]),
    "gp_mll_and_grad": (C.c_int, [C.POINTER(GpKernel), C.POINTER(GpMllOpts), _P, _P, _I64,
                                  C.POINTER(_D), C.POINTER(_D), C.POINTER(GpMllInfo), _P, _SZ, _P]),
    "gp_lanczos_cache": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _P, _I64, _I32, _P, C.POINTER(_I32),
                                   _P, _SZ, _P]),
    "gp_predict": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _I64, _P, _P, _I32, _P, _I64, _P, _P,
                             _P, _SZ, _P]),
    "gp_predict_model_bytes": (C.c_size_t, [C.POINTER(GpKernel), _I32, _I64, _I32]),
    "gp_predict_prepare": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _I64, _P, _P, _I32, _P, _SZ, _P]),
    "gp_predict_run": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _I64, _I32, _P, _I64, _P, _P, _P, _SZ, _P]),
    "gp_lanczos_quadrature": (C.c_int, [C.POINTER(_D), C.POINTER(_D), _I32, _I32, C.POINTER(_D)]),
    "gp_nystrom_precond": (C.c_int, [C.POINTER(GpKernel), _P, _I64, C.POINTER(C.c_int64), _I32, _P, _P,
                                     _P, _SZ, _P]),
    "gp_nystrom_apply": (C.c_int, [_P, _P, _I64, _I32, _D, _P, _I32, _P, _P, _SZ, _P]),
    "gp_exact_mll_and_grad": (C.c_int, [C.POINTER(GpKernel), _P, _P, _I64, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double), _P, _P, _SZ, _P]),
    "gp_bcg": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _I64, _P, _P, _I32, _P, _I64, _I32, _I32, _D, _P, _I64,
                         C.POINTER(_I32), C.POINTER(_D), _P, _SZ, _P]),
    "gp_nystrom_chol_precond": (C.c_int, [C.POINTER(GpKernel), _P, _I64, C.POINTER(C.c_int64), _I32, _P, _P, _SZ,
                                          _P]),
    "gp_bpcg": (C.c_int, [C.POINTER(GpKernel), _I32, _P, _I64, _P, _I32, _P, _I64, _I32, _I32, _D, _P, _I64,
                          C.POINTER(_I32), C.POINTER(_D), _P, _SZ, _P]),
    "gp_workspace_bytes": (C.c_size_t, [_I32, _I64, _I64, _I32, _I32, _I32, _I32]),
    "gp_profile_enable": (C.c_int, [_I32]),
    "gp_profile_read": (C.c_int, [C.POINTER(_I64), C.POINTER(_D), C.POINTER(_D), _I32]),
    "gp_profile_records": (C.c_int, [_I64, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I32), C.POINTER(_D),
                                     C.POINTER(_I64)]),
    "gp_last_error": (C.c_char_p, []),
    "gp_version": (C.c_char_p, []),
}

_LIB = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the built library; raises if it has not been built (no fallback exists)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"libgpkmm.so is not built ({path}); run paper_2109_09817_amd/build.py")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class GpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(code: int) -> int:
    if code < 0:
        raise GpError(code, load().gp_last_error().decode())
    return code


def kernel_struct(kind: int, lengthscale, outputscale: float, noise: float):
    """A gp_kernel plus the host array it points to (keep both alive during the call)."""
    import numpy as np
    ell = np.ascontiguousarray(np.asarray(lengthscale, dtype=np.float64))
    k = GpKernel(int(kind), int(ell.shape[0]), ell.ctypes.data_as(C.POINTER(C.c_double)),
                 float(outputscale), float(noise))
    return k, ell
