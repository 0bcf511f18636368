"""Python entry points over the C ABI (include/gpkmm.h).

Argument marshalling only: every step of the computation runs in libgpkmm's
HIP kernels.  PyTorch supplies device memory and the current HIP stream.

Layouts (as in the C ABI):
* X (n, d) and query rows Z (m, d): float64, row-major, on the GPU.
* A block of t vectors of length n is a (t, n) float64 tensor: row c of the
  tensor is vector c (the ABI's column-major n x t block with ld = n).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib

PRECISION = {"fp32": _lib.GP_PREC_FP32, "bf16x3": _lib.GP_PREC_BF16X3}
KINDS = {"matern52": _lib.GP_MATERN52, "rbf": _lib.GP_RBF}


@dataclasses.dataclass
class Kernel:
    """ARD stationary kernel: s_f m(r) with r^2 = sum ((x - z)/l)^2, plus noise sigma^2 on K_hat."""

    lengthscale: Sequence[float]
    outputscale: float = 1.0
    noise: float = 0.0
    kind: str = "matern52"

    def struct(self):
        return _lib.kernel_struct(KINDS[self.kind], self.lengthscale, self.outputscale, self.noise)

    @property
    def d(self) -> int:
        return int(np.asarray(self.lengthscale).shape[0])


def _prec(p) -> int:
    return PRECISION[p] if isinstance(p, str) else int(p)


def _stream(dev: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _need(t: torch.Tensor, name: str, shape=None, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def kmm(kern: Kernel, X: torch.Tensor, V: torch.Tensor, Z: Optional[torch.Tensor] = None,
        precision="bf16x3", out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """K_hat V (Z is None) or K(Z, X) V.  X (n, d); V (t, n); returns (t, rows)."""
    lib = _lib.load()
    n, d = X.shape
    _need(X, "X", (n, kern.d))
    t = V.shape[0]
    _need(V, "V", (t, n))
    rows = n if Z is None else Z.shape[0]
    if Z is not None:
        _need(Z, "Z", (rows, kern.d))
    if out is None:
        out = torch.empty((t, rows), dtype=torch.float64, device=X.device)
    _need(out, "out", (t, rows))
    p = _prec(precision)
    ws_bytes = lib.gp_workspace_bytes(_lib.GP_OP_KMM, n, 0 if Z is None else rows, kern.d, t, 0, p)
    ws = workspace(ws_bytes, X.device)
    ks, _keep = kern.struct()
    _lib.check(lib.gp_kmm(C.byref(ks), p, X.data_ptr(), n, _ptr(Z), rows if Z is not None else 0,
                          V.data_ptr(), n, t, out.data_ptr(), rows, ws.data_ptr(), ws.numel(),
                          _stream(X.device)))
    return out
