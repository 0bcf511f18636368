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

PRECISION = {"fp32": _lib.GP_PREC_FP32, "bf16x3": _lib.GP_PREC_BF16X3, "fp64": _lib.GP_PREC_FP64}
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


def kmm_noalloc(kern: Kernel, X: torch.Tensor, V: torch.Tensor, out: torch.Tensor, Z: Optional[torch.Tensor] = None,
                precision="bf16x3") -> torch.Tensor:
    """gp_kmm_noalloc: K_hat V or K(Z, X) V into the caller's ``out`` (t, rows), with the library's
    fixed device scratch instead of a workspace (no allocation in the call)."""
    lib = _lib.load()
    n, d = X.shape
    _need(X, "X", (n, kern.d))
    t = V.shape[0]
    _need(V, "V", (t, n))
    rows = n if Z is None else Z.shape[0]
    if Z is not None:
        _need(Z, "Z", (rows, kern.d))
    _need(out, "out", (t, rows))
    ks, _keep = kern.struct()
    _lib.check(lib.gp_kmm_noalloc(C.byref(ks), _prec(precision), X.data_ptr(), n, _ptr(Z),
                                  rows if Z is not None else 0, V.data_ptr(), n, t, out.data_ptr(), rows,
                                  _stream(X.device)))
    return out


def kmm_grad(kern: Kernel, X: torch.Tensor, U: torch.Tensor, W: torch.Tensor, colw, precision="fp32") -> np.ndarray:
    """sum_c colw[c] U_c^T (dK_hat/dlog theta) W_c for theta = (l_1..l_d, s_f, sigma^2); U, W (t, n)."""
    lib = _lib.load()
    n = X.shape[0]
    t = U.shape[0]
    _need(X, "X", (n, kern.d))
    _need(U, "U", (t, n))
    _need(W, "W", (t, n))
    w = np.ascontiguousarray(np.asarray(colw, dtype=np.float64))
    if w.shape != (t,):
        raise ValueError("colw must have t entries")
    g = np.zeros(kern.d + 2)
    p = _prec(precision)
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_KMM_GRAD, n, 0, kern.d, t, 0, p), X.device)
    ks, _keep = kern.struct()
    _lib.check(lib.gp_kmm_grad(C.byref(ks), p, X.data_ptr(), n, U.data_ptr(), n, W.data_ptr(), n, t,
                               w.ctypes.data_as(C.POINTER(C.c_double)), g.ctypes.data_as(C.POINTER(C.c_double)),
                               ws.data_ptr(), ws.numel(), _stream(X.device)))
    return g


@dataclasses.dataclass
class Precond:
    """Pivoted-Cholesky preconditioner P = L L^T + sigma^2 I (L: (k, n) = n x k column-major)."""

    L: torch.Tensor
    Cchol: torch.Tensor  # (k, k): row j of the tensor is column j of the lower factor
    pivots: np.ndarray
    rank: int
    logdet: float

    def struct(self):
        return _lib.GpPrecond(self.L.shape[0], self.L.data_ptr(), self.Cchol.data_ptr())


def pivchol(kern: Kernel, X: torch.Tensor, k: int) -> Precond:
    lib = _lib.load()
    n = X.shape[0]
    _need(X, "X", (n, kern.d))
    L = torch.empty((k, n), dtype=torch.float64, device=X.device)
    Cc = torch.empty((k, k), dtype=torch.float64, device=X.device)
    piv = np.zeros(k, dtype=np.int64)
    rank = C.c_int32(0)
    ld = C.c_double(0.0)
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_PIVCHOL, n, 0, kern.d, 1, k, 0), X.device)
    ks, _keep = kern.struct()
    _lib.check(lib.gp_pivchol_precond(C.byref(ks), X.data_ptr(), n, k, L.data_ptr(), Cc.data_ptr(),
                                      piv.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(rank), C.byref(ld),
                                      ws.data_ptr(), ws.numel(), _stream(X.device)))
    return Precond(L, Cc, piv, int(rank.value), float(ld.value))


def probe_block(y: torch.Tensor, t: int, seed: int, noise: float, pc: Optional[Precond] = None) -> torch.Tensor:
    """[y | b_1..b_t] as a (t+1, n) tensor."""
    lib = _lib.load()
    n = y.shape[0]
    _need(y, "y", (n,))
    B = torch.empty((t + 1, n), dtype=torch.float64, device=y.device)
    k = 0 if pc is None else pc.L.shape[0]
    _lib.check(lib.gp_probe_block(y.data_ptr(), n, t, None if pc is None else pc.L.data_ptr(), k, noise,
                                  C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), B.data_ptr(), _stream(y.device)))
    return B


@dataclasses.dataclass
class MbcgResult:
    U: torch.Tensor
    Z0: Optional[torch.Tensor]
    alpha: np.ndarray  # (iters, s)
    beta: np.ndarray
    iters: np.ndarray
    relres: np.ndarray
    gamma0: np.ndarray
    status: int


def mbcg(kern: Kernel, X: torch.Tensor, B: torch.Tensor, max_iter: int, tol: float,
         pc: Optional[Precond] = None, precision="bf16x3", want_z0: bool = True) -> MbcgResult:
    lib = _lib.load()
    n = X.shape[0]
    s = B.shape[0]
    _need(X, "X", (n, kern.d))
    _need(B, "B", (s, n))
    U = torch.empty_like(B)
    Z0 = torch.empty_like(B) if want_z0 else None
    al = np.zeros((max_iter, s))
    be = np.zeros((max_iter, s))
    it = np.zeros(s, dtype=np.int32)
    rr = np.zeros(s)
    g0 = np.zeros(s)
    dp = C.POINTER(C.c_double)
    out = _lib.GpMbcgOut(al.ctypes.data_as(dp), be.ctypes.data_as(dp), it.ctypes.data_as(C.POINTER(C.c_int32)),
                         rr.ctypes.data_as(dp), g0.ctypes.data_as(dp), 0)
    p = _prec(precision)
    k = 0 if pc is None else pc.L.shape[0]
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_MBCG, n, 0, kern.d, s, k, p), X.device)
    ks, _keep = kern.struct()
    pcs = pc.struct() if pc is not None else None
    rc = _lib.check(lib.gp_mbcg(C.byref(ks), p, X.data_ptr(), n, None if pcs is None else C.byref(pcs),
                                B.data_ptr(), s, max_iter, tol, U.data_ptr(), _ptr(Z0), C.byref(out),
                                ws.data_ptr(), ws.numel(), _stream(X.device)))
    J = out.total_iters
    return MbcgResult(U, Z0, al[:J].copy(), be[:J].copy(), it, rr, g0, rc)


@dataclasses.dataclass
class MllResult:
    mll: float
    grad: Optional[np.ndarray]
    info: dict
    status: int


def mll_and_grad(kern: Kernel, X: torch.Tensor, y: torch.Tensor, probes: int, rank: int, max_iter: int,
                 tol: float, seed: int, precision="bf16x3", with_grad: bool = True) -> MllResult:
    lib = _lib.load()
    n = X.shape[0]
    _need(X, "X", (n, kern.d))
    _need(y, "y", (n,))
    p = _prec(precision)
    opts = _lib.GpMllOpts(probes, rank, max_iter, p, tol, C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF))
    info = _lib.GpMllInfo()
    mll = C.c_double(0.0)
    g = np.zeros(kern.d + 2)
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_MLL, n, 0, kern.d, probes, rank, p), X.device)
    ks, _keep = kern.struct()
    rc = _lib.check(lib.gp_mll_and_grad(C.byref(ks), C.byref(opts), X.data_ptr(), y.data_ptr(), n, C.byref(mll),
                                        g.ctypes.data_as(C.POINTER(C.c_double)) if with_grad else None,
                                        C.byref(info), ws.data_ptr(), ws.numel(), _stream(X.device)))
    inf = {f: getattr(info, f) for f, _ in _lib.GpMllInfo._fields_}
    return MllResult(float(mll.value), g if with_grad else None, inf, rc)


@dataclasses.dataclass
class Nystrom:
    """AltBBMM preconditioner over r landmark rows: P^{-1/2} = sigma^{-1} I + Z^T diag(g) Z."""

    Z: torch.Tensor         # (r, n): rows beyond the kept rank are zero; sum_m Z_m Z_m^T = K_XM K_MM^+ K_MX
    g: torch.Tensor         # (r,): zero beyond the kept rank
    landmarks: np.ndarray
    noise: float

    @property
    def rank(self) -> int:
        """Landmarks r (the size of Z and g)."""
        return self.Z.shape[0]

    @property
    def kept(self) -> int:
        """Directions of K_MM kept by its eigenvalue cut."""
        return int(torch.count_nonzero(self.g).item())


def nystrom_precond(kern: Kernel, X: torch.Tensor, landmarks) -> Nystrom:
    lib = _lib.load()
    n = X.shape[0]
    _need(X, "X", (n, kern.d))
    M = np.ascontiguousarray(np.asarray(landmarks, dtype=np.int64))
    r = M.shape[0]
    Z = torch.empty((r, n), dtype=torch.float64, device=X.device)
    g = torch.empty((r,), dtype=torch.float64, device=X.device)
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_NYSTROM, n, 0, kern.d, 0, r, _lib.GP_PREC_FP32), X.device)
    ks, _keep = kern.struct()
    _lib.check(lib.gp_nystrom_precond(C.byref(ks), X.data_ptr(), n, M.ctypes.data_as(C.POINTER(C.c_int64)), r,
                                      Z.data_ptr(), g.data_ptr(), ws.data_ptr(), ws.numel(), _stream(X.device)))
    return Nystrom(Z, g, M, kern.noise)


def nystrom_apply(pc: Nystrom, V: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """P^{-1/2} V for a (s, n) block."""
    lib = _lib.load()
    r, n = pc.Z.shape
    s = V.shape[0]
    _need(V, "V", (s, n))
    if out is None:
        out = torch.empty_like(V)
    _need(out, "out", (s, n))
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_NYSTROM_APPLY, n, 0, 1, s, r, _lib.GP_PREC_FP32), V.device)
    _lib.check(lib.gp_nystrom_apply(pc.Z.data_ptr(), pc.g.data_ptr(), n, r, pc.noise, V.data_ptr(), s,
                                    out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(V.device)))
    return out


@dataclasses.dataclass
class ExactResult:
    mll: float
    grad: Optional[np.ndarray]     # (d + 2,): log l_1..log l_d, log s_f, log sigma^2
    omega: Optional[torch.Tensor]  # (n,): K_hat^{-1} y


def exact_mll_and_grad(kern: Kernel, X: torch.Tensor, y: torch.Tensor, with_grad: bool = True,
                       with_omega: bool = False, ws: Optional[torch.Tensor] = None) -> ExactResult:
    """Exact (dense Cholesky) GP: the log marginal likelihood, its gradient and K_hat^{-1} y."""
    lib = _lib.load()
    n = X.shape[0]
    _need(X, "X", (n, kern.d))
    _need(y, "y", (n,))
    need = lib.gp_workspace_bytes(_lib.GP_OP_EXACT, n, 0, kern.d, 0, 0, _lib.GP_PREC_FP64)
    if ws is None or ws.numel() < need:
        ws = workspace(need, X.device)
    mll = C.c_double(0.0)
    g = np.zeros(kern.d + 2) if with_grad else None
    om = torch.empty((n,), dtype=torch.float64, device=X.device) if with_omega else None
    ks, _keep = kern.struct()
    _lib.check(lib.gp_exact_mll_and_grad(C.byref(ks), X.data_ptr(), y.data_ptr(), n, C.byref(mll),
                                         None if g is None else g.ctypes.data_as(C.POINTER(C.c_double)), _ptr(om),
                                         ws.data_ptr(), ws.numel(), _stream(X.device)))
    return ExactResult(float(mll.value), g, om)


@dataclasses.dataclass
class BcgResult:
    W: torch.Tensor          # (s, n): K_hat^{-1} B
    iters: int
    relres: np.ndarray       # (s,)
    status: int              # GP_OK or GP_WNOCONV


def bcg(kern: Kernel, X: torch.Tensor, B: torch.Tensor, max_iter: int, tol: float,
        pc: Optional[Nystrom] = None, precision="bf16x3") -> BcgResult:
    """AltBBMM: block CG on P^{-1/2} K_hat P^{-1/2} (P Nystrom, or the identity when pc is None)."""
    lib = _lib.load()
    n = X.shape[0]
    _need(X, "X", (n, kern.d))
    s = B.shape[0]
    _need(B, "B", (s, n))
    r = 0 if pc is None else pc.rank
    W = torch.empty_like(B)
    p = _prec(precision)
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_BCG, n, 0, kern.d, s, r, p), X.device)
    it = C.c_int32(0)
    rr = np.zeros(s)
    ks, _keep = kern.struct()
    rc = _lib.check(lib.gp_bcg(C.byref(ks), p, X.data_ptr(), n, _ptr(None if pc is None else pc.Z),
                               _ptr(None if pc is None else pc.g), r, B.data_ptr(), n, s, max_iter, tol,
                               W.data_ptr(), n, C.byref(it), rr.ctypes.data_as(C.POINTER(C.c_double)),
                               ws.data_ptr(), ws.numel(), _stream(X.device)))
    return BcgResult(W, int(it.value), rr, rc)


@dataclasses.dataclass
class NystromChol:
    """AltBBMM preconditioner at large rank: P^{-1} = sigma^{-2} (I - E E^T), E (r, n) = n x r column-major."""

    E: torch.Tensor
    landmarks: np.ndarray
    noise: float

    @property
    def rank(self) -> int:
        return self.E.shape[0]


def nystrom_chol_precond(kern: Kernel, X: torch.Tensor, landmarks) -> NystromChol:
    lib = _lib.load()
    n = X.shape[0]
    _need(X, "X", (n, kern.d))
    M = np.ascontiguousarray(np.asarray(landmarks, dtype=np.int64))
    r = M.shape[0]
    E = torch.empty((r, n), dtype=torch.float64, device=X.device)
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_NYSTROM_CHOL, n, 0, kern.d, 0, r, _lib.GP_PREC_FP64), X.device)
    ks, _keep = kern.struct()
    _lib.check(lib.gp_nystrom_chol_precond(C.byref(ks), X.data_ptr(), n, M.ctypes.data_as(C.POINTER(C.c_int64)), r,
                                           E.data_ptr(), ws.data_ptr(), ws.numel(), _stream(X.device)))
    return NystromChol(E, M, kern.noise)


def bpcg(kern: Kernel, X: torch.Tensor, B: torch.Tensor, max_iter: int, tol: float,
         pc: Optional[NystromChol] = None, precision="bf16x3") -> BcgResult:
    """AltBBMM: block preconditioned CG on K_hat W = B with P^{-1} = sigma^{-2} (I - E E^T) (or P = I)."""
    lib = _lib.load()
    n = X.shape[0]
    _need(X, "X", (n, kern.d))
    s = B.shape[0]
    _need(B, "B", (s, n))
    r = 0 if pc is None else pc.rank
    W = torch.empty_like(B)
    p = _prec(precision)
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_BPCG, n, 0, kern.d, s, r, p), X.device)
    it = C.c_int32(0)
    rr = np.zeros(s)
    ks, _keep = kern.struct()
    rc = _lib.check(lib.gp_bpcg(C.byref(ks), p, X.data_ptr(), n, _ptr(None if pc is None else pc.E), r, B.data_ptr(),
                                n, s, max_iter, tol, W.data_ptr(), n, C.byref(it),
                                rr.ctypes.data_as(C.POINTER(C.c_double)), ws.data_ptr(), ws.numel(),
                                _stream(X.device)))
    return BcgResult(W, int(it.value), rr, rc)


def lanczos_cache(kern: Kernel, X: torch.Tensor, y: torch.Tensor, kc: int, precision="bf16x3"):
    """Variance cache R (kc, n) with R R^T ~ K_hat^{-1} on the Krylov space of y; returns (R, rank)."""
    lib = _lib.load()
    n = X.shape[0]
    _need(X, "X", (n, kern.d))
    _need(y, "y", (n,))
    R = torch.empty((kc, n), dtype=torch.float64, device=X.device)
    p = _prec(precision)
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_LANCZOS, n, 0, kern.d, 1, kc, p), X.device)
    kout = C.c_int32(0)
    ks, _keep = kern.struct()
    _lib.check(lib.gp_lanczos_cache(C.byref(ks), p, X.data_ptr(), y.data_ptr(), n, kc, R.data_ptr(),
                                    C.byref(kout), ws.data_ptr(), ws.numel(), _stream(X.device)))
    return R, int(kout.value)


class PredictModel:
    """A trained model kept resident on the GPU: prepared operands of K(., X) [alpha | R]."""

    def __init__(self, kern: Kernel, X: torch.Tensor, alpha: torch.Tensor, R: Optional[torch.Tensor] = None,
                 precision="bf16x3"):
        lib = _lib.load()
        self.kern = kern
        self.n = X.shape[0]
        _need(X, "X", (self.n, kern.d))
        _need(alpha, "alpha", (self.n,))
        self.kc = 0 if R is None else R.shape[0]
        if R is not None:
            _need(R, "R", (self.kc, self.n))
        self.precision = _prec(precision)
        self.device = X.device
        ks, self._ell = kern.struct()
        self._ks = ks
        nb = lib.gp_predict_model_bytes(C.byref(ks), self.precision, self.n, self.kc)
        if nb == 0:
            raise ValueError("invalid prediction model arguments")
        self.model = workspace(nb, X.device)
        _lib.check(lib.gp_predict_prepare(C.byref(ks), self.precision, X.data_ptr(), self.n, alpha.data_ptr(),
                                          _ptr(R), self.kc, self.model.data_ptr(), self.model.numel(),
                                          _stream(X.device)))

    def workspace_bytes(self, m: int) -> int:
        return _lib.load().gp_workspace_bytes(_lib.GP_OP_PREDICT_RUN, self.n, m, self.kern.d, 0, self.kc,
                                              self.precision)

    def __call__(self, Z: torch.Tensor, with_var: bool = True, ws: Optional[torch.Tensor] = None,
                 mean: Optional[torch.Tensor] = None, var: Optional[torch.Tensor] = None, stream=None):
        lib = _lib.load()
        m = Z.shape[0]
        _need(Z, "Z", (m, self.kern.d))
        if mean is None:
            mean = torch.empty(m, dtype=torch.float64, device=self.device)
        if with_var and self.kc > 0 and var is None:
            var = torch.empty(m, dtype=torch.float64, device=self.device)
        if not with_var or self.kc == 0:
            var = None
        need = self.workspace_bytes(m)
        if ws is None or ws.numel() < need:
            ws = workspace(need, self.device)
        st = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(self.device)
        _lib.check(lib.gp_predict_run(C.byref(self._ks), self.precision, self.model.data_ptr(), self.n, self.kc,
                                      Z.data_ptr(), m, mean.data_ptr(), _ptr(var), ws.data_ptr(), ws.numel(), st))
        return mean, var


def predict(kern: Kernel, X: torch.Tensor, alpha: torch.Tensor, Z: torch.Tensor, R: Optional[torch.Tensor] = None,
            precision="bf16x3"):
    """One-shot predictive mean (and variance when a cache R is given) at query rows Z."""
    lib = _lib.load()
    n = X.shape[0]
    m = Z.shape[0]
    _need(X, "X", (n, kern.d))
    _need(alpha, "alpha", (n,))
    _need(Z, "Z", (m, kern.d))
    kc = 0 if R is None else R.shape[0]
    if R is not None:
        _need(R, "R", (kc, n))
    p = _prec(precision)
    mean = torch.empty(m, dtype=torch.float64, device=X.device)
    var = torch.empty(m, dtype=torch.float64, device=X.device) if kc > 0 else None
    ws = workspace(lib.gp_workspace_bytes(_lib.GP_OP_PREDICT, n, m, kern.d, 0, kc, p), X.device)
    ks, _keep = kern.struct()
    _lib.check(lib.gp_predict(C.byref(ks), p, X.data_ptr(), n, alpha.data_ptr(), _ptr(R), kc, Z.data_ptr(), m,
                              mean.data_ptr(), _ptr(var), ws.data_ptr(), ws.numel(), _stream(X.device)))
    return mean, var


def profile_enable(on: bool = True) -> None:
    _lib.check(_lib.load().gp_profile_enable(1 if on else 0))


def profile_read(reset: bool = True):
    """(launches, total_ms, nominal_flops) of the timed tile sweeps since the last reset."""
    n = C.c_int64(0)
    ms = C.c_double(0.0)
    fl = C.c_double(0.0)
    _lib.check(_lib.load().gp_profile_read(C.byref(n), C.byref(ms), C.byref(fl), 1 if reset else 0))
    return int(n.value), float(ms.value), float(fl.value)


def profile_records(cap: int = 4096):
    """Per-launch (n, m, t, ms) records of the timed tile sweeps (oldest first)."""
    n = np.zeros(cap, dtype=np.int64)
    m = np.zeros(cap, dtype=np.int64)
    t = np.zeros(cap, dtype=np.int32)
    ms = np.zeros(cap)
    cnt = C.c_int64(0)
    _lib.check(_lib.load().gp_profile_records(cap, n.ctypes.data_as(C.POINTER(C.c_int64)),
                                              m.ctypes.data_as(C.POINTER(C.c_int64)),
                                              t.ctypes.data_as(C.POINTER(C.c_int32)),
                                              ms.ctypes.data_as(C.POINTER(C.c_double)), C.byref(cnt)))
    k = int(cnt.value)
    return [(int(n[i]), int(m[i]), int(t[i]), float(ms[i])) for i in range(k)]
