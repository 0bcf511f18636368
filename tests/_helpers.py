"""Shared helpers of the test-suite (tolerances, device transfer, building the library)."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def ensure_built() -> str:
    """Path of libgpkmm.so, building it only when nothing is built yet."""
    from paper_2109_09817_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2109_09817_amd import build
        build.build()
    return _lib.LIB_PATH


def col_rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max over vectors (rows of a (t, n) block) of ||got - ref||_2 / ||ref||_2."""
    got = np.atleast_2d(got)
    ref = np.atleast_2d(ref)
    num = np.linalg.norm(got - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(num / den))


def dev(a, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()
