"""Error metric for comparing an FP32 transform with the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per transform b: ``rel_l2(b) = ||Y_b - X_b||_2 / ||X_b||_2`` in FP64 with the
FP32 result promoted.  The gate is ``max_b rel_l2(b) <= 1e-6 * log2(N)``
(the accuracy bound the build is held to; the paper itself states none).  When
``||X_b|| == 0`` the absolute error must be 0 and the reported value is the
absolute error.
"""
from __future__ import annotations

import math

import numpy as np


def rel_l2_per_transform(y, x, n_axes: int = 1) -> np.ndarray:
    """Relative L2 error of each transform; the last ``n_axes`` axes form one transform."""
    y = np.asarray(y).astype(np.complex128)
    x = np.asarray(x).astype(np.complex128)
    if y.shape != x.shape:
        raise ValueError(f"shape mismatch {y.shape} vs {x.shape}")
    axes = tuple(range(-n_axes, 0))
    num = np.sqrt(np.sum(np.abs(y - x) ** 2, axis=axes))
    den = np.sqrt(np.sum(np.abs(x) ** 2, axis=axes))
    out = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
    return np.atleast_1d(out)


def tolerance(n_points: int) -> float:
    """``1e-6 * log2(N)`` with N the number of points of one transform (real-valued log)."""
    return 1e-6 * max(math.log2(n_points), 1.0)


def check(y, x, n_points: int, n_axes: int = 1, factor: float = 1.0):
    """Return (max, median, tol) and raise AssertionError when max exceeds tol."""
    e = rel_l2_per_transform(y, x, n_axes)
    tol = factor * tolerance(n_points)
    mx, md = float(np.max(e)), float(np.median(e))
    if not (mx <= tol):
        raise AssertionError(f"max rel L2 {mx:.3e} > tol {tol:.3e} (median {md:.3e})")
    return mx, md, tol
