"""FP64 CPU oracle for batched complex FFTs -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never imports it and shares no code with it.

What it computes (paper, Background, "FFT Basics"): the DFT
``X(k) = sum_n x(n) w_N^{nk}`` with ``w_N = exp(-2 i pi / N)`` for the forward
direction and the sign of the exponent flipped for the backward one, with no
normalisation.  ``sign`` is that sign: -1 forward, +1 backward.

Functions (all return complex128 numpy arrays of the input's shape):

* ``dft_naive``   -- the definition written out, O(N^2).
* ``fft_radix2``  -- recursive radix-2 decimation in time (powers of two).
* ``fft_mixed``   -- recursive smallest-prime-factor decimation in time.
* ``fft``         -- ``fft_radix2`` for powers of two, else ``fft_mixed``.
* ``fft2d``       -- separable 2-D transform (rows, then columns).
* ``transpose``   -- ``out[b][c][r] = in[b][r][c]``.
* ``range_compress`` -- SAR range compression (the matched filter): the
  circular cross-correlation of every row with the pulse replica, scaled by n
  (what B(F(x) * conj(F(ref))) gives with the unnormalised backward
  transform), evaluated from its definition.
* ``fourstep_reference`` -- the four-step identity written out with numpy
  (column DFTs, twiddle, row DFTs, transposed read-out), used only to locate
  index mistakes; its sub-DFTs call ``fft``.

The C part lives in ``fft_oracle.c`` and is built by ``build()`` with gcc
(``-O2``, no fast-math) into ``liboracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fft_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``fft_oracle.c`` into ``liboracle.so`` (gcc, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=gnu11",
               "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    for name in ("oracle_dft_naive", "oracle_fft_radix2", "oracle_fft_mixed"):
        fn = getattr(lib, name)
        fn.argtypes = [dp, dp, i64, i64, ctypes.c_int, ctypes.c_int]
        fn.restype = ctypes.c_int
    lib.oracle_fft2d.argtypes = [dp, dp, i64, i64, i64, ctypes.c_int, ctypes.c_int]
    lib.oracle_fft2d.restype = ctypes.c_int
    lib.oracle_transpose.argtypes = [dp, dp, i64, i64, i64]
    lib.oracle_transpose.restype = ctypes.c_int
    lib.oracle_unit_root.argtypes = [i64, i64, ctypes.c_int, dp]
    lib.oracle_unit_root.restype = None
    lib.oracle_range_compress.argtypes = [dp, dp, i64, i64, dp, i64, ctypes.c_int]
    lib.oracle_range_compress.restype = ctypes.c_int
    lib.oracle_nthreads.argtypes = []
    lib.oracle_nthreads.restype = ctypes.c_int
    _lib = lib
    return lib


def _as_c128(x) -> np.ndarray:
    x = np.asarray(x)
    if not np.iscomplexobj(x):
        x = x.astype(np.complex128)
    return np.ascontiguousarray(x, dtype=np.complex128)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_sign(sign: int) -> None:
    if sign not in (-1, 1):
        raise ValueError("sign must be -1 (forward) or +1 (backward)")


def _batched(fn_name: str, x, sign: int, threads: int) -> np.ndarray:
    _check_sign(sign)
    a = _as_c128(x)
    if a.ndim == 0:
        raise ValueError("need at least one dimension")
    n = a.shape[-1]
    batch = a.size // n if n else 0
    out = np.empty_like(a)
    if a.size == 0:
        return out
    rc = getattr(_load(), fn_name)(_ptr(a), _ptr(out), n, batch, sign, threads)
    if rc == 2:
        raise ValueError(f"{fn_name}: length {n} is not a power of two")
    if rc != 0:
        raise RuntimeError(f"{fn_name} failed (status {rc})")
    return out


def dft_naive(x, sign: int = -1, threads: int = 0) -> np.ndarray:
    """The DFT definition over the last axis, O(N^2) (Background, FFT Basics)."""
    return _batched("oracle_dft_naive", x, sign, threads)


def fft_radix2(x, sign: int = -1, threads: int = 0) -> np.ndarray:
    """Recursive radix-2 DIT over the last axis (power-of-two lengths)."""
    return _batched("oracle_fft_radix2", x, sign, threads)


def fft_mixed(x, sign: int = -1, threads: int = 0) -> np.ndarray:
    """Recursive smallest-prime-factor DIT over the last axis (any length)."""
    return _batched("oracle_fft_mixed", x, sign, threads)


def fft(x, sign: int = -1, threads: int = 0) -> np.ndarray:
    """Radix-2 for power-of-two lengths, the mixed-radix recursion otherwise."""
    n = np.asarray(x).shape[-1]
    if n >= 1 and (n & (n - 1)) == 0:
        return fft_radix2(x, sign, threads)
    return fft_mixed(x, sign, threads)


def fft2d(x, sign: int = -1, threads: int = 0) -> np.ndarray:
    """2-D transform over the last two axes (rows, then columns)."""
    _check_sign(sign)
    a = _as_c128(x)
    if a.ndim < 2:
        raise ValueError("fft2d needs at least two dimensions")
    rows, cols = a.shape[-2], a.shape[-1]
    batch = a.size // (rows * cols)
    out = np.empty_like(a)
    rc = _load().oracle_fft2d(_ptr(a), _ptr(out), rows, cols, batch, sign, threads)
    if rc != 0:
        raise RuntimeError(f"oracle_fft2d failed (status {rc})")
    return out


def transpose(x) -> np.ndarray:
    """``out[..., c, r] = in[..., r, c]`` on complex values (bit-exact copy)."""
    a = _as_c128(x)
    rows, cols = a.shape[-2], a.shape[-1]
    batch = a.size // (rows * cols)
    out = np.empty(a.shape[:-2] + (cols, rows), dtype=np.complex128)
    rc = _load().oracle_transpose(_ptr(a), _ptr(out), rows, cols, batch)
    if rc != 0:
        raise RuntimeError("oracle_transpose failed")
    return out


def range_compress(x, ref, threads: int = 0) -> np.ndarray:
    """SAR range compression of every row of ``x`` (shape [..., n]) with the
    pulse replica ``ref`` (length L <= n), from the definition
    ``y[m] = n * sum_{l<L} x[(m + l) mod n] * conj(ref[l])`` (paper: the SAR
    application section and Fig. 3, range compression after the range FFT)."""
    a = _as_c128(x)
    r = _as_c128(ref).reshape(-1)
    if a.ndim == 0:
        raise ValueError("need at least one dimension")
    n = a.shape[-1]
    if not 1 <= r.size <= n:
        raise ValueError("replica length must be in [1, n]")
    rows = a.size // n if n else 0
    out = np.empty_like(a)
    if a.size == 0:
        return out
    if _load().oracle_range_compress(_ptr(a), _ptr(out), n, rows, _ptr(r), r.size, threads) != 0:
        raise RuntimeError("oracle_range_compress failed")
    return out


def unit_root(m: int, n: int, sign: int = -1) -> complex:
    """``exp(sign 2 pi i m / n)`` as the definition's table computes it."""
    buf = (ctypes.c_double * 2)()
    _load().oracle_unit_root(m, n, sign, buf)
    return complex(buf[0], buf[1])


def nthreads() -> int:
    """Threads the oracle uses when ``threads`` is 0 (online CPUs, capped at 256)."""
    return int(_load().oracle_nthreads())


def fourstep_reference(x, n1: int, n2: int, sign: int = -1) -> np.ndarray:
    """The four-step identity for N = n1*n2 written out step by step.

    Index map: input ``n = n2_len*n1 + n2`` is viewed as ``A[n1][n2]``; the
    n2-column transforms (length n1) give ``A'[k1][n2]``; each point is
    multiplied by ``exp(sign 2 pi i n2 k1 / N)``; the row transforms (length
    n2) give ``Y[k1][k2]``; and ``X[k1 + n1*k2] = Y[k1][k2]``.  This is the
    splitting of a long transform into shorter ones the paper builds larger
    FFTs from (Approach, "Other FFT sizes").  Used only to locate index
    mistakes; the parity reference for long lengths is ``fft``.
    """
    a = _as_c128(x)
    N = n1 * n2
    if a.shape[-1] != N:
        raise ValueError("last axis must be n1*n2")
    lead = a.shape[:-1]
    A = a.reshape(lead + (n1, n2))
    # column transforms: move n1 to the last axis
    Ac = np.swapaxes(A, -1, -2)                      # [..., n2, n1]
    Ap = fft(np.ascontiguousarray(Ac), sign)         # [..., n2, k1]
    k1 = np.arange(n1, dtype=np.int64)
    n2i = np.arange(n2, dtype=np.int64)
    m = np.outer(n2i, k1) % N                        # [n2, k1]
    tw = np.array([[unit_root(int(v), N, sign) for v in row] for row in m]) if N <= 4096 else \
        np.exp(sign * 2j * np.pi * m / N)
    B = Ap * tw                                      # [..., n2, k1]
    Bt = np.ascontiguousarray(np.swapaxes(B, -1, -2))  # [..., k1, n2]
    Y = fft(Bt, sign)                                # [..., k1, k2]
    X = np.swapaxes(Y, -1, -2)                       # [..., k2, k1] -> index k1 + n1*k2
    return np.ascontiguousarray(X).reshape(lead + (N,))
