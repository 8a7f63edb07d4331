"""Seeded synthetic inputs for the batched FFT path.

This module only draws inputs; it holds none of the transform's arithmetic,
so the tests can hand the same arrays to the FP64 oracle and to the GPU path.

Recipes (the paper publishes no data set; these stand in for the radar data
it processes):

* ``uniform(seed, batch, n)`` -- real and imaginary parts iid uniform[-1, 1]:
  ``numpy.random.default_rng(seed).uniform(-1, 1, (batch, n, 2))`` drawn in
  float64 and rounded once to float32.  The oracle consumes these rounded
  values.
* ``sar(seed, pulses, ranges, ...)`` -- a synthetic range/azimuth matrix for
  the range-Doppler processing chain the paper targets (Background, "Radar
  application"): each row (pulse) is the sum of ``targets`` linear-FM chirps
  ``exp(i pi TB ((n - d_j)/L - 1/2)^2)`` of length ``L = round(alpha*TB)``
  starting at a per-target delay ``d_j`` (drawn once per matrix, stationary
  scatterers) with a unit-modulus phase drawn per (pulse, target), plus
  complex Gaussian noise at the requested SNR (noise variance = mean signal
  power / 10^(snr/10)).
* ``sar_replica(tb, alpha)`` -- the transmitted pulse the ``sar`` echoes are
  made of (the chirp at delay 0, complex64, length L): the reference that
  range compression correlates every row with.
* ``ragged_sizes(seed, ...)`` -- the ragged mix: an equal share of points per
  size, shuffled with the seed.
* ``poisson_trace(seed, ...)`` -- request arrival times and shapes for the
  serving stream: exponential inter-arrival gaps at ``rate``, N = 2^k with k
  uniform on an integer range, batch log-uniform on [1, max_batch],
  direction 50/50.
"""
from __future__ import annotations

import math

import numpy as np


def uniform(seed: int, batch: int, n: int) -> np.ndarray:
    """complex64 array [batch, n] with iid uniform[-1,1] real and imaginary parts."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, (batch, n, 2)).astype(np.float32)
    out = np.empty((batch, n), dtype=np.complex64)
    out.real = u[..., 0]
    out.imag = u[..., 1]
    return out


def sar(seed: int, pulses: int = 4096, ranges: int = 8192, targets: int = 32,
        tb: float = 500.0, alpha: float = 1.25, snr_db: float = 10.0) -> np.ndarray:
    """complex64 [pulses, ranges] SAR-shaped raw matrix (see the module docstring)."""
    rng = np.random.default_rng(seed)
    L = int(round(alpha * tb))
    if L > ranges:
        raise ValueError("chirp longer than a row")
    n = np.arange(L, dtype=np.float64)
    chirp = np.exp(1j * np.pi * tb * (n / L - 0.5) ** 2)
    delays = rng.integers(0, ranges - L + 1, size=targets)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=(pulses, targets))
    sig = np.zeros((pulses, ranges), dtype=np.complex128)
    for j in range(targets):
        d = int(delays[j])
        sig[:, d:d + L] += np.exp(1j * phases[:, j])[:, None] * chirp[None, :]
    p_sig = float(np.mean(np.abs(sig) ** 2))
    sigma2 = p_sig / (10.0 ** (snr_db / 10.0))
    noise = rng.standard_normal((pulses, ranges, 2)) * math.sqrt(sigma2 / 2.0)
    sig.real += noise[..., 0]
    sig.imag += noise[..., 1]
    return sig.astype(np.complex64)


def sar_delays(seed: int, ranges: int = 8192, targets: int = 32, tb: float = 500.0,
               alpha: float = 1.25):
    """The target delays ``sar`` draws for the same seed (first draws of the stream)."""
    rng = np.random.default_rng(seed)
    L = int(round(alpha * tb))
    return rng.integers(0, ranges - L + 1, size=targets)


def sar_replica(tb: float = 500.0, alpha: float = 1.25) -> np.ndarray:
    """complex64 pulse replica: ``exp(i pi TB (n/L - 1/2)^2)``, n < L = round(alpha*TB)."""
    L = int(round(alpha * tb))
    n = np.arange(L, dtype=np.float64)
    return np.exp(1j * np.pi * tb * (n / L - 0.5) ** 2).astype(np.complex64)


RAGGED_POW2 = tuple(2 ** k for k in range(6, 17))
RAGGED_MIXED = (1000, 3072, 6000, 15360)


def ragged_sizes(seed: int, sizes=RAGGED_POW2 + RAGGED_MIXED, total_points: int = 2 ** 28):
    """Shuffled list of transform lengths with an equal share of points per size."""
    rng = np.random.default_rng(seed)
    share = total_points / len(sizes)
    lst = []
    for s in sizes:
        lst.extend([int(s)] * int(round(share / s)))
    arr = np.array(lst, dtype=np.int64)
    rng.shuffle(arr)
    return arr


def poisson_trace(seed: int, rate: float = 2000.0, duration: float = 10.0,
                  k_lo: int = 8, k_hi: int = 22, max_batch: int = 512):
    """Arrival times (s), N, batch and sign (-1/+1) per request."""
    rng = np.random.default_rng(seed)
    count = int(rate * duration * 1.5) + 16
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    keep = t < duration
    t = t[keep]
    m = t.size
    k = rng.integers(k_lo, k_hi + 1, size=m)
    b = np.floor(np.exp(rng.uniform(0.0, math.log(max_batch + 1), size=m))).astype(np.int64)
    b = np.clip(b, 1, max_batch)
    sign = np.where(rng.uniform(size=m) < 0.5, -1, 1)
    return t, (2 ** k).astype(np.int64), b, sign
