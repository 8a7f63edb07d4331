"""The seeded input generators: determinism, shapes and the stated recipes."""
import math

import numpy as np

from paper_1505_08067_amd import inputs
import oracle


def test_uniform_deterministic_and_bounded():
    a = inputs.uniform(0, 4, 64)
    b = inputs.uniform(0, 4, 64)
    c = inputs.uniform(1, 4, 64)
    assert a.dtype == np.complex64 and a.shape == (4, 64)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.all(np.abs(a.real) <= 1) and np.all(np.abs(a.imag) <= 1)
    rng = np.random.default_rng(0)
    u = rng.uniform(-1, 1, (4, 64, 2)).astype(np.float32)
    assert np.array_equal(a.real, u[..., 0]) and np.array_equal(a.imag, u[..., 1])


def test_sar_shape_snr_and_chirp_positions():
    P, R, J = 64, 2048, 4
    x = inputs.sar(2, pulses=P, ranges=R, targets=J)
    assert x.shape == (P, R) and x.dtype == np.complex64
    d = inputs.sar_delays(2, ranges=R, targets=J)
    L = 625
    # range compression by correlation with the chirp peaks at each delay
    n = np.arange(L)
    chirp = np.exp(1j * np.pi * 500 * (n / L - 0.5) ** 2)
    ref = np.zeros(R, complex)
    ref[:L] = chirp
    X = oracle.fft(x.astype(np.complex128), -1)
    H = oracle.fft(ref[None], -1)[0]
    comp = oracle.fft(X * np.conj(H)[None, :], +1) / R
    prof = np.mean(np.abs(comp) ** 2, axis=0)
    top = set(np.argsort(prof)[-J:].tolist())
    assert top == set(int(v) for v in d)
    # SNR: noise power is about 1/10 of the signal power
    sig_pow = J * L / R
    tot = float(np.mean(np.abs(x.astype(np.complex128)) ** 2))
    assert abs(tot / sig_pow - 1.1) < 0.05


def test_ragged_equal_point_share():
    s = inputs.ragged_sizes(3)
    s2 = inputs.ragged_sizes(3)
    assert np.array_equal(s, s2)
    total = int(np.sum(s))
    assert abs(total - 2 ** 28) / 2 ** 28 < 1e-3
    for size in inputs.RAGGED_POW2 + inputs.RAGGED_MIXED:
        pts = int(np.sum(s[s == size]))
        assert abs(pts - 2 ** 28 / 15) / (2 ** 28 / 15) < 0.01


def test_poisson_trace_rate_and_ranges():
    t, n, b, sign = inputs.poisson_trace(4, rate=2000.0, duration=10.0)
    assert abs(t.size / 10.0 - 2000) < 3 * math.sqrt(20000) / 10
    assert np.all(np.diff(t) > 0)
    assert n.min() >= 256 and n.max() <= 2 ** 22
    assert b.min() >= 1 and b.max() <= 512
    assert set(np.unique(sign).tolist()) == {-1, 1}


def test_sar_replica_is_the_chirp_the_echoes_are_made_of():
    # a single noiseless target at delay d: the row equals the replica shifted by d,
    # up to its unit-modulus phase
    ref = inputs.sar_replica()
    assert ref.dtype == np.complex64 and ref.size == 625
    assert np.allclose(np.abs(ref), 1.0, atol=1e-6)
    x = inputs.sar(5, pulses=2, ranges=2048, targets=1, snr_db=200.0)
    d = int(inputs.sar_delays(5, ranges=2048, targets=1)[0])
    for row in x:
        seg = row[d:d + ref.size].astype(np.complex128)
        ratio = seg / ref.astype(np.complex128)
        assert np.allclose(ratio, ratio[0], atol=1e-5) and abs(abs(ratio[0]) - 1) < 1e-5
        assert np.max(np.abs(np.delete(row, np.s_[d:d + ref.size]))) < 1e-6


def test_poisson_trace_batch_is_log_uniform():
    # batch = floor(exp(U[0, ln 513))): P(b <= 22) = ln 23 / ln 513, about one half
    t, n, b, sign = inputs.poisson_trace(9, 2000.0, 20.0)
    frac = np.mean(b <= 22)
    assert abs(frac - np.log(23) / np.log(513)) < 0.02
    assert abs(np.mean(sign == -1) - 0.5) < 0.02
    k = np.log2(n).astype(int)
    assert set(np.unique(k)) == set(range(8, 23))
