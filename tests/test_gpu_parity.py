"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Inputs are seeded and synthetic (uniform[-1,1] parts, or the SAR-shaped
matrix).  Gate: per transform, relative L2 error <= 1e-6 * log2(N) (the 2-D
SAR matrix counts as one transform of P*R points; a round trip gets twice the
tolerance).  The transpose must be bit-exact.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import metrics
from paper_1505_08067_amd import fftblock as fb
from paper_1505_08067_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD, BWD = fb.FORWARD, fb.BACKWARD


def say(*a):
    print(*a, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")


def gpu_fft(x, sign, inplace=False, opts=None):
    x = np.ascontiguousarray(x, dtype=np.complex64)
    n = x.shape[-1]
    batch = x.size // n
    with fb.Plan(n, batch, sign, opts) as plan:
        d = to_dev(x)
        y = plan.execute(d, out=d if inplace else None)
        torch.cuda.synchronize()
        return y.cpu().numpy().reshape(x.shape)


def check(y, ref, n_points, n_axes=1, factor=1.0, label=""):
    mx, md, tol = metrics.check(y, ref, n_points, n_axes=n_axes, factor=factor)
    say(f"  {label}: max rel L2 {mx:.3e}  median {md:.3e}  tol {tol:.1e}")
    return mx


# ----------------------------------------------------------- the block path
def test_cfg1_n1024_batch64_forward_against_definition():
    say("case: N=1024 batch=64 forward seed=0 vs the O(N^2) definition")
    x = inputs.uniform(0, 64, 1024)
    y = gpu_fft(x, FWD)
    ref = oracle.dft_naive(x.astype(np.complex128), FWD)
    check(y, ref, 1024, label="N=1024 x 64")


BLOCK_SIZES = [2 ** k for k in range(1, 15)]


@pytest.mark.parametrize("n", BLOCK_SIZES)
@pytest.mark.parametrize("sign", [FWD, BWD])
def test_block_sizes_against_oracle(n, sign):
    # small batches of 8192 and longer default to four-step: name the limit
    opts = fb.make_opts(block_limit=n) if n >= 8192 else None
    d = fb.plan_query(n, 1, sign, opts)
    assert d["path"] == fb.PATH_BLOCK
    fpb = max(1, d["transforms_per_block"])
    batch = 2 * fpb + 1 if n < 16384 else 3   # a partly filled last workgroup
    say(f"case: block N={n} batch={batch} sign={sign} kernel={d['kernel_name']}")
    x = inputs.uniform(100 + n, batch, n)
    y = gpu_fft(x, sign, opts=opts)
    ref = oracle.fft(x.astype(np.complex128), sign)
    check(y, ref, n, label=f"N={n}")


@pytest.mark.parametrize("n,batch", [(8192, 15), (8192, 16), (16384, 47), (16384, 48), (32768, 63), (32768, 64)])
def test_long_block_default_path_by_batch(n, batch):
    # a long block fills the device only from a minimum batch on (one
    # 32768-point transform takes a whole compute unit); below it the
    # default plan is four-step
    first = {8192: 16, 16384: 48, 32768: 64}[n]
    d = fb.plan_query(n, batch)
    assert d["path"] == (fb.PATH_BLOCK if batch >= first else fb.PATH_FOURSTEP)
    say(f"case: N={n} batch={batch} default path {d['path']} {d['kernel_name']}")
    x = inputs.uniform(150 + batch, batch, n)
    for sign in (FWD, BWD):
        y = gpu_fft(x, sign)
        ref = oracle.fft(x.astype(np.complex128), sign)
        check(y, ref, n, label=f"N={n} batch={batch} sign={sign}")


def test_n1_is_copy():
    x = inputs.uniform(5, 7, 1)
    for sign in (FWD, BWD):
        assert np.array_equal(gpu_fft(x, sign), x)
        assert np.array_equal(gpu_fft(x, sign, inplace=True), x)


@pytest.mark.parametrize("n", [4096, 1 << 20])
def test_cfg2_full_size_forward_and_inverse(n):
    batch = 4096 if n == 4096 else 16
    say(f"case: N={n} batch={batch} forward+inverse, full comparison")
    x = inputs.uniform(1, batch, n)
    xd = x.astype(np.complex128)
    for sign in (FWD, BWD):
        y = gpu_fft(x, sign)
        ref = oracle.fft(xd, sign)
        check(y, ref, n, label=f"N={n} sign={sign}")


@pytest.mark.parametrize("L", list(range(15, 23)))
def test_fourstep_sizes_against_oracle(L):
    n = 1 << L
    batch = 2 if L <= 20 else 1
    d = fb.plan_query(n, batch)
    say(f"case: four-step N=2^{L} = {d['n1']}x{d['n2']} batch={batch}")
    x = inputs.uniform(200 + L, batch, n)
    for sign in (FWD, BWD):
        y = gpu_fft(x, sign)
        ref = oracle.fft(x.astype(np.complex128), sign)
        check(y, ref, n, label=f"N=2^{L} sign={sign}")


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [64, 4096, 1 << 20])
def test_closed_forms_on_gpu(n):
    say(f"case: closed forms N={n}")
    k = np.arange(n)
    x = np.zeros((4, n), np.complex64)
    x[0, 0] = 1                                   # impulse -> all ones
    x[1, 3] = 1                                   # shifted impulse -> w^(3k)
    x[2, :] = 1                                   # constant -> N delta
    x[3] = np.exp(2j * np.pi * 5 * k / n)         # tone -> N delta at 5
    y = gpu_fft(x, FWD)
    exp = np.zeros((4, n), complex)
    exp[0] = 1
    exp[1] = np.exp(-2j * np.pi * ((3 * k) % n) / n)
    exp[2, 0] = n
    ref_tone = oracle.fft(x[3:4].astype(np.complex128), FWD)[0]
    exp[3] = ref_tone
    check(y[:3], exp[:3], n, label="impulse/shift/constant")
    assert abs(y[3, 5] - n) / n < 1e-5
    # Parseval on random input
    r = inputs.uniform(7, 3, n)
    Y = gpu_fft(r, FWD).astype(np.complex128)
    lhs = np.sum(np.abs(Y) ** 2, -1)
    rhs = n * np.sum(np.abs(r.astype(np.complex128)) ** 2, -1)
    assert np.all(np.abs(lhs / rhs - 1) < 2e-6 * math.log2(n))


@pytest.mark.parametrize("n", [1024, 8192, 1 << 18])
def test_roundtrip(n):
    batch = 8 if n < (1 << 18) else 2
    x = inputs.uniform(9, batch, n)
    y = gpu_fft(gpu_fft(x, FWD), BWD) / n
    check(y, x.astype(np.complex128), n, factor=2.0, label=f"round trip N={n}")


# ---------------------------------------------------------- isolation etc.
@pytest.mark.parametrize("n", [256, 1024, 4096, 1 << 16])
def test_batch_isolation_with_poisoned_neighbours(n):
    d = fb.plan_query(n, 1)
    batch = max(8, 2 * d["transforms_per_block"])
    say(f"case: NaN-poisoned neighbours N={n} batch={batch}")
    x = inputs.uniform(11, batch, n)
    x[1::2] = np.nan + 1j * np.inf
    y = gpu_fft(x, FWD)
    good = x[0::2]
    assert np.all(np.isfinite(y[0::2].view(np.float32)))
    check(y[0::2], oracle.fft(good.astype(np.complex128), FWD), n, label="clean slots")


@pytest.mark.parametrize("n,limit", [(512, 0), (4096, 0), (16384, 0), (32768, 32768), (1 << 20, 0)])
def test_in_place_equals_out_of_place(n, limit):
    # 16384 x 3 runs four-step (small batch), 32768 x 3 the single block
    batch = 3
    opts = fb.make_opts(block_limit=limit) if limit else None
    x = inputs.uniform(12, batch, n)
    a = gpu_fft(x, FWD, opts=opts)
    b = gpu_fft(x, FWD, inplace=True, opts=opts)
    assert np.array_equal(a, b)


def test_deterministic_repeat():
    x = inputs.uniform(13, 64, 4096)
    assert np.array_equal(gpu_fft(x, FWD), gpu_fft(x, FWD))


# ---------------------------------------------------------------- transpose
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 100, 37), (1, 64, 64), (2, 65, 129), (2, 66, 130), (2, 130, 66),
                                   (2, 34, 258), (3, 2, 200), (1, 4096, 8192), (1, 8192, 4096)])
def test_transpose_bit_exact(shape):
    say(f"case: transpose {shape}")
    rng = np.random.default_rng(14)
    bits = rng.integers(0, 2 ** 32, size=shape + (2,), dtype=np.uint32)
    x = bits.view(np.float32).view(np.complex64).reshape(shape)
    d = torch.from_numpy(x.copy()).to("cuda")
    t = fb.transpose(d)
    tt = fb.transpose(t)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    ref = oracle.transpose(x.astype(np.complex128)) if x.size < 2e6 else None
    exp = np.ascontiguousarray(np.swapaxes(x, -1, -2))
    assert np.array_equal(got.view(np.uint32), exp.view(np.uint32))
    if ref is not None:
        assert np.array_equal(got[np.isfinite(got)], ref.astype(np.complex64)[np.isfinite(got)])
    assert np.array_equal(tt.cpu().numpy().view(np.uint32), x.view(np.uint32))


@pytest.mark.parametrize("values", [1 << 20, 2 * 1037, 2, (1 << 25) + 6])
def test_copy_probe(values):
    # whole rounds, a ragged last round, one 16-byte element, and three
    # elements past one round of the capped grid (16384 x 1024 x 16 bytes)
    say(f"copy {values} complex64 values")
    g = torch.Generator(device="cuda").manual_seed(15)
    a = torch.randn(values, dtype=torch.complex64, device="cuda", generator=g)
    b = torch.full_like(a, complex(7.0, -7.0))
    guard = torch.full((2 * values + 64,), complex(3.0, 3.0), dtype=torch.complex64, device="cuda")
    fb.copy_(guard[32:32 + values], a)
    fb.copy_(b, a)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.float32), b.view(torch.float32))
    assert torch.equal(guard[32:32 + values].view(torch.float32), a.view(torch.float32))
    assert bool((guard[:32] == complex(3.0, 3.0)).all()) and bool((guard[32 + values:] == complex(3.0, 3.0)).all())


def test_device_query_and_block_limit():
    info = fb.device_query()
    say(f"device: {info}")
    assert info["arch"].startswith("gfx950")
    assert info["warp_size"] == 64
    assert info["lds_per_cu"] == 160 * 1024
    assert info["block_max"] == [16384, 8192, 4096]
    # half exchanges hold half the points in LDS: twice the analytic limit
    assert fb.block_limit() <= 2 * info["block_max"][0]


def test_errors_on_device():
    with fb.Plan(1024, 2) as p:
        x = to_dev(inputs.uniform(1, 2, 1024))
        with pytest.raises(ValueError):
            p.execute(x[:1])
        with pytest.raises(TypeError):
            p.execute(x.to(torch.complex128))
        # partial overlap is rejected by the library
        big = to_dev(inputs.uniform(1, 3, 1024))
        st = fb.load().fft_execute(p.handle, big.data_ptr(), big.data_ptr() + 8 * 1024, None)
        assert st == 1
    with pytest.raises(fb.FFTError) as ei:
        fb.Plan(1001, 1)
    assert ei.value.status == 2


# ------------------------------------------------------------ SAR 2-D chain
def test_sar_range_azimuth_chain_and_roundtrip():
    P, R = 4096, 8192
    say(f"case: SAR {P}x{R} range FFT -> corner turn -> azimuth FFT, and back")
    x = inputs.sar(2, pulses=P, ranges=R)
    xd = to_dev(x)
    with fb.Plan(R, P, FWD) as rf, fb.Plan(P, R, FWD) as af, fb.Plan(P, R, BWD) as ab, fb.Plan(R, P, BWD) as rb:
        a = rf.execute(xd)                 # range FFT per pulse
        t = fb.transpose(a.view(P, R))     # [range][pulse]
        b = af.execute(t)                  # azimuth FFT per range bin
        torch.cuda.synchronize()
        y = b.cpu().numpy().reshape(R, P).T
        ref = oracle.fft2d(x.astype(np.complex128), FWD)
        check(y[None], ref[None], P * R, n_axes=2, label="SAR forward 2-D")
        c = ab.execute(b)
        t2 = fb.transpose(c.view(R, P))
        z = rb.execute(t2)
        torch.cuda.synchronize()
        back = z.cpu().numpy().reshape(P, R) / (P * R)
        check(back[None], x.astype(np.complex128)[None], P * R, n_axes=2, factor=2.0, label="SAR round trip")


def test_execute_pass_timed_matches_and_stamps():
    # the dispatch-stamped launch computes the same result and gives a positive duration
    for n, batch in ((4096, 64), (1 << 20, 2)):
        say(f"case: timed passes n={n} batch={batch}")
        x = to_dev(inputs.uniform(21, batch, n))
        with fb.Plan(n, batch) as p:
            d = p.describe()
            y0 = torch.empty_like(x)
            y1 = torch.empty_like(x)
            sh = torch.cuda.current_stream().cuda_stream
            passes = (1, 2) if d["path"] == fb.PATH_FOURSTEP else (1,)
            for ps in passes:
                p.execute_pass_ptr(ps, x.data_ptr(), y0.data_ptr(), sh)
            torch.cuda.synchronize()
            evs = []
            for ps in passes:
                e0, e1 = fb.Event(), fb.Event()
                p.execute_pass_timed_ptr(ps, x.data_ptr(), y1.data_ptr(), sh, e0, e1)
                evs.append((e0, e1))
            torch.cuda.synchronize()
            for e0, e1 in evs:
                ms = e0.elapsed_ms(e1)
                say(f"  {ms * 1e3:.1f} us")
                assert 0.0 < ms < 1000.0
            assert np.array_equal(y0.cpu().numpy().view(np.uint32), y1.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("n", [3, 1000, 4096, 16384, 1 << 20])
def test_zero_input_gives_exact_zero(n):
    # degenerate case of the error metric: a zero transform must come out exactly zero
    say(f"case: zero input N={n}")
    x = np.zeros((2, n), np.complex64)
    for sign in (FWD, BWD):
        y = gpu_fft(x, sign)
        assert np.all(y == 0), sign
    if n == 4096:
        with fb.Plan(n, 2, FWD, fb.make_opts(storage=fb.STORAGE_F16)) as p:
            z = p.execute(torch.zeros(2 * n, dtype=torch.complex32, device="cuda"))
            assert torch.count_nonzero(torch.view_as_real(z)).item() == 0
        rep = to_dev(inputs.sar_replica())
        with fb.RangeCompressor(n, 2, rep) as rc:
            z = rc.execute(to_dev(x))
            assert torch.count_nonzero(torch.view_as_real(z)).item() == 0


@pytest.mark.parametrize("n", [4096, 1 << 20])
def test_execute_on_a_side_stream(n):
    # work queued on a stream other than the current one gives the same
    # result, and the output allocated for it stays valid until that stream
    # has run (the binding records the stream on the tensors)
    batch = 8 if n == 4096 else 2
    say(f"case: side stream N={n} batch={batch}")
    x = torch.from_numpy(inputs.uniform(60, batch, n)).to("cuda")
    side = torch.cuda.Stream()
    with fb.Plan(n, batch) as p:
        ref = p.execute(x)
        # one plan, one workspace: the side stream starts after the current one
        side.wait_stream(torch.cuda.current_stream())
        ys = [p.execute(x, stream=side) for _ in range(3)]
        ys.append(fb.transpose(x.view(batch, n // 64, 64), stream=side))
        side.synchronize()
        torch.cuda.synchronize()
    for y in ys[:3]:
        assert torch.equal(torch.view_as_real(y), torch.view_as_real(ref))
    tref = x.view(batch, n // 64, 64).transpose(1, 2).contiguous()
    assert torch.equal(torch.view_as_real(ys[3]), torch.view_as_real(tref))
