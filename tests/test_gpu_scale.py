"""The output scale option (fft_plan_opts_t.scale): every output is
multiplied by it in the last store, so a backward plan with scale 1/n is the
normalised inverse, backward(forward(x)) = x.

For each kernel family that writes final outputs (single block, the
all-register cross-lane kernel, the variable-thread kernels, the run-time
schedule kernel, four-step pass 2, FP16 storage and its compact form, range
compression) the scaled result is checked against the unscaled one times the
scale, bit for bit where the scale is a power of two (an exact FP32 product),
and the normalised round trip against the input.  Pass 1 of the four-step
path must not scale its (intermediate) outputs, which the four-step cases
cover.  With FP16 storage the unscaled inverse of a long transform
(n times the input) overflows binary16; the scaled one does not."""
import numpy as np
import pytest

from oracle import metrics
from paper_1505_08067_amd import fftblock as fb
from paper_1505_08067_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


CASES = [
    # (n, batch, planner options besides the scale, storage)
    (4096, 8, {}, fb.STORAGE_C64),
    (1024, 16, {}, fb.STORAGE_C64),                                         # cross-lane default
    (6000, 4, {}, fb.STORAGE_C64),                                          # variable-thread
    (15360, 2, {}, fb.STORAGE_C64),
    (1024, 8, dict(radix=[8, 16, 8], flags=fb.VARIANT_RUNTIME_SCHEDULE), fb.STORAGE_C64),
    (1 << 20, 2, {}, fb.STORAGE_C64),                                       # four-step
    (1 << 16, 3, {}, fb.STORAGE_C64),
    (4096, 8, {}, fb.STORAGE_F16),
    (15360, 2, {}, fb.STORAGE_F16),
    (1 << 20, 1, {}, fb.STORAGE_F16_COMPACT),
]


@pytest.mark.parametrize("n,batch,extra,storage", CASES)
def test_scaled_output_and_normalised_round_trip(n, batch, extra, storage):
    say(f"case: scale n={n} batch={batch} opts={extra} storage={storage}")
    dt = torch.complex32 if storage else torch.complex64
    x = torch.from_numpy(inputs.uniform(1200 + n % 97, batch, n)).to("cuda").to(dt)
    s = 1.0 / n
    with fb.Plan(n, batch, fb.FORWARD, fb.make_opts(storage=storage, **extra)) as f, \
            fb.Plan(n, batch, fb.BACKWARD, fb.make_opts(storage=storage, **extra)) as b, \
            fb.Plan(n, batch, fb.BACKWARD, fb.make_opts(storage=storage, scale=s, **extra)) as bs:
        assert bs.describe()["kernel_name"] == b.describe()["kernel_name"]
        assert np.float32(bs.describe()["scale"]) == np.float32(s)
        y = f.execute(x)
        z = b.execute(y)
        zs = bs.execute(y)
        torch.cuda.synchronize()
    zf = torch.view_as_real(z).float()
    zsf = torch.view_as_real(zs).float()
    pow2 = (n & (n - 1)) == 0
    if storage and n * 2 > 65504:
        # the unscaled FP16 round trip (n times the input) overflows binary16:
        # there the scale is what makes the result representable, and only the
        # normalised round trip below is checked
        assert not torch.isfinite(zf).all()
    elif pow2 and storage == fb.STORAGE_C64:
        # a power-of-two scale is exact in FP32: the same bits as scaling afterwards
        assert torch.equal(zsf, zf * np.float32(s))
    else:
        # one rounding more (a non-power-of-two scale, or FP16 rounding of the
        # scaled rather than the unscaled value)
        ulp = 2.0 ** -10 if storage else 2.0 ** -23
        ref = zf * np.float32(s)
        assert float((zsf - ref).abs().max()) <= 2 * ulp * float(ref.abs().max()) + 1e-30
    # the normalised round trip returns the input
    xin = torch.view_as_real(x).float().cpu().numpy().astype(np.float64)
    back = zsf.cpu().numpy().astype(np.float64)
    xc = (xin[..., 0] + 1j * xin[..., 1]).reshape(batch, n)
    bc = (back[..., 0] + 1j * back[..., 1]).reshape(batch, n)
    err = metrics.rel_l2_per_transform(bc, xc)
    tol = (3 * 2.0 ** -11 if storage else 0.0) + 2 * metrics.tolerance(max(n, 2))
    say(f"  round trip max rel L2 {err.max():.2e} (tol {tol:.1e})")
    assert np.all(err <= tol)


def test_scaled_range_compression():
    n, batch = 8192, 16
    say(f"case: scaled range compression n={n} batch={batch}")
    rep = torch.from_numpy(inputs.sar_replica()).to("cuda")
    x = torch.from_numpy(inputs.uniform(1300, batch, n)).to("cuda")
    with fb.RangeCompressor(n, batch, rep) as r, \
            fb.RangeCompressor(n, batch, rep, fb.make_opts(scale=1.0 / n)) as rs:
        y = r.execute(x)
        ys = rs.execute(x)
        torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(ys), torch.view_as_real(y) * np.float32(1.0 / n))
