"""fft_execute_static, the allocation-free four-step execute, against
fft_execute_ex with a caller-allocated workspace: the same kernels run, so
the outputs must agree bit for bit.  Each plan is called twice in a row, the
second call with a smaller batch (the scratch array keeps the first call's
contents); one case is also checked against the FP64 oracle, and a batch
beyond the array is refused before anything is launched."""
import numpy as np
import pytest

import oracle
from oracle import metrics
from paper_1505_08067_amd import fftblock as fb
from paper_1505_08067_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _bits(t):
    return t.view(torch.float32).view(torch.int32)


@pytest.mark.parametrize("n,batches", [(1 << 20, (8, 3)), (1 << 16, (100, 7)), (1 << 22, (2, 1)),
                                       (4096, (64, 5))])
def test_static_scratch_equals_execute_ex(n, batches):
    lib = fb.load()
    assert lib.fft_static_scratch_bytes() == 64 << 20
    for direction in (fb.FORWARD, fb.BACKWARD):
        with fb.Plan(n, 1, direction) as plan:
            four = plan.describe()["path"] == fb.PATH_FOURSTEP
            assert four == (n > 4096)
            for k, batch in enumerate(batches):
                say(f"case: fft_execute_static n={n} batch={batch} direction={direction} call {k}")
                x = inputs.uniform(700 + k, batch, n)
                xd = torch.from_numpy(x).to("cuda")
                y_static = torch.empty_like(xd)
                y_ex = torch.empty_like(xd)
                ws = torch.empty(n * batch, dtype=torch.complex64, device="cuda")
                torch.cuda.synchronize()
                fb._check(lib.fft_execute_static(plan.handle, batch, xd.data_ptr(), y_static.data_ptr(), None),
                          "fft_execute_static")
                fb._check(lib.fft_execute_ex(plan.handle, batch, xd.data_ptr(), y_ex.data_ptr(),
                                             ws.data_ptr() if four else None, None), "fft_execute_ex")
                torch.cuda.synchronize()
                assert torch.equal(_bits(y_static), _bits(y_ex))
                if n == 1 << 16 and k == 1:
                    metrics.check(y_static.cpu().numpy(), oracle.fft(x.astype(np.complex128), direction), n)


def test_static_scratch_limit_is_refused():
    lib = fb.load()
    n = 1 << 20
    batch = (64 << 20) // 8 // n + 1
    x = torch.zeros(n * batch, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    with fb.Plan(n, 1, fb.FORWARD) as plan:
        say(f"case: fft_execute_static n={n} batch={batch} beyond the scratch array")
        assert lib.fft_execute_static(plan.handle, batch, x.data_ptr(), y.data_ptr(), None) == 7
        assert fb.status_string(7) == "request exceeds the library's static scratch buffer"
        # the largest batch that fits runs
        fb._check(lib.fft_execute_static(plan.handle, batch - 1, x.data_ptr(), y.data_ptr(), None),
                  "fft_execute_static")
        torch.cuda.synchronize()
        assert float(y[: n * (batch - 1)].abs().max()) == 0.0


def test_static_scratch_compact_fp16():
    # the compact FP16 form keeps its workspace in FP16 pairs: 4 bytes per
    # point, so the array holds twice the complex64 batch (16 x 2^20 here)
    lib = fb.load()
    n = 1 << 20
    opts = fb.make_opts(storage=fb.STORAGE_F16_COMPACT)
    with fb.Plan(n, 1, fb.FORWARD, opts=opts) as plan:
        assert plan.describe()["path"] == fb.PATH_FOURSTEP
        for k, batch in enumerate((16, 5)):
            say(f"case: fft_execute_static compact FP16 n={n} batch={batch} call {k}")
            xd = torch.from_numpy(inputs.uniform(900 + k, batch, n)).to("cuda").to(torch.complex32)
            y_static = torch.empty_like(xd)
            y_ex = torch.empty_like(xd)
            ws = torch.empty(n * batch, dtype=torch.complex32, device="cuda")
            torch.cuda.synchronize()
            fb._check(lib.fft_execute_static(plan.handle, batch, xd.data_ptr(), y_static.data_ptr(), None),
                      "fft_execute_static")
            fb._check(lib.fft_execute_ex(plan.handle, batch, xd.data_ptr(), y_ex.data_ptr(), ws.data_ptr(), None),
                      "fft_execute_ex")
            torch.cuda.synchronize()
            assert torch.equal(torch.view_as_real(y_static).view(torch.int16),
                               torch.view_as_real(y_ex).view(torch.int16))
        x = torch.zeros(n * 17, dtype=torch.complex32, device="cuda")
        assert lib.fft_execute_static(plan.handle, 17, x.data_ptr(), x.data_ptr(), None) == 7
