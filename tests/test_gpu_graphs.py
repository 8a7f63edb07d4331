"""Executes captured into a HIP graph (through torch.cuda.CUDAGraph) and
replayed: the library's execute path launches only kernels (no allocation,
no synchronisation, no memset), so a captured execute must give, on every
replay, exactly the eager result of whatever its input buffer then holds.

Each case replays the graph three times with eager work in between (the
output cleared, an unrelated torch kernel), checks every replay bit for bit
against the eager execute of the same input, then rewrites the input and
checks that the next replay transforms the new values.  Covered: a single
block, the four-step path with the plan's workspace, the compact FP16 form,
the allocation-free entry point (its workspace the library's static array)
and the standalone transpose."""
import ctypes

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
    return torch.view_as_real(t).contiguous().view(torch.int16 if t.dtype == torch.complex32 else torch.int32).reshape(-1)


def _replays(launch, x, y, x_new, eager):
    """Capture launch(stream) (reads x, writes y), replay it three times
    between unrelated eager work, then once more after x is rewritten."""
    ref = eager(x)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        launch(side.cuda_stream)  # a warm-up outside the capture, as torch advises
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        launch(torch.cuda.current_stream().cuda_stream)
    scratch = torch.randn(256, 256, device="cuda")
    for r in range(3):
        y.zero_()
        scratch = scratch @ scratch.T * 1e-3
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(_bits(y), _bits(ref)), f"replay {r}"
    x.copy_(x_new)
    ref_new = eager(x)
    y.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(_bits(y), _bits(ref_new)), "replay after the input changed"
    return ref_new


@pytest.mark.parametrize("n,batch,storage", [(4096, 64, fb.STORAGE_C64), (1 << 20, 2, fb.STORAGE_C64),
                                             (1 << 20, 2, fb.STORAGE_F16_COMPACT), (1 << 16, 3, fb.STORAGE_C64)])
def test_captured_execute(n, batch, storage):
    say(f"case: captured fft_execute n={n} batch={batch} storage={storage}")
    dt = torch.complex32 if storage else torch.complex64
    opts = fb.make_opts(storage=storage)
    with fb.Plan(n, batch, fb.FORWARD, opts) as p:
        x = torch.from_numpy(inputs.uniform(800, batch, n)).to("cuda").to(dt)
        x_new = torch.from_numpy(inputs.uniform(801, batch, n)).to("cuda").to(dt)
        y = torch.empty_like(x)
        with fb.Plan(n, batch, fb.FORWARD, opts) as q:
            def eager(xx):
                out = q.execute(xx)
                torch.cuda.synchronize()
                return out
            got = _replays(lambda st: p.execute_ptr(x.data_ptr(), y.data_ptr(), st), x, y, x_new, eager)
        if storage == fb.STORAGE_C64 and n == 1 << 16:
            metrics.check(got.cpu().numpy(), oracle.fft(inputs.uniform(801, batch, n).astype(np.complex128),
                                                        fb.FORWARD), n)


def test_captured_execute_static():
    n, batch = 1 << 20, 4
    say(f"case: captured fft_execute_static n={n} batch={batch}")
    lib = fb.load()
    with fb.Plan(n, 1, fb.BACKWARD) as p:
        assert p.describe()["path"] == fb.PATH_FOURSTEP
        x = torch.from_numpy(inputs.uniform(810, batch, n)).to("cuda")
        x_new = torch.from_numpy(inputs.uniform(811, batch, n)).to("cuda")
        y = torch.empty_like(x)
        ws = torch.empty_like(x)

        def launch(st):
            fb._check(lib.fft_execute_static(p.handle, batch, x.data_ptr(), y.data_ptr(), ctypes.c_void_p(st)),
                      "fft_execute_static")

        def eager(xx):
            out = torch.empty_like(xx)
            fb._check(lib.fft_execute_ex(p.handle, batch, xx.data_ptr(), out.data_ptr(), ws.data_ptr(), None),
                      "fft_execute_ex")
            torch.cuda.synchronize()
            return out
        _replays(launch, x, y, x_new, eager)


def test_captured_transpose():
    rows, cols, batch = 1000, 3000, 2
    say(f"case: captured fft_transpose {rows} x {cols} x {batch}")
    x = torch.from_numpy(inputs.uniform(820, batch, rows * cols)).to("cuda")
    x_new = torch.from_numpy(inputs.uniform(821, batch, rows * cols)).to("cuda")
    y = torch.empty_like(x)

    def eager(xx):
        out = fb.transpose(xx.view(batch, rows, cols))
        torch.cuda.synchronize()
        return out.reshape(-1)

    def launch(st):
        fb._check(fb.load().fft_transpose(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), rows, cols,
                                          batch, ctypes.c_void_p(st)), "fft_transpose")
    got = _replays(launch, x, y, x_new, eager)
    want = x_new.view(batch, rows, cols).transpose(1, 2).reshape(-1)
    assert torch.equal(_bits(got), _bits(want))
