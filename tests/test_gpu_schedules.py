"""The run-time-schedule block kernel against the FP64 oracle.

The schedule search (paper, Approach, "FFT performance model": a shortest
path through the stage graph) can return any sequence of radices 2, 4, 8,
16 whose product is the length; this kernel runs whichever it is.  Every
such schedule of at most 8 stages is checked at N = 64, 256 and 1024 (the
paper's length), seeded samples at 2048 ... 16384, both directions, with a
batch that leaves the last workgroup partly empty, and the schedules the
paper's stage tables name.
"""
import math
import random

import numpy as np
import pytest

import oracle
from oracle import metrics
from paper_1505_08067_amd import fftblock as fb
from paper_1505_08067_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RADICES = (2, 4, 8, 16)


def say(*a):
    print(*a, flush=True)


def compositions(log2n, max_stages=8):
    """Every sequence of radices from RADICES multiplying to 2^log2n."""
    out = []

    def rec(left, acc):
        if left == 0:
            out.append(list(acc))
            return
        if len(acc) == max_stages:
            return
        for r in RADICES:
            lr = int(math.log2(r))
            if lr <= left:
                rec(left - lr, acc + [r])

    rec(log2n, [])
    return out


def _rt_opts(sched):
    return fb.make_opts(radix=sched, flags=fb.VARIANT_RUNTIME_SCHEDULE | fb.VARIANT_NT_LOAD | fb.VARIANT_NT_STORE)


def _check_schedules(n, scheds, signs=(fb.FORWARD, fb.BACKWARD)):
    rt = [k for k in fb.kernels() if k["kind"] == "block" and k["n"] == n and k["flags"] & fb.VARIANT_RUNTIME_SCHEDULE]
    assert len(rt) == 1
    batch = 2 * rt[0]["c"] + 1
    x = inputs.uniform(4000 + n, batch, n)
    xd = torch.from_numpy(x).to("cuda")
    worst = 0.0
    for sign in signs:
        ref = oracle.fft(x.astype(np.complex128), sign)
        for sched in scheds:
            with fb.Plan(n, batch, sign, _rt_opts(sched)) as p:
                d = p.describe()
                assert d["kernel_name"] == rt[0]["name"] and d["radix"] == sched
                y = p.execute(xd)
                torch.cuda.synchronize()
            mx, _, _ = metrics.check(y.cpu().numpy(), ref, n)
            worst = max(worst, mx)
    say(f"  N={n}: {len(scheds)} schedules x {len(signs)} directions, worst rel L2 {worst:.2e} "
        f"(tol {metrics.tolerance(n):.1e})")


@pytest.mark.parametrize("n", [64, 256, 1024])
def test_every_schedule(n):
    scheds = compositions(int(math.log2(n)))
    say(f"case: every schedule of {n}: {len(scheds)}")
    _check_schedules(n, scheds)


@pytest.mark.parametrize("n", [2048, 4096, 8192, 16384])
def test_sampled_schedules(n):
    rng = random.Random(n)
    scheds = rng.sample(compositions(int(math.log2(n))), 12)
    lead = {2048: 8, 4096: 16, 8192: 2, 16384: 4}[n]
    scheds.append([lead] + [16] * ((int(math.log2(n)) - int(math.log2(lead))) // 4))   # radix 16 after one other
    say(f"case: {len(scheds)} sampled schedules of {n}")
    _check_schedules(n, scheds)


def test_paper_schedules_at_1024_in_place():
    # the schedules the paper's stage tables compare (FFT_{8,8,8,2},
    # FFT_{4,8,8,4}, and the additive optimum over the printed tables,
    # [8,8,4,4]), in place
    n, batch = 1024, 9
    x = inputs.uniform(77, batch, n)
    ref = oracle.fft(x.astype(np.complex128), fb.FORWARD)
    for sched in ([8, 8, 8, 2], [4, 8, 8, 4], [8, 8, 4, 4]):
        say(f"case: 1024 schedule {sched} in place")
        buf = torch.from_numpy(x).to("cuda")
        with fb.Plan(n, batch, fb.FORWARD, _rt_opts(sched)) as p:
            p.execute(buf, out=buf)
            torch.cuda.synchronize()
        metrics.check(buf.cpu().numpy(), ref, n)


def test_compositions_counted():
    # paths through the stage graph with edges of 1..4 stages: 401 at 1024
    # (a tetranacci number), ten of them longer than the kernel's 8 stages
    assert len(compositions(10, 10)) == 401 and len(compositions(10)) == 391
