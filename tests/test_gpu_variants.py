"""Every compiled kernel variant against the FP64 oracle.

The planner's defaults are covered by test_gpu_parity.py; the runtime sweep
and the schedule search can select any other compiled (schedule, workgroup
shape, variant), so each of them is held to the same tolerance here,
including the persistent variants with more work units than resident
workgroups and the four-step path forced onto short lengths.
"""
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


def run(n, batch, sign, opts, x):
    with fb.Plan(n, batch, sign, opts) as p:
        d = p.describe()
        xd = torch.from_numpy(x).to("cuda")
        y = p.execute(xd)
        torch.cuda.synchronize()
        return y.cpu().numpy(), d


def _block_variants():
    out = []
    for k in fb.kernels():
        # (the run-time-schedule kernels take the plan's schedule: test_gpu_schedules.py)
        if k["kind"] == "block" and k["n"] >= 2 and not k["flags"] & fb.VARIANT_RUNTIME_SCHEDULE:
            out.append(pytest.param(k, id=k["name"]))
    return out


@pytest.mark.parametrize("k", _block_variants())
def test_block_variant(k):
    n = k["n"]
    persistent = bool(k["flags"] & (fb.VARIANT_PERSISTENT | fb.VARIANT_LOOP))
    batch = 2 * k["c"] + 1
    if persistent:
        batch = max(batch, (1 << 24) // n + 3)   # more units than resident workgroups
    fp16 = bool(k["flags"] & fb.VARIANT_FP16_STORAGE)
    opts = fb.make_opts(radix=k["radix"], flags=k["flags"], c=k["c"],
                        storage=fb.STORAGE_F16 if fp16 else fb.STORAGE_C64,
                        block_limit=n if n > 16384 else 0)   # at any batch
    x = inputs.uniform(300 + n, batch, n)
    for sign in (fb.FORWARD, fb.BACKWARD):
        say(f"{k['name']} batch={batch} sign={sign}")
        if fp16:
            # FP16 storage: against the exact DFT of the FP16-valued input
            with fb.Plan(n, batch, sign, opts) as p:
                d = p.describe()
                xh = torch.from_numpy(x).to("cuda").to(torch.complex32)
                y = torch.view_as_real(p.execute(xh)).float().cpu().numpy().astype(np.float64)
                xr = torch.view_as_real(xh).float().cpu().numpy().astype(np.float64)
            assert d["kernel_name"] == k["name"]
            ref = oracle.fft(xr[..., 0] + 1j * xr[..., 1], sign)
            err = metrics.rel_l2_per_transform(y[..., 0] + 1j * y[..., 1], ref)
            assert np.all(err <= 2.0 ** -11 + metrics.tolerance(max(n, 2)))
            continue
        y, d = run(n, batch, sign, opts, x)
        assert d["kernel_name"] == k["name"]
        ref = oracle.fft(x.astype(np.complex128), sign)
        metrics.check(y, ref, n)


def _pass_combos():
    # 1) at 2^20 = 1024 x 1024: every complex64 pass-1 kernel with a plain pass 2
    #    of each workspace width, and every pass-2 kernel with the default pass 1;
    # 2) every other pass kernel (any length, FP16 storage included) with the
    #    default partner of its storage form, at a split that fits both
    ks = fb.kernels()
    c64 = [k for k in ks if not k["flags"] & fb.VARIANT_FP16_STORAGE]
    p1 = [k for k in c64 if k["kind"] == "pass1" and k["n"] == 1024]
    p2 = [k for k in c64 if k["kind"] == "pass2" and k["n"] == 1024]
    plain2 = [k for k in p2 if k["flags"] == 0]
    default1 = [k for k in p1 if k["is_default"]]
    combos, seen = [], set()

    def add(n1, a, b):
        if (a["name"], b["name"]) not in seen:
            seen.add((a["name"], b["name"]))
            combos.append(pytest.param(n1, a, b, id=f"{a['name']}+{b['name']}"))

    for a, b in [(a, b) for a in p1 for b in plain2] + [(a, b) for a in default1 for b in p2]:
        add(1024, a, b)
    dflt = {}

    def form(k):  # storage form of a pass kernel: complex64, FP16, FP16 with an FP16 workspace
        return (bool(k["flags"] & fb.VARIANT_FP16_STORAGE), bool(k["flags"] & fb.VARIANT_FP16_WORKSPACE))
    for k in ks:
        if k["kind"] in ("pass1", "pass2") and k["is_default"]:
            dflt[(k["kind"], k["n"], form(k))] = k
    for k in ks:
        if k["kind"] == "pass1":
            n1, n2 = k["n"], (2048 if k["n"] <= 1024 else 1024)
            b = dflt.get(("pass2", n2, form(k)))
            if b and n2 % k["c"] == 0 and n1 % b["c"] == 0:
                add(n1, k, b)
        elif k["kind"] == "pass2":
            n1 = 512 if k["n"] <= 2048 else 256
            a = dflt.get(("pass1", n1, form(k)))
            if a and k["n"] % a["c"] == 0 and n1 % k["c"] == 0:
                add(n1, a, k)
    return combos


@pytest.mark.parametrize("n1,k1,k2", _pass_combos())
def test_fourstep_variant_pairs(n1, k1, k2):
    n2 = k2["n"]
    n, batch = n1 * n2, 2
    if (k1["flags"] | k2["flags"]) & fb.VARIANT_LOOP:
        batch = max(batch, (1 << 23) // n)   # more units than resident workgroups
    half = bool(k1["flags"] & fb.VARIANT_FP16_STORAGE)
    compact = bool(k1["flags"] & fb.VARIANT_FP16_WORKSPACE)
    # lengths a single block would take are forced onto the four-step path
    limit = 0 if n > fb.block_limit() else max(1024, n // 2)
    storage = fb.STORAGE_F16_COMPACT if compact else fb.STORAGE_F16 if half else fb.STORAGE_C64
    opts = fb.make_opts(radix=k1["radix"], flags=k1["flags"], c=k1["c"], flags2=k2["flags"], c2=k2["c"], n1=n1,
                        storage=storage, block_limit=limit)
    say(f"case: four-step {n1} x {n2} {k1['name']} + {k2['name']}")
    x = inputs.uniform(400 + n1, batch, n)
    if half:
        with fb.Plan(n, batch, fb.FORWARD, opts) as p:
            d = p.describe()
            xh = torch.from_numpy(x).to("cuda").to(torch.complex32)
            y = torch.view_as_real(p.execute(xh)).float().cpu().numpy().astype(np.float64)
            xr = torch.view_as_real(xh).float().cpu().numpy().astype(np.float64)
        assert (d["kernel_name"], d["kernel_name2"]) == (k1["name"], k2["name"])
        ref = oracle.fft(xr[..., 0] + 1j * xr[..., 1], fb.FORWARD)
        err = metrics.rel_l2_per_transform(y[..., 0] + 1j * y[..., 1], ref)
        # one FP16 rounding at the output, and one more of the workspace in the compact form
        assert np.all(err <= (2 if compact else 1) * 2.0 ** -11 + metrics.tolerance(n))
        return
    y, d = run(n, batch, fb.FORWARD, opts, x)
    assert (d["kernel_name"], d["kernel_name2"]) == (k1["name"], k2["name"])
    ref = oracle.fft(x.astype(np.complex128), fb.FORWARD)
    metrics.check(y, ref, n)


@pytest.mark.parametrize("n", [2048, 4096, 8192, 16384])
@pytest.mark.parametrize("sign", [fb.FORWARD, fb.BACKWARD])
def test_fourstep_forced_on_block_sizes(n, sign):
    opts = fb.make_opts(block_limit=1024)
    d = fb.plan_query(n, 5, sign, opts)
    assert d["path"] == fb.PATH_FOURSTEP
    x = inputs.uniform(500 + n, 5, n)
    y, d = run(n, 5, sign, opts, x)
    say(f"forced four-step N={n} = {d['n1']}x{d['n2']}")
    ref = oracle.fft(x.astype(np.complex128), sign)
    metrics.check(y, ref, n)


def test_kernel_occupancy_fits_the_compute_unit():
    # every catalogue kernel can be resident, and the reported count respects the
    # compute unit's LDS and thread limits
    info = fb.device_query()
    props = torch.cuda.get_device_properties(0)
    max_threads = getattr(props, "max_threads_per_multi_processor", 2048)
    for k in fb.kernels():
        occ = fb.kernel_occupancy(k["name"])
        say(f"{k['name']} occupancy {occ}")
        assert occ >= 1, k["name"]
        assert occ * k["lds_bytes"] <= info["lds_per_cu"], k["name"]
        assert occ * k["threads"] <= max_threads, k["name"]


def test_vec16_needs_aligned_data():
    # sixteen-byte lanes read and write pairs of complex values: a buffer
    # only 8-byte aligned is refused, not read across a pair boundary
    k = next(k for k in fb.kernels() if k["kind"] == "block" and k["flags"] & fb.VARIANT_VEC16)
    n, batch = k["n"], 3
    say(f"case: {k['name']} misaligned")
    opts = fb.make_opts(radix=k["radix"], flags=k["flags"], c=k["c"])
    buf = torch.zeros(n * batch + 1, dtype=torch.complex64, device="cuda")
    out = torch.zeros_like(buf)
    with fb.Plan(n, batch, fb.FORWARD, opts) as p:
        with pytest.raises(fb.FFTError):
            p.execute(buf[1:], out=out[1:])
        p.execute(buf[:-1], out=out[:-1])   # aligned views run
    torch.cuda.synchronize()
