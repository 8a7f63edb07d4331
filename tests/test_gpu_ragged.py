"""Ragged batches (persistent work-list kernels in one graph, the plain path,
the per-length branch graph) and the autotuner, on the GPU, against the oracle."""
import numpy as np
import pytest

import oracle
from oracle import metrics
from paper_1505_08067_amd import fftblock as fb
from paper_1505_08067_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CLASSES = [(64, 5), (1000, 3), (4096, 2), (3, 7), (1 << 16, 1), (15360, 2), (6000, 1), (3072, 3), (1, 4)]


def say(*a):
    print(*a, flush=True)


def _ragged_input(classes, seed):
    parts = [inputs.uniform(seed + i, c, n).reshape(-1) for i, (n, c) in enumerate(classes)]
    return np.concatenate(parts)


def _check_classes(y, x, classes, sign):
    at = 0
    for n, c in classes:
        xs = x[at:at + n * c].reshape(c, n).astype(np.complex128)
        ys = y[at:at + n * c].reshape(c, n)
        ref = oracle.fft(xs, sign)
        mx, _, tol = metrics.check(ys, ref, max(n, 2))
        say(f"  class N={n} x{c}: max rel L2 {mx:.2e} (tol {tol:.1e})")
        at += n * c


@pytest.mark.parametrize("sign", [fb.FORWARD, fb.BACKWARD])
def test_ragged_persistent_plain_and_branches_match_oracle(sign):
    say(f"case: ragged mix {CLASSES} sign={sign}")
    x = _ragged_input(CLASSES, 700)
    xd = torch.from_numpy(x).to("cuda")
    with fb.Ragged(CLASSES, sign) as r:
        yg = r.execute(xd)                               # persistent work-list kernels
        torch.cuda.synchronize()
        d = r.describe()
        say(f"  {d['kernel_nodes']} kernel nodes: {d['persistent_launches']}, fallback {d['fallback_classes']}")
        assert d["total_points"] == x.size and d["graph_nodes"] == d["kernel_nodes"] > 0
        # one launch per LDS-footprint class present; lengths 3 and 1, and the
        # mixed lengths 15360 and 6000 (their own kernels), on nodes of their own
        assert 2 <= len(d["persistent_launches"]) <= 3 and d["fallback_classes"] == 4
        assert d["kernel_nodes"] == len(d["persistent_launches"]) + 4
        yp = r.execute(xd, mode=fb.RAGGED_PLAIN)
        yb = r.execute(xd, mode=fb.RAGGED_BRANCHES)
        torch.cuda.synchronize()
        ygn, ypn, ybn = yg.cpu().numpy(), yp.cpu().numpy(), yb.cpu().numpy()
        # the plain path and its branch graph run the same kernels: bitwise equal
        assert np.array_equal(ybn.view(np.uint32), ypn.view(np.uint32))
        _check_classes(ygn, x, CLASSES, sign)
        _check_classes(ypn, x, CLASSES, sign)
        # new buffers: the graph's node arguments are updated
        x2 = _ragged_input(CLASSES, 800)
        y2 = r.execute(torch.from_numpy(x2).to("cuda"))
        torch.cuda.synchronize()
        _check_classes(y2.cpu().numpy(), x2, CLASSES, sign)
        # in place, launched several times with host work in between
        buf = torch.from_numpy(x).to("cuda")
        for rep in range(3):
            b = buf.clone()
            r.execute(b, out=b)
            torch.cuda.synchronize()
            assert np.array_equal(b.cpu().numpy().view(np.uint32), ygn.view(np.uint32)), rep


def test_persistent_relaunch_back_to_back():
    # the queue counters return to zero at the end of every launch: five
    # launches with no synchronisation in between give five equal results
    say("case: five back-to-back persistent launches")
    x = _ragged_input(CLASSES, 710)
    xd = torch.from_numpy(x).to("cuda")
    y = torch.empty_like(xd)
    outs = []
    with fb.Ragged(CLASSES, fb.FORWARD) as r:
        for _ in range(5):
            r.execute(xd, out=y)
            outs.append(y.clone())
        torch.cuda.synchronize()
    first = outs[0].cpu().numpy()
    _check_classes(first, x, CLASSES, fb.FORWARD)
    for o in outs[1:]:
        assert np.array_equal(o.cpu().numpy().view(np.uint32), first.view(np.uint32))


def test_each_class_alone_equals_in_mix():
    # persistent: a class alone (a one-class ragged plan) equals the same class
    # in the mix, bitwise; plain: each default plan alone equals the plain mix
    x = _ragged_input(CLASSES, 900)
    xd = torch.from_numpy(x).to("cuda")
    with fb.Ragged(CLASSES) as r:
        mix = r.execute(xd).cpu().numpy()
        plain = r.execute(xd, mode=fb.RAGGED_PLAIN).cpu().numpy()
    at = 0
    for n, c in CLASSES:
        say(f"case: class N={n} x{c} alone")
        part = xd[at:at + n * c].clone()
        with fb.Ragged([(n, c)]) as one:
            alone = one.execute(part).cpu().numpy()
        assert np.array_equal(alone.view(np.uint32), mix[at:at + n * c].view(np.uint32)), n
        with fb.Plan(n, c) as p:
            alone = p.execute(part).cpu().numpy()
        assert np.array_equal(alone.view(np.uint32), plain[at:at + n * c].view(np.uint32)), n
        at += n * c


def test_stage_benchmark_positive():
    for radix, stage in ((2, 0), (4, 3), (8, 7), (16, 6)):
        v = fb.stage_benchmark(1024, radix, stage)
        say(f"  stage radix {radix} at {stage}: {v:.3f} ns per transform")
        assert v >= 0.0


def test_autotune_sets_wisdom_and_stays_correct(tmp_path):
    fb.wisdom_clear()
    rep = fb.autotune(1024, 4096)
    say(f"  autotune 1024: predicted {rep['predicted']} cost {rep['predicted_cost']:.2f}; "
        f"chosen {rep['chosen']} {rep['chosen_us']:.1f} us of {len(rep['candidates'])}")
    assert rep["predicted"] and np.prod(rep["predicted"]) == 1024
    assert len(rep["stage_cost"]) == 10 + 9 + 8 + 7
    say(f"  predicted schedule run: {rep['predicted_us']:.1f} us; best compiled schedule on the same "
        f"run-time-schedule kernel: {rep['chosen_schedule_rt_us']:.1f} us")
    assert rep["predicted_us"] > 0 and rep["chosen_schedule_rt_us"] > 0
    name = rep["chosen"].split(":")[0]
    assert rep["chosen"] and fb.wisdom_get(1024) == name
    with fb.Plan(1024, 33) as p:
        d = p.describe()
        assert d["kernel_name"] == name
        if rep["chosen_predicted"]:
            assert d["radix"] == rep["predicted"]
        x = inputs.uniform(1, 33, 1024)
        y = p.execute(torch.from_numpy(x).to("cuda")).cpu().numpy()
    metrics.check(y, oracle.fft(x.astype(np.complex128)), 1024)
    rep2 = fb.autotune(6000, 256)           # mixed length: whole-kernel validation only
    assert rep2["log2n"] == 0 and rep2["predicted"] == [] and rep2["chosen"]
    rep3 = fb.autotune(1 << 20, 4)          # four-step: pass-1 x pass-2 pairs
    say(f"  autotune 2^20: chosen {rep3['chosen']} {rep3['chosen_us']:.1f} us of {len(rep3['candidates'])}")
    assert "+" in rep3["chosen"] and len(rep3["candidates"]) > 1
    with fb.Plan(1 << 20, 2) as p:
        d = p.describe()
        assert d["kernel_name"] + "+" + d["kernel_name2"] == rep3["chosen"]
        x = inputs.uniform(2, 2, 1 << 20)
        y = p.execute(torch.from_numpy(x).to("cuda")).cpu().numpy()
    metrics.check(y, oracle.fft(x.astype(np.complex128)), 1 << 20)
    path = tmp_path / "wisdom.txt"
    fb.wisdom_save(str(path))
    txt = path.read_text()
    assert "\n1024\t" in txt and "\n6000\t" in txt and "\n1048576\t" in txt
    fb.wisdom_clear()


def test_ragged_fp16_storage():
    """The ragged mix in the FP16-storage form: persistent and plain paths each
    within 2^-11 + the FP32 tolerance of the exact DFT of the FP16-valued
    input, and each class alone (a one-class ragged plan) equal to the same
    class in the mix, bitwise."""
    classes = CLASSES
    say(f"case: ragged fp16 {classes}")
    x = _ragged_input(classes, 950)
    xh = torch.from_numpy(x).to("cuda").to(torch.complex32)
    xr = torch.view_as_real(xh).float().cpu().numpy().astype(np.float64)
    xexact = xr[..., 0] + 1j * xr[..., 1]
    with fb.Ragged(classes, storage=fb.STORAGE_F16) as r:
        yg = r.execute(xh)
        yp = r.execute(xh, mode=fb.RAGGED_PLAIN)
        torch.cuda.synchronize()
        g16 = torch.view_as_real(yg).cpu().numpy()
        p16 = torch.view_as_real(yp).cpu().numpy()
    at = 0
    for n, c in classes:
        ref = oracle.fft(xexact[at:at + n * c].reshape(c, n))
        for name, out in (("persistent", g16), ("plain", p16)):
            y = out[at:at + n * c].astype(np.float64)
            err = metrics.rel_l2_per_transform((y[..., 0] + 1j * y[..., 1]).reshape(c, n), ref)
            say(f"  {name} class N={n} x{c}: max rel L2 {err.max():.2e}")
            assert np.all(err <= 2.0 ** -11 + metrics.tolerance(n))
        with fb.Ragged([(n, c)], storage=fb.STORAGE_F16) as one:
            alone = torch.view_as_real(one.execute(xh[at:at + n * c].clone())).cpu().numpy()
        assert np.array_equal(alone.view(np.int16), g16[at:at + n * c].view(np.int16)), n
        at += n * c


def test_full_ragged_mix_sampled_against_oracle():
    # the full mix the bench times (15 lengths, about 2^28 points, one graph
    # launch): the first and the last transform of every length against the oracle
    sizes = inputs.ragged_sizes(3)
    classes = [(int(n), int((sizes == n).sum())) for n in inputs.RAGGED_POW2 + inputs.RAGGED_MIXED]
    total = sum(n * c for n, c in classes)
    say(f"case: full ragged mix, {len(classes)} lengths, {total} points")
    x = torch.empty(total, dtype=torch.complex64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    x.real.uniform_(-1.0, 1.0, generator=gen)
    x.imag.uniform_(-1.0, 1.0, generator=gen)
    with fb.Ragged(classes, fb.FORWARD) as r:
        y = r.execute(x)
        torch.cuda.synchronize()
        d = r.describe()
    # one persistent launch per LDS-footprint class, and the two mixed
    # lengths whose own kernels (stages on different thread counts) run
    # beside them as plain launches
    say(f"  launches: {d['persistent_launches']}, fallback {d['fallback_classes']}")
    assert len(d["persistent_launches"]) <= 3 and d["fallback_classes"] == 2
    assert d["kernel_nodes"] == len(d["persistent_launches"]) + 2
    assert sum(L["classes"] for L in d["persistent_launches"]) == len(classes) - 2 + 1   # 65536: two passes
    at = 0
    for n, c in classes:
        for b in (0, c - 1):
            lo = at + b * n
            xs = x[lo:lo + n].cpu().numpy().astype(np.complex128)[None, :]
            ys = y[lo:lo + n].cpu().numpy()[None, :]
            mx, _, tol = metrics.check(ys, oracle.fft(xs, -1), n)
            say(f"  N={n} transform {b} of {c}: rel L2 {mx:.2e} (tol {tol:.1e})")
        at += n * c
    assert at == total
