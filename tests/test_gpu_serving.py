"""The GPU server: results against the oracle, each request alone equal to
the same request in the mix (bitwise), budget and rejection, continuous
batching, and a short replay of a Poisson arrival stream; plus
fft_execute_ex (per-call batch and workspace) that the server relies on."""
import numpy as np
import pytest

import oracle
from oracle import metrics
from paper_1505_08067_amd import fftblock as fb
from paper_1505_08067_amd import inputs
from paper_1505_08067_amd import serving as sv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_execute_ex_batch_and_workspace():
    # (1024, 4096, 3) and (1024, 2, 4096): the call's batch, not the plan's,
    # picks the block kernel's width (one-wave form below 128 workgroups)
    for n, plan_batch, batch in ((4096, 1, 7), (1000, 2, 5), (1 << 20, 1, 3), (1 << 16, 4, 2), (1024, 4096, 3),
                                 (1024, 2, 4096)):
        say(f"case: execute_ex n={n} plan batch {plan_batch} call batch {batch}")
        x = inputs.uniform(n + 11, batch, n)
        xd = torch.from_numpy(x).to("cuda")
        y = torch.empty_like(xd)
        with fb.Plan(n, plan_batch) as p:
            four = p.describe()["path"] == fb.PATH_FOURSTEP
            ws = torch.empty(n * batch, dtype=torch.complex64, device="cuda") if four else None
            if four and batch > plan_batch:
                with pytest.raises(fb.FFTError):     # the plan's own workspace is too small
                    fb._check(fb.load().fft_execute_ex(p.handle, batch, xd.data_ptr(), y.data_ptr(), None, None),
                              "x")
            fb._check(fb.load().fft_execute_ex(p.handle, batch, xd.data_ptr(), y.data_ptr(),
                                               ws.data_ptr() if ws is not None else None, None), "fft_execute_ex")
            torch.cuda.synchronize()
        metrics.check(y.cpu().numpy(), oracle.fft(x.astype(np.complex128)), n)


def test_submit_waits_for_the_producer_on_the_callers_stream():
    # The input is written on a side torch stream, behind about 2 ms of other
    # work, and submitted at once from that stream without synchronising: the
    # server's launch must wait for the copy (an event on the submitter's
    # stream), or it would transform the zeros the buffer held before.
    n, b = 4096, 64
    x = inputs.uniform(77, b, n)
    src = torch.from_numpy(x).to("cuda")
    ref = oracle.fft(x.astype(np.complex128))
    side = torch.cuda.Stream()
    with sv.Server(hbm_budget=1 << 30, n_streams=4) as srv:
        srv.prepare(n, fb.FORWARD)
        for rep in range(3):
            say(f"case: submit from a side stream, repetition {rep}")
            buf = torch.zeros_like(src)
            junk = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            with torch.cuda.stream(side):
                for _ in range(20):
                    junk.mul_(1.0001)
                buf.copy_(src)
                t = srv.submit(buf, n, b, fb.FORWARD)
            y, info = srv.result(t)
            torch.cuda.synchronize()
            metrics.check(y.cpu().numpy(), ref, n)
            del buf, junk


def _mix(seed, count, sizes, max_batch):
    rng = np.random.default_rng(seed)
    return [(int(rng.choice(sizes)), int(rng.integers(1, max_batch + 1)), int(rng.choice([-1, 1])))
            for _ in range(count)]


def test_server_results_alone_equal_in_mix():
    sizes = [64, 256, 1000, 4096, 6000, 16384, 1 << 16, 1 << 18]
    reqs = _mix(31, 48, sizes, 6)
    data = [torch.from_numpy(inputs.uniform(2000 + i, b, n)).to("cuda") for i, (n, b, _) in enumerate(reqs)]
    say(f"case: server mix of {len(reqs)} requests")
    with sv.Server(hbm_budget=1 << 30, n_streams=4, max_inflight=2, max_coalesce=16) as srv:
        for n in set(n for n, _, _ in reqs):
            srv.prepare(n, -1)
            srv.prepare(n, 1)
        tickets = [srv.submit(data[i], n, b, d) for i, (n, b, d) in enumerate(reqs)]
        outs = []
        for tk in tickets:
            y, info = srv.result(tk)
            assert info["state"] == fb.REQ_DONE and info["t_done"] >= info["t_launch"] >= info["t_arrive"]
            outs.append(y.cpu().numpy())
            srv.release(tk)
        st = srv.stats()
        say(f"  launches {st['launches']} for {st['completed']} requests, coalesced {st['coalesced_requests']}, "
            f"peak in flight {st['peak_inflight_bytes'] / 2**20:.1f} MiB, p50 {st['latency_p50']*1e3:.3f} ms")
        assert st["completed"] == len(reqs) and st["peak_inflight_bytes"] <= 1 << 30
    for i, (n, b, d) in enumerate(reqs):
        x = data[i].cpu().numpy().astype(np.complex128)
        metrics.check(outs[i], oracle.fft(x, d), n)
    # each request alone on a fresh server: bitwise the same as in the mix
    with sv.Server(hbm_budget=1 << 30) as srv:
        for i in (0, 5, 11, 23, 47):
            n, b, d = reqs[i]
            y, info = srv.result(srv.submit(data[i], n, b, d))
            assert info["group_size"] == 1
            assert np.array_equal(y.cpu().numpy().view(np.uint32), outs[i].view(np.uint32)), i


def test_server_coalesces_a_burst_and_respects_the_budget():
    n, count = 1024, 40
    data = torch.from_numpy(inputs.uniform(77, count, n)).to("cuda")
    # one stream with one launch outstanding: the burst queues behind a long
    # request (2^20 x 64, about half a millisecond) and is then batched
    blocker = torch.zeros((64, 1 << 20), dtype=torch.complex64, device="cuda")
    ptrs = [data[i].data_ptr() for i in range(count)]
    with sv.Server(hbm_budget=2 << 30, n_streams=1, max_inflight=1, max_coalesce=16) as srv:
        srv.prepare(n)
        srv.prepare(1 << 20)
        t_block = srv.submit(blocker, 1 << 20, 64)
        tickets = [srv.submit_ptr(p, n, 1) for p in ptrs]
        srv.wait(t_block)
        infos = [srv.wait(t) for t in tickets]
        groups = [i["group_size"] for i in infos]
        say(f"  group sizes {groups}")
        assert max(groups) > 1 and max(groups) <= 16
        ys = [srv.result(t)[0] for t in tickets]
        st = srv.stats()
        assert st["coalesced_requests"] > 0 and st["launches"] < count
    y = torch.cat(ys).cpu().numpy()
    metrics.check(y, oracle.fft(data.cpu().numpy().astype(np.complex128)), n)
    # a request above the budget is rejected, the next one is served
    with sv.Server(hbm_budget=1 << 20, arena_bytes=1 << 22) as srv:
        big = torch.zeros(1 << 16, dtype=torch.complex64, device="cuda")
        t_big = srv.submit(big, 1 << 16, 1)            # 1 MiB in + out + workspace > 1 MiB
        t_ok = srv.submit(data[0], n, 1)
        with pytest.raises(fb.FFTError) as ei:
            srv.wait(t_big)
        assert ei.value.status == 3                     # FFT_ERR_OUT_OF_MEMORY
        y, _ = srv.result(t_ok)
        metrics.check(y.cpu().numpy(), oracle.fft(data[0:1].cpu().numpy().astype(np.complex128)), n)
        assert srv.stats()["rejected"] == 1


def test_replay_short_poisson_stream_pooled_and_plain():
    t, nn, bb, sg = inputs.poisson_trace(4, 2000.0, 0.25, 8, 18, 64)
    trace = [{"t": float(t[i]), "n": int(nn[i]), "batch": int(bb[i]), "direction": int(sg[i])}
             for i in range(t.size)]
    pool_points = 1 << 25
    pool = torch.randn(pool_points, dtype=torch.complex64, device="cuda")
    offs = sv.trace_offsets(5, trace, pool_points)
    res = {}
    for name, kw in (("pooled", {}), ("plain", {"n_streams": 1, "max_inflight": 1, "max_coalesce": 1, "backfill_bytes": 0})):
        with sv.Server(hbm_budget=4 << 30, auto_release=True, **kw) as srv:
            for k in range(8, 19):
                srv.prepare(1 << k, -1)
                srv.prepare(1 << k, 1)
            st = sv.replay(srv, trace, pool, offs)
        say(f"  {name}: {st['completed']} requests, p50 {st['latency_p50']*1e3:.3f} ms, "
            f"p99 {st['latency_p99']*1e3:.3f} ms, launches {st['launches']}")
        assert st["completed"] == len(trace) and st["rejected"] == 0
        res[name] = st
    assert res["pooled"]["latency_p50"] > 0


def test_server_edge_lengths():
    # n = 1 (a copy), a mixed-radix length through its list kernel, the
    # longest four-step length with its workspace from the arena, and 32768
    # at a batch whose own plan would be a single block (served as the
    # server's batch-1 plan: four-step, workspace included)
    cases = [(1, 5, -1), (6000, 3, 1), (1 << 22, 2, -1), (3, 7, 1), (1 << 15, 80, 1)]
    data = [torch.from_numpy(inputs.uniform(3000 + i, b, n)).to("cuda") for i, (n, b, _) in enumerate(cases)]
    with sv.Server(hbm_budget=1 << 30) as srv:
        tickets = [srv.submit(data[i], n, b, d) for i, (n, b, d) in enumerate(cases)]
        for i, ((n, b, d), tk) in enumerate(zip(cases, tickets)):
            say(f"case: server edge n={n} batch={b} sign={d}")
            y, info = srv.result(tk)
            x = data[i].cpu().numpy().astype(np.complex128)
            if n == 1:
                assert np.array_equal(y.cpu().numpy().reshape(-1), data[i].cpu().numpy().reshape(-1))
            else:
                metrics.check(y.cpu().numpy(), oracle.fft(x, d), n)
            srv.release(tk)
        with pytest.raises(fb.FFTError):
            srv.release(tickets[0])                    # already released


def test_server_arena_backpressure_and_oversize():
    # 1 MiB arena: a request whose output can never fit is refused at submit;
    # unreleased outputs hold a later launch back until one is released
    n, b = 4096, 12                        # 384 KiB of output per request
    xs = [torch.from_numpy(inputs.uniform(4100 + i, b, n)).to("cuda") for i in range(3)]
    big = torch.from_numpy(inputs.uniform(4199, 4, 1 << 16)).to("cuda")
    say("case: server arena 1 MiB, three 384 KiB outputs and one 2 MiB output")
    with sv.Server(arena_bytes=1 << 20, hbm_budget=1 << 30, n_streams=2) as srv:
        with pytest.raises(fb.FFTError) as ei:
            srv.submit(big, 1 << 16, 4)
        assert ei.value.status == 3
        ta, tb = srv.submit(xs[0], n, b), srv.submit(xs[1], n, b)
        ya, _ = srv.result(ta)
        yb, _ = srv.result(tb)
        tc = srv.submit(xs[2], n, b)
        with pytest.raises(fb.FFTError) as ei:
            srv.wait(tc, timeout=0.5)          # 768 KiB held, 256 KiB free
        assert ei.value.status == 6
        srv.release(ta)
        yc, info = srv.result(tc)
        assert info["state"] == fb.REQ_DONE
        for x, y in ((xs[0], ya), (xs[1], yb), (xs[2], yc)):
            ref = oracle.fft(x.cpu().numpy().astype(np.complex128))
            metrics.check(y.cpu().numpy(), ref, n)
        srv.release(tb)
        srv.release(tc)


def test_served_stream_slice_sampled_against_oracle():
    # 0.1 s of the full serving stream (N = 2^8 ... 2^22, batch 1 ... 512, both
    # directions, 64 GiB budget, the default pooled server): the first
    # transform of every request against the oracle.  Outputs are read back
    # and released as requests complete, so the arena never fills.
    import collections
    import ctypes
    t, nn, bb, sg = inputs.poisson_trace(4, 2000.0, 0.1, 8, 22, 512)
    trace = [{"t": float(t[i]), "n": int(nn[i]), "batch": int(bb[i]), "direction": int(sg[i])}
             for i in range(t.size)]
    say(f"case: served stream slice, {len(trace)} requests")
    pool_points = (1 << 22) * 512
    pool = torch.empty(pool_points, dtype=torch.complex64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    pool.real.uniform_(-1.0, 1.0, generator=gen)
    pool.imag.uniform_(-1.0, 1.0, generator=gen)
    offs = sv.trace_offsets(5, trace, pool_points)
    lib = fb.load()
    got, pending = {}, collections.deque()
    with sv.Server(hbm_budget=64 << 30) as srv:
        def collect(block):
            while pending:
                i, tk = pending[0]
                out, info = ctypes.c_void_p(), fb.RequestInfo()
                st = lib.fft_server_wait(srv._h, tk, 60.0 if block else 0.0, ctypes.byref(out), ctypes.byref(info))
                if st == 6 and not block:
                    return
                fb._check(st, "fft_server_wait")
                n = trace[i]["n"]
                y = torch.empty(n, dtype=torch.complex64, device="cuda")
                fb._check(lib.fft_copy(out, ctypes.c_void_p(y.data_ptr()), n * 8, None), "fft_copy")
                torch.cuda.synchronize()
                got[i] = y.cpu().numpy()
                srv.release(tk)
                pending.popleft()

        # the arrival loop of serving.replay, without its final drain: the
        # outputs still held must be read and released first
        t0 = srv.clock()
        for i, r in enumerate(trace):
            while srv.clock() < t0 + r["t"]:
                pass
            pending.append((i, srv.submit_ptr(pool.data_ptr() + 8 * offs[i], r["n"], r["batch"], r["direction"])))
            collect(False)
        collect(True)
    assert len(got) == len(trace)
    for i, r in enumerate(trace):
        n = r["n"]
        x = pool[offs[i]:offs[i] + n].cpu().numpy().astype(np.complex128)[None, :]
        metrics.check(got[i][None, :], oracle.fft(x, r["direction"]), n)
