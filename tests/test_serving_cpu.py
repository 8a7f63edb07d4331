"""The serving scheduler on the CPU: admission under the budget, FIFO order,
stream choice, continuous batching and latency accounting, driven on a
virtual clock by a simulated executor (oracle-backed for the data)."""
import numpy as np
import pytest

import oracle
from paper_1505_08067_amd import fftblock as fb
from paper_1505_08067_amd import inputs
from paper_1505_08067_amd import serving as sv

F, B = fb.FORWARD, fb.BACKWARD


def test_options_are_checked():
    for kw in ({"hbm_budget": 0}, {"n_streams": 0}, {"n_streams": 17}, {"max_inflight": 0},
               {"max_coalesce": 0}, {"max_coalesce": 65}, {"max_transforms": 0}):
        with pytest.raises(fb.FFTError) as ei:
            sv.Scheduler(**kw)
        assert ei.value.status == 1, kw


def test_fifo_admission_under_budget_without_bypass():
    with sv.Scheduler(hbm_budget=1000, n_streams=4, max_inflight=4, max_coalesce=1, backfill_bytes=0) as s:
        s.submit(1, 64, 1, F, 600, False, 0.0)
        s.submit(2, 128, 1, F, 600, False, 0.1)
        s.submit(3, 256, 1, F, 300, False, 0.2)
        a = s.next(0.3)
        assert a["requests"] == [1]
        # 2 does not fit next to 1; 3 would, but must not overtake 2
        assert s.next(0.3) is None
        s.complete(a["id"], 1.0)
        b = s.next(1.0)
        assert b["requests"] == [2]
        c = s.next(1.0)
        assert c["requests"] == [3]
        st = s.stats()
        assert st["inflight_bytes"] == 900 and st["peak_inflight_bytes"] == 900
        s.complete(c["id"], 1.5)
        s.complete(b["id"], 2.0)
        st = s.stats()
        assert st["completed"] == 3 and st["inflight_bytes"] == 0
        lat = sorted([1.0, 2.0 - 0.1, 1.5 - 0.2])
        assert st["latency_p50"] == pytest.approx(lat[1]) and st["latency_max"] == pytest.approx(lat[2])
        # queue: launch - arrival (0.3, 0.9, 0.8); device: completion - launch (0.7, 1.0, 0.5)
        assert st["queue_p50"] == pytest.approx(0.8) and st["queue_p99"] == pytest.approx(0.9)
        assert st["device_p50"] == pytest.approx(0.7) and st["device_p99"] == pytest.approx(1.0)
        assert s.request(2)["t_launch"] == pytest.approx(1.0) and s.request(2)["state"] == fb.REQ_DONE


def test_bounded_backfill_past_a_waiting_head():
    # budget 1000, backfill 250: while the 600-byte head waits, requests of at
    # most 250 bytes pass it, with at most 250 bytes of them in flight
    with sv.Scheduler(hbm_budget=1000, n_streams=4, max_inflight=8, max_coalesce=1, backfill_bytes=250) as s:
        s.submit(1, 64, 1, F, 600, False, 0.0)
        s.submit(2, 128, 1, F, 600, False, 0.1)     # waits behind 1
        s.submit(3, 256, 1, F, 300, False, 0.2)     # too large to pass
        s.submit(4, 512, 1, F, 200, False, 0.3)     # passes
        s.submit(5, 1024, 1, F, 100, False, 0.4)    # would exceed 250 in flight by backfill
        a = s.next(0.5)
        assert a["requests"] == [1]
        b = s.next(0.5)
        assert b["requests"] == [4]
        assert s.next(0.5) is None
        assert s.request(4)["state"] == fb.REQ_RUNNING and s.request(2)["state"] == fb.REQ_QUEUED
        s.complete(b["id"], 0.6)
        c = s.next(0.6)
        assert c["requests"] == [5]                 # backfill room again
        s.complete(a["id"], 1.0)
        d = s.next(1.0)
        assert d["requests"] == [2]                 # the head goes first once it fits
        st = s.stats()
        assert st["backfilled_requests"] == 2


def test_backfill_never_starves_a_large_head():
    # budget 1000, backfill 500, a head of 800 bytes: backfill in flight is
    # capped at 1000 - 800 = 200, so a continuous stream of small requests
    # cannot keep the head out once the request launched before it completes
    with sv.Scheduler(hbm_budget=1000, n_streams=4, max_inflight=64, max_coalesce=1, backfill_bytes=500) as s:
        s.submit(1, 64, 1, F, 300, False, 0.0)
        a = s.next(0.0)
        assert a["requests"] == [1]
        s.submit(2, 128, 1, F, 800, False, 0.0)     # the head: waits behind 1
        running, rid, t = [], 100, 0.0
        for step in range(40):
            t += 0.01
            for _ in range(3):                      # small requests keep arriving
                s.submit(rid, 256, 1, F, 100, False, t)
                rid += 1
            while True:
                L = s.next(t)
                if L is None:
                    break
                if L["requests"] == [2]:
                    break
                running.append(L)
            assert sum(r["bytes"] for r in running) <= 200   # never more backfill than the head leaves
            if L is not None and L["requests"] == [2]:
                break
            if running:                              # the oldest backfill completes
                s.complete(running.pop(0)["id"], t)
            if step == 10:
                s.complete(a["id"], t)               # the work ahead of the head completes
        assert s.request(2)["state"] == fb.REQ_RUNNING
        assert s.request(2)["t_launch"] <= 0.13


def test_oversized_request_is_rejected_and_others_proceed():
    with sv.Scheduler(hbm_budget=1000) as s:
        s.submit(1, 64, 1, F, 5000, True, 0.0)
        s.submit(2, 64, 1, F, 100, True, 0.0)
        L = s.next(0.5)
        assert L["requests"] == [2]
        assert s.request(1)["state"] == fb.REQ_REJECTED
        assert s.stats()["rejected"] == 1
    with pytest.raises(fb.FFTError):
        with sv.Scheduler() as s:
            s.submit(7, 64, 1, F, 10, True, 0.0)
            s.submit(7, 64, 1, F, 10, True, 0.0)      # duplicate id


def test_stream_choice_and_inflight_cap():
    with sv.Scheduler(hbm_budget=1 << 30, n_streams=2, max_inflight=1, max_coalesce=1, small_streams=0) as s:
        for i, nb in enumerate((500, 100, 100)):
            s.submit(i, 64 << i, 1, F, nb, False, 0.0)
        a, b = s.next(0.0), s.next(0.0)
        assert (a["stream"], b["stream"]) == (0, 1)
        assert s.next(0.0) is None                    # both streams at their cap
        s.complete(a["id"], 1.0)
        c = s.next(1.0)
        assert c["stream"] == 0 and c["requests"] == [2]
    with sv.Scheduler(hbm_budget=1 << 30, n_streams=2, max_inflight=2, max_coalesce=1, small_streams=0) as s:
        for i, nb in enumerate((500, 100, 100)):
            s.submit(i, 64 << i, 1, F, nb, False, 0.0)
        got = [s.next(0.0) for _ in range(3)]
        # least outstanding bytes: 0 -> s0 (500), 1 -> s1 (100), 2 -> s1 (200 < 500)
        assert [g["stream"] for g in got] == [0, 1, 1]


def test_small_request_lane():
    # stream 0 takes only launches led by requests of at most small_bytes;
    # larger ones use streams 1..n-1; a small launch falls back to any stream
    # when the lane is full
    kw = dict(hbm_budget=1 << 30, max_inflight=1, max_coalesce=1, small_streams=1, small_bytes=100)
    with sv.Scheduler(n_streams=3, **kw) as s:
        for i, nb in enumerate((500, 50, 600, 60, 70)):
            s.submit(i, 64 << i, 1, F, nb, False, 0.0)
        a, b, c = s.next(0.0), s.next(0.0), s.next(0.0)
        assert (a["requests"], a["stream"]) == ([0], 1)
        assert (b["requests"], b["stream"]) == ([1], 0)
        assert (c["requests"], c["stream"]) == ([2], 2)
        assert s.next(0.0) is None                    # every stream at its cap
        s.complete(b["id"], 1.0)
        d = s.next(1.0)
        assert (d["requests"], d["stream"]) == ([3], 0)
        s.complete(a["id"], 1.0)
        e = s.next(1.0)
        assert (e["requests"], e["stream"]) == ([4], 1)   # lane full: any stream
    # a large head never takes the lane
    with sv.Scheduler(n_streams=2, **kw) as s:
        s.submit(0, 64, 1, F, 500, False, 0.0)
        s.submit(1, 128, 1, F, 500, False, 0.0)
        assert s.next(0.0)["stream"] == 1
        assert s.next(0.0) is None
    # one stream: no lane
    with sv.Scheduler(n_streams=1, **kw) as s:
        s.submit(0, 64, 1, F, 500, False, 0.0)
        assert s.next(0.0)["stream"] == 0
    with pytest.raises(fb.FFTError):
        sv.Scheduler(small_streams=-1)


def test_continuous_batching_groups_same_length_and_direction():
    with sv.Scheduler(hbm_budget=1 << 30, n_streams=1, max_inflight=1, max_coalesce=3, max_transforms=10) as s:
        s.submit(0, 1024, 1, F, 16, True, 0.0)
        first = s.next(0.0)                           # occupies the only slot
        reqs = [(1, 1024, 2, F), (2, 512, 1, F), (3, 1024, 3, B), (4, 1024, 4, F), (5, 1024, 1, F),
                (6, 1024, 1, F), (7, 1024, 9, F)]
        for rid, n, b, d in reqs:
            s.submit(rid, n, b, d, 16 * n * b, True, 0.1)
        s.complete(first["id"], 1.0)
        L = s.next(1.0)
        # head 1 (F, 1024) gathers 4 and 5 (3 requests max); 2 and 3 differ
        assert L["requests"] == [1, 4, 5] and L["batch"] == 7 and L["n"] == 1024
        assert all(s.request(r)["group_size"] == 3 for r in (1, 4, 5))
        s.complete(L["id"], 2.0)
        assert s.next(2.0)["requests"] == [2]
    with sv.Scheduler(hbm_budget=1 << 30, n_streams=1, max_inflight=1, max_coalesce=8, max_transforms=10) as s:
        s.submit(0, 64, 1, F, 16, True, 0.0)
        first = s.next(0.0)
        for rid, b in ((1, 6), (2, 5), (3, 4)):
            s.submit(rid, 1024, b, F, 16, True, 0.1)
        s.submit(4, 1024, 1, F, 16, False, 0.1)       # four-step-like: never coalesced
        s.complete(first["id"], 1.0)
        L = s.next(1.0)
        assert L["requests"] == [1, 3] and L["batch"] == 10      # 6 + 5 > 10, 6 + 4 fits
        s.complete(L["id"], 2.0)
        assert s.next(2.0)["requests"] == [2]


def _cfg5_trace(seed, duration, k_hi=22, max_batch=512):
    t, n, b, sign = inputs.poisson_trace(seed, 2000.0, duration, 8, k_hi, max_batch)
    out = []
    for i in range(t.size):
        nn, bb = int(n[i]), int(b[i])
        four = nn > 16384
        out.append({"t": float(t[i]), "n": nn, "batch": bb, "direction": int(sign[i]),
                    "bytes": nn * bb * 8 * (3 if four else 2), "coalescible": not four})
    return out


def _duration(L):
    # executor model: 5 us launch cost plus the bytes at 5 TB/s
    return 5e-6 + 16.0 * L["n"] * L["batch"] * (2 if L["n"] > 16384 else 1) / 5e12


def test_simulated_cfg5_trace_accounting():
    trace = _cfg5_trace(4, 1.0)
    budget = 64 << 30
    seen = {}

    def on_launch(L):
        assert L["bytes"] <= budget
        for r in L["requests"]:
            assert r not in seen
            seen[r] = L["id"]
            assert trace[r]["n"] == L["n"] and trace[r]["direction"] == L["direction"]

    with sv.Scheduler(hbm_budget=budget) as s:
        st = sv.simulate(s, trace, _duration, on_launch)
        assert st["completed"] == len(trace) and st["rejected"] == 0 and len(seen) == len(trace)
        assert st["peak_inflight_bytes"] <= budget and st["inflight_bytes"] == 0
        lat = np.array([s.request(i)["t_done"] - trace[i]["t"] for i in range(len(trace))])
        k = lambda p: np.sort(lat)[int(np.ceil(p * lat.size)) - 1]   # nearest rank
        assert st["latency_p50"] == pytest.approx(k(0.5)) and st["latency_p99"] == pytest.approx(k(0.99))
        q = np.array([s.request(i)["t_launch"] - trace[i]["t"] for i in range(len(trace))])
        d = np.array([s.request(i)["t_done"] - s.request(i)["t_launch"] for i in range(len(trace))])
        kq = lambda p: np.sort(q)[int(np.ceil(p * q.size)) - 1]
        kd = lambda p: np.sort(d)[int(np.ceil(p * d.size)) - 1]
        assert st["queue_p50"] == pytest.approx(kq(0.5)) and st["queue_p99"] == pytest.approx(kq(0.99))
        assert st["device_p50"] == pytest.approx(kd(0.5)) and st["device_p99"] == pytest.approx(kd(0.99))
        assert st["points"] == pytest.approx(sum(r["n"] * r["batch"] for r in trace))
    # the plain path (one stream, one launch at a time, no batching) is never faster at p99
    with sv.Scheduler(hbm_budget=budget, n_streams=1, max_inflight=1, max_coalesce=1, backfill_bytes=0) as s:
        plain = sv.simulate(s, trace, _duration)
    assert plain["completed"] == len(trace) and plain["coalesced_requests"] == 0
    assert st["latency_p99"] <= plain["latency_p99"] * (1 + 1e-9)


def test_oracle_backed_executor_alone_equals_in_mix():
    # small requests with data: the simulated executor computes each launch's
    # requests with the oracle; every request is computed exactly once, and its
    # result in the mix equals the result of the same request served alone
    rng = np.random.default_rng(5)
    trace, data = [], []
    t = 0.0
    for i in range(60):
        n = int(rng.choice([8, 16, 64, 100]))
        b = int(rng.integers(1, 5))
        t += float(rng.exponential(1e-5))
        trace.append({"t": t, "n": n, "batch": b, "direction": int(rng.choice([F, B])),
                      "bytes": 16 * n * b, "coalescible": True})
        data.append(inputs.uniform(1000 + i, b, n))
    def executor(ids, results):
        # ids: scheduler request id -> index of the request's data
        def execute(L):
            for r in L["requests"]:
                assert r not in results
                results[r] = oracle.fft(data[ids[r]].astype(np.complex128), L["direction"])
        return execute

    mix = {}
    with sv.Scheduler(hbm_budget=1 << 20, n_streams=2, max_inflight=1, max_coalesce=8) as s:
        st = sv.simulate(s, trace, lambda L: 2e-5, executor(list(range(len(trace))), mix))
    assert st["completed"] == len(trace) and st["coalesced_requests"] > 0 and len(mix) == len(trace)
    for i in (0, 17, 59):
        alone = {}
        with sv.Scheduler(hbm_budget=1 << 20) as s:
            sv.simulate(s, [dict(trace[i], t=0.0)], lambda L: 2e-5, executor([i], alone))
        assert np.array_equal(alone[0], mix[i])
        assert np.array_equal(mix[i], oracle.fft(data[i].astype(np.complex128), trace[i]["direction"]))
