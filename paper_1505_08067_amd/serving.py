"""Python side of the serving layer (``fft_sched_*`` and ``fft_server_*``).

* ``Scheduler`` -- the host-only scheduler; every call takes the time, so a
  trace can be replayed on a simulated clock (``simulate``).
* ``Server`` -- the GPU server: a dispatcher thread, a stream pool, an HBM
  arena for outputs and workspaces, resident plans.
* ``replay`` -- submit an arrival trace to a ``Server`` in real time and
  return its latency and throughput statistics.

Admission, stream choice and continuous batching are the scheduler's (see
``include/fftblock.h``); this module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import time

from . import fftblock as fb


def sched_opts(hbm_budget=64 << 30, n_streams=4, max_inflight=2, max_coalesce=32, max_transforms=16384,
               backfill_bytes=1 << 30, small_streams=1, small_bytes=64 << 20):
    o = fb.SchedOpts()
    fb.load().fft_sched_opts_init(ctypes.byref(o))
    o.hbm_budget, o.n_streams, o.max_inflight = int(hbm_budget), int(n_streams), int(max_inflight)
    o.max_coalesce, o.max_transforms = int(max_coalesce), int(max_transforms)
    o.backfill_bytes = int(backfill_bytes)
    o.small_streams, o.small_bytes = int(small_streams), int(small_bytes)
    return o


def request_bytes(n: int, batch: int) -> int:
    """Budget bytes the server charges a request: input and output, plus the
    workspace on the four-step path."""
    four = fb.plan_query(n, batch)["path"] == fb.PATH_FOURSTEP
    return n * batch * 8 * (3 if four else 2)


class Scheduler:
    def __init__(self, **kw):
        self._o = sched_opts(**kw)
        h = ctypes.c_void_p()
        fb._check(fb.load().fft_sched_create(ctypes.byref(self._o), ctypes.byref(h)), "fft_sched_create")
        self._h = h

    def submit(self, rid: int, n: int, batch: int, direction: int, nbytes: int, coalescible: bool, now: float):
        fb._check(fb.load().fft_sched_submit(self._h, rid, n, batch, direction, nbytes, 1 if coalescible else 0,
                                             now), "fft_sched_submit")

    def next(self, now: float):
        L, got = fb.Launch(), ctypes.c_int()
        fb._check(fb.load().fft_sched_next(self._h, now, ctypes.byref(L), ctypes.byref(got)), "fft_sched_next")
        if not got.value:
            return None
        d = fb._struct_dict(L)
        d["requests"] = d["requests"][:L.n_requests]
        return d

    def complete(self, launch_id: int, now: float):
        fb._check(fb.load().fft_sched_complete(self._h, launch_id, now), "fft_sched_complete")

    def request(self, rid: int) -> dict:
        r = fb.RequestInfo()
        fb._check(fb.load().fft_sched_request(self._h, rid, ctypes.byref(r)), "fft_sched_request")
        return fb._struct_dict(r)

    def stats(self) -> dict:
        st = fb.SchedStats()
        fb._check(fb.load().fft_sched_stats(self._h, ctypes.byref(st)), "fft_sched_stats")
        return fb._struct_dict(st)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            fb._check(fb.load().fft_sched_destroy(self._h), "fft_sched_destroy")
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(sched: Scheduler, trace, duration_of, on_launch=None):
    """Replay ``trace`` (list of dicts with ``t, n, batch, direction``; ids are
    the list positions) through ``sched`` on a virtual clock.  A launch issued
    at time t on stream s starts when the stream is free (launches on one
    stream run in order) and lasts ``duration_of(launch)`` seconds;
    ``on_launch(launch)`` is called at issue (a simulated executor).  Returns
    the scheduler's statistics."""
    import heapq
    events = []            # (t_done, launch_id)
    stream_free = {}
    i = 0
    now = 0.0
    while i < len(trace) or events:
        t_next_arrival = trace[i]["t"] if i < len(trace) else float("inf")
        t_next_done = events[0][0] if events else float("inf")
        if t_next_arrival <= t_next_done:
            now = t_next_arrival
            r = trace[i]
            sched.submit(i, r["n"], r["batch"], r["direction"], r["bytes"], r.get("coalescible", True), now)
            i += 1
        else:
            now, lid = heapq.heappop(events)
            sched.complete(lid, now)
        while True:
            L = sched.next(now)
            if L is None:
                break
            if on_launch is not None:
                on_launch(L)
            start = max(now, stream_free.get(L["stream"], 0.0))
            done = start + duration_of(L)
            stream_free[L["stream"]] = done
            heapq.heappush(events, (done, L["id"]))
    return sched.stats()


class Server:
    """GPU server (``fft_server_*``) on the current device."""

    def __init__(self, arena_bytes: int = 0, auto_release: bool = False, **sched_kw):
        o = fb.ServerOpts()
        lib = fb.load()
        lib.fft_server_opts_init(ctypes.byref(o))
        o.sched = sched_opts(**sched_kw)
        o.arena_bytes = int(arena_bytes)
        o.auto_release = 1 if auto_release else 0
        h = ctypes.c_void_p()
        fb._check(lib.fft_server_create(ctypes.byref(o), ctypes.byref(h)), "fft_server_create")
        self._h = h

    def prepare(self, n: int, direction: int = fb.FORWARD):
        fb._check(fb.load().fft_server_prepare(self._h, n, direction), f"fft_server_prepare({n})")

    def submit_ptr(self, ptr: int, n: int, batch: int, direction: int = fb.FORWARD, stream=None) -> int:
        """Queue batch transforms of length n at device pointer ``ptr``.  The
        server's launch waits for the work queued on ``stream`` (a raw
        hipStream_t handle; None = torch's current stream) before the call."""
        import torch
        sh = torch.cuda.current_stream().cuda_stream if stream is None else stream
        t = ctypes.c_uint64()
        fb._check(fb.load().fft_server_submit(self._h, n, batch, direction, ctypes.c_void_p(ptr),
                                              ctypes.c_void_p(sh), ctypes.byref(t)), "fft_server_submit")
        return t.value

    def submit(self, x, n: int, batch: int, direction: int = fb.FORWARD) -> int:
        """Queue the transform of ``x`` (complex64 CUDA tensor of batch*n values,
        kept alive and unchanged by the caller until the request completes).
        The work torch has queued on its current stream (what writes ``x``)
        completes before the server reads it."""
        fb._check_tensor(x, "x")
        if x.numel() != n * batch:
            raise ValueError("x has the wrong size")
        return self.submit_ptr(x.data_ptr(), n, batch, direction)

    def wait(self, ticket: int, timeout: float = 60.0) -> dict:
        info, out = fb.RequestInfo(), ctypes.c_void_p()
        fb._check(fb.load().fft_server_wait(self._h, ticket, timeout, ctypes.byref(out), ctypes.byref(info)),
                  "fft_server_wait")
        return fb._struct_dict(info)

    def result(self, ticket: int, timeout: float = 60.0):
        """Wait for the request and return a copy of its output (complex64, [batch, n])."""
        import torch
        info = self.wait(ticket, timeout)
        out = torch.empty((info["batch"], info["n"]), dtype=torch.complex64, device="cuda")
        s = torch.cuda.current_stream()
        fb._check(fb.load().fft_server_read(self._h, ticket, ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(s.cuda_stream)), "fft_server_read")
        s.synchronize()
        return out, info

    def release(self, ticket: int):
        fb._check(fb.load().fft_server_release(self._h, ticket), "fft_server_release")

    def drain(self, timeout: float = 600.0):
        fb._check(fb.load().fft_server_drain(self._h, timeout), "fft_server_drain")

    def stats(self) -> dict:
        st = fb.SchedStats()
        fb._check(fb.load().fft_server_stats(self._h, ctypes.byref(st)), "fft_server_stats")
        return fb._struct_dict(st)

    def clock(self) -> float:
        return fb.load().fft_server_clock(self._h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            fb._check(fb.load().fft_server_destroy(self._h), "fft_server_destroy")
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server: Server, trace, pool, offsets, on_submit=None) -> dict:
    """Submit ``trace`` to ``server`` at its arrival times (seconds from now):
    request i transforms ``batch*n`` values of ``pool`` (a complex64 CUDA
    tensor) from element ``offsets[i]``.  Returns the server statistics after
    the last request completed, plus the wall time of the replay."""
    base = pool.data_ptr()
    t0 = server.clock()
    tickets = []
    for i, r in enumerate(trace):
        target = t0 + r["t"]
        while server.clock() < target:
            pass
        tk = server.submit_ptr(base + 8 * int(offsets[i]), r["n"], r["batch"], r["direction"])
        tickets.append(tk)
        if on_submit is not None:
            on_submit(i, tk)
    server.drain()
    st = server.stats()
    st["wall"] = server.clock() - t0
    st["tickets"] = tickets
    return st


def trace_offsets(seed: int, trace, pool_points: int, align: int = 64):
    """Seeded start offsets of each request's input inside a pool."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for r in trace:
        span = pool_points - r["n"] * r["batch"]
        if span < 0:
            raise ValueError("pool smaller than a request")
        out.append(int(rng.integers(0, span // align + 1)) * align)
    return out
