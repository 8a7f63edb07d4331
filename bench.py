#!/usr/bin/env python3
"""Throughput benchmark of the batched complex64 FFT path on one MI355X.

One step = one pass of the hot path over the plain workload:
  * N = 4096, batch 4096, forward and inverse (single LDS-resident block);
  * N = 2^20, batch 16, forward and inverse (four-step N1 x N2 as planned:
    column block FFTs + twiddle, then row block FFTs + corner-turn store).
Inputs are seeded uniform[-1,1] complex64, resident in HBM before timing;
every launch of the step (each direction of each shape) has its own (in, out)
buffer sets, rotated, so no buffer is reused within 1.75 GiB of traffic, beyond
the 256 MB Infinity Cache (cold-cache timing).

Metric: GFLOP/s counted as 5 N log2 N per transform, over the event-timed
steps.  Per-kernel durations come from the same steps run again with events
the device stamps at each dispatch's own start and end on the launch stream
(what a kernel trace reports); the dominant kernel's algorithmic HBM bytes (16 N per transform and
pass: the data read once and written once) over its average duration give
the roofline fraction against 8 TB/s.  The FP64 oracle is timed on the host
cores on the same step (CPU baseline).  Prints ONE JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "batched c64 FFT GFLOP/s (5Nlog2N) + % HBM peak; serving p50/p99 latency"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print("bench:", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=50, help="untimed steps after the settle phase")
    p.add_argument("--settle-ms", type=float, default=40.0,
                   help="untimed steps until this much device time has passed, before the warmup steps: "
                        "after an idle period the step time rises for 10-15 ms before it settles")
    p.add_argument("--rotate", type=int, default=2,
                   help="(in,out) buffer sets per launch of a step (every launch has its own sets)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0, help="target oracle time for the CPU baseline")
    p.add_argument("--no-extras", action="store_true", help="skip copy probe and SAR chain timing")
    p.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "hbm_traffic_n4096x4096_n2p20x16.md"),
                   help="rocprofv3 traffic summary (measured HBM bytes per launch per kernel)")
    p.add_argument("--no-serving", action="store_true", help="skip the serving stream (profiling runs)")
    p.add_argument("--extras", default=",".join(("copy", "small", "sar", "fp16", "ragged", "schedules", "lanes", "serving")),
                   help="comma list of extras to run: copy, small, sar, fp16, ragged, schedules, lanes, serving")
    p.add_argument("--calibrate", action="store_true",
                   help="also run the copy kernel on 256 MiB three times (counter calibration)")
    return p.parse_args()


def kernel_source_hash() -> str:
    """sha256 over the device code of the transform kernels (the kernel
    templates, their argument layout and the kernel catalogues): what the
    measured traffic figures depend on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1505_08067_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "kernels_*.hip")) +
                   [os.path.join(csrc, f) for f in ("fft_device.hpp", "fft_kernel.hpp", "internal.hpp")])
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path: str, kernel: str):
    """HBM bytes per launch of `kernel` from the traffic summary, or None.

    The summary lists `| kernel | ... | bytes_per_launch |` rows and a
    `source_hash:` line; the figure is used only when the kernel sources still
    hash to that value (a changed kernel makes the counters stale).
    """
    if not path or not os.path.exists(path):
        return None
    rows, src = {}, None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("source_hash:"):
                src = line.split(":", 1)[1].strip()
            elif line.startswith("|") and not line.startswith("|-"):
                cells = [c.strip() for c in line.strip("|").split("|")]
                if len(cells) >= 2 and cells[-1].replace(".", "", 1).isdigit():
                    rows[cells[0]] = float(cells[-1])
    if src != kernel_source_hash():
        return None
    return rows.get(kernel)


def flops(n, batch):
    return 5.0 * n * math.log2(n) * batch if n > 1 else 0.0


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only; the multi-GPU layout (batch sharding and an "
              "all-to-all corner turn) is a design note, not implemented. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1505_08067_amd import fftblock as fb
    from paper_1505_08067_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    fb.load()
    info = fb.device_query()
    log("device", info["arch"], "CUs", info["compute_units"], "LDS/CU", info["lds_per_cu"])

    # ------------------------------------------------------------ workload
    items = [
        ("block N=4096 fwd", 4096, 4096, fb.FORWARD),
        ("block N=4096 inv", 4096, 4096, fb.BACKWARD),
        ("fourstep N=2^20 fwd", 1 << 20, 16, fb.FORWARD),
        ("fourstep N=2^20 inv", 1 << 20, 16, fb.BACKWARD),
    ]
    plans = {}
    bufs = {}
    # Every item of the step (each direction of each shape) has its own
    # `rotate` (in, out) sets, so no launch reads what another launch of the
    # same step read or wrote: between two uses of one buffer the step moves
    # at least rotate * 4 * 256 MiB - 256 MiB >= 1.75 GiB, beyond the 256 MB
    # Infinity Cache and the 32 MB of L2.
    host_x = {}
    for name, n, batch, sign in items:
        plans[name] = fb.Plan(n, batch, sign)
        if (n, batch) not in host_x:
            host_x[(n, batch)] = torch.from_numpy(inputs.uniform(1, batch, n))
        x = host_x[(n, batch)].to("cuda")
        bufs[name] = [(x.clone(), torch.empty_like(x)) for _ in range(args.rotate)]
        del x
    del host_x
    torch.cuda.synchronize()

    # launches of one step: (kernel label, item, pass, shape)
    launches = []
    for name, n, batch, sign in items:
        d = plans[name].describe()
        launches.append((d["kernel_name"], name, 1, (n, batch)))
        if d["path"] != fb.PATH_BLOCK:
            launches.append((d["kernel_name2"], name, 2, (n, batch)))
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    d4 = plans["fourstep N=2^20 fwd"].describe()
    split = f"{d4['n1']}x{d4['n2']}"

    def run_step(s, evs=None):
        k = s % args.rotate
        for li, (_, name, pass_, _) in enumerate(launches):
            xin, xout = bufs[name][k]
            if evs is None or li not in evs:
                plans[name].execute_pass_ptr(pass_, xin.data_ptr(), xout.data_ptr(), sh)
            else:
                # the device stamps the pair at this dispatch's own start and end
                plans[name].execute_pass_timed_ptr(pass_, xin.data_ptr(), xout.data_ptr(), sh, *evs[li])

    # Settle phase.  Measured after an idle period: the first few steps take
    # ~297 us, steps 8-20 take 310-325 us, and from ~15 ms on the step stays
    # at ~295 us (the device's clock and power control reacting to the new
    # load).  A short warmup would put the timed region inside that
    # transient, so whole steps run, untimed, until settle_ms of device time
    # has passed; then come the W warmup steps and the K timed steps.
    settle_steps = 0
    settled_ms = 0.0
    if args.settle_ms > 0:
        # chunks of 10 steps, one always queued behind the one waited on, so
        # the device never idles
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        marks = []
        while True:
            for _ in range(10):
                run_step(settle_steps)
                settle_steps += 1
            marks.append(torch.cuda.Event(enable_timing=True))
            marks[-1].record(stream)
            if len(marks) >= 2:
                marks[-2].synchronize()
                if e0.elapsed_time(marks[-2]) >= args.settle_ms:
                    break
        torch.cuda.synchronize()
        settled_ms = e0.elapsed_time(marks[-1])
        log(f"settle: {settle_steps} steps, {settled_ms:.1f} ms")
    for s in range(args.warmup):
        run_step(s)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")

    # timed region: K steps between two events on the launch stream.  In
    # every step one launch, in turn, is dispatched with two events the device
    # stamps at the kernel's own start and end, so the per-kernel durations
    # are sampled from the timed launches themselves.  A stamped dispatch
    # leaves a gap of several microseconds before the next one, and a kernel
    # that starts after such a gap finds the previous kernel's stores drained
    # and runs faster than back to back; stamping one launch per step keeps
    # each stamped kernel's predecessor an ordinary launch.
    K = args.steps
    nl = len(launches)
    evs = {s: {s % nl: (fb.Event(), fb.Event())} for s in range(K)}
    for li in range(K, nl):  # fewer steps than launches: the last step stamps the rest
        evs[K - 1][li] = (fb.Event(), fb.Event())
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_start.record(stream)
    for s in range(K):
        run_step(s, evs.get(s))
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"timed {K} steps in {wall:.3f} s wall")
    ms_per_step = t_start.elapsed_time(t_end) / K

    # cross-check: the same K steps with ordinary launches (no stamps)
    torch.cuda.synchronize()
    t_start.record(stream)
    for s in range(K):
        run_step(s)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_per_step_plain = t_start.elapsed_time(t_end) / K
    log(f"step {ms_per_step * 1e3:.1f} us stamped, {ms_per_step_plain * 1e3:.1f} us with ordinary launches")
    per = {}
    for s in range(K):
        for li, (e0, e1) in evs[s].items():
            per.setdefault(li, []).append(e0.elapsed_ms(e1))
    for row in evs.values():
        for e0, e1 in row.values():
            e0.close()
            e1.close()
    fl_step = sum(flops(n, b) for _, n, b, _ in items)
    value = fl_step / (ms_per_step * 1e-3) / 1e9

    kernels = {}
    for li, (kname, name, pass_, (n, batch)) in enumerate(launches):
        avg_ms = sum(per[li]) / len(per[li])
        byts = 16.0 * n * batch
        e = kernels.setdefault(kname, {"launches_per_step": 0, "total_ms": 0.0, "bytes_per_launch": byts,
                                       "durations_ms": []})
        e["launches_per_step"] += 1
        e["total_ms"] += avg_ms
        e["durations_ms"].append(avg_ms)
    kinfo = {k["name"]: k for k in fb.kernels()}
    breakdown = {}
    for kname, e in kernels.items():
        avg = e["total_ms"] / e["launches_per_step"]
        gbps = e["bytes_per_launch"] / (avg * 1e-3) / 1e9
        occ = fb.kernel_occupancy(kname)
        durs = sorted(d for li, (k2, _, _, _) in enumerate(launches) if k2 == kname for d in per[li])
        breakdown[kname] = {"avg_us": round(avg * 1e3, 2), "median_us": round(durs[len(durs) // 2] * 1e3, 2),
                            "launches_per_step": e["launches_per_step"],
                            "bytes_per_launch": int(e["bytes_per_launch"]), "GBps": round(gbps, 1),
                            "frac_hbm_peak": round(gbps / HBM_PEAK_GBPS, 4),
                            "workgroups_per_cu": occ, "waves_per_simd": occ * kinfo[kname]["threads"] / 64 / 4,
                            "by_direction": {}}
    # the same rows split by direction (each launch has its own buffers)
    for li, (kname, name, pass_, (n, batch)) in enumerate(launches):
        d = sorted(per[li])
        avg = sum(d) / len(d)
        gbps = 16.0 * n * batch / (avg * 1e-3) / 1e9
        breakdown[kname]["by_direction"][name.rsplit(" ", 1)[1]] = {
            "launch": name + (f" pass {pass_}" if plans[name].describe()["path"] != fb.PATH_BLOCK else ""),
            "samples": len(d), "avg_us": round(avg * 1e3, 2), "median_us": round(d[len(d) // 2] * 1e3, 2),
            "GBps": round(gbps, 1), "frac_hbm_peak": round(gbps / HBM_PEAK_GBPS, 4)}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    dom_avg_ms = kernels[dom]["total_ms"] / kernels[dom]["launches_per_step"]
    achieved = kernels[dom]["bytes_per_launch"] / (dom_avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.traffic, dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic}
    log("per-kernel:", json.dumps(breakdown))

    extras = {}
    if not args.no_extras:
        which = set(t for t in args.extras.split(",") if t)
        if args.no_serving:
            which.discard("serving")
        extras = run_extras(torch, fb, inputs, stream, which)
    sat = (extras.get("serving") or {}).get("saturated") if isinstance(extras.get("serving"), dict) else None
    if isinstance(sat, dict) and sat.get("GFLOPs"):
        # the served mix at saturation against the uniform batches of the step
        sat["GFLOPs_over_uniform_step"] = round(sat["GFLOPs"] / value, 3)
    rg = extras.get("ragged")
    if isinstance(rg, dict) and rg.get("graph_GFLOPs"):
        # the ragged mix's throughput against the uniform batches of the step
        rg["graph_GFLOPs_over_uniform_step"] = round(rg["graph_GFLOPs"] / value, 3)
    cp = extras.get("copy_probe")
    if isinstance(cp, dict) and cp.get("GBps_read_plus_write"):
        # the same kernels against what a plain copy reaches on this device
        for row in breakdown.values():
            row["frac_copy_peak"] = round(row["GBps"] / cp["GBps_read_plus_write"], 4)
        roofline["frac_copy_peak"] = round(achieved / cp["GBps_read_plus_write"], 4)
    if args.calibrate:
        src = torch.empty((1 << 28) // 8, dtype=torch.complex64, device="cuda")
        dst = torch.empty_like(src)
        src.zero_()
        for _ in range(3):
            fb.copy_(dst, src)
        torch.cuda.synchronize()
        del src, dst

    # ------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        # the GPU's outputs of the same inputs, compared with the oracle's
        outs = {}
        for name, n, batch, sign in items:
            xin = bufs[name][0][0]
            outs[name] = plans[name].execute(xin).cpu().numpy().reshape(batch, n)
        cpu = cpu_baseline(items, fl_step, args.cpu_seconds, outs)
        del outs

    rec = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "settle_ms": round(settled_ms, 1),
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched complex64 FFT, N=4096 x batch 4096 forward+inverse (single LDS block) "
                        f"+ N=2^20 x batch 16 forward+inverse (four-step {split})",
            "inputs": "uniform[-1,1] re/im, seed 1",
            "buffer_sets_per_launch": args.rotate,
            "flops_per_step": fl_step,
            "hbm_bytes_per_step": int(sum(16.0 * n * b for _, _, _, (n, b) in launches)),
            "device": info["arch"],
            "kernel_source_hash": kernel_source_hash(),
            "ms_per_step_unstamped_launches": round(ms_per_step_plain, 5),
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": breakdown,
        "extras": extras,
    }
    print(json.dumps(rec), flush=True)
    for p in plans.values():
        p.close()


EXTRAS = ("copy", "small", "sar", "fp16", "ragged", "schedules", "lanes", "serving")


def run_extras(torch, fb, inputs, stream, which=EXTRAS):
    out = {}
    todo = [("copy_probe", "copy", lambda: run_copy(torch, fb, stream)),
            ("fourstep_1024x1024", "copy", lambda: run_split(torch, fb, inputs, stream)),
            ("small_batches", "small", lambda: run_small(torch, fb, inputs, stream)),
            ("sar", "sar", lambda: run_sar(torch, fb, inputs, stream)),
            ("fp16_storage", "fp16", lambda: run_fp16(torch, fb, inputs, stream)),
            ("ragged", "ragged", lambda: run_ragged(torch, fb, inputs, stream)),
            ("schedule_model", "schedules", lambda: run_schedule_model(torch, fb, stream)),
            ("lanes", "lanes", lambda: run_lanes(torch, fb, stream)),
            ("serving", "serving", lambda: run_serving(torch, fb, inputs))]
    for key, tag, fn in todo:
        if tag not in which:
            continue
        try:
            res = fn()
        except (fb.FFTError, RuntimeError, ValueError) as e:
            # a failed extra is reported, not fatal to the headline line
            res = {"error": f"{type(e).__name__}: {e}"}
            log(f"{key} failed: {type(e).__name__}: {e}")
            torch.cuda.synchronize()
        if key == "sar" and "error" not in res:
            out.update(res)
        else:
            out[key] = res
    return out


def run_split(torch, fb, inputs, stream):
    """N = 2^20 x 16 forward + inverse at the balanced split 1024 x 1024 (the
    planner's default is measured faster and is what the step uses)."""
    n, batch = 1 << 20, 16
    sets = [(torch.from_numpy(inputs.uniform(1, batch, n)).to("cuda"), None) for _ in range(1)]
    x = sets[0][0]
    xs = [x.clone() for _ in range(4)]
    ys = [torch.empty_like(x) for _ in range(4)]
    sh = stream.cuda_stream
    res = {}
    for name, n1 in (("balanced", 1024), ("planner", 0)):
        with fb.Plan(n, batch, fb.FORWARD, fb.make_opts(n1=n1)) as pf, \
                fb.Plan(n, batch, fb.BACKWARD, fb.make_opts(n1=n1)) as pb:
            d = pf.describe()
            k = [0]

            def step():
                i = k[0] % 4
                k[0] += 1
                pf.execute_ptr(xs[i].data_ptr(), ys[i].data_ptr(), sh)
                pb.execute_ptr(xs[i].data_ptr(), ys[i].data_ptr(), sh)
            t = _timed(torch, stream, step, reps=20)
        res[name] = {"split": f"{d['n1']}x{d['n2']}", "kernels": [d["kernel_name"], d["kernel_name2"]],
                     "us_fwd_plus_inv": round(t * 1e6, 1),
                     "GFLOPs": round(2 * 5.0 * n * 20 * batch / t / 1e9, 1),
                     "frac_hbm_peak": round(2 * 32.0 * n * batch / t / 1e9 / HBM_PEAK_GBPS, 4)}
    del xs, ys, x
    log("four-step splits", json.dumps(res))
    return res


def run_copy(torch, fb, stream):
    """HBM copy probe: 1 GiB, read + write counted."""
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    a.zero_()
    for _ in range(3):
        fb.copy_(b, a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record(stream)
    for _ in range(reps):
        fb.copy_(b, a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    res = {"bytes": nbytes, "GBps_read_plus_write": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}
    del a, b
    log("copy probe", res)
    return res


def run_sar(torch, fb, inputs, stream):
    """The radar chain on 4096 pulses x 8192 range samples, and range compression."""
    out = {}
    # SAR chain: range FFT (8192 x 4096) -> corner turn -> azimuth FFT (4096 x 8192), and back
    P, R = 4096, 8192
    x = torch.from_numpy(inputs.sar(2, pulses=P, ranges=R)).to("cuda")
    rf, af = fb.Plan(R, P, fb.FORWARD), fb.Plan(P, R, fb.FORWARD)
    ab, rb = fb.Plan(P, R, fb.BACKWARD), fb.Plan(R, P, fb.BACKWARD)
    t1, t2, t3 = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    sh = stream.cuda_stream
    steps = [("range_fft", lambda: rf.execute_ptr(x.data_ptr(), t1.data_ptr(), sh)),
             ("corner_turn", lambda: fb.transpose(t1.view(P, R), out=t2.view(R, P))),
             ("azimuth_fft", lambda: af.execute_ptr(t2.data_ptr(), t3.data_ptr(), sh)),
             ("azimuth_ifft", lambda: ab.execute_ptr(t3.data_ptr(), t2.data_ptr(), sh)),
             ("corner_turn_back", lambda: fb.transpose(t2.view(R, P), out=t1.view(P, R))),
             ("range_ifft", lambda: rb.execute_ptr(t1.data_ptr(), t3.data_ptr(), sh))]
    for _ in range(2):
        for _, f in steps:
            f()
    torch.cuda.synchronize()
    reps = 10
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(steps) + 1)] for _ in range(reps)]
    for r in range(reps):
        for i, (_, f) in enumerate(steps):
            evs[r][i].record(stream)
            f()
        evs[r][len(steps)].record(stream)
    torch.cuda.synchronize()
    pts = P * R
    sar = {}
    for i, (name, _) in enumerate(steps):
        ms = sum(evs[r][i].elapsed_time(evs[r][i + 1]) for r in range(reps)) / reps
        sar[name] = {"us": round(ms * 1e3, 1), "GBps": round(16.0 * pts / (ms * 1e-3) / 1e9, 1)}
    fwd_ms = sum(sar[k]["us"] for k in ("range_fft", "corner_turn", "azimuth_fft")) / 1e3
    inv_ms = sum(sar[k]["us"] for k in ("azimuth_ifft", "corner_turn_back", "range_ifft")) / 1e3
    fl = 5.0 * pts * math.log2(pts)
    sar["forward_GFLOPs"] = round(fl / (fwd_ms * 1e-3) / 1e9, 1)
    sar["inverse_GFLOPs"] = round(fl / (inv_ms * 1e-3) / 1e9, 1)
    sar["forward_frac_hbm_at_48B_per_point"] = round(48.0 * pts / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
    sar["shape"] = f"{P} pulses x {R} range samples"
    out["sar_chain"] = sar
    # range compression (matched filter), fused into one pass over the rows,
    # then the corner turn and the azimuth FFT: the compressed forward chain
    rep = torch.from_numpy(inputs.sar_replica()).to("cuda")
    with fb.RangeCompressor(R, P, rep) as rc:
        kname = rc.describe()["kernel_name"]
        chain = [("range_compress", lambda: rc.execute_ptr(x.data_ptr(), t1.data_ptr(), sh)),
                 ("corner_turn", lambda: fb.transpose(t1.view(P, R), out=t2.view(R, P))),
                 ("azimuth_fft", lambda: af.execute_ptr(t2.data_ptr(), t3.data_ptr(), sh))]
        for _ in range(2):
            for _, f in chain:
                f()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(chain) + 1)] for _ in range(reps)]
        for r in range(reps):
            for i, (_, f) in enumerate(chain):
                evs[r][i].record(stream)
                f()
            evs[r][len(chain)].record(stream)
        torch.cuda.synchronize()
    comp = {"kernel": kname}
    for i, (name, _) in enumerate(chain):
        ms = sum(evs[r][i].elapsed_time(evs[r][i + 1]) for r in range(reps)) / reps
        comp[name] = {"us": round(ms * 1e3, 1), "GBps": round(16.0 * pts / (ms * 1e-3) / 1e9, 1),
                      "frac_hbm_peak": round(16.0 * pts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    rc_s = comp["range_compress"]["us"] * 1e-6
    # two transforms per row (forward and backward) plus the product
    comp["range_compress"]["GFLOPs"] = round(2 * 5.0 * pts * math.log2(R) / rc_s / 1e9, 1)
    out["sar_range_compression"] = comp
    log("range compression", json.dumps(comp))
    for p in (rf, af, ab, rb):
        p.close()
    del x, t1, t2, t3
    log("SAR", json.dumps(sar))
    return out


def run_small(torch, fb, inputs, stream):
    """Batches too small to be HBM-bound: N=1024 x 64 forward (launch-bound),
    five more small batches, and the paper's own workload N=1024 x 1024
    (16 MiB in + out, resident in the Infinity Cache).  Per-call time is 50
    back-to-back launches between two events (it includes the gaps between
    launches); where the planner picks the one-wave form of a kernel, or the
    four-step path for a long length, the full-width single block is timed
    beside it.  Kernel durations of the same launches
    come from a kernel trace (dispatch-stamped events have a floor of about
    4 us, above these kernels)."""
    res = {}
    sh = stream.cuda_stream
    ks = {k["name"]: k for k in fb.kernels()}
    cases = (("n1024x64_launch_bound", 1024, 64, 0), ("n512x64", 512, 64, 0), ("n256x256", 256, 256, 0),
             ("n3072x64", 3072, 64, 0), ("n16384x1", 16384, 1, 2), ("n32768x16", 32768, 16, 3),
             ("n1024x1024_cache_resident", 1024, 1024, 1))
    for name, n, batch, seed in cases:
        x = torch.from_numpy(inputs.uniform(seed, batch, n)).to("cuda")
        y = torch.empty_like(x)
        row = {}
        wide = ks[fb.plan_query(n, 1 << 14)["kernel_name"]]
        forms = [("planner", None)]
        planned = fb.plan_query(n, batch)
        if planned["kernel_name"] != wide["name"]:
            # the one-wave form, or for long lengths the four-step path: the
            # full-width single block beside it
            alt = "single_block" if planned["path"] == fb.PATH_FOURSTEP else "full_width"
            forms.append((alt, fb.make_opts(radix=wide["radix"], flags=wide["flags"], c=wide["c"])))
        for form, opts in forms:
            with fb.Plan(n, batch, fb.FORWARD, opts) as p:
                t = _timed(torch, stream, lambda: p.execute_ptr(x.data_ptr(), y.data_ptr(), sh), reps=50)
                d = p.describe()
                kname = d["kernel_name"] + ("+" + d["kernel_name2"] if d["path"] == fb.PATH_FOURSTEP else "")
                row[form] = {"kernel": kname, "per_call_us": round(t * 1e6, 2),
                             "GFLOPs_per_call": round(flops(n, batch) / t / 1e9, 1)}
        res[name] = row
        del x, y
    log("small batches", json.dumps(res))
    return res


def _timed(torch, stream, fn, reps=10):
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def run_fp16(torch, fb, inputs, stream):
    """FP16 storage (FP32 arithmetic): 4096 x 4096 and 2^20 x 16 forward, 8 B per point per pass."""
    res = {}
    sh = stream.cuda_stream
    for n, batch, storage in ((4096, 4096, fb.STORAGE_F16), (1 << 20, 16, fb.STORAGE_F16),
                              (1 << 20, 16, fb.STORAGE_F16_COMPACT)):
        x = torch.from_numpy(inputs.uniform(1, batch, n)).to("cuda").to(torch.complex32)
        y = torch.empty_like(x)
        with fb.Plan(n, batch, fb.FORWARD, fb.make_opts(storage=storage)) as p:
            d = p.describe()
            t = _timed(torch, stream, lambda: p.execute_ptr(x.data_ptr(), y.data_ptr(), sh))
        passes = 2 if d["path"] == fb.PATH_FOURSTEP else 1
        compact = storage == fb.STORAGE_F16_COMPACT
        # bytes per point: 4 in + 4 out per pass, the workspace complex64 (8 + 8) unless compact
        bpp = 8.0 if passes == 1 else 16.0 if compact else 24.0
        res[f"{n}x{batch}" + ("_compact" if compact else "")] = {
            "kernels": [d["kernel_name"]] + ([d["kernel_name2"]] if passes == 2 else []),
            "us": round(t * 1e6, 1), "GFLOPs": round(5.0 * n * math.log2(n) * batch / t / 1e9, 1),
            "bytes_per_point": bpp, "GBps": round(bpp * n * batch / t / 1e9, 1),
            "note": ("pass-1 output and pass-2 input FP16 as well" if compact else
                     "pass-1 output and pass-2 input stay complex64") if passes == 2 else ""}
        del x, y
    sizes = inputs.ragged_sizes(3)
    classes = [(int(n), int((sizes == n).sum())) for n in inputs.RAGGED_POW2 + inputs.RAGGED_MIXED]
    total = sum(n * c for n, c in classes)
    x = torch.randn(total, dtype=torch.complex64, device="cuda").to(torch.complex32)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    log(f"fp16 ragged buffers x={x.data_ptr():#x} y={y.data_ptr():#x} bytes={4 * total}")
    with fb.Ragged(classes, fb.FORWARD, storage=fb.STORAGE_F16) as r:
        t = _timed(torch, stream, lambda: r.execute(x, out=y), reps=20)
        t_plain = _timed(torch, stream, lambda: r.execute(x, out=y, mode=fb.RAGGED_PLAIN), reps=20)
    fl = sum(5.0 * n * math.log2(n) * c for n, c in classes)
    res["ragged_mix"] = {"total_points": total, "t_graph_us": round(t * 1e6, 1), "GFLOPs": round(fl / t / 1e9, 1),
                         "t_plain_sequential_us": round(t_plain * 1e6, 1)}
    log("fp16", json.dumps(res))
    return res


def run_serving(torch, fb, inputs):
    """Poisson arrivals at 2000 requests/s for 10 s (after a 1 s warm-up on a
    separate server): N = 2^k, k uniform on 8..22, batch log-uniform on
    [1, 512], direction 50/50, inputs from a pre-generated pool; 64 GiB HBM
    admission budget.  The pooled server (4 streams, continuous batching,
    bounded backfill of requests up to 1 GiB past a waiting head) and the
    plain path (one stream, one launch at a time, strict FIFO) replay the
    same trace."""
    from paper_1505_08067_amd import serving as sv

    def trace_of(seed, duration):
        t, n, b, sg = inputs.poisson_trace(seed, 2000.0, duration, 8, 22, 512)
        return [{"t": float(t[i]), "n": int(n[i]), "batch": int(b[i]), "direction": int(sg[i])}
                for i in range(t.size)]

    pool_points = (1 << 22) * 512
    pool = torch.empty(pool_points, dtype=torch.complex64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    pool.real.uniform_(-1.0, 1.0, generator=gen)
    pool.imag.uniform_(-1.0, 1.0, generator=gen)
    warm, trace = trace_of(40, 1.0), trace_of(4, 10.0)
    w_offs, offs = sv.trace_offsets(41, warm, pool_points), sv.trace_offsets(5, trace, pool_points)
    pts = sum(r["n"] * r["batch"] for r in trace)
    fl = sum(5.0 * r["n"] * math.log2(r["n"]) * r["batch"] for r in trace)
    res = {"requests": len(trace), "rate_per_s": 2000.0, "duration_s": 10.0, "budget_bytes": 64 << 30}
    for name, kw in (("pooled", {}), ("plain", {"n_streams": 1, "max_inflight": 1, "max_coalesce": 1, "backfill_bytes": 0})):
        for phase, tr, of in (("warmup", warm, w_offs), ("timed", trace, offs)):
            with sv.Server(hbm_budget=64 << 30, auto_release=True, **kw) as srv:
                for k in range(8, 23):
                    srv.prepare(1 << k, fb.FORWARD)
                    srv.prepare(1 << k, fb.BACKWARD)
                st = sv.replay(srv, tr, pool, of)
            log(f"serving {name} {phase}: {st['completed']} requests in {st['wall']:.2f} s")
        res[name] = {
            "completed": st["completed"], "rejected": st["rejected"], "launches": st["launches"],
            "coalesced_requests": st["coalesced_requests"], "backfilled_requests": st["backfilled_requests"],
            "p50_ms": round(st["latency_p50"] * 1e3, 3), "p99_ms": round(st["latency_p99"] * 1e3, 3),
            "mean_ms": round(st["latency_mean"] * 1e3, 3), "max_ms": round(st["latency_max"] * 1e3, 3),
            "queue_p50_ms": round(st["queue_p50"] * 1e3, 3), "queue_p99_ms": round(st["queue_p99"] * 1e3, 3),
            "device_p50_ms": round(st["device_p50"] * 1e3, 3), "device_p99_ms": round(st["device_p99"] * 1e3, 3),
            "peak_inflight_GiB": round(st["peak_inflight_bytes"] / 2 ** 30, 2),
            "wall_s": round(st["wall"], 3), "GFLOPs": round(fl / st["wall"] / 1e9, 1),
            "points_per_s": round(pts / st["wall"], 1)}
    # saturation: a 2 s slice of the same stream (about 4000 requests)
    # submitted at once (every arrival time 0) to the pooled server: the
    # throughput the served mix sustains when requests are always waiting
    burst = [dict(r, t=0.0) for r in trace_of(42, 2.0)]
    b_offs = sv.trace_offsets(43, burst, pool_points)
    bfl = sum(5.0 * r["n"] * math.log2(r["n"]) * r["batch"] for r in burst)
    with sv.Server(hbm_budget=64 << 30, auto_release=True) as srv:
        for k in range(8, 23):
            srv.prepare(1 << k, fb.FORWARD)
            srv.prepare(1 << k, fb.BACKWARD)
        st = sv.replay(srv, burst, pool, b_offs)
    log(f"serving saturated: {st['completed']} requests in {st['wall']:.2f} s")
    res["saturated"] = {"requests": len(burst), "completed": st["completed"], "wall_s": round(st["wall"], 3),
                        "GFLOPs": round(bfl / st["wall"] / 1e9, 1), "launches": st["launches"],
                        "coalesced_requests": st["coalesced_requests"],
                        "p99_ms": round(st["latency_p99"] * 1e3, 3)}
    # the plain uniform-batch rate of the same mix: each length as one batch
    # of 2^26 points (forward; the inverse costs the same), and the burst's
    # points of each length at that rate, summed
    out = torch.empty(1 << 26, dtype=torch.complex64, device="cuda")
    sh = torch.cuda.current_stream().cuda_stream
    t_uniform = 0.0
    per_n = {}
    for k in range(8, 23):
        n = 1 << k
        b = (1 << 26) // n
        with fb.Plan(n, b, fb.FORWARD) as p:
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            for _ in range(3):
                p.execute_ptr(pool.data_ptr(), out.data_ptr(), sh)
            ev[0].record()
            for _ in range(10):
                p.execute_ptr(pool.data_ptr(), out.data_ptr(), sh)
            ev[1].record()
            torch.cuda.synchronize()
            rate = n * b / (ev[0].elapsed_time(ev[1]) / 10 * 1e-3)      # points per second
        pts_n = sum(r["n"] * r["batch"] for r in burst if r["n"] == n)
        per_n[n] = round(5.0 * math.log2(n) * rate / 1e9, 1)
        t_uniform += pts_n / rate
    del out
    res["saturated"]["uniform_batches_same_mix_GFLOPs"] = round(bfl / t_uniform / 1e9, 1)
    res["saturated"]["over_uniform_same_mix"] = round(t_uniform / st["wall"], 3)
    res["saturated"]["uniform_GFLOPs_by_n"] = per_n
    del pool
    log("serving", json.dumps(res))
    return res


def run_ragged(torch, fb, inputs, stream):
    """The ragged mix: 15 lengths with an equal share of about 2^28 points.

    Each length is autotuned first (the paper's stage model plus whole-kernel
    validation; the fastest kernel becomes the wisdom the plain plans use).
    Then the whole mix runs as one graph of persistent work-list kernels (one
    launch per LDS-footprint class) and is compared with the plain path: every
    length as its own batched execute, timed separately and summed; the
    per-length kernels on four graph branches are timed beside it.
    """
    sizes = inputs.ragged_sizes(3)
    classes = [(int(n), int((sizes == n).sum())) for n in inputs.RAGGED_POW2 + inputs.RAGGED_MIXED]
    tuned = {}
    for n, c in classes:
        # the class's own batch: 2^28 / 15 points, 143 MB each way, so the
        # candidates are timed against HBM rather than the Infinity Cache
        rep = fb.autotune(n, c)
        tuned[n] = {"kernel": rep["chosen"], "chosen_us": round(rep["chosen_us"], 2),
                    "predicted_schedule": rep["predicted"],
                    "predicted_us": None if rep["predicted_us"] is None else round(rep["predicted_us"], 2),
                    "chosen_schedule_rt_us": None if rep["chosen_schedule_rt_us"] is None
                    else round(rep["chosen_schedule_rt_us"], 2),
                    "chosen_is_predicted": rep["chosen_predicted"]}
    total = sum(n * c for n, c in classes)
    x = torch.empty(total, dtype=torch.complex64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    x.real.uniform_(-1.0, 1.0, generator=gen)
    x.imag.uniform_(-1.0, 1.0, generator=gen)
    y = torch.empty_like(x)
    sh = stream.cuda_stream

    def timed(fn, reps=10, warm=2):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    t_plain, at = 0.0, 0
    per_class = {}
    for n, c in classes:
        with fb.Plan(n, c, fb.FORWARD) as p:
            xi, yi = x[at:at + n * c], y[at:at + n * c]
            t = timed(lambda: p.execute_ptr(xi.data_ptr(), yi.data_ptr(), sh))
        per_class[n] = round(t * 1e6, 2)
        t_plain += t
        at += n * c
    with fb.Ragged(classes, fb.FORWARD) as r:
        # the first launches of a freshly built graph run slower: warm it up
        t_graph = timed(lambda: r.execute(x, out=y, mode=fb.RAGGED_PERSISTENT), reps=20, warm=10)
        t_branch = timed(lambda: r.execute(x, out=y, mode=fb.RAGGED_BRANCHES), reps=20, warm=10)
        t_seq = timed(lambda: r.execute(x, out=y, mode=fb.RAGGED_PLAIN), reps=20, warm=10)
        d = r.describe()
    fl = sum(5.0 * n * math.log2(n) * c for n, c in classes)
    res = {
        "classes": [[n, c] for n, c in classes], "total_points": total,
        "graph_nodes": d["kernel_nodes"], "persistent_launches": d["persistent_launches"],
        "t_plain_sum_us": round(t_plain * 1e6, 1), "t_graph_us": round(t_graph * 1e6, 1),
        "t_per_length_branch_graph_us": round(t_branch * 1e6, 1),
        "per_length_branch_graph_nodes": d["branch_graph_nodes"],
        "t_sequential_us": round(t_seq * 1e6, 1),
        "ratio_plain_over_graph": round(t_plain / t_graph, 3),
        "graph_GFLOPs": round(fl / t_graph / 1e9, 1),
        "graph_GBps_one_pass": round(16.0 * total / t_graph / 1e9, 1),
        "per_class_plain_us": per_class, "autotuned": tuned,
    }
    # the same 15 lengths at 1/256 of the counts (about 1 M points): launch
    # rather than HBM bound, where one launch per footprint class replaces
    # fifteen per-length launches
    small = [(n, max(1, c // 256)) for n, c in classes]
    tot_s = sum(n * c for n, c in small)
    xs, ys = x[:tot_s], y[:tot_s]
    t_plain_s, at = 0.0, 0
    for n, c in small:
        with fb.Plan(n, c, fb.FORWARD) as p:
            xi, yi = xs[at:at + n * c], ys[at:at + n * c]
            t_plain_s += timed(lambda: p.execute_ptr(xi.data_ptr(), yi.data_ptr(), sh), reps=50, warm=5)
        at += n * c
    with fb.Ragged(small, fb.FORWARD) as r:
        t_graph_s = timed(lambda: r.execute(xs, out=ys, mode=fb.RAGGED_PERSISTENT), reps=50, warm=10)
        t_branch_s = timed(lambda: r.execute(xs, out=ys, mode=fb.RAGGED_BRANCHES), reps=50, warm=10)
        t_seq_s = timed(lambda: r.execute(xs, out=ys, mode=fb.RAGGED_PLAIN), reps=50, warm=10)
        d_s = r.describe()
    res["small_mix"] = {"classes": [[n, c] for n, c in small], "total_points": tot_s,
                        "graph_nodes": d_s["kernel_nodes"], "t_plain_sum_us": round(t_plain_s * 1e6, 1),
                        "t_graph_us": round(t_graph_s * 1e6, 1), "t_per_length_branch_graph_us": round(t_branch_s * 1e6, 1),
                        "t_sequential_us": round(t_seq_s * 1e6, 1),
                        "ratio_plain_over_graph": round(t_plain_s / t_graph_s, 3)}
    log("ragged", json.dumps({k: v for k, v in res.items() if k not in ("autotuned", "per_class_plain_us")}))
    fb.wisdom_clear()
    return res


def run_schedule_model(torch, fb, stream):
    """The paper's performance model tested on this GPU at its own length,
    N = 1024: the stage costs measured one stage at a time give every
    schedule (sequence of radices 2, 4, 8, 16) an additive cost; every
    schedule of at most 8 stages (391) is then run whole on the
    run-time-schedule kernel (16384 transforms, 128 MiB each way, four
    rotating buffer sets) and the model's ranking is compared with the
    measured one (Spearman rank correlation), with the model's optimum, the
    measured optimum and the schedules the paper's tables compare."""
    import numpy as np
    n, batch = 1024, 16384
    rep = fb.autotune(n, batch)
    cost = rep["stage_cost"]                      # (radix, start stage) -> ns per transform
    scheds = []

    def rec(left, acc):
        if left == 0:
            scheds.append(list(acc))
            return
        if len(acc) == 8:
            return
        for r in (2, 4, 8, 16):
            if int(math.log2(r)) <= left:
                rec(left - int(math.log2(r)), acc + [r])

    rec(10, [])
    sets = [(torch.empty(2 * n * batch, dtype=torch.float32, device="cuda").uniform_(-1, 1).view(torch.complex64),
             torch.empty(n * batch, dtype=torch.complex64, device="cuda")) for _ in range(4)]
    sh = stream.cuda_stream
    flags = fb.VARIANT_RUNTIME_SCHEDULE | fb.VARIANT_NT_LOAD | fb.VARIANT_NT_STORE
    model, measured = [], []
    for sc in scheds:
        at, c = 0, 0.0
        for r in sc:
            c += cost[(r, at)]
            at += int(math.log2(r))
        with fb.Plan(n, batch, fb.FORWARD, fb.make_opts(radix=sc, flags=flags)) as p:
            k = [0]

            def step():
                xi, yi = sets[k[0] % 4]
                k[0] += 1
                p.execute_ptr(xi.data_ptr(), yi.data_ptr(), sh)
            t = _timed(torch, stream, step, reps=12)
        model.append(c)
        measured.append(t * 1e6)
    # the kernel the autotuner chose and the planner's default, timed the
    # same way as the schedules, in interleaved rounds
    p_tuned = fb.Plan(n, batch, fb.FORWARD)
    fb.wisdom_clear()
    p_dflt = fb.Plan(n, batch, fb.FORWARD)
    chosen_name, dflt_name = p_tuned.describe()["kernel_name"], p_dflt.describe()["kernel_name"]
    tt = {"tuned": [], "default": []}
    for _ in range(5):
        for lab, p in (("tuned", p_tuned), ("default", p_dflt)):
            k = [0]

            def step_c():
                xi, yi = sets[k[0] % 4]
                k[0] += 1
                p.execute_ptr(xi.data_ptr(), yi.data_ptr(), sh)
            tt[lab].append(_timed(torch, stream, step_c, reps=12) * 1e6)
    p_tuned.close()
    p_dflt.close()
    t_chosen = sorted(tt["tuned"])[2]
    t_dflt = sorted(tt["default"])[2]
    del sets
    model, measured = np.array(model), np.array(measured)
    rk = lambda v: np.argsort(np.argsort(v))
    rho = float(np.corrcoef(rk(model), rk(measured))[0, 1])
    order = np.argsort(measured)
    pi = scheds.index(rep["predicted"]) if rep["predicted"] in scheds else None
    key = lambda sc: ",".join(str(v) for v in sc)
    res = {"n": n, "batch": batch, "schedules": len(scheds), "spearman_model_vs_measured": round(rho, 3),
           "predicted": rep["predicted"],
           "predicted_us": None if pi is None else round(float(measured[pi]), 2),
           "predicted_measured_rank": None if pi is None else int(np.where(order == pi)[0][0]) + 1,
           "best_measured": scheds[int(order[0])], "best_measured_us": round(float(measured[order[0]]), 2),
           "worst_measured_us": round(float(measured[order[-1]]), 2),
           "autotuned_kernel": chosen_name, "autotuned_kernel_us": round(t_chosen, 2),
           "default_kernel": dflt_name, "default_kernel_us": round(t_dflt, 2),
           "paper_schedules_us": {key(sc): round(float(measured[scheds.index(sc)]), 2)
                                  for sc in ([8, 8, 8, 2], [4, 8, 8, 4], [8, 8, 4, 4], [16, 16, 4])}}
    log("schedule model", json.dumps(res))
    return res


def run_lanes(torch, fb, stream, rounds=7, reps=20):
    """Global-access width and exchange form of the block kernels: 2^24
    points per launch at every length (128 MiB read, 128 MiB written),
    forward, four rotating (in, out) sets so every launch reads and writes
    HBM.  The planner's kernel against the same schedule with 16-byte lanes
    (neighbouring lanes swapping halves by DPP) and, where one exists, the
    kernels whose intra-wave exchanges are register permutations, with the
    LDS kernels of their schedule.  The candidates of a length are timed in
    turn, `rounds` times `reps` launches each; the median round is reported
    (and the spread, max - min, over the rounds)."""
    sh = stream.cuda_stream
    npts = 1 << 24
    sets = [(torch.empty(2 * npts, dtype=torch.float32, device="cuda").uniform_(-1, 1).view(torch.complex64),
             torch.empty(npts, dtype=torch.complex64, device="cuda")) for _ in range(4)]
    kinfo = [k for k in fb.kernels() if k["kind"] == "block" and not k["flags"] & fb.VARIANT_FP16_STORAGE]
    res = {}

    def fits(n, batch):
        # the launches below take raw pointers: every one must stay inside a set
        if n * batch > npts:
            raise ValueError(f"{n} x {batch} exceeds the {npts}-point buffer sets")
    for n in (256, 1024, 2048, 4096, 8192):
        batch = npts // n
        fits(n, batch)
        with fb.Plan(n, batch, fb.FORWARD) as p0:
            d0 = p0.describe()
        base = next(k for k in kinfo if k["name"] == d0["kernel_name"])
        cands = [("planner", base)]
        for k in kinfo:
            if k["n"] == n and k["radix"] == base["radix"] and k["c"] == base["c"] and k is not base \
                    and k["flags"] == (base["flags"] | fb.VARIANT_VEC16):
                cands.append(("vec16", k))
        xl = [k for k in kinfo if k["n"] == n and k["flags"] & fb.VARIANT_CROSS_LANE]
        if xl:
            # the same schedule with LDS exchanges (barriers, and wave-synchronous)
            for k in kinfo:
                if k["n"] == n and k["radix"] == xl[0]["radix"] and k["c"] == xl[0]["c"] \
                        and not k["flags"] & fb.VARIANT_CROSS_LANE:
                    cands.append((f"lds_exchanges_v{k['flags']}", k))
            for k in xl:
                lab = "cross_lane_then_lds" if k["flags"] & fb.VARIANT_WAVE_SYNC else "cross_lane_all"
                cands.append((lab, k))
        plans = [(lab, fb.Plan(n, batch, fb.FORWARD, fb.make_opts(radix=k["radix"], flags=k["flags"], c=k["c"])))
                 for lab, k in cands]
        times = {lab: [] for lab, _ in plans}
        for _ in range(rounds):
            for lab, p in plans:
                it = [0]

                def step():
                    xi, yi = sets[it[0] % 4]
                    it[0] += 1
                    p.execute_ptr(xi.data_ptr(), yi.data_ptr(), sh)
                times[lab].append(_timed(torch, stream, step, reps=reps) * 1e6)
        row = {}
        for lab, p in plans:
            ts = sorted(times[lab])
            med = ts[len(ts) // 2]
            row[lab] = {"kernel": p.describe()["kernel_name"], "us": round(med, 2),
                        "spread_us": round(ts[-1] - ts[0], 2),
                        "frac_hbm_peak": round(16.0 * npts / (med * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4)}
            p.close()
        res[f"{n}x{batch}"] = row
    # the long single blocks: every compiled complex64 form
    for n in (16384, 32768):
        batch = npts // n
        fits(n, batch)
        with fb.Plan(n, batch, fb.FORWARD, fb.make_opts(block_limit=n)) as p0:
            d0 = p0.describe()
        cands = [k for k in kinfo if k["n"] == n and not k["flags"] & (fb.VARIANT_FP16_STORAGE |
                 fb.VARIANT_RUNTIME_SCHEDULE)]
        plans = [(k["name"], fb.Plan(n, batch, fb.FORWARD, fb.make_opts(radix=k["radix"], flags=k["flags"], c=k["c"],
                                                                         block_limit=n))) for k in cands]
        times = {lab: [] for lab, _ in plans}
        for _ in range(rounds):
            for lab, p in plans:
                it = [0]

                def step_l():
                    xi, yi = sets[it[0] % 4]
                    it[0] += 1
                    p.execute_ptr(xi.data_ptr(), yi.data_ptr(), sh)
                times[lab].append(_timed(torch, stream, step_l, reps=reps) * 1e6)
        row = {"planner": d0["kernel_name"]}
        for lab, p in plans:
            ts = sorted(times[lab])
            med = ts[len(ts) // 2]
            row[lab] = {"us": round(med, 2), "spread_us": round(ts[-1] - ts[0], 2),
                        "frac_hbm_peak": round(16.0 * n * batch / (med * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4),
                        "workgroups_per_cu": fb.kernel_occupancy(lab)}
            p.close()
        res[f"{n}x{batch}"] = row
    # mixed-radix lengths: the planner's kernel against the kernels whose
    # stages run on different thread counts
    for n in (6000, 15360):
        batch = npts // n
        fits(n, batch)
        with fb.Plan(n, batch, fb.FORWARD) as p0:
            d0 = p0.describe()
        base = next(k for k in kinfo if k["name"] == d0["kernel_name"])
        cands = [("planner", base)] + [(k["name"], k) for k in kinfo
                                       if k["n"] == n and k["flags"] & fb.VARIANT_VAR_THREADS]
        plans = [(lab, fb.Plan(n, batch, fb.FORWARD, fb.make_opts(radix=k["radix"], flags=k["flags"], c=k["c"])))
                 for lab, k in cands]
        times = {lab: [] for lab, _ in plans}
        for _ in range(rounds):
            for lab, p in plans:
                it = [0]

                def step_m():
                    xi, yi = sets[it[0] % 4]
                    it[0] += 1
                    p.execute_ptr(xi.data_ptr(), yi.data_ptr(), sh)
                times[lab].append(_timed(torch, stream, step_m, reps=reps) * 1e6)
        row = {}
        for lab, p in plans:
            ts = sorted(times[lab])
            med = ts[len(ts) // 2]
            name = p.describe()["kernel_name"]
            row[lab] = {"kernel": name, "us": round(med, 2), "spread_us": round(ts[-1] - ts[0], 2),
                        "frac_hbm_peak": round(16.0 * n * batch / (med * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4),
                        "workgroups_per_cu": fb.kernel_occupancy(name)}
            p.close()
        res[f"{n}x{batch}"] = row
    # four-step pass 1 at 2^20 x 16 (512-point columns): the planner's
    # kernel against the other compiled 512-point pass-1 forms with the same
    # schedule (wider tiles, workgroups looping over tiles)
    n, batch = 1 << 20, 16
    fits(n, batch)
    with fb.Plan(n, batch, fb.FORWARD) as p0:
        d0 = p0.describe()
    base = next(k for k in fb.kernels() if k["name"] == d0["kernel_name"])
    cands = [("planner", base)] + [(f"v{k['flags']}_C{k['c']}", k) for k in fb.kernels()
                                   if k["kind"] == "pass1" and k["n"] == base["n"] and k["radix"] == base["radix"]
                                   and k is not base and not k["flags"] & fb.VARIANT_FP16_STORAGE]
    plans = [(lab, fb.Plan(n, batch, fb.FORWARD, fb.make_opts(radix=k["radix"], flags=k["flags"], c=k["c"],
                                                              n1=base["n"])))
             for lab, k in cands]
    times = {lab: [] for lab, _ in plans}
    for _ in range(rounds):
        for lab, p in plans:
            it = [0]

            def step1():
                xi, yi = sets[it[0] % 4]
                it[0] += 1
                p.execute_pass_ptr(1, xi.data_ptr(), yi.data_ptr(), sh)
            times[lab].append(_timed(torch, stream, step1, reps=reps) * 1e6)
    row = {}
    for lab, p in plans:
        ts = sorted(times[lab])
        med = ts[len(ts) // 2]
        row[lab] = {"kernel": p.describe()["kernel_name"], "us": round(med, 2), "spread_us": round(ts[-1] - ts[0], 2),
                    "frac_hbm_peak": round(16.0 * npts / (med * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4)}
        p.close()
    res["fourstep_pass1_2^20x16"] = row
    # pass 2 (2048-point rows) the same way: the planner's kernel against the
    # other compiled forms of its schedule and width
    base2 = next(k for k in fb.kernels() if k["name"] == d0["kernel_name2"])
    cands = [("planner", base2)] + [(f"v{k['flags']}_C{k['c']}", k) for k in fb.kernels()
                                    if k["kind"] == "pass2" and k["n"] == base2["n"] and k["radix"] == base2["radix"]
                                    and k["c"] == base2["c"] and k is not base2
                                    and not k["flags"] & fb.VARIANT_FP16_STORAGE]
    plans = [(lab, fb.Plan(n, batch, fb.FORWARD, fb.make_opts(n1=base["n"], flags2=k["flags"], c2=k["c"])))
             for lab, k in cands]
    times = {lab: [] for lab, _ in plans}
    for _ in range(rounds):
        for lab, p in plans:
            it = [0]

            def step2():
                xi, yi = sets[it[0] % 4]
                it[0] += 1
                p.execute_pass_ptr(2, xi.data_ptr(), yi.data_ptr(), sh)
            times[lab].append(_timed(torch, stream, step2, reps=reps) * 1e6)
    row = {}
    for lab, p in plans:
        ts = sorted(times[lab])
        med = ts[len(ts) // 2]
        row[lab] = {"kernel": p.describe()["kernel_name2"], "us": round(med, 2),
                    "spread_us": round(ts[-1] - ts[0], 2),
                    "frac_hbm_peak": round(16.0 * npts / (med * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4)}
        p.close()
    res["fourstep_pass2_2^20x16"] = row
    # range compression (2^24 points per launch): every compiled filter kernel
    # at 4096, 8192 and 16384 samples per row
    from paper_1505_08067_amd import inputs
    rep = torch.from_numpy(inputs.sar_replica()).to("cuda")
    for n in (4096, 8192, 16384):
        batch = npts // n
        fits(n, batch)
        with fb.RangeCompressor(n, batch, rep) as r0:
            dflt = r0.describe()["kernel_name"]
        cands = [k for k in fb.kernels() if k["kind"] == "filter" and k["n"] == n]
        comps = [(k["name"], fb.RangeCompressor(n, batch, rep, fb.make_opts(radix=k["radix"], flags=k["flags"],
                                                                             c=k["c"]))) for k in cands]
        times = {lab: [] for lab, _ in comps}
        for _ in range(rounds):
            for lab, rc in comps:
                it = [0]

                def step_f():
                    xi, yi = sets[it[0] % 4]
                    it[0] += 1
                    rc.execute_ptr(xi.data_ptr(), yi.data_ptr(), sh)
                times[lab].append(_timed(torch, stream, step_f, reps=reps) * 1e6)
        row = {"planner": dflt}
        for lab, rc in comps:
            ts = sorted(times[lab])
            med = ts[len(ts) // 2]
            row[lab] = {"us": round(med, 2), "spread_us": round(ts[-1] - ts[0], 2),
                        "frac_hbm_peak": round(16.0 * npts / (med * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4),
                        "workgroups_per_cu": fb.kernel_occupancy(lab)}
            rc.close()
        res[f"range_compress_{n}x{batch}"] = row
    del sets
    log("lanes", json.dumps(res))
    return res


def cpu_baseline(items, fl_step, target_s, gpu_outs=None):
    """The FP64 oracle (radix-2 recursion, all host threads) on the same step,
    repeated ~target_s.  The first repetition's results are also compared with
    the GPU's outputs of the same inputs (relative L2 per transform)."""
    import numpy as np

    import oracle
    from oracle import metrics
    from paper_1505_08067_amd import inputs

    data = {}
    for _, n, batch, _ in items:
        if (n, batch) not in data:
            data[(n, batch)] = inputs.uniform(1, batch, n).astype(np.complex128)
    reps, t_total, err = 0, 0.0, {}
    while t_total < target_s or reps == 0:
        t0 = time.perf_counter()
        res = [oracle.fft_radix2(data[(n, batch)], sign) for _, n, batch, sign in items]
        t_total += time.perf_counter() - t0
        if reps == 0 and gpu_outs:
            for (name, n, _, _), ref in zip(items, res):
                e = metrics.rel_l2_per_transform(gpu_outs[name], ref)
                err[name] = {"max_rel_l2": float(f"{np.max(e):.3e}"), "median_rel_l2": float(f"{np.median(e):.3e}"),
                             "tolerance": float(f"{metrics.tolerance(n):.3e}")}
        del res
        reps += 1
        if reps >= 50:
            break
    value = fl_step * reps / t_total / 1e9
    log(f"cpu baseline: {reps} steps in {t_total:.2f} s")
    out = {"value": round(value, 3), "unit": "GFLOP/s", "cores": oracle.nthreads(), "kind": "oracle",
           "sample": f"{reps} full step(s) of the same workload (4096x4096 fwd+inv, 2^20x16 fwd+inv) "
                     f"through the FP64 radix-2 oracle, {t_total:.1f} s"}
    if err:
        out["gpu_error_vs_oracle"] = err
    return out


if __name__ == "__main__":
    main()
