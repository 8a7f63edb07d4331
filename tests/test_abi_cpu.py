"""The C-ABI library on the CPU: it loads, exports what the header declares,
checks arguments before any HIP call, and plans without a device."""
import ctypes
import math
import os
import re
import subprocess

import pytest

from paper_1505_08067_amd import fftblock as fb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fftblock.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fft_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = fb.load()
    declared = header_functions()
    assert set(declared) == set(fb.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", fb.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fft_\w+)", out))
    assert set(declared) <= exported


def test_header_is_plain_c():
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", HEADER],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(fb, "_lib", None)
    monkeypatch.setattr(fb, "LIB_PATH", os.path.join(ROOT, "does_not_exist.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        fb.load()


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1505_08067_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), f
                assert "fft_oracle" not in txt and "liboracle" not in txt, f


def test_status_strings():
    for code in range(6):
        assert fb.status_string(code)
    assert fb.status_string(99) == "unknown status"


@pytest.mark.parametrize("k,expect", [(1, 16384), (2, 8192), (4, 4096)])
def test_block_max_for_160k_lds(k, expect):
    # pow2floor(160 KiB / (8 B * 17/16 * k))
    assert fb.load().fft_block_max(160 * 1024, k) == expect


def test_block_max_other_sizes():
    lib = fb.load()
    assert lib.fft_block_max(64 * 1024, 1) == 4096
    assert lib.fft_block_max(64 * 1024, 2) == 2048
    assert lib.fft_block_max(100, 1) == 8
    assert lib.fft_block_max(8, 1) == 0
    assert lib.fft_block_max(160 * 1024, 0) == 0


def test_plan_query_block_and_fourstep():
    limit = fb.block_limit()
    assert limit == 32768
    for L in range(1, 23):
        n = 1 << L
        d = fb.plan_query(n, 64)
        # from 8192 on a transform fills a large share of a compute unit, so
        # small batches go four-step (checked below); 64 take the block
        if n <= limit:
            assert d["path"] == fb.PATH_BLOCK and d["kernels_per_execute"] == 1
            assert math.prod(d["radix"]) == n
            assert d["workspace_bytes"] == 0
            assert d["lds_bytes"] <= 160 * 1024
        else:
            assert d["path"] == fb.PATH_FOURSTEP and d["kernels_per_execute"] == 2
            assert d["n1"] * d["n2"] == n
            # rows (pass 2) up to 2048, columns (pass 1) at least 256
            assert d["n2"] == min(2048, n // 256) and d["n1"] == n // d["n2"]
            assert math.prod(d["radix"]) == d["n1"] and math.prod(d["radix2"]) == d["n2"]
            assert d["workspace_bytes"] == 8 * n * 64
            assert d["lds_bytes"] <= 160 * 1024
    for n, first in ((2048, 1), (4096, 1), (8192, 16), (16384, 48), (32768, 64)):
        for batch in (1, first - 1, first, 1024):
            if batch < 1:
                continue
            d = fb.plan_query(n, batch)
            assert d["path"] == (fb.PATH_BLOCK if batch >= first else fb.PATH_FOURSTEP), (n, batch)
            if d["path"] == fb.PATH_BLOCK:
                assert math.prod(d["radix"]) == n and d["workspace_bytes"] == 0
                assert d["lds_bytes"] <= 160 * 1024
            else:
                assert d["n1"] * d["n2"] == n and d["workspace_bytes"] == 8 * n * batch
    f16 = fb.make_opts(storage=fb.STORAGE_F16)
    for n, first in ((8192, 1), (16384, 32), (32768, 48)):
        for batch in (first - 1, first):
            if batch >= 1:
                d = fb.plan_query(n, batch, opts=f16)
                assert d["path"] == (fb.PATH_BLOCK if batch >= first else fb.PATH_FOURSTEP), (n, batch)
    assert fb.plan_query(limit, 64)["threads_per_block"] == limit // 32
    # an explicit block limit, or options naming a block kernel, keep the
    # single block at any batch
    assert fb.plan_query(limit, 1, opts=fb.make_opts(block_limit=limit))["path"] == fb.PATH_BLOCK
    assert fb.plan_query(16384, 1, opts=fb.make_opts(flags=1059))["path"] == fb.PATH_BLOCK
    assert fb.plan_query(8192, 1, opts=fb.make_opts(c=1))["path"] == fb.PATH_BLOCK
    assert fb.plan_query(limit, 1024, opts=fb.make_opts(block_limit=16384))["path"] == fb.PATH_FOURSTEP
    d = fb.plan_query(1 << 20, 16)
    assert (d["n1"], d["n2"]) == (512, 2048)
    d = fb.plan_query(1 << 20, 16, opts=fb.make_opts(n1=1024))
    assert (d["n1"], d["n2"]) == (1024, 1024)
    with pytest.raises(fb.FFTError):
        fb.plan_query(1 << 20, 16, opts=fb.make_opts(n1=3))
    assert fb.plan_query(1, 5)["path"] == fb.PATH_BLOCK


def test_block_limit_env_override():
    code = ("from paper_1505_08067_amd import fftblock as f; "
            "print(f.block_limit(), f.plan_query(8192, 1)['path'], f.plan_query(4096, 1)['path'])")
    env = dict(os.environ, FFTBLOCK_BLOCK_MAX="4096")
    out = subprocess.run(["python", "-c", code], env=env, cwd=ROOT, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["4096", "2", "1"]


@pytest.mark.parametrize("args,status", [
    ((0, 1, -1), 1), ((8, 0, -1), 1), ((8, 1, 0), 1), ((8, 1, 2), 1),
    ((7, 1, -1), 2), ((1001, 1, -1), 2), ((3000, 1, -1), 2), ((1 << 23, 1, -1), 2),
])
def test_plan_argument_errors_without_device(args, status):
    with pytest.raises(fb.FFTError) as ei:
        fb.plan_query(*args)
    assert ei.value.status == status
    # fft_plan_create rejects the same arguments before any HIP call
    h = ctypes.c_void_p(123)
    assert fb.load().fft_plan_create(*args, ctypes.byref(h)) == status
    assert h.value is None


def test_null_and_unknown_handles():
    lib = fb.load()
    assert lib.fft_plan_create(8, 1, -1, None) == 1
    assert lib.fft_execute(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == 5
    assert lib.fft_execute(ctypes.c_void_p(0xdead0), ctypes.c_void_p(16), ctypes.c_void_p(16), None) == 5
    assert lib.fft_plan_destroy(None) == 5
    assert lib.fft_plan_destroy(ctypes.c_void_p(0xdead0)) == 5
    assert lib.fft_plan_describe(None, None) == 5
    assert lib.fft_plan_query(8, 1, -1, None) == 1
    assert lib.fft_device_query(0, None) == 1
    occ = ctypes.c_int(-7)
    assert lib.fft_kernel_occupancy(0, None) == 1
    assert lib.fft_kernel_occupancy(-1, ctypes.byref(occ)) == 1
    assert lib.fft_kernel_occupancy(lib.fft_kernel_count(), ctypes.byref(occ)) == 1
    assert occ.value == -7


def test_transpose_and_copy_argument_errors_without_device():
    lib = fb.load()
    vp = ctypes.c_void_p
    assert lib.fft_transpose(None, vp(0x10000), 4, 4, 1, None) == 1
    assert lib.fft_transpose(vp(0x10000), vp(0x20000), 0, 4, 1, None) == 1
    assert lib.fft_transpose(vp(0x10000), vp(0x20000), 4, 0, 1, None) == 1
    assert lib.fft_transpose(vp(0x10000), vp(0x20000), 4, 4, 0, None) == 1
    assert lib.fft_transpose(vp(0x10004), vp(0x20000), 4, 4, 1, None) == 1      # misaligned
    assert lib.fft_transpose(vp(0x10000), vp(0x10008), 4, 4, 1, None) == 1      # overlap
    assert lib.fft_copy(vp(0x10000), vp(0x20000), 24, None) == 1                 # not a multiple of 16
    assert lib.fft_copy(vp(0x10008), vp(0x20000), 32, None) == 1                 # misaligned
    assert lib.fft_copy(vp(0x10000), vp(0x10010), 32, None) == 1                 # overlap
    assert lib.fft_copy(None, vp(0x20000), 32, None) == 1


def test_fp16_storage_planning_without_device():
    for n in (2, 16, 60, 1000, 4096, 16384):
        d = fb.plan_query(n, 3, opts=fb.make_opts(storage=fb.STORAGE_F16))
        assert d["storage"] == 1 and "_f16" in d["kernel_name"], n
        assert d["flags"] & fb.VARIANT_FP16_STORAGE
    d = fb.plan_query(32768, 64, opts=fb.make_opts(storage=fb.STORAGE_F16))
    assert d["path"] == fb.PATH_BLOCK and "_f16" in d["kernel_name"]
    for L in (15, 20, 22):
        d = fb.plan_query(1 << L, 1, opts=fb.make_opts(storage=fb.STORAGE_F16))
        assert d["path"] == fb.PATH_FOURSTEP
        assert "_f16" in d["kernel_name"] and "_f16" in d["kernel_name2"]
        assert d["workspace_bytes"] == 8 << L          # the workspace stays complex64
    # complex64 plans never pick an FP16 kernel
    assert "_f16" not in fb.plan_query(4096, 1)["kernel_name"]
    assert fb.plan_query(4096, 1)["storage"] == 0
    with pytest.raises(fb.FFTError) as ei:
        fb.plan_query(4096, 1, opts=fb.make_opts(storage=3))
    assert ei.value.status == 1
    # the compact FP16 form: FP16 workspace passes on the four-step path (both
    # passes, the storage's own kernels), the FP16 blocks otherwise
    d = fb.plan_query(1 << 20, 16, opts=fb.make_opts(storage=fb.STORAGE_F16_COMPACT))
    assert d["path"] == fb.PATH_FOURSTEP and "_f16w" in d["kernel_name"] and "_f16w" in d["kernel_name2"]
    assert d["workspace_bytes"] == 4 << 24                   # FP16 pairs
    assert fb.plan_query(4096, 4, opts=fb.make_opts(storage=fb.STORAGE_F16_COMPACT))["kernel_name"] == \
        fb.plan_query(4096, 4, opts=fb.make_opts(storage=fb.STORAGE_F16))["kernel_name"]
    with pytest.raises(fb.FFTError) as ei:                  # an FP32-workspace pass 2 with the compact form
        fb.plan_query(1 << 20, 16, opts=fb.make_opts(storage=fb.STORAGE_F16_COMPACT, flags2=98, c2=16, n1=1024))
    assert ei.value.status == 1
    with pytest.raises(fb.FFTError):                         # no ragged batches in the compact form
        fb.Ragged([(1024, 2)], storage=fb.STORAGE_F16_COMPACT)
    with pytest.raises(fb.FFTError) as ei:                  # FP16 flag on a complex64 plan
        fb.plan_query(4096, 1, opts=fb.make_opts(flags=fb.VARIANT_FP16_STORAGE | 35))
    assert ei.value.status == 1
    with pytest.raises(fb.FFTError) as ei:                  # complex64 kernel on an FP16 plan
        fb.plan_query(4096, 1, opts=fb.make_opts(flags=35, storage=fb.STORAGE_F16))
    assert ei.value.status == 1
    d = fb.plan_query(4096, 1, opts=fb.make_opts(device_twiddles=True))
    assert d["device_twiddles"] == 1 and d["storage"] == 0


def test_plan_twiddles_argument_errors_without_device():
    lib = fb.load()
    cnt = ctypes.c_size_t(7)
    assert lib.fft_plan_twiddles(None, None, 0, ctypes.byref(cnt)) == 5
    assert lib.fft_plan_twiddles(ctypes.c_void_p(0xdead0), None, 0, ctypes.byref(cnt)) == 5


def test_filter_planning_without_device():
    for n in (64, 1024, 8192, 16384):
        d = fb.filter_query(n, 7, 625 if n >= 1024 else n // 2)
        assert d["path"] == fb.PATH_FILTER and d["kernel_name"].startswith("range_compress<")
        assert d["workspace_bytes"] == 0 and d["kernels_per_execute"] == 1
        assert d["twiddle_bytes"] >= 8 * n          # stage table + the replica spectrum
    for args, status in (((8192, 0, 10), 1), ((8192, 1, 0), 1), ((8192, 1, 8193), 1),
                         ((100, 1, 10), 2), ((32, 1, 10), 2), ((32768, 1, 10), 2)):
        with pytest.raises(fb.FFTError) as ei:
            fb.filter_query(*args)
        assert ei.value.status == status, args
    with pytest.raises(fb.FFTError) as ei:
        fb.filter_query(8192, 1, 10, fb.make_opts(storage=fb.STORAGE_F16))
    assert ei.value.status == 1
    lib = fb.load()
    h = ctypes.c_void_p(5)
    assert lib.fft_filter_create(8192, 1, None, 10, None, ctypes.byref(h)) == 1
    assert lib.fft_filter_create(8192, 1, ctypes.c_void_p(0x10004), 10, None, ctypes.byref(h)) == 1
    assert lib.fft_filter_create(8192, 1, ctypes.c_void_p(0x10000), 10, None, None) == 1
    assert h.value is None


def test_every_handle_entry_point_rejects_null_and_unknown_handles():
    lib = fb.load()
    vp = ctypes.c_void_p
    bogus = vp(0xdead0)
    u64 = ctypes.c_uint64()
    for h in (None, bogus):
        assert lib.fft_execute_ex(h, 1, vp(16), vp(16), None, None) == 5
        assert lib.fft_execute_pass(h, 1, vp(16), vp(16), None) == 5
        assert lib.fft_execute_pass_timed(h, 1, vp(16), vp(16), None, vp(8), vp(8)) == 5
        assert lib.fft_plan_twiddles(h, None, 0, ctypes.byref(ctypes.c_size_t())) == 5
        assert lib.fft_ragged_execute(h, vp(16), vp(16), None, 0) == 5
        assert lib.fft_ragged_describe(h, None, None) == 5
        assert lib.fft_ragged_destroy(h) == 5
        assert lib.fft_sched_submit(h, 1, 8, 1, -1, 16, 1, 0.0) == 5
        assert lib.fft_sched_destroy(h) == 5
        assert lib.fft_server_submit(h, 8, 1, -1, vp(16), None, ctypes.byref(u64)) == 5
        assert lib.fft_server_wait(h, 1, 0.0, None, None) == 5
        assert lib.fft_server_release(h, 1) == 5
        assert lib.fft_server_drain(h, 0.0) == 5
        assert lib.fft_server_destroy(h) == 5
        assert lib.fft_server_clock(h) == -1.0
    # events: null arguments are rejected before any HIP call
    assert lib.fft_event_create(None) == 1
    assert lib.fft_event_destroy(None) == 1
    assert lib.fft_event_elapsed(None, None, None) == 1


def test_scheduler_host_only_lifecycle():
    # the scheduler makes no HIP call: it runs here without a device
    from paper_1505_08067_amd import serving as sv
    with sv.Scheduler(hbm_budget=1 << 20) as s:
        s.submit(1, 1024, 2, fb.FORWARD, 32768, True, 0.0)
        L = s.next(0.0)
        assert L["requests"] == [1] and L["batch"] == 2
        s.complete(L["id"], 0.5)
        assert s.request(1)["state"] == fb.REQ_DONE and s.stats()["completed"] == 1


def test_small_batches_take_the_one_wave_form():
    # fewer than 128 workgroups of the full-width kernel: the narrowest compiled
    # form of the same schedule and variant; otherwise the full-width default
    ks = {k["name"]: k for k in fb.kernels()}
    for n in (16, 32, 64, 128, 256, 512, 1024, 2048, 1000, 3072):
        wide = fb.plan_query(n, 1 << 16)
        kw = ks[wide["kernel_name"]]
        assert kw["is_default"], n
        small_batch = 127 * kw["c"]                    # 127 workgroups
        full_batch = 127 * kw["c"] + 1                 # 128 workgroups
        narrow = fb.plan_query(n, small_batch)
        kn = ks[narrow["kernel_name"]]
        assert kn["c"] < kw["c"] and kn["radix"] == kw["radix"] and kn["flags"] == kw["flags"], n
        assert kn["threads"] < kw["threads"]
        assert narrow["transforms_per_block"] == kn["c"]
        assert fb.plan_query(n, full_batch)["kernel_name"] == kw["name"], n
    # lengths without a narrower form, FP16 storage and explicit options keep the default
    assert fb.plan_query(4096, 1)["kernel_name"] == fb.plan_query(4096, 4096)["kernel_name"]
    assert fb.plan_query(1024, 1, opts=fb.make_opts(storage=fb.STORAGE_F16))["transforms_per_block"] == 4
    assert fb.plan_query(1024, 1, opts=fb.make_opts(radix=[16, 16, 4], flags=35))["transforms_per_block"] == 4
    # wisdom names one kernel for every batch
    fb.wisdom_clear()
    alt = ks[fb.plan_query(1024, 1 << 16)["kernel_name"]]
    fb.wisdom_set(1024, alt["name"])
    try:
        assert fb.plan_query(1024, 8)["kernel_name"] == alt["name"]
    finally:
        fb.wisdom_clear()


def test_variant_constants_match_the_header():
    import re
    text = open(HEADER).read()
    defs = dict((m.group(1), int(m.group(2))) for m in re.finditer(r"#define FFT_VARIANT_(\w+)\s+(\d+)", text))
    assert defs, "no variant flags found"
    for name, value in defs.items():
        assert getattr(fb, "VARIANT_" + name) == value, name


def test_kernel_names_are_unique():
    # wisdom, fft_kernel_occupancy and the kernel-trace summaries resolve a
    # kernel by its name, so no two catalogue entries may share one (a
    # 1024-thread form of 16384 with two transforms per workgroup once carried
    # the name of the 512-thread default and was found in its place)
    names = [k["name"] for k in fb.kernels()]
    dup = sorted({n for n in names if names.count(n) > 1})
    assert not dup, dup
    # and a name recorded as wisdom plans exactly that entry
    k2 = next(k for k in fb.kernels() if k["n"] == 16384 and k["c"] == 2 and k["kind"] == "block"
              and not k["flags"] & fb.VARIANT_FP16_STORAGE)
    k1 = next(k for k in fb.kernels() if k["n"] == 16384 and k["is_default"] and k["kind"] == "block"
              and not k["flags"] & fb.VARIANT_FP16_STORAGE)
    assert k1["c"] == 1 and k1["name"] != k2["name"]
    fb.wisdom_clear()
    try:
        fb.wisdom_set(16384, k1["name"])
        d = fb.plan_query(16384, 1024)
        assert d["kernel_name"] == k1["name"] and d["transforms_per_block"] == 1
    finally:
        fb.wisdom_clear()


def test_output_scale_option():
    # 0 means none (1); any finite value is kept; NaN and infinities are refused;
    # ragged plans take no scale
    assert fb.plan_query(4096, 8)["scale"] == 1.0
    assert fb.plan_query(4096, 8, fb.BACKWARD, opts=fb.make_opts(scale=1.0 / 4096))["scale"] == 2.0 ** -12
    assert fb.plan_query(1 << 20, 2, opts=fb.make_opts(scale=-0.5))["scale"] == -0.5
    for bad in (float("nan"), float("inf"), -float("inf")):
        with pytest.raises(fb.FFTError) as ei:
            fb.plan_query(1024, 4, opts=fb.make_opts(scale=bad))
        assert ei.value.status == 1
    lib = fb.load()
    sizes, counts = (ctypes.c_size_t * 1)(1024), (ctypes.c_size_t * 1)(2)
    h = ctypes.c_void_p()
    o = fb.make_opts(scale=0.5)
    assert lib.fft_ragged_create_ex(sizes, counts, 1, fb.FORWARD, ctypes.byref(o), ctypes.byref(h)) == 1
    assert not h.value
