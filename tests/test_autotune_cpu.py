"""The C++ schedule search against the reference model and the paper's tables,
and the wisdom file, on the CPU (no device calls)."""
import math
import os
import random

import pytest

from oracle import plan_dag
from paper_1505_08067_amd import fftblock as fb


def _table(golden_dir, name):
    return plan_dag.load_stage_table(os.path.join(golden_dir, name))


@pytest.mark.parametrize("name,cost", [("stage_costs_ivybridge.txt", 19785), ("stage_costs_haswell.txt", 18218)])
def test_schedule_search_on_printed_tables(golden_dir, name, cost):
    c = _table(golden_dir, name)
    total, sched = fb.schedule_search(10, c, radices=(2, 4, 8))
    assert sched == [8, 8, 4, 4] and total == cost
    assert (total, sched) == plan_dag.dijkstra(10, c)


def test_schedule_search_matches_reference_on_random_tables():
    rnd = random.Random(11)
    for L in range(1, 13):
        for _ in range(5):
            costs = {(r, s): rnd.randint(1, 30) for r in (2, 4, 8, 16) for s in range(L)
                     if s + int(math.log2(r)) <= L}
            got = fb.schedule_search(L, costs)
            ref = plan_dag.dijkstra(L, costs, radices=(2, 4, 8, 16))
            assert got[0] == ref[0] and got[1] == ref[1], (L, costs)


def test_schedule_search_errors():
    with pytest.raises(fb.FFTError):
        fb.schedule_search(4, {}, radices=(2,))          # no edges: unreachable sink
    with pytest.raises(fb.FFTError):
        fb.schedule_search(4, {(3, 0): 1.0}, radices=(3,))  # not a power of two


def test_wisdom_roundtrip(tmp_path):
    fb.wisdom_clear()
    assert fb.wisdom_get(4096) is None
    alt = [k["name"] for k in fb.kernels() if k["kind"] == "block" and k["n"] == 4096 and not k["is_default"]][0]
    fb.wisdom_set(4096, alt)
    assert fb.wisdom_get(4096) == alt
    assert fb.plan_query(4096, 8)["kernel_name"] == alt
    p = tmp_path / "w.txt"
    fb.wisdom_save(str(p))
    fb.wisdom_clear()
    assert fb.plan_query(4096, 8)["kernel_name"] != alt
    fb.wisdom_load(str(p))
    assert fb.wisdom_get(4096) == alt
    # a stale entry is skipped and reported
    p.write_text("4096 block_fft<4096,[no such],v0>\n1024 " + fb.plan_query(1024, 1)["kernel_name"] + "\n")
    fb.wisdom_clear()
    with pytest.raises(fb.FFTError):
        fb.wisdom_load(str(p))
    assert fb.wisdom_get(4096) is None and fb.wisdom_get(1024) is not None
    fb.wisdom_clear()
    with pytest.raises(fb.FFTError):
        fb.wisdom_set(4096, [k["name"] for k in fb.kernels() if k["n"] == 1024][0])


def test_wisdom_pair_for_fourstep(tmp_path):
    fb.wisdom_clear()
    ks = [k for k in fb.kernels() if not k["flags"] & fb.VARIANT_FP16_STORAGE]   # wisdom is for complex64
    p1 = [k["name"] for k in ks if k["kind"] == "pass1" and k["n"] == 1024 and not k["is_default"] and k["c"] == 8][0]
    p2 = [k["name"] for k in ks if k["kind"] == "pass2" and k["n"] == 1024 and not k["is_default"] and k["c"] == 16][0]
    path = tmp_path / "w.txt"
    path.write_text(f"1048576\t{p1}\t{p2}\n")
    fb.wisdom_load(str(path))
    d = fb.plan_query(1 << 20, 4)
    assert (d["kernel_name"], d["kernel_name2"]) == (p1, p2)
    assert d["transforms_per_block"] == 8 and d["c2"] == 16
    fb.wisdom_save(str(path))
    assert p1 in path.read_text() and p2 in path.read_text()
    fb.wisdom_clear()
    d = fb.plan_query(1 << 20, 4)
    assert (d["kernel_name"], d["kernel_name2"]) != (p1, p2)


def test_runtime_schedule_planning_without_device():
    # a schedule no compiled kernel has runs on the run-time-schedule kernel,
    # whose table follows the plan's schedule; a compiled one keeps its kernel
    import math
    d = fb.plan_query(1024, 64, opts=fb.make_opts(radix=[2, 16, 16, 2]))
    assert d["kernel_name"] == "block_fft_rt<1024>" and d["radix"] == [2, 16, 16, 2]
    assert d["flags"] & fb.VARIANT_RUNTIME_SCHEDULE
    # exact rows: stage s >= 1 holds Ns * R entries (2*16 + 32*16 + 512*2), padded to 32
    assert d["twiddle_bytes"] == 8 * ((32 + 512 + 1024 + 31) // 32 * 32)
    assert fb.plan_query(1024, 64, opts=fb.make_opts(radix=[16, 16, 4]))["kernel_name"].startswith("block_fft<1024")
    # ... unless the run-time-schedule kernel is asked for
    d = fb.plan_query(1024, 64, opts=fb.make_opts(radix=[16, 16, 4], flags=fb.VARIANT_RUNTIME_SCHEDULE | 3))
    assert d["kernel_name"] == "block_fft_rt<1024>" and d["radix"] == [16, 16, 4]
    for n, sched in ((64, [2] * 6), (256, [2] * 8), (4096, [2, 2, 2, 2, 16, 16]), (16384, [2, 2, 16, 16, 16])):
        d = fb.plan_query(n, 3, opts=fb.make_opts(radix=sched))
        assert d["kernel_name"] == f"block_fft_rt<{n}>" and d["radix"] == sched and math.prod(sched) == n
    for bad in ([32, 32], [16, 16], [3, 4, 4], [2] * 8):
        with pytest.raises(fb.FFTError) as ei:
            fb.plan_query(1024, 1, opts=fb.make_opts(radix=bad))
        assert ei.value.status == 2, bad
    with pytest.raises(fb.FFTError):      # complex64 only
        fb.plan_query(1024, 1, opts=fb.make_opts(radix=[2, 16, 16, 2], storage=fb.STORAGE_F16))


def test_wisdom_with_a_runtime_schedule(tmp_path):
    fb.wisdom_clear()
    path = tmp_path / "w.txt"
    path.write_text("1024\tblock_fft_rt<1024>:2,16,16,2\n")
    fb.wisdom_load(str(path))
    d = fb.plan_query(1024, 512)
    assert d["kernel_name"] == "block_fft_rt<1024>" and d["radix"] == [2, 16, 16, 2]
    fb.wisdom_save(str(path))
    assert "block_fft_rt<1024>:2,16,16,2" in path.read_text()
    # a schedule that does not multiply to the length is refused
    path.write_text("1024\tblock_fft_rt<1024>:16,16\n")
    with pytest.raises(fb.FFTError):
        fb.wisdom_load(str(path))
    fb.wisdom_clear()
    assert fb.plan_query(1024, 512)["kernel_name"] != "block_fft_rt<1024>"
