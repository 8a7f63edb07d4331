"""Python binding of the C ABI in ``include/fftblock.h`` (ctypes).

Argument marshalling only: every step of a transform runs in the HIP kernels
of ``libfftblock.so``.  PyTorch provides device memory and the stream
(``torch.cuda.current_stream()``).  There is no CPU fallback: if the library
is missing or a call fails, an exception is raised.

    plan = Plan(n, batch, FORWARD)        # fft_plan_create
    y = plan.execute(x)                   # fft_execute on the current stream
    t = transpose(m)                      # fft_transpose (corner turn)
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfftblock.so")

FORWARD = -1
BACKWARD = +1
PATH_BLOCK = 1
PATH_FOURSTEP = 2
PATH_FILTER = 3

STATUS = {
    0: "FFT_SUCCESS",
    1: "FFT_ERR_INVALID_ARG",
    2: "FFT_ERR_UNSUPPORTED_SIZE",
    3: "FFT_ERR_OUT_OF_MEMORY",
    4: "FFT_ERR_DEVICE",
    5: "FFT_ERR_INVALID_PLAN",
    6: "FFT_ERR_TIMEOUT",
    7: "FFT_ERR_SCRATCH_LIMIT",
}

# Every symbol include/fftblock.h declares.
EXPORTS = (
    "fft_plan_create", "fft_execute", "fft_execute_pass", "fft_transpose", "fft_plan_destroy", "fft_status_string",
    "fft_plan_describe", "fft_plan_query", "fft_device_query", "fft_block_max", "fft_block_limit",
    "fft_copy", "fft_plan_opts_init", "fft_plan_create_ex", "fft_plan_query_ex", "fft_kernel_count",
    "fft_kernel_info", "fft_kernel_occupancy", "fft_schedule_search", "fft_stage_benchmark", "fft_autotune",
    "fft_wisdom_set", "fft_wisdom_get", "fft_wisdom_clear", "fft_wisdom_save", "fft_wisdom_load",
    "fft_ragged_create", "fft_ragged_execute", "fft_ragged_describe", "fft_ragged_destroy",
    "fft_plan_twiddles", "fft_ragged_create_ex", "fft_filter_create", "fft_filter_query", "fft_execute_ex",
    "fft_sched_opts_init", "fft_sched_create", "fft_sched_destroy", "fft_sched_submit", "fft_sched_next",
    "fft_sched_complete", "fft_sched_request", "fft_sched_stats",
    "fft_execute_pass_timed", "fft_event_create", "fft_event_destroy", "fft_event_elapsed",
    "fft_server_opts_init", "fft_server_create", "fft_server_prepare", "fft_server_submit", "fft_server_wait",
    "fft_server_read", "fft_server_release", "fft_server_drain", "fft_server_stats", "fft_server_clock", "fft_server_destroy",
    "fft_execute_static", "fft_static_scratch_bytes", "fft_ragged_describe_ex",
)

VARIANT_NT_LOAD = 1
VARIANT_NT_STORE = 2
VARIANT_PERSISTENT = 4
VARIANT_SWIZZLE = 8
VARIANT_STAGED = 16
VARIANT_TWIDDLE_POWERS = 32
VARIANT_FP16_STORAGE = 64
VARIANT_XCD_ORDER = 128
VARIANT_STAGE_STRIDE = 256
VARIANT_WAVE_SYNC = 512
VARIANT_HALF_EXCHANGE = 1024
VARIANT_FIT_REGISTERS = 2048
VARIANT_LOOP = 4096
VARIANT_RUNTIME_SCHEDULE = 8192
VARIANT_VEC16 = 16384
VARIANT_CROSS_LANE = 32768
VARIANT_VAR_THREADS = 65536
VARIANT_FP16_WORKSPACE = 524288
STORAGE_C64 = 0
STORAGE_F16 = 1
STORAGE_F16_COMPACT = 2
KERNEL_KINDS = {0: "block", 1: "pass1", 2: "pass2", 3: "filter", 4: "list"}


class FFTError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_size_t), ("batch", ctypes.c_size_t),
        ("direction", ctypes.c_int), ("path", ctypes.c_int),
        ("n1", ctypes.c_size_t), ("n2", ctypes.c_size_t),
        ("n_radix", ctypes.c_int), ("radix", ctypes.c_int * 8),
        ("n_radix2", ctypes.c_int), ("radix2", ctypes.c_int * 8),
        ("threads_per_block", ctypes.c_int), ("transforms_per_block", ctypes.c_int),
        ("lds_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
        ("twiddle_bytes", ctypes.c_size_t), ("kernels_per_execute", ctypes.c_int),
        ("kernel_name", ctypes.c_char_p), ("kernel_name2", ctypes.c_char_p),
        ("flags", ctypes.c_int), ("flags2", ctypes.c_int), ("c2", ctypes.c_int),
        ("grid", ctypes.c_longlong), ("storage", ctypes.c_int), ("device_twiddles", ctypes.c_int),
        ("scale", ctypes.c_float),
    ]


class PlanOpts(ctypes.Structure):
    _fields_ = [
        ("block_limit", ctypes.c_size_t), ("n_radix", ctypes.c_int), ("radix", ctypes.c_int * 8),
        ("flags", ctypes.c_int), ("c", ctypes.c_int), ("flags2", ctypes.c_int), ("c2", ctypes.c_int),
        ("n1", ctypes.c_size_t), ("storage", ctypes.c_int), ("device_twiddles", ctypes.c_int),
        ("scale", ctypes.c_float),
    ]


class KernelInfo(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int), ("n", ctypes.c_int), ("e", ctypes.c_int), ("c", ctypes.c_int),
        ("flags", ctypes.c_int), ("n_radix", ctypes.c_int), ("radix", ctypes.c_int * 8),
        ("threads", ctypes.c_int), ("lds_bytes", ctypes.c_size_t), ("is_default", ctypes.c_int),
        ("name", ctypes.c_char_p),
    ]


class DeviceInfo(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int), ("arch", ctypes.c_char * 64),
        ("compute_units", ctypes.c_int), ("warp_size", ctypes.c_int),
        ("lds_per_cu", ctypes.c_size_t), ("lds_per_block", ctypes.c_size_t),
        ("global_mem", ctypes.c_size_t), ("clock_khz", ctypes.c_int),
        ("mem_clock_khz", ctypes.c_int), ("mem_bus_width", ctypes.c_int),
        ("block_max", ctypes.c_size_t * 3),
    ]


class TuneReport(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_size_t), ("log2n", ctypes.c_int),
        ("stage_cost", (ctypes.c_double * 16) * 4),
        ("predicted", ctypes.c_int * 16), ("n_predicted", ctypes.c_int), ("predicted_cost", ctypes.c_double),
        ("n_candidates", ctypes.c_int), ("candidate_kernel", ctypes.c_int * 32),
        ("candidate_kernel2", ctypes.c_int * 32),
        ("candidate_us", ctypes.c_double * 32), ("chosen_kernel", ctypes.c_int), ("chosen_kernel2", ctypes.c_int),
        ("chosen_us", ctypes.c_double), ("predicted_us", ctypes.c_double), ("chosen_schedule_rt_us", ctypes.c_double),
        ("chosen_predicted", ctypes.c_int),
    ]


class SchedOpts(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t), ("n_streams", ctypes.c_int), ("max_inflight", ctypes.c_int),
        ("max_coalesce", ctypes.c_int), ("max_transforms", ctypes.c_size_t), ("backfill_bytes", ctypes.c_size_t),
        ("small_streams", ctypes.c_int), ("small_bytes", ctypes.c_size_t),
    ]


LAUNCH_MAX_REQUESTS = 64
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_REJECTED = 0, 1, 2, 3


class Launch(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_longlong), ("stream", ctypes.c_int), ("n", ctypes.c_size_t), ("direction", ctypes.c_int),
        ("batch", ctypes.c_size_t), ("bytes", ctypes.c_size_t), ("n_requests", ctypes.c_int),
        ("requests", ctypes.c_uint64 * LAUNCH_MAX_REQUESTS),
    ]


class RequestInfo(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_uint64), ("n", ctypes.c_size_t), ("batch", ctypes.c_size_t), ("direction", ctypes.c_int),
        ("state", ctypes.c_int), ("bytes", ctypes.c_size_t), ("t_arrive", ctypes.c_double),
        ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double), ("launch", ctypes.c_longlong),
        ("stream", ctypes.c_int), ("group_size", ctypes.c_int),
    ]


class SchedStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_size_t), ("completed", ctypes.c_size_t), ("rejected", ctypes.c_size_t),
        ("queued", ctypes.c_size_t), ("running_launches", ctypes.c_size_t), ("launches", ctypes.c_size_t),
        ("coalesced_requests", ctypes.c_size_t), ("backfilled_requests", ctypes.c_size_t),
        ("inflight_bytes", ctypes.c_size_t),
        ("peak_inflight_bytes", ctypes.c_size_t), ("points", ctypes.c_double), ("t_last_done", ctypes.c_double),
        ("latency_p50", ctypes.c_double), ("latency_p99", ctypes.c_double), ("latency_mean", ctypes.c_double),
        ("latency_max", ctypes.c_double), ("queue_p50", ctypes.c_double), ("queue_p99", ctypes.c_double),
        ("device_p50", ctypes.c_double), ("device_p99", ctypes.c_double),
    ]


class ServerOpts(ctypes.Structure):
    _fields_ = [("sched", SchedOpts), ("arena_bytes", ctypes.c_size_t), ("auto_release", ctypes.c_int)]


class RaggedDesc(ctypes.Structure):
    _fields_ = [("total_points", ctypes.c_size_t), ("graph_nodes", ctypes.c_int),
                ("persistent_launches", ctypes.c_int), ("fallback_classes", ctypes.c_int),
                ("kernel_name", ctypes.c_char_p * 8), ("units", ctypes.c_uint * 8), ("grid", ctypes.c_uint * 8),
                ("classes", ctypes.c_int * 8), ("threads", ctypes.c_int * 8), ("lds_bytes", ctypes.c_size_t * 8),
                ("branch_graph_nodes", ctypes.c_size_t)]


RAGGED_PERSISTENT, RAGGED_PLAIN, RAGGED_BRANCHES = 0, 1, 2


def _struct_dict(st) -> dict:
    out = {}
    for name, _ in st._fields_:
        v = getattr(st, name)
        out[name] = list(v) if isinstance(v, ctypes.Array) else v
    return out


_lib = None


def load():
    """Load ``libfftblock.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1505_08067_amd/build.py "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    sz, vp, i = ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int
    lib.fft_plan_create.argtypes = [sz, sz, i, ctypes.POINTER(vp)]
    lib.fft_execute.argtypes = [vp, vp, vp, vp]
    lib.fft_execute_pass.argtypes = [vp, i, vp, vp, vp]
    lib.fft_transpose.argtypes = [vp, vp, sz, sz, sz, vp]
    lib.fft_plan_destroy.argtypes = [vp]
    lib.fft_status_string.argtypes = [i]
    lib.fft_status_string.restype = ctypes.c_char_p
    lib.fft_plan_describe.argtypes = [vp, ctypes.POINTER(PlanDesc)]
    lib.fft_plan_query.argtypes = [sz, sz, i, ctypes.POINTER(PlanDesc)]
    lib.fft_device_query.argtypes = [i, ctypes.POINTER(DeviceInfo)]
    lib.fft_block_max.argtypes = [sz, i]
    lib.fft_block_max.restype = sz
    lib.fft_block_limit.argtypes = []
    lib.fft_block_limit.restype = sz
    lib.fft_copy.argtypes = [vp, vp, sz, vp]
    lib.fft_plan_opts_init.argtypes = [ctypes.POINTER(PlanOpts)]
    lib.fft_plan_opts_init.restype = None
    lib.fft_plan_create_ex.argtypes = [sz, sz, i, ctypes.POINTER(PlanOpts), ctypes.POINTER(vp)]
    lib.fft_plan_query_ex.argtypes = [sz, sz, i, ctypes.POINTER(PlanOpts), ctypes.POINTER(PlanDesc)]
    lib.fft_filter_create.argtypes = [sz, sz, vp, sz, ctypes.POINTER(PlanOpts), ctypes.POINTER(vp)]
    lib.fft_execute_ex.argtypes = [vp, sz, vp, vp, vp, vp]
    lib.fft_execute_static.argtypes = [vp, sz, vp, vp, vp]
    lib.fft_static_scratch_bytes.argtypes = []
    lib.fft_static_scratch_bytes.restype = sz
    lib.fft_execute_pass_timed.argtypes = [vp, i, vp, vp, vp, vp, vp]
    lib.fft_event_create.argtypes = [ctypes.POINTER(vp)]
    lib.fft_event_destroy.argtypes = [vp]
    lib.fft_event_elapsed.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_float)]
    lib.fft_filter_query.argtypes = [sz, sz, sz, ctypes.POINTER(PlanOpts), ctypes.POINTER(PlanDesc)]
    lib.fft_kernel_count.argtypes = []
    lib.fft_kernel_count.restype = i
    lib.fft_kernel_info.argtypes = [i, ctypes.POINTER(KernelInfo)]
    lib.fft_kernel_occupancy.argtypes = [i, ctypes.POINTER(i)]
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.fft_schedule_search.argtypes = [i, ip, i, dp, ip, ip, dp]
    lib.fft_stage_benchmark.argtypes = [sz, i, i, i, dp]
    lib.fft_autotune.argtypes = [sz, sz, ctypes.POINTER(TuneReport)]
    lib.fft_wisdom_set.argtypes = [sz, i]
    lib.fft_wisdom_get.argtypes = [sz]
    lib.fft_wisdom_get.restype = i
    lib.fft_wisdom_clear.argtypes = []
    lib.fft_wisdom_clear.restype = None
    lib.fft_wisdom_save.argtypes = [ctypes.c_char_p]
    lib.fft_wisdom_load.argtypes = [ctypes.c_char_p]
    szp = ctypes.POINTER(ctypes.c_size_t)
    lib.fft_ragged_create.argtypes = [szp, szp, sz, i, ctypes.POINTER(vp)]
    lib.fft_ragged_execute.argtypes = [vp, vp, vp, vp, i]
    lib.fft_ragged_describe.argtypes = [vp, szp, szp]
    lib.fft_ragged_describe_ex.argtypes = [vp, ctypes.POINTER(RaggedDesc)]
    lib.fft_ragged_describe_ex.restype = ctypes.c_int
    lib.fft_ragged_destroy.argtypes = [vp]
    lib.fft_plan_twiddles.argtypes = [vp, vp, sz, szp]
    lib.fft_ragged_create_ex.argtypes = [szp, szp, sz, i, vp, ctypes.POINTER(vp)]
    lib.fft_ragged_create_ex.restype = ctypes.c_int
    lib.fft_plan_twiddles.restype = ctypes.c_int
    u64, dbl = ctypes.c_uint64, ctypes.c_double
    lib.fft_sched_opts_init.argtypes = [ctypes.POINTER(SchedOpts)]
    lib.fft_sched_opts_init.restype = None
    lib.fft_sched_create.argtypes = [ctypes.POINTER(SchedOpts), ctypes.POINTER(vp)]
    lib.fft_sched_destroy.argtypes = [vp]
    lib.fft_sched_submit.argtypes = [vp, u64, sz, sz, i, sz, i, dbl]
    lib.fft_sched_next.argtypes = [vp, dbl, ctypes.POINTER(Launch), ctypes.POINTER(i)]
    lib.fft_sched_complete.argtypes = [vp, ctypes.c_longlong, dbl]
    lib.fft_sched_request.argtypes = [vp, u64, ctypes.POINTER(RequestInfo)]
    lib.fft_sched_stats.argtypes = [vp, ctypes.POINTER(SchedStats)]
    lib.fft_server_opts_init.argtypes = [ctypes.POINTER(ServerOpts)]
    lib.fft_server_opts_init.restype = None
    lib.fft_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    lib.fft_server_prepare.argtypes = [vp, sz, i]
    lib.fft_server_submit.argtypes = [vp, sz, sz, i, vp, vp, ctypes.POINTER(u64)]
    lib.fft_server_wait.argtypes = [vp, u64, dbl, ctypes.POINTER(vp), ctypes.POINTER(RequestInfo)]
    lib.fft_server_release.argtypes = [vp, u64]
    lib.fft_server_read.argtypes = [vp, u64, vp, vp]
    lib.fft_server_drain.argtypes = [vp, dbl]
    lib.fft_server_stats.argtypes = [vp, ctypes.POINTER(SchedStats)]
    lib.fft_server_clock.argtypes = [vp]
    lib.fft_server_clock.restype = dbl
    lib.fft_server_destroy.argtypes = [vp]
    for name in ("fft_schedule_search", "fft_stage_benchmark", "fft_autotune", "fft_wisdom_set",
                 "fft_wisdom_save", "fft_wisdom_load", "fft_ragged_create", "fft_ragged_execute",
                 "fft_ragged_describe", "fft_ragged_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("fft_plan_create", "fft_execute", "fft_execute_pass", "fft_transpose", "fft_plan_destroy",
                 "fft_plan_describe", "fft_plan_query", "fft_device_query", "fft_copy",
                 "fft_plan_create_ex", "fft_plan_query_ex", "fft_kernel_info", "fft_kernel_occupancy"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int, where: str) -> None:
    if status != 0:
        raise FFTError(status, where)


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _record(stream, *tensors) -> None:
    """Work queued on a stream other than the current one: the caching
    allocator must not hand these tensors' blocks out again before that
    stream has used them."""
    if stream is None:
        return
    import torch
    for t in tensors:
        if stream != torch.cuda.current_stream(t.device):
            t.record_stream(stream)


def _check_tensor(x, name: str, storage: int = 0):
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    want = torch.complex64 if storage == 0 else torch.complex32
    if x.dtype != want:
        raise TypeError(f"{name} must be {want}, got {x.dtype}")
    if not x.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if x.data_ptr() % 8:
        raise ValueError(f"{name} must be 8-byte aligned")


def _desc_dict(d: "PlanDesc") -> dict:
    return {
        "n": d.n, "batch": d.batch, "direction": d.direction, "path": d.path,
        "n1": d.n1, "n2": d.n2,
        "radix": list(d.radix[: d.n_radix]), "radix2": list(d.radix2[: d.n_radix2]),
        "threads_per_block": d.threads_per_block, "transforms_per_block": d.transforms_per_block,
        "lds_bytes": d.lds_bytes, "workspace_bytes": d.workspace_bytes,
        "twiddle_bytes": d.twiddle_bytes, "kernels_per_execute": d.kernels_per_execute,
        "kernel_name": d.kernel_name.decode() if d.kernel_name else None,
        "kernel_name2": d.kernel_name2.decode() if d.kernel_name2 else None,
        "flags": d.flags, "flags2": d.flags2, "c2": d.c2, "grid": d.grid,
        "storage": d.storage, "device_twiddles": d.device_twiddles, "scale": d.scale,
    }


def make_opts(block_limit=0, radix=None, flags=-1, c=0, flags2=-1, c2=0, storage=0, device_twiddles=False, n1=0,
              scale=0.0):
    """Planner options (``fft_plan_opts_t``); every default means "planner's choice".
    ``scale`` multiplies every output in the last store (0: none; ``1.0 / n`` with
    BACKWARD gives the normalised inverse)."""
    o = PlanOpts()
    load().fft_plan_opts_init(ctypes.byref(o))
    o.block_limit = block_limit
    if radix:
        o.n_radix = len(radix)
        for k, r in enumerate(radix):
            o.radix[k] = r
    o.flags, o.c, o.flags2, o.c2 = flags, c, flags2, c2
    o.storage, o.device_twiddles = storage, 1 if device_twiddles else 0
    o.n1 = int(n1)
    o.scale = float(scale)
    return o


def kernels() -> list:
    """The compiled transform kernels (``fft_kernel_count`` / ``fft_kernel_info``)."""
    lib = load()
    out = []
    for idx in range(lib.fft_kernel_count()):
        k = KernelInfo()
        _check(lib.fft_kernel_info(idx, ctypes.byref(k)), "fft_kernel_info")
        out.append({"kind": KERNEL_KINDS[k.kind], "n": k.n, "e": k.e, "c": k.c, "flags": k.flags,
                    "radix": list(k.radix[: k.n_radix]), "threads": k.threads, "lds_bytes": k.lds_bytes,
                    "is_default": bool(k.is_default), "name": k.name.decode()})
    return out


def kernel_occupancy(name: str) -> int:
    """Workgroups per compute unit of the named catalogue kernel on the current
    device (``fft_kernel_occupancy``)."""
    lib = load()
    for idx in range(lib.fft_kernel_count()):
        k = KernelInfo()
        _check(lib.fft_kernel_info(idx, ctypes.byref(k)), "fft_kernel_info")
        if k.name.decode() == name:
            occ = ctypes.c_int()
            _check(lib.fft_kernel_occupancy(idx, ctypes.byref(occ)), "fft_kernel_occupancy")
            return occ.value
    raise FFTError(f"no kernel named {name}")


def plan_query(n: int, batch: int, direction: int = FORWARD, opts: "PlanOpts | None" = None) -> dict:
    """What ``fft_plan_create`` would choose, without a device (``fft_plan_query[_ex]``)."""
    d = PlanDesc()
    if opts is None:
        st = load().fft_plan_query(n, batch, direction, ctypes.byref(d))
    else:
        st = load().fft_plan_query_ex(n, batch, direction, ctypes.byref(opts), ctypes.byref(d))
    _check(st, f"fft_plan_query(n={n})")
    return _desc_dict(d)


class Plan:
    """Batched 1-D complex64 FFT plan (``fft_plan_create``)."""

    def __init__(self, n: int, batch: int, direction: int = FORWARD, opts: "PlanOpts | None" = None):
        lib = load()
        h = ctypes.c_void_p()
        if opts is None:
            st = lib.fft_plan_create(n, batch, direction, ctypes.byref(h))
        else:
            st = lib.fft_plan_create_ex(n, batch, direction, ctypes.byref(opts), ctypes.byref(h))
        _check(st, f"fft_plan_create(n={n}, batch={batch})")
        self._h = h
        self.n, self.batch, self.direction = int(n), int(batch), int(direction)
        self.storage = int(opts.storage) if opts is not None else 0

    @property
    def handle(self):
        return self._h

    def describe(self) -> dict:
        d = PlanDesc()
        _check(load().fft_plan_describe(self._h, ctypes.byref(d)), "fft_plan_describe")
        return _desc_dict(d)

    def execute(self, x, out=None, stream=None):
        """Transform ``x`` (complex64, ``batch*n`` values) into ``out`` (new tensor if None)."""
        import torch
        _check_tensor(x, "x", self.storage)
        if x.numel() != self.n * self.batch:
            raise ValueError(f"x has {x.numel()} values, plan expects {self.n * self.batch}")
        if out is None:
            out = torch.empty_like(x)
        _check_tensor(out, "out", self.storage)
        if out.numel() != x.numel():
            raise ValueError("out has the wrong size")
        if out.device != x.device:
            raise ValueError("x and out are on different devices")
        st = _stream_handle(stream)
        _check(load().fft_execute(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), st),
               "fft_execute")
        _record(stream, x, out)
        return out

    def execute_ptr(self, in_ptr: int, out_ptr: int, stream_handle: int = 0) -> None:
        """Raw-pointer variant (device addresses as ints) for benchmarks."""
        _check(load().fft_execute(self._h, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                                  ctypes.c_void_p(stream_handle)), "fft_execute")

    def execute_pass_timed_ptr(self, pass_: int, in_ptr: int, out_ptr: int, stream_handle, start, stop) -> None:
        """``fft_execute_pass_timed``: the device stamps ``start`` / ``stop`` (Event objects) at the
        kernel's own start and end."""
        _check(load().fft_execute_pass_timed(self._h, pass_, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                                             ctypes.c_void_p(stream_handle), start.handle, stop.handle),
               f"fft_execute_pass_timed({pass_})")

    def execute_pass_ptr(self, pass_: int, in_ptr: int, out_ptr: int, stream_handle: int = 0) -> None:
        """Run one kernel of the plan (``fft_execute_pass``): 1 = block / four-step pass 1, 2 = pass 2."""
        _check(load().fft_execute_pass(self._h, pass_, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                                       ctypes.c_void_p(stream_handle)), f"fft_execute_pass({pass_})")

    def twiddles(self):
        """The plan's twiddle table as a complex64 numpy array (``fft_plan_twiddles``)."""
        import numpy as np
        cnt = ctypes.c_size_t()
        _check(load().fft_plan_twiddles(self._h, None, 0, ctypes.byref(cnt)), "fft_plan_twiddles")
        out = np.zeros(cnt.value, dtype=np.complex64)
        if cnt.value:
            _check(load().fft_plan_twiddles(self._h, ctypes.c_void_p(out.ctypes.data), cnt.value, ctypes.byref(cnt)),
                   "fft_plan_twiddles")
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().fft_plan_destroy(self._h), "fft_plan_destroy")
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


class Event:
    """A timing event of the library's HIP runtime (``fft_event_*``)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(load().fft_event_create(ctypes.byref(h)), "fft_event_create")
        self.handle = h

    def elapsed_ms(self, stop: "Event") -> float:
        """Milliseconds from this event to ``stop`` (waits for ``stop``)."""
        ms = ctypes.c_float()
        _check(load().fft_event_elapsed(self.handle, stop.handle, ctypes.byref(ms)), "fft_event_elapsed")
        return ms.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().fft_event_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def filter_query(n: int, batch: int, replica_len: int, opts: "PlanOpts | None" = None) -> dict:
    """What ``fft_filter_create`` would choose, without a device."""
    d = PlanDesc()
    _check(load().fft_filter_query(n, batch, replica_len, ctypes.byref(opts) if opts is not None else None,
                                   ctypes.byref(d)), f"fft_filter_query(n={n})")
    return _desc_dict(d)


class RangeCompressor(Plan):
    """Range compression of ``batch`` rows of length ``n`` against a pulse
    replica (``fft_filter_create``): ``y = B(F(x) * conj(F(replica)))`` per
    row, i.e. ``n`` times the circular cross-correlation with the replica,
    in one kernel.  ``replica`` is a complex64 CUDA tensor of at most ``n``
    values; it is only read while the plan is created."""

    def __init__(self, n: int, batch: int, replica, opts: "PlanOpts | None" = None):
        import torch
        _check_tensor(replica, "replica")
        if not replica.is_cuda or not replica.is_contiguous():
            raise ValueError("replica must be a contiguous CUDA tensor")
        h = ctypes.c_void_p()
        torch.cuda.synchronize(replica.device)
        _check(load().fft_filter_create(n, batch, ctypes.c_void_p(replica.data_ptr()), replica.numel(),
                                        ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)),
               f"fft_filter_create(n={n}, batch={batch})")
        self._h = h
        self.n, self.batch, self.direction = int(n), int(batch), FORWARD
        self.storage = STORAGE_C64


def transpose(x, out=None, stream=None):
    """Corner turn of the last two axes: ``out[..., c, r] = x[..., r, c]`` (``fft_transpose``)."""
    import torch
    _check_tensor(x, "x")
    if x.dim() < 2:
        raise ValueError("need at least two dimensions")
    rows, cols = x.shape[-2], x.shape[-1]
    batch = x.numel() // (rows * cols) if rows * cols else 0
    if out is None:
        out = torch.empty(x.shape[:-2] + (cols, rows), dtype=x.dtype, device=x.device)
    _check_tensor(out, "out")
    _check(load().fft_transpose(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                rows, cols, batch, _stream_handle(stream)), "fft_transpose")
    _record(stream, x, out)
    return out


def copy_(dst, src, stream=None):
    """HBM copy probe (``fft_copy``): byte copy of ``src`` into ``dst``."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    _check(load().fft_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                           _stream_handle(stream)), "fft_copy")
    _record(stream, src, dst)
    return dst


def device_query(device: int = -1) -> dict:
    info = DeviceInfo()
    _check(load().fft_device_query(device, ctypes.byref(info)), "fft_device_query")
    return {
        "device": info.device, "arch": info.arch.decode(), "compute_units": info.compute_units,
        "warp_size": info.warp_size, "lds_per_cu": info.lds_per_cu, "lds_per_block": info.lds_per_block,
        "global_mem": info.global_mem, "clock_khz": info.clock_khz, "mem_clock_khz": info.mem_clock_khz,
        "mem_bus_width": info.mem_bus_width, "block_max": list(info.block_max),
    }


def block_limit() -> int:
    return int(load().fft_block_limit())


def status_string(status: int) -> str:
    return load().fft_status_string(status).decode()


# ------------------------------------------------------------ schedule search
RADICES = (2, 4, 8, 16)


def schedule_search(log2n: int, costs: dict, radices=RADICES):
    """Shortest path over the stage DAG (``fft_schedule_search``).

    ``costs`` maps (radix, start_stage) to a cost; missing entries are absent
    edges.  Returns (total cost, radix list).
    """
    lib = load()
    nr = len(radices)
    arr = (ctypes.c_double * (nr * log2n))(*([-1.0] * (nr * log2n)))
    for i, r in enumerate(radices):
        for s_ in range(log2n):
            if (r, s_) in costs:
                arr[i * log2n + s_] = float(costs[(r, s_)])
    rad = (ctypes.c_int * nr)(*radices)
    out = (ctypes.c_int * max(1, log2n))()
    n_out = ctypes.c_int()
    total = ctypes.c_double()
    _check(lib.fft_schedule_search(log2n, rad, nr, arr, out, ctypes.byref(n_out), ctypes.byref(total)),
           "fft_schedule_search")
    return total.value, list(out[: n_out.value])


def stage_benchmark(n: int, radix: int, start_stage: int, reps: int = 8) -> float:
    """GPU cost of one radix stage in ns per transform (``fft_stage_benchmark``)."""
    v = ctypes.c_double()
    _check(load().fft_stage_benchmark(n, radix, start_stage, reps, ctypes.byref(v)), "fft_stage_benchmark")
    return v.value


def autotune(n: int, batch: int) -> dict:
    """Stage model + whole-kernel validation for length n (``fft_autotune``); updates the wisdom."""
    r = TuneReport()
    _check(load().fft_autotune(n, batch, ctypes.byref(r)), f"fft_autotune({n})")
    names = kernels()
    stage = {}
    for i, rad in enumerate(RADICES):
        for s_ in range(16):
            if r.stage_cost[i][s_] >= 0:
                stage[(rad, s_)] = r.stage_cost[i][s_]
    return {
        "n": r.n, "log2n": r.log2n, "stage_cost": stage,
        "predicted": list(r.predicted[: r.n_predicted]), "predicted_cost": r.predicted_cost,
        "candidates": [(names[r.candidate_kernel[k]]["name"] +
                        ("+" + names[r.candidate_kernel2[k]]["name"] if r.candidate_kernel2[k] >= 0 else ""),
                        r.candidate_us[k]) for k in range(r.n_candidates)],
        "chosen": (names[r.chosen_kernel]["name"] +
                   ("+" + names[r.chosen_kernel2]["name"] if r.chosen_kernel2 >= 0 else "") +
                   (":" + ",".join(str(v) for v in r.predicted[: r.n_predicted]) if r.chosen_predicted else ""))
        if r.chosen_kernel >= 0 else None,
        "chosen_us": r.chosen_us,
        "predicted_us": r.predicted_us if r.predicted_us >= 0 else None,
        "chosen_schedule_rt_us": r.chosen_schedule_rt_us if r.chosen_schedule_rt_us >= 0 else None,
        "chosen_predicted": bool(r.chosen_predicted),
    }


def wisdom_set(n: int, kernel_name: str) -> None:
    names = [k["name"] for k in kernels()]
    _check(load().fft_wisdom_set(n, names.index(kernel_name)), "fft_wisdom_set")


def wisdom_get(n: int):
    idx = load().fft_wisdom_get(n)
    return None if idx < 0 else kernels()[idx]["name"]


def wisdom_clear() -> None:
    load().fft_wisdom_clear()


def wisdom_save(path: str) -> None:
    _check(load().fft_wisdom_save(path.encode()), "fft_wisdom_save")


def wisdom_load(path: str) -> None:
    _check(load().fft_wisdom_load(path.encode()), "fft_wisdom_load")


# ------------------------------------------------------------------- ragged
class Ragged:
    """Batches of several lengths in one submission (``fft_ragged_*``).

    ``classes`` is a list of (length, count); the data of one execute is the
    concatenation of the classes' batches in that order.
    """

    def __init__(self, classes, direction: int = FORWARD, storage: int = STORAGE_C64, device_twiddles: bool = False):
        lib = load()
        self.classes = [(int(n), int(c)) for n, c in classes]
        k = len(self.classes)
        sizes = (ctypes.c_size_t * k)(*[n for n, _ in self.classes])
        counts = (ctypes.c_size_t * k)(*[c for _, c in self.classes])
        h = ctypes.c_void_p()
        if storage == STORAGE_C64 and not device_twiddles:
            st = lib.fft_ragged_create(sizes, counts, k, direction, ctypes.byref(h))
        else:
            o = make_opts(storage=storage, device_twiddles=device_twiddles)
            st = lib.fft_ragged_create_ex(sizes, counts, k, direction, ctypes.byref(o), ctypes.byref(h))
        _check(st, "fft_ragged_create")
        self.storage = storage
        self._h = h
        self.direction = direction
        self.total_points = sum(n * c for n, c in self.classes)

    def offsets(self):
        out, at = [], 0
        for n, c in self.classes:
            out.append(at)
            at += n * c
        return out

    def execute(self, x, out=None, stream=None, graph: bool = True, mode=None):
        """mode: RAGGED_PERSISTENT (default; graph=False means RAGGED_PLAIN),
        RAGGED_PLAIN or RAGGED_BRANCHES (``fft_ragged_execute``)."""
        import torch
        if mode is None:
            mode = RAGGED_PERSISTENT if graph else RAGGED_PLAIN
        _check_tensor(x, "x", self.storage)
        if x.numel() != self.total_points:
            raise ValueError(f"x has {x.numel()} values, ragged plan expects {self.total_points}")
        if out is None:
            out = torch.empty_like(x)
        _check_tensor(out, "out", self.storage)
        _check(load().fft_ragged_execute(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         _stream_handle(stream), int(mode)), "fft_ragged_execute")
        _record(stream, x, out)
        return out

    def describe(self) -> dict:
        tp, gn = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().fft_ragged_describe(self._h, ctypes.byref(tp), ctypes.byref(gn)), "fft_ragged_describe")
        d = RaggedDesc()
        _check(load().fft_ragged_describe_ex(self._h, ctypes.byref(d)), "fft_ragged_describe_ex")
        k = d.persistent_launches
        launches = [{"kernel": d.kernel_name[i].decode(), "units": d.units[i], "grid": d.grid[i],
                     "classes": d.classes[i], "threads": d.threads[i], "lds_bytes": d.lds_bytes[i]}
                    for i in range(min(k, 8))]
        return {"total_points": tp.value, "graph_nodes": gn.value, "classes": list(self.classes),
                "kernel_nodes": d.graph_nodes, "persistent_launches": launches,
                "fallback_classes": d.fallback_classes, "branch_graph_nodes": d.branch_graph_nodes}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().fft_ragged_destroy(self._h), "fft_ragged_destroy")
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
