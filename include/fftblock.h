/*
 * fftblock.h -- C ABI of the MI355X (gfx950) batched complex FFT library.
 *
 * The library computes batched one-dimensional discrete Fourier transforms of
 * single-precision complex data, following the definition in the paper's
 * Background section ("FFT Basics"):
 *
 *     X(k) = sum_{n=0}^{N-1} x(n) * w_N^{n k},   w_N = exp(-2 i pi / N)
 *
 * and the backward transform obtained by flipping the sign of the exponent.
 * Neither direction is normalised: backward(forward(x)) = N * x, unless the
 * planner option `scale` (fft_plan_opts_t) multiplies the outputs, e.g. by 1/N
 * for the normalised inverse.
 *
 * Method (paper, Approach): one elementary FFT block sized to what one
 * compute unit holds on chip (registers + the 160 KB LDS of a gfx950 CU) runs
 * a whole transform per workgroup ("Top level analysis": read, compute,
 * write).  Longer transforms are composed from two layers of such blocks by
 * the four-step split N = N1 * N2 ("Other FFT sizes": larger FFTs from the
 * fixed block): N2 column transforms of length N1 with a fused twiddle
 * multiply, then N1 row transforms of length N2 with the corner turn fused
 * into the store.  The data transpose used between the range and azimuth
 * passes of the radar chain ("Radar application description") is
 * fft_transpose.
 *
 * Data conventions (all entry points):
 *   - complex values are interleaved (re, im) pairs of IEEE float32, 8 bytes
 *     each (the layout of float2 and of torch.complex64);
 *   - a batch is contiguous and batch-major: element k of transform b is at
 *     index b * n + k;
 *   - pointers named `in`/`out` are DEVICE pointers on the plan's device;
 *     `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *   - output is always in natural order.
 *
 * Errors: every call returns an fft_status_t; nothing is thrown across the
 * ABI.  Argument checks run before any HIP call.  Launches are asynchronous:
 * a kernel fault surfaces at the caller's next synchronisation, not here.
 * Thread safety: distinct plans may be used from distinct host threads; one
 * plan must not be executed concurrently (it owns one workspace).
 */
#ifndef FFTBLOCK_H
#define FFTBLOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fft_plan_s* fft_plan_t;   /* opaque; created and freed by this API */

typedef enum {
    FFT_SUCCESS = 0,
    FFT_ERR_INVALID_ARG = 1,       /* zero size/batch, bad direction, null pointer, overlap */
    FFT_ERR_UNSUPPORTED_SIZE = 2,  /* a length the library has no kernels for */
    FFT_ERR_OUT_OF_MEMORY = 3,     /* hipMalloc failed */
    FFT_ERR_DEVICE = 4,            /* any other HIP runtime error (launch, copy, device query) */
    FFT_ERR_INVALID_PLAN = 5,      /* null or destroyed plan (or scheduler / server) handle */
    FFT_ERR_TIMEOUT = 6,           /* a wait of the serving layer ran out of time */
    FFT_ERR_SCRATCH_LIMIT = 7      /* fft_execute_static: the workspace exceeds the static scratch */
} fft_status_t;

/* Direction = sign of the exponent in the definition above. */
#define FFT_FORWARD (-1)
#define FFT_BACKWARD (+1)

/* Execution path chosen by the planner. */
#define FFT_PATH_BLOCK 1      /* one LDS-resident block per transform (N <= block limit 32768) */
#define FFT_PATH_FOURSTEP 2   /* two block passes, N = N1 * N2 */
#define FFT_PATH_FILTER 3     /* range compression: forward, filter, backward in one block */

/*
 * fft_plan_create -- plan `batch` transforms of length `n` in `direction`
 * on the calling thread's current HIP device.
 *
 *   n          transform length: powers of two from 1 to 2^22 (the single
 *              block path covers n <= the LDS block limit, longer lengths
 *              use the four-step path), and the compiled mixed-radix lengths
 *              3, 5, 6, 10, 12, 15, 20, 60, 100, 1000, 3072, 6000 and 15360
 *              (single block).  Other lengths: UNSUPPORTED_SIZE.  Long
 *              blocks hold a large share of a compute unit's LDS per
 *              transform, so small batches of them go four-step: the block
 *              path needs at least 16 transforms at n = 8192, 48 at 16384
 *              and 64 at 32768 (FP16 storage: 32 at 16384, 48 at 32768),
 *              unless fft_plan_create_ex's options give a block limit or
 *              name a block kernel (radix, flags or c).
 *   batch      number of transforms per execute (>= 1).  On the block path
 *              the default kernel's width follows it: a batch that would
 *              give the full-width kernel fewer than 128 workgroups runs
 *              the one-wave form of the same schedule and variant (fewer
 *              transforms per workgroup, more compute units busy); the
 *              same rule applies to the batch of each fft_execute_ex call.
 *   direction  FFT_FORWARD or FFT_BACKWARD.
 *   plan_out   receives the plan handle.
 *
 * The plan allocates (hipMalloc) its twiddle tables, generated in FP64 on the
 * host and rounded once to FP32, and for the four-step path a workspace of
 * batch * n complex values.  Returns INVALID_ARG (n == 0, batch == 0, bad
 * direction, null plan_out), UNSUPPORTED_SIZE, OUT_OF_MEMORY or DEVICE.
 */
fft_status_t fft_plan_create(size_t n, size_t batch, int direction, fft_plan_t* plan_out);

/*
 * fft_execute -- run the planned transforms on `stream`.
 *
 *   in   device pointer to batch * n complex values (read only), complex64
 *        or, for FFT_STORAGE_F16 plans, FP16 pairs.
 *   out  device pointer to batch * n complex values of the same storage;
 *        out == in is allowed (in-place).  Partial overlap other than
 *        out == in is INVALID_ARG.
 *
 * Both pointers must be aligned to the element size (8 or 4 bytes).  Asynchronous; returns DEVICE when a
 * launch fails, INVALID_PLAN for a null plan.
 */
fft_status_t fft_execute(fft_plan_t plan, const void* in, void* out, void* stream);

/*
 * fft_execute_pass -- run one kernel of a plan, for per-kernel timing.
 *   pass 1: block path: the whole transform (same as fft_execute);
 *           four-step: the column transforms + twiddle, `in` -> plan workspace
 *           (`out` is not touched).
 *   pass 2: four-step only: the row transforms + corner turn, plan workspace
 *           -> `out` (`in` is not touched); INVALID_ARG on the block path.
 * fft_execute(plan, in, out) == pass 1 then pass 2 on the same stream.
 * Same pointer rules and errors as fft_execute.
 */
fft_status_t fft_execute_pass(fft_plan_t plan, int pass, const void* in, void* out, void* stream);

/*
 * fft_execute_pass_timed -- fft_execute_pass with two events (from
 * fft_event_create) that the device stamps at the start and at the end of
 * the kernel's dispatch itself, so their difference is the kernel's duration
 * without the gaps between launches (what a kernel-trace profiler reports).
 * Both events are required (INVALID_ARG otherwise).
 */
fft_status_t fft_execute_pass_timed(fft_plan_t plan, int pass, const void* in, void* out, void* stream,
                                    void* start_event, void* stop_event);

/* Timing events of the library's runtime: create, destroy, and the time in
 * milliseconds between two recorded events (waits for stop_event). */
fft_status_t fft_event_create(void** event);
fft_status_t fft_event_destroy(void* event);
fft_status_t fft_event_elapsed(void* start_event, void* stop_event, float* ms);

/*
 * fft_transpose -- corner turn of `batch` row-major complex64 matrices:
 *     out[b][c][r] = in[b][r][c],  0 <= r < rows, 0 <= c < cols.
 * The values are copied bit for bit.  `in` and `out` must not overlap
 * (INVALID_ARG).  Asynchronous on `stream`.
 */
fft_status_t fft_transpose(const void* in, void* out, size_t rows, size_t cols, size_t batch,
                           void* stream);

/*
 * fft_plan_destroy -- synchronise the plan's device, free its tables and
 * workspace, and invalidate the handle.  Null handle: INVALID_PLAN.
 */
fft_status_t fft_plan_destroy(fft_plan_t plan);

/* Static English text for a status code (never NULL). */
const char* fft_status_string(fft_status_t s);

/* ---------------------------------------------------------------------------
 * Introspection.
 * ------------------------------------------------------------------------- */
typedef struct {
    size_t n, batch;
    int direction;
    int path;                 /* FFT_PATH_BLOCK, FFT_PATH_FOURSTEP or FFT_PATH_FILTER */
    size_t n1, n2;            /* four-step split (n1: pass-1 column length); 0 for block */
    int n_radix;              /* radix schedule of the block kernel (pass 1 for four-step) */
    int radix[8];
    int n_radix2;             /* radix schedule of pass 2 (four-step only) */
    int radix2[8];
    int threads_per_block;    /* workgroup size of the (first) kernel */
    int transforms_per_block; /* transforms (or columns) one workgroup handles */
    size_t lds_bytes;         /* static LDS of the (first) kernel */
    size_t workspace_bytes;   /* device workspace owned by the plan */
    size_t twiddle_bytes;     /* device twiddle tables owned by the plan */
    int kernels_per_execute;  /* 1 (block) or 2 (four-step) */
    const char* kernel_name;  /* symbolic name of the (first) kernel */
    const char* kernel_name2; /* symbolic name of the pass-2 kernel (four-step), else NULL */
    int flags;                /* variant flags (FFT_VARIANT_*) of the (first) kernel */
    int flags2;               /* variant flags of the pass-2 kernel */
    int c2;                   /* pass-2 rows per workgroup = workspace block width */
    long long grid;           /* workgroups of the (first) launch; 0 from fft_plan_query */
    int storage;              /* FFT_STORAGE_C64, FFT_STORAGE_F16 or FFT_STORAGE_F16_COMPACT */
    int device_twiddles;      /* tables evaluated on the GPU */
    float scale;              /* output multiplier (1: none) */
} fft_plan_desc_t;

/* ---------------------------------------------------------------------------
 * Kernel variants and planner options (the runtime sweep and the schedule
 * search pick among compiled variants; the defaults need none of this).
 * ------------------------------------------------------------------------- */
#define FFT_VARIANT_NT_LOAD 1     /* non-temporal (streaming) loads of the data */
#define FFT_VARIANT_NT_STORE 2    /* non-temporal stores of the data */
#define FFT_VARIANT_PERSISTENT 4  /* persistent workgroups prefetching the next unit */
#define FFT_VARIANT_SWIZZLE 8     /* XOR-swizzled unpadded LDS layout */
#define FFT_VARIANT_STAGED 16     /* four-step pass 1: outputs staged through LDS, contiguous stores */
#define FFT_VARIANT_TWIDDLE_POWERS 32 /* stage twiddles from per-row powers w^(2^i) and products */
#define FFT_VARIANT_FP16_STORAGE 64   /* data stored as FP16 pairs, FP32 arithmetic */
#define FFT_VARIANT_XCD_ORDER 128     /* work units ordered so neighbours share an XCD (and its L2) */
#define FFT_VARIANT_STAGE_STRIDE 256  /* four-step pass 1: LDS stride residue for the staged store */
#define FFT_VARIANT_WAVE_SYNC 512     /* one transform per wavefront: exchanges without workgroup barriers */
#define FFT_VARIANT_HALF_EXCHANGE 1024 /* every stage but the last runs an even number of butterflies
                                          per thread: exchanges (and the pass-1 staged store) in two
                                          rounds through half the LDS */
#define FFT_VARIANT_FIT_REGISTERS 2048 /* with HALF_EXCHANGE: registers fitted to every workgroup the
                                          halved LDS allows, spilling if need be */
#define FFT_VARIANT_LOOP 4096         /* persistent workgroups (as many as are resident) looping over
                                         the units in launch order, without prefetch */
#define FFT_VARIANT_RUNTIME_SCHEDULE 8192 /* block kernel (lengths 64..16384, 16 values per thread)
                                             that takes its radix schedule at run time: any
                                             sequence of radices 2, 4, 8, 16 whose product is n.
                                             Chosen for a schedule (fft_plan_opts_t.radix) no
                                             compiled kernel has, or when flags include it */
#define FFT_VARIANT_VEC16 16384       /* block kernel: 16-byte global loads and stores (two
                                         consecutive complex values per lane; neighbouring lanes
                                         swap halves by a DPP lane permutation).  fft_execute
                                         returns FFT_ERR_INVALID_ARG unless in and out are 16-byte
                                         aligned */
#define FFT_VARIANT_CROSS_LANE 32768  /* block kernel, one transform per wave64 (N = 1024,
                                         schedule [16,4,16]): exchanges between the lanes of the
                                         wave are register permutations (DPP, v_permlane16/32_swap)
                                         instead of LDS round trips; with WAVE_SYNC the exchange
                                         over lane bits 0..3 still goes through LDS */
#define FFT_VARIANT_VAR_THREADS 65536 /* block kernel whose stages run on different numbers of
                                         threads (each stage's butterflies split evenly over at
                                         most the workgroup's threads), so a mixed-radix length
                                         holds few values per thread (15360 = [15,16,16,4] on
                                         1024 threads: 16 values, not 60); one transform per
                                         workgroup */
#define FFT_VARIANT_FP16_WORKSPACE 524288 /* four-step passes of FFT_STORAGE_F16_COMPACT: FP16 workspace */

/* Storage of the transform data (fft_plan_opts_t.storage). */
#define FFT_STORAGE_C64 0   /* interleaved FP32 (re, im), 8 bytes per value */
#define FFT_STORAGE_F16 1   /* interleaved IEEE FP16 (re, im), 4 bytes per value; arithmetic stays FP32
                               (values are widened on load and rounded to nearest even on store);
                               the four-step workspace stays FP32.  The transform is unnormalised,
                               so an output can reach n * max|x|: outputs beyond 65504 in magnitude
                               become +-inf (uniform [-1, 1] data stays far below that: its spectrum
                               has rms sqrt(2n/3)) */
#define FFT_STORAGE_F16_COMPACT 2 /* FP16 data as FFT_STORAGE_F16, and on the four-step path an FP16
                                     workspace as well (16 bytes of HBM traffic per point instead of
                                     24): the pass-1 outputs are rounded to FP16 once more, which adds
                                     at most 2^-11 to the relative error bound.  Single-block lengths
                                     run as with FFT_STORAGE_F16.  Not available for ragged batches */

typedef struct {
    size_t block_limit;  /* longest single-block length (power of two, 1024..32768); 0 =
                            fft_block_limit() with the small-batch rule of fft_plan_create;
                            nonzero: the single block at every batch up to this length */
    int n_radix;         /* schedule of the single block (four-step: of pass 1): 0 = default, else radix[0..n_radix) */
    int radix[8];
    int flags;           /* variant of the block kernel / pass 1; -1 = default */
    int c;               /* transforms per workgroup of the block kernel, or four-step pass-1
                            columns per workgroup; 0 = default */
    int flags2;          /* variant of pass 2; -1 = default */
    int c2;              /* pass-2 rows per workgroup (workspace block width); 0 = default */
    size_t n1;           /* four-step split n = n1 * n2 (a power of two); 0 = the planner's split
                            (rows n2 up to 2048, columns n1 at least 256) */
    int storage;         /* FFT_STORAGE_C64 (default), FFT_STORAGE_F16 or FFT_STORAGE_F16_COMPACT */
    int device_twiddles; /* nonzero: evaluate the twiddle tables in FP64 on the GPU
                            (default: FP64 on the host); both round each table entry once
                            to FP32.  Kernels with FFT_VARIANT_TWIDDLE_POWERS (most
                            defaults) then form w^r from the entries w^(2^i) with at most
                            popcount(r) - 1 FP32 complex products, and the four-step long
                            twiddle as b * s^m; the exact-row variants multiply by entries
                            rounded once */
    float scale;         /* multiplier applied to every output in the last store, in FP32
                            (1.0f / n with FFT_BACKWARD gives the normalised inverse,
                            backward(forward(x)) = x); 0 = none (1).  Must be finite.
                            Not accepted for ragged plans (INVALID_ARG). */
} fft_plan_opts_t;

/* Fill `opts` with "use the defaults". */
void fft_plan_opts_init(fft_plan_opts_t* opts);

/* fft_plan_create with planner options (NULL = defaults).  A combination no
 * compiled kernel provides returns UNSUPPORTED_SIZE. */
fft_status_t fft_plan_create_ex(size_t n, size_t batch, int direction, const fft_plan_opts_t* opts,
                                fft_plan_t* plan_out);

/* fft_plan_query with planner options (no device needed). */
fft_status_t fft_plan_query_ex(size_t n, size_t batch, int direction, const fft_plan_opts_t* opts,
                               fft_plan_desc_t* desc);

#define FFT_KERNEL_BLOCK 0
#define FFT_KERNEL_PASS1 1
#define FFT_KERNEL_PASS2 2
#define FFT_KERNEL_FILTER 3

typedef struct {
    int kind;            /* FFT_KERNEL_* */
    int n;               /* length of the transforms one thread group computes */
    int e;               /* complex values per thread */
    int c;               /* transforms (block) or columns/rows (passes) per workgroup */
    int flags;           /* FFT_VARIANT_* */
    int n_radix;
    int radix[8];
    int threads;         /* workgroup size */
    size_t lds_bytes;
    int is_default;      /* the planner's default for (kind, n) */
    const char* name;
} fft_kernel_info_t;

/* Number of compiled transform kernels, and the description of one. */
int fft_kernel_count(void);
fft_status_t fft_kernel_info(int index, fft_kernel_info_t* info);

/*
 * fft_kernel_occupancy -- workgroups of catalogue kernel `index` that one
 * compute unit of the current device keeps resident at once, as the HIP
 * runtime's occupancy calculator gives it from the kernel's registers, its
 * LDS and the wave slots (four SIMDs, 64-wide waves).  A report about the
 * implementation, not an operation of the paper: it tells how many
 * workgroups overlap their LDS exchanges with other workgroups' loads.
 *   workgroups_per_cu  HOST pointer, written on success.
 * INVALID_ARG for a null pointer or an index outside [0, fft_kernel_count());
 * DEVICE if there is no device or the runtime reports zero.
 */
fft_status_t fft_kernel_occupancy(int index, int* workgroups_per_cu);

/* Fill `desc` for a plan.  INVALID_PLAN / INVALID_ARG on null arguments. */
fft_status_t fft_plan_describe(fft_plan_t plan, fft_plan_desc_t* desc);

/*
 * fft_execute_ex -- fft_execute with the batch and the workspace given per call.
 *   batch      transforms of this call, any number >= 1 (0 = the plan's batch);
 *              the plan's tables do not depend on it.
 *   workspace  four-step plans: DEVICE pointer to n * batch complex64 values
 *              (FP16 pairs in the compact FP16 form; 8-byte aligned,
 *              overlapping neither in nor out) used instead
 *              of the plan's own workspace, or NULL for the plan's own (then
 *              batch must not exceed the plan's).  Ignored on other paths.
 * With an external workspace one plan may run on several streams at once.
 * Errors as fft_execute, plus INVALID_ARG for a batch the plan's workspace
 * cannot hold or a bad workspace pointer.
 */
fft_status_t fft_execute_ex(fft_plan_t plan, size_t batch, const void* in, void* out, void* workspace,
                            void* stream);

/*
 * fft_execute_static -- fft_execute_ex whose four-step workspace is the
 * library's own static device array (fft_static_scratch_bytes() = 64 MiB per
 * GPU, held from module load until the process ends) instead of the plan's
 * or a caller's buffer.  For callers that cannot allocate device memory at
 * execute time (code under HIP graph capture, tight serving loops,
 * allocation-free harnesses): the call makes no hipMalloc/hipFree or other
 * allocating call; the plan (created beforehand, e.g. with batch 1) supplies
 * only its tables.  The caller still passes in and out (DEVICE pointers, as
 * fft_execute).  batch: transforms of this call (0 = the plan's).
 * Single-block plans need no workspace and run exactly as fft_execute_ex.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (two streams, two threads) race on it and must be ordered by
 * the caller.  Pass 1 writes every workspace value pass 2 reads, so nothing
 * needs clearing between calls.  Returns SCRATCH_LIMIT when n * batch * 8
 * bytes (4 in the compact FP16 form) exceed the array (nothing is launched),
 * else as fft_execute_ex.
 */
fft_status_t fft_execute_static(fft_plan_t plan, size_t batch, const void* in, void* out, void* stream);
size_t fft_static_scratch_bytes(void);

/* Copy the plan's twiddle table (complex64 entries) to host memory: the
 * number of entries goes to *n_entries; with host_dst NULL only the count is
 * returned; max_entries below the count is INVALID_ARG.  Synchronous. */
fft_status_t fft_plan_twiddles(fft_plan_t plan, void* host_dst, size_t max_entries, size_t* n_entries);

/* Dry-run planning: fill `desc` with the path, split and kernels that
 * fft_plan_create would choose for (n, batch, direction), without touching a
 * device (no HIP call, no allocation).  Same argument errors as
 * fft_plan_create. */
fft_status_t fft_plan_query(size_t n, size_t batch, int direction, fft_plan_desc_t* desc);

typedef struct {
    int device;
    char arch[64];            /* gcnArchName, e.g. "gfx950:sramecc+:xnack-" */
    int compute_units;
    int warp_size;
    size_t lds_per_cu;        /* bytes of LDS per compute unit */
    size_t lds_per_block;     /* max LDS bytes one workgroup may allocate */
    size_t global_mem;
    int clock_khz;
    int mem_clock_khz;
    int mem_bus_width;
    /* Analytic block limit (paper, Approach: the largest FFT a compute unit's
     * local memory holds): pow2floor(lds_per_cu / (8 * (1 + 1/16) * k)) for
     * k = 1, 2, 4 workgroups resident per CU (8 bytes per complex value plus
     * one pad value per 16). */
    size_t block_max[3];
} fft_device_info_t;

/* Query the current device (device < 0) or device `device`. */
fft_status_t fft_device_query(int device, fft_device_info_t* info);

/* The analytic block limit for `lds_bytes` of local memory per compute unit
 * and k resident workgroups: pow2floor(lds_bytes / (8 * (17/16) * k)); 0 if
 * k < 1 or nothing fits.  Pure arithmetic, no device needed. */
size_t fft_block_max(size_t lds_bytes, int k);

/* Largest length the single-block path handles: 32768, twice the analytic
 * limit for one workgroup per CU, since the half-exchange kernels stage only
 * half the points in LDS at a time; the runtime sweep confirms each step
 * (block faster than four-step at 2048..32768 for large batches).  The
 * environment variable FFTBLOCK_BLOCK_MAX (power of two, 1024..32768) may
 * lower it. */
size_t fft_block_limit(void);

/* ---------------------------------------------------------------------------
 * Bandwidth probe (the analogue of the paper's memory benchmark, Approach,
 * bottom-level analysis): copy `bytes` (multiple of 16, 16-byte aligned
 * pointers, no overlap) from `in` to `out` with 16-byte streaming
 * (non-temporal) vector loads and stores, the access form of the transforms.
 * ------------------------------------------------------------------------- */
fft_status_t fft_copy(const void* in, void* out, size_t bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Schedule search (paper, Approach, bottom-level analysis, "FFT performance
 * model"): radix stages as edges of a DAG over stage indices 0..log2 N, a
 * radix-R stage starting at stage s weighted by its measured cost; under the
 * hypothesis that a stage's cost depends only on (radix, start stage), the
 * best mixed-radix schedule is the shortest source-to-sink path (Dijkstra).
 * ------------------------------------------------------------------------- */

/* Shortest path over the stage DAG.  costs[i * log2n + s] is the cost of
 * radix radices[i] (a power of two) starting at stage s; a negative, NaN or
 * infinite cost means "no such edge".  Ties go to fewer stages, then to the
 * lexicographically larger radix list.  Writes the schedule (at most log2n
 * radices) to sched_out, its length to n_sched_out and its cost to total_out
 * (may be NULL).  Pure host code.  INVALID_ARG on bad arguments,
 * UNSUPPORTED_SIZE when no path reaches the sink. */
fft_status_t fft_schedule_search(int log2n, const int* radices, int n_radices, const double* costs,
                                 int* sched_out, int* n_sched_out, double* total_out);

/* GPU microbenchmark of one radix-R Stockham stage (R = 2, 4, 8, 16)
 * starting at stage index start_stage on an LDS-resident power-of-two
 * transform of length n (256..16384): nanoseconds per stage per transform,
 * measured as the difference between repeating the stage `reps` times and
 * not at all.  Allocates and frees its own device buffers; synchronous. */
fft_status_t fft_stage_benchmark(size_t n, int radix, int start_stage, int reps, double* ns_per_stage);

typedef struct {
    size_t n;
    int log2n;                    /* 0 for lengths that are not powers of two */
    double stage_cost[4][16];     /* ns per stage per transform for radix 2,4,8,16 by start stage; <0 = none */
    int predicted[16];            /* shortest-path schedule over stage_cost */
    int n_predicted;
    double predicted_cost;
    int n_candidates;             /* compiled kernels (four-step: kernel pairs) timed whole */
    int candidate_kernel[32];     /* catalogue indices (fft_kernel_info): block or pass-1 kernel */
    int candidate_kernel2[32];    /* pass-2 kernel of a four-step candidate, else -1 */
    double candidate_us[32];      /* microseconds per execute of `batch` transforms, rotating over
                                     buffer sets of up to 512 MiB per side (data from HBM) */
    int chosen_kernel;            /* fastest candidate; recorded as wisdom for n */
    int chosen_kernel2;
    double chosen_us;
    double predicted_us;          /* the predicted schedule run whole on the run-time-schedule kernel
                                     (FFT_VARIANT_RUNTIME_SCHEDULE), same batch; < 0 = not run */
    double chosen_schedule_rt_us; /* the fastest compiled kernel's schedule on that same kernel: the
                                     model's choice against the measured one on one code path */
    int chosen_predicted;         /* 1: the predicted schedule beat every compiled kernel; chosen_kernel
                                     is then the run-time-schedule kernel and the wisdom holds the
                                     schedule */
} fft_tune_report_t;

/* Autotune length n on the current device: stage microbenchmarks and the
 * shortest-path schedule (the paper's model), then every compiled block kernel
 * for n -- or, for four-step lengths, every compiled pass-1 x pass-2 pair,
 * which also chooses the column and row widths -- timed as a whole on `batch`
 * transforms (runtime validation), and the predicted schedule itself on the
 * run-time-schedule kernel; the fastest becomes the wisdom entry
 * fft_plan_create uses for n.  Synchronous; allocates temporary buffers. */
fft_status_t fft_autotune(size_t n, size_t batch, fft_tune_report_t* report);

/* Wisdom: the kernel (four-step: kernel pair) chosen per length.
 * fft_plan_create uses it when no explicit options are given.  The file
 * format is one "length<TAB>kernel[<TAB>pass-2 kernel]" line per entry
 * (a space may separate length and kernel); entries naming kernels the
 * library does not contain are skipped
 * (INVALID_ARG is returned after loading the rest).  The environment variable
 * FFTBLOCK_WISDOM names a file loaded before the first plan is created. */
fft_status_t fft_wisdom_set(size_t n, int kernel_index);
int fft_wisdom_get(size_t n);          /* catalogue index, or -1 */
void fft_wisdom_clear(void);
fft_status_t fft_wisdom_save(const char* path);
fft_status_t fft_wisdom_load(const char* path);

/* ---------------------------------------------------------------------------
 * Range compression (radar chain, "Radar application description", Fig. 3:
 * the range lines are compressed after the range FFT by the matched filter).
 * ------------------------------------------------------------------------- */

/*
 * fft_filter_create -- plan the range compression of `batch` rows of length n
 * against a transmitted pulse replica of replica_len <= n samples:
 *
 *     y = B(F(x) .* conj(F(r)))   per row,  r = replica zero-padded to n,
 *
 * F the forward and B the unnormalised backward transform, which equals the
 * circular cross-correlation y[m] = n * sum_{l<L} x[(m + l) mod n] conj(r[l]);
 * a target echo delayed by d samples compresses to a peak at m = d.  One
 * workgroup runs the forward transform, the product and the backward
 * transform of a row in LDS, so a row is read and written once.
 *
 *   replica  DEVICE pointer to replica_len complex64 values (8-byte aligned);
 *            read during this call only (the plan keeps F(r) in its table,
 *            computed on the device with this library's forward transform).
 *   opts     may be NULL; flags / radix select a catalogue variant,
 *            device_twiddles as for fft_plan_create_ex; storage must be 0.
 *
 * n: a power of two from 64 to 16384.  Execute with fft_execute(plan, in,
 * out, stream) (direction is ignored; in == out allowed).  Synchronous.
 * Errors: INVALID_ARG (null or misaligned pointers, zero sizes, replica_len
 * > n, storage != 0), UNSUPPORTED_SIZE (other n), OUT_OF_MEMORY, DEVICE.
 */
fft_status_t fft_filter_create(size_t n, size_t batch, const void* replica, size_t replica_len,
                               const fft_plan_opts_t* opts, fft_plan_t* plan_out);

/* Dry run of fft_filter_create's planning (no device needed). */
fft_status_t fft_filter_query(size_t n, size_t batch, size_t replica_len, const fft_plan_opts_t* opts,
                              fft_plan_desc_t* desc);

/* ---------------------------------------------------------------------------
 * Ragged batches: transforms of several lengths in one submission (paper,
 * Approach, "Top level analysis": many independent FFT tasks, each reading its
 * inputs, computing and writing its outputs, mapped onto the compute units).
 * ------------------------------------------------------------------------- */
typedef struct fft_ragged_s* fft_ragged_t;

/*
 * fft_ragged_create -- plan n_classes batches: counts[c] transforms of length
 * sizes[c] each, all in `direction`, on the current device.  Every length must
 * be one fft_plan_create accepts.  Data layout for execute: the classes'
 * batches concatenated in the given order, class c starting at complex
 * element sum_{j<c} sizes[j] * counts[j].
 *
 * Each class is matched to a case of a persistent work-list kernel (one per
 * LDS-footprint class: lengths up to 8192, 1000, 3072 and 256-point four-step
 * rows in a 256-thread kernel with four workgroups per CU; 6000, 15360,
 * 16384, 32768 and 256-point four-step columns in a 512-thread kernel with
 * one workgroup per CU).  The classes of one kernel form one launch whose
 * resident workgroups take work units (a workgroup's share of transforms, or
 * a four-step tile) from one device queue, largest units first; a four-step
 * length (65536 = 256 x 256) has its pass-1 tiles in the first launch and its
 * pass-2 tiles in the second.  A length no case covers runs its own plan's
 * kernels beside them.  Allocates the classes' plans (tables, four-step
 * workspaces), the work lists and two counters per launch.
 */
fft_status_t fft_ragged_create(const size_t* sizes, const size_t* counts, size_t n_classes, int direction,
                               fft_ragged_t* out);

/* As fft_ragged_create; of `opts` (may be NULL) only `storage` and
 * `device_twiddles` are used, for every class.  With FFT_STORAGE_F16 the data
 * of execute are FP16 pairs (4 bytes per value, 4-byte alignment). */
fft_status_t fft_ragged_create_ex(const size_t* sizes, const size_t* counts, size_t n_classes, int direction,
                                  const fft_plan_opts_t* opts, fft_ragged_t* out);

/*
 * fft_ragged_execute -- transform every class from `in` to `out` on `stream`
 * (device pointers aligned to the element size, in == out allowed, other overlap
 * INVALID_ARG).  Asynchronous.
 *   mode 0: one hipGraphLaunch of a graph whose kernel nodes are the
 *           persistent launches and then the kernels of every class with no
 *           persistent case (the lengths whose own kernels beat any shared
 *           case), all in sequence; built on the first call, and on a call with other
 *           buffers only the nodes' arguments change.  Launches of one plan
 *           must not overlap in time (they share the queue counters).
 *   mode 1: the plain path -- every class through its own default plan (the
 *           autotuner's wisdom for its length), one after another on `stream`.
 *   mode 2: those default plans' kernels in one graph on four parallel
 *           branches (re-captured when the buffers change).
 */
fft_status_t fft_ragged_execute(fft_ragged_t r, const void* in, void* out, void* stream, int mode);

/* Total complex values of one execute, and kernel nodes of the mode-0 graph
 * (0 before its first execute).  Either pointer may be NULL. */
fft_status_t fft_ragged_describe(fft_ragged_t r, size_t* total_points, size_t* graph_nodes);

typedef struct {
    size_t total_points;
    int graph_nodes;            /* kernel nodes of the mode-0 graph */
    int persistent_launches;    /* of which persistent work-list kernels (at most 8 described) */
    int fallback_classes;       /* classes run by their own plan's kernels */
    const char* kernel_name[8]; /* per persistent launch, in launch order */
    unsigned units[8];          /* work units of the launch */
    unsigned grid[8];           /* workgroups launched (the resident capacity, at most units) */
    int classes[8];             /* length classes (four-step passes count once each) */
    int threads[8];             /* workgroup size */
    size_t lds_bytes[8];        /* static LDS per workgroup */
    size_t branch_graph_nodes;  /* nodes of the mode-2 graph (0 before its first execute) */
} fft_ragged_desc_t;

fft_status_t fft_ragged_describe_ex(fft_ragged_t r, fft_ragged_desc_t* desc);

/* Synchronise the device and free the plans, graph, streams and events. */
fft_status_t fft_ragged_destroy(fft_ragged_t r);

/* ---------------------------------------------------------------------------
 * Serving: a request scheduler and a GPU server built on it.  Not an
 * operation of the paper: its top-level analysis runs one batch of
 * same-size FFTs (one FFT per processing element, read / compute / write);
 * serving extends that to requests of any size arriving over time.
 *
 * Requests (n, batch, direction) arrive over time.  The scheduler admits them
 * in arrival order while the bytes of the requests in flight (input, output
 * and four-step workspace) stay within an HBM budget; a request larger than
 * the budget is rejected, one that does not fit yet waits at the head of the
 * queue, and while it waits only small requests (backfill_bytes) may pass it.
 * Each launch goes to the stream with the fewest outstanding bytes among
 * those with fewer than max_inflight launches outstanding; the first
 * small_streams streams are kept for launches led by short requests.
 * Continuous batching: queued requests of the same (n, direction) on the
 * single-block path join the head request's launch (one list launch), in
 * arrival order, up to max_coalesce requests and max_transforms transforms.
 * Latency = completion time - arrival time.
 *
 * The scheduler alone (fft_sched_*) is a host-only state machine: it makes
 * no HIP call and takes every time as an argument (seconds, any monotonic
 * clock), so it can be driven by a simulated executor.  The server
 * (fft_server_*) runs it on a dispatcher thread against the device.
 * ------------------------------------------------------------------------- */
#define FFT_LAUNCH_MAX_REQUESTS 64

/* Request states. */
#define FFT_REQ_QUEUED 0
#define FFT_REQ_RUNNING 1
#define FFT_REQ_DONE 2
#define FFT_REQ_REJECTED 3   /* larger than the whole budget */

typedef struct {
    size_t hbm_budget;   /* bytes in flight at most (default 64 GiB) */
    int n_streams;       /* 1..16 (default 4) */
    int max_inflight;    /* launches outstanding per stream, >= 1 (default 2) */
    int max_coalesce;    /* requests per launch, 1..FFT_LAUNCH_MAX_REQUESTS (default 32; 1 = off) */
    size_t max_transforms;  /* transforms per coalesced launch (default 16384) */
    size_t backfill_bytes;  /* while the head request waits for room, later requests of at most this
                               many bytes may pass it, at most this many bytes of them in flight and
                               never more than the budget minus the head's bytes, so the head fits as
                               soon as the work launched before it completes (default 1 GiB; 0 =
                               strict FIFO) */
    int small_streams;      /* streams [0, small_streams) take only launches led by a request of at
                               most small_bytes, so short requests never queue on a stream behind a
                               long transform (they use any stream when these are full); default 1,
                               0 = none, capped at n_streams - 1 */
    size_t small_bytes;     /* default 64 MiB */
} fft_sched_opts_t;

typedef struct {
    long long id;        /* launch id, for fft_sched_complete */
    int stream;          /* 0..n_streams-1 */
    size_t n;
    int direction;
    size_t batch;        /* transforms of the launch (sum over its requests) */
    size_t bytes;        /* budget bytes of the launch */
    int n_requests;
    uint64_t requests[FFT_LAUNCH_MAX_REQUESTS];   /* request ids, arrival order */
} fft_launch_t;

typedef struct {
    uint64_t id;
    size_t n, batch;
    int direction;
    int state;           /* FFT_REQ_* */
    size_t bytes;
    double t_arrive, t_launch, t_done;   /* seconds; -1 = not yet */
    long long launch;    /* -1 until launched */
    int stream;
    int group_size;      /* requests in its launch */
} fft_request_info_t;

typedef struct {
    size_t submitted, completed, rejected, queued;
    size_t running_launches, launches;
    size_t coalesced_requests;    /* requests that shared a launch with others */
    size_t backfilled_requests;   /* requests admitted past a waiting head */
    size_t inflight_bytes, peak_inflight_bytes;
    double points;                /* transform points completed (n * batch summed) */
    double t_last_done;
    double latency_p50, latency_p99, latency_mean, latency_max;   /* seconds, nearest rank */
    double queue_p50, queue_p99;    /* seconds from arrival to launch (admission and stream wait) */
    double device_p50, device_p99;  /* seconds from launch to completion (on the device, with
                                       whatever shares it) */
} fft_sched_stats_t;

typedef struct fft_sched_s* fft_sched_t;

void fft_sched_opts_init(fft_sched_opts_t* opts);
/* INVALID_ARG for options out of range. */
fft_status_t fft_sched_create(const fft_sched_opts_t* opts, fft_sched_t* out);
fft_status_t fft_sched_destroy(fft_sched_t s);
/* Queue a request (ids must be unique); `coalescible` marks requests that may
 * share a list launch.  INVALID_ARG for zero sizes, a bad direction or a
 * duplicate id. */
fft_status_t fft_sched_submit(fft_sched_t s, uint64_t id, size_t n, size_t batch, int direction, size_t bytes,
                              int coalescible, double now);
/* The next launch to issue at time `now`, if any (*got = 1).  The caller
 * issues it and reports its completion with fft_sched_complete. */
fft_status_t fft_sched_next(fft_sched_t s, double now, fft_launch_t* launch, int* got);
fft_status_t fft_sched_complete(fft_sched_t s, long long launch_id, double now);
fft_status_t fft_sched_request(fft_sched_t s, uint64_t id, fft_request_info_t* info);
fft_status_t fft_sched_stats(fft_sched_t s, fft_sched_stats_t* stats);

typedef struct {
    fft_sched_opts_t sched;
    size_t arena_bytes;  /* device memory for outputs and workspaces; 0 = sched.hbm_budget */
    int auto_release;    /* nonzero: outputs are dropped at completion (load generation) */
} fft_server_opts_t;

/* A server's calls may come from any host threads; fft_server_destroy must
 * not overlap another call on the same server. */
typedef struct fft_server_s* fft_server_t;

void fft_server_opts_init(fft_server_opts_t* opts);
/* Allocates the arena, the stream pool and the list-descriptor buffers on the
 * current device and starts the dispatcher thread. */
fft_status_t fft_server_create(const fft_server_opts_t* opts, fft_server_t* out);
/* Create the plan for (n, direction) now rather than at its first request
 * (plans and twiddle tables stay resident for the server's lifetime). */
fft_status_t fft_server_prepare(fft_server_t s, size_t n, int direction);
/* Queue a request; `in` is a DEVICE pointer to batch * n complex64 values that
 * must stay valid and unchanged until the request completes.  `stream` is the
 * submitter's hipStream_t (NULL = the null stream): the server records an event
 * there at submission and its launch waits for it, so work queued on `stream`
 * before the call (the kernel or copy that writes `in`) completes before the
 * server reads the input; the submitting thread need not synchronise.  The
 * output (and,
 * for four-step lengths, the workspace) is allocated from the server's arena
 * when the request is issued; outputs stay there until fft_server_release (or
 * completion, with auto_release), and a full arena holds later launches back
 * until room is freed.  Non-blocking.  OUT_OF_MEMORY at once for a request
 * whose output (and workspace) can never fit the arena; INVALID_ARG for a null
 * or misaligned pointer, zero sizes or a bad direction; UNSUPPORTED_SIZE for a
 * length the planner has no kernels for. */
fft_status_t fft_server_submit(fft_server_t s, size_t n, size_t batch, int direction, const void* in,
                               void* stream, uint64_t* ticket);
/* Block until the request completes (TIMEOUT after timeout_s seconds);
 * *out = its output in the arena (valid until fft_server_release), *info its
 * record.  OUT_OF_MEMORY for a rejected request.  Not for auto_release
 * servers. */
fft_status_t fft_server_wait(fft_server_t s, uint64_t ticket, double timeout_s, void** out,
                             fft_request_info_t* info);
/* Copy a completed request's output (batch * n complex64) to the DEVICE
 * pointer dst on `stream` (asynchronous; NULL = the null stream). */
fft_status_t fft_server_read(fft_server_t s, uint64_t ticket, void* dst, void* stream);
/* Free a completed request's output and record. */
fft_status_t fft_server_release(fft_server_t s, uint64_t ticket);
/* Block until every submitted request has completed. */
fft_status_t fft_server_drain(fft_server_t s, double timeout_s);
fft_status_t fft_server_stats(fft_server_t s, fft_sched_stats_t* stats);
/* The server's clock (seconds since creation), the time base of its records. */
double fft_server_clock(fft_server_t s);
/* Drain, stop the dispatcher and free everything. */
fft_status_t fft_server_destroy(fft_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* FFTBLOCK_H */
