// Internal interface between the host planner (fftblock_api.hip) and the
// kernel translation units.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

struct fft_plan_s;

namespace fb {

// Longest length one workgroup transforms from LDS (the block path's limit).
constexpr size_t kMaxBlockLen = 32768;

// Arguments shared by every transform kernel (one struct so all launchers
// have the same signature).
struct KArgs {
    const float2* in;
    float2* out;
    const float2* tw;      // stage twiddle rows of the kernel's radix schedule
    long long batch;       // block: transforms; four-step passes: long transforms
    long long nbig;        // four-step: N = N1 * N2
    long long n_other;     // pass 1: N2 (input row stride); pass 2: N1 (output stride)
    int tiles;             // four-step: work units per long transform
    int cw_bits;           // four-step workspace block width 2^cw_bits (= pass-2 rows per unit)
    int lo_bits;           // long twiddle split m = hi * 2^lo_bits + lo
    const float2* tw_hi;   // exp(-2 pi i hi 2^lo_bits / N)
    const float2* tw_lo;   // exp(-2 pi i lo / N)
    const float2* tw_col;  // pass 1, power variant: row col holds exp(-2 pi i col T 2^i / N)
    const float2* flt;     // range compression: spectrum of the pulse replica (n entries)
    const void* list;      // list kernels: one ListEnt per transform
    float sg;              // +1 forward, -1 backward (conjugation on entry and exit)
    unsigned sched;        // run-time-schedule kernels: log2 radix per stage, 4 bits each, stage 0 lowest
    float scale = 1.0f;    // multiplier of the final outputs (1: none); pass 1 applies it only to an
                           // FP16 workspace (then pass 2 gets 1)
};

// start / stop: optional events the device stamps at the dispatch's own start
// and end (nullptr: an ordinary launch).
using KLaunch = hipError_t (*)(const KArgs& a, long long grid, hipStream_t st, hipEvent_t start, hipEvent_t stop);
using KOccupancy = int (*)();   // resident workgroups per CU (hipOccupancy...), 0 on error

enum : int { kKindBlock = 0, kKindPass1 = 1, kKindPass2 = 2, kKindFilter = 3, kKindList = 4 };

// Descriptor of one transform of a list launch (several requests' batches,
// anywhere in memory, in one launch).
struct ListEnt {
    const float2* in;
    float2* out;
};

struct KEntry {
    int kind;          // kKindBlock, kKindPass1, kKindPass2, kKindFilter
    int n;             // transform length handled by one group of threads
    int e;             // complex values per thread
    int c;             // transforms per workgroup (block) / columns or rows per workgroup (passes)
    int flags;         // kNtLoad | kNtStore | kPipe
    int nr;            // radix stages
    int radix[8];
    int tw_size;       // complex entries of the stage table
    int threads;       // workgroup size
    size_t lds;        // static LDS bytes
    bool is_default;   // the planner's choice for (kind, n)
    KLaunch launch;
    KOccupancy occupancy;
    const char* name;
    const void* fn;    // the kernel itself (graph kernel nodes)
};

// Work units a launch must cover (block: workgroups of c transforms;
// passes: batch * tiles).
long long kernel_units(const KEntry& k, const KArgs& a);

const KEntry* kernel_table(int* count);
// Default kernel for (kind, n); for the passes `c` > 0 restricts the width.
const KEntry* kernel_default(int kind, int n, int c, int storage = 0);
// Kernel with exactly this schedule / width / flags (c or flags < 0: any).
const KEntry* kernel_find(int kind, int n, const int* radix, int nr, int c, int flags);

// Registration hooks of the kernel translation units.
const KEntry* block_entries(int* count);
const KEntry* pass_entries(int* count);
const KEntry* filter_entries(int* count);
const KEntry* list_entries(int* count);
const KEntry* rt_entries(int* count);
const KEntry* xlane_entries(int* count);
const KEntry* vt_entries(int* count);

// Kernel the wisdom (autotuner or FFTBLOCK_WISDOM file) chose for length n, or
// nullptr; for the run-time-schedule kernel also its schedule (radix[0..*nr)).
const KEntry* wisdom_kernel(size_t n, int* radix, int* nr);
// Four-step kernels the wisdom chose for length n (false if none); their
// lengths give the split n = k1->n * k2->n.
bool wisdom_pair(size_t n, const KEntry** k1, const KEntry** k2);

// One segment of a plan's twiddle table: entries [offset, offset + count)
// hold exp(-2 pi i m / n) rounded once from FP64 to FP32, with (m, n) a
// function of the entry index e:
//   kSegRows  (a = Ns, b = R):             k = e / R, r = e % R, m = r k, n = Ns R
//   kSegPow   (a = Ns, b = R, c = row, d = P): k = e / row, i = e % row,
//                                           m = k 2^i, n = Ns R (zero for i >= P)
//   kSegHi    (a = N, b = lo_bits):         m = e 2^lo_bits, n = N
//   kSegLo    (a = N):                      m = e, n = N
//   kSegCol   (a = N, b = T, c = row, d = E): col = e / row, i = e % row,
//                                           m = col T 2^i mod N, n = N (zero if 2^i >= E)
// Entries covered by no segment are zero.
enum : int { kSegRows = 0, kSegPow = 1, kSegHi = 2, kSegLo = 3, kSegCol = 4 };
struct TwSeg {
    int type;
    long long offset, count;
    long long a, b, c, d;
};
// exp(-2 pi i m / n) in FP64 on the host (quadrant reduction, quarter turns
// exact), and the same rounded once to FP32: every host-side twiddle value.
void root_fwd(long long m, long long n, double* re, double* im);
float2 root_f32(long long m, long long n);

// Evaluate the segments on the device in FP64 into dst (total entries).
hipError_t generate_twiddles_device(float2* dst, long long total, const TwSeg* segs, int nseg, hipStream_t st);

// List launch of a block plan's kernel: `transforms` descriptors at `list`
// (device memory).  hipErrorNotSupported if the plan's kernel has no list form.
hipError_t plan_launch_list(fft_plan_s* plan, const void* list, long long transforms, hipStream_t st);
// Kernel, arguments and grid of launch `pass` (1, or 2 on the four-step
// path) of a plan's own batch from in to out (the four-step workspace is the
// plan's, between the passes).  false if the plan has no such launch.
bool plan_launch_params(const fft_plan_s* plan, int pass, const void* in, void* out, const KEntry** k, KArgs* a,
                        long long* grid);
// Length, direction and path of a plan (for the serving layer).
void plan_shape(const fft_plan_s* plan, size_t* n, int* direction, int* path, bool* has_list);

hipError_t launch_transpose(const float2* in, float2* out, long long rows, long long cols, long long batch,
                            hipStream_t st);
hipError_t launch_copy(const void* in, void* out, size_t bytes, hipStream_t st);

}  // namespace fb
