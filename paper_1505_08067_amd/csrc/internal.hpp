// Internal interface between the host planner (fftblock_api.hip) and the
// kernel translation units.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace fb {

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
    float sg;              // +1 forward, -1 backward (conjugation on entry and exit)
};

using KLaunch = hipError_t (*)(const KArgs& a, long long grid, hipStream_t st);
using KOccupancy = int (*)();   // resident workgroups per CU (hipOccupancy...), 0 on error

enum : int { kKindBlock = 0, kKindPass1 = 1, kKindPass2 = 2 };

struct KEntry {
    int kind;          // kKindBlock, kKindPass1, kKindPass2
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
};

// Work units a launch must cover (block: workgroups of c transforms;
// passes: batch * tiles).
long long kernel_units(const KEntry& k, const KArgs& a);

const KEntry* kernel_table(int* count);
// Default kernel for (kind, n); for the passes `c` > 0 restricts the width.
const KEntry* kernel_default(int kind, int n, int c);
// Kernel with exactly this schedule / width / flags (c or flags < 0: any).
const KEntry* kernel_find(int kind, int n, const int* radix, int nr, int c, int flags);

// Registration hooks of the two kernel translation units.
const KEntry* block_entries(int* count);
const KEntry* pass_entries(int* count);

// Kernel the wisdom (autotuner or FFTBLOCK_WISDOM file) chose for length n, or nullptr.
const KEntry* wisdom_kernel(size_t n);
// Four-step kernels the wisdom chose for length n = n1 * n2 (false if none).
bool wisdom_pair(size_t n, size_t n1, size_t n2, const KEntry** k1, const KEntry** k2);

hipError_t launch_transpose(const float2* in, float2* out, long long rows, long long cols, long long batch,
                            hipStream_t st);
hipError_t launch_copy(const void* in, void* out, size_t bytes, hipStream_t st);

}  // namespace fb
