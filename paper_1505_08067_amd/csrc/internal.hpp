// Internal interface between the host planner (fftblock.cpp) and the kernel
// translation units.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace fb {

// ---------------------------------------------------------------- block path
using BlockLaunch = hipError_t (*)(const float2* in, float2* out, const float2* tw, long long batch,
                                   float sg, hipStream_t st);

struct BlockEntry {
    int n;            // transform length
    int e;            // complex values held per thread
    int fpb;          // transforms per workgroup
    int nr;           // number of radix stages
    int radix[8];
    int tw_size;      // complex entries of the stage twiddle table
    int threads;      // workgroup size
    size_t lds;       // static LDS bytes
    BlockLaunch launch;
    const char* name;
};

// Default (planner) kernel for length n, or nullptr.
const BlockEntry* block_default(int n);
// Every compiled block kernel (for the sweep / schedule search).
const BlockEntry* block_table(int* count);

// ------------------------------------------------------------ four-step path
struct FourStepArgs {
    long long batch;     // number of long transforms
    long long nbig;      // N = N1 * N2
    long long n_other;   // pass 1: N2 (row stride); pass 2: N1 (output stride)
    int tiles;           // workgroups per long transform
    int lo_bits;         // split of the long twiddle exponent m = hi * 2^lo_bits + lo
    const float2* tw_hi; // exp(-2 pi i hi 2^lo_bits / N)
    const float2* tw_lo; // exp(-2 pi i lo / N)
    float sg;            // +1 forward, -1 backward (conjugation on entry / exit)
};

using TileLaunch = hipError_t (*)(const float2* in, float2* out, const float2* tw, const FourStepArgs& a,
                                  hipStream_t st);

struct TileEntry {
    int pass;         // 1: column transforms + twiddle, 2: row transforms + corner-turn store
    int n;            // length of the short transforms
    int e;            // values per thread
    int c;            // transforms (columns / rows) per workgroup
    int nr;
    int radix[8];
    int tw_size;
    int threads;
    size_t lds;
    TileLaunch launch;
    const char* name;
};

const TileEntry* tile_find(int pass, int n, int c);
const TileEntry* tile_table(int* count);

// ------------------------------------------------------------------ misc
hipError_t launch_transpose(const float2* in, float2* out, long long rows, long long cols, long long batch,
                            hipStream_t st);
hipError_t launch_copy(const void* in, void* out, size_t bytes, hipStream_t st);

}  // namespace fb
