// Corner-turn transpose and the HBM copy probe.
//
// Transpose (paper, Approach, "Top level analysis": a large matrix transpose
// split into smaller blocks): each workgroup moves one tile of complex values
// (64 x 64, or 32 x 128 for matrices wider than tall) through LDS.  Reads
// walk rows and writes walk columns of the input, so both sides are
// coalesced; the LDS tile has one pad column so the column-wise LDS reads hit
// distinct banks.  The values are copied bit for bit.
//
// Tile order: workgroup w of tile row tr takes tile column w XOR tr (w + tr
// modulo the count when that is no power of two).  The resident workgroups
// span few tile rows, so with tile columns in plain order their writes start
// at only a few distinct offsets within the output rows (whose pitch is a
// large power of two); spreading them measured 105-106 us against 113 us
// for a cold 4096 x 8192 transpose (diagonal shift: 107 us).
//
// Copy probe (the analogue of the paper's CPU-to-iGPU memory benchmark):
// 16-byte vector loads and stores, grid-stride, used to measure the practical
// HBM bandwidth next to the 8 TB/s specification.
#include <cstdint>

#include "internal.hpp"

namespace fb {

constexpr int kTile = 64;
constexpr int kTransposeThreads = 256;

// The tile (tr, tc) of workgroup blk: tile rows in order, tile columns
// permuted within each tile row (a bijection on [0, tiles_c)).
__device__ __forceinline__ void tile_of(long long rem, long long tiles_c, long long& tr, long long& tc)
{
    tr = rem / tiles_c;
    const long long w = rem - tr * tiles_c;
    if ((tiles_c & (tiles_c - 1)) == 0)
        tc = w ^ (tr & (tiles_c - 1));
    else
        tc = (w + tr) % tiles_c;
}

__global__ void __launch_bounds__(kTransposeThreads)
k_transpose(const float2* __restrict__ in, float2* __restrict__ out, long long rows, long long cols,
            long long tiles_r, long long tiles_c)
{
    __shared__ float2 tile[kTile][kTile + 1];
    const long long blk = blockIdx.x;
    const long long per_mat = tiles_r * tiles_c;
    const long long b = blk / per_mat;
    const long long rem = blk - b * per_mat;
    long long tr, tc;
    tile_of(rem, tiles_c, tr, tc);
    const long long r0 = tr * kTile, c0 = tc * kTile;
    const int tx = threadIdx.x % kTile;
    const int ty = threadIdx.x / kTile;
    constexpr int step = kTransposeThreads / kTile;
    const float2* __restrict__ src = in + b * rows * cols;
    float2* __restrict__ dst = out + b * rows * cols;

    const bool full = (r0 + kTile <= rows) && (c0 + kTile <= cols);
    if (full) {
#pragma unroll
        for (int i = ty; i < kTile; i += step) tile[i][tx] = src[(r0 + i) * cols + c0 + tx];
    } else {
        for (int i = ty; i < kTile; i += step)
            if (r0 + i < rows && c0 + tx < cols) tile[i][tx] = src[(r0 + i) * cols + c0 + tx];
    }
    __syncthreads();
    if (full) {
#pragma unroll
        for (int i = ty; i < kTile; i += step) dst[(c0 + i) * rows + r0 + tx] = tile[tx][i];
    } else {
        for (int i = ty; i < kTile; i += step)
            if (c0 + i < cols && r0 + tx < rows) dst[(c0 + i) * rows + r0 + tx] = tile[tx][i];
    }
}

// Even row and column counts with 16-byte aligned buffers: each lane moves
// two complex values (16 bytes) per access on both sides; tiles hanging over
// the matrix edge are guarded per pair (pairs never straddle the edge since
// both counts are even).  A tile is TR rows by TC columns of the input: the
// reads run TC * 8 bytes along an input row, the writes TR * 8 bytes along an
// output row.
template <int TR, int TC>
__global__ void __launch_bounds__(kTransposeThreads)
k_transpose16(const float2* __restrict__ in, float2* __restrict__ out, long long rows, long long cols,
              long long tiles_r, long long tiles_c)
{
    __shared__ float2 tile[TR][TC + 1];
    const long long blk = blockIdx.x;
    const long long per_mat = tiles_r * tiles_c;
    const long long b = blk / per_mat;
    const long long rem = blk - b * per_mat;
    long long tr, tc;
    tile_of(rem, tiles_c, tr, tc);
    const long long r0 = tr * TR, c0 = tc * TC;
    const float2* __restrict__ src = in + b * rows * cols;
    float2* __restrict__ dst = out + b * rows * cols;
    const bool full = (r0 + TR <= rows) && (c0 + TC <= cols);
    {
        constexpr int PX = TC / 2;  // pairs along an input row
        const int tx = threadIdx.x % PX, ty = threadIdx.x / PX;
        for (int i = ty; i < TR; i += kTransposeThreads / PX) {
            if (full || (r0 + i < rows && c0 + 2 * tx < cols)) {
                const float4 v = *reinterpret_cast<const float4*>(src + (r0 + i) * cols + c0 + 2 * tx);
                tile[i][2 * tx] = make_float2(v.x, v.y);
                tile[i][2 * tx + 1] = make_float2(v.z, v.w);
            }
        }
    }
    __syncthreads();
    {
        constexpr int QX = TR / 2;  // pairs along an output row
        const int ux = threadIdx.x % QX, uy = threadIdx.x / QX;
        for (int i = uy; i < TC; i += kTransposeThreads / QX) {
            if (full || (c0 + i < cols && r0 + 2 * ux < rows)) {
                const float2 a = tile[2 * ux][i], c = tile[2 * ux + 1][i];
                *reinterpret_cast<float4*>(dst + (c0 + i) * rows + r0 + 2 * ux) = make_float4(a.x, a.y, c.x, c.y);
            }
        }
    }
}

// Wider than tall: 32 x 128 tiles (1 KB read runs), measured 103.3 against
// 106.8 us for 4096 x 8192 (cold, XOR order); otherwise 64 x 64 (8192 x 4096:
// 106.4 against 109.2 for 32 x 128).
hipError_t launch_transpose(const float2* in, float2* out, long long rows, long long cols, long long batch,
                            hipStream_t st)
{
    const bool vec = (rows % 2 == 0) && (cols % 2 == 0) && ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0);
    const bool wide = vec && cols > rows;
    const long long TR = wide ? 32 : kTile, TC = wide ? 128 : kTile;
    const long long tr = (rows + TR - 1) / TR;
    const long long tc = (cols + TC - 1) / TC;
    const long long grid = tr * tc * batch;
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    if (wide)
        hipLaunchKernelGGL((k_transpose16<32, 128>), dim3((unsigned)grid), dim3(kTransposeThreads), 0, st, in, out,
                           rows, cols, tr, tc);
    else if (vec)
        hipLaunchKernelGGL((k_transpose16<kTile, kTile>), dim3((unsigned)grid), dim3(kTransposeThreads), 0, st, in,
                           out, rows, cols, tr, tc);
    else
        hipLaunchKernelGGL(k_transpose, dim3((unsigned)grid), dim3(kTransposeThreads), 0, st, in, out, rows, cols,
                           tr, tc);
    return hipGetLastError();
}

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;
typedef float v4f_t __attribute__((ext_vector_type(4)));

// Streaming (non-temporal) 16-byte loads and stores, as the transform kernels
// use for data touched once: the copy then measures the rate those kernels
// can reach (6.1 TB/s on 1 GiB against 5.4 TB/s with cached accesses).
__global__ void __launch_bounds__(kCopyThreads)
k_copy(const v4f_t* __restrict__ in, v4f_t* __restrict__ out, long long n16)
{
    const long long stride = (long long)gridDim.x * kCopyThreads * kCopyUnroll;
    for (long long base = (long long)blockIdx.x * kCopyThreads * kCopyUnroll + threadIdx.x; base < n16;
         base += stride) {
        v4f_t r[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const long long i = base + (long long)u * kCopyThreads;
            if (i < n16) r[u] = __builtin_nontemporal_load(in + i);
        }
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const long long i = base + (long long)u * kCopyThreads;
            if (i < n16) __builtin_nontemporal_store(r[u], out + i);
        }
    }
}

hipError_t launch_copy(const void* in, void* out, size_t bytes, hipStream_t st)
{
    const long long n16 = (long long)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    long long blocks = (n16 + kCopyThreads * kCopyUnroll - 1) / (kCopyThreads * kCopyUnroll);
    if (blocks > 256LL * 64) blocks = 256LL * 64;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kCopyThreads), 0, st, (const v4f_t*)in, (v4f_t*)out,
                       n16);
    return hipGetLastError();
}

}  // namespace fb

namespace fb {

// FP64 evaluation of a plan's twiddle table on the device (the precision form:
// the tables are the only FP64 work on the GPU).  Each entry is
// exp(-2 pi i m / n) for the (m, n) its segment assigns, computed with an
// exact quadrant reduction and double-precision sin/cos, then rounded once to
// FP32; entries outside every segment are zero.
__device__ float2 root_f64_to_f32(long long m, long long n)
{
    m %= n;
    if (m < 0) m += n;
    const long long q = (4 * m) / n, rem = 4 * m - q * n;
    const double hp = 1.57079632679489661923132169163975144;
    double c, s;
    if (2 * rem <= n) {
        const double phi = hp * ((double)rem / (double)n);
        c = cos(phi);
        s = sin(phi);
    } else {
        const double phi = hp * ((double)(n - rem) / (double)n);
        c = sin(phi);
        s = cos(phi);
    }
    const double cr = q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
    const double sr = q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
    return make_float2((float)cr, (float)(-sr));
}

__global__ void __launch_bounds__(256) k_twiddle_gen(float2* __restrict__ dst, long long total,
                                                     const TwSeg* __restrict__ segs, int nseg)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < total; i += (long long)gridDim.x * 256) {
        float2 v = make_float2(0.f, 0.f);
        for (int g = 0; g < nseg; ++g) {
            const TwSeg sg = segs[g];
            if (i < sg.offset || i >= sg.offset + sg.count) continue;
            const long long e = i - sg.offset;
            long long m = 0, n = 1;
            bool have = true;
            switch (sg.type) {
                case kSegRows: m = (e % sg.b) * (e / sg.b); n = sg.a * sg.b; break;
                case kSegPow: {
                    const long long k = e % sg.c;
                    have = k < sg.d;
                    m = (e / sg.c) << k;
                    n = sg.a * sg.b;
                    break;
                }
                case kSegHi: m = e << sg.b; n = sg.a; break;
                case kSegLo: m = e; n = sg.a; break;
                case kSegCol: {
                    const long long k = e % sg.c;
                    have = (1LL << k) < sg.d;
                    m = (((e / sg.c) * sg.b) << k) % sg.a;
                    n = sg.a;
                    break;
                }
                default: have = false;
            }
            if (have) v = root_f64_to_f32(m, n);
            break;
        }
        dst[i] = v;
    }
}

hipError_t generate_twiddles_device(float2* dst, long long total, const TwSeg* segs, int nseg, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    long long blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_twiddle_gen, dim3((unsigned)blocks), dim3(256), 0, st, dst, total, segs, nseg);
    return hipGetLastError();
}

}  // namespace fb
