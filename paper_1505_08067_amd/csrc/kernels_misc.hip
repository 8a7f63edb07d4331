// Corner-turn transpose and the HBM copy probe.
//
// Transpose (paper, Approach, "Top level analysis": a large matrix transpose
// split into smaller blocks): each workgroup moves one TILE x TILE tile of
// complex values through LDS.  Reads walk rows and writes walk columns of the
// input, so both sides are coalesced; the LDS tile has one pad column so the
// column-wise LDS reads hit distinct banks.  The values are copied bit for bit.
//
// Copy probe (the analogue of the paper's CPU-to-iGPU memory benchmark):
// 16-byte vector loads and stores, grid-stride, used to measure the practical
// HBM bandwidth next to the 8 TB/s specification.
#include <cstdint>

#include "internal.hpp"

namespace fb {

constexpr int kTile = 64;
constexpr int kTransposeThreads = 256;

__global__ void __launch_bounds__(kTransposeThreads)
k_transpose(const float2* __restrict__ in, float2* __restrict__ out, long long rows, long long cols,
            long long tiles_r, long long tiles_c)
{
    __shared__ float2 tile[kTile][kTile + 1];
    const long long blk = blockIdx.x;
    const long long per_mat = tiles_r * tiles_c;
    const long long b = blk / per_mat;
    const long long rem = blk - b * per_mat;
    const long long tr = rem / tiles_c;
    const long long tc = rem - tr * tiles_c;
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
// both counts are even).
__global__ void __launch_bounds__(kTransposeThreads)
k_transpose16(const float2* __restrict__ in, float2* __restrict__ out, long long rows, long long cols,
              long long tiles_r, long long tiles_c)
{
    __shared__ float2 tile[kTile][kTile + 1];
    const long long blk = blockIdx.x;
    const long long per_mat = tiles_r * tiles_c;
    const long long b = blk / per_mat;
    const long long rem = blk - b * per_mat;
    const long long tr = rem / tiles_c;
    const long long tc = rem - tr * tiles_c;
    const long long r0 = tr * kTile, c0 = tc * kTile;
    const int tx = threadIdx.x % (kTile / 2);
    const int ty = threadIdx.x / (kTile / 2);
    constexpr int step = kTransposeThreads / (kTile / 2);
    const float2* __restrict__ src = in + b * rows * cols;
    float2* __restrict__ dst = out + b * rows * cols;
    const bool full = (r0 + kTile <= rows) && (c0 + kTile <= cols);
    for (int i = ty; i < kTile; i += step) {
        if (full || (r0 + i < rows && c0 + 2 * tx < cols)) {
            const float4 v = *reinterpret_cast<const float4*>(src + (r0 + i) * cols + c0 + 2 * tx);
            tile[i][2 * tx] = make_float2(v.x, v.y);
            tile[i][2 * tx + 1] = make_float2(v.z, v.w);
        }
    }
    __syncthreads();
    for (int i = ty; i < kTile; i += step) {
        if (full || (c0 + i < cols && r0 + 2 * tx < rows)) {
            const float2 a = tile[2 * tx][i], c = tile[2 * tx + 1][i];
            *reinterpret_cast<float4*>(dst + (c0 + i) * rows + r0 + 2 * tx) = make_float4(a.x, a.y, c.x, c.y);
        }
    }
}

hipError_t launch_transpose(const float2* in, float2* out, long long rows, long long cols, long long batch,
                            hipStream_t st)
{
    const long long tr = (rows + kTile - 1) / kTile;
    const long long tc = (cols + kTile - 1) / kTile;
    const long long grid = tr * tc * batch;
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool vec = (rows % 2 == 0) && (cols % 2 == 0) && ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0);
    if (vec)
        hipLaunchKernelGGL(k_transpose16, dim3((unsigned)grid), dim3(kTransposeThreads), 0, st, in, out, rows, cols,
                           tr, tc);
    else
        hipLaunchKernelGGL(k_transpose, dim3((unsigned)grid), dim3(kTransposeThreads), 0, st, in, out, rows, cols,
                           tr, tc);
    return hipGetLastError();
}

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;

__global__ void __launch_bounds__(kCopyThreads)
k_copy(const float4* __restrict__ in, float4* __restrict__ out, long long n16)
{
    const long long stride = (long long)gridDim.x * kCopyThreads * kCopyUnroll;
    for (long long base = (long long)blockIdx.x * kCopyThreads * kCopyUnroll + threadIdx.x; base < n16;
         base += stride) {
        float4 r[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const long long i = base + (long long)u * kCopyThreads;
            if (i < n16) r[u] = in[i];
        }
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const long long i = base + (long long)u * kCopyThreads;
            if (i < n16) out[i] = r[u];
        }
    }
}

hipError_t launch_copy(const void* in, void* out, size_t bytes, hipStream_t st)
{
    const long long n16 = (long long)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    long long blocks = (n16 + kCopyThreads * kCopyUnroll - 1) / (kCopyThreads * kCopyUnroll);
    if (blocks > 256LL * 64) blocks = 256LL * 64;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kCopyThreads), 0, st, (const float4*)in, (float4*)out,
                       n16);
    return hipGetLastError();
}

}  // namespace fb
