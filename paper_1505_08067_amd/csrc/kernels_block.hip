// Single-block batched FFT: one LDS-resident transform per group of threads.
//
// Paper, Approach: the elementary FFT block is sized to what one compute
// unit holds on chip, and each task reads all its inputs, computes, and
// writes all its outputs ("Top level analysis": Read / Compute / Write).  On
// gfx950 a workgroup of T = N/E threads holds E complex values per thread in
// VGPRs; radix stages run in registers, and between stages the values are
// exchanged through the CU's LDS (160 KB) with one barrier pair per stage.
// The first stage reads global memory directly and the last stage writes it
// directly; both are coalesced (consecutive lanes touch consecutive complex
// values) because Stockham's first-stage input stride and last-stage output
// stride are both N/R.
//
// FPB transforms share one workgroup when N is small, so a workgroup always
// has at least 64 threads (one wave64).
#include "fft_device.hpp"
#include "internal.hpp"

namespace fb {

template <int N, int E, int FPB, class S>
__global__ void __launch_bounds__((N / E) * FPB)
k_block(const float2* __restrict__ in, float2* __restrict__ out, const float2* __restrict__ tw,
        long long batch, float sg)
{
    constexpr int T = N / E;
    constexpr int NST = S::count;
    constexpr int LDSN = lds_pad(N) + 1;
    static_assert(S::n() == N, "schedule does not multiply to N");
    __shared__ float2 lds[NST > 1 ? FPB * LDSN : 1];

    const int tid = threadIdx.x;
    const int f = tid / T;
    const int t = tid - f * T;
    const long long b = (long long)blockIdx.x * FPB + f;
    const bool act = b < batch;
    const float2* __restrict__ src = in + (act ? b : 0) * (long long)N;
    float2* __restrict__ dst = out + b * (long long)N;
    float2* L = lds + (NST > 1 ? f * LDSN : 0);

    float2 v[E];
    {
        constexpr int R = S::r(0);
#pragma unroll
        for (int i = 0; i < E / R; ++i)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 a = act ? src[t + i * T + r * (N / R)] : make_float2(0.f, 0.f);
                a.y *= sg;
                v[i * R + r] = a;
            }
    }

    sfor<0, NST>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int R = S::r(s);
        constexpr int Ns = S::ns(s);
        if constexpr (s > 0) {
#pragma unroll
            for (int i = 0; i < E / R; ++i)
#pragma unroll
                for (int r = 0; r < R; ++r) v[i * R + r] = L[lds_pad(t + i * T + r * (N / R))];
#pragma unroll
            for (int i = 0; i < E / R; ++i) {
                const int k = (t + i * T) % Ns;
                apply_row<R>(&v[i * R], tw + S::tw_off(s) + k * R);
            }
        }
#pragma unroll
        for (int i = 0; i < E / R; ++i) Dft<R>::run(&v[i * R]);
        if constexpr (s < NST - 1) {
            if constexpr (s > 0) __syncthreads();
#pragma unroll
            for (int i = 0; i < E / R; ++i) {
                const int j = t + i * T;
                const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
                for (int q = 0; q < R; ++q) L[lds_pad(base + q * Ns)] = v[i * R + q];
            }
            __syncthreads();
        } else {
            if (act) {
#pragma unroll
                for (int i = 0; i < E / R; ++i)
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        float2 a = v[i * R + q];
                        a.y *= sg;
                        dst[t + i * T + q * Ns] = a;
                    }
            }
        }
    });
}

template <int N, int E, int FPB, class S>
hipError_t launch_block(const float2* in, float2* out, const float2* tw, long long batch, float sg, hipStream_t st)
{
    const long long grid = (batch + FPB - 1) / FPB;
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_block<N, E, FPB, S>), dim3((unsigned)grid), dim3((N / E) * FPB), 0, st, in, out, tw,
                       batch, sg);
    return hipGetLastError();
}

template <int N, int E, int FPB, class S>
constexpr BlockEntry block_entry(const char* name)
{
    BlockEntry b{};
    b.n = N;
    b.e = E;
    b.fpb = FPB;
    b.nr = S::count;
    for (int i = 0; i < S::count && i < 8; ++i) b.radix[i] = S::r(i);
    b.tw_size = S::tw_size();
    b.threads = (N / E) * FPB;
    b.lds = S::count > 1 ? (size_t)FPB * (lds_pad(N) + 1) * sizeof(float2) : sizeof(float2);
    b.launch = &launch_block<N, E, FPB, S>;
    b.name = name;
    return b;
}

#define FB_BLOCK(N, E, FPB, ...) block_entry<N, E, FPB, Sched<__VA_ARGS__>>("block_fft<" #N ",[" #__VA_ARGS__ "]>")

// The first entry for each N is the planner's default schedule.
static const BlockEntry kBlocks[] = {
    FB_BLOCK(2, 2, 256, 2),
    FB_BLOCK(4, 4, 256, 4),
    FB_BLOCK(8, 8, 256, 8),
    FB_BLOCK(16, 16, 256, 16),
    FB_BLOCK(32, 16, 128, 16, 2),
    FB_BLOCK(64, 16, 64, 16, 4),
    FB_BLOCK(128, 16, 32, 16, 8),
    FB_BLOCK(256, 16, 16, 16, 16),
    FB_BLOCK(512, 16, 8, 16, 16, 2),
    FB_BLOCK(1024, 16, 4, 16, 16, 4),
    FB_BLOCK(2048, 16, 2, 16, 16, 8),
    FB_BLOCK(4096, 16, 1, 16, 16, 16),
    FB_BLOCK(8192, 32, 1, 32, 16, 16),
    FB_BLOCK(16384, 16, 1, 16, 16, 16, 4),
    // alternative schedules (radix search / sweep)
    FB_BLOCK(512, 8, 4, 8, 8, 8),
    FB_BLOCK(1024, 16, 4, 4, 16, 16),
    FB_BLOCK(1024, 8, 2, 4, 8, 8, 4),
    FB_BLOCK(1024, 8, 2, 8, 8, 4, 4),
    FB_BLOCK(1024, 8, 2, 8, 8, 8, 2),
    FB_BLOCK(4096, 8, 1, 8, 8, 8, 8),
    FB_BLOCK(4096, 16, 1, 4, 16, 16, 4),
    FB_BLOCK(8192, 16, 1, 16, 16, 16, 2),
    FB_BLOCK(8192, 32, 1, 16, 16, 32),
    FB_BLOCK(16384, 32, 1, 32, 32, 16),
};

const BlockEntry* block_default(int n)
{
    for (const BlockEntry& b : kBlocks)
        if (b.n == n) return &b;
    return nullptr;
}

const BlockEntry* block_table(int* count)
{
    *count = (int)(sizeof(kBlocks) / sizeof(kBlocks[0]));
    return kBlocks;
}

}  // namespace fb
