// Block kernels whose radix schedule is a run-time argument (paper, Approach,
// "FFT performance model": the schedule is the shortest path through the
// stage graph, whichever composition of radices that turns out to be).  The
// compiled kernels cover a fixed catalogue of schedules; the shortest path
// over measured stage costs can be any sequence of radices 2, 4, 8 and 16
// whose product is the length, so it runs here.
//
// The kernel is the Stockham form of the compiled block kernel with sixteen
// values per thread (every radix of the set divides 16): each stage reads its
// inputs from LDS (stage 0 from global memory), multiplies by its twiddle row
// (exact rows w_{Ns R}^{k r}, one FP64-to-FP32 rounding each), runs R-point
// DFTs and writes to LDS (the last stage to global memory, natural order).
// A stage dispatches on its radix to a body compiled for that radix, so the
// sixteen values stay in registers; what varies at run time is only the
// stride Ns, a power of two (shifts and masks).
#include "fft_kernel.hpp"

namespace fb {

namespace {

constexpr int kRtE = 16;

// Stage s > 0 of radix R: gather from LDS, twiddle.
template <int R, int N, int T, int FL>
__device__ __forceinline__ void rt_gather(float2 (&v)[kRtE], const float2* L, const float2* __restrict__ row0,
                                          int t, int lns)
{
#pragma unroll
    for (int i = 0; i < kRtE / R; ++i)
#pragma unroll
        for (int r = 0; r < R; ++r) v[i * R + r] = L[lds_at<FL>(t + i * T + r * (N / R))];
#pragma unroll
    for (int i = 0; i < kRtE / R; ++i) {
        const int k = (t + i * T) & ((1 << lns) - 1);
        apply_row<R>(&v[i * R], row0 + k * R);
    }
}

template <int R>
__device__ __forceinline__ void rt_dft(float2 (&v)[kRtE])
{
#pragma unroll
    for (int i = 0; i < kRtE / R; ++i) Dft<R>::run(&v[i * R]);
}

// Outputs of a radix-R stage after Ns = 2^lns points, to LDS: butterfly
// j = t + i T writes slots Ns (R floor(j / Ns)) + j mod Ns + q Ns.
template <int R, int T, int FL>
__device__ __forceinline__ void rt_scatter(const float2 (&v)[kRtE], float2* L, int t, int lns)
{
    constexpr int LR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
#pragma unroll
    for (int i = 0; i < kRtE / R; ++i) {
        const int j = t + i * T;
        const int base = ((j >> lns) << (lns + LR)) + (j & ((1 << lns) - 1));
#pragma unroll
        for (int q = 0; q < R; ++q) L[lds_at<FL>(base + (q << lns))] = v[i * R + q];
    }
}

// Stage-0 inputs x[t + i T + r N / R0] from global memory.
template <int R, int N, int T, int FL>
__device__ __forceinline__ void rt_load(float2 (&v)[kRtE], const float2* src, int t)
{
#pragma unroll
    for (int i = 0; i < kRtE / R; ++i)
#pragma unroll
        for (int r = 0; r < R; ++r) v[i * R + r] = gload<FL>(src + t + i * T + r * (N / R));
}

// Last-stage outputs X[t + i T + q N / R] to global memory.
template <int R, int N, int T, int FL>
__device__ __forceinline__ void rt_store(const float2 (&v)[kRtE], float2* dst, int t)
{
#pragma unroll
    for (int i = 0; i < kRtE / R; ++i)
#pragma unroll
        for (int q = 0; q < R; ++q) gstore<FL>(dst + t + i * T + q * (N / R), v[i * R + q]);
}

}  // namespace

// a.sched: log2 of each stage's radix, four bits per stage, stage 0 in the
// lowest bits; a zero nibble ends the schedule.  The twiddle block of stage
// s >= 1 (Ns R entries) follows those of the earlier stages.
template <int N, int C, int FL>
__global__ void __launch_bounds__((N / kRtE) * C) k_fft_rt(KArgs a)
{
    constexpr int T = N / kRtE;
    constexpr int LDSN = lds_stride<N, FL, false, C, T>();
    __shared__ __attribute__((aligned(16))) float2 lds[C * LDSN];
    const int tid = threadIdx.x;
    const int f = tid / T, t = tid % T;
    float2* L = lds + f * LDSN;
    const long long b = (long long)blockIdx.x * C + f;
    const bool act = b < a.batch;
    const float2* src = a.in + (act ? b : 0) * N;
    float2* dst = a.out + (act ? b : 0) * N;
    const bool bwd = a.sg < 0.f;
    const unsigned sched = a.sched;
    int nst = 0;
    while (nst < 8 && ((sched >> (4 * nst)) & 15u) != 0) ++nst;

    float2 v[kRtE];
    if (act) {
        switch (sched & 15u) {
            case 1: rt_load<2, N, T, FL>(v, src, t); break;
            case 2: rt_load<4, N, T, FL>(v, src, t); break;
            case 3: rt_load<8, N, T, FL>(v, src, t); break;
            default: rt_load<16, N, T, FL>(v, src, t); break;
        }
    } else {
#pragma unroll
        for (int e = 0; e < kRtE; ++e) v[e] = make_float2(0.f, 0.f);
    }
    if (bwd) {
#pragma unroll
        for (int e = 0; e < kRtE; ++e) v[e].y = -v[e].y;
    }
    int lns = 0;         // log2 of the points combined before this stage
    long long toff = 0;  // this stage's twiddle block
    for (int s = 0; s < nst; ++s) {
        const int lr = (int)((sched >> (4 * s)) & 15u);
        if (s > 0) {
            const float2* row0 = a.tw + toff;
            switch (lr) {
                case 1: rt_gather<2, N, T, FL>(v, L, row0, t, lns); break;
                case 2: rt_gather<4, N, T, FL>(v, L, row0, t, lns); break;
                case 3: rt_gather<8, N, T, FL>(v, L, row0, t, lns); break;
                default: rt_gather<16, N, T, FL>(v, L, row0, t, lns); break;
            }
            toff += 1LL << (lns + lr);
        }
        switch (lr) {
            case 1: rt_dft<2>(v); break;
            case 2: rt_dft<4>(v); break;
            case 3: rt_dft<8>(v); break;
            default: rt_dft<16>(v); break;
        }
        if (s < nst - 1) {
            if (s > 0) __syncthreads();  // every read of the last exchange precedes these writes
            switch (lr) {
                case 1: rt_scatter<2, T, FL>(v, L, t, lns); break;
                case 2: rt_scatter<4, T, FL>(v, L, t, lns); break;
                case 3: rt_scatter<8, T, FL>(v, L, t, lns); break;
                default: rt_scatter<16, T, FL>(v, L, t, lns); break;
            }
            __syncthreads();
        } else if (act) {
            if (bwd) {
#pragma unroll
                for (int e = 0; e < kRtE; ++e) v[e].y = -v[e].y;
            }
            if (a.scale != 1.f) {
#pragma unroll
                for (int e = 0; e < kRtE; ++e) v[e] = make_float2(v[e].x * a.scale, v[e].y * a.scale);
            }
            int ts = t;  // see the compiled kernel's store: keeps the store offsets out of the stages
            asm volatile("" : "+v"(ts));
            __builtin_assume(ts >= 0 && ts < T);
            switch (lr) {
                case 1: rt_store<2, N, T, FL>(v, dst, ts); break;
                case 2: rt_store<4, N, T, FL>(v, dst, ts); break;
                case 3: rt_store<8, N, T, FL>(v, dst, ts); break;
                default: rt_store<16, N, T, FL>(v, dst, ts); break;
            }
        }
        lns += lr;
    }
}

template <int N, int C, int FL>
hipError_t launch_fft_rt(const KArgs& a, long long grid, hipStream_t st, hipEvent_t start, hipEvent_t stop)
{
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    if (start || stop)
        hipExtLaunchKernelGGL((k_fft_rt<N, C, FL>), dim3((unsigned)grid), dim3((N / kRtE) * C), 0, st, start, stop, 0,
                              a);
    else
        hipLaunchKernelGGL((k_fft_rt<N, C, FL>), dim3((unsigned)grid), dim3((N / kRtE) * C), 0, st, a);
    return hipGetLastError();
}

template <int N, int C, int FL>
int occupancy_fft_rt()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void*)&k_fft_rt<N, C, FL>, (N / kRtE) * C, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

// Catalogue entry: no fixed schedule (nr = 0); the plan supplies it.
template <int N, int C, int FL>
constexpr KEntry make_rt_entry(const char* name)
{
    KEntry k{};
    k.kind = kKindBlock;
    k.n = N;
    k.e = kRtE;
    k.c = C;
    k.flags = FL | kRtSched;
    k.nr = 0;
    k.tw_size = 0;
    k.threads = (N / kRtE) * C;
    k.lds = (size_t)C * lds_stride<N, FL, false, C, N / kRtE>() * sizeof(float2);
    k.is_default = false;
    k.launch = &launch_fft_rt<N, C, FL>;
    k.occupancy = &occupancy_fft_rt<N, C, FL>;
    k.name = name;
    k.fn = reinterpret_cast<const void*>(&k_fft_rt<N, C, FL>);
    return k;
}

// Streaming loads and stores (3), as the compiled defaults; 256 threads per
// workgroup up to 4096, one transform per workgroup beyond.
static const KEntry kRt[] = {
    make_rt_entry<64, 64, 3>("block_fft_rt<64>"),
    make_rt_entry<128, 32, 3>("block_fft_rt<128>"),
    make_rt_entry<256, 16, 3>("block_fft_rt<256>"),
    make_rt_entry<512, 8, 3>("block_fft_rt<512>"),
    make_rt_entry<1024, 4, 3>("block_fft_rt<1024>"),
    make_rt_entry<2048, 2, 3>("block_fft_rt<2048>"),
    make_rt_entry<4096, 1, 3>("block_fft_rt<4096>"),
    make_rt_entry<8192, 1, 3>("block_fft_rt<8192>"),
    make_rt_entry<16384, 1, 3>("block_fft_rt<16384>"),
};

const KEntry* rt_entries(int* count)
{
    *count = (int)(sizeof(kRt) / sizeof(kRt[0]));
    return kRt;
}

}  // namespace fb
