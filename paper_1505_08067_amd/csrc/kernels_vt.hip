// Block kernels whose stages run on different numbers of threads (paper,
// Approach: the elementary FFT block, mixed radices when N is not a power
// of one radix).
//
// In the Stockham form every thread holds E values and runs E/R butterflies
// of a radix-R stage, so E must be a multiple of every radix of the
// schedule: a length with factors 2, 3 and 5 (15360 = 2^10 * 3 * 5) needs 60
// values per thread, which takes the whole register file of a SIMD for one
// wave.  Here the workgroup has T threads and stage s runs its N/R_s
// butterflies on T_s <= T of them, b_s = ceil((N/R_s) / T) per thread, so a
// thread holds at most max_s b_s R_s values (16 for 15360 as
// [15, 16, 16, 4] on 1024 threads).  The threads a stage leaves idle keep
// to its barriers.  Stage formulas, twiddle table and LDS layout are those
// of the Stockham kernel: butterfly j of stage s (Ns points combined before
// it) reads slots j + r N/R_s and writes slots (j / Ns) Ns R_s + j mod Ns +
// q Ns.  One transform per workgroup.
//
// Half exchanges (kHalfX): when every stage but the last runs an even number
// of butterflies per thread and every stage after the first has an even
// radix, the butterflies j < N/2R of a stage (the first half of each
// thread's) write exactly the lower N/2 slots, and the next stage's inputs
// r < R'/2 are exactly those slots, so each exchange runs in two rounds
// through N/2 slots: half the LDS per workgroup.
#include <type_traits>

#include "fft_kernel.hpp"

namespace fb {

namespace {

template <int N, int T, class S>
struct VtShape {
    static constexpr int bpt(int s) { return (N / S::r(s) + T - 1) / T; }  // butterflies per thread
    static constexpr int ts(int s) { return (N / S::r(s)) / bpt(s); }       // threads the stage uses
    static constexpr int es(int s) { return bpt(s) * S::r(s); }             // values per thread
    static constexpr int emax()
    {
        int m = 1;
        for (int s = 0; s < S::count; ++s) m = es(s) > m ? es(s) : m;
        return m;
    }
    static constexpr bool valid()
    {
        for (int s = 0; s < S::count; ++s)
            if ((N / S::r(s)) % bpt(s) != 0 || ts(s) > T) return false;
        return S::n() == N;
    }
    static constexpr bool half_ok()
    {
        for (int s = 0; s + 1 < S::count; ++s)
            if (bpt(s) % 2 != 0 || S::r(s + 1) % 2 != 0) return false;
        return true;
    }
};

}  // namespace

template <int N, int T, class S, int FL>
__global__ void __launch_bounds__(T) k_fft_vt(KArgs a)
{
    using V = VtShape<N, T, S>;
    static_assert(V::valid(), "every stage must split its butterflies evenly over at most T threads");
    constexpr bool HX = (FL & kHalfX) != 0;
    static_assert(!HX || V::half_ok(), "half exchanges need even butterfly counts and even radices after stage 0");
    constexpr int E = V::emax();
    constexpr int NST = S::count;
    constexpr int LDSN = lds_pad(HX ? N / 2 : N) + 1;
    __shared__ __attribute__((aligned(16))) float2 L[LDSN];

    const int t = threadIdx.x;
    const long long b = blockIdx.x;
    const bool act = b < a.batch;  // the same in the whole workgroup
    // complex64 or FP16 pairs in HBM (FP32 arithmetic either way)
    using TD = std::conditional_t<(FL & kF16Data) != 0, h2_t, float2>;
    const TD* src = reinterpret_cast<const TD*>(a.in) + (act ? b : 0) * N;
    TD* dst = reinterpret_cast<TD*>(a.out) + (act ? b : 0) * N;
    const bool bwd = a.sg < 0.f;

    float2 v[E];
    sfor<0, NST>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int R = S::r(s);
        constexpr int Ns = S::ns(s);
        constexpr int BP = V::bpt(s);
        constexpr int TS = V::ts(s);
        const bool on = t < TS;
        if constexpr (s == 0) {
            if (on && act) {
#pragma unroll
                for (int i = 0; i < BP; ++i)
#pragma unroll
                    for (int r = 0; r < R; ++r) v[i * R + r] = gload<FL>(src + t + i * TS + r * (N / R));
                if (bwd) {
#pragma unroll
                    for (int e = 0; e < BP * R; ++e) v[e].y = -v[e].y;
                }
            }
        } else if (on) {
            if constexpr (!HX) {
#pragma unroll
                for (int i = 0; i < BP; ++i)
#pragma unroll
                    for (int r = 0; r < R; ++r) v[i * R + r] = L[lds_pad(t + i * TS + r * (N / R))];
            }  // half exchanges read this stage's inputs during the exchange itself
#pragma unroll
            for (int i = 0; i < BP; ++i) {
                const int k = (t + i * TS) % Ns;
                if constexpr ((FL & kTwPow) != 0)
                    apply_pow_row<R>(&v[i * R], a.tw + S::ptw_off(s) + k * S::p_row(s));
                else
                    apply_row<R>(&v[i * R], a.tw + S::tw_off(s) + k * R);
            }
        }
        if (on) {
#pragma unroll
            for (int i = 0; i < BP; ++i) Dft<R>::run(&v[i * R]);
        }
        if constexpr (s < NST - 1 && !HX) {
            if constexpr (s > 0) __syncthreads();  // every read of the last exchange precedes these writes
            if (on) {
#pragma unroll
                for (int i = 0; i < BP; ++i) {
                    const int j = t + i * TS;
                    const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
                    for (int q = 0; q < R; ++q) L[lds_pad(base + q * Ns)] = v[i * R + q];
                }
            }
            __syncthreads();
        } else if constexpr (s < NST - 1) {
            // round h: butterflies [h BP/2, (h+1) BP/2) of this stage write
            // half h of the slots; the next stage reads its inputs
            // r in [h R2/2, (h+1) R2/2) from them
            constexpr int R2 = S::r(s + 1);
            constexpr int BP2 = V::bpt(s + 1);
            constexpr int TS2 = V::ts(s + 1);
            float2 w[E];
            sfor<0, 2>([&](auto hc) {
                constexpr int h = decltype(hc)::value;
                if constexpr (h > 0 || s > 0) __syncthreads();  // earlier reads precede these writes
                if (on) {
#pragma unroll
                    for (int i = h * (BP / 2); i < (h + 1) * (BP / 2); ++i) {
                        const int j = t + i * TS;
                        const int base = (j / Ns) * Ns * R + (j % Ns) - h * (N / 2);
#pragma unroll
                        for (int q = 0; q < R; ++q) L[lds_pad(base + q * Ns)] = v[i * R + q];
                    }
                }
                __syncthreads();
                if (t < TS2) {
#pragma unroll
                    for (int i2 = 0; i2 < BP2; ++i2)
#pragma unroll
                        for (int r = h * (R2 / 2); r < (h + 1) * (R2 / 2); ++r)
                            w[i2 * R2 + r] = L[lds_pad(t + i2 * TS2 + r * (N / R2) - h * (N / 2))];
                }
            });
#pragma unroll
            for (int e = 0; e < BP2 * R2; ++e) v[e] = w[e];
        } else if (on && act) {
            // last stage: Ns R = N, so output q of butterfly j is X[j + q Ns]
            if (bwd) {
#pragma unroll
                for (int e = 0; e < BP * R; ++e) v[e].y = -v[e].y;
            }
            if (a.scale != 1.f) {
#pragma unroll
                for (int e = 0; e < BP * R; ++e) v[e] = make_float2(v[e].x * a.scale, v[e].y * a.scale);
            }
            int tsx = t;  // store offsets formed afresh (not kept live from the stages)
            asm volatile("" : "+v"(tsx));
            __builtin_assume(tsx >= 0 && tsx < TS);
#pragma unroll
            for (int i = 0; i < BP; ++i)
#pragma unroll
                for (int q = 0; q < R; ++q) gstore<FL>(dst + tsx + i * TS + q * Ns, v[i * R + q]);
        }
    });
}

template <int N, int T, class S, int FL>
hipError_t launch_fft_vt(const KArgs& a, long long grid, hipStream_t st, hipEvent_t start, hipEvent_t stop)
{
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    if (start || stop)
        hipExtLaunchKernelGGL((k_fft_vt<N, T, S, FL>), dim3((unsigned)grid), dim3(T), 0, st, start, stop, 0, a);
    else
        hipLaunchKernelGGL((k_fft_vt<N, T, S, FL>), dim3((unsigned)grid), dim3(T), 0, st, a);
    return hipGetLastError();
}

template <int N, int T, class S, int FL>
int occupancy_fft_vt()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void*)&k_fft_vt<N, T, S, FL>, T, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

template <int N, int T, class S, int FL>
constexpr KEntry make_vt_entry(bool is_default, const char* name)
{
    KEntry k{};
    k.kind = kKindBlock;
    k.n = N;
    k.e = VtShape<N, T, S>::emax();
    k.c = 1;
    k.flags = FL;
    k.nr = S::count;
    for (int i = 0; i < S::count && i < 8; ++i) k.radix[i] = S::r(i);
    k.tw_size = (FL & kTwPow) != 0 ? S::ptw_size() : S::tw_size();
    k.threads = T;
    k.lds = (size_t)(lds_pad((FL & kHalfX) != 0 ? N / 2 : N) + 1) * sizeof(float2);
    k.is_default = is_default;
    k.launch = &launch_fft_vt<N, T, S, FL>;
    k.occupancy = &occupancy_fft_vt<N, T, S, FL>;
    k.name = name;
    k.fn = reinterpret_cast<const void*>(&k_fft_vt<N, T, S, FL>);
    return k;
}

#define FB_VT(DEF, FL, N, T, ...) \
    make_vt_entry<N, T, Sched<__VA_ARGS__>, FL>(DEF, "block_fft_vt<" #N ",T" #T ",[" #__VA_ARGS__ "],v" #FL ">")
#define FB_VTH(DEF, FL, N, T, ...) \
    make_vt_entry<N, T, Sched<__VA_ARGS__>, FL>(DEF, "block_fft_vt_f16<" #N ",T" #T ",[" #__VA_ARGS__ "],v" #FL ">")

// 35 = streaming loads and stores + power-row twiddles; 65536 = stages on
// different thread counts.  The defaults for 15360 and 6000 (complex64):
// 2^24 points, 70.4 (half exchanges, 512 threads) and 72.2 (1024 threads)
// against 106.2 us for [12,20,4,4,4] at 60 values per thread, and 59.8
// against 65.1 us for [10,10,10,6] at 30.  Exact twiddle
// rows instead of power rows: 89.5 against 72.3 us at 15360, 66.7 against
// 62.2 at 6000 (the rows' cache traffic).
static const KEntry kVt[] = {
    FB_VT(false, 65571, 15360, 1024, 15, 16, 16, 4),
    FB_VT(false, 65571, 15360, 1024, 16, 16, 15, 4),
    FB_VT(false, 65571, 15360, 1024, 16, 15, 16, 4),
    // half exchanges: 512 threads, two workgroups per CU (70.4 against 72.2 us)
    FB_VT(true, 66595, 15360, 512, 15, 16, 16, 4),
    FB_VT(false, 65571, 6000, 600, 10, 10, 10, 6),
    FB_VT(true, 65571, 6000, 600, 12, 10, 10, 5),
    // FP16 storage (64): the same kernels reading and writing FP16 pairs.
    // Defaults (FP16, 2^24 points, interleaved medians): 15360 on 1024
    // threads 51.9 against 86.0 us for the fixed-E kernel (60 values per
    // thread; 56.9 with half exchanges on 512 threads), 6000 as [10,10,10,6]
    // 45.8 against 51.5 us
    FB_VTH(false, 66659, 15360, 512, 15, 16, 16, 4),
    FB_VTH(true, 65635, 15360, 1024, 16, 16, 15, 4),
    FB_VTH(false, 65635, 6000, 600, 12, 10, 10, 5),
    FB_VTH(true, 65635, 6000, 600, 10, 10, 10, 6),
};

const KEntry* vt_entries(int* count)
{
    *count = (int)(sizeof(kVt) / sizeof(kVt[0]));
    return kVt;
}

}  // namespace fb
