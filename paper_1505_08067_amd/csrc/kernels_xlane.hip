// Block kernels whose intra-wave exchanges are register permutations
// (paper, Approach: the elementary FFT block; the radix stages run in
// registers and exchange data between stages).  When a whole transform lives
// in one wavefront, an exchange only moves values between the lanes and
// registers of that wavefront, which the VALU can do directly instead of a
// round trip through LDS.
//
// N = 1024, one transform per wave64, sixteen values per lane, schedule
// [16, 4, 16] in decimation-in-frequency order.  With n = a + 16 b + 64 c
// (a < 16, b < 4, c < 16) and k = d + 16 e + 64 f (d < 16, e < 4, f < 16):
//
//   X[k] = sum_a w16^{a f} w64^{a e} sum_b w4^{b e} w1024^{(a + 16 b) d}
//                                            sum_c w16^{c d} x[n]
//
// Lane l, register r first hold x[l + 64 r]: l = a + 16 b, r = c.
//   stage 1: 16-point DFTs over the registers (c -> d), then w1024^{l d};
//   exchange 1: lane bits 4, 5 (b) swap with register bits 2, 3 (d2, d3);
//   stage 2: 4-point DFTs over register bits 2, 3 (b -> e), then w64^{a e};
//   exchange 2: lane bits 0..3 (a) swap with the four register bits;
//   stage 3: 16-point DFTs over the registers (a -> f).
// The twiddle factors are the power rows of the Stockham schedule [16, 4, 16]
// (its stage-2 rows are w1024^{k 2^i}, k < 64, its stage-1 rows w64^{k 2^i},
// k < 16), so the plan builds the same table for both.
//
// Swapping lane bit m with register bit p: for each register pair
// (A = v[r], B = v[r + 2^p], bit p of r clear), with h = lane bit m,
//   A' = h ? B of lane l ^ 2^m : A,      B' = h ? B : A of lane l ^ 2^m.
// Lane bits 5 and 4 (the other half-wave, the other row of 16 lanes) are one
// gfx950 v_permlane32_swap / v_permlane16_swap per 32-bit register pair; lane
// bits 3 and 2 (the other bank of four lanes in the row) are one DPP row
// shift per value with a bank mask selecting the lanes it writes; lane bits 1
// and 0 (within a bank of four lanes) are a DPP quad permutation and a
// select per value.
//
// Two forms of exchange 2: through LDS (wave-synchronous, no workgroup
// barrier; slot 65 a + d + 16 e, read back as 16 values per lane at
// 65 a + l', which leaves lane l' = d + 16 e holding k = l' + 64 f), or in
// registers (no LDS at all; the outputs are then in lane order
// l = d0 + 2 d1 + 4 e0 + 8 e1 + 16 d2 + 32 d3, still 64 consecutive values
// per store instruction).
#include <type_traits>

#include "fft_kernel.hpp"

namespace fb {

namespace {

constexpr int kXlN = 1024;
constexpr int kXlE = 16;
constexpr int kXlSlots = 1040;  // LDS slots per transform for exchange 2 (65 * 15 + 64, even)

template <int CTRL, int BANK>
__device__ __forceinline__ float upd(float old, float src)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), CTRL, 0xF, BANK, false));
}

template <int QP>
__device__ __forceinline__ float qperm(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), QP, 0xF, 0xF, true));
}

// Exchange lane bit M with the register bit that separates A and B.
template <int M>
__device__ __forceinline__ void swap_bit(float& A, float& B, bool h)
{
    if constexpr (M == 5) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(A), __float_as_uint(B), false, false);
        A = __uint_as_float(r[0]);
        B = __uint_as_float(r[1]);
    } else if constexpr (M == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(A), __float_as_uint(B), false, false);
        A = __uint_as_float(r[0]);
        B = __uint_as_float(r[1]);
    } else if constexpr (M == 3) {
        // row_shr:8 (lane i reads i - 8) into banks 2, 3; row_shl:8 into banks 0, 1
        const float a2 = upd<0x118, 0xC>(A, B);
        const float b2 = upd<0x108, 0x3>(B, A);
        A = a2;
        B = b2;
    } else if constexpr (M == 2) {
        // row_shr:4 into banks 1, 3; row_shl:4 into banks 0, 2
        const float a2 = upd<0x114, 0xA>(A, B);
        const float b2 = upd<0x104, 0x5>(B, A);
        A = a2;
        B = b2;
    } else {
        // quad_perm [2,3,0,1] (lane ^ 2) or [1,0,3,2] (lane ^ 1)
        constexpr int QP = M == 1 ? 0x4E : 0xB1;
        const float pa = qperm<QP>(A), pb = qperm<QP>(B);
        A = h ? pb : A;
        B = h ? B : pa;
    }
}

template <int M, int P>
__device__ __forceinline__ void swap_bits(float2 (&v)[kXlE], int lane)
{
    const bool h = ((lane >> M) & 1) != 0;
#pragma unroll
    for (int r = 0; r < kXlE; ++r) {
        if ((r >> P) & 1) continue;
        swap_bit<M>(v[r].x, v[r + (1 << P)].x, h);
        swap_bit<M>(v[r].y, v[r + (1 << P)].y, h);
    }
}

}  // namespace

// LDSX: exchange 2 through LDS (true) or in registers (false); C transforms
// (waves) per workgroup.
template <int FL, bool LDSX, int C>
__global__ void __launch_bounds__(64 * C) k_fft_xl1024(KArgs a)
{
    constexpr int N = kXlN;
    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63;
    const long long b = (long long)blockIdx.x * C + w;
    const bool act = b < a.batch;  // the same in every lane of the wave
    // complex64 or FP16 pairs in HBM (FP32 arithmetic either way)
    using TD = std::conditional_t<(FL & kF16Data) != 0, h2_t, float2>;
    const TD* src = reinterpret_cast<const TD*>(a.in) + (act ? b : 0) * N;
    TD* dst = reinterpret_cast<TD*>(a.out) + (act ? b : 0) * N;
    const bool bwd = a.sg < 0.f;

    float2 v[kXlE];
    if (act) {
#pragma unroll
        for (int r = 0; r < kXlE; ++r) v[r] = gload<FL>(src + l + 64 * r);
    } else {
#pragma unroll
        for (int r = 0; r < kXlE; ++r) v[r] = make_float2(0.f, 0.f);
    }
    if (bwd) {
#pragma unroll
        for (int r = 0; r < kXlE; ++r) v[r].y = -v[r].y;
    }

    // stage 1: c -> d, then w1024^{l d} (power row l of the table's second block)
    Dft<16>::run(v);
    apply_pow_row<16>(v, a.tw + 32 + l * 4);

    // exchange 1: b (lane bits 4, 5) into register bits 2, 3
    swap_bits<5, 3>(v, l);
    swap_bits<4, 2>(v, l);

    // stage 2: b -> e over register bits 2, 3, then w64^{a e} (power row a of the first block)
    {
        const float2* row = a.tw + (l & 15) * 2;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float2 u[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) u[i] = v[q + 4 * i];
            Dft<4>::run(u);
            apply_pow_row<4>(u, row);
#pragma unroll
            for (int i = 0; i < 4; ++i) v[q + 4 * i] = u[i];
        }
    }

    int ks;  // the lane's output offset: k = ks + 64 f
    if constexpr (LDSX) {
        // exchange 2 through this wave's own LDS slots (wave-synchronous)
        __shared__ __attribute__((aligned(16))) float2 lds[C * kXlSlots];
        float2* L = lds + w * kXlSlots;
        const int dhi = ((l >> 4) & 3) << 2;  // d2, d3
#pragma unroll
        for (int r = 0; r < kXlE; ++r) {
            const int d = (r & 3) | dhi, e = r >> 2;
            L[65 * (l & 15) + d + 16 * e] = v[r];
        }
        exch_sync<true>();
#pragma unroll
        for (int r = 0; r < kXlE; ++r) v[r] = L[65 * r + l];
        ks = l;
    } else {
        // exchange 2 in registers: lane bits 0..3 (a) with register bits 0..3
        swap_bits<3, 3>(v, l);
        swap_bits<2, 2>(v, l);
        swap_bits<1, 1>(v, l);
        swap_bits<0, 0>(v, l);
        ks = (l & 3) | (((l >> 2) & 3) << 4) | (((l >> 4) & 3) << 2);
    }

    // stage 3: a -> f
    Dft<16>::run(v);
    if (act) {
        if (bwd) {
#pragma unroll
            for (int r = 0; r < kXlE; ++r) v[r].y = -v[r].y;
        }
        if (a.scale != 1.f) {
#pragma unroll
            for (int r = 0; r < kXlE; ++r) v[r] = make_float2(v[r].x * a.scale, v[r].y * a.scale);
        }
        asm volatile("" : "+v"(ks));
#pragma unroll
        for (int r = 0; r < kXlE; ++r) gstore<FL>(dst + ks + 64 * r, v[r]);
    }
}

template <int FL, bool LDSX, int C>
hipError_t launch_fft_xl(const KArgs& a, long long grid, hipStream_t st, hipEvent_t start, hipEvent_t stop)
{
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    if (start || stop)
        hipExtLaunchKernelGGL((k_fft_xl1024<FL, LDSX, C>), dim3((unsigned)grid), dim3(64 * C), 0, st, start, stop, 0,
                              a);
    else
        hipLaunchKernelGGL((k_fft_xl1024<FL, LDSX, C>), dim3((unsigned)grid), dim3(64 * C), 0, st, a);
    return hipGetLastError();
}

template <int FL, bool LDSX, int C>
int occupancy_fft_xl()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void*)&k_fft_xl1024<FL, LDSX, C>, 64 * C, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

// Catalogue entry: schedule [16, 4, 16] with power-row twiddles (the plan
// builds that schedule's table).
template <int FL, bool LDSX, int C>
constexpr KEntry make_xl_entry(bool is_default, const char* name)
{
    using S = Sched<16, 4, 16>;
    KEntry k{};
    k.kind = kKindBlock;
    k.n = kXlN;
    k.e = kXlE;
    k.c = C;
    k.flags = FL;
    k.nr = S::count;
    for (int i = 0; i < S::count; ++i) k.radix[i] = S::r(i);
    k.tw_size = S::ptw_size();
    k.threads = 64 * C;
    k.lds = LDSX ? (size_t)C * kXlSlots * sizeof(float2) : 0;
    k.is_default = is_default;
    k.launch = &launch_fft_xl<FL, LDSX, C>;
    k.occupancy = &occupancy_fft_xl<FL, LDSX, C>;
    k.name = name;
    k.fn = reinterpret_cast<const void*>(&k_fft_xl1024<FL, LDSX, C>);
    return k;
}

static_assert(Sched<16, 4, 16>::ptw_off(2) == 32 && Sched<16, 4, 16>::p_row(2) == 4 &&
                  Sched<16, 4, 16>::p_row(1) == 2,
              "the kernel reads the power rows of [16, 4, 16] at these offsets");

// 35 = streaming loads and stores + power-row twiddles; 32768 = cross-lane
// exchanges; with 512 (wave-synchronous) the second exchange uses LDS.  The
// all-register form is the default at 1024 (complex64): on random data,
// 2^24 points cold, 46.0 against 49.7 us for [16,16,4] with LDS exchanges
// in the autotuner's timing, 45.7-46.9 against 46.4-50.1 in the bench's;
// its one-wave form (C = 1) serves small batches.
static const KEntry kXl[] = {
    make_xl_entry<35 | kCrossLane | kWaveSync, true, 4>(false, "block_fft_xl<1024,[16, 4, 16],v33315>"),
    make_xl_entry<35 | kCrossLane, false, 4>(true, "block_fft_xl<1024,[16, 4, 16],v32803>"),
    make_xl_entry<35 | kCrossLane, false, 1>(false, "block_fft_xl<1024,C1,[16, 4, 16],v32803>"),
    // FP16 storage (64): the same kernel reading and writing FP16 pairs
    // (1024 x 16384: 28.8 against 30.2 us for the FP16 default, within the
    // 2.2-2.7 us spread of the rounds, so not the default)
    make_xl_entry<99 | kCrossLane, false, 4>(false, "block_fft_xl_f16<1024,[16, 4, 16],v32867>"),
    make_xl_entry<99 | kCrossLane, false, 1>(false, "block_fft_xl_f16<1024,C1,[16, 4, 16],v32867>"),
};

const KEntry* xlane_entries(int* count)
{
    *count = (int)(sizeof(kXl) / sizeof(kXl[0]));
    return kXl;
}

}  // namespace fb
