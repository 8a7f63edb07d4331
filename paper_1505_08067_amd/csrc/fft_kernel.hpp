// The transform kernel shared by the single-block path and the two four-step
// passes (paper, Approach: one elementary FFT block per compute unit; each
// task reads all its inputs, computes, and writes all its outputs).
//
// A workgroup runs C transforms of length N with T = N/E threads each; every
// thread holds E complex values in VGPRs.  The radix stages of the schedule
// S run in registers; between stages the values are exchanged through LDS
// with a barrier pair.  The first stage reads global memory directly and the
// last stage writes it directly, so the only difference between the block
// kernel and the four-step passes is the address map (the policy P):
//
//   PolBlock : transform f of unit u is contiguous at (u*C + f) * N;
//              threads of one transform are consecutive lanes.
//   PolPass1 : column c0+f of a long transform viewed as N1 x N2 (row-major);
//              sample n at n*N2 + c0 + f.  Lanes run over f first, so every
//              wave reads runs of C consecutive complex values.  Outputs are
//              multiplied by exp(-2 pi i (c0+f) k / N) and written to the
//              workspace in blocks of CW consecutive k (layout
//              W[k / CW][n2][k mod CW]), so a block of rows is contiguous.
//   PolPass2 : row k1 = g*CW + f of the workspace; sample n2 at
//              g*N2*CW + n2*CW + f (contiguous across the workgroup).  Output
//              k2 goes to k1 + N1*k2: the corner turn is fused into the store.
//
// Variant flags (kNtLoad, kNtStore, kPipe, kSwz): non-temporal global loads
// and stores, persistent workgroups that prefetch the next unit's stage-0
// inputs while the current unit computes, and an XOR-swizzled unpadded LDS
// layout (one transform per 16-aligned bank group).
#pragma once

#include <hip/hip_ext.h>

#include "fft_device.hpp"
#include "internal.hpp"

namespace fb {

enum : int {
    kF16Data = 64,  // FP16 pairs in HBM (kernels that take their element type from the flags)
    kSwz = 8, kStaged = 16, kTwPow = 32, kXcd = 128, kStageStride = 256, kWaveSync = 512, kHalfX = 1024,
    kFitRegs = 2048,  // with kHalfX: registers fitted to every workgroup the halved LDS allows
    kLoop = 4096,     // persistent workgroups looping over units, without prefetch
    kRtSched = 8192,  // the radix schedule is a run-time argument (KArgs::sched)
    kVec16 = 16384,   // block layout: 16-byte global accesses, pairs of lanes swapping halves
    kCrossLane = 32768,  // intra-wave exchanges as register permutations (DPP, lane swaps)
    kVarThreads = 65536,  // stages on different thread counts (values per thread per stage)
    kF16Work = 524288     // four-step passes: the workspace holds FP16 pairs (with FP16 storage)
};

// Half exchanges (kHalfX): when every stage but the last runs an even number
// of butterflies per thread, the butterflies of one half write exactly the
// slots that hold one half of every input of the next stage, so each
// exchange (and the staged store of pass 1) runs in two rounds through an
// LDS buffer of N/2 values per transform: half the LDS per workgroup, more
// workgroups per CU.
template <int N, int FL>
__host__ __device__ constexpr int lds_points()
{
    return (FL & kHalfX) != 0 ? N / 2 : N;
}

// Synchronisation of an LDS exchange.  When every thread that exchanges
// through a buffer belongs to one wavefront (a whole transform per wave), its
// LDS operations are performed in issue order, so a compiler-level barrier
// is enough and the workgroup barrier is skipped: the wavefronts of a
// workgroup then run their stages independently.
template <bool WS>
__device__ __forceinline__ void exch_sync()
{
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Workgroup b of a grid of G is dispatched to XCD b mod 8.  The XCD-ordered
// variants give each XCD a contiguous range of work units, so neighbouring
// units (which share cache lines at the edges of their column or row
// ranges) meet in the same L2.  A bijection on [0, G) when 8 divides G, the
// identity otherwise.
__device__ __forceinline__ long long xcd_unit(long long b, long long G)
{
    if ((G & 7) != 0) return b;
    return (b & 7) * (G >> 3) + (b >> 3);
}

// LDS index map: padded (default) or XOR-swizzled within 16-value groups.
template <int FL>
__device__ __forceinline__ int lds_at(int i)
{
    if constexpr ((FL & kSwz) != 0) {
        return i ^ ((i >> 4) & 15);
    } else {
        return lds_pad(i);
    }
}

// Distance between the LDS buffers of the C transforms of a workgroup.
// Lanes that share a 16-lane group differ in their transform index f and in
// their position t: with f-fast lanes (C values of f, 16/C of t) the stride
// is made congruent to 16/C modulo 16, with t-fast lanes and T < 16 threads
// per transform it is made congruent to T, so every such group hits 16
// distinct 8-byte bank pairs.
template <int N, int FL, bool FFAST, int C, int T>
__host__ __device__ constexpr int lds_stride()
{
    if constexpr ((FL & kSwz) != 0) {
        return N;
    } else {
        int want = FFAST ? (C < 16 ? 16 / C : 1) : (T < 16 ? T : 1);
        // staged pass-1 stores read 16-lane groups spanning two transforms
        // CW = 8 values apart: a residue 8 larger (still odd for C = 16, so
        // the exchanges keep 16 distinct bank pairs) separates the two halves
        if constexpr ((FL & kStageStride) != 0) want += 8;
        int s = lds_pad(N);
        while ((s & 15) != (want & 15)) ++s;
        return s;
    }
}

// ----------------------------------------------------------------- policies
// TI / TO: element type of the data in HBM -- float2 (complex64) or h2_t
// (two FP16 values, the storage-only half precision form); arithmetic is
// always FP32.  The four-step workspace is always complex64.
template <typename TI, typename TO>
struct PolBlockT {
    static constexpr bool f_fast = false;
    static constexpr bool conj_in = true;
    static constexpr bool conj_out = true;
    static constexpr int kind = kKindBlock;
    struct Ctx {
        const TI* src;
        TO* dst;
        bool act;
    };
    template <int N, int C>
    __device__ static Ctx ctx(const KArgs& a, long long unit, int f)
    {
        const long long b = unit * C + f;
        Ctx c;
        c.act = b < a.batch;
        const long long bb = c.act ? b : 0;
        c.src = reinterpret_cast<const TI*>(a.in) + bb * N;
        c.dst = reinterpret_cast<TO*>(a.out) + bb * N;
        return c;
    }
    template <int C>
    __device__ static const TI* in_at(const KArgs&, const Ctx& c, int n)
    {
        return c.src + n;
    }
    template <int N, int E, int T, int RL, int NsL, int FL>
    __device__ static void twiddle_outputs(const KArgs&, const Ctx&, int, float2 (&)[E])
    {
    }
    template <int FL>
    __device__ static void store(const KArgs&, const Ctx& c, int k, float2 x)
    {
        gstore<FL>(c.dst + k, x);
    }
    __host__ __device__ static long long units(const KArgs& a, int C) { return (a.batch + C - 1) / C; }
};
using PolBlock = PolBlockT<float2, float2>;
using PolBlockH = PolBlockT<h2_t, h2_t>;

// List launches: transform b of the launch reads and writes where its
// descriptor points (the block layout otherwise).  The descriptors are read
// through the constant address space: pointers loaded from it are taken to
// address global memory, so the data accesses are global instructions (a
// pointer loaded from ordinary memory could point anywhere, and accesses
// through it would be flat ones, which also hold up every LDS wait).
struct PolList : PolBlock {
    static constexpr int kind = kKindList;
    template <int N, int C>
    __device__ static Ctx ctx(const KArgs& a, long long unit, int f)
    {
        using ListEntC = __attribute__((address_space(4))) const ListEnt;
        const long long b = unit * C + f;
        Ctx c;
        c.act = b < a.batch;
        ListEntC* e = (ListEntC*)a.list + (c.act ? b : 0);
        c.src = e->in;
        c.dst = e->out;
        return c;
    }
};

// Range compression: the block layout, a forward transform, the product with
// the conjugate replica spectrum and the backward transform, all in one
// workgroup (the conjugations are explicit, not direction dependent).
struct PolFilt : PolBlock {
    static constexpr bool conj_in = false;
    static constexpr bool conj_out = false;
    static constexpr int kind = kKindFilter;
};

// TW: element type of the four-step workspace (complex64, or FP16 pairs for
// the compact FP16 form).
template <typename TI, typename TW = float2>
struct PolPass1T {
    static constexpr bool f_fast = true;
    static constexpr bool conj_in = true;
    static constexpr bool conj_out = false;
    static constexpr int kind = kKindPass1;
    struct Ctx {
        const TI* src;
        TW* dst;
        unsigned col;
        bool act;
    };
    template <int N, int C>
    __device__ static Ctx ctx(const KArgs& a, long long unit, int f)
    {
        const long long bt = unit / a.tiles;
        const int tile = (int)(unit - bt * a.tiles);
        Ctx c;
        c.col = (unsigned)(tile * C + f);
        c.act = true;
        c.src = reinterpret_cast<const TI*>(a.in) + bt * a.nbig + c.col;
        c.dst = reinterpret_cast<TW*>(a.out) + bt * a.nbig + ((long long)c.col << a.cw_bits);
        return c;
    }
    template <int C>
    __device__ static const TI* in_at(const KArgs& a, const Ctx& c, int n)
    {
        return c.src + (long long)n * a.n_other;
    }
    // the same for n = t + nc with nc the same in every lane: one per-thread
    // base, then a stride the scalar unit forms (no 64-bit multiply per load)
    template <int C>
    __device__ static const TI* in_at_split(const KArgs& a, const Ctx& c, int t, int nc)
    {
        return c.src + (long long)t * a.n_other + (long long)nc * a.n_other;
    }
    // x * exp(-2 pi i col k / N)
    __device__ static float2 twiddled(const KArgs& a, const Ctx& c, int k, float2 x)
    {
        const unsigned m = (c.col * (unsigned)k) & (unsigned)(a.nbig - 1);
        const float2 w = cmul(a.tw_hi[m >> a.lo_bits], a.tw_lo[m & ((1u << a.lo_bits) - 1u)]);
        return cmul(x, w);
    }
    // Multiplies every output of the thread by its long twiddle.  Output
    // (i, q) of the last stage is k = t + T*m with m = i + q*(E/RL), so
    // exp(-2 pi i col k / N) = exp(-2 pi i col t / N) * s^m with
    // s = exp(-2 pi i col T / N); the power variant reads s^(2^i) from the
    // per-column table and forms s^m by products, the plain one gathers every
    // twiddle from the hi/lo tables.
    template <int N, int E, int T, int RL, int NsL, int FL>
    __device__ static void twiddle_outputs(const KArgs& a, const Ctx& c, int t, float2 (&v)[E])
    {
        if constexpr ((FL & kTwPow) != 0) {
            constexpr int LP = E == 2 ? 1 : E == 4 ? 2 : E == 8 ? 3 : E == 16 ? 4 : 5;  // log2 E
            constexpr int ROW = (LP + 1) & ~1;
            const unsigned m0 = (c.col * (unsigned)t) & (unsigned)(a.nbig - 1);
            const float2 b = cmul(a.tw_hi[m0 >> a.lo_bits], a.tw_lo[m0 & ((1u << a.lo_bits) - 1u)]);
            float2 p[ROW];  // s^(2^j), j < log2 E
            const float4* row4 = reinterpret_cast<const float4*>(a.tw_col + (long long)c.col * ROW);
#pragma unroll
            for (int j = 0; j < ROW; j += 2) {
                const float4 w = row4[j / 2];
                p[j] = make_float2(w.x, w.y);
                p[j + 1] = make_float2(w.z, w.w);
            }
            // m = r + L h: s^m = s^(L h) s^r, with G[h] = b s^(L h) formed
            // first and the low powers s^r one at a time, so only H + log2 L
            // factors stay live next to the values (not all E powers)
            constexpr int L = E < 8 ? E : 8;
            constexpr int LL = L == 2 ? 1 : L == 4 ? 2 : 3;
            constexpr int H = E / L;
            float2 G[H];
            G[0] = b;
            sfor<1, H>([&](auto hc) {
                constexpr int h = decltype(hc)::value;
                constexpr int hb = h >= 2 ? 1 : 0;  // highest set bit of h (h < 4)
                if constexpr (h == (1 << hb))
                    G[h] = cmul(b, p[LL + hb]);
                else
                    G[h] = cmul(G[h - (1 << hb)], p[LL + hb]);
            });
            float2 low[L];
            low[0] = make_float2(1.f, 0.f);
            sfor<0, L>([&](auto rc) {
                constexpr int r = decltype(rc)::value;
                if constexpr (r > 0) {
                    constexpr int rb = r >= 4 ? 2 : r >= 2 ? 1 : 0;
                    if constexpr (r == (1 << rb))
                        low[r] = p[rb];
                    else
                        low[r] = cmul(p[rb], low[r - (1 << rb)]);
                }
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    constexpr int D = E / RL;
                    const int m = r + L * h;
                    float2& x = v[(m % D) * RL + m / D];
                    x = cmul(x, r == 0 ? G[h] : cmul(G[h], low[r]));
                }
            });
        } else {
#pragma unroll
            for (int i = 0; i < E / RL; ++i)
#pragma unroll
                for (int q = 0; q < RL; ++q) v[i * RL + q] = twiddled(a, c, t + i * T + q * NsL, v[i * RL + q]);
        }
    }
    template <int FL>
    __device__ static void store(const KArgs& a, const Ctx& c, int k, float2 x)
    {
        const long long blk = (long long)(k >> a.cw_bits) * (a.n_other << a.cw_bits);
        gstore<FL>(c.dst + blk + (k & ((1 << a.cw_bits) - 1)), x);
    }
    // Contiguous store of the workgroup's outputs from LDS (natural order per
    // column): for each block g of CW rows the C columns x CW values are one
    // contiguous run of the workspace.  The LDS holds outputs k0 .. k0 + N - 1
    // of every column (k0 a multiple of CW).
    template <int N, int C, int FL, int LDSN, int NT>
    __device__ static void staged_store(const KArgs& a, long long unit, const float2* lds, int tid, int k0)
    {
        const long long bt = unit / a.tiles;
        const int tile = (int)(unit - bt * a.tiles);
        const long long gstride = a.n_other << a.cw_bits;
        TW* base = reinterpret_cast<TW*>(a.out) + bt * a.nbig + ((long long)(tile * C) << a.cw_bits) +
                   (k0 >> a.cw_bits) * gstride;
        const int cwm = (1 << a.cw_bits) - 1;
        const int blk_bits = a.cw_bits + __builtin_ctz(C);
        const unsigned gs24 = (unsigned)gstride;
#pragma unroll
        for (int m = 0; m < N * C / NT; ++m) {
            const int e = tid + m * NT;
            const int g = e >> blk_bits;
            const int w = e & ((1 << blk_bits) - 1);
            const int ff = w >> a.cw_bits;
            const int k = (g << a.cw_bits) + (w & cwm);
            // the offset within one transform is below N <= 2^22, so a
            // 24-bit multiply in 32 bits forms it (no 64-bit multiply)
            gstore<FL>(base + (long long)(int)(__umul24(g, gs24) + w), lds[ff * LDSN + lds_at<FL>(k)]);
        }
    }
    __host__ __device__ static long long units(const KArgs& a, int) { return a.batch * a.tiles; }
};
using PolPass1 = PolPass1T<float2>;
using PolPass1H = PolPass1T<h2_t>;
using PolPass1HW = PolPass1T<h2_t, h2_t>;

template <typename TO, typename TW = float2>
struct PolPass2T {
    static constexpr bool f_fast = true;
    static constexpr bool conj_in = false;
    static constexpr bool conj_out = true;
    static constexpr int kind = kKindPass2;
    struct Ctx {
        const TW* src;
        TO* dst;
        bool act;
    };
    template <int N, int C>
    __device__ static Ctx ctx(const KArgs& a, long long unit, int f)
    {
        const long long bt = unit / a.tiles;
        const int g = (int)(unit - bt * a.tiles);
        Ctx c;
        c.act = true;
        c.src = reinterpret_cast<const TW*>(a.in) + bt * a.nbig + (long long)g * N * C + f;
        c.dst = reinterpret_cast<TO*>(a.out) + bt * a.nbig + (long long)g * C + f;
        return c;
    }
    template <int C>
    __device__ static const TW* in_at(const KArgs&, const Ctx& c, int n)
    {
        return c.src + (long long)n * C;
    }
    template <int N, int E, int T, int RL, int NsL, int FL>
    __device__ static void twiddle_outputs(const KArgs&, const Ctx&, int, float2 (&)[E])
    {
    }
    template <int FL>
    __device__ static void store(const KArgs& a, const Ctx& c, int k, float2 x)
    {
        gstore<FL>(c.dst + (long long)k * a.n_other, x);
    }
    // the same for k = t + kc with kc the same in every lane (see in_at_split)
    template <int FL>
    __device__ static void store_split(const KArgs& a, const Ctx& c, int t, int kc, float2 x)
    {
        gstore<FL>(c.dst + (long long)t * a.n_other + (long long)kc * a.n_other, x);
    }
    __host__ __device__ static long long units(const KArgs& a, int) { return a.batch * a.tiles; }
};
using PolPass2 = PolPass2T<float2>;
using PolPass2H = PolPass2T<h2_t>;
using PolPass2HW = PolPass2T<h2_t, h2_t>;

// Address of element t + c (t per lane, c the same in every lane) through the
// policy's split form where it has one, else its plain one.
template <class P, int C, class Ctx>
__device__ __forceinline__ auto in_at_split(const KArgs& a, const Ctx& cx, int t, int c)
{
    if constexpr (requires { P::template in_at_split<C>(a, cx, t, c); })
        return P::template in_at_split<C>(a, cx, t, c);
    else
        return P::template in_at<C>(a, cx, t + c);
}
template <class P, int FL, class Ctx>
__device__ __forceinline__ void store_split(const KArgs& a, const Ctx& cx, int t, int c, float2 x)
{
    if constexpr (requires { P::template store_split<FL>(a, cx, t, c, x); })
        P::template store_split<FL>(a, cx, t, c, x);
    else
        P::template store<FL>(a, cx, t + c, x);
}

// --------------------------------------------------------------- the stages
// v holds the stage-0 inputs x[t + i*T + r*N/R0] on entry and the outputs
// X[t + i*T + q*Ns_last] on exit.
// Twiddle rows from the factorised table in LDS (persistent kernels).
template <class S, int s, int R>
__device__ __forceinline__ void apply_lds_tw(float2* v, const float2* Ltw, int k)
{
    static_assert(R % 2 == 0, "persistent variants need even radices");
    const float4* A;
    if constexpr (S::f_full(s)) {
        A = reinterpret_cast<const float4*>(Ltw + S::ftw_off(s) + k * R);
#pragma unroll
        for (int r = 0; r < R; r += 2) {
            const float4 w = A[r / 2];
            if (r > 0) v[r] = cmul(v[r], make_float2(w.x, w.y));
            v[r + 1] = cmul(v[r + 1], make_float2(w.z, w.w));
        }
    } else {
        constexpr int M = S::fm(s);
        constexpr int Q = S::fq(s);
        const int q = k / M, p = k % M;
        A = reinterpret_cast<const float4*>(Ltw + S::ftw_off(s) + q * R);
        const float4* B = reinterpret_cast<const float4*>(Ltw + S::ftw_off(s) + Q * R + p * R);
#pragma unroll
        for (int r = 0; r < R; r += 2) {
            const float4 wa = A[r / 2], wb = B[r / 2];
            if (r > 0) v[r] = cmul(v[r], cmul(make_float2(wa.x, wa.y), make_float2(wb.x, wb.y)));
            v[r + 1] = cmul(v[r + 1], cmul(make_float2(wa.z, wa.w), make_float2(wb.z, wb.w)));
        }
    }
}

// on: this thread takes part (false for the idle threads of a persistent
// kernel whose workgroup is wider than the case it runs: they keep to every
// barrier but write nothing).
template <int N, int E, class S, int FL, bool WS = false>
__device__ __forceinline__ void run_stages(float2 (&v)[E], float2* L, const float2* __restrict__ tw,
                                           const float2* Ltw, int t, bool on = true)
{
    constexpr int T = N / E;
    constexpr int NST = S::count;

    sfor<0, NST>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int R = S::r(s);
        constexpr int Ns = S::ns(s);
        if constexpr (s > 0) {
            if constexpr ((FL & kHalfX) == 0) {
#pragma unroll
                for (int i = 0; i < E / R; ++i)
#pragma unroll
                    for (int r = 0; r < R; ++r) v[i * R + r] = L[lds_at<FL>(t + i * T + r * (N / R))];
            }  // half exchanges read this stage's inputs during the exchange itself
#pragma unroll
            for (int i = 0; i < E / R; ++i) {
                const int k = (t + i * T) % Ns;
                if constexpr ((FL & kPipe) != 0)
                    apply_lds_tw<S, s, R>(&v[i * R], Ltw, k);
                else if constexpr ((FL & kTwPow) != 0)
                    apply_pow_row<R>(&v[i * R], tw + S::ptw_off(s) + k * S::p_row(s));
                else
                    apply_row<R>(&v[i * R], tw + S::tw_off(s) + k * R);
            }
        }
#pragma unroll
        for (int i = 0; i < E / R; ++i) Dft<R>::run(&v[i * R]);
        if constexpr (s < NST - 1 && (FL & kHalfX) == 0) {
            if constexpr (s > 0) exch_sync<WS>();
            if (on) {
#pragma unroll
                for (int i = 0; i < E / R; ++i) {
                    const int j = t + i * T;
                    const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
                    for (int q = 0; q < R; ++q) L[lds_at<FL>(base + q * Ns)] = v[i * R + q];
                }
            }
            exch_sync<WS>();
        } else if constexpr (s < NST - 1) {
            // Half exchange through N/2 slots.  Butterfly i of this stage
            // (j = t + i T) writes slots Ns (R (j / Ns) + q) + j mod Ns, which
            // lie in the upper half exactly when j >= N / 2R, i.e. i >= E / 2R;
            // the next stage's input r of its butterfly i2 sits at slot
            // t + i2 T + r N / R2, in the upper half exactly when r >= R2 / 2.
            // Round h writes butterflies [h E/2R, (h+1) E/2R) and reads the
            // inputs r in [h R2/2, (h+1) R2/2) of every butterfly.
            constexpr int R2 = S::r(s + 1);
            static_assert(E % (2 * R) == 0 && R2 % 2 == 0 && (FL & kPipe) == 0,
                          "half exchanges need an even number of butterflies per thread");
            float2 w[E];
            sfor<0, 2>([&](auto hc) {
                constexpr int h = decltype(hc)::value;
                if constexpr (h > 0 || s > 0) exch_sync<WS>();  // earlier reads precede these writes
                if (on) {
#pragma unroll
                    for (int i = h * (E / (2 * R)); i < (h + 1) * (E / (2 * R)); ++i) {
                        const int j = t + i * T;
                        const int base = (j / Ns) * Ns * R + (j % Ns) - h * (N / 2);
#pragma unroll
                        for (int q = 0; q < R; ++q) L[lds_at<FL>(base + q * Ns)] = v[i * R + q];
                    }
                }
                exch_sync<WS>();
#pragma unroll
                for (int i2 = 0; i2 < E / R2; ++i2)
#pragma unroll
                    for (int r = h * (R2 / 2); r < (h + 1) * (R2 / 2); ++r)
                        w[i2 * R2 + r] = L[lds_at<FL>(t + i2 * T + r * (N / R2) - h * (N / 2))];
            });
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = w[e];
        }
    });
}

// LDS layout of a kernel: C exchange buffers of lds_stride values, then (for
// persistent variants) the factorised twiddle table, 16-byte aligned.
template <int N, int C, class S, int FL, bool FFAST, int T>
__host__ __device__ constexpr int k_tw_base()
{
    return (S::count > 1 ? ((C * lds_stride<lds_points<N, FL>(), FL, FFAST, C, T>() + 1) & ~1) : 0);
}
template <int N, int C, class S, int FL, bool FFAST, int T>
__host__ __device__ constexpr int k_lds_elems()
{
    const int tw = (FL & kPipe) != 0 ? S::ftw_size() : 0;
    const int n = k_tw_base<N, C, S, FL, FFAST, T>() + tw;
    return n > 0 ? n : 1;
}

// Waves per SIMD the LDS footprint allows (160 KB per CU, 4 SIMDs); the
// persistent variants ask the register allocator for that occupancy.
template <int N, int E, int C, class S, int FL, bool FFAST>
__host__ __device__ constexpr int k_min_waves()
{
    if ((FL & kHalfX) != 0) {
        // ask the register allocator for the residency the halved LDS allows
        const int lds = k_lds_elems<N, C, S, FL, FFAST, N / E>() * 8;
        const int wgs = 163840 / lds;
        const int waves = wgs * (((N / E) * C + 63) / 64) / 4;
        const int cap = (FL & kFitRegs) != 0 ? 8 : 3;
        return waves < 1 ? 1 : waves > cap ? cap : waves;
    }
    if ((FL & kPipe) == 0) return 1;
    const int lds = k_lds_elems<N, C, S, FL, FFAST, N / E>() * 8;
    const int wgs = 163840 / lds;
    const int waves = wgs * (((N / E) * C + 63) / 64) / 4;
    return waves < 1 ? 1 : waves > 8 ? 8 : waves;
}

// One work unit of a transform kernel (C transforms, or C columns / rows of
// a four-step pass), shared by the one-unit-per-workgroup kernel k_fft, its
// looping variants and the persistent ragged kernels.  `lds` holds the C
// exchange buffers (and, for kPipe, the factorised twiddles at TWB); `on` is
// false for the idle threads of a workgroup wider than T * C: they keep to
// every barrier of the unit but read and write no global memory and write no
// LDS.
template <int N, int E, int C, class S, class P, int FL>
struct FftBody {
    static constexpr int T = N / E;
    static constexpr int threads = T * C;
    static constexpr int NST = S::count;
    static constexpr int LDSN = lds_stride<lds_points<N, FL>(), FL, P::f_fast, C, T>();
    static constexpr int R0 = S::r(0);
    static constexpr int RL = S::r(NST - 1);
    static constexpr int NsL = S::ns(NST - 1);
    static constexpr int TWB = k_tw_base<N, C, S, FL, P::f_fast, T>();
    static constexpr int lds_elems = k_lds_elems<N, C, S, FL, P::f_fast, T>();
    // wave-synchronous exchanges: t-fast lanes, whole transforms per wavefront
    static constexpr bool WS = (FL & kWaveSync) != 0 && !P::f_fast && T <= 64 && 64 % T == 0 && (FL & kPipe) == 0;
    static_assert(S::n() == N, "schedule does not multiply to N");

    // the thread's transform (or column / row) f and position t in it
    __device__ static __forceinline__ void place(int tid, int& f, int& t)
    {
        f = P::f_fast ? tid % C : tid / T;
        t = P::f_fast ? tid / C : tid % T;
    }

    // Sixteen-byte lanes (kVec16).  Stage-0 input e = i R0 + r of thread t is
    // x[t + off_in(e)], last-stage output e = i RL + q goes to X[t + off_out(e)],
    // so threads t and t + 1 (t even: lanes 2m and 2m + 1 of one transform)
    // want neighbouring elements for every e.  The pair moves them two at a
    // time: the even lane the pair's values e < E/2, the odd lane those
    // e >= E/2, which lie a constant D further on (half the stage's
    // butterflies, or half of each butterfly's inputs when a thread runs one
    // butterfly); then each value crosses to the lane that owns it by one DPP
    // lane permutation (a VALU operand, no LDS).  The thread-to-butterfly map,
    // and so every LDS exchange, is unchanged.
    static constexpr int off_in(int e) { return (e / R0) * T + (e % R0) * (N / R0); }
    static constexpr int off_out(int e) { return (e / RL) * T + (e % RL) * NsL; }
    static constexpr bool kPairs = (FL & kVec16) != 0;
    static_assert(!kPairs || ((P::kind == kKindBlock) && !P::f_fast && T % 2 == 0 &&
                              (E / R0 == 1 || (E / R0) % 2 == 0) && (E / RL == 1 || (E / RL) % 2 == 0)),
                  "16-byte lanes: block layout, an even number of threads per transform, and one or an even "
                  "number of butterflies per thread in the first and last stage");

    template <class Ctx>
    __device__ static __forceinline__ void load_pairs(const Ctx& cx, int t, float2 (&v)[E])
    {
        constexpr int D = off_in(E / 2);
        const bool odd = (t & 1) != 0;
        const float2* p = cx.src + ((t & ~1) + (odd ? D : 0));
        float2 lo[E / 2], hi[E / 2];
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const float4 q = gload2<FL>(p + off_in(e));
            lo[e] = make_float2(q.x, q.y);
            hi[e] = make_float2(q.z, q.w);
        }
        // even lane: lo = its own value e, hi = the odd lane's; odd lane:
        // lo = the even lane's value e + E/2, hi = its own
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const float2 xl = lane_xor1(lo[e]), xh = lane_xor1(hi[e]);
            v[e] = odd ? xh : lo[e];
            v[e + E / 2] = odd ? hi[e] : xl;
        }
    }

    template <class Ctx>
    __device__ static __forceinline__ void store_pairs(const Ctx& cx, int t, const float2 (&v)[E])
    {
        constexpr int D = off_out(E / 2);
        const bool odd = (t & 1) != 0;
        float2* p = cx.dst + ((t & ~1) + (odd ? D : 0));
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const float2 xl = lane_xor1(v[e]), xh = lane_xor1(v[e + E / 2]);
            gstore2<FL>(p + off_out(e), odd ? xh : v[e], odd ? v[e + E / 2] : xl);
        }
    }

    // The backward transform is conj(forward(conj(x))): the conjugations are
    // skipped by a uniform branch in the forward direction.
    __device__ static __forceinline__ void load(const KArgs& a, long long unit, int f, int t, bool on,
                                                float2 (&v)[E])
    {
        const bool bwd = a.sg < 0.f;
        const auto cx = P::template ctx<N, C>(a, unit, f);
        if (cx.act && on) {
            if constexpr ((FL & kVec16) != 0) {
                load_pairs(cx, t, v);
            } else {
#pragma unroll
                for (int i = 0; i < E / R0; ++i)
#pragma unroll
                    for (int r = 0; r < R0; ++r)
                        v[i * R0 + r] = gload<FL>(in_at_split<P, C>(a, cx, t, i * T + r * (N / R0)));
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = make_float2(0.f, 0.f);
        }
        if constexpr (P::conj_in) {
            if (bwd) {
#pragma unroll
                for (int e = 0; e < E; ++e) v[e].y = -v[e].y;
            }
        }
    }

    __device__ static __forceinline__ void finish(const KArgs& a, long long unit, float2* lds, int tid, int f,
                                                  int t, bool on, float2 (&v)[E])
    {
        const bool bwd = a.sg < 0.f;
        float2* L = lds + (NST > 1 ? f * LDSN : 0);
        const float2* Ltw = lds + TWB;
        run_stages<N, E, S, FL, WS>(v, L, a.tw, Ltw, t, on);
        static_assert(P::kind != kKindFilter || (FL & kHalfX) == 0 || R0 == RL,
                      "the filter's round trip between the transforms needs N slots");
        if constexpr (P::kind == kKindFilter) {
            // Z = X conj(H) is transformed back as conj(F(conj Z)), and
            // conj Z = conj(X) H: X[k] sits at v[i RL + q], k = t + i T + q NsL.
            int tp = t;  // (offsets of the product formed afresh as well)
            asm volatile("" : "+v"(tp));
            __builtin_assume(tp >= 0 && tp < T);
            const float2* flt = a.flt + tp;
#pragma unroll
            for (int i = 0; i < E / RL; ++i)
#pragma unroll
                for (int q = 0; q < RL; ++q) {
                    const float2 h = flt[i * T + q * NsL];
                    const float2 x = v[i * RL + q];
                    v[i * RL + q] = cmul(make_float2(x.x, -x.y), h);
                }
            if constexpr (NST > 1) {
                exch_sync<WS>();  // every read of the last stage precedes the next writes
                if constexpr (R0 != RL) {
                    // natural order through LDS, then the stage-0 gather
                    if (on) {
#pragma unroll
                        for (int i = 0; i < E / RL; ++i)
#pragma unroll
                            for (int q = 0; q < RL; ++q) L[lds_at<FL>(t + i * T + q * NsL)] = v[i * RL + q];
                    }
                    exch_sync<WS>();
#pragma unroll
                    for (int i = 0; i < E / R0; ++i)
#pragma unroll
                        for (int r = 0; r < R0; ++r) v[i * R0 + r] = L[lds_at<FL>(t + i * T + r * (N / R0))];
                    exch_sync<WS>();
                }
                // with R0 == RL the outputs already sit where stage 0 wants its inputs
            }
            // the second transform's thread index behind an empty asm, so its
            // LDS and twiddle offsets are formed afresh rather than kept live
            // from the first transform's
            int t2 = t;
            asm volatile("" : "+v"(t2));
            __builtin_assume(t2 >= 0 && t2 < T);
            run_stages<N, E, S, FL, WS>(v, L, a.tw, Ltw, t2, on);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e].y = -v[e].y;
        }
        const auto cx = P::template ctx<N, C>(a, unit, f);
        P::template twiddle_outputs<N, E, T, RL, NsL, FL>(a, cx, t, v);
        if constexpr (P::kind == kKindPass1 && (FL & kF16Work) != 0) {
            // an FP16 workspace takes the output scale before pass 2 (whose
            // inputs would otherwise overflow binary16 in a long inverse)
            if (a.scale != 1.f) {
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = make_float2(v[e].x * a.scale, v[e].y * a.scale);
            }
        }
        if constexpr ((FL & kStaged) != 0 && (FL & kHalfX) != 0) {
            // the same in two rounds of N/2 outputs: output (i, q) of the last
            // stage is k = t + i T + q NsL, in the upper half exactly when
            // q >= RL / 2; round h stores those at k - h N/2
            static_assert(P::kind == kKindPass1 && RL % 2 == 0, "staged store is a pass-1 variant");
            sfor<0, 2>([&](auto hc) {
                constexpr int h = decltype(hc)::value;
                __syncthreads();
                if (on) {
#pragma unroll
                    for (int i = 0; i < E / RL; ++i)
#pragma unroll
                        for (int q = h * (RL / 2); q < (h + 1) * (RL / 2); ++q)
                            L[lds_at<FL>(t + i * T + q * NsL - h * (N / 2))] = v[i * RL + q];
                }
                __syncthreads();
                if (on) P::template staged_store<N / 2, C, FL, LDSN, T * C>(a, unit, lds, tid, h * (N / 2));
            });
        } else if constexpr ((FL & kStaged) != 0) {
            // outputs (twiddled) to LDS in natural order, then contiguous stores
            static_assert(P::kind == kKindPass1, "staged store is a pass-1 variant");
            __syncthreads();
            if (on) {
#pragma unroll
                for (int i = 0; i < E / RL; ++i)
#pragma unroll
                    for (int q = 0; q < RL; ++q) {
                        const int k = t + i * T + q * NsL;
                        L[lds_at<FL>(k)] = v[i * RL + q];
                    }
            }
            __syncthreads();
            if (on) P::template staged_store<N, C, FL, LDSN, T * C>(a, unit, lds, tid, 0);
        } else {
            if constexpr (P::conj_out) {
                if (bwd) {
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e].y = -v[e].y;
                }
            }
            if constexpr (P::kind != kKindPass1) {
                if (a.scale != 1.f) {  // uniform: unscaled launches skip it
#pragma unroll
                    for (int e = 0; e < E; ++e) v[e] = make_float2(v[e].x * a.scale, v[e].y * a.scale);
                }
            }
            if (cx.act && on) {
                // a copy of t the compiler cannot see through: otherwise it
                // shares the store offsets t + i T + q NsL with the LDS
                // indices of the stages and keeps them live all along
                int ts = t;
                asm volatile("" : "+v"(ts));
                if constexpr (kPairs) {
                    store_pairs(cx, ts, v);
                } else {
#pragma unroll
                    for (int i = 0; i < E / RL; ++i)
#pragma unroll
                        for (int q = 0; q < RL; ++q)
                            store_split<P, FL>(a, cx, ts, i * T + q * NsL, v[i * RL + q]);
                }
            }
        }
    }
};

template <int N, int E, int C, class S, class P, int FL>
__global__ void __launch_bounds__((N / E) * C)
__attribute__((amdgpu_waves_per_eu(k_min_waves<N, E, C, S, FL, P::f_fast>())))
k_fft(KArgs a)
{
    using B = FftBody<N, E, C, S, P, FL>;
    constexpr int T = B::T;
    __shared__ __attribute__((aligned(16))) float2 lds[B::lds_elems];

    const int tid = threadIdx.x;
    int f, t;
    B::place(tid, f, t);

    if constexpr ((FL & kLoop) != 0) {
        static_assert((FL & kPipe) == 0 && (FL & kXcd) == 0, "the loop form takes units in launch order");
        // One workgroup per resident slot walks units b, b + G, ...: the next
        // unit's loads issue as soon as this unit's stores are issued, with no
        // workgroup exit and dispatch in between.
        const long long units = P::units(a, C);
        for (long long u = blockIdx.x; u < units; u += gridDim.x) {
            // the thread's indices are re-derived in every iteration (the
            // empty asm hides that they repeat), so the many per-thread LDS
            // and global offsets are not hoisted out of the loop and kept
            // live across it, which would spill
            int tl = tid;
            asm volatile("" : "+v"(tl));
            B::place(tl, f, t);
            float2 v[E];
            B::load(a, u, f, t, true, v);
            B::finish(a, u, lds, tl, f, t, true, v);
            __syncthreads();  // the next unit's first LDS writes follow every thread's last LDS reads
        }
    } else if constexpr ((FL & kPipe) == 0) {
        float2 v[E];
        long long unit = blockIdx.x;
        if constexpr ((FL & kXcd) != 0) unit = xcd_unit(unit, gridDim.x);
        B::load(a, unit, f, t, true, v);
        B::finish(a, unit, lds, tid, f, t, true, v);
    } else {
        const long long units = P::units(a, C);
        long long u = blockIdx.x;
        if (u >= units) return;
        float2* Ltw = lds + B::TWB;
        constexpr int TWN = S::ftw_size();
        float2 twv[(TWN + T * C - 1) / (T * C) > 0 ? (TWN + T * C - 1) / (T * C) : 1];
#pragma unroll
        for (int m = 0; m * T * C < TWN; ++m) {
            const int i = tid + m * T * C;
            if (i < TWN) twv[m] = a.tw[i];
        }
        float2 nx[E];
        B::load(a, u, f, t, true, nx);
#pragma unroll
        for (int m = 0; m * T * C < TWN; ++m) {
            const int i = tid + m * T * C;
            if (i < TWN) Ltw[i] = twv[m];
        }
        for (;;) {
            float2 v[E];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = nx[e];
            const long long un = u + gridDim.x;
            if (un < units) B::load(a, un, f, t, true, nx);
            B::finish(a, u, lds, tid, f, t, true, v);
            if (un >= units) break;
            u = un;
            __syncthreads();  // the next unit's first LDS writes follow every thread's last LDS reads
        }
    }
}

template <int N, int E, int C, class S, class P, int FL>
hipError_t launch_fft(const KArgs& a, long long grid, hipStream_t st, hipEvent_t start, hipEvent_t stop)
{
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    if (start || stop)
        hipExtLaunchKernelGGL((k_fft<N, E, C, S, P, FL>), dim3((unsigned)grid), dim3((N / E) * C), 0, st, start,
                              stop, 0, a);
    else
        hipLaunchKernelGGL((k_fft<N, E, C, S, P, FL>), dim3((unsigned)grid), dim3((N / E) * C), 0, st, a);
    return hipGetLastError();
}

template <int N, int E, int C, class S, class P, int FL>
int occupancy_fft()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void*)&k_fft<N, E, C, S, P, FL>,
                                                     (N / E) * C, 0) != hipSuccess)
        return 0;
    return blocks;
}

template <int N, int E, int C, class S, class P, int FL>
constexpr KEntry make_entry(bool is_default, const char* name)
{
    KEntry k{};
    k.kind = P::kind;
    k.n = N;
    k.e = E;
    k.c = C;
    k.flags = FL;
    k.nr = S::count;
    for (int i = 0; i < S::count && i < 8; ++i) k.radix[i] = S::r(i);
    k.tw_size = (FL & kPipe) != 0 ? S::ftw_size() : (FL & kTwPow) != 0 ? S::ptw_size() : S::tw_size();
    k.threads = (N / E) * C;
    k.lds = (size_t)k_lds_elems<N, C, S, FL, P::f_fast, N / E>() * sizeof(float2);
    k.is_default = is_default;
    k.launch = &launch_fft<N, E, C, S, P, FL>;
    k.occupancy = &occupancy_fft<N, E, C, S, P, FL>;
    k.name = name;
    k.fn = reinterpret_cast<const void*>(&k_fft<N, E, C, S, P, FL>);
    return k;
}

}  // namespace fb
