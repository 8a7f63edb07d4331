// Persistent kernels for ragged batches: transforms of several lengths in one
// launch (paper, Approach, "Top level analysis": many independent FFT tasks,
// each reading all its inputs, computing, and writing all its outputs, mapped
// onto the compute units).
//
// A launch holds as many workgroups as are resident.  The work list is a
// sequence of units: unit u belongs to class c when u0[c] <= u < u0[c+1], and
// class c runs case cs[c] of the kernel (one compiled length, schedule,
// width and variant) with the class's own kernel arguments.  A head of the
// list is dealt round-robin to the workgroups; the rest is taken one unit at
// a time from an atomic counter, so the workgroups finish together.  The
// host orders the classes (largest units first, so the last units to finish
// are short).  A case narrower than the workgroup runs on its first T * C
// threads; the others keep to its barriers.
//
// The counter returns to zero when the last workgroup leaves, so the launch
// can be replayed (a captured graph) without a reset node.
#pragma once

#include "fft_kernel.hpp"

namespace fb {

// One length class of a persistent launch (device memory).  rel bit 0 / 1:
// a.in / a.out hold byte offsets from the launch's in / out base (the ragged
// batch the caller passes) rather than absolute addresses (a plan's own
// workspace).
struct RagEnt {
    KArgs a;
    long long u0;  // first unit of the class
    int cs;        // case index within the kernel
    int rel;
};

constexpr int kRagMaxEnt = 16;

// The class table rides in the kernel arguments (first unit and case of each
// class), so finding a unit's class touches no memory.
struct RagArgs {
    const RagEnt* ent;
    int nent;
    unsigned units;      // total units of the launch
    unsigned nstatic;    // units [0, nstatic) are dealt round-robin, the rest from the queue
    unsigned* ctr;       // [0]: next queued unit - nstatic, [1]: workgroups that have left (8-byte aligned)
    const char* in;      // base of the ragged input
    char* out;           // base of the ragged output
    unsigned u0[kRagMaxEnt];
};

// One case: a compiled transform configuration (as in the plain catalogue).
template <int N_, int E_, int C_, class S_, class P_, int FL_>
struct RCase {
    static constexpr int N = N_, E = E_, C = C_, FL = FL_;
    using S = S_;
    using P = P_;
    using Body = FftBody<N, E, C, S, P, FL>;
};

template <class... Cs>
__host__ __device__ constexpr int rag_lds_elems()
{
    int m = 1;
    ((m = Cs::Body::lds_elems > m ? Cs::Body::lds_elems : m), ...);
    return m;
}

template <class Cs0>
__device__ __forceinline__ void rag_run(const KArgs& a, long long unit, float2* lds, int tid)
{
    using B = typename Cs0::Body;
    const bool on = tid < B::threads;
    int f, t;
    B::place(on ? tid : 0, f, t);
    float2 v[Cs0::E];
    B::load(a, unit, f, t, on, v);
    B::finish(a, unit, lds, tid, f, t, on, v);
}

template <int I, class C0, class... Cs>
__device__ __forceinline__ void rag_dispatch(int cs, const KArgs& a, long long unit, float2* lds, int tid)
{
    if (cs == I) {
        rag_run<C0>(a, unit, lds, tid);
    } else if constexpr (sizeof...(Cs) > 0) {
        rag_dispatch<I + 1, Cs...>(cs, a, unit, lds, tid);
    }
}

// A pointer loaded from ordinary memory may point anywhere, so accesses
// through it would be flat instructions, which count against the LDS counter
// too: every LDS wait and barrier would then also wait for the HBM loads and
// stores in flight.  Pointers loaded from the constant address space (where
// kernel arguments live) are taken to address global memory, so the class
// entries -- read-only for the kernel's lifetime -- are read through it.
using RagEntC = __attribute__((address_space(4))) const RagEnt;

// The class's kernel arguments, field by field (no reference may bind to the
// constant address space).
__device__ __forceinline__ KArgs rag_args(RagEntC& e)
{
    KArgs a;
    a.in = e.a.in;
    a.out = e.a.out;
    a.tw = e.a.tw;
    a.batch = e.a.batch;
    a.nbig = e.a.nbig;
    a.n_other = e.a.n_other;
    a.tiles = e.a.tiles;
    a.cw_bits = e.a.cw_bits;
    a.lo_bits = e.a.lo_bits;
    a.tw_hi = e.a.tw_hi;
    a.tw_lo = e.a.tw_lo;
    a.tw_col = e.a.tw_col;
    a.flt = e.a.flt;
    a.list = e.a.list;
    a.sg = e.a.sg;
    a.sched = e.a.sched;
    return a;
}

// One unit u (uniform): its class (from the class table, copied to LDS at
// the start so it occupies no registers across the loop), then its case.
template <int NT, class... Cs>
__device__ __forceinline__ void rag_unit(const RagArgs& r, unsigned u, const unsigned* su0, float2* lds, int tid)
{
    int c = 0;
#pragma unroll
    for (int j = 1; j < kRagMaxEnt; ++j) c += su0[j] <= u ? 1 : 0;
    c = __builtin_amdgcn_readfirstlane(c);
    RagEntC& e = ((RagEntC*)r.ent)[c];
    KArgs a = rag_args(e);
    const int rel = e.rel;
    if (rel & 1) a.in = reinterpret_cast<const float2*>(r.in + reinterpret_cast<size_t>(a.in));
    if (rel & 2) a.out = reinterpret_cast<float2*>(r.out + reinterpret_cast<size_t>(a.out));
    // the thread index re-derived in every unit behind an empty asm:
    // otherwise the per-thread offsets of every case are hoisted out of the
    // workgroup's loop and kept live across it (they spill)
    int tl = tid;
    asm volatile("" : "+v"(tl));
    __builtin_assume(tl >= 0 && tl < NT);  // what the asm hides: the range of a thread index
    rag_dispatch<0, Cs...>(e.cs, a, (long long)u - (long long)e.u0, lds, tl);
}

// Workgroup w first takes units w, w + G, ... below nstatic (no atomics: the
// host orders the list so these are a balanced share), then units from the
// queue, one at a time; thread 0 asks the queue for the next unit as soon as
// it starts the current one, so the atomic's latency overlaps the unit's
// loads.  One loop, so every case is instantiated once.
template <int NT, int MINW, class... Cs>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MINW))) k_ragged(RagArgs r)
{
    static_assert(((Cs::Body::threads <= NT) && ...), "a case is wider than the workgroup");
    __shared__ __attribute__((aligned(16))) float2 lds[rag_lds_elems<Cs...>()];
    __shared__ unsigned s_unit;
    __shared__ unsigned su0[kRagMaxEnt];
    const int tid = threadIdx.x;
    const unsigned G = gridDim.x;
    // the class table; entries past nent hold `units` (no unit reaches them)
    if (tid < kRagMaxEnt) su0[tid] = r.u0[tid];
    __syncthreads();
    unsigned u = blockIdx.x;
    if (u >= r.nstatic) {
        if (tid == 0) s_unit = r.nstatic + atomicAdd(&r.ctr[0], 1u);
        __syncthreads();
        u = __builtin_amdgcn_readfirstlane(s_unit);
    }
    while (u < r.units) {
        // the next unit: dealt (uniform), or asked of the queue now
        const bool dealt = u + G < r.nstatic;
        // The raw result only, and only in thread 0: arithmetic on it here, or
        // giving the register a value in the other threads, would make the
        // wave wait for the atomic -- and, since stores count in the same
        // counter, for the previous unit's stores -- before the unit's loads.
        const bool ask = !dealt && tid == 0;
        unsigned nxt;
        // (a wrapping increment, which the compiler's atomic optimizer does
        // not turn into a wave-aggregated add whose result is used at once)
        if (ask) nxt = atomicInc(&r.ctr[0], 0xffffffffu);
        rag_unit<NT, Cs...>(r, u, su0, lds, tid);
        // every thread has finished the unit's LDS reads (and read s_unit)
        __syncthreads();
        if (dealt) {
            u += G;
        } else {
            if (ask) s_unit = r.nstatic + nxt;
            __syncthreads();
            u = __builtin_amdgcn_readfirstlane(s_unit);
        }
    }
    if (tid == 0) {
        // The last workgroup to leave returns both counters to zero.  No
        // fence is needed (an agent-scope fence would write back and
        // invalidate the L2 at every workgroup's exit): a workgroup's last
        // queue atomic has returned its value, so it has been performed,
        // before the workgroup counts itself out, and the reset is an atomic
        // (it completes before the launch ends).
        if (atomicAdd(&r.ctr[1], 1u) == G - 1)
            __hip_atomic_store(reinterpret_cast<unsigned long long*>(r.ctr), 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);  // both counters, not waited for
    }
}

// Catalogue entry of a persistent kernel: its cases (matched against plain
// catalogue entries, whose plans supply the twiddle tables), launcher and
// occupancy.
struct RKCase {
    int kind, n, e, c, flags, nr;
    int radix[8];
};
using RKLaunch = hipError_t (*)(const RagArgs& r, unsigned grid, hipStream_t st);
struct RKEntry {
    const char* name;
    int threads;
    size_t lds;
    int ncase;
    RKCase cases[16];
    RKLaunch launch;
    KOccupancy occupancy;
    const void* fn;  // the kernel itself (graph kernel nodes)
};

const RKEntry* ragged_entries(int* count);

template <int NT, int MINW, class... Cs>
hipError_t launch_ragged(const RagArgs& r, unsigned grid, hipStream_t st)
{
    if (grid == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_ragged<NT, MINW, Cs...>), dim3(grid), dim3(NT), 0, st, r);
    return hipGetLastError();
}

template <int NT, int MINW, class... Cs>
int occupancy_ragged()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void*)&k_ragged<NT, MINW, Cs...>, NT, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

template <class Cs0>
constexpr RKCase rk_case()
{
    RKCase k{};
    k.kind = Cs0::P::kind;
    k.n = Cs0::N;
    k.e = Cs0::E;
    k.c = Cs0::C;
    k.flags = Cs0::FL;
    k.nr = Cs0::S::count;
    for (int i = 0; i < Cs0::S::count && i < 8; ++i) k.radix[i] = Cs0::S::r(i);
    return k;
}

template <int NT, int MINW, class... Cs>
constexpr RKEntry make_rk_entry(const char* name)
{
    static_assert(sizeof...(Cs) <= 16, "too many cases");
    RKEntry k{};
    k.name = name;
    k.threads = NT;
    k.lds = (size_t)rag_lds_elems<Cs...>() * sizeof(float2);
    k.ncase = (int)sizeof...(Cs);
    int i = 0;
    ((k.cases[i++] = rk_case<Cs>()), ...);
    k.launch = &launch_ragged<NT, MINW, Cs...>;
    k.occupancy = &occupancy_ragged<NT, MINW, Cs...>;
    k.fn = reinterpret_cast<const void*>(&k_ragged<NT, MINW, Cs...>);
    return k;
}

}  // namespace fb
