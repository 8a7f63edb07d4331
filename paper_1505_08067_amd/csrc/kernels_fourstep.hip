// Four-step passes for transforms longer than one LDS-resident block.
//
// Paper, Approach ("Other FFT sizes"): a transform larger than the block is
// built from block-sized transforms by splitting its stages, at the price of
// more data exchange.  With N = N1 * N2, input index n = N2*n1 + n2 and
// output index k = k1 + N1*k2:
//
//   pass 1: for every column n2, the N1-point transform over n1 of
//           x[N2*n1 + n2], each result multiplied by exp(-2 pi i n2 k1 / N),
//           stored to a workspace W[k1][n2] (row-major, row length N2);
//   pass 2: for every row k1, the N2-point transform over n2 of W[k1][n2],
//           stored to X[k1 + N1*k2] (the corner turn fused into the store).
//
// One workgroup handles C adjacent columns (pass 1) or C adjacent rows
// (pass 2), so every global access moves runs of C contiguous complex values
// (C*8 bytes) on the strided side and long contiguous runs on the other.
// Loads and stores go through LDS, which decouples the global access order
// from the butterfly order: load phase -> radix stages (register butterflies,
// LDS exchanges) -> store phase.  The long twiddle exp(-2 pi i m / N),
// m = n2*k1 mod N, is the product of two small FP32 tables (FP64-generated):
// hi[m >> b] * lo[m & (2^b - 1)].
#include "fft_device.hpp"
#include "internal.hpp"

namespace fb {

template <int PASS, int N, int E, int C, class S>
__global__ void __launch_bounds__((N / E) * C)
k_fourstep(const float2* __restrict__ in, float2* __restrict__ out, const float2* __restrict__ tw, FourStepArgs a)
{
    constexpr int T = N / E;
    constexpr int NT = T * C;
    constexpr int NST = S::count;
    constexpr int LDSN = lds_pad(N) + 1;
    static_assert(S::n() == N, "schedule does not multiply to N");
    __shared__ float2 lds[C * LDSN];

    const int tid = threadIdx.x;
    const long long bt = blockIdx.x / a.tiles;
    const int tile = blockIdx.x - (int)(bt * a.tiles);
    const int c0 = tile * C;
    const float2* __restrict__ src = in + bt * a.nbig;
    float2* __restrict__ dst = out + bt * a.nbig;

    // ---- load phase
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = tid + m * NT;
        if constexpr (PASS == 1) {
            const int n = e / C, ff = e % C;  // column c0+ff, row n
            float2 x = src[(long long)n * a.n_other + c0 + ff];
            x.y *= a.sg;
            lds[ff * LDSN + lds_pad(n)] = x;
        } else {
            const int ff = e / N, n = e % N;  // row c0+ff, column n
            lds[ff * LDSN + lds_pad(n)] = src[(long long)(c0 + ff) * N + n];
        }
    }
    __syncthreads();

    // ---- radix stages, LDS to LDS
    const int f = tid / T;
    const int t = tid - f * T;
    float2* L = lds + f * LDSN;
    float2 v[E];
    sfor<0, NST>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int R = S::r(s);
        constexpr int Ns = S::ns(s);
#pragma unroll
        for (int i = 0; i < E / R; ++i)
#pragma unroll
            for (int r = 0; r < R; ++r) v[i * R + r] = L[lds_pad(t + i * T + r * (N / R))];
        if constexpr (s > 0) {
#pragma unroll
            for (int i = 0; i < E / R; ++i) {
                const int k = (t + i * T) % Ns;
                apply_row<R>(&v[i * R], tw + S::tw_off(s) + k * R);
            }
        }
#pragma unroll
        for (int i = 0; i < E / R; ++i) Dft<R>::run(&v[i * R]);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < E / R; ++i) {
            const int j = t + i * T;
            const int base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
            for (int q = 0; q < R; ++q) L[lds_pad(base + q * Ns)] = v[i * R + q];
        }
        __syncthreads();
    });

    // ---- store phase
    const unsigned mask_all = (unsigned)(a.nbig - 1);
    const unsigned mask_lo = (1u << a.lo_bits) - 1u;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = tid + m * NT;
        const int k = e / C, ff = e % C;
        float2 x = lds[ff * LDSN + lds_pad(k)];
        if constexpr (PASS == 1) {
            const unsigned mm = ((unsigned)(c0 + ff) * (unsigned)k) & mask_all;
            const float2 w = cmul(a.tw_hi[mm >> a.lo_bits], a.tw_lo[mm & mask_lo]);
            dst[(long long)k * a.n_other + c0 + ff] = cmul(x, w);
        } else {
            x.y *= a.sg;
            dst[(long long)k * a.n_other + c0 + ff] = x;
        }
    }
}

template <int PASS, int N, int E, int C, class S>
hipError_t launch_fourstep(const float2* in, float2* out, const float2* tw, const FourStepArgs& a, hipStream_t st)
{
    const long long grid = a.batch * (long long)a.tiles;
    if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_fourstep<PASS, N, E, C, S>), dim3((unsigned)grid), dim3((N / E) * C), 0, st, in, out,
                       tw, a);
    return hipGetLastError();
}

template <int PASS, int N, int E, int C, class S>
constexpr TileEntry tile_entry(const char* name)
{
    TileEntry t{};
    t.pass = PASS;
    t.n = N;
    t.e = E;
    t.c = C;
    t.nr = S::count;
    for (int i = 0; i < S::count && i < 8; ++i) t.radix[i] = S::r(i);
    t.tw_size = S::tw_size();
    t.threads = (N / E) * C;
    t.lds = (size_t)C * (lds_pad(N) + 1) * sizeof(float2);
    t.launch = &launch_fourstep<PASS, N, E, C, S>;
    t.name = name;
    return t;
}

#define FB_TILE(P, N, E, C, ...) \
    tile_entry<P, N, E, C, Sched<__VA_ARGS__>>("fourstep_pass" #P "<" #N ",C" #C ",[" #__VA_ARGS__ "]>")

static const TileEntry kTiles[] = {
    FB_TILE(1, 32, 16, 16, 16, 2),
    FB_TILE(1, 64, 16, 16, 16, 4),
    FB_TILE(1, 128, 16, 16, 16, 8),
    FB_TILE(1, 256, 16, 16, 16, 16),
    FB_TILE(1, 512, 16, 16, 16, 16, 2),
    FB_TILE(1, 1024, 16, 16, 16, 16, 4),
    FB_TILE(1, 1024, 16, 8, 16, 16, 4),
    FB_TILE(1, 2048, 16, 8, 16, 16, 8),
    FB_TILE(2, 32, 16, 16, 16, 2),
    FB_TILE(2, 64, 16, 16, 16, 4),
    FB_TILE(2, 128, 16, 16, 16, 8),
    FB_TILE(2, 256, 16, 16, 16, 16),
    FB_TILE(2, 512, 16, 16, 16, 16, 2),
    FB_TILE(2, 1024, 16, 16, 16, 16, 4),
    FB_TILE(2, 1024, 16, 8, 16, 16, 4),
    FB_TILE(2, 2048, 16, 8, 16, 16, 8),
};

const TileEntry* tile_find(int pass, int n, int c)
{
    for (const TileEntry& t : kTiles)
        if (t.pass == pass && t.n == n && (c <= 0 || t.c == c)) return &t;
    return nullptr;
}

const TileEntry* tile_table(int* count)
{
    *count = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
    return kTiles;
}

}  // namespace fb
