// Device-side building blocks of the block FFT (gfx950, wave64).
//
// * In-register DFTs of radix 2, 4, 8, 16 and 32 (forward sign; the backward
//   transform is run as conj(forward(conj(x))), which is exact in FP32 since
//   negation does not round).  Larger radices are built from smaller ones by
//   the same split N = N1*N2 used between kernels (paper, Approach, "Other FFT
//   sizes": larger transforms from smaller blocks), with the inner twiddles
//   as compile-time constants and the multiplications by 1, -1, +-i and
//   (+-1 +-i)/sqrt(2) written out so they cost no general complex multiply.
// * The schedule type Sched<R0, R1, ...>: a list of radices whose product is
//   the transform length, with the per-stage strides and twiddle-table
//   offsets (paper, Background: a mixed-radix FFT as a sequence of radix
//   stages; Approach: a radix stage's inputs held in the private memory
//   (registers) of one processing element).
//
// A Stockham stage (autosort, natural-order output) of radix R after
// Ns = R0*...*R_{s-1} points have been combined maps butterfly j to inputs
// x[j + r*N/R], r < R, multiplies input r by exp(-2 pi i r (j mod Ns)/(Ns R)),
// takes the R-point DFT and writes output q to
// ((j / Ns) * Ns * R + j mod Ns) + q * Ns.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace fb {

template <int I>
using ic = std::integral_constant<int, I>;

// Compile-time loop: calls f(ic<B>), f(ic<B+1>), ..., f(ic<E-1>).
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f)
{
    if constexpr (B < E) {
        f(ic<B>{});
        sfor<B + 1, E>(f);
    }
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// a * w
__device__ __forceinline__ float2 cmul(float2 a, float2 w)
{
    return make_float2(fmaf(a.x, w.x, -(a.y * w.y)), fmaf(a.x, w.y, a.y * w.x));
}
// a * (c + i s) with compile-time c, s
__device__ __forceinline__ float2 cmul_cs(float2 a, float c, float s)
{
    return make_float2(fmaf(a.x, c, -(a.y * s)), fmaf(a.x, s, a.y * c));
}

// cos(2 pi u / 32) for u = 0..8 (the first quadrant of the 32nd roots of unity)
__host__ __device__ constexpr double cos32(int u)
{
    constexpr double t[9] = {1.0,
                             0.98078528040323044913,
                             0.92387953251128675613,
                             0.83146961230254523708,
                             0.70710678118654752440,
                             0.55557023301960222474,
                             0.38268343236508977173,
                             0.19509032201612826785,
                             0.0};
    return t[u];
}
// cos and sin of 2 pi q / 32 by quadrant symmetry
__host__ __device__ constexpr double cos_q32(int q)
{
    const int h = (q & 31) >> 3, u = q & 7;
    const double c = cos32(u), s = cos32(8 - u);
    return h == 0 ? c : h == 1 ? -s : h == 2 ? -c : s;
}
__host__ __device__ constexpr double sin_q32(int q)
{
    const int h = (q & 31) >> 3, u = q & 7;
    const double c = cos32(u), s = cos32(8 - u);
    return h == 0 ? s : h == 1 ? c : h == 2 ? -s : -c;
}

// Compile-time cos/sin of 2 pi q / R for any integer q and R > 0: quadrant
// reduction (exact at multiples of a quarter turn), then Taylor series on an
// angle of at most pi/4 (error below 1e-16 after 12 terms).
constexpr double kHalfPi = 1.57079632679489661923132169163975144;
__host__ __device__ constexpr double ct_sin_small(double x)
{
    double x2 = x * x, term = x, sum = x;
    for (int i = 1; i < 12; ++i) {
        term *= -x2 / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}
__host__ __device__ constexpr double ct_cos_small(double x)
{
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int i = 1; i < 12; ++i) {
        term *= -x2 / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}
// {cos, sin}(2 pi q / R)
__host__ __device__ constexpr double ct_cs(int q, int R, bool want_sin)
{
    int m = q % R;
    if (m < 0) m += R;
    const int quad = (4 * m) / R;
    const int rem = 4 * m - quad * R;  // angle within the quadrant = (pi/2) rem / R
    double c = 1.0, s = 0.0;
    if (rem != 0) {
        if (2 * rem <= R) {
            const double phi = kHalfPi * ((double)rem / (double)R);
            c = ct_cos_small(phi);
            s = ct_sin_small(phi);
        } else {
            const double phi = kHalfPi * ((double)(R - rem) / (double)R);
            c = ct_sin_small(phi);
            s = ct_cos_small(phi);
        }
    }
    const double cr = quad == 0 ? c : quad == 1 ? -s : quad == 2 ? -c : s;
    const double sr = quad == 0 ? s : quad == 1 ? c : quad == 2 ? -s : -c;
    return want_sin ? sr : cr;
}

// v * exp(-2 pi i Q / R).  Multiples of a quarter turn and odd multiples of
// an eighth turn are written without a general complex multiply.
template <int Q, int R>
__device__ __forceinline__ float2 mul_root(float2 v)
{
    constexpr int q0 = ((Q % R) + R) % R;
    constexpr bool eighth = (8 * q0) % R == 0;
    constexpr int q = eighth ? (8 * q0) / R * 4 : -1;  // in 32nds when on the eighth grid
    constexpr float h = 0.70710678118654752440f;
    if constexpr (q0 == 0) {
        return v;
    } else if constexpr (q == 8) {
        return make_float2(v.y, -v.x);
    } else if constexpr (q == 16) {
        return make_float2(-v.x, -v.y);
    } else if constexpr (q == 24) {
        return make_float2(-v.y, v.x);
    } else if constexpr (q == 4) {
        return make_float2(h * (v.x + v.y), h * (v.y - v.x));
    } else if constexpr (q == 12) {
        return make_float2(h * (v.y - v.x), -h * (v.x + v.y));
    } else if constexpr (q == 20) {
        return make_float2(-h * (v.x + v.y), h * (v.x - v.y));
    } else if constexpr (q == 28) {
        return make_float2(h * (v.x - v.y), h * (v.x + v.y));
    } else {
        constexpr float c = (float)ct_cs(q0, R, false);
        constexpr float sn = (float)(-ct_cs(q0, R, true));
        return cmul_cs(v, c, sn);
    }
}

// ------------------------------------------------------------ small DFTs
// Dft<R>::run(v) replaces v[0..R) by its forward R-point DFT, natural order.
template <int R>
struct Dft;

template <>
struct Dft<1> {
    static __device__ __forceinline__ void run(float2*) {}
};

template <>
struct Dft<2> {
    static __device__ __forceinline__ void run(float2* v)
    {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <>
struct Dft<4> {
    static __device__ __forceinline__ void run(float2* v)
    {
        const float2 t0 = cadd(v[0], v[2]);
        const float2 t1 = csub(v[0], v[2]);
        const float2 t2 = cadd(v[1], v[3]);
        const float2 d = csub(v[1], v[3]);
        const float2 t3 = make_float2(d.y, -d.x);  // (v1 - v3) * (-i)
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

// 3-point DFT: X1,2 = x0 - (x1+x2)/2 -/+ i (sqrt(3)/2)(x1 - x2).
template <>
struct Dft<3> {
    static __device__ __forceinline__ void run(float2* v)
    {
        constexpr float s3 = 0.86602540378443864676f;
        const float2 a = cadd(v[1], v[2]);
        const float2 b = csub(v[1], v[2]);
        const float2 m = make_float2(fmaf(-0.5f, a.x, v[0].x), fmaf(-0.5f, a.y, v[0].y));
        v[0] = cadd(v[0], a);
        v[1] = make_float2(fmaf(s3, b.y, m.x), fmaf(-s3, b.x, m.y));
        v[2] = make_float2(fmaf(-s3, b.y, m.x), fmaf(s3, b.x, m.y));
    }
};

// 5-point DFT with the symmetric pairs (x1, x4) and (x2, x3):
//   X1,4 = x0 + c1 a1 + c2 a2 -/+ i (s1 b1 + s2 b2)
//   X2,3 = x0 + c2 a1 + c1 a2 -/+ i (s2 b1 - s1 b2)
// with a = sums, b = differences, c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5).
template <>
struct Dft<5> {
    static __device__ __forceinline__ void run(float2* v)
    {
        constexpr float c1 = (float)ct_cs(1, 5, false), c2 = (float)ct_cs(2, 5, false);
        constexpr float s1 = (float)ct_cs(1, 5, true), s2 = (float)ct_cs(2, 5, true);
        const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
        const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        const float2 x0 = v[0];
        const float2 m1 = make_float2(fmaf(c2, a2.x, fmaf(c1, a1.x, x0.x)), fmaf(c2, a2.y, fmaf(c1, a1.y, x0.y)));
        const float2 m2 = make_float2(fmaf(c1, a2.x, fmaf(c2, a1.x, x0.x)), fmaf(c1, a2.y, fmaf(c2, a1.y, x0.y)));
        const float2 n1 = make_float2(fmaf(s2, b2.x, s1 * b1.x), fmaf(s2, b2.y, s1 * b1.y));
        const float2 n2 = make_float2(fmaf(-s1, b2.x, s2 * b1.x), fmaf(-s1, b2.y, s2 * b1.y));
        v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
        v[1] = make_float2(m1.x + n1.y, m1.y - n1.x);  // m1 - i n1
        v[4] = make_float2(m1.x - n1.y, m1.y + n1.x);  // m1 + i n1
        v[2] = make_float2(m2.x + n2.y, m2.y - n2.x);
        v[3] = make_float2(m2.x - n2.y, m2.y + n2.x);
    }
};

__host__ __device__ constexpr int dft_split(int R)
{
    return R == 8 ? 4 : R == 16 ? 4 : R == 32 ? 8 : R == 6 ? 2 : R == 10 ? 2 : R == 12 ? 4 : R == 15 ? 3 : R == 20 ? 4 : 1;
}

// R = R1 * R2: with n = R2*n1 + n2 and k = k1 + R1*k2,
//   X[k] = sum_{n2} w_R2^{n2 k2} [ w_R^{n2 k1} sum_{n1} x[R2 n1 + n2] w_R1^{n1 k1} ].
template <int R>
struct Dft {
    static constexpr int R1 = dft_split(R);
    static constexpr int R2 = R / R1;
    static_assert(R1 > 1 && R2 > 1, "unsupported radix");
    static __device__ __forceinline__ void run(float2* v)
    {
        float2 a[R];
        sfor<0, R2>([&](auto n2c) {
            constexpr int n2 = decltype(n2c)::value;
            float2 u[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) u[n1] = v[R2 * n1 + n2];
            Dft<R1>::run(u);
            sfor<0, R1>([&](auto k1c) {
                constexpr int k1 = decltype(k1c)::value;
                a[n2 * R1 + k1] = mul_root<n2 * k1, R>(u[k1]);
            });
        });
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            float2 w[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) w[n2] = a[n2 * R1 + k1];
            Dft<R2>::run(w);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = w[k2];
        }
    }
};

// --------------------------------------------------------------- schedule
template <int... Rs>
struct Sched {
    static constexpr int count = sizeof...(Rs);
    static constexpr int r(int s)
    {
        constexpr int a[] = {Rs...};
        return a[s];
    }
    // points already combined before stage s
    static constexpr int ns(int s)
    {
        int p = 1;
        for (int i = 0; i < s; ++i) p *= r(i);
        return p;
    }
    static constexpr int n() { return ns(count); }
    // offset of stage s's twiddle rows (stage 0 needs none): rows k < Ns of R entries
    // (each stage's block is padded to an even number of entries)
    static constexpr int tw_off(int s)
    {
        int o = 0;
        for (int i = 1; i < s; ++i) o += (ns(i) * r(i) + 1) & ~1;
        return o;
    }
    static constexpr int tw_size() { return tw_off(count); }
    // Factorised layout (persistent kernels keep it in LDS): a stage with
    // Ns <= 16 keeps its full rows; a larger one stores A[q][r] = w_{Q R}^{r q}
    // for q < Q, then B[p][r] = w_{Ns R}^{r p} for p < M, with Ns = Q M and Q
    // the largest power of two whose square is <= Ns, so that
    // w_{Ns R}^{r (q M + p)} = A[q][r] * B[p][r].
    static constexpr bool f_full(int s) { return ns(s) <= 16; }
    static constexpr int fq(int s)
    {
        int q = 1;
        while (4 * q * q <= ns(s)) q *= 2;
        return f_full(s) ? ns(s) : q;
    }
    static constexpr int fm(int s) { return f_full(s) ? 1 : ns(s) / fq(s); }
    static constexpr int f_size(int s) { return f_full(s) ? ns(s) * r(s) : (fq(s) + fm(s)) * r(s); }
    static constexpr int ftw_off(int s)
    {
        int o = 0;
        for (int i = 1; i < s; ++i) o += f_size(i);
        return o;
    }
    static constexpr int ftw_size() { return ftw_off(count); }
    // Power layout: row k of stage s holds w^(2^i), i < log2(R), for
    // w = w_{Ns R}^k (padded to an even count for 16-byte loads); the other
    // powers are formed by products (binary decomposition of the exponent).
    static constexpr int bits(int v) { return v <= 0 ? 0 : 1 + bits(v / 2); }
    static constexpr int p_row(int s) { return (bits(r(s) - 1) + 1) & ~1; }
    static constexpr int ptw_off(int s)
    {
        int o = 0;
        for (int i = 1; i < s; ++i) o += ns(i) * p_row(i);
        return o;
    }
    static constexpr int ptw_size() { return ptw_off(count); }
    static constexpr int max_r()
    {
        int m = 1;
        for (int i = 0; i < count; ++i) m = r(i) > m ? r(i) : m;
        return m;
    }
};

// LDS index with one pad slot per 16 complex values (keeps stride-16 and
// stride-R butterfly accesses on distinct banks).
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }

// Multiplies the R inputs of one butterfly by its twiddle row
// tw[k*R + r] = exp(-2 pi i r k / (Ns R)); even radices load 16-byte pairs
// (rows start on even entries), odd radices single entries.
template <int R>
__device__ __forceinline__ void apply_row(float2* v, const float2* __restrict__ row)
{
    if constexpr (R == 1) {
        return;
    } else if constexpr (R % 2 == 0) {
        const float4* row4 = reinterpret_cast<const float4*>(row);
#pragma unroll
        for (int r = 0; r < R; r += 2) {
            const float4 w = row4[r / 2];
            if (r > 0) v[r] = cmul(v[r], make_float2(w.x, w.y));
            v[r + 1] = cmul(v[r + 1], make_float2(w.z, w.w));
        }
    } else {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], row[r]);
    }
}

// ------------------------------------------------------ global accesses
// Variant flags of the transform kernels.
enum : int {
    kNtLoad = 1,   // non-temporal (streaming) global loads of the transform data
    kNtStore = 2,  // non-temporal global stores of the transform data
    kPipe = 4,     // persistent workgroups that prefetch the next unit's inputs
};

typedef float v2f_t __attribute__((ext_vector_type(2)));
// Two IEEE half values: the storage element of the FP16-storage form.
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

template <int FL>
__device__ __forceinline__ float2 gload(const float2* p)
{
    if constexpr ((FL & kNtLoad) != 0) {
        const v2f_t t = __builtin_nontemporal_load(reinterpret_cast<const v2f_t*>(p));
        return make_float2(t.x, t.y);
    } else {
        return *p;
    }
}

// FP16 storage: widened to FP32 on load, rounded to nearest even on store.
template <int FL>
__device__ __forceinline__ float2 gload(const h2_t* p)
{
    h2_t h;
    if constexpr ((FL & kNtLoad) != 0)
        h = __builtin_nontemporal_load(p);
    else
        h = *p;
    return make_float2((float)h.x, (float)h.y);
}

template <int FL>
__device__ __forceinline__ void gstore(h2_t* p, float2 v)
{
    h2_t h;
    h.x = (_Float16)v.x;
    h.y = (_Float16)v.y;
    if constexpr ((FL & kNtStore) != 0)
        __builtin_nontemporal_store(h, p);
    else
        *p = h;
}

template <int FL>
__device__ __forceinline__ void gstore(float2* p, float2 v)
{
    if constexpr ((FL & kNtStore) != 0) {
        v2f_t t;
        t.x = v.x;
        t.y = v.y;
        __builtin_nontemporal_store(t, reinterpret_cast<v2f_t*>(p));
    } else {
        *p = v;
    }
}

// Sixteen-byte accesses: two consecutive complex values in one lane.
typedef float v4f_t __attribute__((ext_vector_type(4)));

template <int FL>
__device__ __forceinline__ float4 gload2(const float2* p)
{
    if constexpr ((FL & kNtLoad) != 0) {
        const v4f_t t = __builtin_nontemporal_load(reinterpret_cast<const v4f_t*>(p));
        return make_float4(t.x, t.y, t.z, t.w);
    } else {
        return *reinterpret_cast<const float4*>(p);
    }
}

template <int FL>
__device__ __forceinline__ void gstore2(float2* p, float2 lo, float2 hi)
{
    v4f_t t;
    t.x = lo.x;
    t.y = lo.y;
    t.z = hi.x;
    t.w = hi.y;
    if constexpr ((FL & kNtStore) != 0)
        __builtin_nontemporal_store(t, reinterpret_cast<v4f_t*>(p));
    else
        *reinterpret_cast<v4f_t*>(p) = t;
}

// The value of the neighbouring lane (lane ^ 1), by a DPP quad permutation
// [1,0,3,2]: a VALU operand modifier, no LDS traffic.  Every lane of the pair
// must be active.
__device__ __forceinline__ float2 lane_xor1(float2 v)
{
    float2 r;
    r.x = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.x), 0xB1, 0xF, 0xF, true));
    r.y = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v.y), 0xB1, 0xF, 0xF, true));
    return r;
}

// Powers w^r, r < R, from the row w^(2^i), 2^i < R (FP64-generated,
// FP32-stored): w^r = w^h * w^(r-h) with h the highest power of two in r, so
// each power carries at most popcount(r) - 1 complex products.
template <int R>
__device__ __forceinline__ void powers_from_row(float2 (&w)[R], const float2* __restrict__ row)
{
    constexpr int P = (R - 1) >= 16 ? 5 : (R - 1) >= 8 ? 4 : (R - 1) >= 4 ? 3 : (R - 1) >= 2 ? 2 : 1;
    constexpr int PP = (P + 1) & ~1;
    float2 p[PP];
    const float4* row4 = reinterpret_cast<const float4*>(row);
#pragma unroll
    for (int i = 0; i < PP; i += 2) {
        const float4 q = row4[i / 2];
        p[i] = make_float2(q.x, q.y);
        p[i + 1] = make_float2(q.z, q.w);
    }
    w[0] = make_float2(1.f, 0.f);
    sfor<1, R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        constexpr int h = (r >= 16) ? 16 : (r >= 8) ? 8 : (r >= 4) ? 4 : (r >= 2) ? 2 : 1;
        constexpr int hi = (h == 16) ? 4 : (h == 8) ? 3 : (h == 4) ? 2 : (h == 2) ? 1 : 0;
        if constexpr (r == h)
            w[r] = p[hi];
        else
            w[r] = cmul(w[h], w[r - h]);
    });
}

// Multiplies input r of one radix-R butterfly by w^r (powers from the row).
template <int R>
__device__ __forceinline__ void apply_pow_row(float2* v, const float2* __restrict__ row)
{
    if constexpr (R > 1) {
        float2 w[R];
        powers_from_row<R>(w, row);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
    }
}

}  // namespace fb
