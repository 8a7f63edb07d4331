// Host side of the C ABI declared in include/fftblock.h: argument checks,
// the planner (block limit, path, kernel choice, four-step split), FP64
// twiddle generation, plan lifetime and launches.
//
// Planner (paper, Approach): the largest transform one compute unit holds is
// derived from the local-memory size -- on gfx950 the LDS, 160 KB per CU --
// as pow2floor(LDS / (8 B * (1 + 1/16) * k)) for k resident workgroups; the
// runtime sweep then confirms which single-block lengths actually win (the
// paper pairs the analytic bound with a measurement in the same way).
// Lengths up to the limit run as one block per transform; longer
// power-of-two lengths run the four-step split N = N1 * N2 (powers of two,
// the split chosen by measurement, see plan_choose).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "../../include/fftblock.h"
#include "internal.hpp"

using namespace fb;

struct fft_plan_s {
    size_t n = 0, batch = 0;
    int direction = FFT_FORWARD;
    int path = 0;
    int device = 0;
    const KEntry* k1 = nullptr;     // block kernel, or four-step pass 1
    const KEntry* k2 = nullptr;     // four-step pass 2
    size_t n1 = 0, n2 = 0;
    int lo_bits = 0;
    int cw_bits = 0;
    long long grid1 = 0, grid2 = 0;
    float2* tw = nullptr;           // one allocation holding every table
    size_t tw_bytes = 0;
    size_t off_s1 = 0, off_s2 = 0, off_hi = 0, off_lo = 0, off_col = 0;  // in complex entries
    size_t off_flt = 0;             // range compression: spectrum of the pulse replica
    float2* work = nullptr;
    size_t work_bytes = 0;
    std::vector<TwSeg> segs;        // layout of the twiddle table
    int storage = 0;                // 0: complex64 data, 1: FP16 pairs, 2: FP16 pairs and workspace
    int device_twiddles = 0;        // tables generated on the device
    float scale = 1.0f;             // multiplier of the final outputs
    int cus = 0;                    // compute units of the plan's device
    const KEntry* klist = nullptr;  // list form of k1 (same schedule and shape), if compiled
    const KEntry* kn = nullptr;     // one-wave form of a default k1, for small batches
    int rt_nr = 0;                  // run-time-schedule kernel: the plan's schedule
    int rt_radix[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace fb {

static std::vector<KEntry> build_table()
{
    std::vector<KEntry> v;
    int nb = 0, np = 0, nf = 0, nl = 0, nr = 0;
    const KEntry* b = block_entries(&nb);
    const KEntry* p = pass_entries(&np);
    const KEntry* f = filter_entries(&nf);
    const KEntry* l = list_entries(&nl);
    const KEntry* r = rt_entries(&nr);
    int nx = 0, nv = 0;
    const KEntry* x = xlane_entries(&nx);
    const KEntry* vt = vt_entries(&nv);
    v.insert(v.end(), b, b + nb);
    v.insert(v.end(), p, p + np);
    v.insert(v.end(), f, f + nf);
    v.insert(v.end(), l, l + nl);
    v.insert(v.end(), r, r + nr);
    v.insert(v.end(), x, x + nx);
    v.insert(v.end(), vt, vt + nv);
    return v;
}

static const std::vector<KEntry>& table()
{
    static const std::vector<KEntry> t = build_table();
    return t;
}

const KEntry* kernel_table(int* count)
{
    *count = (int)table().size();
    return table().data();
}

// Bytes per point of the four-step workspace: complex64, or FP16 pairs in
// the compact form.
size_t work_elem(int storage) { return storage == FFT_STORAGE_F16_COMPACT ? 2 * sizeof(uint16_t) : sizeof(float2); }

const KEntry* kernel_default(int kind, int n, int c, int storage)
{
    // the compact FP16 form differs from FP16 storage only in the four-step workspace
    const bool ws = storage == FFT_STORAGE_F16_COMPACT && (kind == kKindPass1 || kind == kKindPass2);
    const KEntry* any = nullptr;
    for (const KEntry& k : table()) {
        if (k.kind != kind || k.n != n || (c > 0 && k.c != c)) continue;
        if (((k.flags & FFT_VARIANT_FP16_STORAGE) != 0) != (storage != 0)) continue;
        if (((k.flags & FFT_VARIANT_FP16_WORKSPACE) != 0) != ws) continue;
        if (k.is_default) return &k;
        if (!any && (k.flags & ~(FFT_VARIANT_FP16_STORAGE | FFT_VARIANT_FP16_WORKSPACE)) == 0) any = &k;
    }
    return any;
}

const KEntry* kernel_find(int kind, int n, const int* radix, int nr, int c, int flags)
{
    for (const KEntry& k : table()) {
        if (k.kind != kind || k.n != n) continue;
        if (c > 0 && k.c != c) continue;
        if (flags >= 0 && k.flags != flags) continue;
        if (nr > 0) {
            if (k.nr != nr) continue;
            bool same = true;
            for (int i = 0; i < nr; ++i) same = same && k.radix[i] == radix[i];
            if (!same) continue;
        }
        return &k;
    }
    return nullptr;
}

long long kernel_units(const KEntry& k, const KArgs& a)
{
    if (k.kind == kKindBlock || k.kind == kKindFilter || k.kind == kKindList) return (a.batch + k.c - 1) / k.c;
    return a.batch * a.tiles;
}

// exp(-2 pi i m / n) in FP64 by quadrant reduction: the angle handed to
// cos/sin never exceeds pi/4, and multiples of a quarter turn are exact.
void root_fwd(long long m, long long n, double* re, double* im)
{
    m %= n;
    if (m < 0) m += n;
    const long long q = (4 * m) / n;
    const long long rem = 4 * m - q * n;  // angle within the quadrant = (pi/2) * rem / n
    const double half_pi = 1.57079632679489661923132169163975144;
    double c, s;
    if (2 * rem <= n) {
        const double phi = half_pi * ((double)rem / (double)n);
        c = std::cos(phi);
        s = std::sin(phi);
    } else {
        const double phi = half_pi * ((double)(n - rem) / (double)n);
        c = std::sin(phi);
        s = std::cos(phi);
    }
    double cr, sr;
    switch (q) {
        case 0: cr = c; sr = s; break;
        case 1: cr = -s; sr = c; break;
        case 2: cr = -c; sr = -s; break;
        default: cr = s; sr = -c; break;
    }
    *re = cr;
    *im = -sr;
}

float2 root_f32(long long m, long long n)
{
    double re, im;
    root_fwd(m, n, &re, &im);
    return make_float2((float)re, (float)im);  // one round-to-nearest-even from FP64
}

}  // namespace fb

namespace {

std::mutex g_mu;
std::unordered_set<fft_plan_s*> g_plans;

bool plan_live(fft_plan_s* p)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return p != nullptr && g_plans.count(p) != 0;
}

fft_status_t from_hip(hipError_t e)
{
    if (e == hipSuccess) return FFT_SUCCESS;
    if (e == hipErrorOutOfMemory) return FFT_ERR_OUT_OF_MEMORY;
    return FFT_ERR_DEVICE;
}

bool is_pow2(size_t n) { return n != 0 && (n & (n - 1)) == 0; }

int ilog2(size_t n)
{
    int l = 0;
    while ((size_t(1) << l) < n) ++l;
    return l;
}

// (m, n) of one table entry, per segment type (see TwSeg in internal.hpp).
bool seg_entry(const TwSeg& g, long long e, long long* m, long long* n)
{
    switch (g.type) {
        case kSegRows: *m = (e % g.b) * (e / g.b); *n = g.a * g.b; return true;
        case kSegPow: {
            const long long i = e % g.c;
            if (i >= g.d) return false;
            *m = (e / g.c) << i;
            *n = g.a * g.b;
            return true;
        }
        case kSegHi: *m = e << g.b; *n = g.a; return true;
        case kSegLo: *m = e; *n = g.a; return true;
        case kSegCol: {
            const long long i = e % g.c;
            if ((1LL << i) >= g.d) return false;
            *m = (((e / g.c) * g.b) << i) % g.a;
            *n = g.a;
            return true;
        }
    }
    return false;
}

void eval_segments_host(const std::vector<TwSeg>& segs, float2* dst)
{
    for (const TwSeg& g : segs)
        for (long long e = 0; e < g.count; ++e) {
            long long m = 0, n = 1;
            dst[g.offset + e] = seg_entry(g, e, &m, &n) ? root_f32(m, n) : make_float2(0.f, 0.f);
        }
}

int bits_of(int v)
{
    int b = 0;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

// Segments of a kernel's stage table starting at `at` (entries); returns the end.
long long stage_segments(const KEntry* k, long long at, std::vector<TwSeg>& segs)
{
    long long ns = k->radix[0];
    for (int s = 1; s < k->nr; ++s) {
        const long long R = k->radix[s];
        if (k->flags & FFT_VARIANT_PERSISTENT) {
            // factorised rows: full rows for Ns <= 16, else A (Q rows of the
            // Q R-th roots) then B (the first M rows of the Ns R-th roots)
            if (ns <= 16) {
                segs.push_back({kSegRows, at, ns * R, ns, R, 0, 0});
                at += ns * R;
            } else {
                long long Q = 1;
                while (4 * Q * Q <= ns) Q *= 2;
                const long long M = ns / Q;
                segs.push_back({kSegRows, at, Q * R, Q, R, 0, 0});
                at += Q * R;
                segs.push_back({kSegRows, at, M * R, ns, R, 0, 0});
                at += M * R;
            }
        } else if (k->flags & FFT_VARIANT_TWIDDLE_POWERS) {
            // power rows: w^(2^i) for 2^i < R, padded to an even count
            const int P = bits_of((int)R - 1);
            const int row = (P + 1) & ~1;
            segs.push_back({kSegPow, at, ns * row, ns, R, row, P});
            at += ns * row;
        } else {
            // exact rows, each stage's block padded to an even count
            segs.push_back({kSegRows, at, ns * R, ns, R, 0, 0});
            at += (ns * R + 1) & ~1LL;
        }
        ns *= R;
    }
    return at;
}

size_t env_size(const char* name, size_t dflt)
{
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    char* end = nullptr;
    const unsigned long long x = std::strtoull(v, &end, 10);
    return (end && *end == 0 && x > 0) ? (size_t)x : dflt;
}

constexpr size_t kMaxN = size_t(1) << 22;
// Longest single block: with half exchanges 32768 points fit the LDS of one
// workgroup (16384 exchange slots).
constexpr size_t kDefaultBlockLimit = kMaxBlockLen;
// Longest length with a compiled list form, filter and mixed-radix blocks.
constexpr size_t kLongBlock = 16384;

// Smallest batch at which the default plan of a power-of-two length takes the
// single block.  From 8192 on a transform holds a large share of a compute
// unit's LDS (half of it at 16384, all of it at 32768), so a small batch
// occupies few compute units, while the four-step path spreads every
// transform over many workgroups.  Measured crossovers (microseconds per
// execute, block against four-step): 8192 x 4: 9.0 / 7.8, x 16: 8.3 / 8.4;
// 16384 x 1: 11.2 / 7.6, x 32: 12.2 / 10.6, x 64: 12.7 / 13.9; 32768 x 1:
// 19.4 / 8.1, x 48: 22.1 / 18.0, x 96: 23.8 / 26.5.  FP16 storage halves
// the block's bytes but not the four-step workspace's, which moves the
// crossovers down: 8192 x 1: 7.4 / 8.3; 16384 x 24: 10.7 / 10.6, x 32:
// 10.6 / 11.2; 32768 x 32: 17.7 / 14.1, x 48: 18.0 / 18.1.  Options that name
// a block kernel or a block limit keep the block at any batch.
size_t block_min_batch(size_t n, int storage)
{
    if (storage)
        return n >= 32768 ? 48 : n >= 16384 ? 32 : 1;
    return n >= 32768 ? 64 : n >= 16384 ? 48 : n >= 8192 ? 16 : 1;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t sanitize_limit(size_t lim)
{
    if (!is_pow2(lim) || lim < 1024 || lim > kMaxBlockLen) return kDefaultBlockLimit;
    return lim;
}

// Entries per row of a power table for exponents below e: log2(e), padded even.
int col_row(int e)
{
    int lg = 0;
    while ((1 << lg) < e) ++lg;
    return (lg + 1) & ~1;
}

int log2i(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

extern "C" {

const char* fft_status_string(fft_status_t s)
{
    switch (s) {
        case FFT_SUCCESS: return "success";
        case FFT_ERR_INVALID_ARG: return "invalid argument";
        case FFT_ERR_UNSUPPORTED_SIZE: return "unsupported transform size";
        case FFT_ERR_OUT_OF_MEMORY: return "device out of memory";
        case FFT_ERR_DEVICE: return "HIP runtime error";
        case FFT_ERR_INVALID_PLAN: return "invalid plan handle";
        case FFT_ERR_TIMEOUT: return "timed out";
        case FFT_ERR_SCRATCH_LIMIT: return "request exceeds the library's static scratch buffer";
    }
    return "unknown status";
}

size_t fft_block_limit(void) { return sanitize_limit(env_size("FFTBLOCK_BLOCK_MAX", kDefaultBlockLimit)); }

void fft_plan_opts_init(fft_plan_opts_t* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->flags = -1;
    o->flags2 = -1;
    o->storage = 0;
    o->device_twiddles = 0;
}

size_t fft_block_max(size_t lds_bytes, int k)
{
    if (k < 1) return 0;
    const double per = 8.0 * (1.0 + 1.0 / 16.0) * (double)k;
    const size_t v = (size_t)((double)lds_bytes / per);
    if (v == 0) return 0;
    size_t p2 = 1;
    while (p2 * 2 <= v) p2 *= 2;
    return p2;
}

int fft_kernel_count(void)
{
    int c = 0;
    kernel_table(&c);
    return c;
}

fft_status_t fft_kernel_info(int index, fft_kernel_info_t* info)
{
    if (info == nullptr) return FFT_ERR_INVALID_ARG;
    int c = 0;
    const KEntry* t = kernel_table(&c);
    if (index < 0 || index >= c) return FFT_ERR_INVALID_ARG;
    const KEntry& k = t[index];
    std::memset(info, 0, sizeof(*info));
    info->kind = k.kind;
    info->n = k.n;
    info->e = k.e;
    info->c = k.c;
    info->flags = k.flags;
    info->n_radix = k.nr;
    for (int i = 0; i < k.nr; ++i) info->radix[i] = k.radix[i];
    info->threads = k.threads;
    info->lds_bytes = k.lds;
    info->is_default = k.is_default ? 1 : 0;
    info->name = k.name;
    return FFT_SUCCESS;
}

fft_status_t fft_kernel_occupancy(int index, int* workgroups_per_cu)
{
    if (workgroups_per_cu == nullptr) return FFT_ERR_INVALID_ARG;
    int c = 0;
    const KEntry* t = kernel_table(&c);
    if (index < 0 || index >= c) return FFT_ERR_INVALID_ARG;
    const int occ = t[index].occupancy ? t[index].occupancy() : 0;
    if (occ <= 0) return FFT_ERR_DEVICE;
    *workgroups_per_cu = occ;
    return FFT_SUCCESS;
}

// Small batches: below this many workgroups of the full-width kernel (half
// the compute units of a 256-CU device) the one-wave form of the same
// schedule and variant, with fewer transforms per workgroup, spreads the
// batch over more CUs.  Measured (kernel trace, N = 256 ... 3072): 1.06 to
// 1.32 times faster below the threshold, within 3 % either way above it.
static constexpr long long kNarrowBelow = 128;

// The one-wave (narrowest) form of block kernel k, if compiled.
static const KEntry* narrow_of(const KEntry* k)
{
    const KEntry* best = nullptr;
    int c = 0;
    const KEntry* t = kernel_table(&c);
    for (int i = 0; i < c; ++i) {
        const KEntry& q = t[i];
        if (q.kind != kKindBlock || q.n != k->n || q.e != k->e || q.flags != k->flags || q.nr != k->nr ||
            q.c >= k->c)
            continue;
        bool same = true;
        for (int r = 0; r < q.nr; ++r) same = same && q.radix[r] == k->radix[r];
        if (same && (!best || q.c < best->c)) best = &q;
    }
    return best;
}

// The block-path kernel that runs `batch` transforms.
static const KEntry* block_kernel(const fft_plan_s* p, size_t batch)
{
    if (p->kn && (long long)((batch + (size_t)p->k1->c - 1) / (size_t)p->k1->c) < kNarrowBelow) return p->kn;
    return p->k1;
}

// Pure host planning: path, kernels, four-step split and table layout.
// Makes no HIP call, so it is usable (and testable) without a device.
static fft_status_t plan_choose(size_t n, size_t batch, int direction, const fft_plan_opts_t* opts,
                                fft_plan_s* p, size_t* table_entries)
{
    if (n == 0 || batch == 0) return FFT_ERR_INVALID_ARG;
    if (direction != FFT_FORWARD && direction != FFT_BACKWARD) return FFT_ERR_INVALID_ARG;
    if (n > kMaxN) return FFT_ERR_UNSUPPORTED_SIZE;
    if (!is_pow2(n) && (n > kLongBlock || !kernel_default(kKindBlock, (int)n, 0, 0)))
        return FFT_ERR_UNSUPPORTED_SIZE;  // other lengths: the compiled mixed-radix blocks only
    if (batch > ((size_t)1 << 40) / n) return FFT_ERR_INVALID_ARG;
    fft_plan_opts_t o;
    fft_plan_opts_init(&o);
    if (opts) o = *opts;
    if (o.n_radix < 0 || o.n_radix > 8) return FFT_ERR_INVALID_ARG;
    p->n = n;
    p->batch = batch;
    p->direction = direction;
    if (o.storage != FFT_STORAGE_C64 && o.storage != FFT_STORAGE_F16 && o.storage != FFT_STORAGE_F16_COMPACT)
        return FFT_ERR_INVALID_ARG;
    if (o.flags >= 0 && (((o.flags & FFT_VARIANT_FP16_STORAGE) != 0) != (o.storage != 0))) return FFT_ERR_INVALID_ARG;
    p->storage = o.storage;
    p->device_twiddles = o.device_twiddles ? 1 : 0;
    if (!std::isfinite(o.scale)) return FFT_ERR_INVALID_ARG;
    p->scale = o.scale == 0.0f ? 1.0f : o.scale;
    const int sto = o.storage;
    const size_t limit = o.block_limit ? sanitize_limit(o.block_limit) : fft_block_limit();
    long long off = 0;
    p->segs.clear();
    if (n == 1) {
        p->path = FFT_PATH_BLOCK;
    } else if (!is_pow2(n) ||
               (n <= limit && (batch >= block_min_batch(n, sto) || o.block_limit || o.n_radix || o.flags >= 0 || o.c > 0))) {
        p->path = FFT_PATH_BLOCK;
        if (o.n_radix == 0 && o.flags < 0 && o.c <= 0) {
            p->k1 = sto ? nullptr : wisdom_kernel(n, p->rt_radix, &p->rt_nr);
            if (!p->k1) {
                p->k1 = kernel_default(kKindBlock, (int)n, 0, sto);
                if (p->k1) p->kn = narrow_of(p->k1);   // same table layout (same schedule and variant)
            }
        } else {
            const bool want_rt = o.flags >= 0 && (o.flags & FFT_VARIANT_RUNTIME_SCHEDULE) != 0;
            const int fl = o.flags < 0 ? (sto ? FFT_VARIANT_FP16_STORAGE : 0) : o.flags;
            if (!want_rt) p->k1 = kernel_find(kKindBlock, (int)n, o.radix, o.n_radix, o.c, fl);
            // a schedule no compiled kernel has (or one asked for this way):
            // the run-time-schedule kernel, for radices 2, 4, 8 and 16
            if (!p->k1 && o.n_radix > 0 && sto == 0 && (o.flags < 0 || want_rt)) {
                size_t prod = 1;
                bool ok = o.n_radix <= 8;
                for (int i = 0; i < o.n_radix && ok; ++i) {
                    const int R = o.radix[i];
                    ok = R == 2 || R == 4 || R == 8 || R == 16;
                    prod *= ok ? (size_t)R : 1;
                }
                if (!ok || prod != n) return FFT_ERR_UNSUPPORTED_SIZE;
                for (const KEntry& k : table())
                    if (k.kind == kKindBlock && (size_t)k.n == n && (k.flags & FFT_VARIANT_RUNTIME_SCHEDULE) &&
                        (o.c <= 0 || k.c == o.c))
                        p->k1 = &k;
                if (!p->k1) return FFT_ERR_UNSUPPORTED_SIZE;
                p->rt_nr = o.n_radix;
                for (int i = 0; i < o.n_radix; ++i) p->rt_radix[i] = o.radix[i];
            }
        }
        if (!p->k1) return FFT_ERR_UNSUPPORTED_SIZE;
        if (p->rt_nr > 0) {
            // exact rows for the plan's schedule, laid out as the kernel walks them
            KEntry sk = *p->k1;
            sk.nr = p->rt_nr;
            for (int i = 0; i < p->rt_nr; ++i) sk.radix[i] = p->rt_radix[i];
            sk.flags = 0;
            off = stage_segments(&sk, 0, p->segs);
        } else {
            off = stage_segments(p->k1, 0, p->segs);
        }
    } else {
        p->path = FFT_PATH_FOURSTEP;
        const int L = ilog2(n);
        if (o.n1 != 0 && (!is_pow2(o.n1) || o.n1 < 2 || o.n1 > n / 2)) return FFT_ERR_INVALID_ARG;
        // Default split: rows (pass 2, contiguous) as long as the compiled
        // passes allow (2048, or the block limit), columns (pass 1, strided,
        // LDS-bound to one workgroup per CU at 1024 and beyond) no longer than
        // needed but at least 256 so each column read is 128-byte runs of 16
        // columns over many rows.  Measured on 2^15..2^22 it is the fastest
        // split everywhere (e.g. 2^21: 1024 x 2048 121 us vs 2048 x 1024
        // 144 us).  Short forced four-step lengths keep the balanced split.
        // FP16 storage halves the output runs of pass 2 (CW rows x 4 bytes), so
        // its rows stop at 1024 where 16-row tiles still fit the LDS
        size_t n1 = size_t(1) << ((L + 1) / 2);
        const size_t rows_max = std::min<size_t>(o.storage ? 1024 : 2048, limit);
        const size_t cand = std::max<size_t>(256, n / rows_max);
        if (cand <= std::min<size_t>(2048, limit) && n / cand >= 32 && n / cand <= rows_max) n1 = cand;
        p->n1 = o.n1 ? o.n1 : n1;
        p->n2 = n / p->n1;
        const int c1 = o.c > 0 ? o.c : (int)env_size("FFTBLOCK_FOURSTEP_C", 0);
        const int c2 = o.c2 > 0 ? o.c2 : (int)env_size("FFTBLOCK_FOURSTEP_C2", 0);
        const bool explicit_opts = o.flags >= 0 || o.flags2 >= 0 || o.c > 0 || o.c2 > 0 || o.n1 != 0 || o.n_radix > 0;
        if (!explicit_opts && !sto && wisdom_pair(n, &p->k1, &p->k2)) {
            p->n1 = (size_t)p->k1->n;   // the wisdom fixes the split too
            p->n2 = (size_t)p->k2->n;
        } else {
            // radix / n_radix select the pass-1 schedule on this path
            const KEntry* d1 = kernel_default(kKindPass1, (int)p->n1, c1, sto);
            const int fl1 = o.flags >= 0 ? o.flags : d1 ? d1->flags : -1;
            p->k1 = (o.flags < 0 && o.n_radix == 0)
                        ? kernel_default(kKindPass1, (int)p->n1, c1, sto)
                        : kernel_find(kKindPass1, (int)p->n1, o.n_radix ? o.radix : nullptr, o.n_radix, c1, fl1);
            p->k2 = o.flags2 < 0 ? kernel_default(kKindPass2, (int)p->n2, c2, sto)
                                 : kernel_find(kKindPass2, (int)p->n2, nullptr, 0, c2, o.flags2);
        }
        if (!p->k1 || !p->k2) return FFT_ERR_UNSUPPORTED_SIZE;
        if (((p->k1->flags & FFT_VARIANT_FP16_STORAGE) != 0) != (sto != 0)) return FFT_ERR_INVALID_ARG;
        if (((p->k2->flags & FFT_VARIANT_FP16_STORAGE) != 0) != (sto != 0)) return FFT_ERR_INVALID_ARG;
        // both passes agree on the workspace form, and it is the storage's
        const bool ws = sto == FFT_STORAGE_F16_COMPACT;
        if (((p->k1->flags & FFT_VARIANT_FP16_WORKSPACE) != 0) != ws) return FFT_ERR_INVALID_ARG;
        if (((p->k2->flags & FFT_VARIANT_FP16_WORKSPACE) != 0) != ws) return FFT_ERR_INVALID_ARG;
        if (p->n2 % p->k1->c || p->n1 % p->k2->c) return FFT_ERR_UNSUPPORTED_SIZE;
        p->lo_bits = (L + 1) / 2;
        p->cw_bits = log2i(p->k2->c);
        const long long N = (long long)n;
        p->off_s1 = 0;
        off = (long long)round_up((size_t)stage_segments(p->k1, 0, p->segs), 32);
        p->off_s2 = (size_t)off;
        off = (long long)round_up((size_t)stage_segments(p->k2, off, p->segs), 32);
        p->off_hi = (size_t)off;
        p->segs.push_back({kSegHi, off, N >> p->lo_bits, N, p->lo_bits, 0, 0});
        off += (long long)round_up((size_t)(N >> p->lo_bits), 32);
        p->off_lo = (size_t)off;
        p->segs.push_back({kSegLo, off, 1LL << p->lo_bits, N, 0, 0, 0});
        off += (long long)round_up(size_t(1) << p->lo_bits, 32);
        if (p->k1->flags & FFT_VARIANT_TWIDDLE_POWERS) {
            // row col: exp(-2 pi i col T 2^i / N) for 2^i < E, T = N1 / E threads per column
            const int row = col_row(p->k1->e);
            p->off_col = (size_t)off;
            p->segs.push_back({kSegCol, off, (long long)p->n2 * row, N, (long long)p->n1 / p->k1->e, row, p->k1->e});
            off += (long long)round_up(p->n2 * (size_t)row, 32);
        }
        p->work_bytes = n * batch * work_elem(p->storage);
    }
    off = (long long)round_up((size_t)off, 32);
    p->tw_bytes = (size_t)off * sizeof(float2);
    *table_entries = (size_t)off;
    return FFT_SUCCESS;
}

static KArgs make_args(const fft_plan_s* p, int pass, const float2* in, float2* out)
{
    KArgs a{};
    a.in = in;
    a.out = out;
    a.batch = (long long)p->batch;
    a.sg = p->direction == FFT_FORWARD ? 1.0f : -1.0f;
    // the output scale: in the last store (single blocks, range compression,
    // four-step pass 2), or in pass 1 before an FP16 four-step workspace
    a.scale = p->scale;
    if (p->path == FFT_PATH_FOURSTEP) {
        const bool ws16 = p->storage == FFT_STORAGE_F16_COMPACT;
        a.scale = (ws16 == (pass == 1)) ? p->scale : 1.0f;
    }
    for (int i = 0; i < p->rt_nr; ++i) a.sched |= (unsigned)log2i(p->rt_radix[i]) << (4 * i);
    if (p->path == FFT_PATH_BLOCK || p->path == FFT_PATH_FILTER) {
        a.tw = p->tw + p->off_s1;
        if (p->path == FFT_PATH_FILTER) a.flt = p->tw + p->off_flt;
        return a;
    }
    a.nbig = (long long)p->n;
    a.lo_bits = p->lo_bits;
    a.cw_bits = p->cw_bits;
    a.tw_hi = p->tw + p->off_hi;
    a.tw_lo = p->tw + p->off_lo;
    a.tw_col = p->tw + p->off_col;
    if (pass == 1) {
        a.tw = p->tw + p->off_s1;
        a.n_other = (long long)p->n2;
        a.tiles = (int)(p->n2 / p->k1->c);
    } else {
        a.tw = p->tw + p->off_s2;
        a.n_other = (long long)p->n1;
        a.tiles = (int)(p->n1 / p->k2->c);
    }
    return a;
}

static void describe(const fft_plan_s* plan, fft_plan_desc_t* d)
{
    std::memset(d, 0, sizeof(*d));
    d->n = plan->n;
    d->batch = plan->batch;
    d->direction = plan->direction;
    d->path = plan->path;
    d->n1 = plan->n1;
    d->n2 = plan->n2;
    d->workspace_bytes = plan->work_bytes;
    d->twiddle_bytes = plan->tw_bytes;
    d->kernels_per_execute = plan->path == FFT_PATH_FOURSTEP ? 2 : 1;
    d->grid = plan->grid1;
    d->storage = plan->storage;
    d->device_twiddles = plan->device_twiddles;
    d->scale = plan->scale;
    if (!plan->k1) {
        d->kernel_name = "copy";
        return;
    }
    const KEntry* k1 = plan->path == FFT_PATH_BLOCK ? block_kernel(plan, plan->batch) : plan->k1;
    d->n_radix = k1->nr;
    for (int i = 0; i < k1->nr; ++i) d->radix[i] = k1->radix[i];
    if (plan->rt_nr > 0) {
        d->n_radix = plan->rt_nr;
        for (int i = 0; i < plan->rt_nr; ++i) d->radix[i] = plan->rt_radix[i];
    }
    d->threads_per_block = k1->threads;
    d->transforms_per_block = k1->c;
    d->lds_bytes = k1->lds;
    d->kernel_name = k1->name;
    d->flags = k1->flags;
    if (plan->k2) {
        d->n_radix2 = plan->k2->nr;
        for (int i = 0; i < plan->k2->nr; ++i) d->radix2[i] = plan->k2->radix[i];
        d->kernel_name2 = plan->k2->name;
        d->flags2 = plan->k2->flags;
        d->c2 = plan->k2->c;
    }
}

fft_status_t fft_plan_query_ex(size_t n, size_t batch, int direction, const fft_plan_opts_t* opts,
                               fft_plan_desc_t* desc)
{
    if (desc == nullptr) return FFT_ERR_INVALID_ARG;
    fft_plan_s tmp;
    size_t entries = 0;
    const fft_status_t s = plan_choose(n, batch, direction, opts, &tmp, &entries);
    if (s != FFT_SUCCESS) return s;
    describe(&tmp, desc);
    return FFT_SUCCESS;
}

fft_status_t fft_plan_query(size_t n, size_t batch, int direction, fft_plan_desc_t* desc)
{
    return fft_plan_query_ex(n, batch, direction, nullptr, desc);
}

// Workgroups of a launch: one per unit, or for persistent variants the
// resident capacity of the device (units beyond it are looped over).
static long long grid_for(const KEntry* k, const KArgs& a, int cus)
{
    const long long units = kernel_units(*k, a);
    if ((k->flags & (FFT_VARIANT_PERSISTENT | FFT_VARIANT_LOOP)) == 0) return units;
    const int occ = k->occupancy ? k->occupancy() : 0;
    const long long cap = (long long)(occ > 0 ? occ : 1) * (cus > 0 ? cus : 1);
    return units < cap ? units : cap;
}

// Device resources of a chosen plan (table of `off` entries, workspace),
// then registration.  Takes ownership of p (deleted on failure).
static fft_status_t plan_materialize(fft_plan_s* p, size_t off, fft_plan_t* plan_out)
{
    hipError_t e = hipGetDevice(&p->device);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) {
        delete p;
        return from_hip(e);
    }
    if (p->k1)
        p->grid1 = grid_for(p->path == FFT_PATH_BLOCK ? block_kernel(p, p->batch) : p->k1,
                            make_args(p, 1, nullptr, nullptr), cus);
    if (p->k2) p->grid2 = grid_for(p->k2, make_args(p, 2, nullptr, nullptr), cus);
    p->cus = cus;
    if (p->path == FFT_PATH_BLOCK && p->k1 && p->storage == 0 && (p->k1->flags & FFT_VARIANT_PERSISTENT) == 0) {
        int c = 0;
        const KEntry* t = kernel_table(&c);
        for (int i = 0; i < c && !p->klist; ++i) {
            const KEntry& k = t[i];
            if (k.kind != kKindList || k.n != p->k1->n || k.e != p->k1->e || k.c != p->k1->c ||
                k.flags != p->k1->flags || k.nr != p->k1->nr)
                continue;
            bool same = true;
            for (int r = 0; r < k.nr; ++r) same = same && k.radix[r] == p->k1->radix[r];
            if (same) p->klist = &k;
        }
    }

    if (off > 0) {
        e = hipMalloc((void**)&p->tw, p->tw_bytes);
        if (e == hipSuccess && p->device_twiddles) {
            // FP64 evaluation on the device (the only FP64 step on the GPU)
            TwSeg* dsegs = nullptr;
            e = hipMalloc((void**)&dsegs, p->segs.size() * sizeof(TwSeg));
            if (e == hipSuccess)
                e = hipMemcpy(dsegs, p->segs.data(), p->segs.size() * sizeof(TwSeg), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = generate_twiddles_device(p->tw, (long long)off, dsegs, (int)p->segs.size(), nullptr);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            if (dsegs) (void)hipFree(dsegs);
        } else if (e == hipSuccess) {
            float2* host = (float2*)std::calloc(off, sizeof(float2));
            if (!host) {
                (void)hipFree(p->tw);
                delete p;
                return FFT_ERR_OUT_OF_MEMORY;
            }
            eval_segments_host(p->segs, host);
            e = hipMemcpy(p->tw, host, p->tw_bytes, hipMemcpyHostToDevice);
            std::free(host);
        }
        if (e != hipSuccess) {
            if (p->tw) (void)hipFree(p->tw);
            delete p;
            return from_hip(e);
        }
    }
    if (p->work_bytes) {
        e = hipMalloc((void**)&p->work, p->work_bytes);
        if (e != hipSuccess) {
            (void)hipFree(p->tw);
            delete p;
            return from_hip(e);
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_plans.insert(p);
    }
    *plan_out = p;
    return FFT_SUCCESS;
}

fft_status_t fft_plan_create_ex(size_t n, size_t batch, int direction, const fft_plan_opts_t* opts,
                                fft_plan_t* plan_out)
{
    if (plan_out == nullptr) return FFT_ERR_INVALID_ARG;
    *plan_out = nullptr;
    fft_plan_s* p = new (std::nothrow) fft_plan_s();
    if (!p) return FFT_ERR_OUT_OF_MEMORY;
    size_t off = 0;
    const fft_status_t st = plan_choose(n, batch, direction, opts, p, &off);
    if (st != FFT_SUCCESS) {
        delete p;
        return st;
    }
    return plan_materialize(p, off, plan_out);
}

// Range compression plan: the kernel, its stage table, then n entries for the
// replica's spectrum (zero until the plan computes it).
static fft_status_t filter_choose(size_t n, size_t batch, size_t replica_len, const fft_plan_opts_t* opts,
                                  fft_plan_s* p, size_t* table_entries)
{
    if (n == 0 || batch == 0 || replica_len == 0 || replica_len > n) return FFT_ERR_INVALID_ARG;
    if (batch > ((size_t)1 << 40) / n) return FFT_ERR_INVALID_ARG;
    fft_plan_opts_t o;
    fft_plan_opts_init(&o);
    if (opts) o = *opts;
    if (o.storage != 0 || o.n_radix < 0 || o.n_radix > 8) return FFT_ERR_INVALID_ARG;
    if (n > kLongBlock) return FFT_ERR_UNSUPPORTED_SIZE;
    p->n = n;
    p->batch = batch;
    p->direction = FFT_FORWARD;
    p->path = FFT_PATH_FILTER;
    p->device_twiddles = o.device_twiddles ? 1 : 0;
    if (!std::isfinite(o.scale)) return FFT_ERR_INVALID_ARG;
    p->scale = o.scale == 0.0f ? 1.0f : o.scale;
    p->segs.clear();
    if (o.n_radix == 0 && o.flags < 0)
        p->k1 = kernel_default(kKindFilter, (int)n, 0, 0);
    else
        p->k1 = kernel_find(kKindFilter, (int)n, o.radix, o.n_radix, 0, o.flags);
    if (!p->k1) return FFT_ERR_UNSUPPORTED_SIZE;
    size_t off = round_up((size_t)stage_segments(p->k1, 0, p->segs), 32);
    p->off_flt = off;
    off = round_up(off + n, 32);
    p->tw_bytes = off * sizeof(float2);
    *table_entries = off;
    return FFT_SUCCESS;
}

fft_status_t fft_filter_query(size_t n, size_t batch, size_t replica_len, const fft_plan_opts_t* opts,
                              fft_plan_desc_t* desc)
{
    if (desc == nullptr) return FFT_ERR_INVALID_ARG;
    fft_plan_s tmp;
    size_t entries = 0;
    const fft_status_t s = filter_choose(n, batch, replica_len, opts, &tmp, &entries);
    if (s != FFT_SUCCESS) return s;
    describe(&tmp, desc);
    return FFT_SUCCESS;
}

fft_status_t fft_filter_create(size_t n, size_t batch, const void* replica, size_t replica_len,
                               const fft_plan_opts_t* opts, fft_plan_t* plan_out)
{
    if (plan_out == nullptr) return FFT_ERR_INVALID_ARG;
    *plan_out = nullptr;
    if (replica == nullptr || ((uintptr_t)replica & 7u)) return FFT_ERR_INVALID_ARG;
    fft_plan_s* p = new (std::nothrow) fft_plan_s();
    if (!p) return FFT_ERR_OUT_OF_MEMORY;
    size_t off = 0;
    fft_status_t st = filter_choose(n, batch, replica_len, opts, p, &off);
    if (st != FFT_SUCCESS) {
        delete p;
        return st;
    }
    fft_plan_t plan = nullptr;
    st = plan_materialize(p, off, &plan);
    if (st != FFT_SUCCESS) return st;
    // spectrum of the zero-padded replica, by this library's forward transform
    float2* spec = plan->tw + plan->off_flt;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != plan->device) e = hipSetDevice(plan->device);
    if (e == hipSuccess)
        e = hipMemcpy(spec, replica, replica_len * sizeof(float2), hipMemcpyDeviceToDevice);
    if (e != hipSuccess) st = from_hip(e);
    fft_plan_t fwd = nullptr;
    if (st == FFT_SUCCESS) st = fft_plan_create(n, 1, FFT_FORWARD, &fwd);
    if (st == FFT_SUCCESS) st = fft_execute(fwd, spec, spec, nullptr);
    if (st == FFT_SUCCESS) st = from_hip(hipDeviceSynchronize());
    if (fwd) (void)fft_plan_destroy(fwd);
    if (cur != plan->device) (void)hipSetDevice(cur);
    if (st != FFT_SUCCESS) {
        (void)fft_plan_destroy(plan);
        return st;
    }
    *plan_out = plan;
    return FFT_SUCCESS;
}

fft_status_t fft_plan_create(size_t n, size_t batch, int direction, fft_plan_t* plan_out)
{
    return fft_plan_create_ex(n, batch, direction, nullptr, plan_out);
}

fft_status_t fft_plan_destroy(fft_plan_t plan)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (plan == nullptr || g_plans.erase(plan) == 0) return FFT_ERR_INVALID_PLAN;
    }
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != plan->device) e = hipSetDevice(plan->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (plan->tw) (void)hipFree(plan->tw);
    if (plan->work) (void)hipFree(plan->work);
    if (cur != plan->device) (void)hipSetDevice(cur);
    delete plan;
    return from_hip(e);
}

fft_status_t fft_plan_twiddles(fft_plan_t plan, void* host_dst, size_t max_entries, size_t* n_entries)
{
    if (!plan_live(plan)) return FFT_ERR_INVALID_PLAN;
    if (!n_entries) return FFT_ERR_INVALID_ARG;
    const size_t cnt = plan->tw_bytes / sizeof(float2);
    *n_entries = cnt;
    if (!host_dst || cnt == 0) return FFT_SUCCESS;
    if (max_entries < cnt) return FFT_ERR_INVALID_ARG;
    return from_hip(hipMemcpy(host_dst, plan->tw, plan->tw_bytes, hipMemcpyDeviceToHost));
}

fft_status_t fft_plan_describe(fft_plan_t plan, fft_plan_desc_t* d)
{
    if (!plan_live(plan)) return FFT_ERR_INVALID_PLAN;
    if (!d) return FFT_ERR_INVALID_ARG;
    describe(plan, d);
    return FFT_SUCCESS;
}

// batch: transforms of this call (0 = the plan's); work: four-step workspace
// (nullptr = the plan's own, which then bounds batch).
static fft_status_t execute_impl(fft_plan_t plan, int passes, size_t batch, const void* in, void* out, void* work,
                                 void* stream, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    if (!plan_live(plan)) return FFT_ERR_INVALID_PLAN;
    if (in == nullptr || out == nullptr) return FFT_ERR_INVALID_ARG;
    if (!plan->storage && (((uintptr_t)in & 7u) || ((uintptr_t)out & 7u))) return FFT_ERR_INVALID_ARG;
    if (passes == 2 && plan->path != FFT_PATH_FOURSTEP) return FFT_ERR_INVALID_ARG;
    const size_t elem = plan->storage ? 4 : sizeof(float2);
    if (plan->storage && (((uintptr_t)in & 3u) || ((uintptr_t)out & 3u))) return FFT_ERR_INVALID_ARG;
    if (batch == 0) batch = plan->batch;
    if (batch > ((size_t)1 << 40) / plan->n) return FFT_ERR_INVALID_ARG;
    const size_t bytes = plan->n * batch * elem;
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if (a != b && a < b + bytes && b < a + bytes) return FFT_ERR_INVALID_ARG;
    float2* ws = plan->work;
    if (plan->path == FFT_PATH_FOURSTEP) {
        if (work) {
            const uintptr_t w = (uintptr_t)work, wb = plan->n * batch * work_elem(plan->storage);
            if (w & 7u) return FFT_ERR_INVALID_ARG;
            if ((w < a + bytes && a < w + wb) || (w < b + bytes && b < w + wb)) return FFT_ERR_INVALID_ARG;
            ws = (float2*)work;
        } else if (batch > plan->batch) {
            return FFT_ERR_INVALID_ARG;
        }
    }

    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return from_hip(e);
    if (cur != plan->device && (e = hipSetDevice(plan->device)) != hipSuccess) return from_hip(e);
    hipStream_t st = (hipStream_t)stream;
    const float2* x = (const float2*)in;
    float2* y = (float2*)out;
    const bool run1 = passes == 0 || passes == 1;
    const bool run2 = passes == 0 || passes == 2;
    const bool own = batch == plan->batch;
    auto grid = [&](const KEntry* k, const KArgs& ka, long long g) { return own ? g : grid_for(k, ka, plan->cus); };

    if (plan->path == FFT_PATH_BLOCK || plan->path == FFT_PATH_FILTER) {
        if (plan->n == 1) {
            e = (in == out) ? hipSuccess : hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, st);
        } else {
            KArgs ka = make_args(plan, 1, x, y);
            ka.batch = (long long)batch;
            const KEntry* k = plan->path == FFT_PATH_BLOCK ? block_kernel(plan, batch) : plan->k1;
            if ((k->flags & FFT_VARIANT_VEC16) != 0 && ((a | b) & 15u) != 0) {
                if (cur != plan->device) (void)hipSetDevice(cur);
                return FFT_ERR_INVALID_ARG;  // sixteen-byte lanes need 16-byte aligned data
            }
            e = k->launch(ka, grid(k, ka, plan->grid1), st, ev0, ev1);
        }
    } else {
        if (run1) {
            KArgs ka = make_args(plan, 1, x, ws);
            ka.batch = (long long)batch;
            e = plan->k1->launch(ka, grid(plan->k1, ka, plan->grid1), st, ev0, ev1);
        }
        if (e == hipSuccess && run2) {
            KArgs ka = make_args(plan, 2, ws, y);
            ka.batch = (long long)batch;
            e = plan->k2->launch(ka, grid(plan->k2, ka, plan->grid2), st, ev0, ev1);
        }
    }
    if (cur != plan->device) (void)hipSetDevice(cur);
    return from_hip(e);
}

fft_status_t fft_execute(fft_plan_t plan, const void* in, void* out, void* stream)
{
    return execute_impl(plan, 0, 0, in, out, nullptr, stream);
}

fft_status_t fft_execute_pass_timed(fft_plan_t plan, int pass, const void* in, void* out, void* stream,
                                    void* start_event, void* stop_event)
{
    if (pass != 1 && pass != 2) return plan_live(plan) ? FFT_ERR_INVALID_ARG : FFT_ERR_INVALID_PLAN;
    if (!start_event || !stop_event) return FFT_ERR_INVALID_ARG;
    return execute_impl(plan, pass, 0, in, out, nullptr, stream, (hipEvent_t)start_event, (hipEvent_t)stop_event);
}

fft_status_t fft_event_create(void** event)
{
    if (!event) return FFT_ERR_INVALID_ARG;
    *event = nullptr;
    hipEvent_t e = nullptr;
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return from_hip(r);
    *event = e;
    return FFT_SUCCESS;
}

fft_status_t fft_event_destroy(void* event)
{
    if (!event) return FFT_ERR_INVALID_ARG;
    return from_hip(hipEventDestroy((hipEvent_t)event));
}

fft_status_t fft_event_elapsed(void* start_event, void* stop_event, float* ms)
{
    if (!start_event || !stop_event || !ms) return FFT_ERR_INVALID_ARG;
    hipError_t r = hipEventSynchronize((hipEvent_t)stop_event);
    if (r == hipSuccess) r = hipEventElapsedTime(ms, (hipEvent_t)start_event, (hipEvent_t)stop_event);
    return from_hip(r);
}

fft_status_t fft_execute_ex(fft_plan_t plan, size_t batch, const void* in, void* out, void* workspace, void* stream)
{
    return execute_impl(plan, 0, batch, in, out, workspace, stream);
}

}  // extern "C"

namespace fb {

hipError_t plan_launch_list(fft_plan_s* plan, const void* list, long long transforms, hipStream_t st)
{
    if (!plan->klist || transforms <= 0) return hipErrorNotSupported;
    KArgs ka = make_args(plan, 1, nullptr, nullptr);
    ka.batch = transforms;
    ka.list = list;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != plan->device) e = hipSetDevice(plan->device);
    if (e == hipSuccess) e = plan->klist->launch(ka, kernel_units(*plan->klist, ka), st, nullptr, nullptr);
    if (cur != plan->device) (void)hipSetDevice(cur);
    return e;
}

bool plan_launch_params(const fft_plan_s* p, int pass, const void* in, void* out, const KEntry** k, KArgs* a,
                        long long* grid)
{
    if (p->path == FFT_PATH_FOURSTEP) {
        if (pass == 1) {
            *k = p->k1;
            *a = make_args(p, 1, static_cast<const float2*>(in), p->work);
            *grid = p->grid1;
        } else if (pass == 2) {
            *k = p->k2;
            *a = make_args(p, 2, p->work, static_cast<float2*>(out));
            *grid = p->grid2;
        } else {
            return false;
        }
        return *k != nullptr;
    }
    if (pass != 1 || p->n == 1 || !p->k1) return false;
    *k = block_kernel(p, p->batch);
    *a = make_args(p, 1, static_cast<const float2*>(in), static_cast<float2*>(out));
    *grid = p->grid1;
    return true;
}

void plan_shape(const fft_plan_s* plan, size_t* n, int* direction, int* path, bool* has_list)
{
    *n = plan->n;
    *direction = plan->direction;
    *path = plan->path;
    *has_list = plan->klist != nullptr;
}

}  // namespace fb

extern "C" {

fft_status_t fft_execute_pass(fft_plan_t plan, int pass, const void* in, void* out, void* stream)
{
    if (pass != 1 && pass != 2) return plan_live(plan) ? FFT_ERR_INVALID_ARG : FFT_ERR_INVALID_PLAN;
    return execute_impl(plan, pass, 0, in, out, nullptr, stream);
}

fft_status_t fft_transpose(const void* in, void* out, size_t rows, size_t cols, size_t batch, void* stream)
{
    if (in == nullptr || out == nullptr || rows == 0 || cols == 0 || batch == 0) return FFT_ERR_INVALID_ARG;
    if (((uintptr_t)in & 7u) || ((uintptr_t)out & 7u)) return FFT_ERR_INVALID_ARG;
    if (rows > ((size_t)1 << 32) || cols > ((size_t)1 << 32) || batch > ((size_t)1 << 32))
        return FFT_ERR_INVALID_ARG;
    const size_t bytes = rows * cols * batch * sizeof(float2);
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if (a < b + bytes && b < a + bytes) return FFT_ERR_INVALID_ARG;
    return from_hip(launch_transpose((const float2*)in, (float2*)out, (long long)rows, (long long)cols,
                                     (long long)batch, (hipStream_t)stream));
}

fft_status_t fft_copy(const void* in, void* out, size_t bytes, void* stream)
{
    if (in == nullptr || out == nullptr || bytes == 0 || (bytes & 15u)) return FFT_ERR_INVALID_ARG;
    if (((uintptr_t)in & 15u) || ((uintptr_t)out & 15u)) return FFT_ERR_INVALID_ARG;
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if (a < b + bytes && b < a + bytes) return FFT_ERR_INVALID_ARG;
    return from_hip(launch_copy(in, out, bytes, (hipStream_t)stream));
}

}  // extern "C"

// ------------------------------------------------ allocation-free execute
// The four-step workspace of fft_execute_static: one fixed array in the code
// object, so the call allocates nothing.  Each GPU the library runs on holds
// its own copy (64 MiB, zero at module load) until the process ends; in host
// code the name `scratch` is only a stand-in, so the device address of each
// copy is looked up once per device and kept.
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) float2 scratch[kScratchBytes / sizeof(float2)];

std::mutex g_scratch_mu;
std::vector<std::pair<int, float2*>> g_scratch_at;  // (device, address of its copy)

// Address of the calling thread's current device's copy of `scratch`.
hipError_t scratch_address(int device, float2** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    for (const auto& d : g_scratch_at)
        if (d.first == device) {
            *out = d.second;
            return hipSuccess;
        }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_at.emplace_back(device, static_cast<float2*>(p));
    *out = static_cast<float2*>(p);
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t fft_static_scratch_bytes(void) { return kScratchBytes; }

fft_status_t fft_execute_static(fft_plan_t plan, size_t batch, const void* in, void* out, void* stream)
{
    if (!plan_live(plan)) return FFT_ERR_INVALID_PLAN;
    if (in == nullptr || out == nullptr) return FFT_ERR_INVALID_ARG;
    if (plan->path != FFT_PATH_FOURSTEP) return execute_impl(plan, 0, batch, in, out, nullptr, stream);
    const size_t b = batch ? batch : plan->batch;
    if (b > kScratchBytes / work_elem(plan->storage) / plan->n) return FFT_ERR_SCRATCH_LIMIT;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return from_hip(e);
    if (cur != plan->device && (e = hipSetDevice(plan->device)) != hipSuccess) return from_hip(e);
    float2* ws = nullptr;
    e = scratch_address(plan->device, &ws);
    if (cur != plan->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return from_hip(e);
    return execute_impl(plan, 0, b, in, out, ws, stream);
}

fft_status_t fft_device_query(int device, fft_device_info_t* info)
{
    if (info == nullptr) return FFT_ERR_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    hipError_t e = hipSuccess;
    if (device < 0) e = hipGetDevice(&device);
    if (e != hipSuccess) return from_hip(e);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return from_hip(e);
    info->device = device;
    std::strncpy(info->arch, prop.gcnArchName, sizeof(info->arch) - 1);
    info->compute_units = prop.multiProcessorCount;
    info->warp_size = prop.warpSize;
    info->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
    info->lds_per_block = prop.sharedMemPerBlock;
    info->global_mem = prop.totalGlobalMem;
    info->clock_khz = prop.clockRate;
    info->mem_clock_khz = prop.memoryClockRate;
    info->mem_bus_width = prop.memoryBusWidth;
    for (int i = 0; i < 3; ++i) info->block_max[i] = fft_block_max(info->lds_per_cu, 1 << i);
    return FFT_SUCCESS;
}

}  // extern "C"
