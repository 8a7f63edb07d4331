// Host side of the C ABI declared in include/fftblock.h: argument checks,
// the planner (block limit, path, radix schedule, four-step split), FP64
// twiddle generation, plan lifetime and launches.
//
// Planner (paper, Approach): the largest transform one compute unit holds is
// derived from the local-memory size -- on gfx950 the LDS, 160 KB per CU --
// as pow2floor(LDS / (8 B * (1 + 1/16) * k)) for k resident workgroups; the
// runtime sweep then confirms which single-block lengths actually win
// ("a mix of analytic approach and runtime validation").  Lengths up to the
// limit run as one block per transform; longer power-of-two lengths run the
// four-step split N = N1 * N2 with N1 >= N2, both powers of two.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_set>

#include "../../include/fftblock.h"
#include "internal.hpp"

using namespace fb;

struct fft_plan_s {
    size_t n = 0, batch = 0;
    int direction = FFT_FORWARD;
    int path = 0;
    int device = 0;
    const BlockEntry* blk = nullptr;
    const TileEntry* p1 = nullptr;
    const TileEntry* p2 = nullptr;
    size_t n1 = 0, n2 = 0;
    int lo_bits = 0;
    float2* tw = nullptr;           // one allocation holding every table
    size_t tw_bytes = 0;
    size_t off_s1 = 0, off_s2 = 0, off_hi = 0, off_lo = 0;  // in complex entries
    float2* work = nullptr;
    size_t work_bytes = 0;
};

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

// Stage twiddle rows of a radix schedule: for stage s >= 1 with radix R and
// Ns points already combined, row k < Ns holds exp(-2 pi i r k / (Ns R)), r < R.
void fill_stage_table(const int* radix, int nr, float2* dst)
{
    size_t at = 0;
    long long ns = radix[0];
    for (int s = 1; s < nr; ++s) {
        const int R = radix[s];
        for (long long k = 0; k < ns; ++k)
            for (int r = 0; r < R; ++r) dst[at++] = root_f32((long long)r * k, ns * R);
        ns *= R;
    }
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
constexpr size_t kDefaultBlockLimit = 16384;

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

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
    }
    return "unknown status";
}

size_t fft_block_limit(void)
{
    size_t lim = env_size("FFTBLOCK_BLOCK_MAX", kDefaultBlockLimit);
    if (!is_pow2(lim) || lim < 1024) lim = kDefaultBlockLimit;
    if (lim > kDefaultBlockLimit) lim = kDefaultBlockLimit;
    return lim;
}

// Pure host planning: path, kernels, four-step split and table layout.
// Makes no HIP call, so it is usable (and testable) without a device.
static fft_status_t plan_choose(size_t n, size_t batch, int direction, fft_plan_s* p, size_t* table_entries)
{
    if (n == 0 || batch == 0) return FFT_ERR_INVALID_ARG;
    if (direction != FFT_FORWARD && direction != FFT_BACKWARD) return FFT_ERR_INVALID_ARG;
    if (!is_pow2(n) || n > kMaxN) return FFT_ERR_UNSUPPORTED_SIZE;
    if (batch > ((size_t)1 << 40) / n) return FFT_ERR_INVALID_ARG;
    p->n = n;
    p->batch = batch;
    p->direction = direction;
    const size_t limit = fft_block_limit();
    size_t off = 0;
    if (n == 1) {
        p->path = FFT_PATH_BLOCK;
    } else if (n <= limit) {
        p->path = FFT_PATH_BLOCK;
        p->blk = block_default((int)n);
        if (!p->blk) return FFT_ERR_UNSUPPORTED_SIZE;
        p->off_s1 = 0;
        off = round_up((size_t)p->blk->tw_size, 32);
    } else {
        p->path = FFT_PATH_FOURSTEP;
        const int L = ilog2(n);
        p->n1 = size_t(1) << ((L + 1) / 2);
        p->n2 = n / p->n1;
        const int c = (int)env_size("FFTBLOCK_FOURSTEP_C", 0);
        p->p1 = tile_find(1, (int)p->n1, c);
        p->p2 = tile_find(2, (int)p->n2, c);
        if (!p->p1) p->p1 = tile_find(1, (int)p->n1, 0);
        if (!p->p2) p->p2 = tile_find(2, (int)p->n2, 0);
        if (!p->p1 || !p->p2 || p->n2 % p->p1->c || p->n1 % p->p2->c) return FFT_ERR_UNSUPPORTED_SIZE;
        p->lo_bits = (L + 1) / 2;
        p->off_s1 = 0;
        off = round_up((size_t)p->p1->tw_size, 32);
        p->off_s2 = off;
        off += round_up((size_t)p->p2->tw_size, 32);
        p->off_hi = off;
        off += round_up(n >> p->lo_bits, 32);
        p->off_lo = off;
        off += round_up(size_t(1) << p->lo_bits, 32);
        p->work_bytes = n * batch * sizeof(float2);
    }
    p->tw_bytes = off * sizeof(float2);
    *table_entries = off;
    return FFT_SUCCESS;
}

static void describe(const fft_plan_s* plan, fft_plan_desc_t* d);

fft_status_t fft_plan_query(size_t n, size_t batch, int direction, fft_plan_desc_t* desc)
{
    if (desc == nullptr) return FFT_ERR_INVALID_ARG;
    fft_plan_s tmp;
    size_t entries = 0;
    const fft_status_t s = plan_choose(n, batch, direction, &tmp, &entries);
    if (s != FFT_SUCCESS) return s;
    describe(&tmp, desc);
    return FFT_SUCCESS;
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

fft_status_t fft_plan_create(size_t n, size_t batch, int direction, fft_plan_t* plan_out)
{
    if (plan_out == nullptr) return FFT_ERR_INVALID_ARG;
    *plan_out = nullptr;
    fft_plan_s* p = new (std::nothrow) fft_plan_s();
    if (!p) return FFT_ERR_OUT_OF_MEMORY;
    size_t off = 0;
    const fft_status_t st = plan_choose(n, batch, direction, p, &off);
    if (st != FFT_SUCCESS) { delete p; return st; }

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { delete p; return from_hip(e); }

    if (off > 0) {
        float2* host = (float2*)std::calloc(off, sizeof(float2));
        if (!host) { delete p; return FFT_ERR_OUT_OF_MEMORY; }
        if (p->path == FFT_PATH_BLOCK) {
            fill_stage_table(p->blk->radix, p->blk->nr, host + p->off_s1);
        } else {
            fill_stage_table(p->p1->radix, p->p1->nr, host + p->off_s1);
            fill_stage_table(p->p2->radix, p->p2->nr, host + p->off_s2);
            const long long N = (long long)n;
            for (long long a = 0; a < (N >> p->lo_bits); ++a) host[p->off_hi + a] = root_f32(a << p->lo_bits, N);
            for (long long b = 0; b < (1LL << p->lo_bits); ++b) host[p->off_lo + b] = root_f32(b, N);
        }
        p->tw_bytes = off * sizeof(float2);
        e = hipMalloc((void**)&p->tw, p->tw_bytes);
        if (e == hipSuccess) e = hipMemcpy(p->tw, host, p->tw_bytes, hipMemcpyHostToDevice);
        std::free(host);
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
    if (plan->path == FFT_PATH_BLOCK) {
        d->kernels_per_execute = 1;
        if (plan->blk) {
            d->n_radix = plan->blk->nr;
            for (int i = 0; i < plan->blk->nr; ++i) d->radix[i] = plan->blk->radix[i];
            d->threads_per_block = plan->blk->threads;
            d->transforms_per_block = plan->blk->fpb;
            d->lds_bytes = plan->blk->lds;
            d->kernel_name = plan->blk->name;
        } else {
            d->kernel_name = "copy";
        }
    } else {
        d->kernels_per_execute = 2;
        d->n_radix = plan->p1->nr;
        for (int i = 0; i < plan->p1->nr; ++i) d->radix[i] = plan->p1->radix[i];
        d->n_radix2 = plan->p2->nr;
        for (int i = 0; i < plan->p2->nr; ++i) d->radix2[i] = plan->p2->radix[i];
        d->threads_per_block = plan->p1->threads;
        d->transforms_per_block = plan->p1->c;
        d->lds_bytes = plan->p1->lds;
        d->kernel_name = plan->p1->name;
        d->kernel_name2 = plan->p2->name;
    }
}

fft_status_t fft_plan_describe(fft_plan_t plan, fft_plan_desc_t* d)
{
    if (!plan_live(plan)) return FFT_ERR_INVALID_PLAN;
    if (!d) return FFT_ERR_INVALID_ARG;
    describe(plan, d);
    return FFT_SUCCESS;
}

static fft_status_t execute_impl(fft_plan_t plan, int passes, const void* in, void* out, void* stream)
{
    if (!plan_live(plan)) return FFT_ERR_INVALID_PLAN;
    if (in == nullptr || out == nullptr) return FFT_ERR_INVALID_ARG;
    if (((uintptr_t)in & 7u) || ((uintptr_t)out & 7u)) return FFT_ERR_INVALID_ARG;
    if (passes == 2 && plan->path != FFT_PATH_FOURSTEP) return FFT_ERR_INVALID_ARG;
    const size_t bytes = plan->n * plan->batch * sizeof(float2);
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if (a != b && a < b + bytes && b < a + bytes) return FFT_ERR_INVALID_ARG;

    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return from_hip(e);
    if (cur != plan->device && (e = hipSetDevice(plan->device)) != hipSuccess) return from_hip(e);
    hipStream_t st = (hipStream_t)stream;
    const float sg = plan->direction == FFT_FORWARD ? 1.0f : -1.0f;
    const float2* x = (const float2*)in;
    float2* y = (float2*)out;
    const bool run1 = passes == 0 || passes == 1;
    const bool run2 = passes == 0 || passes == 2;

    if (plan->path == FFT_PATH_BLOCK) {
        if (plan->n == 1) {
            e = (in == out) ? hipSuccess : hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, st);
        } else {
            e = plan->blk->launch(x, y, plan->tw + plan->off_s1, (long long)plan->batch, sg, st);
        }
    } else {
        FourStepArgs a1{};
        a1.batch = (long long)plan->batch;
        a1.nbig = (long long)plan->n;
        a1.n_other = (long long)plan->n2;
        a1.tiles = (int)(plan->n2 / plan->p1->c);
        a1.lo_bits = plan->lo_bits;
        a1.tw_hi = plan->tw + plan->off_hi;
        a1.tw_lo = plan->tw + plan->off_lo;
        a1.sg = sg;
        if (run1) e = plan->p1->launch(x, plan->work, plan->tw + plan->off_s1, a1, st);
        if (e == hipSuccess && run2) {
            FourStepArgs a2 = a1;
            a2.n_other = (long long)plan->n1;
            a2.tiles = (int)(plan->n1 / plan->p2->c);
            e = plan->p2->launch(plan->work, y, plan->tw + plan->off_s2, a2, st);
        }
    }
    if (cur != plan->device) (void)hipSetDevice(cur);
    return from_hip(e);
}

fft_status_t fft_execute(fft_plan_t plan, const void* in, void* out, void* stream)
{
    return execute_impl(plan, 0, in, out, stream);
}

fft_status_t fft_execute_pass(fft_plan_t plan, int pass, const void* in, void* out, void* stream)
{
    if (pass != 1 && pass != 2) return plan_live(plan) ? FFT_ERR_INVALID_ARG : FFT_ERR_INVALID_PLAN;
    return execute_impl(plan, pass, in, out, stream);
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
