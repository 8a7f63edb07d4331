// Schedule search after the paper's performance model (Approach, bottom-level
// analysis, "FFT performance model"), plus runtime validation and wisdom.
//
// * Stage microbenchmarks: the cost of one radix-R Stockham stage starting at
//   stage index s (Ns = 2^s points already combined) on an LDS-resident
//   N-point transform, measured on the GPU as the difference between a kernel
//   that repeats the stage `reps` times and one that does not, per stage and
//   transform.
// * The stage DAG: states 0..log2 N, a radix-R edge from s to s + log2 R
//   weighted by its measured cost; under the paper's hypothesis (a stage's cost
//   depends only on its radix and start stage) the best schedule is the
//   shortest source-to-sink path, found with Dijkstra's algorithm.
// * Runtime validation: every compiled kernel for N is timed as a whole (the
//   hypothesis does not hold exactly once stages are fused into one kernel);
//   the fastest becomes the wisdom entry the planner uses for N.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "../../include/fftblock.h"
#include "fft_device.hpp"
#include "internal.hpp"

namespace fb {

// ------------------------------------------------------------ stage kernel
// One workgroup per transform, T = N/16 threads, 16 values per thread.  The
// transform is loaded into LDS once; then `reps` times: every thread reads the
// inputs of its 16/R butterflies (Stockham positions j + r N/R), applies the
// stage twiddles w^(r (j mod Ns)) from power rows, runs the R-point DFT and
// writes the outputs back ((j/Ns) Ns R + j mod Ns + q Ns).  The result is
// stored so the work cannot be removed.
template <int R>
__global__ void __launch_bounds__(1024) k_stage(float2* __restrict__ data, const float2* __restrict__ pw, int n, int ns,
                                                int reps)
{
    extern __shared__ float2 sh[];
    constexpr int E = 16;
    constexpr int P = (R - 1) >= 16 ? 5 : (R - 1) >= 8 ? 4 : (R - 1) >= 4 ? 3 : (R - 1) >= 2 ? 2 : 1;
    constexpr int ROW = (P + 1) & ~1;
    const int T = n / E;
    const int t = threadIdx.x;
    float2* x = data + (long long)blockIdx.x * n;
    for (int i = t; i < n; i += T) sh[i + (i >> 4)] = x[i];
    __syncthreads();
    float2 v[E];
    for (int rep = 0; rep < reps; ++rep) {
#pragma unroll
        for (int b = 0; b < E / R; ++b) {
            const int j = t + b * T;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = j + r * (n / R);
                v[b * R + r] = sh[i + (i >> 4)];
            }
            apply_pow_row<R>(&v[b * R], pw + (long long)(j % ns) * ROW);
            Dft<R>::run(&v[b * R]);
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < E / R; ++b) {
            const int j = t + b * T;
            const int base = (j / ns) * ns * R + (j % ns);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int i = base + q * ns;
                sh[i + (i >> 4)] = v[b * R + q];
            }
        }
        __syncthreads();
    }
    for (int i = t; i < n; i += T) x[i] = sh[i + (i >> 4)];
}

using StageFn = void (*)(float2*, const float2*, int, int, int);

static StageFn stage_fn(int radix)
{
    switch (radix) {
        case 2: return k_stage<2>;
        case 4: return k_stage<4>;
        case 8: return k_stage<8>;
        case 16: return k_stage<16>;
        default: return nullptr;
    }
}

// ---------------------------------------------------------------- wisdom
struct Wisdom {
    std::mutex mu;
    std::map<size_t, std::pair<std::string, std::string>> choice;  // length -> (block or pass-1, pass-2)
};
// Timing inputs: values in [-1, 1) from a counter-based hash of the index
// (the transforms' time depends on the data: on all-zero inputs some kernels
// run several per cent faster than on the signals they tune for).
__global__ void __launch_bounds__(256) k_fill_tuning(float* p, long long n, unsigned seed)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        unsigned h = (unsigned)i * 0x9E3779B1u ^ (unsigned)(i >> 32) ^ seed;
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        h *= 0xC2B2AE35u;
        h ^= h >> 16;
        p[i] = (float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f;
    }
}

static hipError_t fill_tuning(float2* x, size_t values, unsigned seed)
{
    const long long nf = (long long)values * 2;
    const long long blocks = std::min<long long>((nf + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_tuning, dim3((unsigned)blocks), dim3(256), 0, nullptr, reinterpret_cast<float*>(x), nf,
                       seed);
    return hipGetLastError();
}

static Wisdom& wisdom()
{
    static Wisdom w;
    return w;
}

// Wisdom applies to complex64 plans: FP16-storage kernels are never chosen.
static bool wisdom_eligible(const KEntry& k) { return (k.flags & FFT_VARIANT_FP16_STORAGE) == 0; }

// A block choice is a kernel name, followed for the run-time-schedule kernel
// by ':' and its schedule ("block_fft_rt<1024>:16,16,4").  Splits it; false
// for a malformed schedule (radices 2, 4, 8, 16 whose product is n).
static bool split_choice(const std::string& s, size_t n, std::string* name, std::vector<int>* sched)
{
    sched->clear();
    const size_t colon = s.find(':');
    *name = s.substr(0, colon);
    if (colon == std::string::npos) return true;
    size_t prod = 1, at = colon + 1;
    while (at <= s.size()) {
        const size_t comma = s.find(',', at);
        const std::string tok = s.substr(at, comma == std::string::npos ? std::string::npos : comma - at);
        const int R = std::atoi(tok.c_str());
        if (R != 2 && R != 4 && R != 8 && R != 16) return false;
        sched->push_back(R);
        prod *= (size_t)R;
        if (comma == std::string::npos) break;
        at = comma + 1;
    }
    return !sched->empty() && sched->size() <= 8 && prod == n;
}

static const KEntry* find_named(int kind, size_t n, const std::string& choice, std::vector<int>* sched = nullptr)
{
    std::string name;
    std::vector<int> sc;
    if (!split_choice(choice, n, &name, &sc)) return nullptr;
    int c = 0;
    const KEntry* t = kernel_table(&c);
    for (int i = 0; i < c; ++i)
        if (t[i].kind == kind && (size_t)t[i].n == n && name == t[i].name && wisdom_eligible(t[i])) {
            // the run-time-schedule kernel needs its schedule, the others none
            if (((t[i].flags & FFT_VARIANT_RUNTIME_SCHEDULE) != 0) != !sc.empty()) return nullptr;
            if (sched) *sched = sc;
            return &t[i];
        }
    return nullptr;
}

static void load_env_wisdom()
{
    static std::once_flag env_once;
    std::call_once(env_once, [] {
        const char* path = std::getenv("FFTBLOCK_WISDOM");
        if (path && *path) (void)fft_wisdom_load(path);
    });
}

const KEntry* wisdom_kernel(size_t n, int* radix, int* nr)
{
    load_env_wisdom();
    Wisdom& w = wisdom();
    std::string name;
    {
        std::lock_guard<std::mutex> lk(w.mu);
        auto it = w.choice.find(n);
        if (it == w.choice.end() || !it->second.second.empty()) return nullptr;
        name = it->second.first;
    }
    std::vector<int> sc;
    const KEntry* k = find_named(kKindBlock, n, name, &sc);
    if (nr) *nr = (int)sc.size();
    for (size_t i = 0; radix && i < sc.size(); ++i) radix[i] = sc[i];
    return k;
}

bool wisdom_pair(size_t n, const KEntry** k1, const KEntry** k2)
{
    load_env_wisdom();
    Wisdom& w = wisdom();
    std::pair<std::string, std::string> names;
    {
        std::lock_guard<std::mutex> lk(w.mu);
        auto it = w.choice.find(n);
        if (it == w.choice.end() || it->second.second.empty()) return false;
        names = it->second;
    }
    int c = 0;
    const KEntry* t = kernel_table(&c);
    *k1 = *k2 = nullptr;
    for (int i = 0; i < c; ++i) {
        if (t[i].kind == kKindPass1 && names.first == t[i].name && wisdom_eligible(t[i])) *k1 = &t[i];
        if (t[i].kind == kKindPass2 && names.second == t[i].name && wisdom_eligible(t[i])) *k2 = &t[i];
    }
    return *k1 && *k2 && (size_t)(*k1)->n * (size_t)(*k2)->n == n;
}

}  // namespace fb

using namespace fb;

extern "C" {

fft_status_t fft_schedule_search(int log2n, const int* radices, int n_radices, const double* costs, int* sched_out,
                                 int* n_sched_out, double* total_out)
{
    if (log2n < 1 || log2n > 30 || !radices || n_radices < 1 || n_radices > 8 || !costs || !sched_out ||
        !n_sched_out)
        return FFT_ERR_INVALID_ARG;
    std::vector<int> step(n_radices);
    for (int i = 0; i < n_radices; ++i) {
        int l = 0;
        while ((1 << l) < radices[i]) ++l;
        if (radices[i] < 2 || (1 << l) != radices[i]) return FFT_ERR_INVALID_ARG;
        step[i] = l;
    }
    // label: (cost, stages, radix list negated for "larger list wins ties")
    struct Label {
        double cost;
        int stages;
        std::vector<int> neg;
        bool operator>(const Label& o) const
        {
            if (cost != o.cost) return cost > o.cost;
            if (stages != o.stages) return stages > o.stages;
            return neg > o.neg;
        }
    };
    std::vector<bool> have(log2n + 1, false), done(log2n + 1, false);
    std::vector<Label> best(log2n + 1);
    using Item = std::pair<Label, int>;
    auto cmp = [](const Item& a, const Item& b) { return a.first > b.first; };
    std::priority_queue<Item, std::vector<Item>, decltype(cmp)> pq(cmp);
    best[0] = Label{0.0, 0, {}};
    have[0] = true;
    pq.push({best[0], 0});
    while (!pq.empty()) {
        const Item it = pq.top();
        pq.pop();
        const int node = it.second;
        if (done[node]) continue;
        done[node] = true;
        if (node == log2n) break;
        for (int i = 0; i < n_radices; ++i) {
            const int nxt = node + step[i];
            if (nxt > log2n) continue;
            const double c = costs[i * log2n + node];
            if (!(c >= 0.0) || std::isinf(c)) continue;  // absent edge
            Label cand = it.first;
            cand.cost += c;
            cand.stages += 1;
            cand.neg.push_back(-radices[i]);
            if (!have[nxt] || best[nxt] > cand) {
                best[nxt] = cand;
                have[nxt] = true;
                pq.push({cand, nxt});
            }
        }
    }
    if (!have[log2n]) return FFT_ERR_UNSUPPORTED_SIZE;
    const Label& b = best[log2n];
    for (size_t i = 0; i < b.neg.size(); ++i) sched_out[i] = -b.neg[i];
    *n_sched_out = (int)b.neg.size();
    if (total_out) *total_out = b.cost;
    return FFT_SUCCESS;
}

fft_status_t fft_stage_benchmark(size_t n, int radix, int start_stage, int reps, double* ns_per_stage)
{
    if (!ns_per_stage || reps < 1 || n < 256 || n > 16384 || (n & (n - 1)) || start_stage < 0) return FFT_ERR_INVALID_ARG;
    StageFn fn = stage_fn(radix);
    if (!fn) return FFT_ERR_INVALID_ARG;
    int lg = 0, lr = 0;
    while (((size_t)1 << lg) < n) ++lg;
    while ((1 << lr) < radix) ++lr;
    if (start_stage + lr > lg) return FFT_ERR_INVALID_ARG;
    const int ns = 1 << start_stage;
    const int P = (radix - 1) >= 16 ? 5 : (radix - 1) >= 8 ? 4 : (radix - 1) >= 4 ? 3 : (radix - 1) >= 2 ? 2 : 1;
    const int row = (P + 1) & ~1;
    std::vector<float2> pw((size_t)ns * row, make_float2(0.f, 0.f));
    for (int k = 0; k < ns; ++k)
        for (int i = 0; i < P; ++i) pw[(size_t)k * row + i] = root_f32((long long)k << i, (long long)ns * radix);
    const size_t batch = std::max<size_t>((size_t)1 << 22, n) / n;
    float2 *d = nullptr, *dpw = nullptr;
    hipError_t e = hipMalloc(&d, batch * n * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&dpw, pw.size() * sizeof(float2));
    if (e == hipSuccess) e = hipMemcpy(dpw, pw.data(), pw.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = fill_tuning(d, batch * n, 0x57A6Eu);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const size_t shmem = (n + n / 16) * sizeof(float2);
    const int threads = (int)(n / 16);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    float ms_base = 0.f, ms_reps = 0.f;
    for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {  // pass 0 warms up
        for (int which = 0; which < 2 && e == hipSuccess; ++which) {
            const int r = which == 0 ? 0 : reps;
            e = hipEventRecord(e0, nullptr);
            hipLaunchKernelGGL(fn, dim3((unsigned)batch), dim3(threads), shmem, nullptr, d, dpw, (int)n, ns, r);
            if (e == hipSuccess) e = hipGetLastError();
            if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (pass > 0) (which == 0 ? ms_base : ms_reps) += ms;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d) (void)hipFree(d);
    if (dpw) (void)hipFree(dpw);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_OUT_OF_MEMORY : FFT_ERR_DEVICE;
    const double per = ((double)ms_reps - (double)ms_base) / 2.0 * 1e6 / ((double)reps * (double)batch);
    *ns_per_stage = per > 0 ? per : 0.0;
    return FFT_SUCCESS;
}

fft_status_t fft_autotune(size_t n, size_t batch, fft_tune_report_t* rep)
{
    if (!rep || n < 2 || batch < 1) return FFT_ERR_INVALID_ARG;
    std::memset(rep, 0, sizeof(*rep));
    rep->n = n;
    rep->chosen_kernel = -1;
    rep->chosen_kernel2 = -1;
    rep->predicted_us = -1.0;
    rep->chosen_schedule_rt_us = -1.0;
    int lg = 0;
    while (((size_t)1 << lg) < n) ++lg;
    const bool pow2 = ((size_t)1 << lg) == n;
    rep->log2n = pow2 ? lg : 0;
    for (int i = 0; i < 4; ++i)
        for (int s = 0; s < 16; ++s) rep->stage_cost[i][s] = -1.0;
    // 1) the paper's model: stage costs, DAG, Dijkstra (power-of-two lengths)
    static const int kRad[4] = {2, 4, 8, 16};
    if (pow2 && n >= 256 && n <= 16384) {
        for (int i = 0; i < 4; ++i) {
            int lr = 0;
            while ((1 << lr) < kRad[i]) ++lr;
            for (int s = 0; s + lr <= lg; ++s) {
                double c = -1.0;
                const fft_status_t st = fft_stage_benchmark(n, kRad[i], s, 8, &c);
                if (st != FFT_SUCCESS) return st;
                rep->stage_cost[i][s] = c;
            }
        }
        std::vector<double> costs(4 * lg, -1.0);
        for (int i = 0; i < 4; ++i)
            for (int s = 0; s < lg; ++s) costs[i * lg + s] = rep->stage_cost[i][s];
        int ns = 0;
        if (fft_schedule_search(lg, kRad, 4, costs.data(), rep->predicted, &ns, &rep->predicted_cost) == FFT_SUCCESS)
            rep->n_predicted = ns;
    }
    // 2) runtime validation: every compiled block kernel for n, timed whole
    int count = 0;
    const KEntry* t = kernel_table(&count);
    // Rotating (in, out) sets, up to 512 MiB on each side: the transforms
    // this tunes for stream their data from HBM, and one pair re-used
    // launch after launch would sit in the 256 MB Infinity Cache and favour
    // variants that win only on cached data.
    const size_t bytes = n * batch * sizeof(float2);
    const int nsets = (int)std::min<size_t>(8, std::max<size_t>(1, ((size_t)512 << 20) / bytes));
    std::vector<float2*> xs(nsets, nullptr), ys(nsets, nullptr);
    hipError_t e = hipSuccess;
    for (int k = 0; k < nsets && e == hipSuccess; ++k) {
        e = hipMalloc(&xs[k], bytes);
        if (e == hipSuccess) e = hipMalloc(&ys[k], bytes);
        if (e == hipSuccess) e = fill_tuning(xs[k], n * batch, 0x5EEDu + (unsigned)k);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best = 1e300;
    auto time_plan = [&](fft_plan_t p) -> double {
        for (int w = 0; w < nsets; ++w) fft_execute(p, xs[w], ys[w], nullptr);
        const int reps = 16;
        e = hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            if (fft_execute(p, xs[r % nsets], ys[r % nsets], nullptr) != FFT_SUCCESS) e = hipErrorUnknown;
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        return (double)ms * 1e3 / reps;
    };
    // Candidates are timed in interleaved rounds (every candidate once per
    // round) and ranked by their median round: kernels within a few per cent
    // of each other would otherwise be ranked by the drift of the clocks
    // between one timing and the next.
    constexpr int kRounds = 5;
    struct Cand {
        fft_plan_t p;
        int i, j;
        double t[kRounds];
    };
    std::vector<Cand> cands;
    auto median_of = [](double* v, int m) {
        std::sort(v, v + m);
        return v[m / 2];
    };
    fft_plan_desc_t dq;
    const bool four = fft_plan_query(n, batch, FFT_FORWARD, &dq) == FFT_SUCCESS && dq.path == FFT_PATH_FOURSTEP;
    if (four) {
        // the default split with every pass-1 x pass-2 pair (schedules,
        // column/row widths, variants), then the neighbouring splits with
        // their default passes
        const size_t d1 = dq.n1;
        const size_t splits[3] = {d1, d1 / 2, d1 * 2};
        for (int sp = 0; sp < 3; ++sp) {
        const size_t n1 = splits[sp], n2 = n / n1;
        if (n1 < 2 || n2 < 2 || n1 * n2 != n) continue;
        for (int i = 0; i < count && e == hipSuccess; ++i) {
            if (t[i].kind != kKindPass1 || (size_t)t[i].n != n1 || n2 % t[i].c || !wisdom_eligible(t[i])) continue;
            if (sp > 0 && !t[i].is_default) continue;
            for (int j = 0; j < count && e == hipSuccess && rep->n_candidates < (sp == 0 ? 28 : 32); ++j) {
                if (t[j].kind != kKindPass2 || (size_t)t[j].n != n2 || n1 % t[j].c || !wisdom_eligible(t[j])) continue;
                if (sp > 0 && !t[j].is_default) continue;
                fft_plan_opts_t o;
                fft_plan_opts_init(&o);
                // a length the single block could take (a small batch put it
                // on this path) stays four-step under explicit kernel options
                if (n <= kMaxBlockLen) o.block_limit = std::max<size_t>(1024, n / 2);
                o.n1 = n1;
                o.n_radix = t[i].nr;
                for (int r = 0; r < t[i].nr; ++r) o.radix[r] = t[i].radix[r];
                o.flags = t[i].flags;
                o.c = t[i].c;
                o.flags2 = t[j].flags;
                o.c2 = t[j].c;
                fft_plan_t p = nullptr;
                if (fft_plan_create_ex(n, batch, FFT_FORWARD, &o, &p) != FFT_SUCCESS) continue;
                fft_plan_desc_t d;
                fft_plan_describe(p, &d);
                const bool same = std::strcmp(d.kernel_name, t[i].name) == 0 && std::strcmp(d.kernel_name2, t[j].name) == 0;
                if (!same) {
                    fft_plan_destroy(p);
                    continue;
                }
                cands.push_back({p, i, j, {}});
                rep->n_candidates++;
            }
        }
        }
    }
    for (int i = 0; i < count && e == hipSuccess && rep->n_candidates < 32 && !four; ++i) {
        if (t[i].kind != kKindBlock || (size_t)t[i].n != n || !wisdom_eligible(t[i]) ||
            (t[i].flags & FFT_VARIANT_RUNTIME_SCHEDULE) != 0)
            continue;
        fft_plan_opts_t o;
        fft_plan_opts_init(&o);
        o.n_radix = t[i].nr;
        for (int r = 0; r < t[i].nr; ++r) o.radix[r] = t[i].radix[r];
        o.flags = t[i].flags;
        o.c = t[i].c;
        o.block_limit = kMaxBlockLen;
        fft_plan_t p = nullptr;
        fft_status_t st = fft_plan_create_ex(n, batch, FFT_FORWARD, &o, &p);
        if (st != FFT_SUCCESS) continue;
        fft_plan_desc_t d;
        fft_plan_describe(p, &d);
        if (std::strcmp(d.kernel_name, t[i].name) != 0) {
            fft_plan_destroy(p);
            continue;
        }
        cands.push_back({p, i, -1, {}});
        rep->n_candidates++;
    }
    for (int r = 0; r < kRounds && e == hipSuccess; ++r)
        for (Cand& c : cands) c.t[r] = time_plan(c.p);
    for (size_t k = 0; k < cands.size(); ++k) {
        Cand& c = cands[k];
        const double us = e == hipSuccess ? median_of(c.t, kRounds) : -1.0;
        fft_plan_destroy(c.p);
        rep->candidate_kernel[k] = c.i;
        rep->candidate_kernel2[k] = c.j;
        rep->candidate_us[k] = us;
        if (e == hipSuccess && us < best) {
            best = us;
            rep->chosen_kernel = c.i;
            rep->chosen_kernel2 = c.j;
            rep->chosen_us = us;
        }
    }
    // 3) the model's own choice, run: the predicted schedule on the
    // run-time-schedule kernel, and the fastest compiled schedule on the same
    // kernel (the two schedules compared on one code path); the predicted
    // schedule becomes the wisdom when it beats every compiled kernel
    int rt_index = -1;
    for (int i = 0; i < count; ++i)
        if (t[i].kind == kKindBlock && (size_t)t[i].n == n && (t[i].flags & FFT_VARIANT_RUNTIME_SCHEDULE) != 0)
            rt_index = i;
    if (!four && rep->n_predicted > 0 && rt_index >= 0 && e == hipSuccess) {
        auto time_rt = [&](const int* sched, int nr) -> double {
            fft_plan_opts_t o;
            fft_plan_opts_init(&o);
            o.n_radix = nr;
            for (int r = 0; r < nr; ++r) o.radix[r] = sched[r];
            o.flags = t[rt_index].flags;
            o.block_limit = kMaxBlockLen;
            fft_plan_t p = nullptr;
            if (fft_plan_create_ex(n, batch, FFT_FORWARD, &o, &p) != FFT_SUCCESS) return -1.0;
            double ts[kRounds];
            for (int r = 0; r < kRounds; ++r) ts[r] = time_plan(p);
            fft_plan_destroy(p);
            return median_of(ts, kRounds);
        };
        rep->predicted_us = time_rt(rep->predicted, rep->n_predicted);
        const KEntry* ck = rep->chosen_kernel >= 0 ? &t[rep->chosen_kernel] : nullptr;
        bool rt_ok = ck && ck->nr > 0;
        for (int r = 0; rt_ok && r < ck->nr; ++r)
            rt_ok = ck->radix[r] == 2 || ck->radix[r] == 4 || ck->radix[r] == 8 || ck->radix[r] == 16;
        if (rt_ok && e == hipSuccess) rep->chosen_schedule_rt_us = time_rt(ck->radix, ck->nr);
        if (e == hipSuccess && rep->predicted_us > 0.0 && rep->predicted_us < best) {
            best = rep->predicted_us;
            rep->chosen_kernel = rt_index;
            rep->chosen_kernel2 = -1;
            rep->chosen_us = rep->predicted_us;
            rep->chosen_predicted = 1;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (int k = 0; k < nsets; ++k) {
        if (xs[k]) (void)hipFree(xs[k]);
        if (ys[k]) (void)hipFree(ys[k]);
    }
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? FFT_ERR_OUT_OF_MEMORY : FFT_ERR_DEVICE;
    if (rep->chosen_kernel < 0) return FFT_ERR_UNSUPPORTED_SIZE;
    {
        std::string name = t[rep->chosen_kernel].name;
        if (rep->chosen_predicted) {
            name += ':';
            for (int r = 0; r < rep->n_predicted; ++r) name += (r ? "," : "") + std::to_string(rep->predicted[r]);
        }
        Wisdom& w = wisdom();
        std::lock_guard<std::mutex> lk(w.mu);
        w.choice[n] = {name, rep->chosen_kernel2 >= 0 ? t[rep->chosen_kernel2].name : ""};
    }
    return FFT_SUCCESS;
}

fft_status_t fft_wisdom_set(size_t n, int kernel_index)
{
    int c = 0;
    const KEntry* t = kernel_table(&c);
    if (kernel_index < 0 || kernel_index >= c || t[kernel_index].kind != kKindBlock || (size_t)t[kernel_index].n != n ||
        !wisdom_eligible(t[kernel_index]) || (t[kernel_index].flags & FFT_VARIANT_RUNTIME_SCHEDULE) != 0)
        return FFT_ERR_INVALID_ARG;
    Wisdom& w = wisdom();
    std::lock_guard<std::mutex> lk(w.mu);
    w.choice[n] = {t[kernel_index].name, ""};
    return FFT_SUCCESS;
}

void fft_wisdom_clear(void)
{
    Wisdom& w = wisdom();
    std::lock_guard<std::mutex> lk(w.mu);
    w.choice.clear();
}

int fft_wisdom_get(size_t n)
{
    const KEntry* k = wisdom_kernel(n, nullptr, nullptr);
    if (!k) return -1;
    int c = 0;
    const KEntry* t = kernel_table(&c);
    return (int)(k - t);
}

fft_status_t fft_wisdom_save(const char* path)
{
    if (!path) return FFT_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "w");
    if (!f) return FFT_ERR_INVALID_ARG;
    Wisdom& w = wisdom();
    std::lock_guard<std::mutex> lk(w.mu);
    std::fprintf(f, "# fftblock wisdom: length kernel [pass-2 kernel, tab separated]\n");
    for (const auto& kv : w.choice)
        std::fprintf(f, "%zu\t%s\t%s\n", kv.first, kv.second.first.c_str(), kv.second.second.c_str());
    std::fclose(f);
    return FFT_SUCCESS;
}

fft_status_t fft_wisdom_load(const char* path)
{
    if (!path) return FFT_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "r");
    if (!f) return FFT_ERR_INVALID_ARG;
    char line[512];
    int c = 0;
    const KEntry* t = kernel_table(&c);
    fft_status_t st = FFT_SUCCESS;
    Wisdom& w = wisdom();
    std::lock_guard<std::mutex> lk(w.mu);
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        // "length<TAB>name[<TAB>name2]" (a space also separates length and name)
        char* end = nullptr;
        const size_t n = std::strtoull(line, &end, 10);
        if (end == line) {
            st = FFT_ERR_INVALID_ARG;
            continue;
        }
        while (*end == ' ' || *end == '\t') ++end;
        std::string rest(end);
        while (!rest.empty() && (rest.back() == '\n' || rest.back() == '\r')) rest.pop_back();
        std::string a = rest, b;
        const size_t tab = rest.find('\t');
        if (tab != std::string::npos) {
            a = rest.substr(0, tab);
            b = rest.substr(tab + 1);
        }
        bool known = false;
        if (b.empty()) {
            known = find_named(kKindBlock, n, a) != nullptr;
        } else {
            bool k1 = false, k2 = false;
            for (int i = 0; i < c; ++i) {
                k1 = k1 || (t[i].kind == kKindPass1 && a == t[i].name && wisdom_eligible(t[i]));
                k2 = k2 || (t[i].kind == kKindPass2 && b == t[i].name && wisdom_eligible(t[i]));
            }
            known = k1 && k2;
        }
        if (!known) {
            st = FFT_ERR_INVALID_ARG;  // stale entry (kernel no longer compiled): skipped
            continue;
        }
        w.choice[n] = {a, b};
    }
    std::fclose(f);
    return st;
}

}  // extern "C"
