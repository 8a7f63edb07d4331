// Ragged batches: transforms of several lengths in one submission.
//
// A ragged plan holds one ordinary plan per length class (each uses the
// wisdom the autotuner recorded, so radix, block size and workgroup shape are
// the measured best for that length).  The first execute with a given
// (in, out) pair captures every class's kernels into one hipGraph whose
// classes hang off a fork event on up to four parallel branches, so the
// device may overlap classes; every later execute with the same buffers is a
// single hipGraphLaunch.  Data layout: the classes' batches are concatenated
// in the order given, class c starting at element offset
// sum_{j<c} sizes[j] * counts[j].
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "../../include/fftblock.h"
#include "internal.hpp"

struct fft_ragged_s {
    int direction = FFT_FORWARD;
    size_t elem = 8;  // bytes per value: 8 (complex64) or 4 (FP16 pairs)
    int device = 0;
    std::vector<size_t> sizes, counts, offsets;
    size_t total_points = 0;
    std::vector<fft_plan_t> plans;
    std::vector<hipStream_t> branches;
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    const void* g_in = nullptr;
    void* g_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t graph_nodes = 0;
};

namespace {

std::mutex g_rmu;
std::unordered_set<fft_ragged_s*> g_ragged;

bool live(fft_ragged_s* r)
{
    std::lock_guard<std::mutex> lk(g_rmu);
    return r && g_ragged.count(r);
}

fft_status_t st_of(hipError_t e)
{
    return e == hipSuccess ? FFT_SUCCESS : e == hipErrorOutOfMemory ? FFT_ERR_OUT_OF_MEMORY : FFT_ERR_DEVICE;
}

void release(fft_ragged_s* r)
{
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    for (fft_plan_t p : r->plans)
        if (p) fft_plan_destroy(p);
    for (hipStream_t s : r->branches)
        if (s) (void)hipStreamDestroy(s);
    if (r->cap) (void)hipStreamDestroy(r->cap);
    if (r->fork) (void)hipEventDestroy(r->fork);
    for (hipEvent_t e : r->joins)
        if (e) (void)hipEventDestroy(e);
    delete r;
}

// Record every class's launches into a graph for (in, out).
fft_status_t capture(fft_ragged_s* r, const void* in, void* out)
{
    if (r->exec) {
        (void)hipGraphExecDestroy(r->exec);
        r->exec = nullptr;
    }
    if (r->graph) {
        (void)hipGraphDestroy(r->graph);
        r->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return st_of(e);
    fft_status_t st = FFT_SUCCESS;
    e = hipEventRecord(r->fork, r->cap);
    const size_t nb = r->branches.size();
    for (size_t b = 0; b < nb && e == hipSuccess; ++b) e = hipStreamWaitEvent(r->branches[b], r->fork, 0);
    for (size_t c = 0; c < r->plans.size() && e == hipSuccess && st == FFT_SUCCESS; ++c) {
        const char* x = (const char*)in + r->offsets[c] * r->elem;
        char* y = (char*)out + r->offsets[c] * r->elem;
        st = fft_execute(r->plans[c], x, y, r->branches[c % nb]);
    }
    for (size_t b = 0; b < nb && e == hipSuccess; ++b) {
        e = hipEventRecord(r->joins[b], r->branches[b]);
        if (e == hipSuccess) e = hipStreamWaitEvent(r->cap, r->joins[b], 0);
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(r->cap, &g);
    if (e == hipSuccess) e = e2;
    if (st != FFT_SUCCESS || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != FFT_SUCCESS ? st : st_of(e);
    }
    r->graph = g;
    e = hipGraphInstantiate(&r->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return st_of(e);
    size_t nodes = 0;
    (void)hipGraphGetNodes(g, nullptr, &nodes);
    r->graph_nodes = nodes;
    r->g_in = in;
    r->g_out = out;
    return FFT_SUCCESS;
}

}  // namespace

extern "C" {

fft_status_t fft_ragged_create(const size_t* sizes, const size_t* counts, size_t n_classes, int direction,
                               fft_ragged_t* out)
{
    return fft_ragged_create_ex(sizes, counts, n_classes, direction, nullptr, out);
}

fft_status_t fft_ragged_create_ex(const size_t* sizes, const size_t* counts, size_t n_classes, int direction,
                                  const fft_plan_opts_t* opts, fft_ragged_t* out)
{
    if (!out) return FFT_ERR_INVALID_ARG;
    *out = nullptr;
    if (!sizes || !counts || n_classes == 0 || n_classes > 4096) return FFT_ERR_INVALID_ARG;
    if (direction != FFT_FORWARD && direction != FFT_BACKWARD) return FFT_ERR_INVALID_ARG;
    size_t total = 0;
    // only the storage form and the twiddle source apply to a ragged plan
    fft_plan_opts_t po;
    fft_plan_opts_init(&po);
    if (opts) {
        po.storage = opts->storage;
        po.device_twiddles = opts->device_twiddles;
    }
    for (size_t c = 0; c < n_classes; ++c) {
        if (counts[c] == 0 || sizes[c] == 0) return FFT_ERR_INVALID_ARG;
        fft_plan_desc_t d;
        const fft_status_t st = fft_plan_query_ex(sizes[c], counts[c], direction, &po, &d);
        if (st != FFT_SUCCESS) return st;
        if (sizes[c] > ((size_t)1 << 40) / counts[c] || total > ((size_t)1 << 40)) return FFT_ERR_INVALID_ARG;
        total += sizes[c] * counts[c];
    }
    fft_ragged_s* r = new (std::nothrow) fft_ragged_s();
    if (!r) return FFT_ERR_OUT_OF_MEMORY;
    r->direction = direction;
    r->elem = po.storage ? 4 : 8;
    r->total_points = total;
    size_t at = 0;
    for (size_t c = 0; c < n_classes; ++c) {
        r->sizes.push_back(sizes[c]);
        r->counts.push_back(counts[c]);
        r->offsets.push_back(at);
        at += sizes[c] * counts[c];
    }
    hipError_t e = hipGetDevice(&r->device);
    for (size_t c = 0; c < n_classes && e == hipSuccess; ++c) {
        fft_plan_t p = nullptr;
        const fft_status_t st = opts ? fft_plan_create_ex(sizes[c], counts[c], direction, &po, &p)
                                     : fft_plan_create(sizes[c], counts[c], direction, &p);
        if (st != FFT_SUCCESS) {
            release(r);
            return st;
        }
        r->plans.push_back(p);
    }
    const size_t nb = n_classes < 4 ? n_classes : 4;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking);
    for (size_t b = 0; b < nb && e == hipSuccess; ++b) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) r->branches.push_back(s);
        hipEvent_t j = nullptr;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        if (e == hipSuccess) r->joins.push_back(j);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        release(r);
        return st_of(e);
    }
    {
        std::lock_guard<std::mutex> lk(g_rmu);
        g_ragged.insert(r);
    }
    *out = r;
    return FFT_SUCCESS;
}

fft_status_t fft_ragged_execute(fft_ragged_t r, const void* in, void* out, void* stream, int mode)
{
    if (!live(r)) return FFT_ERR_INVALID_PLAN;
    if (!in || !out || (mode != 0 && mode != 1)) return FFT_ERR_INVALID_ARG;
    if (((uintptr_t)in & (r->elem - 1)) || ((uintptr_t)out & (r->elem - 1))) return FFT_ERR_INVALID_ARG;
    const size_t bytes = r->total_points * r->elem;
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if (a != b && a < b + bytes && b < a + bytes) return FFT_ERR_INVALID_ARG;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return st_of(e);
    if (cur != r->device && (e = hipSetDevice(r->device)) != hipSuccess) return st_of(e);
    fft_status_t st = FFT_SUCCESS;
    if (mode == 1) {
        // plain path: every class launched in order on the caller's stream
        for (size_t c = 0; c < r->plans.size() && st == FFT_SUCCESS; ++c)
            st = fft_execute(r->plans[c], (const char*)in + r->offsets[c] * r->elem,
                             (char*)out + r->offsets[c] * r->elem, stream);
    } else {
        if (!r->exec || r->g_in != in || r->g_out != out) st = capture(r, in, out);
        if (st == FFT_SUCCESS) st = st_of(hipGraphLaunch(r->exec, (hipStream_t)stream));
    }
    if (cur != r->device) (void)hipSetDevice(cur);
    return st;
}

fft_status_t fft_ragged_describe(fft_ragged_t r, size_t* total_points, size_t* graph_nodes)
{
    if (!live(r)) return FFT_ERR_INVALID_PLAN;
    if (total_points) *total_points = r->total_points;
    if (graph_nodes) *graph_nodes = r->graph_nodes;
    return FFT_SUCCESS;
}

fft_status_t fft_ragged_destroy(fft_ragged_t r)
{
    {
        std::lock_guard<std::mutex> lk(g_rmu);
        if (!r || g_ragged.erase(r) == 0) return FFT_ERR_INVALID_PLAN;
    }
    int cur = 0;
    const int dev = r->device;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    release(r);
    if (cur != dev) (void)hipSetDevice(cur);
    return st_of(e);
}

}  // extern "C"
