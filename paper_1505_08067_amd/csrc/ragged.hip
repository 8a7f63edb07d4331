// Ragged batches: transforms of several lengths in one submission.
//
// Default form (mode 0): persistent kernels over a device work list (paper,
// Approach, "Top level analysis": independent FFT tasks mapped onto the
// compute units).  Each length class is matched to a case of a persistent
// kernel of the catalogue (kernels_ragged.hip); the classes of one kernel
// become one launch whose workgroups (as many as are resident) take the
// classes' work units from one queue, largest units first.  A four-step
// length puts its pass-1 units in one launch and its pass-2 units in a later
// one, so the launch boundary orders the two passes.  The launches are the
// kernel nodes of one hipGraph, built once; when a later execute passes other
// buffers only the nodes' arguments are updated (no re-capture).  A class no
// persistent case covers runs its own plan's kernels as extra nodes.
//
// Each class has an ordinary plan built with exactly its case's kernel, which
// holds the case's twiddle table (and, four-step, its workspace).  Mode 1
// runs the classes' default plans (the autotuner's wisdom) one after another
// on the caller's stream; mode 2 replays a graph of those plans' kernels on
// four parallel branches (the per-length form, kept for comparison).
//
// Data layout: the classes' batches concatenated in the order given, class c
// starting at element offset sum_{j<c} sizes[j] * counts[j].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "../../include/fftblock.h"
#include "internal.hpp"
#include "ragged_kernel.hpp"

namespace {

struct RagLaunch {
    const fb::RKEntry* k = nullptr;
    std::vector<fb::RagEnt> ents;  // host copy; in / out as offsets (rel)
    unsigned units = 0, grid = 0, nstatic = 0;
    fb::RagEnt* d_ents = nullptr;
    unsigned* d_ctr = nullptr;
    bool has_pass1 = false, has_pass2 = false;
};

// Length-1 classes are the identity: a copy of their words (in == out allowed:
// every word is read and written back by the same thread).
__global__ void __launch_bounds__(256) k_identity(const unsigned* in, unsigned* out, long long words)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < words; i += (long long)gridDim.x * 256)
        out[i] = in[i];
}

struct IdArgs {
    const unsigned* in;
    unsigned* out;
    long long words;
};

// A kernel node of the mode-0 graph and the arguments it was last given.
struct Node {
    hipGraphNode_t node = nullptr;
    int launch = -1;         // persistent launch index, or -1: a plain kernel (or a copy)
    int cls = -1, pass = 0;  // plain kernel: class and pass (pass 0: length 1, a copy)
    fb::RagArgs rargs{};
    fb::KArgs kargs{};
    IdArgs ida{};
    void* argp[3] = {nullptr, nullptr, nullptr};
};

}  // namespace

struct fft_ragged_s {
    int direction = FFT_FORWARD;
    size_t elem = 8;  // bytes per value: 8 (complex64) or 4 (FP16 pairs)
    int storage = 0, device_twiddles = 0;
    int device = 0;
    std::vector<size_t> sizes, counts, offsets;
    size_t total_points = 0;
    std::vector<fft_plan_t> case_plans;   // per class: the plan of its persistent case (or fallback)
    std::vector<fft_plan_t> plain_plans;  // per class: default plans (modes 1 and 2), made on first use
    std::vector<RagLaunch> launches;
    std::vector<int> fallback;            // classes with no persistent case
    char* dmem = nullptr;                 // work lists and counters
    // mode 0 graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Node> nodes;
    const void* g_in = nullptr;
    void* g_out = nullptr;
    hipEvent_t done = nullptr;  // recorded after every graph launch
    bool launched = false;
    // mode 2 graph (per-class kernels on branches)
    std::vector<hipStream_t> branches;
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    hipGraph_t graph2 = nullptr;
    hipGraphExec_t exec2 = nullptr;
    const void* g2_in = nullptr;
    void* g2_out = nullptr;
    size_t graph2_nodes = 0;
};

namespace {

using namespace fb;

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
    if (r->exec2) (void)hipGraphExecDestroy(r->exec2);
    if (r->graph2) (void)hipGraphDestroy(r->graph2);
    for (fft_plan_t p : r->case_plans)
        if (p) fft_plan_destroy(p);
    for (fft_plan_t p : r->plain_plans)
        if (p) fft_plan_destroy(p);
    if (r->dmem) (void)hipFree(r->dmem);
    if (r->done) (void)hipEventDestroy(r->done);
    for (hipStream_t s : r->branches)
        if (s) (void)hipStreamDestroy(s);
    if (r->cap) (void)hipStreamDestroy(r->cap);
    if (r->fork) (void)hipEventDestroy(r->fork);
    for (hipEvent_t e : r->joins)
        if (e) (void)hipEventDestroy(e);
    delete r;
}

bool case_storage(const RKCase& c, int storage) { return ((c.flags & FFT_VARIANT_FP16_STORAGE) != 0) == (storage != 0); }

// Persistent kernel and case of kernel kind `kind` at length n (storage st).
const RKEntry* find_case(int kind, size_t n, int st, int* cs)
{
    int cnt = 0;
    const RKEntry* t = ragged_entries(&cnt);
    for (int i = 0; i < cnt; ++i) {
        for (int j = 0; j < t[i].ncase; ++j) {
            const RKCase& c = t[i].cases[j];
            if (c.kind == kind && (size_t)c.n == n && case_storage(c, st)) {
                *cs = j;
                return &t[i];
            }
        }
    }
    return nullptr;
}

void case_opts(const RKCase& c, fft_plan_opts_t* o)
{
    o->n_radix = c.nr;
    for (int i = 0; i < c.nr && i < 8; ++i) o->radix[i] = c.radix[i];
    o->flags = c.flags;
    o->c = c.c;
}

// Host planning: every class's case, plan and entry; launches grouped by
// kernel, pass-1 launches first, entries largest units first.
fft_status_t plan_classes(fft_ragged_s* r)
{
    struct Item {
        const RKEntry* k;
        RagEnt e;
        double unit_bytes;
        long long units;
        int pass;  // 0 block, 1 / 2 four-step pass
    };
    std::vector<Item> items;
    for (size_t c = 0; c < r->sizes.size(); ++c) {
        const size_t n = r->sizes[c], cnt = r->counts[c];
        fft_plan_opts_t o;
        fft_plan_opts_init(&o);
        o.storage = r->storage;
        o.device_twiddles = r->device_twiddles;
        int cs = -1, cs1 = -1, cs2 = -1;
        const RKEntry* kb = find_case(kKindBlock, n, r->storage, &cs);
        const RKEntry *k1 = nullptr, *k2 = nullptr;
        if (!kb) {
            // four-step: pass 1 at n1 and pass 2 at n / n1, in two different kernels
            int nk = 0;
            const RKEntry* t = ragged_entries(&nk);
            for (int i = 0; i < nk && !k1; ++i)
                for (int j = 0; j < t[i].ncase && !k1; ++j) {
                    const RKCase& a = t[i].cases[j];
                    if (a.kind != kKindPass1 || !case_storage(a, r->storage)) continue;
                    if (n % (size_t)a.n || n / (size_t)a.n < 2) continue;
                    int j2 = -1;
                    const RKEntry* q = find_case(kKindPass2, n / (size_t)a.n, r->storage, &j2);
                    if (q && q != &t[i]) {
                        k1 = &t[i];
                        cs1 = j;
                        k2 = q;
                        cs2 = j2;
                    }
                }
        }
        fft_plan_t p = nullptr;
        fft_status_t st;
        if (kb) {
            case_opts(kb->cases[cs], &o);
            o.block_limit = kMaxBlockLen;
            st = fft_plan_create_ex(n, cnt, r->direction, &o, &p);
        } else if (k1) {
            const RKCase &a1 = k1->cases[cs1], &a2 = k2->cases[cs2];
            case_opts(a1, &o);
            o.n1 = (size_t)a1.n;
            o.flags2 = a2.flags;
            o.c2 = a2.c;
            o.block_limit = 1024;  // below n: the four-step path
            st = fft_plan_create_ex(n, cnt, r->direction, &o, &p);
        } else {
            // no persistent case: the class's default plan runs as its own nodes
            st = fft_plan_create_ex(n, cnt, r->direction, &o, &p);
        }
        if (st != FFT_SUCCESS) return st;
        r->case_plans.push_back(p);
        if (!kb && !k1) {
            r->fallback.push_back((int)c);
            continue;
        }
        const size_t off = r->offsets[c] * r->elem;
        for (int pass = 1; pass <= (kb ? 1 : 2); ++pass) {
            const KEntry* ke = nullptr;
            KArgs a{};
            long long grid = 0;
            // in / out as byte offsets into the ragged buffers; the four-step
            // workspace between the passes stays an absolute address
            if (!plan_launch_params(p, pass, reinterpret_cast<const void*>(off), reinterpret_cast<void*>(off), &ke, &a,
                                    &grid))
                return FFT_ERR_DEVICE;
            const RKEntry* k = kb ? kb : pass == 1 ? k1 : k2;
            const int cse = kb ? cs : pass == 1 ? cs1 : cs2;
            const RKCase& rc = k->cases[cse];
            bool same = ke->n == rc.n && ke->e == rc.e && ke->c == rc.c && ke->flags == rc.flags &&
                        ke->kind == rc.kind && ke->nr == rc.nr;
            for (int i = 0; same && i < rc.nr; ++i) same = ke->radix[i] == rc.radix[i];
            if (!same) return FFT_ERR_DEVICE;  // the plan did not take the case's kernel
            Item it;
            it.k = k;
            it.e.a = a;
            it.e.cs = cse;
            it.e.rel = kb ? 3 : pass == 1 ? 1 : 2;
            it.e.u0 = 0;
            it.units = kernel_units(*ke, a);
            it.unit_bytes = (double)ke->n * ke->c * 16.0;
            it.pass = kb ? 0 : pass;
            items.push_back(it);
        }
    }
    // within a launch, the largest units first
    std::stable_sort(items.begin(), items.end(),
                     [](const Item& a, const Item& b) { return a.unit_bytes > b.unit_bytes; });
    for (const Item& it : items) {
        RagLaunch* L = nullptr;
        for (RagLaunch& q : r->launches)
            if (q.k == it.k && q.ents.size() < (size_t)kRagMaxEnt) L = &q;
        if (!L) {
            r->launches.emplace_back();
            L = &r->launches.back();
            L->k = it.k;
        }
        RagEnt e = it.e;
        e.u0 = (long long)L->units;
        if ((long long)L->units + it.units >= (1LL << 31)) return FFT_ERR_INVALID_ARG;
        L->units += (unsigned)it.units;
        L->ents.push_back(e);
        if (it.pass == 1) L->has_pass1 = true;
        if (it.pass == 2) L->has_pass2 = true;
    }
    // launches holding pass 1 of a four-step class run first; one launch
    // cannot hold both passes (nothing would order them)
    for (const RagLaunch& L : r->launches)
        if (L.has_pass1 && L.has_pass2) return FFT_ERR_UNSUPPORTED_SIZE;
    std::stable_sort(r->launches.begin(), r->launches.end(),
                     [](const RagLaunch& a, const RagLaunch& b) { return a.has_pass1 && !b.has_pass1; });
    return FFT_SUCCESS;
}

// Share of a launch's units dealt round-robin before the queue takes over
// (FFTBLOCK_RAGGED_STATIC overrides it, in percent).  Measured on the
// 2^28-point mix: 1110 us with 75 %, 1126 with 90 %, 1211 with none (all
// queued).
constexpr size_t kStaticPct = 75;

size_t env_pct(const char* name, size_t dflt)
{
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    char* end = nullptr;
    const unsigned long x = std::strtoul(v, &end, 10);
    return (end && *end == 0) ? (size_t)x : dflt;
}

// Device memory: every launch's work list and its two counters (zero).
fft_status_t materialize(fft_ragged_s* r)
{
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, r->device);
    if (e != hipSuccess) return st_of(e);
    size_t bytes = 0;
    for (const RagLaunch& L : r->launches) bytes += (L.ents.size() * sizeof(RagEnt) + 255) & ~(size_t)255;
    const size_t ctr_off = bytes;
    bytes += r->launches.size() * 256;
    if (bytes == 0) return FFT_SUCCESS;
    e = hipMalloc((void**)&r->dmem, bytes);
    if (e == hipSuccess) e = hipMemset(r->dmem + ctr_off, 0, r->launches.size() * 256);
    size_t at = 0;
    for (size_t i = 0; i < r->launches.size() && e == hipSuccess; ++i) {
        RagLaunch& L = r->launches[i];
        L.d_ents = reinterpret_cast<RagEnt*>(r->dmem + at);
        e = hipMemcpy(L.d_ents, L.ents.data(), L.ents.size() * sizeof(RagEnt), hipMemcpyHostToDevice);
        at += (L.ents.size() * sizeof(RagEnt) + 255) & ~(size_t)255;
        L.d_ctr = reinterpret_cast<unsigned*>(r->dmem + ctr_off + i * 256);
        const int occ = L.k->occupancy ? L.k->occupancy() : 0;
        if (occ <= 0) return FFT_ERR_DEVICE;
        const unsigned slots = (unsigned)occ * (unsigned)(cus > 0 ? cus : 1);
        L.grid = std::min(L.units, slots);
        // a head of whole rounds is dealt round-robin, the rest queued
        const unsigned pct = (unsigned)std::min<size_t>(env_pct("FFTBLOCK_RAGGED_STATIC", kStaticPct), 100);
        L.nstatic = (unsigned)((unsigned long long)L.units * pct / 100 / L.grid * L.grid);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return st_of(e);
}

// Kernel-node parameters of node nd for the buffers (in, out).
bool node_params(fft_ragged_s* r, Node& nd, const void* in, void* out, hipKernelNodeParams* p)
{
    std::memset(p, 0, sizeof(*p));
    if (nd.launch >= 0) {
        const RagLaunch& L = r->launches[(size_t)nd.launch];
        nd.rargs.ent = L.d_ents;
        nd.rargs.nent = (int)L.ents.size();
        nd.rargs.units = L.units;
        nd.rargs.nstatic = L.nstatic;
        nd.rargs.ctr = L.d_ctr;
        for (int j = 0; j < kRagMaxEnt; ++j)
            nd.rargs.u0[j] = j < nd.rargs.nent ? (unsigned)L.ents[(size_t)j].u0 : L.units;
        nd.rargs.in = static_cast<const char*>(in);
        nd.rargs.out = static_cast<char*>(out);
        nd.argp[0] = &nd.rargs;
        p->func = const_cast<void*>(L.k->fn);
        p->gridDim = dim3(L.grid);
        p->blockDim = dim3((unsigned)L.k->threads);
    } else if (nd.pass == 0) {
        const size_t off = r->offsets[(size_t)nd.cls] * r->elem;
        nd.ida.in = reinterpret_cast<const unsigned*>(static_cast<const char*>(in) + off);
        nd.ida.out = reinterpret_cast<unsigned*>(static_cast<char*>(out) + off);
        nd.ida.words = (long long)(r->counts[(size_t)nd.cls] * r->elem / 4);
        nd.argp[0] = &nd.ida.in;
        nd.argp[1] = &nd.ida.out;
        nd.argp[2] = &nd.ida.words;
        p->func = reinterpret_cast<void*>(&k_identity);
        p->gridDim = dim3((unsigned)std::min<long long>((nd.ida.words + 255) / 256, 1024));
        p->blockDim = dim3(256);
    } else {
        const size_t off = r->offsets[(size_t)nd.cls] * r->elem;
        const KEntry* k = nullptr;
        long long grid = 0;
        if (!plan_launch_params(r->case_plans[(size_t)nd.cls], nd.pass, static_cast<const char*>(in) + off,
                                static_cast<char*>(out) + off, &k, &nd.kargs, &grid) ||
            grid <= 0 || grid > 0x7fffffffLL)
            return false;
        nd.argp[0] = &nd.kargs;
        p->func = const_cast<void*>(k->fn);
        p->gridDim = dim3((unsigned)grid);
        p->blockDim = dim3((unsigned)k->threads);
    }
    p->sharedMemBytes = 0;
    p->kernelParams = nd.argp;
    p->extra = nullptr;
    return true;
}

// The mode-0 graph: the persistent launches in sequence, then each fallback
// class's kernels, also in sequence (pass 2 after pass 1).  A persistent
// launch fills every resident slot, so a kernel beside it would only take
// slots from it (measured: 1059 us with the fallback kernels on branches of
// their own against the sequence).
fft_status_t build_graph(fft_ragged_s* r, const void* in, void* out)
{
    hipError_t e = hipGraphCreate(&r->graph, 0);
    if (e != hipSuccess) return st_of(e);
    r->nodes.clear();
    for (size_t i = 0; i < r->launches.size(); ++i) {
        Node nd;
        nd.launch = (int)i;
        r->nodes.push_back(nd);
    }
    for (int c : r->fallback) {
        size_t n = 0;
        int dir = 0, path = 0;
        bool list = false;
        plan_shape(r->case_plans[(size_t)c], &n, &dir, &path, &list);
        if (n == 1) {
            Node nd;
            nd.cls = c;
            nd.pass = 0;  // the identity: a copy kernel
            r->nodes.push_back(nd);
            continue;
        }
        for (int pass = 1; pass <= (path == FFT_PATH_FOURSTEP ? 2 : 1); ++pass) {
            Node nd;
            nd.cls = c;
            nd.pass = pass;
            r->nodes.push_back(nd);
        }
    }
    hipGraphNode_t prev = nullptr;
    for (size_t i = 0; i < r->nodes.size(); ++i) {
        Node& nd = r->nodes[i];
        hipKernelNodeParams p;
        if (!node_params(r, nd, in, out, &p)) return FFT_ERR_DEVICE;
        hipGraphNode_t dep = prev;  // every node after the one before it
        e = hipGraphAddKernelNode(&nd.node, r->graph, dep ? &dep : nullptr, dep ? 1 : 0, &p);
        if (e != hipSuccess) return st_of(e);
        prev = nd.node;
    }
    e = hipGraphInstantiate(&r->exec, r->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return st_of(e);
    r->g_in = in;
    r->g_out = out;
    return FFT_SUCCESS;
}

// New buffers: update every node's arguments in the executable graph, once
// its last launch has completed (the runtime may keep a node's arguments in
// one place, which a launch still queued would read).
fft_status_t rebind_graph(fft_ragged_s* r, const void* in, void* out)
{
    if (r->launched) {
        const hipError_t e = hipEventSynchronize(r->done);
        if (e != hipSuccess) return st_of(e);
    }
    for (Node& nd : r->nodes) {
        hipKernelNodeParams p;
        if (!node_params(r, nd, in, out, &p)) return FFT_ERR_DEVICE;
        const hipError_t e = hipGraphExecKernelNodeSetParams(r->exec, nd.node, &p);
        if (e != hipSuccess) return st_of(e);
    }
    r->g_in = in;
    r->g_out = out;
    return FFT_SUCCESS;
}

fft_status_t plain_plans(fft_ragged_s* r)
{
    if (!r->plain_plans.empty()) return FFT_SUCCESS;
    for (size_t c = 0; c < r->sizes.size(); ++c) {
        fft_plan_opts_t o;
        fft_plan_opts_init(&o);
        o.storage = r->storage;
        o.device_twiddles = r->device_twiddles;
        fft_plan_t p = nullptr;
        const fft_status_t st = fft_plan_create_ex(r->sizes[c], r->counts[c], r->direction, &o, &p);
        if (st != FFT_SUCCESS) {
            for (fft_plan_t q : r->plain_plans) fft_plan_destroy(q);
            r->plain_plans.clear();
            return st;
        }
        r->plain_plans.push_back(p);
    }
    return FFT_SUCCESS;
}

// Mode 2: the default plans' kernels captured on four branches.
fft_status_t capture_branches(fft_ragged_s* r, const void* in, void* out)
{
    hipError_t e = hipSuccess;
    if (!r->cap) {
        const size_t nb = std::min<size_t>(r->sizes.size(), 4);
        e = hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking);
        for (size_t b = 0; b < nb && e == hipSuccess; ++b) {
            hipStream_t s = nullptr;
            e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (e == hipSuccess) r->branches.push_back(s);
            hipEvent_t j = nullptr;
            if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
            if (e == hipSuccess) r->joins.push_back(j);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&r->fork, hipEventDisableTiming);
        if (e != hipSuccess) return st_of(e);
    }
    if (r->exec2) {
        // a launch of the old graph may still be queued or running
        if (r->launched) {
            e = hipEventSynchronize(r->done);
            if (e != hipSuccess) return st_of(e);
        }
        (void)hipGraphExecDestroy(r->exec2);
        r->exec2 = nullptr;
    }
    if (r->graph2) {
        (void)hipGraphDestroy(r->graph2);
        r->graph2 = nullptr;
    }
    e = hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return st_of(e);
    fft_status_t st = FFT_SUCCESS;
    e = hipEventRecord(r->fork, r->cap);
    const size_t nb = r->branches.size();
    for (size_t b = 0; b < nb && e == hipSuccess; ++b) e = hipStreamWaitEvent(r->branches[b], r->fork, 0);
    for (size_t c = 0; c < r->plain_plans.size() && e == hipSuccess && st == FFT_SUCCESS; ++c) {
        const char* x = (const char*)in + r->offsets[c] * r->elem;
        char* y = (char*)out + r->offsets[c] * r->elem;
        st = fft_execute(r->plain_plans[c], x, y, r->branches[c % nb]);
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
    r->graph2 = g;
    e = hipGraphInstantiate(&r->exec2, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return st_of(e);
    size_t nodes = 0;
    (void)hipGraphGetNodes(g, nullptr, &nodes);
    r->graph2_nodes = nodes;
    r->g2_in = in;
    r->g2_out = out;
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
        if (opts->scale != 0.0f && opts->scale != 1.0f) return FFT_ERR_INVALID_ARG;  // no output scale here
    }
    // the compact FP16 form has no persistent cases (their pass-1 tiles write
    // a complex64 workspace)
    if (po.storage != FFT_STORAGE_C64 && po.storage != FFT_STORAGE_F16) return FFT_ERR_INVALID_ARG;
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
    r->storage = po.storage;
    r->device_twiddles = po.device_twiddles;
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
    fft_status_t st = e == hipSuccess ? plan_classes(r) : st_of(e);
    if (st == FFT_SUCCESS) st = materialize(r);
    if (st != FFT_SUCCESS) {
        release(r);
        return st;
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
    if (!in || !out || mode < 0 || mode > 2) return FFT_ERR_INVALID_ARG;
    if (((uintptr_t)in & (r->elem - 1)) || ((uintptr_t)out & (r->elem - 1))) return FFT_ERR_INVALID_ARG;
    const size_t bytes = r->total_points * r->elem;
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if (a != b && a < b + bytes && b < a + bytes) return FFT_ERR_INVALID_ARG;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return st_of(e);
    if (cur != r->device && (e = hipSetDevice(r->device)) != hipSuccess) return st_of(e);
    hipStream_t st_h = (hipStream_t)stream;
    fft_status_t st = FFT_SUCCESS;
    if (!r->done && mode != 1) {
        e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming);
        if (e != hipSuccess) st = st_of(e);
    }
    if (st != FFT_SUCCESS) {
    } else if (mode == 0) {
        if (!r->exec)
            st = build_graph(r, in, out);
        else if (r->g_in != in || r->g_out != out)
            st = rebind_graph(r, in, out);
        if (st == FFT_SUCCESS) st = st_of(hipGraphLaunch(r->exec, st_h));
        if (st == FFT_SUCCESS) st = st_of(hipEventRecord(r->done, st_h));
        if (st == FFT_SUCCESS) r->launched = true;
    } else {
        st = plain_plans(r);
        if (st == FFT_SUCCESS && mode == 1) {
            // plain path: every class launched in order on the caller's stream
            for (size_t c = 0; c < r->plain_plans.size() && st == FFT_SUCCESS; ++c)
                st = fft_execute(r->plain_plans[c], (const char*)in + r->offsets[c] * r->elem,
                                 (char*)out + r->offsets[c] * r->elem, stream);
        } else if (st == FFT_SUCCESS) {
            if (!r->exec2 || r->g2_in != in || r->g2_out != out) st = capture_branches(r, in, out);
            if (st == FFT_SUCCESS) st = st_of(hipGraphLaunch(r->exec2, st_h));
            if (st == FFT_SUCCESS) st = st_of(hipEventRecord(r->done, st_h));
            if (st == FFT_SUCCESS) r->launched = true;
        }
    }
    if (cur != r->device) (void)hipSetDevice(cur);
    return st;
}

fft_status_t fft_ragged_describe(fft_ragged_t r, size_t* total_points, size_t* graph_nodes)
{
    if (!live(r)) return FFT_ERR_INVALID_PLAN;
    if (total_points) *total_points = r->total_points;
    if (graph_nodes) *graph_nodes = r->exec ? r->nodes.size() : 0;
    return FFT_SUCCESS;
}

fft_status_t fft_ragged_describe_ex(fft_ragged_t r, fft_ragged_desc_t* d)
{
    if (!live(r)) return FFT_ERR_INVALID_PLAN;
    if (!d) return FFT_ERR_INVALID_ARG;
    std::memset(d, 0, sizeof(*d));
    d->total_points = r->total_points;
    d->persistent_launches = (int)r->launches.size();
    size_t fb_nodes = 0;
    for (int c : r->fallback) {
        size_t n = 0;
        int dir = 0, path = 0;
        bool list = false;
        plan_shape(r->case_plans[(size_t)c], &n, &dir, &path, &list);
        fb_nodes += path == FFT_PATH_FOURSTEP ? 2 : 1;
    }
    d->graph_nodes = (int)(r->launches.size() + fb_nodes);
    d->fallback_classes = (int)r->fallback.size();
    for (size_t i = 0; i < r->launches.size() && i < 8; ++i) {
        const RagLaunch& L = r->launches[i];
        d->kernel_name[i] = L.k->name;
        d->units[i] = L.units;
        d->grid[i] = L.grid;
        d->classes[i] = (int)L.ents.size();
        d->threads[i] = L.k->threads;
        d->lds_bytes[i] = L.k->lds;
    }
    d->branch_graph_nodes = r->graph2_nodes;
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
