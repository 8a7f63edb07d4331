// Serving layer: a request scheduler (a host-only state machine, driven by
// explicit timestamps so it runs and is tested without a device) and a GPU
// server that feeds it from a dispatcher thread.
//
// Scheduling rules (fft_sched_next):
//   * requests are admitted in arrival order (FIFO); a request larger than
//     the whole budget is rejected, a request that does not fit the bytes
//     still free waits at the head of the queue;
//   * while the head waits, later requests of at most backfill_bytes may
//     pass it, with at most backfill_bytes of such requests in flight at a
//     time and never more than the head leaves of the budget: once the work
//     launched before the head completes, the head fits beside whatever
//     backfill is in flight, so it is delayed by little and never starved
//     (backfill_bytes = 0: strict FIFO);
//   * the launch goes to the stream with the fewest outstanding bytes among
//     those with fewer than max_inflight launches outstanding; the first
//     small_streams streams take only launches led by requests of at most
//     small_bytes (a lane for short requests, which would otherwise wait on a
//     stream behind a long transform), and such a launch uses any stream
//     when the lane is full;
//   * continuous batching: queued requests of the same (n, direction) that
//     the library can run as one list launch join the head's launch, in
//     arrival order, up to max_coalesce requests / max_transforms transforms
//     and within the budget.
// Latency of a request = completion time - arrival time, in the caller's
// clock (the server maps device completion events onto the host clock).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/fftblock.h"
#include "internal.hpp"

namespace {

struct SReq {
    uint64_t id = 0;
    size_t n = 0, batch = 0, bytes = 0;
    int dir = FFT_FORWARD;
    bool coalescible = false;
    int state = FFT_REQ_QUEUED;
    double t_arrive = 0.0, t_launch = -1.0, t_done = -1.0;
    long long launch = -1;
    int stream = -1;
    int group = 0;
    uint64_t seq = 0;   // arrival order
};

struct SLaunch {
    long long id = -1;
    int stream = 0;
    size_t n = 0, batch = 0, bytes = 0;
    int dir = FFT_FORWARD;
    bool backfill = false;
    std::vector<uint64_t> reqs;
};

class Scheduler {
public:
    explicit Scheduler(const fft_sched_opts_t& o)
        : o_(o), out_((size_t)o.n_streams, 0), outb_((size_t)o.n_streams, 0)
    {
    }

    fft_status_t submit(uint64_t id, size_t n, size_t batch, int dir, size_t bytes, bool coalescible, double now)
    {
        if (n == 0 || batch == 0 || (dir != FFT_FORWARD && dir != FFT_BACKWARD)) return FFT_ERR_INVALID_ARG;
        if (reqs_.count(id)) return FFT_ERR_INVALID_ARG;
        SReq r;
        r.id = id;
        r.n = n;
        r.batch = batch;
        r.dir = dir;
        r.bytes = bytes;
        r.coalescible = coalescible && batch <= o_.max_transforms;
        r.t_arrive = now;
        r.seq = next_seq_++;
        reqs_[id] = r;
        queue_.push_back(id);
        ++submitted_;
        return FFT_SUCCESS;
    }

    bool next(double now, SLaunch* L)
    {
        while (!queue_.empty() && reqs_[queue_.front()].bytes > o_.hbm_budget) {
            SReq& r = reqs_[queue_.front()];
            r.state = FFT_REQ_REJECTED;
            r.t_done = now;
            ++rejected_;
            queue_.pop_front();
        }
        if (queue_.empty()) return false;
        // the head, or -- while the head waits for room -- the first small
        // request that fits (backfill, bounded so the head is not starved)
        auto pick = queue_.begin();
        bool backfill = false;
        // backfill in flight may take at most what the head leaves of the budget
        size_t bf_cap = o_.backfill_bytes;
        if (inflight_ + reqs_[*pick].bytes > o_.hbm_budget) {
            if (o_.backfill_bytes == 0) return false;
            bf_cap = std::min(bf_cap, o_.hbm_budget - reqs_[*pick].bytes);
            for (++pick; pick != queue_.end(); ++pick) {
                const SReq& r = reqs_[*pick];
                if (r.bytes + backfill_inflight_ <= bf_cap && inflight_ + r.bytes <= o_.hbm_budget) break;
            }
            if (pick == queue_.end()) return false;
            backfill = true;
        }
        SReq& head = reqs_[*pick];
        const int s = pick_stream(head.bytes);
        if (s < 0) return false;
        L->id = next_launch_++;
        L->stream = s;
        L->n = head.n;
        L->dir = head.dir;
        L->batch = head.batch;
        L->bytes = head.bytes;
        L->backfill = backfill;
        L->reqs.assign(1, head.id);
        auto after = queue_.erase(pick);
        if (head.coalescible && o_.max_coalesce > 1) {
            for (auto it = backfill ? after : queue_.begin(); it != queue_.end() && (int)L->reqs.size() < o_.max_coalesce;) {
                const SReq& r = reqs_[*it];
                const bool room = backfill ? backfill_inflight_ + L->bytes + r.bytes <= bf_cap : true;
                if (r.coalescible && r.n == L->n && r.dir == L->dir && L->batch + r.batch <= o_.max_transforms &&
                    room && inflight_ + L->bytes + r.bytes <= o_.hbm_budget) {
                    L->reqs.push_back(r.id);
                    L->batch += r.batch;
                    L->bytes += r.bytes;
                    it = queue_.erase(it);
                } else {
                    ++it;
                }
            }
        }
        inflight_ += L->bytes;
        if (backfill) {
            backfill_inflight_ += L->bytes;
            backfilled_ += L->reqs.size();
        }
        peak_ = std::max(peak_, inflight_);
        out_[(size_t)s] += 1;
        outb_[(size_t)s] += L->bytes;
        for (uint64_t id : L->reqs) {
            SReq& r = reqs_[id];
            r.state = FFT_REQ_RUNNING;
            r.t_launch = now;
            r.launch = L->id;
            r.stream = s;
            r.group = (int)L->reqs.size();
        }
        ++launches_;
        if (L->reqs.size() > 1) coalesced_ += L->reqs.size();
        running_[L->id] = *L;
        return true;
    }

    // Stream for a launch led by a request of `bytes`: the fewest outstanding
    // bytes among streams below max_inflight.  Streams [0, lane) take only
    // small launches (at most small_bytes), so short requests do not queue on
    // a stream behind a long transform; a small launch falls back to any
    // stream when the lane is full.  -1: none free.
    int pick_stream(size_t bytes) const
    {
        const int lane = std::min(o_.small_streams, o_.n_streams - 1);
        const bool small = lane > 0 && bytes <= o_.small_bytes;
        auto best = [&](int lo, int hi) {
            int s = -1;
            for (int i = lo; i < hi; ++i)
                if (out_[(size_t)i] < o_.max_inflight && (s < 0 || outb_[(size_t)i] < outb_[(size_t)s])) s = i;
            return s;
        };
        if (!small) return best(lane, o_.n_streams);
        const int s = best(0, lane);
        return s >= 0 ? s : best(0, o_.n_streams);
    }

    // Undo a next() whose launch could not be issued: the requests go back to
    // the head of the queue in their order.
    void requeue(const SLaunch& L)
    {
        auto it = running_.find(L.id);
        if (it == running_.end()) return;
        for (uint64_t id : L.reqs) {
            SReq& q = reqs_[id];
            q.state = FFT_REQ_QUEUED;
            q.t_launch = -1.0;
            q.launch = -1;
            q.stream = -1;
            q.group = 0;
            // back to its place in arrival order
            auto at = queue_.begin();
            while (at != queue_.end() && reqs_[*at].seq < q.seq) ++at;
            queue_.insert(at, id);
        }
        if (L.backfill) {
            backfill_inflight_ -= L.bytes;
            backfilled_ -= L.reqs.size();
        }
        inflight_ -= L.bytes;
        out_[(size_t)L.stream] -= 1;
        outb_[(size_t)L.stream] -= L.bytes;
        --launches_;
        if (L.reqs.size() > 1) coalesced_ -= L.reqs.size();
        running_.erase(it);
    }

    fft_status_t complete(long long launch, double now, std::vector<uint64_t>* done)
    {
        auto it = running_.find(launch);
        if (it == running_.end()) return FFT_ERR_INVALID_ARG;
        const SLaunch& L = it->second;
        for (uint64_t id : L.reqs) {
            SReq& r = reqs_[id];
            r.state = FFT_REQ_DONE;
            r.t_done = now;
            lat_.push_back(now - r.t_arrive);
            wait_.push_back(r.t_launch - r.t_arrive);
            run_.push_back(now - r.t_launch);
            points_ += (double)r.n * (double)r.batch;
            ++completed_;
            if (done) done->push_back(id);
        }
        inflight_ -= L.bytes;
        if (L.backfill) backfill_inflight_ -= L.bytes;
        out_[(size_t)L.stream] -= 1;
        outb_[(size_t)L.stream] -= L.bytes;
        t_last_ = std::max(t_last_, now);
        running_.erase(it);
        return FFT_SUCCESS;
    }

    bool info(uint64_t id, fft_request_info_t* o) const
    {
        auto it = reqs_.find(id);
        if (it == reqs_.end()) return false;
        const SReq& r = it->second;
        o->id = r.id;
        o->n = r.n;
        o->batch = r.batch;
        o->direction = r.dir;
        o->state = r.state;
        o->bytes = r.bytes;
        o->t_arrive = r.t_arrive;
        o->t_launch = r.t_launch;
        o->t_done = r.t_done;
        o->launch = r.launch;
        o->stream = r.stream;
        o->group_size = r.group;
        return true;
    }

    void forget(uint64_t id) { reqs_.erase(id); }
    size_t queued() const { return queue_.size(); }
    size_t running() const { return running_.size(); }

    void stats(fft_sched_stats_t* s) const
    {
        std::memset(s, 0, sizeof(*s));
        s->submitted = submitted_;
        s->completed = completed_;
        s->rejected = rejected_;
        s->queued = queue_.size();
        s->running_launches = running_.size();
        s->launches = launches_;
        s->coalesced_requests = coalesced_;
        s->backfilled_requests = backfilled_;
        s->inflight_bytes = inflight_;
        s->peak_inflight_bytes = peak_;
        s->points = points_;
        s->t_last_done = t_last_;
        if (!lat_.empty()) {
            // nearest rank: the smallest value with at least p of the samples at or below it
            auto pct = [](const std::vector<double>& v, double p) {
                size_t k = (size_t)std::ceil(p * (double)v.size());
                if (k < 1) k = 1;
                return v[k - 1];
            };
            std::vector<double> v = lat_, w = wait_, r = run_;
            std::sort(v.begin(), v.end());
            std::sort(w.begin(), w.end());
            std::sort(r.begin(), r.end());
            double sum = 0.0;
            for (double x : v) sum += x;
            s->latency_p50 = pct(v, 0.50);
            s->latency_p99 = pct(v, 0.99);
            s->latency_mean = sum / (double)v.size();
            s->latency_max = v.back();
            s->queue_p50 = pct(w, 0.50);
            s->queue_p99 = pct(w, 0.99);
            s->device_p50 = pct(r, 0.50);
            s->device_p99 = pct(r, 0.99);
        }
    }

private:
    fft_sched_opts_t o_;
    std::unordered_map<uint64_t, SReq> reqs_;
    std::deque<uint64_t> queue_;
    std::map<long long, SLaunch> running_;
    std::vector<int> out_;
    std::vector<size_t> outb_;
    size_t inflight_ = 0, peak_ = 0, backfill_inflight_ = 0, backfilled_ = 0;
    uint64_t next_seq_ = 0;
    size_t submitted_ = 0, completed_ = 0, rejected_ = 0, launches_ = 0, coalesced_ = 0;
    long long next_launch_ = 0;
    double points_ = 0.0, t_last_ = 0.0;
    std::vector<double> lat_, wait_, run_;  // arrival->done, arrival->launch, launch->done
};

bool opts_ok(const fft_sched_opts_t& o)
{
    return o.hbm_budget > 0 && o.n_streams >= 1 && o.n_streams <= 16 && o.max_inflight >= 1 &&
           o.max_coalesce >= 1 && o.max_coalesce <= FFT_LAUNCH_MAX_REQUESTS && o.max_transforms >= 1 &&
           o.small_streams >= 0;
}

}  // namespace

struct fft_sched_s {
    explicit fft_sched_s(const fft_sched_opts_t& o) : s(o) {}
    Scheduler s;
};

namespace {

std::mutex g_smu;
std::unordered_set<const void*> g_live;

bool live(const void* p)
{
    std::lock_guard<std::mutex> lk(g_smu);
    return p && g_live.count(p);
}
void track(const void* p)
{
    std::lock_guard<std::mutex> lk(g_smu);
    g_live.insert(p);
}
bool untrack(const void* p)
{
    std::lock_guard<std::mutex> lk(g_smu);
    return p && g_live.erase(p) == 1;
}

void fill_launch(const SLaunch& L, fft_launch_t* o)
{
    std::memset(o, 0, sizeof(*o));
    o->id = L.id;
    o->stream = L.stream;
    o->n = L.n;
    o->direction = L.dir;
    o->batch = L.batch;
    o->bytes = L.bytes;
    o->n_requests = (int)L.reqs.size();
    for (size_t i = 0; i < L.reqs.size() && i < FFT_LAUNCH_MAX_REQUESTS; ++i) o->requests[i] = L.reqs[i];
}

}  // namespace

extern "C" {

void fft_sched_opts_init(fft_sched_opts_t* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->hbm_budget = (size_t)64 << 30;
    o->n_streams = 4;
    o->max_inflight = 2;
    o->max_coalesce = 32;
    o->max_transforms = 16384;
    o->backfill_bytes = (size_t)1 << 30;
    o->small_streams = 1;
    o->small_bytes = (size_t)64 << 20;
}

fft_status_t fft_sched_create(const fft_sched_opts_t* opts, fft_sched_t* out)
{
    if (!out) return FFT_ERR_INVALID_ARG;
    *out = nullptr;
    fft_sched_opts_t o;
    fft_sched_opts_init(&o);
    if (opts) o = *opts;
    if (!opts_ok(o)) return FFT_ERR_INVALID_ARG;
    fft_sched_s* s = new (std::nothrow) fft_sched_s(o);
    if (!s) return FFT_ERR_OUT_OF_MEMORY;
    track(s);
    *out = s;
    return FFT_SUCCESS;
}

fft_status_t fft_sched_destroy(fft_sched_t s)
{
    if (!untrack(s)) return FFT_ERR_INVALID_PLAN;
    delete s;
    return FFT_SUCCESS;
}

fft_status_t fft_sched_submit(fft_sched_t s, uint64_t id, size_t n, size_t batch, int direction, size_t bytes,
                              int coalescible, double now)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    return s->s.submit(id, n, batch, direction, bytes, coalescible != 0, now);
}

fft_status_t fft_sched_next(fft_sched_t s, double now, fft_launch_t* launch, int* got)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    if (!launch || !got) return FFT_ERR_INVALID_ARG;
    SLaunch L;
    *got = s->s.next(now, &L) ? 1 : 0;
    if (*got) fill_launch(L, launch);
    return FFT_SUCCESS;
}

fft_status_t fft_sched_complete(fft_sched_t s, long long launch_id, double now)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    return s->s.complete(launch_id, now, nullptr);
}

fft_status_t fft_sched_request(fft_sched_t s, uint64_t id, fft_request_info_t* info)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    if (!info) return FFT_ERR_INVALID_ARG;
    return s->s.info(id, info) ? FFT_SUCCESS : FFT_ERR_INVALID_ARG;
}

fft_status_t fft_sched_stats(fft_sched_t s, fft_sched_stats_t* st)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    if (!st) return FFT_ERR_INVALID_ARG;
    s->s.stats(st);
    return FFT_SUCCESS;
}

}  // extern "C"

// ------------------------------------------------------------------ server
namespace {

// First-fit allocator over one device allocation (offsets, 256-byte units).
class Arena {
public:
    void reset(size_t bytes)
    {
        free_.clear();
        if (bytes) free_[0] = bytes;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

private:
    std::map<size_t, size_t> free_;
};

struct SrvReq {
    const float2* in = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream: the input is written
    size_t out_off = 0, out_bytes = 0;
    size_t ws_off = 0, ws_bytes = 0;
    bool has_out = false, has_ws = false;
    bool done = false, released = false;
    fft_request_info_t info{};
};

struct InFlight {
    SLaunch L;
    hipEvent_t done = nullptr;
    int chunk = -1;
};

constexpr int kChunks = 16;

}  // namespace

struct fft_server_s {
    explicit fft_server_s(const fft_server_opts_t& o) : opts(o), sched(o.sched) {}
    fft_server_opts_t opts;
    Scheduler sched;
    int device = 0;
    std::vector<hipStream_t> streams;
    char* arena_base = nullptr;
    Arena arena;
    fb::ListEnt* host_desc = nullptr;  // pinned, kChunks * max_transforms
    fb::ListEnt* dev_desc = nullptr;
    std::vector<int> free_chunks;
    std::map<std::pair<size_t, int>, fft_plan_t> plans;
    std::deque<InFlight> inflight;
    std::vector<hipEvent_t> event_pool;
    std::vector<hipEvent_t> ready_pool;  // input-ready events (no timing)
    std::unordered_map<uint64_t, SrvReq> reqs;
    uint64_t next_id = 1;
    std::thread worker;
    std::mutex mu;
    std::condition_variable wake, done_cv;
    bool stop = false;
    fft_status_t error = FFT_SUCCESS;
    std::chrono::steady_clock::time_point t0;
    hipEvent_t ref = nullptr;
    double t_ref = 0.0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

fft_status_t st_of(hipError_t e)
{
    return e == hipSuccess ? FFT_SUCCESS : e == hipErrorOutOfMemory ? FFT_ERR_OUT_OF_MEMORY : FFT_ERR_DEVICE;
}

// Options of the server's plans: single blocks up to 16384 at every batch
// (their list forms coalesce same-length requests), four-step above.
fft_plan_opts_t server_plan_opts()
{
    fft_plan_opts_t o;
    fft_plan_opts_init(&o);
    o.block_limit = std::min<size_t>(fft_block_limit(), 16384);
    return o;
}

// Plan for (n, direction), created on first use (batch 1: the tables; the
// per-request batch and workspace are given at execute).
fft_status_t get_plan(fft_server_s* s, size_t n, int dir, fft_plan_t* p)
{
    auto key = std::make_pair(n, dir);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) {
        *p = it->second;
        return FFT_SUCCESS;
    }
    fft_plan_t q = nullptr;
    const fft_plan_opts_t o = server_plan_opts();
    const fft_status_t st = fft_plan_create_ex(n, 1, dir, &o, &q);
    if (st != FFT_SUCCESS) return st;
    s->plans[key] = q;
    *p = q;
    return FFT_SUCCESS;
}

bool plan_is_fourstep(fft_plan_t p)
{
    size_t n = 0;
    int dir = 0, path = 0;
    bool list = false;
    fb::plan_shape(p, &n, &dir, &path, &list);
    return path == FFT_PATH_FOURSTEP;
}

bool plan_has_list(fft_plan_t p)
{
    size_t n = 0;
    int dir = 0, path = 0;
    bool list = false;
    fb::plan_shape(p, &n, &dir, &path, &list);
    return list;
}

// The request's input-ready event back to the pool (its launch has completed,
// or it was never issued).
void drop_ready(fft_server_s* s, SrvReq& r)
{
    if (r.ready) {
        s->ready_pool.push_back(r.ready);
        r.ready = nullptr;
    }
}

void free_request_memory(fft_server_s* s, SrvReq& r, bool out_too)
{
    if (r.has_ws) {
        s->arena.release(r.ws_off, r.ws_bytes);
        r.has_ws = false;
    }
    if (out_too && r.has_out) {
        s->arena.release(r.out_off, r.out_bytes);
        r.has_out = false;
    }
}

// Issue one scheduled launch (lock held).  false: resources not available
// now (the launch is requeued); an error is made sticky in s->error.
bool issue(fft_server_s* s, const SLaunch& L)
{
    fft_plan_t plan = nullptr;
    fft_status_t st = get_plan(s, L.n, L.dir, &plan);
    if (st != FFT_SUCCESS) {
        s->error = st;
        return false;
    }
    const bool four = plan_is_fourstep(plan);
    // output (and workspace) memory for every request
    std::vector<uint64_t> got;
    bool ok = true;
    for (uint64_t id : L.reqs) {
        SrvReq& r = s->reqs[id];
        r.out_bytes = L.n * r.info.batch * sizeof(float2);
        ok = s->arena.alloc(r.out_bytes, &r.out_off);
        if (!ok) break;
        r.has_out = true;
        if (four) {
            r.ws_bytes = r.out_bytes;
            ok = s->arena.alloc(r.ws_bytes, &r.ws_off);
            if (!ok) break;
            r.has_ws = true;
        }
        got.push_back(id);
    }
    // every single-block request goes through the list form of the plan's
    // kernel, alone or coalesced, so its result does not depend on the mix
    int chunk = -1;
    const bool list = !four && plan_has_list(plan) && L.batch <= s->opts.sched.max_transforms;
    if (ok && list) {
        if (s->free_chunks.empty()) {
            ok = false;
        } else {
            chunk = s->free_chunks.back();
            s->free_chunks.pop_back();
        }
    }
    if (!ok) {
        for (uint64_t id : L.reqs) free_request_memory(s, s->reqs[id], true);
        if (chunk >= 0) s->free_chunks.push_back(chunk);
        return false;
    }
    hipStream_t stream = s->streams[(size_t)L.stream];
    hipError_t e = hipSuccess;
    // the launch reads each request's input only after the work the submitter
    // had queued on its stream before submitting (the producer of the input)
    for (uint64_t id : L.reqs) {
        const SrvReq& r = s->reqs[id];
        if (e == hipSuccess && r.ready) e = hipStreamWaitEvent(stream, r.ready, 0);
    }
    if (e == hipSuccess && list) {
        const size_t cap = s->opts.sched.max_transforms;
        fb::ListEnt* h = s->host_desc + (size_t)chunk * cap;
        fb::ListEnt* d = s->dev_desc + (size_t)chunk * cap;
        size_t at = 0;
        for (uint64_t id : L.reqs) {
            SrvReq& r = s->reqs[id];
            float2* out = reinterpret_cast<float2*>(s->arena_base + r.out_off);
            for (size_t b = 0; b < r.info.batch; ++b) h[at++] = {r.in + b * L.n, out + b * L.n};
        }
        e = hipMemcpyAsync(d, h, at * sizeof(fb::ListEnt), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = fb::plan_launch_list(plan, d, (long long)at, stream);
    } else if (e == hipSuccess) {
        for (uint64_t id : L.reqs) {
            SrvReq& r = s->reqs[id];
            void* out = s->arena_base + r.out_off;
            void* ws = r.has_ws ? (void*)(s->arena_base + r.ws_off) : nullptr;
            st = fft_execute_ex(plan, r.info.batch, r.in, out, ws, stream);
            if (st != FFT_SUCCESS) {
                e = hipErrorUnknown;
                break;
            }
        }
    }
    InFlight f;
    f.L = L;
    f.chunk = chunk;
    if (e == hipSuccess) {
        if (s->event_pool.empty()) {
            e = hipEventCreate(&f.done);
        } else {
            f.done = s->event_pool.back();
            s->event_pool.pop_back();
        }
    }
    if (e == hipSuccess) e = hipEventRecord(f.done, stream);
    if (e != hipSuccess) {
        s->error = st_of(e) == FFT_SUCCESS ? FFT_ERR_DEVICE : st_of(e);
        if (f.done) s->event_pool.push_back(f.done);
        // the launch may be partly queued: wait for the stream before freeing
        (void)hipStreamSynchronize(stream);
        for (uint64_t id : L.reqs) free_request_memory(s, s->reqs[id], true);
        if (chunk >= 0) s->free_chunks.push_back(chunk);
        return false;
    }
    s->inflight.push_back(f);
    return true;
}

void finish_launch(fft_server_s* s, InFlight& f, double t_done)
{
    std::vector<uint64_t> done;
    (void)s->sched.complete(f.L.id, t_done, &done);
    for (uint64_t id : done) {
        SrvReq& r = s->reqs[id];
        drop_ready(s, r);
        free_request_memory(s, r, s->opts.auto_release != 0);
        (void)s->sched.info(id, &r.info);
        r.done = true;
        if (s->opts.auto_release) {
            s->sched.forget(id);
            s->reqs.erase(id);
        }
    }
    if (f.chunk >= 0) s->free_chunks.push_back(f.chunk);
    s->event_pool.push_back(f.done);
}

void worker_loop(fft_server_s* s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        for (auto it = s->inflight.begin(); it != s->inflight.end();) {
            const hipError_t q = hipEventQuery(it->done);
            if (q == hipErrorNotReady) {
                ++it;
                continue;
            }
            float ms = 0.f;
            if (q != hipSuccess || hipEventElapsedTime(&ms, s->ref, it->done) != hipSuccess) {
                if (q != hipSuccess) s->error = FFT_ERR_DEVICE;
                ms = (float)((s->now() - s->t_ref) * 1e3);
            }
            finish_launch(s, *it, s->t_ref + (double)ms * 1e-3);
            it = s->inflight.erase(it);
            progress = true;
        }
        if (progress) s->done_cv.notify_all();
        if (s->error == FFT_SUCCESS) {
            SLaunch L;
            while (s->sched.next(s->now(), &L)) {
                if (!issue(s, L)) {
                    s->sched.requeue(L);
                    break;
                }
                progress = true;
            }
        }
        // stopping: whatever could be issued has been; with nothing in flight
        // no completion can free room for what is still queued
        if (s->stop && s->inflight.empty()) break;
        if (!progress) {
            if (s->inflight.empty())
                s->wake.wait_for(lk, std::chrono::milliseconds(5));
            else
                s->wake.wait_for(lk, std::chrono::microseconds(20));
        }
    }
    s->done_cv.notify_all();
}

void server_free(fft_server_s* s)
{
    for (auto& kv : s->plans) (void)fft_plan_destroy(kv.second);
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->ready_pool) (void)hipEventDestroy(e);
    for (auto& kv : s->reqs)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    for (auto& f : s->inflight)
        if (f.done) (void)hipEventDestroy(f.done);
    if (s->ref) (void)hipEventDestroy(s->ref);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->dev_desc) (void)hipFree(s->dev_desc);
    if (s->host_desc) (void)hipHostFree(s->host_desc);
    delete s;
}

}  // namespace

extern "C" {

void fft_server_opts_init(fft_server_opts_t* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    fft_sched_opts_init(&o->sched);
    o->arena_bytes = 0;
    o->auto_release = 0;
}

fft_status_t fft_server_create(const fft_server_opts_t* opts, fft_server_t* out)
{
    if (!out) return FFT_ERR_INVALID_ARG;
    *out = nullptr;
    fft_server_opts_t o;
    fft_server_opts_init(&o);
    if (opts) o = *opts;
    if (!opts_ok(o.sched)) return FFT_ERR_INVALID_ARG;
    if (o.arena_bytes == 0) o.arena_bytes = o.sched.hbm_budget;
    fft_server_s* s = new (std::nothrow) fft_server_s(o);
    if (!s) return FFT_ERR_OUT_OF_MEMORY;
    hipError_t e = hipGetDevice(&s->device);
    for (int i = 0; i < o.sched.n_streams && e == hipSuccess; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
    }
    if (e == hipSuccess) e = hipMalloc((void**)&s->arena_base, o.arena_bytes);
    const size_t desc = (size_t)kChunks * o.sched.max_transforms * sizeof(fb::ListEnt);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->host_desc, desc, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&s->dev_desc, desc);
    if (e == hipSuccess) e = hipEventCreate(&s->ref);
    // host time of the reference event: between the record call and the
    // return of its synchronisation (completion times inherit that error)
    s->t0 = std::chrono::steady_clock::now();
    const double before = s->now();
    if (e == hipSuccess) e = hipEventRecord(s->ref, s->streams[0]);
    if (e == hipSuccess) e = hipEventSynchronize(s->ref);
    if (e != hipSuccess) {
        const fft_status_t st = st_of(e);
        server_free(s);
        return st;
    }
    s->t_ref = 0.5 * (before + s->now());
    s->arena.reset(o.arena_bytes);
    for (int c = kChunks - 1; c >= 0; --c) s->free_chunks.push_back(c);
    try {
        s->worker = std::thread(worker_loop, s);
    } catch (...) {
        server_free(s);
        return FFT_ERR_OUT_OF_MEMORY;
    }
    track(s);
    *out = s;
    return FFT_SUCCESS;
}

fft_status_t fft_server_prepare(fft_server_t s, size_t n, int direction)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    if (direction != FFT_FORWARD && direction != FFT_BACKWARD) return FFT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    fft_plan_t p = nullptr;
    return get_plan(s, n, direction, &p);
}

fft_status_t fft_server_submit(fft_server_t s, size_t n, size_t batch, int direction, const void* in,
                               void* stream, uint64_t* ticket)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    if (!ticket || !in || ((uintptr_t)in & 7u) || n == 0 || batch == 0) return FFT_ERR_INVALID_ARG;
    if (direction != FFT_FORWARD && direction != FFT_BACKWARD) return FFT_ERR_INVALID_ARG;
    fft_plan_desc_t d;
    fft_status_t st = fft_plan_query(n, batch, direction, &d);   // validates the batch
    if (st != FFT_SUCCESS) return st;
    // the path of the server's own plan for n (as get_plan creates it)
    const fft_plan_opts_t so = server_plan_opts();
    st = fft_plan_query_ex(n, 1, direction, &so, &d);
    if (st != FFT_SUCCESS) return st;
    const bool four = d.path == FFT_PATH_FOURSTEP;
    const size_t bytes = n * batch * sizeof(float2) * (four ? 3 : 2);  // in + out (+ workspace)
    // arena space it takes when issued (output, and workspace, in 256-byte
    // units): a request that can never fit would hold the queue's head forever
    const size_t part = (n * batch * sizeof(float2) + 255) & ~(size_t)255;
    if (part * (four ? 2 : 1) > s->opts.arena_bytes) return FFT_ERR_OUT_OF_MEMORY;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error != FFT_SUCCESS) return s->error;
    // mark the submitter's stream: the server's launch waits for this point
    hipEvent_t ready = nullptr;
    if (!s->ready_pool.empty()) {
        ready = s->ready_pool.back();
        s->ready_pool.pop_back();
    } else {
        const hipError_t e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
        if (e != hipSuccess) return st_of(e);
    }
    const hipError_t er = hipEventRecord(ready, (hipStream_t)stream);
    if (er != hipSuccess) {
        s->ready_pool.push_back(ready);
        return st_of(er);
    }
    const uint64_t id = s->next_id++;
    // a list launch exists for every default single-block length
    st = s->sched.submit(id, n, batch, direction, bytes, !four, s->now());
    if (st != FFT_SUCCESS) {
        s->ready_pool.push_back(ready);
        return st;
    }
    SrvReq r;
    r.in = (const float2*)in;
    r.ready = ready;
    (void)s->sched.info(id, &r.info);
    s->reqs[id] = r;
    *ticket = id;
    s->wake.notify_one();
    return FFT_SUCCESS;
}

fft_status_t fft_server_wait(fft_server_t s, uint64_t ticket, double timeout_s, void** out,
                             fft_request_info_t* info)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return FFT_ERR_INVALID_ARG;
    const auto limit = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (true) {
        it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return FFT_ERR_INVALID_ARG;
        (void)s->sched.info(ticket, &it->second.info);
        if (it->second.done || it->second.info.state == FFT_REQ_REJECTED) break;
        if (s->error != FFT_SUCCESS) return s->error;
        if (s->done_cv.wait_until(lk, limit) == std::cv_status::timeout) return FFT_ERR_TIMEOUT;
    }
    SrvReq& r = it->second;
    if (info) *info = r.info;
    if (r.info.state == FFT_REQ_REJECTED) return FFT_ERR_OUT_OF_MEMORY;
    if (out) *out = r.has_out ? (void*)(s->arena_base + r.out_off) : nullptr;
    return FFT_SUCCESS;
}

fft_status_t fft_server_read(fft_server_t s, uint64_t ticket, void* dst, void* stream)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    if (!dst) return FFT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || !it->second.done || !it->second.has_out) return FFT_ERR_INVALID_ARG;
    const SrvReq& r = it->second;
    return st_of(hipMemcpyAsync(dst, s->arena_base + r.out_off, r.out_bytes, hipMemcpyDeviceToDevice,
                                (hipStream_t)stream));
}

fft_status_t fft_server_release(fft_server_t s, uint64_t ticket)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return FFT_ERR_INVALID_ARG;
    SrvReq& r = it->second;
    if (!r.done && r.info.state != FFT_REQ_REJECTED) return FFT_ERR_INVALID_ARG;  // still queued or running
    drop_ready(s, r);
    free_request_memory(s, r, true);
    s->sched.forget(ticket);
    s->reqs.erase(it);
    return FFT_SUCCESS;
}

fft_status_t fft_server_drain(fft_server_t s, double timeout_s)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    std::unique_lock<std::mutex> lk(s->mu);
    const auto limit = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (s->sched.queued() > 0 || !s->inflight.empty()) {
        if (s->error != FFT_SUCCESS) return s->error;
        s->wake.notify_one();
        if (s->done_cv.wait_until(lk, limit) == std::cv_status::timeout) return FFT_ERR_TIMEOUT;
    }
    return s->error;
}

fft_status_t fft_server_stats(fft_server_t s, fft_sched_stats_t* st)
{
    if (!live(s)) return FFT_ERR_INVALID_PLAN;
    if (!st) return FFT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    s->sched.stats(st);
    return FFT_SUCCESS;
}

double fft_server_clock(fft_server_t s)
{
    if (!live(s)) return -1.0;
    return s->now();
}

fft_status_t fft_server_destroy(fft_server_t s)
{
    if (!untrack(s)) return FFT_ERR_INVALID_PLAN;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->wake.notify_one();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    const hipError_t e = hipDeviceSynchronize();
    const fft_status_t st = s->error != FFT_SUCCESS ? s->error : st_of(e);
    server_free(s);
    return st;
}

}  // extern "C"
