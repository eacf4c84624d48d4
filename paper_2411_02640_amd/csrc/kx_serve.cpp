// kx_serve.cpp -- continuous-batching request server.
//
// Mechanisms are made resident with kx_server_add_mech: their device tables
// are copied into the server's arena (so they count against its HBM budget)
// and the launch graphs of their batches are captured at once.  Requests
// (device-resident inputs, any resident mechanism, op and precision) are
// queued in arrival order.  A scheduler thread
//   1. retires finished batches (event query) and marks their requests DONE;
//   2. admits queued requests in order while a slot is free and the output
//      arena has room for the request's outputs (admission by HBM footprint);
//   3. while a stream is idle, takes the oldest admitted request's
//      (mechanism, precision) group -- up to kMaxBatch requests -- writes the
//      batch work list into that stream's pinned staging buffer, copies it to
//      the stream's device work list and launches the batch: a batch of fewer
//      than kBigBatchPoints points replays the stream's HIP graph for the
//      group (zero counters, work-stealing rates kernel, work-stealing
//      transport kernel; captured once per (stream, mechanism, precision, ops)
//      because the work list and counters live at fixed addresses and the
//      grids do not depend on the batch), a bigger one is launched directly
//      with one workgroup per tile (the grids are the batch's tile counts; the
//      work-stealing kernels measured 3 to 10 percent slower per tile).
// Batches of different groups run on different streams and overlap on the
// device; requests that arrive meanwhile join the next batch of their group.
// The scheduler holds the server lock only while it changes request state:
// work-list copies, graph launches and event records run without it, so
// clients submitting and polling are not held up by HIP calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "kx_internal.h"

namespace kx {
namespace {

constexpr int kStreams = 4;
constexpr double kSimSecondsPerPoint = 5e-9;
// A batch of at least this many points fills the GPU on its own: two such
// batches are not run at the same time (they would only compete for the CUs,
// and their kernels' caches and LDS), while smaller batches overlap anything.
constexpr int64_t kBigBatchPoints = 1 << 17;

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, capacity) in 256-byte units.
class Arena {
  public:
    explicit Arena(size_t cap) : cap_(cap)
    {
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t capacity() const { return cap_; }

  private:
    size_t cap_, used_ = 0;
    std::map<size_t, size_t> free_;
};

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

struct Req {
    kx_ticket id;
    kx_request r;
    int state = KX_REQ_QUEUED;
    size_t off = 0, bytes = 0;
    bool has_mem = false;
    double t_arrival = 0, t_admit = 0, t_launch = 0, t_done = 0;
    double *wdot = nullptr, *mu = nullptr, *lam = nullptr, *Dmix = nullptr;
};

using GraphKey = std::tuple<uint64_t, int, int>;  // (mechanism uid, precision, ops)

// A mechanism resident on the server: its tables copied into the arena.
struct ServedMech {
    MechDev dev;             // table pointers into the server's copy
    size_t off = 0, bytes = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    WorkList *d_wl = nullptr;   // device work list
    WorkList *h_wl = nullptr;   // pinned staging
    int *d_counter = nullptr;   // kBatchCounters tile counters (rates per XCD, transport)
    bool busy = false;
    bool big = false;           // the running batch has >= kBigBatchPoints points
    double sim_done_at = 0;
    std::vector<Req *> reqs;
    std::map<GraphKey, hipGraphExec_t> graphs;
};

}  // namespace
}  // namespace kx

using namespace kx;

struct kx_server {
    int device = 0;
    bool simulate = false;
    int max_slots = 1;
    char *arena_base = nullptr;
    Arena arena{0};
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Req *> pending;
    std::vector<Req *> admitted;
    std::unordered_map<kx_ticket, Req *> reqs;
    int in_flight = 0;
    Slot slots[kStreams];
    std::thread thread;
    bool stop = false;
    kx_ticket next_id = 1;
    kx_server_stats stats{};
    std::unordered_map<const kx_mech *, ServedMech> mechs;  // resident mechanisms
    size_t resident_bytes = 0;
    std::mutex add_mu;  // serialises kx_server_add_mech
};

namespace kx {
namespace {

size_t footprint(const kx_request &r, int ns)
{
    size_t doubles = (size_t)ns;                            // wdot
    if (r.ops & KX_OP_TRANSPORT) doubles += (size_t)ns + 2;  // mu, lambda, Dmix
    return round256((size_t)r.n * 8 * doubles);
}

void place_outputs(kx_server *s, Req *q)
{
    if (s->simulate) return;  // no device memory behind a simulated arena
    const int ns = q->r.mech->n_species;
    char *base = s->arena_base + q->off;
    const int64_t n = q->r.n;
    q->wdot = reinterpret_cast<double *>(base);
    if (q->r.ops & KX_OP_TRANSPORT) {
        q->Dmix = q->wdot + (size_t)ns * n;
        q->mu = q->Dmix + (size_t)ns * n;
        q->lam = q->mu + n;
    }
}

// Capture the launch sequence of one batch of (mechanism, precision, ops) on
// slot `sl`'s work list and counters; captured on `cap` (any idle stream: the
// graph does not belong to a stream).
kx_status build_graph(const MechDev &dev, Slot &sl, int prec, int ops, hipStream_t cap,
                      hipGraphExec_t *out)
{
    // kernel attributes are set outside the capture
    kx_status pst = prepare_rates_batch(dev, prec);
    if (pst == KX_OK && (ops & KX_OP_TRANSPORT)) pst = prepare_transport_batch(dev, prec);
    if (pst != KX_OK) return pst;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    kx_status st = launch_zero(sl.d_counter, kBatchCounters, cap);
    if (st == KX_OK) st = launch_rates_batch(dev, sl.d_wl, sl.d_counter, prec, kRatesBatchGrid, cap);
    if (st == KX_OK && (ops & KX_OP_TRANSPORT))
        st = launch_transport_batch(dev, sl.d_wl, sl.d_counter + kXcds, prec, kTransportBatchGrid,
                                    cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap, &g);
    if (st != KX_OK) {
        if (g) hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return KX_OK;
}

// Mark a batch as launched on slot `sl`.  Called with the lock held.
void begin_batch(kx_server *s, Slot &sl, std::vector<Req *> &batch)
{
    const double t = now_s();
    for (Req *q : batch) {
        q->state = KX_REQ_RUNNING;
        q->t_launch = t;
    }
    sl.reqs = batch;
    sl.busy = true;
    int64_t pts = 0;
    for (Req *q : batch) pts += q->r.n;
    sl.big = pts >= kBigBatchPoints;
    s->stats.batches++;
    if (s->simulate) {
        double work = 0;
        for (Req *q : batch) work += (double)q->r.n * ((q->r.ops & KX_OP_TRANSPORT) ? 2 : 1);
        sl.sim_done_at = t + work * kSimSecondsPerPoint;
    }
}

// Enqueue a begun batch on its slot's stream: waits on the inputs' events, the
// work list, then a graph replay (or, for a big batch, the one-tile kernels),
// and the completion event.  Called WITHOUT the lock: it reads only the
// requests of this batch (fixed while they run) and the slot, which no other
// thread touches while it is busy.  Returns whether the batch was enqueued
// (false: nothing usable was, and the stream has drained); *used_graph tells
// whether a graph replay runs it.
bool enqueue_batch(kx_server *s, Slot &sl, const ServedMech &sm, hipGraphExec_t graph,
                   hipGraphExec_t *new_graph, bool *used_graph)
{
    const std::vector<Req *> &batch = sl.reqs;
    const int prec = batch[0]->r.precision;
    int ops = 0;
    for (Req *q : batch) ops |= q->r.ops;
    WorkList &w = *sl.h_wl;
    std::memset(&w, 0, sizeof w);
    w.nitems = (int)batch.size();
    const int tpr = rates_tile_points(sm.dev);
    const int tpt = transport_tile_points(sm.dev, prec);
    int tr = 0, tt = 0;
    for (size_t r = 0; r < batch.size(); ++r) {
        const Req *q = batch[r];
        WorkItem &it = w.items[r];
        it.T = q->r.T;
        it.p = q->r.p;
        it.Y = q->r.Y;
        it.wdot = q->wdot;
        it.mu = q->mu;
        it.lam = q->lam;
        it.Dmix = q->Dmix;
        it.n = q->r.n;
        w.start[0][r] = tr;
        w.start[1][r] = tt;
        tr += (int)((q->r.n + tpr - 1) / tpr);
        if (q->r.ops & KX_OP_TRANSPORT) tt += (int)((q->r.n + tpt - 1) / tpt);
    }
    w.start[0][batch.size()] = w.ntiles[0] = tr;
    w.start[1][batch.size()] = w.ntiles[1] = tt;

    bool ok_launch = true;
    for (const Req *q : batch)
        if (ok_launch && q->r.inputs_ready)
            ok_launch = hipStreamWaitEvent(sl.stream, q->r.inputs_ready, 0) == hipSuccess;
    if (ok_launch)
        ok_launch = hipMemcpyAsync(sl.d_wl, sl.h_wl, sizeof(WorkList), hipMemcpyHostToDevice,
                                   sl.stream) == hipSuccess;
    *used_graph = false;
    *new_graph = nullptr;
    if (ok_launch && sl.big) {
        // one workgroup per tile, rates then transport
        ok_launch = launch_rates_items(sm.dev, sl.d_wl, tr, prec, sl.stream) == KX_OK &&
                    (!(ops & KX_OP_TRANSPORT) ||
                     launch_transport_items(sm.dev, sl.d_wl, tt, prec, sl.stream) == KX_OK);
    } else if (ok_launch) {
        if (!graph) {
            // captured when the mechanism was added; built here only if that
            // failed (the caller files it under the lock)
            if (build_graph(sm.dev, sl, prec, ops, sl.stream, new_graph) == KX_OK)
                graph = *new_graph;
        }
        if (graph) {
            ok_launch = hipGraphLaunch(graph, sl.stream) == hipSuccess;
            *used_graph = ok_launch;
        } else {
            // direct launches (graph capture unavailable)
            ok_launch = prepare_rates_batch(sm.dev, prec) == KX_OK &&
                        prepare_transport_batch(sm.dev, prec) == KX_OK &&
                        launch_zero(sl.d_counter, kBatchCounters, sl.stream) == KX_OK &&
                        launch_rates_batch(sm.dev, sl.d_wl, sl.d_counter, prec, kRatesBatchGrid,
                                           sl.stream) == KX_OK &&
                        (!(ops & KX_OP_TRANSPORT) ||
                         launch_transport_batch(sm.dev, sl.d_wl, sl.d_counter + kXcds, prec,
                                                kTransportBatchGrid, sl.stream) == KX_OK);
        }
    }
    if (ok_launch) ok_launch = hipEventRecord(sl.done, sl.stream) == hipSuccess;
    if (!ok_launch) hipStreamSynchronize(sl.stream);  // drained before the slot is reused
    (void)s;
    return ok_launch;
}

// Fail a batch whose launch did not go through.  Called with the lock held.
void fail_batch(kx_server *s, Slot &sl)
{
    for (Req *q : sl.reqs) {
        q->state = KX_REQ_FAILED;
        q->t_done = now_s();
        s->in_flight--;
        s->stats.failed++;
    }
    sl.reqs.clear();
    sl.busy = false;
    s->cv_done.notify_all();
}

void scheduler(kx_server *s)
{
    if (!s->simulate) hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        const double t = now_s();
        // 1. retire finished batches
        bool any_busy = false;
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            bool done = false, failed = false;
            if (s->simulate) {
                done = t >= sl.sim_done_at;
            } else {
                const hipError_t e = hipEventQuery(sl.done);
                done = e != hipErrorNotReady;
                failed = done && e != hipSuccess;
            }
            if (!done) {
                any_busy = true;
                continue;
            }
            for (Req *q : sl.reqs) {
                q->state = failed ? KX_REQ_FAILED : KX_REQ_DONE;
                q->t_done = t;
                s->in_flight--;
                if (failed)
                    s->stats.failed++;
                else
                    s->stats.completed++;
            }
            sl.reqs.clear();
            sl.busy = false;
            s->cv_done.notify_all();
        }
        if (s->stop && !any_busy) break;
        if (!s->stop) {
            // 2. admit in arrival order (strict FIFO: no request overtakes an
            // older one that is waiting for memory)
            while (!s->pending.empty() && s->in_flight < s->max_slots) {
                Req *q = s->pending.front();
                size_t off = 0;
                if (q->bytes && !s->arena.alloc(q->bytes, &off)) break;
                q->off = off;
                q->has_mem = q->bytes > 0;
                place_outputs(s, q);
                q->state = KX_REQ_ADMITTED;
                q->t_admit = t;
                s->pending.pop_front();
                s->admitted.push_back(q);
                s->in_flight++;
            }
            // 3. one batch per idle stream, oldest group first; a big batch
            // waits while another big batch runs (younger groups' small batches
            // may go ahead of it)
            for (Slot &sl : s->slots) {
                if (sl.busy || s->admitted.empty()) continue;
                bool big_running = false;
                for (const Slot &o : s->slots) big_running = big_running || (o.busy && o.big);
                const kx_mech *m = nullptr;
                int prec = 0;
                std::vector<std::pair<const kx_mech *, int>> tried;
                for (const Req *q : s->admitted) {
                    const std::pair<const kx_mech *, int> g{q->r.mech, q->r.precision};
                    if (std::find(tried.begin(), tried.end(), g) != tried.end()) continue;
                    tried.push_back(g);
                    int64_t pts = 0;
                    int cnt = 0;
                    for (const Req *o : s->admitted)
                        if (cnt < kMaxBatch && o->r.mech == g.first && o->r.precision == g.second) {
                            pts += o->r.n;
                            ++cnt;
                        }
                    if (pts < kBigBatchPoints || !big_running) {
                        m = g.first;
                        prec = g.second;
                        break;
                    }
                }
                if (!m) break;  // only big batches are waiting, behind a big one
                std::vector<Req *> batch, rest;
                for (Req *q : s->admitted) {
                    if ((int)batch.size() < kMaxBatch && q->r.mech == m && q->r.precision == prec)
                        batch.push_back(q);
                    else
                        rest.push_back(q);
                }
                s->admitted.swap(rest);
                begin_batch(s, sl, batch);
                any_busy = true;
                if (s->simulate) continue;
                // resident mechanisms are never removed, so the record stays
                // valid (map nodes do not move); the slot's graphs are read and
                // filed under the lock only
                const ServedMech &sm = s->mechs.at(m);
                int ops = 0;
                for (Req *q : batch) ops |= q->r.ops;
                const GraphKey key{m->uid, prec, ops};
                auto git = sl.graphs.find(key);
                hipGraphExec_t graph = git == sl.graphs.end() ? nullptr : git->second;
                lk.unlock();
                bool used_graph = false;
                hipGraphExec_t new_graph = nullptr;
                const bool launched = enqueue_batch(s, sl, sm, graph, &new_graph, &used_graph);
                lk.lock();
                if (new_graph && !sl.graphs.emplace(key, new_graph).second)
                    hipGraphExecDestroy(new_graph);
                if (used_graph) s->stats.graph_launches++;
                if (!launched) fail_batch(s, sl);
            }
        }
        // Nothing running and nothing launchable: requests still queued wait for
        // memory or slots, which only kx_release / kx_cancel / kx_submit free or
        // change, and those notify.
        const bool idle = !any_busy && s->admitted.empty();
        if (idle && !s->stop)
            s->cv_sched.wait(lk);
        else
            s->cv_sched.wait_for(lk, std::chrono::microseconds(20));
    }
}

kx_server_stats snapshot(kx_server *s)
{
    kx_server_stats st = s->stats;
    st.queued = (int64_t)s->pending.size();
    st.in_flight = s->in_flight;
    st.arena_in_use = (int64_t)s->arena.used();
    st.arena_capacity = (int64_t)s->arena.capacity();
    st.resident_mechs = (int64_t)s->mechs.size();
    st.resident_bytes = (int64_t)s->resident_bytes;
    return st;
}

void fill_result(const Req *q, kx_result *res)
{
    if (!res) return;
    std::memset(res, 0, sizeof *res);
    res->state = q->state;
    const bool out = q->state == KX_REQ_DONE;
    res->wdot = out ? q->wdot : nullptr;
    res->mu = out ? q->mu : nullptr;
    res->lambda = out ? q->lam : nullptr;
    res->Dmix = out ? q->Dmix : nullptr;
    res->t_arrival = q->t_arrival;
    res->t_admit = q->t_admit;
    res->t_launch = q->t_launch;
    res->t_done = q->t_done;
}

bool finished(int state)
{
    return state == KX_REQ_DONE || state == KX_REQ_CANCELLED || state == KX_REQ_FAILED;
}

}  // namespace
}  // namespace kx

extern "C" {

double kx_server_clock(void) { return now_s(); }

kx_status kx_server_create(int device, int64_t hbm_budget, int32_t max_slots, int32_t flags,
                           kx_server **out)
{
    if (!out) return fail(KX_EINVAL, "kx_server_create: out is NULL");
    *out = nullptr;
    if (hbm_budget <= 0 || max_slots <= 0)
        return fail(KX_EINVAL, "kx_server_create: budget and slots must be > 0");
    kx_server *s = new kx_server;
    s->device = device;
    s->simulate = (flags & KX_SERVER_SIMULATE) != 0;
    s->max_slots = max_slots;
    s->arena = Arena((size_t)hbm_budget & ~size_t(255));
    if (!s->simulate) {
        int prev = 0;
        hipGetDevice(&prev);
        hipError_t e = hipSetDevice(device);
        bool okc = e == hipSuccess;
        if (okc) okc = hipMalloc((void **)&s->arena_base, (size_t)hbm_budget) == hipSuccess;
        for (Slot &sl : s->slots) {
            if (!okc) break;
            okc = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
                  hipMalloc((void **)&sl.d_wl, sizeof(WorkList)) == hipSuccess &&
                  hipMalloc((void **)&sl.d_counter, kBatchCounters * sizeof(int)) == hipSuccess &&
                  hipHostMalloc((void **)&sl.h_wl, sizeof(WorkList), hipHostMallocDefault) ==
                      hipSuccess;
        }
        hipSetDevice(prev);
        if (!okc) {
            for (Slot &sl : s->slots) {
                if (sl.stream) hipStreamDestroy(sl.stream);
                if (sl.done) hipEventDestroy(sl.done);
                if (sl.d_wl) hipFree(sl.d_wl);
                if (sl.d_counter) hipFree(sl.d_counter);
                if (sl.h_wl) hipHostFree(sl.h_wl);
            }
            if (s->arena_base) hipFree(s->arena_base);
            delete s;
            return fail(KX_ENOMEM, "kx_server_create: device resources unavailable");
        }
    }
    s->thread = std::thread(scheduler, s);
    *out = s;
    return ok();
}

kx_status kx_server_destroy(kx_server *s)
{
    if (!s) return ok();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (Req *q : s->pending) {
            q->state = KX_REQ_CANCELLED;
            s->stats.cancelled++;
        }
        for (Req *q : s->admitted) {
            q->state = KX_REQ_CANCELLED;
            s->stats.cancelled++;
            s->in_flight--;
        }
        s->pending.clear();
        s->admitted.clear();
    }
    s->cv_sched.notify_all();
    s->thread.join();
    s->cv_done.notify_all();
    if (!s->simulate) {
        int prev = 0;
        hipGetDevice(&prev);
        hipSetDevice(s->device);
        for (Slot &sl : s->slots) {
            hipStreamSynchronize(sl.stream);
            for (auto &g : sl.graphs) hipGraphExecDestroy(g.second);
            hipStreamDestroy(sl.stream);
            hipEventDestroy(sl.done);
            hipFree(sl.d_wl);
            hipFree(sl.d_counter);
            hipHostFree(sl.h_wl);
        }
        hipFree(s->arena_base);
        hipSetDevice(prev);
    }
    for (auto &kv : s->reqs) delete kv.second;
    delete s;
    return ok();
}

kx_status kx_server_add_mech(kx_server *s, const kx_mech *m)
{
    if (!s || !m) return fail(KX_EINVAL, "kx_server_add_mech: NULL argument");
    if (!s->simulate && (!m->blob || m->device != s->device))
        return fail(KX_EINVAL, "kx_server_add_mech: mechanism has no tables on the server's device");
    if (m->dev.nq > 0)
        return fail(KX_EUNSUPPORTED, "kx_server_add_mech: mechanisms with QSS species are not served");
    std::lock_guard<std::mutex> add_lk(s->add_mu);
    const size_t bytes = round256((size_t)m->bytes);
    size_t off = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(KX_EINVAL, "kx_server_add_mech: server is shutting down");
        if (s->mechs.count(m)) return ok();
        if (!s->arena.alloc(bytes, &off))
            return fail(KX_ENOMEM, "kx_server_add_mech: the mechanism's tables (" +
                                       std::to_string(bytes) + " bytes) do not fit in the "
                                       "server's free HBM budget");
    }
    ServedMech sm;
    sm.off = off;
    sm.bytes = bytes;
    sm.dev = m->dev;
    std::vector<std::pair<Slot *, std::pair<GraphKey, hipGraphExec_t>>> graphs;
    kx_status st = KX_OK;
    if (!s->simulate) {
        int prev = 0;
        hipGetDevice(&prev);
        hipError_t e = hipSetDevice(s->device);
        if (e != hipSuccess) st = hip_fail(e, "kx_server_add_mech: hipSetDevice");
        char *dst = s->arena_base + off;
        if (st == KX_OK &&
            (e = hipMemcpy(dst, m->blob, (size_t)m->bytes, hipMemcpyDeviceToDevice)) != hipSuccess)
            st = hip_fail(e, "kx_server_add_mech: table copy");
        if (st == KX_OK && !rebase_tables(m, dst, &sm.dev))
            st = fail(KX_EINVAL, "kx_server_add_mech: internal error: table pointers not moved");
        // every (stream, precision, ops) graph of this mechanism, captured now
        hipStream_t cap = nullptr;
        if (st == KX_OK && (e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess)
            st = hip_fail(e, "kx_server_add_mech: hipStreamCreate");
        for (Slot &sl : s->slots)
            for (int prec : {(int)KX_FP64, (int)KX_MIXED})
                for (int ops : {(int)KX_OP_RATES, (int)(KX_OP_RATES | KX_OP_TRANSPORT)}) {
                    if (st != KX_OK) break;
                    hipGraphExec_t ex = nullptr;
                    st = build_graph(sm.dev, sl, prec, ops, cap, &ex);
                    if (st == KX_OK) graphs.push_back({&sl, {GraphKey{m->uid, prec, ops}, ex}});
                }
        if (cap) hipStreamDestroy(cap);
        hipSetDevice(prev);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (st != KX_OK) {
        for (auto &g : graphs) hipGraphExecDestroy(g.second.second);
        s->arena.release(off, bytes);
        return st;
    }
    for (auto &g : graphs) g.first->graphs.emplace(g.second.first, g.second.second);
    s->mechs.emplace(m, sm);
    s->resident_bytes += bytes;
    return ok();
}

kx_status kx_submit(kx_server *s, const kx_request *r, kx_ticket *ticket)
{
    if (!s || !r || !ticket) return fail(KX_EINVAL, "kx_submit: NULL argument");
    if (!r->mech) return fail(KX_EINVAL, "kx_submit: mech is NULL");
    if (r->n < 0) return fail(KX_EINVAL, "kx_submit: n < 0");
    if (!(r->ops & KX_OP_RATES) || (r->ops & ~(KX_OP_RATES | KX_OP_TRANSPORT)))
        return fail(KX_EINVAL, "kx_submit: ops must be KX_OP_RATES [| KX_OP_TRANSPORT]");
    if (r->precision != KX_FP64 && r->precision != KX_MIXED)
        return fail(KX_EINVAL, "kx_submit: unknown precision");
    if (!s->simulate && r->n > 0 && (!r->T || !r->p || !r->Y))
        return fail(KX_EINVAL, "kx_submit: NULL input array");
    if (!s->simulate && r->mech->device != s->device)
        return fail(KX_EINVAL, "kx_submit: mechanism lives on another device");
    if (r->mech->dev.nq > 0)
        return fail(KX_EUNSUPPORTED, "kx_submit: mechanisms with QSS species are not served");
    const size_t bytes = r->n > 0 ? footprint(*r, r->mech->n_species) : 0;
    Req *q = new Req;
    q->r = *r;
    q->bytes = bytes;
    q->t_arrival = r->arrival_s >= 0 ? r->arrival_s : now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete q;
            return fail(KX_EINVAL, "kx_submit: server is shutting down");
        }
        if (!s->mechs.count(r->mech)) {
            delete q;
            return fail(KX_EINVAL, "kx_submit: mechanism is not resident on this server "
                                   "(kx_server_add_mech)");
        }
        if (bytes > s->arena.capacity() - s->resident_bytes) {
            delete q;
            return fail(KX_ENOMEM, "kx_submit: request outputs exceed the server's HBM budget "
                                   "left after its resident mechanisms");
        }
        q->id = s->next_id++;
        s->reqs[q->id] = q;
        s->stats.submitted++;
        if (r->n == 0) {
            q->state = KX_REQ_DONE;
            q->t_admit = q->t_launch = q->t_done = now_s();
            s->stats.completed++;
        } else {
            s->pending.push_back(q);
        }
        *ticket = q->id;
    }
    s->cv_sched.notify_all();
    return ok();
}

kx_status kx_poll(kx_server *s, kx_ticket t, kx_result *res)
{
    if (!s) return fail(KX_EINVAL, "kx_poll: server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(t);
    if (it == s->reqs.end()) return fail(KX_EINVAL, "kx_poll: unknown ticket");
    fill_result(it->second, res);
    return ok();
}

kx_status kx_wait(kx_server *s, kx_ticket t, double timeout_s, kx_result *res)
{
    if (!s) return fail(KX_EINVAL, "kx_wait: server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(t);
    if (it == s->reqs.end()) return fail(KX_EINVAL, "kx_wait: unknown ticket");
    Req *q = it->second;
    auto pred = [&] { return finished(q->state); };
    if (timeout_s < 0) {
        s->cv_done.wait(lk, pred);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
        fill_result(q, res);
        return fail(KX_EAGAIN, "kx_wait: timed out");
    }
    fill_result(q, res);
    return ok();
}

kx_status kx_cancel(kx_server *s, kx_ticket t)
{
    if (!s) return fail(KX_EINVAL, "kx_cancel: server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(t);
        if (it == s->reqs.end()) return fail(KX_EINVAL, "kx_cancel: unknown ticket");
        Req *q = it->second;
        if (q->state == KX_REQ_QUEUED) {
            s->pending.erase(std::find(s->pending.begin(), s->pending.end(), q));
        } else if (q->state == KX_REQ_ADMITTED) {
            s->admitted.erase(std::find(s->admitted.begin(), s->admitted.end(), q));
            s->in_flight--;
            if (q->has_mem) {
                s->arena.release(q->off, q->bytes);
                q->has_mem = false;
            }
        } else {
            return fail(KX_EAGAIN, "kx_cancel: request already launched or finished");
        }
        q->state = KX_REQ_CANCELLED;
        q->t_done = now_s();
        s->stats.cancelled++;
    }
    s->cv_done.notify_all();
    s->cv_sched.notify_all();
    return ok();
}

kx_status kx_result_copy(kx_server *s, kx_ticket t, double *wdot, double *mu, double *lam,
                         double *Dmix, hipStream_t stream)
{
    if (!s) return fail(KX_EINVAL, "kx_result_copy: server is NULL");
    if (s->simulate) return fail(KX_EUNSUPPORTED, "kx_result_copy: simulated server");
    Req *q = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(t);
        if (it == s->reqs.end()) return fail(KX_EINVAL, "kx_result_copy: unknown ticket");
        q = it->second;
        if (q->state != KX_REQ_DONE) return fail(KX_EAGAIN, "kx_result_copy: not done");
    }
    const size_t ns = (size_t)q->r.mech->n_species, n = (size_t)q->r.n;
    const bool tr = (q->r.ops & KX_OP_TRANSPORT) != 0;
    hipError_t e = hipSuccess;
    if (wdot && e == hipSuccess)
        e = hipMemcpyAsync(wdot, q->wdot, ns * n * 8, hipMemcpyDefault, stream);
    if (tr && mu && e == hipSuccess)
        e = hipMemcpyAsync(mu, q->mu, n * 8, hipMemcpyDefault, stream);
    if (tr && lam && e == hipSuccess)
        e = hipMemcpyAsync(lam, q->lam, n * 8, hipMemcpyDefault, stream);
    if (tr && Dmix && e == hipSuccess)
        e = hipMemcpyAsync(Dmix, q->Dmix, ns * n * 8, hipMemcpyDefault, stream);
    if (e != hipSuccess) return hip_fail(e, "kx_result_copy");
    return ok();
}

kx_status kx_release(kx_server *s, kx_ticket t)
{
    if (!s) return fail(KX_EINVAL, "kx_release: server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(t);
        if (it == s->reqs.end()) return fail(KX_EINVAL, "kx_release: unknown ticket");
        Req *q = it->second;
        if (!finished(q->state)) return fail(KX_EAGAIN, "kx_release: request not finished");
        if (q->has_mem) s->arena.release(q->off, q->bytes);
        s->reqs.erase(it);
        delete q;
    }
    s->cv_sched.notify_all();
    return ok();
}

kx_status kx_server_stats_get(kx_server *s, kx_server_stats *st)
{
    if (!s || !st) return fail(KX_EINVAL, "kx_server_stats_get: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *st = snapshot(s);
    return ok();
}

}  // extern "C"
