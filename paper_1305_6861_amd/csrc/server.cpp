// Served execution: a request loop with admission by device footprint and
// continuous batching by time slice.
//
// The paper's master hands spin blocks to whichever compute node is free
// and learns that a block is finished only after the superposition process
// has integrated it, which bounds what is in flight (sections 5.3.2, 6.3 and
// 7.3.1).  The MI355X analogue: requests are compiled at submission, queued,
// and admitted while their device footprint fits under a cap.  Each
// scheduler iteration advances every admitted request by one time slice in
// one batched round (persistent kernel + finalize, batch.cpp), so requests
// that arrive while long ones run join at the next iteration instead of
// waiting for them to finish.  Spin state stays in HBM between slices.
// A request is bitwise the same alone or in any mix: its tiling and slice
// plan depend only on itself.
//
// The loop keeps two short iterations in flight: the slice plan of every request
// is fixed at submission, so the host knows which requests an iteration
// finishes without waiting for the device, and plans, uploads and launches
// iteration i + 1 while iteration i runs.  Each in-flight iteration has its
// own launch records, staging buffers and events (two slots, used in turn);
// the host waits on the device only to reuse a slot, whose completed
// iteration it then retires (finished requests are signalled and their
// memory returns to the pool).  An iteration's launches are replayed from a
// HIP graph of the slot, one per launch topology (the kernels of its
// spins-per-lane classes and finalize passes); a known topology only gets
// its kernel-node arguments updated, and the slot's previous replay has
// completed by then.  The graph holds kernel nodes only: the queue counters
// are zeroed by the records' upload.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/parspin.h"
#include "batch.h"
#include "ps_runtime.h"

namespace ps {

using Clock = std::chrono::steady_clock;

enum ReqState : int32_t { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2, RQ_FAILED = 3, RQ_CANCELLED = 4 };

struct Request {
    uint64_t ticket = 0;
    ReqPlan plan;
    int32_t state = RQ_QUEUED;
    ps_status status = PS_OK;
    bool cancel = false;
    size_t enqueued = 0;               // slices launched so far
    size_t completed = 0;              // slices whose iteration has completed
    int inflight = 0;                  // iterations in flight that hold one of its slices
    bool tables_up = false;            // op tables uploaded
    void* mem = nullptr;
    size_t mem_bytes = 0;
    size_t footprint = 0;
    bool large = false;                // see kLargeWork
    double t_submit = 0, t_admit = -1, t_done = -1;
    double t_kernel = 0;               // device time of the iterations it ran in
    std::string error;
    // device work of the request: one slice per iteration (an empty object
    // is one zero fill)
    size_t n_slices() const {
        if (plan.prog.n_samples == 0) return 0;
        return plan.obj.n_spins > 0 ? plan.prog.slices.size() : 1;
    }
};

// Requests of at least this many spin-steps (a few ms of the whole device)
// run one at a time: sharing the device among several of them only delays
// them all, while small requests keep joining every iteration beside the
// one that runs.
constexpr double kLargeWork = 2.5e10;

// An iteration of at most this many spin-steps (about a millisecond of the
// device) has the next one launched before it completes.
constexpr double kAheadWork = 1e10;

// Elementary intervals per spin in slice k of a request (ps_count's unit).
static int64_t slice_steps(const ReqPlan& p, size_t k) {
    if (k >= p.prog.slices.size()) return 0;
    const Slice& sl = p.prog.slices[k];
    int64_t w = 0;
    for (int64_t i = sl.op_begin; i < sl.op_end; ++i) {
        const Op& op = p.prog.ops[i];
        w += (op.kind == OP_ADC || op.kind == OP_ADCT || op.kind == OP_SHAPE) ? op.n : 1;
    }
    return w;
}

// Device memory for admitted requests: freed blocks are kept and reused.
struct Pool {
    std::multimap<size_t, void*> free_blocks;
    bool stand_in = false;             // scheduler test: addresses that are never dereferenced
    uintptr_t next_token = 0;
    ps_status get(size_t n, void** out) {
        if (stand_in) {
            next_token += (n + 4095) / 4096 * 4096 + 4096;
            *out = reinterpret_cast<void*>(next_token);
            return PS_OK;
        }
        auto it = free_blocks.lower_bound(n);
        if (it != free_blocks.end() && it->first <= 2 * n) {
            *out = it->second;
            free_blocks.erase(it);
            return PS_OK;
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) return fail(PS_E_NO_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
        *out = p;
        return PS_OK;
    }
    void put(void* p, size_t n) { if (p && !stand_in) free_blocks.emplace(n, p); }
    void release() {
        for (auto& kv : free_blocks) (void)hipFree(kv.second);
        free_blocks.clear();
    }
};

// A HIP graph of one launch topology (the kernels of an iteration, in order).
struct RoundGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        nodes.clear();
    }
};

// Resources of one in-flight iteration.
struct IterSlot {
    DevBuf records;
    HostBuf staging_rec, staging_tab;
    hipEvent_t ev_start = nullptr, ev_end = nullptr;   // timing of its kernels
    hipEvent_t done = nullptr;                         // completion of all its work
    bool busy = false;
    bool timed = false;                                // ev_start / ev_end recorded
    double work = 0.0;                                 // spin-steps of its slices
    Clock::time_point stand_in_done;                   // scheduler test: completion instant
    bool stand_in_fails = false;                       // scheduler test: injected device error
    std::vector<std::shared_ptr<Request>> members;     // requests with work in it
    std::map<std::vector<const void*>, RoundGraph> graphs;
    std::vector<unsigned char> img;                    // host image of its records
};

struct Server {
    Ctx* ctx = nullptr;
    std::thread thr;
    std::mutex mu;
    std::condition_variable wake, changed;
    std::deque<std::shared_ptr<Request>> queue;
    std::vector<std::shared_ptr<Request>> active;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_ticket = 1;
    size_t used = 0;
    bool stop = false;
    Clock::time_point t0;
    // device side, touched by the scheduler thread only
    hipStream_t stream = nullptr;
    IterSlot slots[2];
    int next_slot = 0;
    std::deque<int> inflight;          // slots in launch order
    Pool pool;
    // counters
    uint64_t iterations = 0;

    bool stand_in = false;             // scheduler-test context (no device)
    int64_t launched = 0;              // iterations launched so far

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void loop();
    ps_status stand_in_launch(IterSlot& sl, std::vector<ReqPlan*>& plans, std::vector<size_t>& first,
                              std::vector<double*>& zero_fill, std::vector<int64_t>& zero_n);
    void finish(const std::shared_ptr<Request>& r, int32_t state, ps_status st, const std::string& err);
    ps_status launch_iteration(IterSlot& sl, std::vector<ReqPlan*>& fresh, std::vector<ReqPlan*>& plans,
                               std::vector<size_t>& first, std::vector<double*>& zero_fill,
                               std::vector<int64_t>& zero_n);
    ps_status launch_nodes(IterSlot& sl, std::vector<KernelNode>& nodes);
    void retire_oldest(bool block, ps_status* err);
};

void Server::finish(const std::shared_ptr<Request>& r, int32_t state, ps_status st, const std::string& err) {
    r->state = state;
    r->status = st;
    r->error = err;
    r->t_done = now();
    if (r->mem) {
        pool.put(r->mem, r->mem_bytes);
        r->mem = nullptr;
        used -= r->footprint;
    }
}

// Replay (or build) the slot's graph for this launch topology.
ps_status Server::launch_nodes(IterSlot& sl, std::vector<KernelNode>& nodes) {
    if (nodes.empty()) return PS_OK;
    hipError_t e;
    if (ctx->cfg.flags & PS_CFG_SERVE_DIRECT) {
        for (KernelNode& n : nodes)
            if ((e = n.launch(stream)) != hipSuccess) return hip_fail(e, "server launch");
        return PS_OK;
    }
    std::vector<const void*> key;
    for (const KernelNode& n : nodes) key.push_back(n.func);
    RoundGraph& g = sl.graphs[key];
    if (!g.exec) {
        e = hipGraphCreate(&g.graph, 0);
        for (size_t i = 0; i < nodes.size() && e == hipSuccess; ++i) {
            const hipKernelNodeParams p = nodes[i].params();
            hipGraphNode_t node = nullptr;
            e = hipGraphAddKernelNode(&node, g.graph, i ? &g.nodes.back() : nullptr, i ? 1 : 0, &p);
            if (e == hipSuccess) g.nodes.push_back(node);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            g.release();
            sl.graphs.erase(key);
            return hip_fail(e, "server graph");
        }
    } else {
        for (size_t i = 0; i < nodes.size(); ++i) {
            const hipKernelNodeParams p = nodes[i].params();
            if ((e = hipGraphExecKernelNodeSetParams(g.exec, g.nodes[i], &p)) != hipSuccess)
                return hip_fail(e, "server graph update");
        }
    }
    if ((e = hipGraphLaunch(g.exec, stream)) != hipSuccess) return hip_fail(e, "server graph launch");
    return PS_OK;
}

// Scheduler test: the iteration's slices write the stand-in pattern into the
// requests' (host) signals right away; the iteration completes
// iteration_seconds after its launch (after the previous one).
ps_status Server::stand_in_launch(IterSlot& sl, std::vector<ReqPlan*>& plans, std::vector<size_t>& first,
                                  std::vector<double*>& zero_fill, std::vector<int64_t>& zero_n) {
    for (size_t i = 0; i < zero_fill.size(); ++i)
        for (int64_t j = 0; j < zero_n[i]; ++j) zero_fill[i][j] = 0.0;
    for (size_t i = 0; i < plans.size(); ++i) {
        const ReqPlan& p = *plans[i];
        const Slice& slc = p.prog.slices[first[i]];
        for (int64_t n = slc.sample_begin; n < slc.sample_begin + slc.n_samples; ++n) {
            p.signal[2 * n] = (double)p.obj.n_spins + (double)n;
            p.signal[2 * n + 1] = (double)first[i];
        }
    }
    const auto dur = std::chrono::duration_cast<Clock::duration>(
        std::chrono::duration<double>(ctx->test_backend.iteration_seconds));
    Clock::time_point start = Clock::now();
    if (!inflight.empty()) start = std::max(start, slots[inflight.back()].stand_in_done);
    sl.stand_in_done = start + dur;
    sl.stand_in_fails = ctx->test_backend.fail_iteration == launched;
    sl.timed = !plans.empty();
    return PS_OK;
}

// Upload the fresh requests' tables and this iteration's records through the
// slot's staging, then launch: zero fills of empty objects, the round's
// graph, with the timing and completion events around them.
ps_status Server::launch_iteration(IterSlot& sl, std::vector<ReqPlan*>& fresh, std::vector<ReqPlan*>& plans,
                                   std::vector<size_t>& first, std::vector<double*>& zero_fill,
                                   std::vector<int64_t>& zero_n) {
    ps_status st = PS_OK;
    hipError_t e;
    if (!fresh.empty() && (st = upload_tables(fresh, sl.staging_tab, 0, stream)) != PS_OK) return st;
    for (size_t i = 0; i < zero_fill.size(); ++i)
        if ((e = launch_fill_zero(zero_fill[i], zero_n[i], stream)) != hipSuccess) return hip_fail(e, "fill");
    sl.timed = false;
    if (!plans.empty()) {
        std::vector<size_t> count(plans.size(), 1);
        std::vector<RoundImage> rounds;
        if ((st = build_rounds(ctx, plans, first, count, &sl.img, &rounds)) != PS_OK) return st;
        if (!sl.img.empty()) {
            if ((st = sl.records.reserve(sl.img.size())) != PS_OK) return st;
            if ((st = sl.staging_rec.reserve(sl.img.size())) != PS_OK) return st;
            std::memcpy(sl.staging_rec.ptr, sl.img.data(), sl.img.size());
            if ((e = hipMemcpyAsync(sl.records.ptr, sl.staging_rec.ptr, sl.img.size(), hipMemcpyHostToDevice,
                                    stream)) != hipSuccess)
                return hip_fail(e, "hipMemcpyAsync(server records)");
            std::vector<KernelNode> nodes;
            for (const RoundImage& R : rounds)
                if ((st = round_nodes(ctx, R, reinterpret_cast<unsigned char*>(sl.records.ptr), &nodes)) != PS_OK)
                    return st;
            if ((e = hipEventRecord(sl.ev_start, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
            if ((st = launch_nodes(sl, nodes)) != PS_OK) return st;
            if ((e = hipEventRecord(sl.ev_end, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
            sl.timed = true;
        }
    }
    if ((e = hipEventRecord(sl.done, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return PS_OK;
}

// Retire the oldest in-flight iteration once it has completed (block: wait
// for it); its members advance, and those whose last slice it ran finish.
void Server::retire_oldest(bool block, ps_status* err) {
    if (inflight.empty()) return;
    IterSlot& sl = slots[inflight.front()];
    ps_status st = PS_OK;
    double iter_kernel_s = 0.0;
    if (stand_in) {
        if (!block && Clock::now() < sl.stand_in_done) return;
        std::this_thread::sleep_until(sl.stand_in_done);
        if (sl.stand_in_fails) st = fail(PS_E_DEVICE, "injected device error (scheduler test)");
        else if (sl.timed) iter_kernel_s = ctx->test_backend.iteration_seconds;
    } else {
        hipError_t e = block ? hipEventSynchronize(sl.done) : hipEventQuery(sl.done);
        if (e == hipErrorNotReady) return;
        if (e != hipSuccess) st = hip_fail(e, "server iteration");
        if (st == PS_OK && sl.timed) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, sl.ev_start, sl.ev_end) == hipSuccess) iter_kernel_s = 1e-3 * ms;
        }
    }
    const std::string msg = st == PS_OK ? "" : ps_last_error();
    {
        std::lock_guard<std::mutex> lk(mu);
        ++iterations;
        for (auto& r : sl.members) {
            r->inflight -= 1;
            r->completed += 1;
            if (r->plan.obj.n_spins > 0) r->t_kernel += iter_kernel_s;
            if (r->state >= RQ_DONE) continue;
            bool done = false;
            if (st != PS_OK) { finish(r, RQ_FAILED, st, msg); done = true; }
            else if (r->completed >= r->n_slices()) { finish(r, RQ_DONE, PS_OK, ""); done = true; }
            else if (r->cancel && r->inflight == 0) { finish(r, RQ_CANCELLED, PS_E_CANCELLED, "cancelled"); done = true; }
            if (done) active.erase(std::find(active.begin(), active.end(), r));
        }
        changed.notify_all();
    }
    sl.members.clear();
    sl.busy = false;
    inflight.pop_front();
    if (err && st != PS_OK) *err = st;
}

void Server::loop() {
    if (!stand_in) (void)hipSetDevice(ctx->cfg.device);
    for (;;) {
        // retire what the device has completed, without waiting
        for (size_t n = inflight.size(); n > 0; --n) retire_oldest(false, nullptr);
        std::vector<std::shared_ptr<Request>> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            auto runnable = [&] {
                for (auto& r : active)
                    if (r->enqueued < r->n_slices() && !r->cancel) return true;
                    else if (r->cancel && r->inflight == 0) return true;
                return false;
            };
            if (inflight.empty())
                wake.wait(lk, [&] { return stop || !queue.empty() || runnable(); });
            if (stop) break;
            // cancellations of running requests take effect between
            // iterations: no further slice is launched, and the request
            // finishes once its slices in flight have completed
            for (auto it = active.begin(); it != active.end();) {
                if ((*it)->cancel && (*it)->inflight == 0) {
                    finish(*it, RQ_CANCELLED, PS_E_CANCELLED, "cancelled");
                    it = active.erase(it);
                } else {
                    ++it;
                }
            }
            // admission in submission order while the footprint fits; a large
            // request waits (without holding up the small ones behind it)
            // while another large one runs
            bool large_active = false;
            for (auto& r : active) large_active = large_active || r->large;
            for (auto it = queue.begin(); it != queue.end();) {
                auto& r = *it;
                if (r->cancel) {
                    finish(r, RQ_CANCELLED, PS_E_CANCELLED, "cancelled");
                    it = queue.erase(it);
                    continue;
                }
                if (r->large && large_active) { ++it; continue; }
                if (used + r->footprint > (size_t)ctx->cfg.max_footprint_bytes) break;
                used += r->footprint;
                large_active = large_active || r->large;
                admitted.push_back(r);
                it = queue.erase(it);
            }
            changed.notify_all();
        }
        // place newly admitted requests
        for (auto& r : admitted) {
            ps_status st = pool.get(std::max<size_t>(r->plan.device_bytes(), 256), &r->mem);
            std::lock_guard<std::mutex> lk(mu);
            if (st != PS_OK) {
                used -= r->footprint;
                finish(r, RQ_FAILED, st, ps_last_error());
                changed.notify_all();
                continue;
            }
            r->mem_bytes = std::max<size_t>(r->plan.device_bytes(), 256);
            r->plan.bind(reinterpret_cast<unsigned char*>(r->mem));
            r->state = RQ_RUNNING;
            r->t_admit = now();
            if (r->n_slices() == 0) {            // no samples: nothing to run
                finish(r, RQ_DONE, PS_OK, "");
                changed.notify_all();
                continue;
            }
            active.push_back(r);
        }
        // the next iteration: one slice of every running request
        std::vector<std::shared_ptr<Request>> members;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto& r : active)
                if (!r->cancel && r->enqueued < r->n_slices()) members.push_back(r);
        }
        if (members.empty()) {
            if (!inflight.empty()) retire_oldest(true, nullptr);
            continue;
        }
        // Launch ahead only while iterations are short: there the host's
        // retire-plan-launch gap would idle the device for a noticeable part
        // of each iteration.  A long iteration first completes, so that a
        // request arriving meanwhile joins the very next one.
        if (!inflight.empty() &&
            ((ctx->cfg.flags & PS_CFG_SERVE_DIRECT) || slots[inflight.back()].work > kAheadWork)) {
            retire_oldest(true, nullptr);
            continue;
        }
        if (slots[next_slot].busy) retire_oldest(true, nullptr);   // two in flight: wait for the older
        IterSlot& sl = slots[next_slot];
        std::vector<ReqPlan*> fresh, plans;
        std::vector<size_t> first;
        std::vector<double*> zero_fill;
        std::vector<int64_t> zero_n;
        sl.work = 0.0;
        for (auto& r : members) {
            ReqPlan& p = r->plan;
            sl.work += (double)p.obj.n_spins * (double)slice_steps(p, r->enqueued);
            if (p.obj.n_spins == 0) {
                zero_fill.push_back(p.signal);
                zero_n.push_back(2 * p.prog.n_samples);
                continue;
            }
            if (!r->tables_up) fresh.push_back(&p);
            plans.push_back(&p);
            first.push_back(r->enqueued);
        }
        ps_status st = stand_in ? stand_in_launch(sl, plans, first, zero_fill, zero_n)
                                : launch_iteration(sl, fresh, plans, first, zero_fill, zero_n);
        ++launched;
        if (st != PS_OK) {
            // the stream may hold part of the iteration: let it drain, then
            // fail the requests that had work in it
            const std::string msg = ps_last_error();
            if (!stand_in) (void)hipStreamSynchronize(stream);
            while (!inflight.empty()) retire_oldest(true, nullptr);
            std::lock_guard<std::mutex> lk(mu);
            for (auto& r : members) {
                if (r->state >= RQ_DONE) continue;
                finish(r, RQ_FAILED, st, msg);
                active.erase(std::find(active.begin(), active.end(), r));
            }
            changed.notify_all();
            continue;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto& r : members) {
                r->tables_up = true;
                r->enqueued += 1;
                r->inflight += 1;
            }
        }
        sl.members = std::move(members);
        sl.busy = true;
        inflight.push_back(next_slot);
        next_slot ^= 1;
    }
    // the device may still run launched iterations: let them complete
    while (!inflight.empty()) retire_oldest(true, nullptr);
}

void destroy_runtime(Ctx* ctx) {
    Server* s = ctx->server.load(std::memory_order_acquire);
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->wake.notify_all();
    if (s->thr.joinable()) s->thr.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& r : s->active) s->finish(r, RQ_CANCELLED, PS_E_CANCELLED, "context destroyed");
        for (auto& r : s->queue) s->finish(r, RQ_CANCELLED, PS_E_CANCELLED, "context destroyed");
        s->active.clear();
        s->queue.clear();
        s->changed.notify_all();
    }
    for (IterSlot& sl : s->slots) {
        for (auto& kv : sl.graphs) kv.second.release();
        if (sl.ev_start) (void)hipEventDestroy(sl.ev_start);
        if (sl.ev_end) (void)hipEventDestroy(sl.ev_end);
        if (sl.done) (void)hipEventDestroy(sl.done);
        sl.records.release();
        sl.staging_rec.release();
        sl.staging_tab.release();
    }
    if (s->stream) (void)hipStreamDestroy(s->stream);
    s->pool.release();
    delete s;
    ctx->server.store(nullptr, std::memory_order_release);
}

static ps_status ensure_server(Ctx* ctx) {
    if (ctx->server.load(std::memory_order_acquire)) return PS_OK;
    Server* s = new (std::nothrow) Server();
    if (!s) return fail(PS_E_NO_MEMORY, "server allocation");
    s->ctx = ctx;
    s->t0 = Clock::now();
    if (ctx->scheduler_test) {
        s->stand_in = true;
        s->pool.stand_in = true;
        s->thr = std::thread([s] { s->loop(); });
        ctx->server.store(s, std::memory_order_release);
        return PS_OK;
    }
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    for (IterSlot& sl : s->slots) {
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreate(&sl.ev_start);
        if (e == hipSuccess) e = hipEventCreate(&sl.ev_end);
    }
    if (e != hipSuccess) {
        for (IterSlot& sl : s->slots) {
            if (sl.ev_end) (void)hipEventDestroy(sl.ev_end);
            if (sl.ev_start) (void)hipEventDestroy(sl.ev_start);
            if (sl.done) (void)hipEventDestroy(sl.done);
        }
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return hip_fail(e, "server stream/event");
    }
    s->thr = std::thread([s] { s->loop(); });
    ctx->server.store(s, std::memory_order_release);
    return PS_OK;
}

static std::shared_ptr<Request> find(Server* s, uint64_t t) {
    auto it = s->all.find(t);
    return it == s->all.end() ? nullptr : it->second;
}

}  // namespace ps

using namespace ps;

extern "C" {

ps_status ps_submit(ps_ctx* handle, const ps_object* obj, const ps_sequence* seq, double* signal,
                    int64_t n_samples, uint64_t* ticket) {
    clear_error();
    if (!handle || !ticket) return fail(PS_E_INVALID_ARG, "ctx or ticket is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    auto r = std::make_shared<Request>();
    ps_status st;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        std::unique_ptr<DeviceGuard> g;
        if (!ctx->scheduler_test) g.reset(new DeviceGuard(ctx->cfg.device));
        if ((st = ensure_server(ctx)) != PS_OK) return st;
        const int64_t steps = ctx->cfg.max_slice_steps;
        if ((st = plan_request(ctx, obj, seq, n_samples, signal, steps, &r->plan)) != PS_OK) return st;
    }
    r->footprint = r->plan.footprint();
    r->large = (double)r->plan.obj.n_spins * (double)r->plan.prog.n_steps >= kLargeWork;
    if (r->footprint > (size_t)ctx->cfg.max_footprint_bytes)
        return fail(PS_E_TOO_LARGE, "request footprint " + std::to_string(r->footprint) +
                                        " bytes exceeds the cap of " + std::to_string(ctx->cfg.max_footprint_bytes));
    Server* s = ctx->server.load(std::memory_order_acquire);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        r->t_submit = s->now();
        s->queue.push_back(r);
        s->all.emplace(r->ticket, r);
        *ticket = r->ticket;
    }
    s->wake.notify_all();
    return PS_OK;
}

ps_status ps_poll(ps_ctx* handle, uint64_t ticket, int32_t* done) {
    clear_error();
    if (!handle || !done) return fail(PS_E_INVALID_ARG, "ctx or done is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    Server* s = ctx->server.load(std::memory_order_acquire);
    if (!s) return fail(PS_E_INVALID_ARG, "unknown ticket");
    std::lock_guard<std::mutex> lk(s->mu);
    auto r = find(s, ticket);
    if (!r) return fail(PS_E_INVALID_ARG, "unknown ticket");
    *done = r->state >= RQ_DONE ? 1 : 0;
    return PS_OK;
}

ps_status ps_wait(ps_ctx* handle, uint64_t ticket, double timeout_s) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    Server* s = ctx->server.load(std::memory_order_acquire);
    if (!s) return fail(PS_E_INVALID_ARG, "unknown ticket");
    std::unique_lock<std::mutex> lk(s->mu);
    auto r = find(s, ticket);
    if (!r) return fail(PS_E_INVALID_ARG, "unknown ticket");
    auto pred = [&] { return r->state >= RQ_DONE; };
    if (timeout_s < 0) {
        s->changed.wait(lk, pred);
    } else if (!s->changed.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
        return fail(PS_E_NOT_READY, "timed out");
    }
    if (r->status != PS_OK) return fail(r->status, r->error);
    return PS_OK;
}

ps_status ps_cancel(ps_ctx* handle, uint64_t ticket) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    Server* s = ctx->server.load(std::memory_order_acquire);
    if (!s) return fail(PS_E_INVALID_ARG, "unknown ticket");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto r = find(s, ticket);
        if (!r) return fail(PS_E_INVALID_ARG, "unknown ticket");
        if (r->state < RQ_DONE) r->cancel = true;
    }
    s->wake.notify_all();
    return PS_OK;
}

ps_status ps_request_info(ps_ctx* handle, uint64_t ticket, ps_request_info_t* out) {
    clear_error();
    if (!handle || !out) return fail(PS_E_INVALID_ARG, "ctx or out is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    Server* s = ctx->server.load(std::memory_order_acquire);
    if (!s) return fail(PS_E_INVALID_ARG, "unknown ticket");
    std::lock_guard<std::mutex> lk(s->mu);
    auto r = find(s, ticket);
    if (!r) return fail(PS_E_INVALID_ARG, "unknown ticket");
    std::memset(out, 0, sizeof(*out));
    out->state = r->state;
    out->status = r->status;
    out->t_submit = r->t_submit;
    out->t_admit = r->t_admit;
    out->t_done = r->t_done;
    out->n_slices = (int64_t)r->plan.prog.slices.size();
    out->footprint_bytes = (int64_t)r->footprint;
    out->n_spins = r->plan.obj.n_spins;
    out->n_steps_per_spin = r->plan.prog.n_steps;
    out->t_kernel = r->state >= RQ_DONE ? r->t_kernel : -1.0;
    return PS_OK;
}

ps_status ps_stats(ps_ctx* handle, uint64_t ticket, double* t_queue, double* t_kernel, double* t_e2e) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    Server* s = ctx->server.load(std::memory_order_acquire);
    if (!s) return fail(PS_E_INVALID_ARG, "unknown ticket");
    std::lock_guard<std::mutex> lk(s->mu);
    auto r = find(s, ticket);
    if (!r) return fail(PS_E_INVALID_ARG, "unknown ticket");
    const bool done = r->state >= RQ_DONE;
    if (t_queue) *t_queue = r->t_admit >= 0 ? r->t_admit - r->t_submit : -1.0;
    if (t_kernel) *t_kernel = done ? r->t_kernel : -1.0;
    if (t_e2e) *t_e2e = done ? r->t_done - r->t_submit : -1.0;
    return PS_OK;
}

ps_status ps_release(ps_ctx* handle, uint64_t ticket) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    Server* s = ctx->server.load(std::memory_order_acquire);
    if (!s) return fail(PS_E_INVALID_ARG, "unknown ticket");
    std::lock_guard<std::mutex> lk(s->mu);
    auto r = find(s, ticket);
    if (!r) return fail(PS_E_INVALID_ARG, "unknown ticket");
    if (r->state < RQ_DONE) return fail(PS_E_NOT_READY, "request still in flight");
    s->all.erase(ticket);
    return PS_OK;
}

ps_status ps_server_stats(ps_ctx* handle, ps_server_stats_t* out) {
    clear_error();
    if (!handle || !out) return fail(PS_E_INVALID_ARG, "ctx or out is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    std::memset(out, 0, sizeof(*out));
    Server* s = ctx->server.load(std::memory_order_acquire);
    if (!s) return PS_OK;
    std::lock_guard<std::mutex> lk(s->mu);
    out->iterations = (int64_t)s->iterations;
    out->queued = (int64_t)s->queue.size();
    out->running = (int64_t)s->active.size();
    out->footprint_in_use = (int64_t)s->used;
    out->now = s->now();
    return PS_OK;
}

}  // extern "C"
