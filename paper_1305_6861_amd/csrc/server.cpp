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
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
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
    size_t next_slice = 0;
    void* mem = nullptr;
    size_t mem_bytes = 0;
    size_t footprint = 0;
    bool large = false;                // see kLargeWork
    double t_submit = 0, t_admit = -1, t_done = -1;
    double t_kernel = 0;               // device time of the iterations it ran in
    std::string error;
};

// Requests of at least this many spin-steps (a few ms of the whole device)
// run one at a time: sharing the device among several of them only delays
// them all, while small requests keep joining every iteration beside the
// one that runs.
constexpr double kLargeWork = 2.5e10;

// Device memory for admitted requests: freed blocks are kept and reused.
struct Pool {
    std::multimap<size_t, void*> free_blocks;
    ps_status get(size_t n, void** out) {
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
    void put(void* p, size_t n) { if (p) free_blocks.emplace(n, p); }
    void release() {
        for (auto& kv : free_blocks) hipFree(kv.second);
        free_blocks.clear();
    }
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
    hipEvent_t ev = nullptr;
    hipEvent_t ev_start = nullptr, ev_end = nullptr;   // timing of one iteration's kernels
    DevBuf records;
    HostBuf staging_rec, staging_tab;
    Pool pool;
    // counters
    uint64_t iterations = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void loop();
    void finish(const std::shared_ptr<Request>& r, int32_t state, ps_status st, const std::string& err);
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

void Server::loop() {
    hipSetDevice(ctx->cfg.device);
    for (;;) {
        std::vector<std::shared_ptr<Request>> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            wake.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
            if (stop) break;
            // cancellations of running requests take effect between iterations
            for (auto it = active.begin(); it != active.end();) {
                if ((*it)->cancel) {
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
        // place and upload newly admitted requests
        std::vector<ReqPlan*> fresh;
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
            active.push_back(r);
            if (r->plan.obj.n_spins > 0) fresh.push_back(&r->plan);
        }
        std::vector<std::shared_ptr<Request>> running;
        {
            std::lock_guard<std::mutex> lk(mu);
            running = active;
        }
        if (running.empty()) continue;
        ps_status st = PS_OK;
        if (!fresh.empty()) st = upload_tables(fresh, staging_tab, 0, stream);
        // one slice of every running request (empty objects only zero-fill)
        std::vector<ReqPlan*> plans;
        std::vector<size_t> first, count;
        for (auto& r : running) {
            ReqPlan& p = r->plan;
            if (p.prog.n_samples == 0) continue;
            if (p.obj.n_spins == 0) {
                if (r->next_slice == 0 && st == PS_OK) {
                    hipError_t e = launch_fill_zero(p.signal, 2 * p.prog.n_samples, stream);
                    if (e != hipSuccess) st = hip_fail(e, "fill");
                }
                continue;
            }
            plans.push_back(&p);
            first.push_back(r->next_slice);
            count.push_back(1);
        }
        const bool timed = st == PS_OK && !plans.empty();
        if (timed) {
            hipError_t e = hipEventRecord(ev_start, stream);
            if (e != hipSuccess) st = hip_fail(e, "hipEventRecord");
        }
        if (st == PS_OK && !plans.empty())
            st = run_rounds(ctx, plans, first, count, stream, records, staging_rec, nullptr);
        if (timed && st == PS_OK) {
            hipError_t e = hipEventRecord(ev_end, stream);
            if (e != hipSuccess) st = hip_fail(e, "hipEventRecord");
        }
        if (st == PS_OK) {
            hipError_t e = hipEventRecord(ev, stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev);
            if (e != hipSuccess) st = hip_fail(e, "server iteration");
        }
        double iter_kernel_s = 0.0;
        if (timed && st == PS_OK) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev_start, ev_end) == hipSuccess) iter_kernel_s = 1e-3 * ms;
        }
        std::string err = st == PS_OK ? "" : ps_last_error();
        {
            std::lock_guard<std::mutex> lk(mu);
            ++iterations;
            for (auto it = active.begin(); it != active.end();) {
                auto& r = *it;
                bool in_iter = std::find(running.begin(), running.end(), r) != running.end();
                if (!in_iter) { ++it; continue; }
                if (st != PS_OK) {
                    finish(r, RQ_FAILED, st, err);
                    it = active.erase(it);
                    continue;
                }
                r->next_slice += 1;
                if (r->plan.obj.n_spins > 0 && r->plan.prog.n_samples > 0) r->t_kernel += iter_kernel_s;
                const size_t n_sl = r->plan.obj.n_spins > 0 ? r->plan.prog.slices.size() : 1;
                if (r->plan.prog.n_samples == 0 || r->next_slice >= n_sl) {
                    finish(r, RQ_DONE, PS_OK, "");
                    it = active.erase(it);
                } else {
                    ++it;
                }
            }
            changed.notify_all();
        }
    }
}

void destroy_runtime(Ctx* ctx) {
    Server* s = ctx->server;
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
    if (s->ev) hipEventDestroy(s->ev);
    if (s->ev_start) hipEventDestroy(s->ev_start);
    if (s->ev_end) hipEventDestroy(s->ev_end);
    if (s->stream) hipStreamDestroy(s->stream);
    s->records.release();
    s->staging_rec.release();
    s->staging_tab.release();
    s->pool.release();
    delete s;
    ctx->server = nullptr;
}

static ps_status ensure_server(Ctx* ctx) {
    if (ctx->server) return PS_OK;
    Server* s = new (std::nothrow) Server();
    if (!s) return fail(PS_E_NO_MEMORY, "server allocation");
    s->ctx = ctx;
    s->t0 = Clock::now();
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&s->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&s->ev_end);
    if (e != hipSuccess) {
        if (s->ev_end) hipEventDestroy(s->ev_end);
        if (s->ev_start) hipEventDestroy(s->ev_start);
        if (s->ev) hipEventDestroy(s->ev);
        if (s->stream) hipStreamDestroy(s->stream);
        delete s;
        return hip_fail(e, "server stream/event");
    }
    ctx->server = s;
    s->thr = std::thread([s] { s->loop(); });
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
        DeviceGuard g(ctx->cfg.device);
        if ((st = ensure_server(ctx)) != PS_OK) return st;
        const int64_t steps = ctx->cfg.max_slice_steps;
        if ((st = plan_request(ctx, obj, seq, n_samples, signal, steps, &r->plan)) != PS_OK) return st;
    }
    r->footprint = r->plan.footprint();
    r->large = (double)r->plan.obj.n_spins * (double)r->plan.prog.n_steps >= kLargeWork;
    if (r->footprint > (size_t)ctx->cfg.max_footprint_bytes)
        return fail(PS_E_TOO_LARGE, "request footprint " + std::to_string(r->footprint) +
                                        " bytes exceeds the cap of " + std::to_string(ctx->cfg.max_footprint_bytes));
    Server* s = ctx->server;
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
    Server* s = ctx->server;
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
    Server* s = ctx->server;
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
    Server* s = ctx->server;
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
    Server* s = ctx->server;
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
    Server* s = ctx->server;
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
    Server* s = ctx->server;
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
    Server* s = ctx->server;
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
