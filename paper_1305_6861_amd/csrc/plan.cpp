// Compiled plans: one request compiled once, its kernel launches captured in
// a HIP graph, replayed by ps_plan_launch.
//
// A plan owns its device tables (operations, shaped-pulse rows) and work
// buffers (partial-sum rows, slice state, finalize scratch), uploaded and
// allocated when it is created, so a replay is a single graph launch with no
// host compile, no copy and no allocation.  The object, receive and output
// pointers are baked into the graph; the caller may change the data behind
// them between replays (e.g. new tissue parameters for the same geometry).
#include <hip/hip_runtime_api.h>

#include <string>

#include "../../include/parspin.h"
#include "ps_kernels.h"
#include "ps_runtime.h"

namespace ps {

struct Plan {
    Ctx* ctx = nullptr;
    Single r;
    DevBuf ops, rows, traj, partial, state, fin;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;       // completion of the last replay
    bool launched = false;
};

static void plan_free(Plan* p) {
    if (!p) return;
    if (p->launched && p->done) hipEventSynchronize(p->done);
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->done) hipEventDestroy(p->done);
    p->ops.release(); p->rows.release(); p->traj.release(); p->partial.release(); p->state.release(); p->fin.release();
    delete p;
}

}  // namespace ps

using namespace ps;

extern "C" {

ps_status ps_plan_create(ps_ctx* handle, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                         double* signal, int64_t n_samples, ps_plan** out) {
    clear_error();
    if (!handle || !out) return fail(PS_E_INVALID_ARG, "ctx or out is NULL");
    *out = nullptr;
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) return fail(PS_E_INVALID_ARG, "a scheduler-test context runs no kernels");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    Plan* p = new Plan();
    p->ctx = ctx;
    ps_status st = autotune_if_new(ctx, obj, seq, rx, nullptr);
    if (st != PS_OK) { plan_free(p); return st; }
    st = plan_single(ctx, obj, seq, rx, signal, n_samples, nullptr, -1, nullptr, &p->r);
    if (st != PS_OK) { plan_free(p); return st; }
    const Program& prog = p->r.prog;
    hipError_t e;
    if ((e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming)) != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "hipEventCreate");
    }
    SingleBuffers b;
    if (!p->r.empty()) {
        const size_t ops_bytes = prog.ops.size() * sizeof(Op), rows_bytes = prog.rows.size() * sizeof(double);
        const size_t traj_bytes = prog.traj.size() * sizeof(double);
        if ((st = p->ops.reserve(ops_bytes)) != PS_OK || (st = p->rows.reserve(rows_bytes)) != PS_OK ||
            (st = p->traj.reserve(traj_bytes)) != PS_OK ||
            (st = p->partial.reserve(p->r.partial_bytes)) != PS_OK ||
            (p->r.fin_bytes && (st = p->fin.reserve(p->r.fin_bytes)) != PS_OK) ||
            (p->r.state_bytes && (st = p->state.reserve(p->r.state_bytes)) != PS_OK)) {
            plan_free(p);
            return st;
        }
        if ((ops_bytes && (e = hipMemcpy(p->ops.ptr, prog.ops.data(), ops_bytes, hipMemcpyHostToDevice)) != hipSuccess) ||
            (rows_bytes && (e = hipMemcpy(p->rows.ptr, prog.rows.data(), rows_bytes, hipMemcpyHostToDevice)) != hipSuccess) ||
            (traj_bytes && (e = hipMemcpy(p->traj.ptr, prog.traj.data(), traj_bytes, hipMemcpyHostToDevice)) != hipSuccess)) {
            plan_free(p);
            return hip_fail(e, "hipMemcpy(plan tables)");
        }
        b = SingleBuffers{p->ops.ptr, p->rows.ptr, p->traj.ptr, p->partial.ptr, p->state.ptr,
                          reinterpret_cast<double*>(p->fin.ptr)};
    }
    // capture the launches on a private stream (default priority)
    hipStream_t cap = nullptr;
    if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "hipStreamCreate");
    }
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        hipStreamDestroy(cap);
        plan_free(p);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    st = enqueue_single(ctx, p->r, b, cap, nullptr);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap, &graph);
    hipStreamDestroy(cap);
    p->graph = graph;
    if (st != PS_OK) { plan_free(p); return st; }
    if (e != hipSuccess) { plan_free(p); return hip_fail(e, "hipStreamEndCapture"); }
    if ((e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0)) != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = reinterpret_cast<ps_plan*>(p);
    return PS_OK;
}

ps_status ps_plan_launch(ps_plan* handle, void* stream) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "plan is NULL");
    Plan* p = reinterpret_cast<Plan*>(handle);
    DeviceGuard g(p->ctx->cfg.device);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if ((e = hipGraphLaunch(p->exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if ((e = hipEventRecord(p->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->launched = true;
    return PS_OK;
}

void ps_plan_destroy(ps_plan* handle) {
    if (!handle) return;
    Plan* p = reinterpret_cast<Plan*>(handle);
    DeviceGuard g(p->ctx->cfg.device);
    plan_free(p);
}

}  // extern "C"
