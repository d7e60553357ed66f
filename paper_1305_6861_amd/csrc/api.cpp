// C ABI implementation: contexts, validation, compilation, device buffers
// and the per-request launch sequence (step kernel + finalize per slice).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/parspin.h"
#include "compile.h"
#include "ps_kernels.h"
#include "calib.h"
#include "ps_runtime.h"

static_assert(sizeof(ps_event) == 64, "ps_event ABI size");
static_assert(sizeof(ps_rf_shape) == 56, "ps_rf_shape ABI size");
static_assert(sizeof(ps_config) == 40, "ps_config ABI size");
static_assert(sizeof(ps_object) == 64, "ps_object ABI size");
static_assert(sizeof(ps_sequence) == 40, "ps_sequence ABI size");
static_assert(sizeof(ps_trajectory) == 24, "ps_trajectory ABI size");
static_assert(sizeof(ps_receive) == 24, "ps_receive ABI size");
static_assert(sizeof(ps_tune_result) == 232, "ps_tune_result ABI size");
static_assert(sizeof(ps_kt_object) == 104, "ps_kt_object ABI size");

namespace ps {

static thread_local std::string g_last_error;

ps_status fail(ps_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

ps_status hip_fail(hipError_t e, const char* what) {
    return fail(PS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) hipSetDevice(dev);
    dev_ = dev;
}
DeviceGuard::~DeviceGuard() {
    if (prev_ >= 0 && prev_ != dev_) hipSetDevice(prev_);
}

ps_status DevBuf::reserve(size_t n) {
    if (n <= bytes) return PS_OK;
    if (ptr) { hipFree(ptr); ptr = nullptr; bytes = 0; }
    size_t want = std::max(n, (size_t)4096);
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) { ptr = nullptr; return fail(PS_E_NO_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e)); }
    bytes = want;
    return PS_OK;
}
void DevBuf::release() {
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

ps_status HostBuf::reserve(size_t n) {
    if (n <= bytes) return PS_OK;
    if (ptr) { hipHostFree(ptr); ptr = nullptr; bytes = 0; }
    size_t want = std::max(n, (size_t)4096);
    hipError_t e = hipHostMalloc(&ptr, want, hipHostMallocDefault);
    if (e != hipSuccess) { ptr = nullptr; return fail(PS_E_NO_MEMORY, std::string("hipHostMalloc: ") + hipGetErrorString(e)); }
    bytes = want;
    return PS_OK;
}
void HostBuf::release() {
    if (ptr) hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

// Whether the FP32 matrix-core readout would sum a run of this sequence's
// readouts: some per-sample step (moment and dwell per sample) shared by two
// readouts of at least kMatrixMinSamples untabulated samples (the compiler's
// rule, see mark_matrix_readouts, without compiling the sequence).
static bool repeated_matrix_readouts(const ps_sequence* seq) {
    if (!seq || !seq->events) return false;
    std::vector<std::array<double, 4>> steps;
    for (int64_t i = 0; i < seq->n_events; ++i) {
        const ps_event& e = seq->events[i];
        if (e.n_adc < kMatrixMinSamples || (e.flags & PS_EV_TRAJECTORY)) continue;
        const double n = (double)e.n_adc;
        steps.push_back({e.dt / n, e.m[0] / n, e.m[1] / n, e.m[2] / n});
    }
    std::sort(steps.begin(), steps.end());
    return std::adjacent_find(steps.begin(), steps.end()) != steps.end();
}

int threshold_spins_per_lane(const Ctx* ctx, int64_t n_spins, const ps_sequence* seq) {
    if (ctx->cfg.spins_per_lane > 0) return ctx->cfg.spins_per_lane;
    // FP32 readouts that take the matrix cores run fastest at one spin per
    // lane (the matrix-only kernel), whatever the object's size
    if (ctx->cfg.precision != 64 && !(ctx->cfg.flags & PS_CFG_NO_MATRIX_READOUT) && repeated_matrix_readouts(seq))
        return 1;
    // Keep at least ~2 waves per SIMD (2 x 1024 SIMDs) while giving each lane
    // as many spins as possible: more spins per lane amortise the per-sample
    // lane-sum + butterfly reduction.  Readouts run 8 spins per lane from
    // S = 2 on (wave groups of 4 at S = 2, of 2 at S = 4), and S = 4 no longer
    // fits two waves per SIMD in registers, nor its propagator slots in LDS,
    // so the automatic choice stops at 2.  (S = 1 runs three waves per SIMD,
    // so objects between the thresholds still fill the chip in one pass.)
    const int64_t target_waves = 2 * 4 * (int64_t)std::max(ctx->n_cu, 1);
    const int maxS = 2;
    int S = 1;
    while (S < maxS && n_spins >= (int64_t)(2 * S) * 64 * target_waves) S *= 2;
    return S;
}

hipEvent_t timing_event(Ctx* ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t ev = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    return ev;
}

ps_status validate_object(const ps_object* obj) {
    if (!obj) return fail(PS_E_INVALID_ARG, "object is NULL");
    if (obj->n_spins < 0) return fail(PS_E_INVALID_ARG, "n_spins < 0");
    if (obj->n_spins > 0 && (!obj->x || !obj->y || !obj->z || !obj->m0 || !obj->t1 || !obj->t2 || !obj->dw))
        return fail(PS_E_INVALID_ARG, "object array pointer is NULL");
    return PS_OK;
}

int shape_cache_slots(const Ctx* ctx, int S, const Program& prog) {
    if (ctx->cfg.flags & PS_CFG_NO_SHAPE_CACHE) return 0;
    return shape_cache_slots_fitting(ctx->cfg.precision, S, (int32_t)(prog.rows.size() / 9),
                                     step_variant(ctx->cfg.precision, S, prog.matrix_only, prog.any_matrix));
}

// Compile + slice a request for a given number of partial-sum rows, spins
// per lane and receive coils (every coil has its own samples in each row).
ps_status prepare(const Ctx* ctx, const ps_sequence* seq, int64_t n_rows, int S, Program* prog, int n_coils,
                  bool snapshots, int64_t max_partial_bytes) {
    std::string err;
    ps_status st = compile_sequence(seq, prog, &err, snapshots);
    if (st != PS_OK) return fail(st, err);
    const int64_t real_bytes = ctx->cfg.precision == 64 ? 8 : 4;
    const int64_t per_sample = std::max<int64_t>(n_rows, 1) * 2 * real_bytes * std::max(n_coils, 1);
    const int64_t budget = max_partial_bytes > 0 ? max_partial_bytes : ctx->cfg.max_partial_bytes;
    int64_t max_samples = budget / per_sample;
    if (max_samples < 64) max_samples = 64;
    plan_slices(prog, max_samples);
    // the readout path first: the matrix-only kernel's LDS sets the slots
    if (ctx->cfg.precision != 64 && !(ctx->cfg.flags & PS_CFG_NO_MATRIX_READOUT)) mark_matrix_readouts(prog);
    assign_shape_slots(prog, shape_cache_slots(ctx, S, *prog));
    if (ctx->cfg.precision != 64) narrow_rotations(&prog->ops);
    return PS_OK;
}

// Upload program tables into a buffer set (stream-ordered).
static ps_status upload(BufSet* b, const Program& prog, hipStream_t stream) {
    const size_t ops_bytes = prog.ops.size() * sizeof(Op);
    const size_t rows_bytes = prog.rows.size() * sizeof(double);
    const size_t traj_bytes = prog.traj.size() * sizeof(double);
    ps_status st;
    if ((st = b->ops.reserve(ops_bytes)) != PS_OK) return st;
    if ((st = b->rows.reserve(rows_bytes)) != PS_OK) return st;
    if ((st = b->traj.reserve(traj_bytes)) != PS_OK) return st;
    if ((st = b->staging.reserve(ops_bytes + rows_bytes + traj_bytes)) != PS_OK) return st;
    unsigned char* h = reinterpret_cast<unsigned char*>(b->staging.ptr);
    if (ops_bytes) std::memcpy(h, prog.ops.data(), ops_bytes);
    if (rows_bytes) std::memcpy(h + ops_bytes, prog.rows.data(), rows_bytes);
    if (traj_bytes) std::memcpy(h + ops_bytes + rows_bytes, prog.traj.data(), traj_bytes);
    hipError_t e;
    if (ops_bytes && (e = hipMemcpyAsync(b->ops.ptr, h, ops_bytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(ops)");
    if (rows_bytes && (e = hipMemcpyAsync(b->rows.ptr, h + ops_bytes, rows_bytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(rows)");
    if (traj_bytes && (e = hipMemcpyAsync(b->traj.ptr, h + ops_bytes + rows_bytes, traj_bytes,
                                          hipMemcpyHostToDevice, stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync(trajectories)");
    return PS_OK;
}

void BufSet::release() {
    ops.release(); rows.release(); traj.release(); partial.release(); state.release(); fin_scratch.release();
    batch_tables.release(); batch_records.release();
    staging.release(); staging2.release();
}

ps_status acquire_set(Ctx* ctx, BufSet** out) {
    for (int k = 0; k < kBufSets; ++k) {
        const int idx = (ctx->next_set + k) % kBufSets;
        BufSet& b = ctx->sets[idx];
        if (b.pending) {
            const hipError_t q = hipEventQuery(b.done);
            if (q == hipErrorNotReady) continue;
            b.pending = false;
            if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
        }
        ctx->next_set = (idx + 1) % kBufSets;
        *out = &b;
        return PS_OK;
    }
    // every set is in use: wait for the oldest
    BufSet& b = ctx->sets[ctx->next_set];
    const hipError_t e = hipEventSynchronize(b.done);
    b.pending = false;
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    ctx->next_set = (ctx->next_set + 1) % kBufSets;
    *out = &b;
    return PS_OK;
}

ps_status release_set_after(BufSet* b, hipStream_t stream) {
    const hipError_t e = hipEventRecord(b->done, stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    b->pending = true;
    return PS_OK;
}

ps_status validate_receive(const ps_receive* rx, const ps_object* obj) {
    if (!rx) return PS_OK;
    if (rx->n_coils < 1) return fail(PS_E_INVALID_ARG, "receive: n_coils < 1");
    if (rx->reserved != 0) return fail(PS_E_INVALID_ARG, "receive: reserved field must be 0");
    if (obj && obj->n_spins > 0 && (!rx->s_x || !rx->s_y))
        return fail(PS_E_INVALID_ARG, "receive: sensitivity array is NULL");
    return PS_OK;
}

// Readout replicas of one tile of a program (ReplicaBound): the work bound
// weighs per-spin estimates in VALU instructions, ~6 per sample and coil
// against ~80 per hard pulse or snapshot and ~30 per shaped-pulse sub-step.
ReplicaBound replica_bound(const Program& p, int n_out) {
    int64_t max_adc = 0;
    for (const Slice& sl : p.slices) {
        int64_t c = 0;
        for (int64_t i = sl.op_begin; i < sl.op_end; ++i) c += p.ops[i].kind == OP_ADC || p.ops[i].kind == OP_ADCT;
        max_adc = std::max(max_adc, c);
    }
    ReplicaBound b;
    b.hard = (int)std::max<int64_t>(1, std::min<int64_t>(max_adc, 64));
    b.work = b.hard;
    // rough per-spin costs in vector instructions: a sample on the vector
    // path or (cheaper) on the matrix cores, a pulse or snapshot, a shaped
    // pulse applied from its cached propagator, a sub-step stepped
    const double per_sample = p.matrix_only ? 3.0 : 6.0;
    double pulses = (double)(p.n_rf + p.n_snapshots), substeps = 0.0;
    for (const Op& op : p.ops)
        if (op.kind == OP_SHAPE) {
            if (op.u.shape.mode == SHAPE_APPLY) pulses += 1.0;
            else substeps += op.n;
        }
    const double readout = per_sample * (double)p.n_samples * std::max(n_out, 1);
    const double other = 80.0 * pulses + 30.0 * substeps;
    if (other > 0) b.work = (int)std::max<int64_t>(1, std::min<int64_t>(b.hard, (int64_t)(readout / other)));
    b.other_share = readout + other > 0 ? other / (readout + other) : 0.0;
    return b;
}

int64_t device_slots(const Ctx* ctx, int S, const Program& p) {
    int32_t slots = 0;
    for (const Slice& sl : p.slices) slots = std::max(slots, sl.n_cache_slots);
    const int v = step_variant(ctx->cfg.precision, S, p.matrix_only, p.any_matrix);
    const size_t dyn = step_dyn_lds_bytes(ctx->cfg.precision, S, (int32_t)(p.rows.size() / 9), slots, v);
    return (int64_t)std::max(ctx->n_cu, 1) * step_workgroups_per_cu(ctx->cfg.precision, S, v, dyn);
}

// Readout replicas for a launch of n_tiles workgroup tiles: none when the
// tiles alone give every CU a workgroup.  Otherwise replicas that each get
// a CU of their own only shorten the launch, whatever stepping they repeat
// (up to n_CU / n_tiles of them); beyond that, about two workgroups per CU
// while the repeated stepping stays below the readout work it splits.
int replicas_for_load(const Ctx* ctx, int64_t n_tiles, ReplicaBound bound, int32_t mode) {
    if ((ctx->cfg.flags & PS_CFG_NO_READOUT_SPLIT) || mode == REPLICAS_NONE) return 1;
    const int64_t n_cu = std::max(ctx->n_cu, 1), want = 2 * n_cu;
    if (n_tiles <= 0 || n_tiles * 2 > want) return 1;
    const int64_t own = n_cu / n_tiles;
    const int64_t shared = std::min<int64_t>((want + n_tiles - 1) / n_tiles, bound.work);
    const int64_t rule = std::max<int64_t>(1, std::min<int64_t>(bound.hard, std::max(own, shared)));
    return (int)(mode == REPLICAS_DOUBLE ? std::min<int64_t>(bound.hard, 2 * rule) : rule);
}

// Whole rounds of workgroup slots after which a launch's tail is not split.
constexpr int64_t kTailSplitRounds = 4;

ReplicaSplit replica_split(const Ctx* ctx, int64_t n_tiles, ReplicaBound bound, int32_t mode, int64_t slots) {
    ReplicaSplit r;
    r.replicas = replicas_for_load(ctx, n_tiles, bound, mode);
    if (r.replicas > 1 || n_tiles <= std::max(ctx->n_cu, 1) || slots <= 0) return r;
    if ((ctx->cfg.flags & PS_CFG_NO_READOUT_SPLIT) || mode == REPLICAS_NONE) return r;
    // More tiles than CUs: the tiles that fill whole rounds of the device's
    // workgroup slots run whole, and the rest, which would leave the last
    // round part-empty, are split over the slots they leave free (at most 8
    // replicas each).  After more than kTailSplitRounds whole rounds the
    // part-empty one is too small a share of the launch to pay for the
    // replicas' repeated stepping (c3: 21 whole rounds, 2 % slower split).
    const int64_t whole = n_tiles / slots * slots, rest = n_tiles - whole;
    if (rest == 0 || whole > kTailSplitRounds * slots) return r;
    int64_t R = std::min<int64_t>({(int64_t)bound.hard, slots / rest, 8});
    if (mode == REPLICAS_DOUBLE) R = std::min<int64_t>(bound.hard, 2 * R);
    if (R < 2) return r;
    r.replicas = (int)R;
    r.n_whole = whole;
    return r;
}

ps_status plan_single(Ctx* ctx, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                      double* signal, int64_t n_samples, void* snaps, int64_t n_snapshots, const Tiling* force,
                      Single* r, int64_t max_partial_bytes) {
    // n_snapshots < 0: snapshot flags are ignored (entry points without them)
    ps_status st = validate_object(obj);
    if (st != PS_OK) return st;
    if ((st = validate_receive(rx, obj)) != PS_OK) return st;
    r->n_coils = rx ? rx->n_coils : 0;
    r->n_out = std::max(r->n_coils, 1);
    const Tiling tl = force ? *force : choose_tiling(ctx, obj->n_spins, seq, r->n_coils);
    r->S = tl.S;
    r->replica_mode = tl.replicas;
    const int64_t spb = spins_per_block_of(r->S);
    r->n_blocks = (obj->n_spins + spb - 1) / spb;
    r->n_rows = r->n_blocks * rows_per_block_of(r->S);
    const bool want_snaps = n_snapshots >= 0;
    if ((st = prepare(ctx, seq, r->n_rows, r->S, &r->prog, r->n_coils, want_snaps, max_partial_bytes)) != PS_OK)
        return st;
    const Program& prog = r->prog;
    if (n_samples != prog.n_samples)
        return fail(PS_E_INVALID_ARG, "n_samples (" + std::to_string(n_samples) + ") differs from the sequence's " +
                                          std::to_string(prog.n_samples));
    if (want_snaps && n_snapshots != prog.n_snapshots)
        return fail(PS_E_INVALID_ARG, "n_snapshots (" + std::to_string(n_snapshots) +
                                          ") differs from the sequence's " + std::to_string(prog.n_snapshots));
    if (want_snaps && prog.n_snapshots > 0 && obj->n_spins > 0 && !snaps)
        return fail(PS_E_INVALID_ARG, "snapshots is NULL");
    if (prog.n_snapshots > 0xffffffffll) return fail(PS_E_TOO_LARGE, "too many snapshots");
    r->any_snaps = want_snaps && prog.n_snapshots > 0 && obj->n_spins > 0;
    if (n_samples > 0 && !signal) return fail(PS_E_INVALID_ARG, "signal is NULL");
    r->obj = *obj;
    r->rx = rx ? *rx : ps_receive{0, 0, nullptr, nullptr};
    r->signal = signal;
    r->n_samples = n_samples;
    r->snaps = r->any_snaps ? snaps : nullptr;
    int64_t max_slice = 0;
    for (const Slice& sl : prog.slices) max_slice = std::max(max_slice, sl.n_samples);
    r->coil_stride = pad_fin(2 * max_slice);   // one block of samples per coil in every row
    r->row_stride = r->coil_stride * r->n_out;
    const int64_t real_bytes = ctx->cfg.precision == 64 ? 8 : 4;
    r->partial_bytes = (size_t)(r->n_rows * r->row_stride * real_bytes);
    r->fin_bytes = (size_t)finalize_scratch_doubles(r->n_rows, r->row_stride) * sizeof(double);
    r->state_bytes = prog.slices.size() > 1
                         ? (size_t)(state_reals_per_spin(prog.n_state_slots) * obj->n_spins * real_bytes)
                         : 0;
    const ReplicaSplit rs = replica_split(ctx, r->n_blocks, replica_bound(r->prog, r->n_out), r->replica_mode,
                                          device_slots(ctx, r->S, r->prog));
    r->n_replicas = rs.replicas;
    r->n_whole = rs.n_whole;
    return PS_OK;
}

bool Single::empty() const { return obj.n_spins == 0 || (n_samples == 0 && !any_snaps); }

ps_status enqueue_single(const Ctx* ctx, const Single& r, const SingleBuffers& b, hipStream_t stream,
                         Ctx* timing_ctx) {
    hipError_t e;
    if (r.obj.n_spins == 0) {
        if (r.n_samples > 0 && (e = launch_fill_zero(r.signal, 2 * r.n_samples * r.n_out, stream)) != hipSuccess)
            return hip_fail(e, "fill");
        return PS_OK;
    }
    if (r.n_samples == 0 && !r.any_snaps) return PS_OK;
    const int precision = ctx->cfg.precision;
    const int64_t real_bytes = precision == 64 ? 8 : 4;
    const Program& prog = r.prog;
    StepArgs a{};
    a.x = r.obj.x; a.y = r.obj.y; a.z = r.obj.z; a.m0 = r.obj.m0; a.t1 = r.obj.t1; a.t2 = r.obj.t2;
    a.dw = r.obj.dw;
    a.n_spins = r.obj.n_spins;
    a.n_shape_rows = (int32_t)(prog.rows.size() / 9);
    a.rows = b.rows;
    a.traj = reinterpret_cast<const double*>(b.traj);
    a.partial = b.partial;
    a.row_stride = r.row_stride;
    a.state = b.state;
    a.n_coils = r.n_coils;
    a.s_x = r.n_coils ? r.rx.s_x : nullptr;
    a.s_y = r.n_coils ? r.rx.s_y : nullptr;
    a.coil_stride = r.coil_stride;
    a.snaps = r.snaps;
    a.n_replicas = r.n_replicas;
    a.n_tiles = r.n_blocks;
    a.n_whole = r.n_whole;
    for (int d = 0; d < 3; ++d) a.mx_mu[d] = prog.matrix_mu[d];
    a.mx_tau = prog.matrix_tau;
    const Op* ops_dev = reinterpret_cast<const Op*>(b.ops);
    for (size_t i = 0; i < prog.slices.size(); ++i) {
        const Slice& sl = prog.slices[i];
        a.ops = ops_dev + sl.op_begin;
        a.n_ops = (int32_t)(sl.op_end - sl.op_begin);
        a.load_state = i > 0;
        a.save_state = i + 1 < prog.slices.size();
        a.anchor_parity = (int32_t)(i & 1);
        a.n_cache_slots = sl.n_cache_slots;
        a.cache_load = sl.cache_load;
        a.cache_save = sl.cache_save;
        hipEvent_t t0 = nullptr, t1 = nullptr, t2 = nullptr;
        if (timing_ctx) {
            t0 = timing_event(timing_ctx); t1 = timing_event(timing_ctx); t2 = timing_event(timing_ctx);
            if (!t0 || !t1 || !t2) return fail(PS_E_DEVICE, "timing event creation failed");
            hipEventRecord(t0, stream);
        }
        if ((e = launch_step(a, precision, r.S, r.n_blocks, stream,
                             step_variant(precision, r.S, prog.matrix_only, prog.any_matrix))) != hipSuccess)
            return hip_fail(e, "step kernel launch");
        if (timing_ctx) hipEventRecord(t1, stream);
        for (int c = 0; c < r.n_out && sl.n_samples > 0; ++c) {
            const unsigned char* part = reinterpret_cast<const unsigned char*>(b.partial) +
                                        (size_t)(c * r.coil_stride * real_bytes);
            if ((e = launch_finalize(part, precision, r.n_rows, r.row_stride, 2 * sl.n_samples,
                                     r.signal + 2 * r.n_samples * c + 2 * sl.sample_begin, b.fin_scratch,
                                     stream)) != hipSuccess)
                return hip_fail(e, "finalize kernel launch");
        }
        if (timing_ctx) {
            hipEventRecord(t2, stream);
            timing_ctx->step_marks.emplace_back(t0, t1);
            timing_ctx->fin_marks.emplace_back(t1, t2);
        }
    }
    return PS_OK;
}

ps_status run_request(Ctx* ctx, const ps_object* obj, const ps_sequence* seq, double* signal,
                      int64_t n_samples, hipStream_t stream, const Tiling* force, const ps_receive* rx,
                      void* snaps, int64_t n_snapshots) {
    Single r;
    ps_status st = plan_single(ctx, obj, seq, rx, signal, n_samples, snaps, n_snapshots, force, &r);
    if (st != PS_OK) return st;
    if (r.empty()) return enqueue_single(ctx, r, SingleBuffers{}, stream, nullptr);
    BufSet* set = nullptr;
    if ((st = acquire_set(ctx, &set)) != PS_OK) return st;
    if ((st = set->partial.reserve(r.partial_bytes)) != PS_OK) return st;
    if (r.fin_bytes > 0 && (st = set->fin_scratch.reserve(r.fin_bytes)) != PS_OK) return st;
    if (r.state_bytes > 0 && (st = set->state.reserve(r.state_bytes)) != PS_OK) return st;
    if ((st = upload(set, r.prog, stream)) != PS_OK) return st;
    SingleBuffers b{set->ops.ptr, set->rows.ptr, set->traj.ptr, set->partial.ptr, set->state.ptr,
                    reinterpret_cast<double*>(set->fin_scratch.ptr)};
    const bool timing = (ctx->cfg.flags & PS_CFG_KERNEL_TIMING) != 0;
    // the set's tables are being copied on `stream`: whatever happens next,
    // the set is not reused before that work completes
    const ps_status enq = enqueue_single(ctx, r, b, stream, timing ? ctx : nullptr);
    st = release_set_after(set, stream);
    return enq != PS_OK ? enq : st;
}

}  // namespace ps

using namespace ps;

extern "C" {

ps_status ps_config_default(ps_config* cfg) {
    if (!cfg) return fail(PS_E_INVALID_ARG, "cfg is NULL");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->precision = 32;
    cfg->spins_per_lane = 0;
    cfg->max_partial_bytes = 2ll << 30;
    cfg->max_footprint_bytes = 64ll << 30;
    cfg->max_slice_steps = 65536;
    return PS_OK;
}

ps_status ps_create(ps_ctx** out, const ps_config* cfg_in) {
    clear_error();
    if (!out) return fail(PS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    ps_config cfg;
    if (cfg_in) cfg = *cfg_in; else ps_config_default(&cfg);
    if (cfg.precision != 32 && cfg.precision != 64) return fail(PS_E_INVALID_ARG, "precision must be 32 or 64");
    if (cfg.spins_per_lane != 0) {
        const int s = cfg.spins_per_lane;
        const bool ok = cfg.precision == 64 ? (s == 1 || s == 2) : (s == 1 || s == 2 || s == 4 || s == 8);
        if (!ok) return fail(PS_E_INVALID_ARG, "spins_per_lane not supported for this precision");
    }
    if (cfg.max_partial_bytes <= 0) cfg.max_partial_bytes = 2ll << 30;
    if (cfg.max_footprint_bytes <= 0) cfg.max_footprint_bytes = 64ll << 30;
    if (cfg.max_slice_steps < 0) return fail(PS_E_INVALID_ARG, "max_slice_steps < 0");
    if (cfg.max_slice_steps == 0) cfg.max_slice_steps = 65536;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(PS_E_NO_DEVICE, "no HIP device visible");
    if (cfg.device < 0 || cfg.device >= count) return fail(PS_E_NO_DEVICE, "device ordinal out of range");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, cfg.device)) != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PS_E_NO_DEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    Ctx* ctx = new (std::nothrow) Ctx();
    if (!ctx) return fail(PS_E_NO_MEMORY, "context allocation");
    ctx->cfg = cfg;
    ctx->n_cu = prop.multiProcessorCount;
    DeviceGuard g(cfg.device);
    for (BufSet& b : ctx->sets) {
        if ((e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming)) != hipSuccess) {
            for (BufSet& c : ctx->sets)
                if (c.done) hipEventDestroy(c.done);
            delete ctx;
            return hip_fail(e, "hipEventCreate");
        }
    }
    // the allocation-free entry point's scratch (device static array, its
    // address taken once per device with the device current) and staging
    void* base = nullptr;
    if ((e = noalloc_scratch(cfg.device, &base)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&ctx->noalloc_done, hipEventDisableTiming)) != hipSuccess) {
        for (BufSet& c : ctx->sets) (void)hipEventDestroy(c.done);
        if (ctx->noalloc_done) (void)hipEventDestroy(ctx->noalloc_done);
        delete ctx;
        return hip_fail(e, "allocation-free scratch set-up");
    }
    ctx->noalloc_base = base;
    if (ctx->noalloc_staging.reserve(kNoAllocStagingBytes) != PS_OK) {
        for (BufSet& c : ctx->sets) (void)hipEventDestroy(c.done);
        (void)hipEventDestroy(ctx->noalloc_done);
        delete ctx;
        return fail(PS_E_NO_MEMORY, "pinned staging of the allocation-free entry point");
    }
    *out = reinterpret_cast<ps_ctx*>(ctx);
    return PS_OK;
}

ps_status ps_create_scheduler_test(ps_ctx** out, const ps_config* cfg_in, const ps_test_backend* backend) {
    clear_error();
    if (!out || !backend) return fail(PS_E_INVALID_ARG, "out or backend is NULL");
    *out = nullptr;
    if (!(backend->iteration_seconds >= 0) || !std::isfinite(backend->iteration_seconds) ||
        backend->fail_iteration < -1)
        return fail(PS_E_INVALID_ARG, "iteration_seconds must be >= 0 and fail_iteration >= -1");
    ps_config cfg;
    if (cfg_in) cfg = *cfg_in; else ps_config_default(&cfg);
    if (cfg.precision != 32 && cfg.precision != 64) return fail(PS_E_INVALID_ARG, "precision must be 32 or 64");
    if (cfg.max_partial_bytes <= 0) cfg.max_partial_bytes = 2ll << 30;
    if (cfg.max_footprint_bytes <= 0) cfg.max_footprint_bytes = 64ll << 30;
    if (cfg.max_slice_steps < 0) return fail(PS_E_INVALID_ARG, "max_slice_steps < 0");
    if (cfg.max_slice_steps == 0) cfg.max_slice_steps = 65536;
    Ctx* ctx = new (std::nothrow) Ctx();
    if (!ctx) return fail(PS_E_NO_MEMORY, "context allocation");
    ctx->cfg = cfg;
    ctx->n_cu = 256;
    ctx->scheduler_test = true;
    ctx->test_backend = *backend;
    *out = reinterpret_cast<ps_ctx*>(ctx);
    return PS_OK;
}

void ps_destroy(ps_ctx* handle) {
    if (!handle) return;
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) {
        destroy_runtime(ctx);
        delete ctx;
        return;
    }
    {
        DeviceGuard g(ctx->cfg.device);
        destroy_runtime(ctx);
        for (BufSet& b : ctx->sets) {
            if (b.pending) hipEventSynchronize(b.done);
            hipEventDestroy(b.done);
        }
        for (auto& m : ctx->step_marks) { hipEventDestroy(m.first); hipEventDestroy(m.second); }
        for (auto& m : ctx->fin_marks) hipEventDestroy(m.second);   // m.first is a step mark
        for (hipEvent_t ev : ctx->ev_pool) hipEventDestroy(ev);
        for (BufSet& b : ctx->sets) b.release();
        if (ctx->noalloc_done) {
            if (ctx->noalloc_pending) (void)hipEventSynchronize(ctx->noalloc_done);
            (void)hipEventDestroy(ctx->noalloc_done);
        }
        ctx->noalloc_staging.release();
    }
    delete ctx;
}

const char* ps_last_error(void) { return g_last_error.c_str(); }

ps_status ps_count(const ps_sequence* seq, int64_t* n_samples, int64_t* n_steps_per_spin) {
    clear_error();
    Program p;
    std::string err;
    ps_status st = compile_sequence(seq, &p, &err);
    if (st != PS_OK) return fail(st, err);
    if (n_samples) *n_samples = p.n_samples;
    if (n_steps_per_spin) *n_steps_per_spin = p.n_steps;
    return PS_OK;
}

ps_status ps_simulate(ps_ctx* handle, const ps_object* obj, const ps_sequence* seq, double* signal,
                      int64_t n_samples, void* stream) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) return fail(PS_E_INVALID_ARG, "a scheduler-test context runs no kernels");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    const ps_status tst = autotune_if_new(ctx, obj, seq, nullptr, reinterpret_cast<hipStream_t>(stream));
    if (tst != PS_OK) return tst;
    return run_request(ctx, obj, seq, signal, n_samples, reinterpret_cast<hipStream_t>(stream), nullptr, nullptr);
}

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

ps_status ps_simulate_noalloc(ps_ctx* handle, const ps_object* obj, const ps_sequence* seq, double* signal,
                              int64_t n_samples, void* stream_v) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) return fail(PS_E_INVALID_ARG, "a scheduler-test context runs no kernels");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
    if (!ctx->noalloc_base) return fail(PS_E_DEVICE, "no static scratch on this context's device");
    // Lay the request out in the scratch: tables, partial rows, finalize
    // row-group sums, slice state.  First with the context's own bound on the
    // partial rows (the time slicing of ps_simulate), then, while it does not
    // fit, with the partial rows held to what the rest leaves (more slices).
    const size_t cap = (size_t)kNoAllocScratchBytes;
    Single r;
    size_t off_rows = 0, off_traj = 0, off_part = 0, off_fin = 0, off_state = 0, total = 0;
    int64_t budget = ctx->cfg.max_partial_bytes;
    for (int attempt = 0;; ++attempt) {
        r = Single();
        ps_status st = plan_single(ctx, obj, seq, nullptr, signal, n_samples, nullptr, -1, nullptr, &r, budget);
        if (st != PS_OK) return st;
        const Program& prog = r.prog;
        off_rows = align256(prog.ops.size() * sizeof(Op));
        off_traj = off_rows + align256(prog.rows.size() * sizeof(double));
        off_part = off_traj + align256(prog.traj.size() * sizeof(double));
        off_fin = off_part + align256(r.partial_bytes);
        off_state = off_fin + align256(r.fin_bytes);
        total = off_state + align256(r.state_bytes);
        if (r.empty() || total <= cap) break;
        const size_t rest = total - align256(r.partial_bytes) - align256(r.fin_bytes);
        // the finalize sums take about 1/32 of the FP32 (1/64 of the FP64) partial rows
        const size_t room = rest < cap ? (cap - rest) * 31 / 32 : 0;
        const int64_t next = std::min<int64_t>((int64_t)room, (int64_t)r.partial_bytes / 2);
        if (attempt >= 16 || next < 4096 || next >= budget)
            return fail(PS_E_TOO_LARGE, "the request needs " + std::to_string(total) +
                                            " bytes of scratch at its smallest time slices; the static scratch holds " +
                                            std::to_string(cap));
        budget = next;
    }
    if (r.empty()) return enqueue_single(ctx, r, SingleBuffers{}, stream, nullptr);
    const Program& prog = r.prog;
    const size_t ops_bytes = prog.ops.size() * sizeof(Op), rows_bytes = prog.rows.size() * sizeof(double);
    const size_t traj_bytes = prog.traj.size() * sizeof(double);
    if (ops_bytes + rows_bytes + traj_bytes > ctx->noalloc_staging.bytes)
        return fail(PS_E_TOO_LARGE, "the request's tables take " + std::to_string(ops_bytes + rows_bytes + traj_bytes) +
                                        " bytes; the staging of the allocation-free entry point holds " +
                                        std::to_string(ctx->noalloc_staging.bytes));
    hipError_t e;
    // the staging is rewritten only after the previous upload from it has run
    if (ctx->noalloc_pending) {
        if ((e = hipEventSynchronize(ctx->noalloc_done)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        ctx->noalloc_pending = false;
    }
    unsigned char* h = reinterpret_cast<unsigned char*>(ctx->noalloc_staging.ptr);
    unsigned char* d = reinterpret_cast<unsigned char*>(ctx->noalloc_base);
    std::memcpy(h, prog.ops.data(), ops_bytes);
    if (rows_bytes) std::memcpy(h + ops_bytes, prog.rows.data(), rows_bytes);
    if (traj_bytes) std::memcpy(h + ops_bytes + rows_bytes, prog.traj.data(), traj_bytes);
    if ((e = hipMemcpyAsync(d, h, ops_bytes, hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (rows_bytes && (e = hipMemcpyAsync(d + off_rows, h + ops_bytes, rows_bytes, hipMemcpyHostToDevice, stream)) !=
                           hipSuccess) ||
        (traj_bytes && (e = hipMemcpyAsync(d + off_traj, h + ops_bytes + rows_bytes, traj_bytes,
                                           hipMemcpyHostToDevice, stream)) != hipSuccess))
        return hip_fail(e, "hipMemcpyAsync(tables into the scratch)");
    SingleBuffers b{d, d + off_rows, d + off_traj, d + off_part, r.state_bytes ? d + off_state : nullptr,
                    r.fin_bytes ? reinterpret_cast<double*>(d + off_fin) : nullptr};
    const ps_status enq = enqueue_single(ctx, r, b, stream, nullptr);
    if ((e = hipEventRecord(ctx->noalloc_done, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    ctx->noalloc_pending = true;
    return enq;
}

ps_status ps_count_snapshots(const ps_sequence* seq, int64_t* n_snapshots) {
    clear_error();
    Program p;
    std::string err;
    ps_status st = compile_sequence(seq, &p, &err);
    if (st != PS_OK) return fail(st, err);
    if (n_snapshots) *n_snapshots = p.n_snapshots;
    return PS_OK;
}

ps_status ps_simulate_ex(ps_ctx* handle, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                         double* signal, int64_t n_samples, void* snapshots, int64_t n_snapshots, void* stream) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    if (n_snapshots < 0) return fail(PS_E_INVALID_ARG, "n_snapshots < 0");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) return fail(PS_E_INVALID_ARG, "a scheduler-test context runs no kernels");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    const ps_status tst = autotune_if_new(ctx, obj, seq, rx, reinterpret_cast<hipStream_t>(stream));
    if (tst != PS_OK) return tst;
    return run_request(ctx, obj, seq, signal, n_samples, reinterpret_cast<hipStream_t>(stream), nullptr, rx, snapshots,
                       n_snapshots);
}

ps_status ps_simulate_rx(ps_ctx* handle, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                         double* signal, int64_t n_samples, void* stream) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) return fail(PS_E_INVALID_ARG, "a scheduler-test context runs no kernels");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    const ps_status tst = autotune_if_new(ctx, obj, seq, rx, reinterpret_cast<hipStream_t>(stream));
    if (tst != PS_OK) return tst;
    return run_request(ctx, obj, seq, signal, n_samples, reinterpret_cast<hipStream_t>(stream), nullptr, rx);
}

ps_status ps_tile(ps_ctx* handle, int64_t n_spins, int32_t* spins_per_lane, int64_t* spins_per_block) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    if (n_spins < 0) return fail(PS_E_INVALID_ARG, "n_spins < 0");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    const int S = threshold_spins_per_lane(ctx, n_spins);
    if (spins_per_lane) *spins_per_lane = S;
    if (spins_per_block) *spins_per_block = spins_per_block_of(S);
    return PS_OK;
}

ps_status ps_valu_peak(ps_ctx* handle, int32_t precision, double* tflops) {
    clear_error();
    if (!handle || !tflops) return fail(PS_E_INVALID_ARG, "ctx or tflops is NULL");
    if (precision != 32 && precision != 64) return fail(PS_E_INVALID_ARG, "precision must be 32 or 64");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) return fail(PS_E_INVALID_ARG, "a scheduler-test context runs no kernels");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    constexpr int64_t kBlocks = 8192;
    constexpr int32_t kIters = 4096;
    void* sink = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&sink, 16);
    if (e == hipSuccess) e = hipStreamCreate(&st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const double nan = std::numeric_limits<double>::quiet_NaN();
    if (e == hipSuccess) e = launch_fma_chain(precision, kBlocks, kIters, nan, sink, st);    // warm-up
    float best = 0.f;
    for (int rep = 0; rep < 5 && e == hipSuccess; ++rep) {
        float ms = 0.f;
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) e = launch_fma_chain(precision, kBlocks, kIters, nan, sink, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && (rep == 0 || ms < best)) best = ms;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const hipError_t first = e;
    if (e1) hipEventDestroy(e1);
    if (e0) hipEventDestroy(e0);
    if (st) hipStreamDestroy(st);
    if (sink) hipFree(sink);
    if (first != hipSuccess) return hip_fail(first, "FMA rate measurement");
    if (!(best > 0.f)) return fail(PS_E_DEVICE, "FMA rate measurement: no elapsed time");
    const double flops = 2.0 * 8.0 * (double)kIters * (double)kBlocks * 256.0;
    *tflops = flops / ((double)best * 1e-3) / 1e12;
    return PS_OK;
}

ps_status ps_kernel_times(ps_ctx* handle, double* step_ms, int64_t capacity, int64_t* n_step,
                          double* finalize_ms) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    if (capacity < 0 || (capacity > 0 && !step_ms)) return fail(PS_E_INVALID_ARG, "bad step_ms/capacity");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    ps_status st = PS_OK;
    double fin = 0.0;
    int64_t n = 0;
    for (auto& m : ctx->step_marks) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(m.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.first, m.second);
        if (e != hipSuccess && st == PS_OK) st = hip_fail(e, "kernel timing");
        if (n < capacity) step_ms[n] = ms;
        ++n;
    }
    for (auto& m : ctx->fin_marks) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(m.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.first, m.second);
        if (e != hipSuccess && st == PS_OK) st = hip_fail(e, "kernel timing");
        fin += ms;
    }
    for (auto& m : ctx->step_marks) { ctx->ev_pool.push_back(m.first); ctx->ev_pool.push_back(m.second); }
    for (auto& m : ctx->fin_marks) ctx->ev_pool.push_back(m.second);
    ctx->step_marks.clear();
    ctx->fin_marks.clear();
    if (n_step) *n_step = n;
    if (finalize_ms) *finalize_ms = fin;
    return st;
}

}  // extern "C"
