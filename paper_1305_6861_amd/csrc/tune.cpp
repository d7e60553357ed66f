// Autotuner of the workgroup tiling.
//
// The paper cuts the spin set into blocks for its compute nodes: small
// enough that every node gets one, and more blocks than nodes so that the
// nodes' different speeds level out (section 5.3.2).  On one GPU the block
// is a workgroup tile of 256 S spins (S spins per lane), and the same
// trade-off decides S: larger tiles amortise the per-sample reduction over
// more spins per lane, smaller ones give the compute units more workgroups;
// readout replicas spread a small object's readouts over idle compute units
// at the price of repeating its RF stepping.  Where the balance lies
// depends on the object size, the readout length, shaped pulses and coils,
// so the tuner times the candidate tilings on the device for one request of
// each class and keeps the fastest in a per-context table that every later
// request of the class uses (ps_simulate*, plans, batches and served
// requests alike, so a request keeps one tiling on every path).
//
// A candidate is timed on a probe: the request's object with a prefix of
// its sequence of bounded work (the whole sequence when it is short), on a
// private stream, in rounds over all candidates (a warm-up round, then
// kTimedRounds timed ones), median of its timed runs.
// The table can be written to a file and read back by a later process on
// the same device model with the same library build.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/parspin.h"
#include "ps_kernels.h"
#include "ps_runtime.h"

#ifndef PS_LIB_HASH
#define PS_LIB_HASH "unversioned"
#endif

namespace ps {

// Timed rounds over the candidates (after one warm-up round).
constexpr int kTimedRounds = 5;
// Probes shorter than this (ms) belong to requests small enough to share
// batched rounds with others.
constexpr double kShortProbeMs = 1.0;

static int floor_log2(int64_t v) {
    int r = -1;
    while (v > 0) { v >>= 1; ++r; }
    return r;
}

static int ceil_log2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

TuneKey tune_key(const Ctx* ctx, int64_t n_spins, const ps_sequence* seq, int n_coils) {
    TuneKey k;
    k.precision = ctx->cfg.precision;
    k.spins_log2 = floor_log2(n_spins);
    int64_t longest = 0;
    int shaped = 0;
    if (seq && seq->events && seq->n_events > 0) {
        for (int64_t i = 0; i < seq->n_events; ++i) {
            const ps_event& e = seq->events[i];
            longest = std::max<int64_t>(longest, (int64_t)e.n_adc);
            shaped |= e.rf_shape >= 0;
        }
    }
    k.readout_log2 = longest > 0 ? floor_log2(longest) : -1;
    k.shaped = shaped;
    k.coils_log2 = n_coils > 1 ? ceil_log2(n_coils) : 0;
    return k;
}

Tiling choose_tiling(const Ctx* ctx, int64_t n_spins, const ps_sequence* seq, int n_coils) {
    const int32_t rep = (ctx->cfg.flags & PS_CFG_NO_READOUT_SPLIT) ? REPLICAS_NONE : REPLICAS_RULE;
    if (ctx->cfg.spins_per_lane > 0) return Tiling{ctx->cfg.spins_per_lane, rep, false};
    auto it = ctx->tuned.find(tune_key(ctx, n_spins, seq, n_coils));
    if (it != ctx->tuned.end()) {
        Tiling t = it->second.tiling;
        if (rep == REPLICAS_NONE) t.replicas = REPLICAS_NONE;
        return t;
    }
    return Tiling{threshold_spins_per_lane(ctx, n_spins, seq), rep, false};
}

// Spin-steps a probe may hold: a few ms of the device at the readout rate.
constexpr double kProbeWork = 6e10;

// Steps one event takes per spin (ps_count's unit).
static int64_t event_steps(const ps_sequence* seq, const ps_event& e) {
    int64_t w = std::max<int64_t>((int64_t)e.n_adc, 1);
    if (e.rf_shape >= 0 && e.rf_shape < seq->n_shapes) w += std::max(seq->shapes[e.rf_shape].n_sub, 1);
    return w;
}

// Number of leading events of the probe: as many as fit kProbeWork (at
// least through the first readout), the whole sequence when it is short.
static int64_t probe_events(const ps_sequence* seq, int64_t n_spins) {
    const double per_step = (double)std::max<int64_t>(n_spins, 1);
    double work = 0.0;
    bool readout = false;
    for (int64_t i = 0; i < seq->n_events; ++i) {
        const ps_event& e = seq->events[i];
        work += per_step * (double)event_steps(seq, e);
        readout = readout || e.n_adc > 0;
        if (readout && work >= kProbeWork) return i + 1;
    }
    return seq->n_events;
}

struct ProbeStream {
    hipStream_t stream = nullptr;
    hipEvent_t after = nullptr;
    ~ProbeStream() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (after) (void)hipEventDestroy(after);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

// Device time of the kernels one probe run launched (the step and finalize
// launches of each time slice, from the context's timing marks), in ms;
// the marks' events go back to the pool.
static ps_status drain_marks(Ctx* ctx, double* ms) {
    double sum = 0.0;
    ps_status st = PS_OK;
    for (size_t i = 0; i < ctx->step_marks.size() && i < ctx->fin_marks.size(); ++i) {
        float f = 0.f;
        hipError_t e = hipEventSynchronize(ctx->fin_marks[i].second);
        if (e == hipSuccess) e = hipEventElapsedTime(&f, ctx->step_marks[i].first, ctx->fin_marks[i].second);
        if (e != hipSuccess && st == PS_OK) st = hip_fail(e, "autotuner timing");
        sum += f;
    }
    for (auto& m : ctx->step_marks) { ctx->ev_pool.push_back(m.first); ctx->ev_pool.push_back(m.second); }
    for (auto& m : ctx->fin_marks) ctx->ev_pool.push_back(m.second);
    ctx->step_marks.clear();
    ctx->fin_marks.clear();
    *ms = sum;
    return st;
}

// Time the candidate tilings of a request's class and enter the fastest in
// the table (ctx->mu held by the caller).
static ps_status tune_request(Ctx* ctx, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                              hipStream_t after, ps_tune_result* res) {
    ps_status st = validate_object(obj);
    if (st != PS_OK) return st;
    if ((st = validate_receive(rx, obj)) != PS_OK) return st;
    {
        Program full;
        std::string err;
        if ((st = compile_sequence(seq, &full, &err)) != PS_OK) return fail(st, err);
    }
    const int n_coils = rx ? rx->n_coils : 0;
    const TuneKey key = tune_key(ctx, obj->n_spins, seq, n_coils);
    const int rule_S = threshold_spins_per_lane(ctx, obj->n_spins, seq);
    const int32_t base_rep = (ctx->cfg.flags & PS_CFG_NO_READOUT_SPLIT) ? REPLICAS_NONE : REPLICAS_RULE;

    ps_sequence probe = *seq;
    probe.n_events = probe_events(seq, obj->n_spins);
    Program pp;
    std::string err;
    if ((st = compile_sequence(&probe, &pp, &err)) != PS_OK) return fail(st, err);
    plan_slices(&pp, int64_t(1) << 40);        // one slice: the readouts a tile's replicas can share
    if (ctx->cfg.precision != 64 && !(ctx->cfg.flags & PS_CFG_NO_MATRIX_READOUT)) mark_matrix_readouts(&pp);
    assign_shape_slots(&pp, kShapeSlots);
    if (res) res->probe_events = probe.n_events;

    // candidates: every spins-per-lane value of the precision with the
    // replica rule, and for tilings whose tiles leave compute units idle
    // also without replicas and with twice the rule's count
    std::vector<Tiling> cands;
    const int max_S = ctx->cfg.precision == 64 ? 2 : 8;
    for (int S = 1; S <= max_S; S *= 2) {
        cands.push_back(Tiling{S, base_rep, true});
        if (base_rep == REPLICAS_NONE || obj->n_spins == 0) continue;
        const int64_t tiles = (obj->n_spins + spins_per_block_of(S) - 1) / spins_per_block_of(S);
        const ReplicaBound b = replica_bound(pp, std::max(n_coils, 1));
        const int64_t slots = device_slots(ctx, S, pp);
        const int rule = replica_split(ctx, tiles, b, REPLICAS_RULE, slots).replicas;
        if (rule > 1) cands.push_back(Tiling{S, REPLICAS_NONE, true});
        if (rule > 1 && replica_split(ctx, tiles, b, REPLICAS_DOUBLE, slots).replicas > rule)
            cands.push_back(Tiling{S, REPLICAS_DOUBLE, true});
    }
    if ((int)cands.size() > PS_TUNE_MAX_CANDIDATES) cands.resize(PS_TUNE_MAX_CANDIDATES);

    const int64_t n_out = std::max(n_coils, 1);
    const size_t sig_bytes = (size_t)std::max<int64_t>(pp.n_samples * 2 * n_out, 1) * sizeof(double);
    DevBuf signal;
    if ((st = signal.reserve(sig_bytes)) != PS_OK) return st;
    ProbeStream ps_;
    hipError_t e = hipStreamCreateWithFlags(&ps_.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ps_.after, hipEventDisableTiming);
    // the probe reads the object: start after the work queued before it
    if (e == hipSuccess) e = hipEventRecord(ps_.after, after);
    if (e == hipSuccess) e = hipStreamWaitEvent(ps_.stream, ps_.after, 0);
    if (e != hipSuccess) { signal.release(); return hip_fail(e, "autotuner stream"); }

    // the probe runs are timed by the context's kernel-timing marks (device
    // time of their step and finalize kernels, not of the host compile);
    // the caller's own marks are set aside meanwhile
    const int32_t flags_saved = ctx->cfg.flags;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> user_step, user_fin;
    std::swap(user_step, ctx->step_marks);
    std::swap(user_fin, ctx->fin_marks);
    ctx->cfg.flags |= PS_CFG_KERNEL_TIMING;
    // rounds over all candidates, so that each is timed in the same device
    // state (clocks ramp up during the first runs: candidates timed one
    // after another favoured the later ones on short probes)
    std::vector<double> ms(cands.size(), 0.0);
    std::vector<std::vector<double>> t(cands.size());
    for (int round = 0; round <= kTimedRounds && st == PS_OK; ++round) {
        for (size_t c = 0; c < cands.size() && st == PS_OK; ++c) {
            st = run_request(ctx, obj, &probe, reinterpret_cast<double*>(signal.ptr), pp.n_samples, ps_.stream,
                             &cands[c], rx);
            double f = 0.0;
            const ps_status dst = drain_marks(ctx, &f);
            if (st == PS_OK) st = dst;
            if (round > 0) t[c].push_back(f);     // the first round warms up
        }
    }
    for (size_t c = 0; c < cands.size() && st == PS_OK; ++c) {
        std::sort(t[c].begin(), t[c].end());
        ms[c] = t[c][t[c].size() / 2];
    }
    ctx->cfg.flags = flags_saved;
    std::swap(user_step, ctx->step_marks);
    std::swap(user_fin, ctx->fin_marks);
    (void)hipStreamSynchronize(ps_.stream);
    signal.release();
    if (st != PS_OK) return st;

    // the rule's tiling is kept unless a candidate beats it by more than 3 %;
    // a small request (probe under kShortProbeMs) needs 15 % to move to
    // another spins-per-lane value: batched and served rounds run one
    // kernel per spins-per-lane class, one after another, so a small class
    // moved off the rule's value stops sharing a persistent kernel with the
    // others, which the probe of one request does not see (c4: two classes
    // moved, each 12-13 % faster alone, made the batch 17 % slower)
    size_t rule_c = 0;
    for (size_t c = 0; c < cands.size(); ++c)
        if (cands[c].S == rule_S && cands[c].replicas == base_rep) rule_c = c;
    size_t best = rule_c;
    for (size_t c = 0; c < cands.size(); ++c) {
        const double need = cands[c].S == rule_S || ms[rule_c] >= kShortProbeMs ? 0.97 : 0.85;
        if (ms[c] < need * ms[rule_c] && ms[c] < ms[best]) best = c;
    }
    TuneEntry ent;
    ent.tiling = cands[best];
    ent.tiling.tuned = true;
    ent.best_ms = ms[best];
    ent.rule_ms = ms[rule_c];
    ctx->tuned[key] = ent;
    if (res) {
        res->n_candidates = (int32_t)cands.size();
        for (size_t c = 0; c < cands.size(); ++c) {
            res->cand_spins_per_lane[c] = cands[c].S;
            res->cand_replicas[c] = cands[c].replicas;
            res->cand_ms[c] = ms[c];
        }
    }
    return PS_OK;
}

static void fill_result(const TuneEntry& ent, ps_tune_result* res) {
    if (!res) return;
    res->spins_per_lane = ent.tiling.S;
    res->replicas = ent.tiling.replicas;
    res->best_ms = ent.best_ms;
    res->rule_ms = ent.rule_ms;
}

ps_status autotune_if_new(Ctx* ctx, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                          hipStream_t after) {
    if (!(ctx->cfg.flags & PS_CFG_AUTOTUNE) || ctx->cfg.spins_per_lane > 0) return PS_OK;
    if (!obj || !seq || obj->n_spins <= 0) return PS_OK;   // invalid requests fail in the call itself
    if (validate_object(obj) != PS_OK || validate_receive(rx, obj) != PS_OK) return PS_OK;
    {
        Program p;
        std::string err;
        if (compile_sequence(seq, &p, &err) != PS_OK || p.n_samples == 0) return PS_OK;
    }
    clear_error();
    if (ctx->tuned.count(tune_key(ctx, obj->n_spins, seq, rx ? rx->n_coils : 0))) return PS_OK;
    return tune_request(ctx, obj, seq, rx, after, nullptr);
}

static const char* kTuneMagic = "parspin-tune 1";

static std::string device_tag(const Ctx* ctx) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->cfg.device) == hipSuccess) arch = prop.gcnArchName;
    for (char& c : arch)
        if (c == ' ') c = '_';
    return arch + " " + std::to_string(ctx->n_cu) + " " + PS_LIB_HASH;
}

}  // namespace ps

using namespace ps;

extern "C" {

ps_status ps_tune(ps_ctx* handle, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                  uint32_t flags, ps_tune_result* out) {
    clear_error();
    if (!handle || !obj || !seq) return fail(PS_E_INVALID_ARG, "ctx, obj or seq is NULL");
    if (flags & ~(uint32_t)PS_TUNE_FORCE) return fail(PS_E_INVALID_ARG, "unknown tune flags");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) return fail(PS_E_INVALID_ARG, "a scheduler-test context runs no kernels");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    if (out) std::memset(out, 0, sizeof(*out));
    if (ctx->cfg.spins_per_lane > 0)
        return fail(PS_E_INVALID_ARG, "the context's spins_per_lane is fixed; the tuner needs 0");
    if (obj->n_spins <= 0) return fail(PS_E_INVALID_ARG, "the tuner needs an object with spins");
    const TuneKey key = tune_key(ctx, obj->n_spins, seq, rx ? rx->n_coils : 0);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end() && !(flags & PS_TUNE_FORCE)) {
        fill_result(it->second, out);
        if (out) out->from_table = 1;
        return PS_OK;
    }
    ps_status st = tune_request(ctx, obj, seq, rx, nullptr, out);
    if (st != PS_OK) return st;
    fill_result(ctx->tuned[key], out);
    return PS_OK;
}

ps_status ps_tile_for(ps_ctx* handle, int64_t n_spins, const ps_sequence* seq, int32_t n_coils,
                      int32_t* spins_per_lane, int32_t* replicas, int32_t* tuned) {
    clear_error();
    if (!handle || !seq) return fail(PS_E_INVALID_ARG, "ctx or seq is NULL");
    if (n_spins < 0 || n_coils < 0) return fail(PS_E_INVALID_ARG, "n_spins or n_coils < 0");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    std::lock_guard<std::mutex> lk(ctx->mu);
    const Tiling t = choose_tiling(ctx, n_spins, seq, n_coils);
    if (spins_per_lane) *spins_per_lane = t.S;
    if (replicas) *replicas = t.replicas;
    if (tuned) *tuned = t.tuned ? 1 : 0;
    return PS_OK;
}

ps_status ps_readout_path(ps_ctx* handle, int64_t n_spins, const ps_sequence* seq, int32_t n_coils,
                          int32_t spins_per_lane, int64_t* n_readouts, int64_t* n_matrix, int32_t* matrix_only,
                          int64_t* n_slices) {
    clear_error();
    if (!handle || !seq) return fail(PS_E_INVALID_ARG, "ctx or seq is NULL");
    if (n_spins < 0) return fail(PS_E_INVALID_ARG, "n_spins < 0");
    if (n_coils < 0) return fail(PS_E_INVALID_ARG, "n_coils < 0");
    if (spins_per_lane != 1 && spins_per_lane != 2 && spins_per_lane != 4 && spins_per_lane != 8)
        return fail(PS_E_INVALID_ARG, "spins_per_lane must be 1, 2, 4 or 8");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    std::lock_guard<std::mutex> lk(ctx->mu);
    // the plan ps_simulate_rx makes for the request at this tiling
    const int64_t spb = spins_per_block_of(spins_per_lane);
    const int64_t n_rows = (n_spins + spb - 1) / spb * rows_per_block_of(spins_per_lane);
    Program p;
    const ps_status st = prepare(ctx, seq, n_rows, spins_per_lane, &p, n_coils);
    if (st != PS_OK) return st;
    const bool fp32 = ctx->cfg.precision != 64;
    int64_t n = 0, m = 0;
    for (const Op& op : p.ops) {
        if (op.kind != OP_ADC && op.kind != OP_ADCT) continue;
        ++n;
        if (fp32 && spins_per_lane == 1 && (op.flags & OPF_MATRIX)) ++m;
    }
    if (n_readouts) *n_readouts = n;
    if (n_matrix) *n_matrix = m;
    if (matrix_only) *matrix_only = fp32 && spins_per_lane == 1 && p.matrix_only ? 1 : 0;
    if (n_slices) *n_slices = (int64_t)p.slices.size();
    return PS_OK;
}

ps_status ps_tune_save(ps_ctx* handle, const char* path) {
    clear_error();
    if (!handle || !path) return fail(PS_E_INVALID_ARG, "ctx or path is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    std::lock_guard<std::mutex> lk(ctx->mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(PS_E_INVALID_ARG, std::string("cannot write ") + path);
    std::fprintf(f, "%s\n%s\n", kTuneMagic, device_tag(ctx).c_str());
    for (const auto& kv : ctx->tuned) {
        const TuneKey& k = kv.first;
        const TuneEntry& v = kv.second;
        std::fprintf(f, "%d %d %d %d %d %d %d %.6f %.6f\n", k.precision, k.spins_log2, k.readout_log2, k.shaped,
                     k.coils_log2, v.tiling.S, v.tiling.replicas, v.best_ms, v.rule_ms);
    }
    const bool ok = std::fflush(f) == 0;
    std::fclose(f);
    return ok ? PS_OK : fail(PS_E_INVALID_ARG, std::string("write error on ") + path);
}

ps_status ps_tune_load(ps_ctx* handle, const char* path, int32_t* n_loaded) {
    clear_error();
    if (!handle || !path) return fail(PS_E_INVALID_ARG, "ctx or path is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (n_loaded) *n_loaded = 0;
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(PS_E_INVALID_ARG, std::string("cannot read ") + path);
    char line[512];
    std::vector<std::pair<TuneKey, TuneEntry>> rows;
    ps_status st = PS_OK;
    if (!std::fgets(line, sizeof line, f) || std::strncmp(line, kTuneMagic, std::strlen(kTuneMagic)) != 0) {
        st = fail(PS_E_INVALID_ARG, std::string(path) + " is not a tiling table");
    } else if (!std::fgets(line, sizeof line, f) ||
               std::string(line).substr(0, std::strcspn(line, "\r\n")) != device_tag(ctx)) {
        st = fail(PS_E_INVALID_ARG, std::string(path) + " was tuned on another device or library build");
    } else {
        const int max_S = ctx->cfg.precision == 64 ? 2 : 8;
        while (std::fgets(line, sizeof line, f)) {
            TuneKey k;
            TuneEntry v;
            int S = 0, rep = 0;
            if (std::sscanf(line, "%d %d %d %d %d %d %d %lf %lf", &k.precision, &k.spins_log2, &k.readout_log2,
                            &k.shaped, &k.coils_log2, &S, &rep, &v.best_ms, &v.rule_ms) != 9 ||
                (S != 1 && S != 2 && S != 4 && S != 8) || rep < REPLICAS_NONE || rep > REPLICAS_DOUBLE) {
                st = fail(PS_E_INVALID_ARG, std::string("malformed line in ") + path);
                break;
            }
            if (k.precision != ctx->cfg.precision || S > max_S) continue;   // another context's entries
            v.tiling = Tiling{S, rep, true};
            rows.emplace_back(k, v);
        }
    }
    std::fclose(f);
    if (st != PS_OK) return st;
    for (auto& r : rows) ctx->tuned[r.first] = r.second;
    if (n_loaded) *n_loaded = (int32_t)rows.size();
    return PS_OK;
}

ps_status ps_tune_clear(ps_ctx* handle) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tuned.clear();
    return PS_OK;
}

}  // extern "C"
