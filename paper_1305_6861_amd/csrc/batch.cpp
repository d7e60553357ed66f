// Batched execution: many independent requests per persistent launch.
//
// The paper spreads spin blocks over workstations dynamically, with more
// blocks than nodes so that faster nodes simply take more (section 5.3.2).
// Here every request is cut into workgroup tiles, all tiles of all requests
// form one queue, and a persistent kernel's workgroups pull from it.  A tile
// writes only its own request's partial rows, and each request keeps the
// tiling and time slicing it would get alone (both depend only on its own
// size), so a request's result is bitwise the same alone (ps_simulate) or in
// any batch.  Requests longer than one time slice run one slice per round,
// their anchors kept in HBM between rounds.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/parspin.h"
#include "batch.h"
#include "ps_kernels.h"
#include "ps_runtime.h"

namespace ps {

static size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

ps_status plan_request(const Ctx* ctx, const ps_object* obj, const ps_sequence* seq, int64_t n_samples,
                       double* signal, int64_t max_slice_steps, ReqPlan* p) {
    ps_status st = validate_object(obj);
    if (st != PS_OK) return st;
    p->obj = *obj;
    p->signal = signal;
    const Tiling tl = choose_tiling(ctx, obj->n_spins, seq, 0);
    p->S = tl.S;
    p->replica_mode = tl.replicas;
    const int64_t spb = spins_per_block_of(p->S);
    p->n_blocks = (obj->n_spins + spb - 1) / spb;
    p->n_rows = p->n_blocks * rows_per_block_of(p->S);
    if ((st = prepare(ctx, seq, p->n_rows, p->S, &p->prog)) != PS_OK) return st;
    if (max_slice_steps > 0) {
        // a second bound for serving: at most max_slice_steps intervals per
        // spin per slice, so that long requests yield the device regularly
        Program& g = p->prog;
        std::vector<Slice> out;
        for (const Slice& sl : g.slices) {
            Slice cur = sl;
            int64_t steps = 0;
            int64_t samples_before = 0;
            for (int64_t i = sl.op_begin; i < sl.op_end; ++i) {
                const Op& op = g.ops[i];
                const int64_t w = (op.kind == OP_ADC || op.kind == OP_ADCT || op.kind == OP_SHAPE) ? op.n : 1;
                if (steps > 0 && steps + w > max_slice_steps) {
                    // cut before op i; ADC offsets restart at the new slice
                    cur.op_end = i;
                    cur.n_samples = samples_before;
                    out.push_back(cur);
                    cur = Slice();
                    cur.op_begin = i;
                    cur.sample_begin = out.back().sample_begin + out.back().n_samples;
                    steps = 0;
                    samples_before = 0;
                }
                if (op.kind == OP_ADC || op.kind == OP_ADCT) {
                    g.ops[i].aux = (uint32_t)samples_before;
                    samples_before += op.n;
                }
                steps += w;
            }
            cur.op_end = sl.op_end;
            cur.n_samples = samples_before;
            out.push_back(cur);
        }
        g.slices = std::move(out);
        assign_shape_slots(&g, shape_cache_slots(ctx, p->S, g));
    }
    p->max_replicas = replica_bound(p->prog, 1);
    if (n_samples != p->prog.n_samples)
        return fail(PS_E_INVALID_ARG, "n_samples (" + std::to_string(n_samples) + ") differs from the sequence's " +
                                          std::to_string(p->prog.n_samples));
    if (n_samples > 0 && !signal) return fail(PS_E_INVALID_ARG, "signal is NULL");
    int64_t max_slice = 0;
    for (const Slice& s : p->prog.slices) max_slice = std::max(max_slice, s.n_samples);
    p->row_stride = pad_fin(2 * max_slice);
    p->n_groups = (p->n_rows + row_group_size() - 1) / row_group_size();
    const size_t rb = ctx->cfg.precision == 64 ? 8 : 4;
    p->bytes_partial = align_up((size_t)(p->n_rows * p->row_stride) * rb);
    p->bytes_state = p->prog.slices.size() > 1
                         ? align_up((size_t)(state_reals_per_spin(p->prog.n_state_slots) * obj->n_spins) * rb)
                         : 0;
    p->bytes_mid = p->n_groups > 1 ? align_up((size_t)(p->n_groups * p->row_stride) * sizeof(double)) : 0;
    p->bytes_ops = align_up(p->prog.ops.size() * sizeof(Op));
    p->bytes_rows = align_up(p->prog.rows.size() * sizeof(double));
    p->bytes_traj = align_up(p->prog.traj.size() * sizeof(double));
    return PS_OK;
}

size_t ReqPlan::device_bytes() const {
    return bytes_partial + bytes_state + bytes_mid + bytes_ops + bytes_rows + bytes_traj;
}

size_t ReqPlan::footprint() const {
    return device_bytes() + (size_t)obj.n_spins * 7 * sizeof(float) + (size_t)prog.n_samples * 2 * sizeof(double);
}

size_t ReqPlan::table_bytes() const { return bytes_ops + bytes_rows + bytes_traj; }

void ReqPlan::bind_work(unsigned char* w) {
    d_partial = w; w += bytes_partial;
    d_state = bytes_state ? w : nullptr; w += bytes_state;
    d_mid = bytes_mid ? reinterpret_cast<double*>(w) : nullptr;
}

void ReqPlan::bind_tables(unsigned char* t) {
    d_ops = reinterpret_cast<Op*>(t); t += bytes_ops;
    d_rows = reinterpret_cast<double*>(t); t += bytes_rows;
    d_traj = reinterpret_cast<double*>(t);
}

void ReqPlan::bind(unsigned char* base) {
    bind_work(base);
    bind_tables(base + bytes_partial + bytes_state + bytes_mid);
}

StepArgs ReqPlan::args_for_slice(size_t k, int n_replicas) const {
    const Slice& sl = prog.slices[k];
    StepArgs a{};
    a.x = obj.x; a.y = obj.y; a.z = obj.z; a.m0 = obj.m0; a.t1 = obj.t1; a.t2 = obj.t2; a.dw = obj.dw;
    a.n_spins = obj.n_spins;
    a.ops = d_ops + sl.op_begin;
    a.n_ops = (int32_t)(sl.op_end - sl.op_begin);
    a.n_shape_rows = (int32_t)(prog.rows.size() / 9);
    a.rows = d_rows;
    a.traj = d_traj;
    a.partial = d_partial;
    a.row_stride = row_stride;
    a.state = d_state;
    a.load_state = k > 0;
    a.save_state = k + 1 < prog.slices.size();
    a.anchor_parity = (int32_t)(k & 1);
    a.n_cache_slots = sl.n_cache_slots;
    a.cache_load = sl.cache_load;
    a.cache_save = sl.cache_save;
    a.n_coils = 0;
    a.s_x = nullptr;
    a.s_y = nullptr;
    a.coil_stride = row_stride;
    a.snaps = nullptr;
    a.n_replicas = std::max(n_replicas, 1);
    a.n_tiles = n_blocks;
    for (int d = 0; d < 3; ++d) a.mx_mu[d] = prog.matrix_mu[d];
    a.mx_tau = prog.matrix_tau;
    return a;
}

// Rough work per spin of one slice of a request: one unit per sample and
// sub-step, a few for every other operation.
static int64_t slice_cost(const ReqPlan& p, size_t k) {
    const Slice& sl = p.prog.slices[k];
    int64_t c = 0;
    for (int64_t i = sl.op_begin; i < sl.op_end; ++i) {
        const Op& op = p.prog.ops[i];
        const bool counted = op.kind == OP_ADC || op.kind == OP_ADCT ||
                             (op.kind == OP_SHAPE && op.u.shape.mode != SHAPE_APPLY);
        c += counted ? (int64_t)op.n : 8;
    }
    return c;
}

ps_status build_rounds(const Ctx* ctx, std::vector<ReqPlan*>& plans, const std::vector<size_t>& first_slice,
                       const std::vector<size_t>& n_slices_this_call, std::vector<unsigned char>* img_out,
                       std::vector<RoundImage>* rounds_out) {
    size_t max_rounds = 0;
    for (size_t i = 0; i < plans.size(); ++i) max_rounds = std::max(max_rounds, n_slices_this_call[i]);
    std::vector<unsigned char>& img = *img_out;
    img.clear();
    auto reserve_bytes = [&](size_t n) {
        const size_t off = align_up(img.size(), 64);
        img.resize(off + n);
        return off;
    };
    std::vector<RoundImage>& rounds = *rounds_out;
    rounds.assign(max_rounds, RoundImage());
    for (size_t k = 0; k < max_rounds; ++k) {
        RoundImage& R = rounds[k];
        // one launch per kernel: spins per lane, and the kernel variant
        // (step_variant) at one spin per lane
        std::map<std::pair<int, int>, std::vector<size_t>> by_S;
        for (size_t i = 0; i < plans.size(); ++i)
            if (k < n_slices_this_call[i] && plans[i]->obj.n_spins > 0) {
                const Program& g = plans[i]->prog;
                by_S[{plans[i]->S, step_variant(ctx->cfg.precision, plans[i]->S, g.matrix_only, g.any_matrix)}]
                    .push_back(i);
            }
        for (auto& kv : by_S) {
            // Longest tiles first: workgroups take items in record order, so
            // the requests whose tiles take longest start first and short
            // ones fill the end of the launch (which workgroup runs an item
            // never changes a result).
            std::vector<int64_t> cost(plans.size(), 0);
            for (size_t i : kv.second) cost[i] = slice_cost(*plans[i], first_slice[i] + k);
            std::stable_sort(kv.second.begin(), kv.second.end(),
                             [&](size_t a, size_t b) { return cost[a] > cost[b]; });
            RoundImage::Class c;
            c.S = kv.first.first;
            c.variant = kv.first.second;
            c.n_req = (int32_t)kv.second.size();
            c.items_off = reserve_bytes(sizeof(BatchItem) * kv.second.size());
            c.counter_off = reserve_bytes(sizeof(unsigned long long));
            int64_t total = 0;
            size_t dyn = 0;
            // readout replicas when the round's tiles of this class leave CUs idle
            int64_t tiles = 0;
            for (size_t q = 0; q < kv.second.size(); ++q) tiles += plans[kv.second[q]]->n_blocks;
            for (size_t q = 0; q < kv.second.size(); ++q) {
                ReqPlan* p = plans[kv.second[q]];
                const int R = replicas_for_load(ctx, tiles, p->max_replicas, p->replica_mode);
                BatchItem it;
                std::memset(&it, 0, sizeof(it));
                it.args = p->args_for_slice(first_slice[kv.second[q]] + k, R);
                it.item_begin = total;
                it.n_items = p->n_blocks * R;
                total += it.n_items;
                dyn = std::max(dyn, step_dyn_lds_bytes(ctx->cfg.precision, c.S, it.args.n_shape_rows,
                                                       it.args.n_cache_slots, c.variant));
                std::memcpy(img.data() + c.items_off + q * sizeof(BatchItem), &it, sizeof(it));
            }
            c.total = total;
            c.dyn_lds = dyn;
            std::memset(img.data() + c.counter_off, 0, sizeof(unsigned long long));
            R.classes.push_back(c);
        }
        // finalize records for requests whose slice k has samples
        std::vector<FinDesc> fd;
        for (size_t i = 0; i < plans.size(); ++i) {
            if (k >= n_slices_this_call[i]) continue;
            ReqPlan* p = plans[i];
            const Slice& sl = p->prog.slices[first_slice[i] + k];
            if (sl.n_samples == 0 || p->obj.n_spins == 0) continue;   // empty objects are zero-filled apart
            FinDesc f;
            std::memset(&f, 0, sizeof(f));
            f.partial = p->d_partial;
            f.n_rows = p->n_rows;
            f.row_stride = p->row_stride;
            f.n_vals = 2 * sl.n_samples;
            f.n_groups = p->n_groups;
            f.out = p->signal + 2 * sl.sample_begin;
            f.mid = p->d_mid;
            fd.push_back(f);
        }
        // prefix sums of the pass-1 blocks (kFinVals values a thread) and
        // pass-2 blocks (one value a thread)
        int64_t t1 = 0, t2 = 0;
        for (FinDesc& f : fd) {
            f.tile_begin1 = t1; f.tile_begin2 = t2;
            t1 += std::max<int64_t>(f.n_groups, 1) * finalize_tiles(f.n_vals);
            if (f.n_groups > 1) t2 += (f.n_vals + 255) / 256;
        }
        R.n_fin = (int32_t)fd.size();
        R.tiles1 = t1; R.tiles2 = t2;
        if (!fd.empty()) {
            R.fin_off = reserve_bytes(sizeof(FinDesc) * fd.size());
            std::memcpy(img.data() + R.fin_off, fd.data(), sizeof(FinDesc) * fd.size());
        }
    }
    return PS_OK;
}

ps_status round_nodes(const Ctx* ctx, const RoundImage& R, unsigned char* dev, std::vector<KernelNode>* nodes) {
    for (const RoundImage::Class& c : R.classes) {
        const hipError_t e = batch_step_nodes(reinterpret_cast<const BatchItem*>(dev + c.items_off), c.n_req,
                                              c.total, reinterpret_cast<unsigned long long*>(dev + c.counter_off),
                                              c.dyn_lds, ctx->cfg.precision, c.S, ctx->n_cu, nodes, c.variant);
        if (e != hipSuccess) return hip_fail(e, "batch step node");
    }
    if (R.n_fin > 0) {
        const hipError_t e = batch_finalize_nodes(reinterpret_cast<const FinDesc*>(dev + R.fin_off), R.n_fin,
                                                  R.tiles1, R.tiles2, ctx->cfg.precision, nodes);
        if (e != hipSuccess) return hip_fail(e, "batch finalize node");
    }
    return PS_OK;
}

ps_status run_rounds(Ctx* ctx, std::vector<ReqPlan*>& plans, const std::vector<size_t>& first_slice,
                     const std::vector<size_t>& n_slices_this_call, hipStream_t stream, DevBuf& arena,
                     HostBuf& staging) {
    // plans[i] runs slices first_slice[i] .. first_slice[i] + n_slices_this_call[i] - 1,
    // one per round.  Tables (ops, rows) must already be resident (uploaded by the caller).
    std::vector<unsigned char> img;
    std::vector<RoundImage> rounds;
    ps_status st = build_rounds(ctx, plans, first_slice, n_slices_this_call, &img, &rounds);
    if (st != PS_OK || img.empty()) return st;
    if ((st = arena.reserve(img.size())) != PS_OK) return st;
    if ((st = staging.reserve(img.size())) != PS_OK) return st;
    std::memcpy(staging.ptr, img.data(), img.size());
    hipError_t e = hipMemcpyAsync(arena.ptr, staging.ptr, img.size(), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch records)");
    unsigned char* dev = reinterpret_cast<unsigned char*>(arena.ptr);
    std::vector<KernelNode> nodes;
    for (const RoundImage& R : rounds) {
        nodes.clear();
        if ((st = round_nodes(ctx, R, dev, &nodes)) != PS_OK) return st;
        for (KernelNode& n : nodes)
            if ((e = n.launch(stream)) != hipSuccess) return hip_fail(e, "batch launch");
    }
    return PS_OK;
}

ps_status upload_tables(std::vector<ReqPlan*>& plans, HostBuf& staging, size_t staging_off, hipStream_t stream) {
    size_t need = 0;
    for (ReqPlan* p : plans) need += p->bytes_ops + p->bytes_rows + p->bytes_traj;
    ps_status st;
    if ((st = staging.reserve(staging_off + need)) != PS_OK) return st;
    unsigned char* h = reinterpret_cast<unsigned char*>(staging.ptr) + staging_off;
    for (ReqPlan* p : plans) {
        const size_t ob = p->prog.ops.size() * sizeof(Op), rb = p->prog.rows.size() * sizeof(double);
        if (ob) {
            std::memcpy(h, p->prog.ops.data(), ob);
            hipError_t e = hipMemcpyAsync(p->d_ops, h, ob, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(ops)");
            h += p->bytes_ops;
        }
        if (rb) {
            std::memcpy(h, p->prog.rows.data(), rb);
            hipError_t e = hipMemcpyAsync(p->d_rows, h, rb, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(rows)");
            h += p->bytes_rows;
        }
        const size_t tb = p->prog.traj.size() * sizeof(double);
        if (tb) {
            std::memcpy(h, p->prog.traj.data(), tb);
            hipError_t e = hipMemcpyAsync(p->d_traj, h, tb, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(trajectories)");
            h += p->bytes_traj;
        }
    }
    return PS_OK;
}

ps_status upload_tables_contiguous(std::vector<ReqPlan*>& plans, void* dev, HostBuf& staging, hipStream_t stream) {
    size_t need = 0;
    for (ReqPlan* p : plans) need += p->table_bytes();
    if (need == 0) return PS_OK;
    ps_status st;
    if ((st = staging.reserve(need)) != PS_OK) return st;
    unsigned char* h0 = reinterpret_cast<unsigned char*>(staging.ptr);
    unsigned char* h = h0;
    for (ReqPlan* p : plans) {
        // the host image mirrors bind_tables: ops, rows, trajectories, each
        // in its 256-byte aligned slot
        if (!p->prog.ops.empty()) std::memcpy(h, p->prog.ops.data(), p->prog.ops.size() * sizeof(Op));
        if (!p->prog.rows.empty())
            std::memcpy(h + p->bytes_ops, p->prog.rows.data(), p->prog.rows.size() * sizeof(double));
        if (!p->prog.traj.empty())
            std::memcpy(h + p->bytes_ops + p->bytes_rows, p->prog.traj.data(), p->prog.traj.size() * sizeof(double));
        h += p->table_bytes();
    }
    hipError_t e = hipMemcpyAsync(dev, h0, need, hipMemcpyHostToDevice, stream);
    return e == hipSuccess ? PS_OK : hip_fail(e, "hipMemcpyAsync(tables)");
}

}  // namespace ps

using namespace ps;

extern "C" ps_status ps_simulate_batch(ps_ctx* handle, int32_t n_requests, const ps_object* objs,
                                       const ps_sequence* seqs, double* const* signals, const int64_t* n_samples,
                                       void* stream_v) {
    clear_error();
    if (!handle) return fail(PS_E_INVALID_ARG, "ctx is NULL");
    if (n_requests < 0) return fail(PS_E_INVALID_ARG, "n_requests < 0");
    if (n_requests == 0) return PS_OK;
    if (!objs || !seqs || !signals || !n_samples) return fail(PS_E_INVALID_ARG, "NULL request array");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) return fail(PS_E_INVALID_ARG, "a scheduler-test context runs no kernels");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);
    for (int32_t i = 0; i < n_requests; ++i) {
        const ps_status tst = autotune_if_new(ctx, &objs[i], &seqs[i], nullptr, stream);
        if (tst != PS_OK) return fail(tst, "request " + std::to_string(i) + ": " + ps_last_error());
    }
    std::vector<ReqPlan> plans((size_t)n_requests);
    {
        // Compiling the requests' sequences is independent host work: spread
        // it over a few threads (errors are thread-local, so each request's
        // message is kept and reported from this thread).
        std::vector<ps_status> sts((size_t)n_requests, PS_OK);
        std::vector<std::string> errs((size_t)n_requests);
        std::atomic<int32_t> next{0};
        auto work = [&]() {
            for (int32_t i; (i = next.fetch_add(1)) < n_requests;) {
                sts[i] = plan_request(ctx, &objs[i], &seqs[i], n_samples[i], signals[i], 0, &plans[i]);
                if (sts[i] != PS_OK) errs[i] = ps_last_error();
            }
        };
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const int n_threads = (int)std::min<unsigned>(std::min<unsigned>(hw, 8u), (unsigned)((n_requests + 7) / 8));
        std::vector<std::thread> pool;
        try {
            for (int t = 1; t < n_threads; ++t) pool.emplace_back(work);
        } catch (...) {
            // no more threads: the calling thread does the rest
        }
        work();
        for (std::thread& t : pool) t.join();
        for (int32_t i = 0; i < n_requests; ++i)
            if (sts[i] != PS_OK) return fail(sts[i], "request " + std::to_string(i) + ": " + errs[i]);
    }
    ps_status st;
    BufSet* set = nullptr;
    if ((st = acquire_set(ctx, &set)) != PS_OK) return st;
    // all requests' tables first (one upload), then their work buffers
    size_t tables = 0, total = 0;
    for (ReqPlan& p : plans) {
        tables += p.table_bytes();
        total += p.device_bytes();
    }
    if ((st = set->batch_tables.reserve(std::max<size_t>(total, 256))) != PS_OK) return st;
    unsigned char* tbase = reinterpret_cast<unsigned char*>(set->batch_tables.ptr);
    unsigned char* base = tbase + tables;
    std::vector<ReqPlan*> ptrs;
    std::vector<ReqPlan*> with_tables;
    std::vector<size_t> first, count;
    for (ReqPlan& p : plans) {
        p.bind_tables(tbase);
        tbase += p.table_bytes();
        p.bind_work(base);
        base += p.device_bytes() - p.table_bytes();
        with_tables.push_back(&p);
        if (p.prog.n_samples == 0) continue;
        if (p.obj.n_spins == 0) {
            hipError_t e = launch_fill_zero(p.signal, 2 * p.prog.n_samples, stream);
            if (e != hipSuccess) return hip_fail(e, "fill");
            continue;
        }
        ptrs.push_back(&p);
        first.push_back(0);
        count.push_back(p.prog.slices.size());
    }
    if (ptrs.empty()) return PS_OK;
    st = upload_tables_contiguous(with_tables, set->batch_tables.ptr, set->staging, stream);
    if (st == PS_OK) st = run_rounds(ctx, ptrs, first, count, stream, set->batch_records, set->staging2);
    // the set's staging may be in a copy on `stream` even after a failure
    const ps_status rel = release_set_after(set, stream);
    return st != PS_OK ? st : rel;
}
