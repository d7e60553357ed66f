// Sequence compiler (host, FP64).
//
// Spin-independent work is done once here rather than per spin, as the
// paper's master process precomputes the trigonometry of RF pulses
// (section 6.3): rotation matrices of hard pulses (eq. 3.19) and of every
// sub-pulse of shaped pulses, and the accumulated gradient moments and times
// since each spin's anchors (see ps_ops.h).  Intervals that contain neither
// a pulse, an ADC nor a spoiler compile to nothing.
#include "compile.h"

#include <cmath>
#include <algorithm>
#include <cstring>
#include <map>
#include <utility>

namespace ps {

void rf_matrix(double a, double p, double r[9]) {
    const double ca = std::cos(a), sa = std::sin(a), cp = std::cos(p), sp = std::sin(p);
    r[0] = cp * cp + sp * sp * ca;  r[1] = sp * cp * (1.0 - ca);     r[2] = -sp * sa;
    r[3] = sp * cp * (1.0 - ca);    r[4] = sp * sp + cp * cp * ca;   r[5] = cp * sa;
    r[6] = sp * sa;                 r[7] = -cp * sa;                 r[8] = ca;
}

void rf_delta(double a, double p, double d[9]) {
    // R - I with 1 - cos(a) = 2 sin^2(a/2) so that small pulses keep full
    // relative precision in every entry.
    const double sa = std::sin(a), cp = std::cos(p), sp = std::sin(p);
    const double h = std::sin(0.5 * a);
    const double v = 2.0 * h * h;          // 1 - cos(a)
    d[0] = -sp * sp * v;  d[1] = sp * cp * v;   d[2] = -sp * sa;
    d[3] = sp * cp * v;   d[4] = -cp * cp * v;  d[5] = cp * sa;
    d[6] = sp * sa;       d[7] = -cp * sa;      d[8] = -v;
}

static bool finite(double v) { return std::isfinite(v); }

static Op blank_op(uint32_t kind) {
    Op op;
    std::memset(&op, 0, sizeof(op));
    op.kind = kind;
    return op;
}

ps_status compile_sequence(const ps_sequence* seq, Program* out, std::string* err, bool snapshots) {
    if (!seq || !out) { *err = "null sequence or output"; return PS_E_INVALID_ARG; }
    if (seq->n_events < 0) { *err = "n_events < 0"; return PS_E_INVALID_ARG; }
    if (seq->n_events > 0 && !seq->events) { *err = "events is NULL"; return PS_E_INVALID_ARG; }
    if (seq->n_shapes < 0) { *err = "n_shapes < 0"; return PS_E_INVALID_ARG; }
    if (seq->n_shapes > 0 && !seq->shapes) { *err = "shapes is NULL"; return PS_E_INVALID_ARG; }
    if (seq->n_trajectories < 0) { *err = "n_trajectories < 0"; return PS_E_INVALID_ARG; }
    if (seq->n_trajectories > 0 && !seq->trajectories) { *err = "trajectories is NULL"; return PS_E_INVALID_ARG; }
    for (int32_t j = 0; j < seq->n_trajectories; ++j) {
        const ps_trajectory& tr = seq->trajectories[j];
        const std::string where = "trajectory " + std::to_string(j) + ": ";
        if (tr.n < 1 || tr.n > 0x7fffffffll || !tr.k || !tr.t) { *err = where + "n < 1 or NULL arrays"; return PS_E_INVALID_ARG; }
        double tp = 0.0;
        for (int64_t q = 0; q < tr.n; ++q) {
            if (!finite(tr.t[q]) || tr.t[q] < tp) { *err = where + "times must be finite, >= 0 and non-decreasing"; return PS_E_INVALID_ARG; }
            tp = tr.t[q];
            if (!finite(tr.k[3 * q]) || !finite(tr.k[3 * q + 1]) || !finite(tr.k[3 * q + 2])) {
                *err = where + "moment not finite"; return PS_E_INVALID_ARG;
            }
        }
    }

    for (int32_t s = 0; s < seq->n_shapes; ++s) {
        const ps_rf_shape& sh = seq->shapes[s];
        if (sh.n_sub < 1 || !sh.alpha || !sh.phase) {
            *err = "shape " + std::to_string(s) + ": n_sub < 1 or NULL alpha/phase";
            return PS_E_INVALID_ARG;
        }
        if (!finite(sh.tau) || sh.tau < 0 || !finite(sh.m_sub[0]) || !finite(sh.m_sub[1]) ||
            !finite(sh.m_sub[2])) {
            *err = "shape " + std::to_string(s) + ": tau or m_sub not finite / negative";
            return PS_E_INVALID_ARG;
        }
        for (int32_t q = 0; q < sh.n_sub; ++q)
            if (!finite(sh.alpha[q]) || !finite(sh.phase[q])) {
                *err = "shape " + std::to_string(s) + ": non-finite sub-pulse";
                return PS_E_INVALID_ARG;
            }
    }

    Program p;
    double K[3] = {0, 0, 0};
    double txy = 0, tz = 0;
    bool mxy_zero = true;
    std::map<int32_t, uint32_t> row_of_shape;   // first row of each shape's block

    for (int64_t e = 0; e < seq->n_events; ++e) {
        const ps_event& ev = seq->events[e];
        const std::string where = "event " + std::to_string(e) + ": ";
        if (!finite(ev.dt) || ev.dt < 0) { *err = where + "dt must be finite and >= 0"; return PS_E_INVALID_ARG; }
        if (!finite(ev.m[0]) || !finite(ev.m[1]) || !finite(ev.m[2])) {
            *err = where + "moment not finite"; return PS_E_INVALID_ARG;
        }
        if (!finite(ev.rf_alpha) || !finite(ev.rf_phase)) {
            *err = where + "RF angle not finite"; return PS_E_INVALID_ARG;
        }
        if (ev.rf_shape < -1 || ev.rf_shape >= seq->n_shapes) {
            *err = where + "rf_shape out of range"; return PS_E_INVALID_ARG;
        }
        if (ev.n_adc > 0x7fffffffu) { *err = where + "n_adc too large"; return PS_E_INVALID_ARG; }
        if (ev.flags & ~(PS_EV_SPOIL | PS_EV_SNAPSHOT | PS_EV_TRAJECTORY)) {
            *err = where + "unknown flag bits"; return PS_E_INVALID_ARG;
        }
        const ps_trajectory* tr = nullptr;
        if (ev.flags & PS_EV_TRAJECTORY) {
            if ((int64_t)ev.trajectory >= seq->n_trajectories) { *err = where + "trajectory out of range"; return PS_E_INVALID_ARG; }
            tr = &seq->trajectories[ev.trajectory];
            if ((int64_t)ev.n_adc != tr->n) { *err = where + "n_adc differs from the trajectory's sample count"; return PS_E_INVALID_ARG; }
            if (tr->t[tr->n - 1] > ev.dt) { *err = where + "trajectory runs past the interval"; return PS_E_INVALID_ARG; }
        } else if (ev.trajectory != 0) {
            *err = where + "trajectory must be 0 without PS_EV_TRAJECTORY"; return PS_E_INVALID_ARG;
        }

        if (ev.rf_shape >= 0) {
            const ps_rf_shape& sh = seq->shapes[ev.rf_shape];
            auto it = row_of_shape.find(ev.rf_shape);
            uint32_t first;
            if (it == row_of_shape.end()) {
                first = (uint32_t)(p.rows.size() / 9);
                for (int32_t q = 0; q < sh.n_sub; ++q) {
                    double r[9];
                    rf_delta(sh.alpha[q], sh.phase[q], r);
                    p.rows.insert(p.rows.end(), r, r + 9);
                }
                row_of_shape.emplace(ev.rf_shape, first);
            } else {
                first = it->second;
            }
            Op op = blank_op(OP_SHAPE);
            std::memcpy(op.k, K, sizeof(K));
            op.txy = txy; op.tz = tz;
            op.u.shape.mu[0] = sh.m_sub[0]; op.u.shape.mu[1] = sh.m_sub[1]; op.u.shape.mu[2] = sh.m_sub[2];
            op.u.shape.tau = sh.tau;
            op.u.shape.rot[0] = 1.0; op.u.shape.rot[1] = 0.0;
            if (ev.rf_phase != 0.0) {
                op.u.shape.rot[0] = std::cos(ev.rf_phase);
                op.u.shape.rot[1] = std::sin(ev.rf_phase);
            }
            op.u.shape.slot = -1;
            op.u.shape.mode = SHAPE_DIRECT;
            op.u.shape.shape_id = ev.rf_shape;
            op.n = (uint32_t)sh.n_sub;
            op.aux = first;
            op.flags = mxy_zero ? OPF_MXY_ZERO : 0u;
            p.ops.push_back(op);
            K[0] = K[1] = K[2] = 0; txy = 0; tz = 0; mxy_zero = false;
            p.n_steps += sh.n_sub;
            p.n_shape_substeps += sh.n_sub;
        }

        if (ev.rf_alpha != 0.0) {
            Op op = blank_op(OP_RF);
            std::memcpy(op.k, K, sizeof(K));
            op.txy = txy; op.tz = tz;
            rf_delta(ev.rf_alpha, ev.rf_phase, op.u.r64);
            op.flags = mxy_zero ? OPF_MXY_ZERO : 0u;
            p.ops.push_back(op);
            K[0] = K[1] = K[2] = 0; txy = 0; tz = 0; mxy_zero = false;
            p.n_rf += 1;
        }

        const int64_t n = (int64_t)ev.n_adc;
        if (tr) {
            // samples at tabulated instants: rows hold absolute (moment, time)
            // since the anchors, so any piece of the op can start anywhere
            Op op = blank_op(OP_ADCT);
            std::memcpy(op.k, K, sizeof(K));
            op.txy = txy;
            op.n = (uint32_t)n;
            op.flags = mxy_zero ? OPF_MXY_ZERO : 0u;
            op.u.tab.row = p.traj.size() / 4;
            // instants on a regular raster (spirals and other trajectories
            // sampled at a fixed dwell) let the kernel step the T2 decay from
            // sample to sample by one factor instead of evaluating it at
            // each sample
            if (n >= 2) {
                const double d = (tr->t[n - 1] - tr->t[0]) / (double)(n - 1);
                bool even = d > 0.0;
                for (int64_t q = 1; even && q < n; ++q)
                    even = std::fabs(tr->t[q] - tr->t[0] - (double)q * d) <= 1e-9 * d;
                if (even) { op.flags |= OPF_EVEN_T; op.u.tab.dt = d; }
            }
            for (int64_t q = 0; q < n; ++q) {
                p.traj.push_back(K[0] + tr->k[3 * q]);
                p.traj.push_back(K[1] + tr->k[3 * q + 1]);
                p.traj.push_back(K[2] + tr->k[3 * q + 2]);
                p.traj.push_back(txy + tr->t[q]);
            }
            p.ops.push_back(op);
            p.n_samples += n;
            p.n_adc_ops += 1;
        } else if (n > 0) {
            Op op = blank_op(OP_ADC);
            const double mu[3] = {ev.m[0] / (double)n, ev.m[1] / (double)n, ev.m[2] / (double)n};
            const double tau = ev.dt / (double)n;
            for (int d = 0; d < 3; ++d) { op.k[d] = K[d] + mu[d]; op.u.adc.mu[d] = mu[d]; }
            op.txy = txy + tau;
            op.u.adc.tau = tau;
            op.n = (uint32_t)n;
            op.flags = mxy_zero ? OPF_MXY_ZERO : 0u;
            p.ops.push_back(op);
            p.n_samples += n;
            p.n_adc_ops += 1;
        }
        K[0] += ev.m[0]; K[1] += ev.m[1]; K[2] += ev.m[2];
        txy += ev.dt; tz += ev.dt;
        // intervals per spin: the samples' pieces, plus the rest of a
        // trajectory interval after its last sample
        p.n_steps += n > 0 ? n + (tr && tr->t[n - 1] < ev.dt ? 1 : 0) : 1;

        if (ev.flags & PS_EV_SPOIL) {
            if (!mxy_zero) p.ops.push_back(blank_op(OP_SPOIL));
            K[0] = K[1] = K[2] = 0; txy = 0; mxy_zero = true;
        }
        if (ev.flags & PS_EV_SNAPSHOT) {
            if (snapshots) {
                Op op = blank_op(OP_SNAP);
                std::memcpy(op.k, K, sizeof(K));
                op.txy = txy; op.tz = tz;
                op.flags = mxy_zero ? OPF_MXY_ZERO : 0u;
                op.aux = (uint32_t)p.n_snapshots;
                p.ops.push_back(op);
            }
            p.n_snapshots += 1;
        }
    }
    // Operations after the last readout or snapshot cannot change an output.
    size_t keep = 0;
    for (size_t i = 0; i < p.ops.size(); ++i)
        if (p.ops[i].kind == OP_ADC || p.ops[i].kind == OP_ADCT || p.ops[i].kind == OP_SNAP) keep = i + 1;
    p.ops.resize(keep);
    if ((int64_t)(p.rows.size() / 9) > kMaxShapeRows) {
        *err = "shaped pulses need " + std::to_string(p.rows.size() / 9) +
               " distinct sub-pulse rotations; at most " + std::to_string(kMaxShapeRows) + " are supported";
        return PS_E_TOO_LARGE;
    }
    *out = std::move(p);
    return PS_OK;
}

void plan_slices(Program* p, int64_t max_samples) {
    if (max_samples < 1) max_samples = 1;
    std::vector<Op> ops;
    ops.reserve(p->ops.size());
    p->slices.clear();
    Slice cur;
    cur.op_begin = 0;
    cur.sample_begin = 0;
    int64_t sample = 0;
    auto close_slice = [&]() {
        cur.op_end = (int64_t)ops.size();
        cur.n_samples = sample - cur.sample_begin;
        p->slices.push_back(cur);
        cur = Slice();
        cur.op_begin = (int64_t)ops.size();
        cur.sample_begin = sample;
    };
    // samples [done, done + take) of readout op0 as one or more ops
    auto emit = [&](const Op& op0, int64_t done, int64_t take) {
        // runs of a Cartesian readout: near-equal lengths of at most kAdcRun
        const int64_t runs = op0.kind == OP_ADC ? (take + kAdcRun - 1) / kAdcRun : 1;
        for (int64_t r = 0; r < runs; ++r) {
            const int64_t b = take * r / runs, e = take * (r + 1) / runs;
            Op op = op0;
            if (op0.kind == OP_ADCT) {
                op.u.tab.row = op0.u.tab.row + (uint64_t)(done + b);
            } else {
                for (int d = 0; d < 3; ++d) op.k[d] = op0.k[d] + (double)(done + b) * op0.u.adc.mu[d];
                op.txy = op0.txy + (double)(done + b) * op0.u.adc.tau;
            }
            op.n = (uint32_t)(e - b);
            op.aux = (uint32_t)(sample - cur.sample_begin);
            ops.push_back(op);
            sample += e - b;
        }
    };
    for (const Op& op0 : p->ops) {
        if (op0.kind != OP_ADC && op0.kind != OP_ADCT) { ops.push_back(op0); continue; }
        const int64_t n = op0.n;
        const int64_t used = sample - cur.sample_begin;
        // a readout that fits a slice of its own starts one rather than
        // being cut at the slice boundary
        if (n <= max_samples && used + n > max_samples && used > 0) close_slice();
        int64_t done = 0;
        while (done < n) {
            int64_t room = max_samples - (sample - cur.sample_begin);
            if (room <= 0) { close_slice(); room = max_samples; }
            const int64_t take = std::min<int64_t>(room, n - done);
            emit(op0, done, take);
            done += take;
        }
    }
    cur.op_end = (int64_t)ops.size();
    cur.n_samples = sample - cur.sample_begin;
    if (cur.op_end > cur.op_begin || p->slices.empty()) p->slices.push_back(cur);
    p->ops = std::move(ops);
}

// Filling a slot steps four vectors through the sub-steps instead of one,
// so a shape pays off from its fifth occurrence in a slice.
constexpr int64_t kMinShapeRepeats = 5;

void assign_shape_slots(Program* p, int max_slots) {
    max_slots = std::max(0, std::min(max_slots, kShapeSlots));
    // shapes that recur often enough in the program, most frequent first
    std::map<int32_t, int64_t> count;
    std::vector<int32_t> order;
    for (const Op& op : p->ops) {
        if (op.kind != OP_SHAPE) continue;
        if (count[op.u.shape.shape_id]++ == 0) order.push_back(op.u.shape.shape_id);
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return count[a] > count[b]; });
    std::map<int32_t, int32_t> slot_of;
    for (int32_t id : order)
        if (count[id] >= kMinShapeRepeats && (int)slot_of.size() < max_slots) {
            const int32_t slot = (int32_t)slot_of.size();
            slot_of[id] = slot;
        }
    // fill or apply, slice by slice; a slot filled in an earlier slice is
    // read back from the slice state instead of filled again
    uint32_t in_state = 0;                       // slots filled in earlier slices
    std::vector<uint32_t> filled(p->slices.size(), 0);
    for (size_t k = 0; k < p->slices.size(); ++k) {
        Slice& sl = p->slices[k];
        uint32_t here = 0, loaded = 0;
        int32_t top = -1;
        for (int64_t i = sl.op_begin; i < sl.op_end; ++i) {
            Op& op = p->ops[i];
            if (op.kind != OP_SHAPE) continue;
            auto& sh = op.u.shape;
            auto it = slot_of.find(sh.shape_id);
            if (it == slot_of.end()) { sh.slot = -1; sh.mode = SHAPE_DIRECT; continue; }
            sh.slot = it->second;
            top = std::max(top, sh.slot);
            const uint32_t bit = 1u << sh.slot;
            if (here & bit) {
                sh.mode = SHAPE_APPLY;
            } else if (in_state & bit) {
                sh.mode = SHAPE_APPLY;
                loaded |= bit;
                here |= bit;
            } else {
                sh.mode = SHAPE_FILL;
                here |= bit;
                filled[k] |= bit;
            }
        }
        sl.n_cache_slots = top + 1;
        sl.cache_load = loaded;
        sl.cache_save = 0;
        in_state |= here;
    }
    // a slot filled in slice k is saved at its end when a later slice loads it
    uint32_t later_loads = 0;
    p->n_state_slots = 0;
    for (size_t k = p->slices.size(); k-- > 0;) {
        Slice& sl = p->slices[k];
        sl.cache_save = filled[k] & later_loads;
        later_loads |= sl.cache_load;
        for (int32_t s = 0; s < kShapeSlots; ++s)
            if ((sl.cache_save | sl.cache_load) & (1u << s)) p->n_state_slots = std::max(p->n_state_slots, s + 1);
    }
}

void narrow_rotations(std::vector<Op>* ops) {
    for (Op& op : *ops) {
        if (op.kind != OP_RF) continue;
        float r[9];
        for (int i = 0; i < 9; ++i) r[i] = (float)op.u.r64[i];
        std::memset(&op.u, 0, sizeof(op.u));
        std::memcpy(op.u.r32, r, sizeof(r));
    }
}

void mark_matrix_readouts(Program* p) {
    std::vector<Op>* ops = &p->ops;
    auto same_step = [](const Op& a, const Op& b) {
        return a.u.adc.tau == b.u.adc.tau && a.u.adc.mu[0] == b.u.adc.mu[0] && a.u.adc.mu[1] == b.u.adc.mu[1] &&
               a.u.adc.mu[2] == b.u.adc.mu[2];
    };
    std::vector<size_t> adc;
    for (size_t i = 0; i < ops->size(); ++i)
        if ((*ops)[i].kind == OP_ADC) adc.push_back(i);
    for (size_t a = 0; a < adc.size(); ++a) {
        Op& op = (*ops)[adc[a]];
        op.flags &= ~OPF_MATRIX;
        if (op.n < (uint32_t)kMatrixMinSamples) continue;
        const bool prev = a > 0 && same_step((*ops)[adc[a - 1]], op);
        const bool next = a + 1 < adc.size() && same_step((*ops)[adc[a + 1]], op);
        if (prev || next) op.flags |= OPF_MATRIX;
    }
    p->any_matrix = false;
    for (size_t a : adc) p->any_matrix = p->any_matrix || ((*ops)[a].flags & OPF_MATRIX);
    p->matrix_only = true;
    const Op* first = nullptr;
    for (const Op& op : *ops) {
        if (op.kind == OP_ADCT || (op.kind == OP_ADC && !(op.flags & OPF_MATRIX))) p->matrix_only = false;
        if (op.kind != OP_ADC) continue;
        if (!first) first = &op;
        else if (!same_step(*first, op)) p->matrix_only = false;
    }
    if (p->matrix_only && first) {
        for (int d = 0; d < 3; ++d) p->matrix_mu[d] = first->u.adc.mu[d];
        p->matrix_tau = first->u.adc.tau;
    }
}

}  // namespace ps
