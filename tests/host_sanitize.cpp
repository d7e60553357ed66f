// The library's host code under AddressSanitizer and UndefinedBehavior-
// Sanitizer: the sequence compiler (compile_sequence, plan_slices,
// assign_shape_slots, narrow_rotations) on seeded random sequences, valid
// and invalid, with the invariants its output must keep, and the K-t
// spin-spacing calculator (ps_kt_extent) on random lattice sequences.
// Built with g++ by tests/test_host_sanitizers.py; no device is involved.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <string>
#include <vector>

#include "../include/parspin.h"
#include "../paper_1305_6861_amd/csrc/compile.h"

// The library's error helpers live in its device-side runtime source; the
// host code under test only needs these two.
namespace ps {
static std::string g_err;
ps_status fail(ps_status st, const std::string& msg) { g_err = msg; return st; }
void clear_error() { g_err.clear(); }
}  // namespace ps

static int g_bad = 0;
#define CHECK(c, what)                                                       \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "case %d: %s (%s:%d)\n", case_no, what, __FILE__, __LINE__); \
            ++g_bad;                                                         \
        }                                                                    \
    } while (0)

struct RandomSeq {
    std::vector<ps_event> ev;
    std::vector<ps_rf_shape> sh;
    std::vector<std::vector<double>> alpha, phase, tk, tt;
    std::vector<ps_trajectory> tr;
    ps_sequence seq{};
};

static void make_sequence(std::mt19937_64& rng, RandomSeq& r, bool corrupt) {
    std::uniform_real_distribution<double> u(0.0, 1.0);
    auto ui = [&](int lo, int hi) { return lo + (int)(rng() % (uint64_t)(hi - lo + 1)); };
    const int n_shapes = ui(0, 2), n_traj = ui(0, 2);
    for (int s = 0; s < n_shapes; ++s) {
        const int n = ui(1, 40);
        r.alpha.emplace_back(n);
        r.phase.emplace_back(n);
        for (int i = 0; i < n; ++i) { r.alpha.back()[i] = u(rng) - 0.5; r.phase.back()[i] = 6.0 * u(rng); }
    }
    for (int s = 0; s < n_shapes; ++s) {
        ps_rf_shape x{};
        x.n_sub = (int32_t)r.alpha[s].size();
        x.tau = 1e-5 * u(rng);
        for (int d = 0; d < 3; ++d) x.m_sub[d] = 10.0 * (u(rng) - 0.5);
        x.alpha = r.alpha[s].data();
        x.phase = r.phase[s].data();
        r.sh.push_back(x);
    }
    for (int j = 0; j < n_traj; ++j) {
        const int n = ui(1, 300);
        r.tk.emplace_back(3 * n);
        r.tt.emplace_back(n);
        double t = 0.0;
        for (int q = 0; q < n; ++q) {
            t += 1e-6 * u(rng);
            r.tt.back()[q] = t;
            for (int d = 0; d < 3; ++d) r.tk.back()[3 * q + d] = 100.0 * (u(rng) - 0.5);
        }
    }
    for (int j = 0; j < n_traj; ++j) r.tr.push_back(ps_trajectory{(int64_t)r.tt[j].size(), r.tk[j].data(), r.tt[j].data()});
    const int n_events = ui(0, 120);
    for (int i = 0; i < n_events; ++i) {
        ps_event e{};
        e.dt = 1e-3 * u(rng);
        for (int d = 0; d < 3; ++d) e.m[d] = 50.0 * (u(rng) - 0.5);
        e.rf_alpha = u(rng) < 0.4 ? 3.0 * (u(rng) - 0.5) : 0.0;
        e.rf_phase = 6.0 * u(rng);
        e.rf_shape = (n_shapes > 0 && u(rng) < 0.3) ? ui(0, n_shapes - 1) : -1;
        e.n_adc = u(rng) < 0.4 ? (uint32_t)ui(1, 3000) : 0u;
        e.flags = (u(rng) < 0.2 ? PS_EV_SPOIL : 0u) | (u(rng) < 0.1 ? PS_EV_SNAPSHOT : 0u);
        if (n_traj > 0 && e.n_adc > 0 && u(rng) < 0.3) {
            e.flags |= PS_EV_TRAJECTORY;
            e.trajectory = (uint32_t)ui(0, n_traj - 1);
            e.n_adc = (uint32_t)r.tt[e.trajectory].size();
            e.dt = r.tt[e.trajectory].back() + 1e-6;
        }
        r.ev.push_back(e);
    }
    if (corrupt && !r.ev.empty()) {
        ps_event& e = r.ev[rng() % r.ev.size()];
        switch (ui(0, 5)) {
            case 0: e.dt = -1.0; break;
            case 1: e.dt = std::numeric_limits<double>::quiet_NaN(); break;
            case 2: e.m[1] = std::numeric_limits<double>::infinity(); break;
            case 3: e.rf_shape = n_shapes + 3; break;
            case 4: e.flags |= 64u; break;
            default: e.flags |= PS_EV_TRAJECTORY; e.trajectory = (uint32_t)(n_traj + 1); break;
        }
    }
    r.seq.n_events = (int64_t)r.ev.size();
    r.seq.events = r.ev.data();
    r.seq.n_shapes = n_shapes;
    r.seq.shapes = r.sh.data();
    r.seq.n_trajectories = n_traj;
    r.seq.trajectories = r.tr.data();
}

static void check_program(int case_no, const ps::Program& p, int64_t max_samples) {
    using namespace ps;
    CHECK(!p.slices.empty(), "no slice");
    int64_t samples = 0, expect_begin = 0;
    for (size_t k = 0; k < p.slices.size(); ++k) {
        const Slice& sl = p.slices[k];
        CHECK(sl.op_begin == expect_begin, "slices not contiguous");
        CHECK(sl.op_end >= sl.op_begin && sl.op_end <= (int64_t)p.ops.size(), "slice ops out of range");
        CHECK(sl.sample_begin == samples, "slice sample offsets");
        CHECK(sl.n_samples <= std::max<int64_t>(max_samples, 1), "slice longer than the bound");
        CHECK(sl.n_cache_slots >= 0 && sl.n_cache_slots <= kShapeSlots, "cache slots");
        int64_t here = 0;
        for (int64_t i = sl.op_begin; i < sl.op_end; ++i) {
            const Op& op = p.ops[i];
            if (op.kind == OP_ADC || op.kind == OP_ADCT) {
                CHECK(op.aux == (uint32_t)here, "ADC offset inside its slice");
                CHECK(op.kind != OP_ADC || op.n <= (uint32_t)kAdcRun, "readout run longer than kAdcRun");
                if (op.kind == OP_ADCT) CHECK(4 * (op.u.tab.row + op.n) <= p.traj.size(), "trajectory rows");
                here += op.n;
            }
            if (op.kind == OP_SHAPE) {
                CHECK(9ull * (op.aux + op.n) <= p.rows.size(), "shape rows");
                CHECK(op.u.shape.slot < sl.n_cache_slots, "shape slot within the slice's slots");
            }
        }
        CHECK(here == sl.n_samples, "slice sample count");
        samples += sl.n_samples;
        expect_begin = sl.op_end;
    }
    CHECK(expect_begin == (int64_t)p.ops.size(), "ops not covered");
    CHECK(samples == p.n_samples, "sample total");
}

int main(int argc, char** argv) {
    const int n_cases = argc > 1 ? std::atoi(argv[1]) : 3000;
    std::mt19937_64 rng(20261203);
    int compiled = 0, refused = 0;
    for (int case_no = 0; case_no < n_cases; ++case_no) {
        RandomSeq r;
        const bool corrupt = case_no % 5 == 4;
        make_sequence(rng, r, corrupt);
        ps::Program p;
        std::string err;
        const bool snaps = (case_no & 1) != 0;
        const ps_status st = ps::compile_sequence(&r.seq, &p, &err, snaps);
        if (st != PS_OK) {
            ++refused;
            CHECK(!err.empty(), "refusal without a message");
            continue;
        }
        ++compiled;
        const int64_t max_samples = 1 + (int64_t)(rng() % 5000);
        ps::plan_slices(&p, max_samples);
        ps::assign_shape_slots(&p, (int)(rng() % 3));
        check_program(case_no, p, max_samples);
        ps::narrow_rotations(&p.ops);
    }
    // the K-t calculator on lattice sequences: moments are multiples of dk
    int kt_ok = 0;
    for (int case_no = 0; case_no < 300; ++case_no) {
        std::uniform_int_distribution<int> q(-3, 3);
        std::vector<ps_event> ev;
        const int n = 1 + (int)(rng() % 12);
        const double dk[3] = {4.0, (case_no & 1) ? 4.0 : 0.0, 0.0};
        for (int i = 0; i < n; ++i) {
            ps_event e{};
            e.dt = 1e-3;
            e.m[0] = dk[0] * q(rng);
            e.m[1] = dk[1] * q(rng);
            e.rf_alpha = (rng() % 3 == 0) ? 0.5 + 0.1 * (double)(rng() % 20) : 0.0;
            e.rf_phase = 0.3 * (double)(rng() % 10);
            e.rf_shape = -1;
            e.n_adc = (rng() % 4 == 0) ? 2u : 0u;
            if (e.n_adc) { e.m[0] = dk[0] * 2 * q(rng); e.m[1] = dk[1] * 2 * q(rng); }
            ev.push_back(e);
        }
        ps_sequence s{};
        s.n_events = (int64_t)ev.size();
        s.events = ev.data();
        const double extent[3] = {0.25, 0.25, 0.0};
        double km[3], dx[3];
        int64_t n_min = 0, peak = 0;
        const ps_status st = ps_kt_extent(&s, dk, 1.0, (case_no % 7 == 0) ? INFINITY : 0.1,
                                          (case_no % 3 == 0) ? 1.0 / 256 : 0.0, extent, km, dx, &n_min, &peak);
        if (st == PS_OK) {
            ++kt_ok;
            CHECK(n_min >= 1 && peak >= 0, "K-t counts");
            for (int d = 0; d < 3; ++d)
                CHECK(km[d] > 0 ? std::fabs(dx[d] * 2.0 * km[d] - 1.0) < 1e-12 : std::isinf(dx[d]),
                      "dx_max = 1 / (2 k_max)");
        }
    }
    std::printf("host-sanitize: %d sequences compiled, %d refused, %d K-t runs, %d failures\n", compiled, refused,
                kt_ok, g_bad);
    return g_bad == 0 ? 0 : 1;
}
