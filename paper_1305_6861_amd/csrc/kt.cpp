// Spin spacing for a sequence (section 5.2), from the K-t formalism
// (section 4.2).
//
// When every gradient moment of a sequence is an integer multiple of a
// lattice step dk per axis, a spin's magnetisation is a finite series over
// lattice orders k whose populations do not depend on position (eq. 4.7 -
// 4.11): transverse F(k) and longitudinal Z(k).  Hard pulses mix the
// triplet (F(k), conj F(-k), Z(k)) of each order with the complex form of
// eq. 3.19 (eq. 4.14), relaxation scales them and feeds Z(0) (eq. 4.15 /
// 4.16), a gradient of moment q dk moves every F(k) to k + q (eq. 4.17).
// Tracking them for one reference tissue gives the largest k-space position
// any configuration reaches (eq. 5.1) and so the largest spin spacing that
// keeps the periodic repetitions of the sampled object's spectrum away from
// every configuration (eq. 5.2); optionally, outer configurations whose
// populations are too small to show in a grey-value image are left out
// (eq. 5.4 / 5.5).  Host code; the GPU path does not need it.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/parspin.h"
#include "compile.h"
#include "kt.h"
#include "ps_runtime.h"

namespace ps {

int64_t kt_pack(int64_t a, int64_t b, int64_t c) {
    const int64_t m = (int64_t(1) << kKtBits) - 1;
    return ((a & m) << (2 * kKtBits)) | ((b & m) << kKtBits) | (c & m);
}

int64_t kt_axis(int64_t key, int d) {
    const int64_t m = (int64_t(1) << kKtBits) - 1;
    int64_t v = (key >> (kKtBits * (2 - d))) & m;
    if (v & (int64_t(1) << (kKtBits - 1))) v -= (int64_t(1) << kKtBits);
    return v;
}

int64_t kt_negate(int64_t key) { return kt_pack(-kt_axis(key, 0), -kt_axis(key, 1), -kt_axis(key, 2)); }

KtPopulations::KtPopulations() { Z[kt_pack(0, 0, 0)] = 1.0; }

void KtPopulations::settle() {
    if (shift_[0] == 0 && shift_[1] == 0 && shift_[2] == 0 && scale_ == cplx(1.0, 0.0)) return;
    std::unordered_map<int64_t, cplx> nF;
    nF.reserve(F_.size());
    each_F([&](int64_t k, cplx f) { nF[k] = f; });
    F_.swap(nF);
    shift_[0] = shift_[1] = shift_[2] = 0;
    scale_ = 1.0;
}

void KtPopulations::spoil() {
    F_.clear();
    shift_[0] = shift_[1] = shift_[2] = 0;
    scale_ = 1.0;
}

void KtPopulations::pulse(double alpha, double phi) {
    if (alpha == 0.0) return;
    settle();
    std::unordered_map<int64_t, cplx>& F = F_;
    double r[9];
    rf_matrix(alpha, phi, r);
    // T = C R C^-1 with C mapping (Mx, My, Mz) to (Mx + j My, Mx - j My, Mz);
    // rows 0 and 2 are needed: F'(k) and Z'(k) from (F(k), conj F(-k), Z(k))
    const cplx j(0.0, 1.0);
    const cplx C[3][3] = {{1.0, j, 0.0}, {1.0, -j, 0.0}, {0.0, 0.0, 1.0}};
    const cplx Ci[3][3] = {{0.5, 0.5, 0.0}, {-0.5 * j, 0.5 * j, 0.0}, {0.0, 0.0, 1.0}};
    cplx CR[3][3], T[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            CR[a][b] = 0.0;
            for (int c = 0; c < 3; ++c) CR[a][b] += C[a][c] * r[3 * c + b];
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            T[a][b] = 0.0;
            for (int c = 0; c < 3; ++c) T[a][b] += CR[a][c] * Ci[c][b];
        }
    std::unordered_set<int64_t> keys;
    keys.reserve(2 * F.size() + Z.size());
    for (auto& kv : F) { keys.insert(kv.first); keys.insert(kt_negate(kv.first)); }
    for (auto& kv : Z) keys.insert(kv.first);
    std::unordered_map<int64_t, cplx> nF, nZ;
    nF.reserve(keys.size());
    nZ.reserve(keys.size());
    for (int64_t k : keys) {
        auto fi = F.find(k), mi = F.find(kt_negate(k));
        auto zi = Z.find(k);
        const cplx u = fi != F.end() ? fi->second : 0.0;
        const cplx v = mi != F.end() ? std::conj(mi->second) : 0.0;
        const cplx w = zi != Z.end() ? zi->second : 0.0;
        const cplx fu = T[0][0] * u + T[0][1] * v + T[0][2] * w;
        const cplx zw = T[2][0] * u + T[2][1] * v + T[2][2] * w;
        if (fu != 0.0) nF[k] = fu;
        if (zw != 0.0) nZ[k] = zw;
    }
    F.swap(nF);
    Z.swap(nZ);
    peak = std::max(peak, F_.size());
}

void KtPopulations::interval(double tau, const int64_t q[3], const KtTissue& t) {
    const double e1 = std::exp(-tau * t.r1), e2 = std::exp(-tau * t.r2);
    // transverse decay and the tissue's uniform off-resonance turn, e^(-j dw tau)
    const cplx turn = t.dw != 0.0 ? e2 * cplx(std::cos(t.dw * tau), -std::sin(t.dw * tau)) : cplx(e2, 0.0);
    for (int d = 0; d < 3; ++d) shift_[d] += q[d];
    scale_ *= turn;
    // keep the pending factor well inside the double range
    if (std::abs(scale_) < 1e-150) settle();
    for (auto& kv : Z) kv.second *= e1;
    Z[kt_pack(0, 0, 0)] += 1.0 - e1;
}

bool kt_lattice(const double m[3], const double dk[3], int64_t q[3]) {
    for (int d = 0; d < 3; ++d) {
        if (dk[d] == 0.0) {
            if (std::fabs(m[d]) > 1e-9) return false;
            q[d] = 0;
            continue;
        }
        const double r = m[d] / dk[d];
        const double n = std::nearbyint(r);
        if (std::fabs(r - n) > 1e-6 * std::max(1.0, std::fabs(r)) || std::fabs(n) > (double)kKtLim / 2) return false;
        q[d] = (int64_t)n;
    }
    return true;
}

namespace {
int64_t iabs(int64_t v) { return v < 0 ? -v : v; }
}  // namespace

}  // namespace ps

using namespace ps;

extern "C" ps_status ps_kt_extent(const ps_sequence* seq, const double dk_in[3], double t1, double t2,
                                  double grey_step, const double extent[3], double k_max[3], double dx_max[3],
                                  int64_t* n_spins_min, int64_t* n_configs_peak) {
    clear_error();
    if (!seq || !dk_in || !k_max || !dx_max) return fail(PS_E_INVALID_ARG, "NULL argument");
    if (n_spins_min && !extent) return fail(PS_E_INVALID_ARG, "n_spins_min needs the object extent");
    if (extent)
        for (int d = 0; d < 3; ++d)
            if (!(extent[d] >= 0) || !std::isfinite(extent[d]))
                return fail(PS_E_INVALID_ARG, "extent must be finite and >= 0");
    if (!(t1 > 0) || !(t2 > 0)) return fail(PS_E_INVALID_ARG, "t1 and t2 must be > 0 (+inf allowed)");
    if (!(grey_step >= 0) || !std::isfinite(grey_step)) return fail(PS_E_INVALID_ARG, "grey_step must be >= 0");
    double dk[3];
    for (int d = 0; d < 3; ++d) {
        if (!(dk_in[d] >= 0) || !std::isfinite(dk_in[d])) return fail(PS_E_INVALID_ARG, "dk must be finite and >= 0");
        dk[d] = dk_in[d];
    }
    {   // the sequence is validated by the compiler
        Program p;
        std::string err;
        ps_status st = compile_sequence(seq, &p, &err);
        if (st != PS_OK) return fail(st, err);
    }
    const KtTissue tis{1.0 / t1, 1.0 / t2, 0.0};
    KtPopulations pop;
    int64_t kmax[3] = {0, 0, 0};
    constexpr double kPopTol = 1e-12;      // rounding left by cancelling terms
    constexpr size_t kCap = size_t(1) << 22;

    auto track_order = [&](int64_t k, cplx f) {
        if (std::abs(f) > kPopTol)
            for (int d = 0; d < 3; ++d) kmax[d] = std::max(kmax[d], iabs(kt_axis(k, d)));
    };
    auto track_all = [&]() {
        pop.each_F(track_order);
        for (auto& kv : pop.Z) track_order(kv.first, kv.second);
    };
    auto track_sample = [&]() {
        if (pop.n_transverse() == 0) return;
        std::vector<std::pair<int64_t, cplx>> F;
        F.reserve(pop.n_transverse());
        pop.each_F([&](int64_t k, cplx f) { F.emplace_back(k, f); });
        double ref = 0.0;
        for (auto& kv : F) ref = std::max(ref, std::abs(kv.second));
        const double budget = 0.5 * grey_step * ref;
        std::vector<std::pair<int64_t, double>> v;
        v.reserve(F.size());
        for (int d = 0; d < 3; ++d) {
            v.clear();
            for (auto& kv : F) v.emplace_back(iabs(kt_axis(kv.first, d)), std::abs(kv.second));
            std::sort(v.begin(), v.end(), [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) {
                return a.first != b.first ? a.first > b.first : a.second > b.second;
            });
            double cut = 0.0;
            int64_t K = 0;
            for (auto& e : v) {
                if (cut + e.second > budget) { K = e.first; break; }
                cut += e.second;
            }
            kmax[d] = std::max(kmax[d], K);
        }
    };
    const bool pruned = grey_step > 0;
    auto too_large = [&]() { return pop.n_transverse() > kCap || pop.Z.size() > kCap; };

    for (int64_t e = 0; e < seq->n_events; ++e) {
        const ps_event& ev = seq->events[e];
        if (ev.rf_shape >= 0) {
            const ps_rf_shape& sh = seq->shapes[ev.rf_shape];
            int64_t q[3];
            if (!kt_lattice(sh.m_sub, dk, q))
                return fail(PS_E_INVALID_ARG, "shape " + std::to_string(ev.rf_shape) +
                                                  ": sub-step moment is not a multiple of dk");
            for (int32_t s = 0; s < sh.n_sub; ++s) {
                pop.pulse(sh.alpha[s], sh.phase[s] + ev.rf_phase);
                if (!pruned) track_all();
                pop.interval(sh.tau, q, tis);
                if (!pruned) track_all();
                if (too_large()) return fail(PS_E_TOO_LARGE, "more than 2^22 configurations");
            }
        }
        pop.pulse(ev.rf_alpha, ev.rf_phase);
        if (!pruned) track_all();
        const int64_t n = (int64_t)ev.n_adc, K = n > 0 ? n : 1;
        const double mu[3] = {ev.m[0] / (double)K, ev.m[1] / (double)K, ev.m[2] / (double)K};
        int64_t q[3];
        if (!kt_lattice(mu, dk, q))
            return fail(PS_E_INVALID_ARG, "event " + std::to_string(e) + ": (per-sample) moment is not a multiple of dk");
        for (int64_t s = 0; s < K; ++s) {
            pop.interval(ev.dt / (double)K, q, tis);
            if (!pruned) track_all();
            else if (n > 0) track_sample();
            if (too_large()) return fail(PS_E_TOO_LARGE, "more than 2^22 configurations");
        }
        if (ev.flags & PS_EV_SPOIL) pop.spoil();
    }
    for (int d = 0; d < 3; ++d) {
        k_max[d] = (double)kmax[d] * dk[d];
        dx_max[d] = k_max[d] > 0 ? 0.5 / k_max[d] : INFINITY;
    }
    if (n_spins_min) {
        // eq. 5.2: isochromats no further apart than dx_max on every axis the
        // object spans, so each such axis needs ceil(extent / dx_max) of them
        constexpr int64_t kMaxSpins = int64_t(1) << 62;
        int64_t n = 1;
        for (int d = 0; d < 3; ++d) {
            if (!(extent[d] > 0) || !std::isfinite(dx_max[d])) continue;
            const double c = std::ceil(extent[d] / dx_max[d]);
            if (c >= (double)kMaxSpins || (double)n * c >= (double)kMaxSpins)
                return fail(PS_E_TOO_LARGE, "spin count beyond 2^62");
            n *= (int64_t)c;
        }
        *n_spins_min = n;
    }
    if (n_configs_peak) *n_configs_peak = (int64_t)pop.peak;
    return PS_OK;
}
