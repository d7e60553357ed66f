// K-t simulation engine (sections 4.2 - 4.4 and 5.1.2).
//
// For sequences whose gradient moments lie on a lattice dk, the signal of an
// object made of tissues (each with uniform T1, T2 and off-resonance) is
//   s(t) = sum over tissues c, sum over lattice orders q of
//          F_c(q, t) W(q) S_c(q dk),                              (eq. 4.19)
// with F_c the transverse configuration populations of tissue c (eq. 4.7),
// S_c(k) = sum over the tissue's spins of m0 exp(-2 pi j k . x) the
// tissue's spatial-frequency function, and W(q) = prod_d sinc(q_d dk_d D_d)
// the spectrum of a box voxel of size D (1 for point spins).  The paper's
// K-t simulation tracks the populations through the sequence independently
// of the object's geometry and superposes, at each instant of interest, the
// spatial-frequency function sampled at the configurations' positions
// (section 5.1.2).  Here the host tracks the populations per tissue
// (kt.h: eq. 4.14 - 4.17) and lists, per ADC sample, the populated
// configurations; the device evaluates every tissue's spatial-frequency
// function at the distinct lattice points met -- the data-parallel part,
// over the object's spins -- and superposes them per sample.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/parspin.h"
#include "compile.h"
#include "kt.h"
#include "ps_kernels.h"
#include "ps_runtime.h"

namespace ps {
namespace {

// Populations below this (per unit M0) are rounding left by cancelling terms.
constexpr double kKtPopFloor = 1e-14;
constexpr int64_t kMaxEntries = int64_t(1) << 28;
constexpr size_t kMaxConfigs = size_t(1) << 22;

double sinc_pi(double u) {
    if (u == 0.0) return 1.0;
    const double a = M_PI * u;
    return std::sin(a) / a;
}

struct PairKey {
    int32_t tissue;
    int64_t key;
    bool operator==(const PairKey& o) const { return tissue == o.tissue && key == o.key; }
};
struct PairKeyHash {
    size_t operator()(const PairKey& p) const { return std::hash<int64_t>()(p.key * 1315423911ll + p.tissue); }
};

struct RawEntry {
    int64_t sample;
    int64_t pair;
    double re, im;
};

}  // namespace
}  // namespace ps

using namespace ps;

extern "C" ps_status ps_kt_simulate(ps_ctx* handle, const ps_kt_object* obj, const ps_sequence* seq,
                                    const double dk_in[3], double* signal, int64_t n_samples, void* stream_v) {
    clear_error();
    if (!handle || !obj || !seq || !dk_in) return fail(PS_E_INVALID_ARG, "ctx, obj, seq or dk is NULL");
    Ctx* ctx = reinterpret_cast<Ctx*>(handle);
    if (ctx->scheduler_test) return fail(PS_E_INVALID_ARG, "a scheduler-test context runs no kernels");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->cfg.device);
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_v);

    // ---- validation
    if (obj->n_tissues < 1 || obj->n_tissues > (1 << 20)) return fail(PS_E_INVALID_ARG, "n_tissues must be 1 .. 2^20");
    if (obj->reserved != 0) return fail(PS_E_INVALID_ARG, "reserved field must be 0");
    if (!obj->t1 || !obj->t2 || !obj->dw || !obj->tissue_begin)
        return fail(PS_E_INVALID_ARG, "tissue arrays must not be NULL");
    if (obj->n_spins < 0) return fail(PS_E_INVALID_ARG, "n_spins < 0");
    if (obj->n_spins > 0 && (!obj->x || !obj->y || !obj->z || !obj->m0))
        return fail(PS_E_INVALID_ARG, "spin array pointer is NULL");
    if (obj->tissue_begin[0] != 0 || obj->tissue_begin[obj->n_tissues] != obj->n_spins)
        return fail(PS_E_INVALID_ARG, "tissue_begin must run from 0 to n_spins");
    for (int32_t c = 0; c < obj->n_tissues; ++c) {
        if (obj->tissue_begin[c + 1] < obj->tissue_begin[c])
            return fail(PS_E_INVALID_ARG, "tissue_begin must not decrease");
        if (!(obj->t1[c] > 0) || !(obj->t2[c] > 0))
            return fail(PS_E_INVALID_ARG, "tissue " + std::to_string(c) + ": t1 and t2 must be > 0 (+inf allowed)");
        if (!std::isfinite(obj->dw[c])) return fail(PS_E_INVALID_ARG, "tissue " + std::to_string(c) + ": dw not finite");
    }
    double dk[3], vox[3];
    for (int d = 0; d < 3; ++d) {
        if (!(dk_in[d] >= 0) || !std::isfinite(dk_in[d])) return fail(PS_E_INVALID_ARG, "dk must be finite and >= 0");
        if (!(obj->voxel[d] >= 0) || !std::isfinite(obj->voxel[d]))
            return fail(PS_E_INVALID_ARG, "voxel size must be finite and >= 0");
        dk[d] = dk_in[d];
        vox[d] = obj->voxel[d];
    }
    Program prog;
    {
        std::string err;
        ps_status st = compile_sequence(seq, &prog, &err);
        if (st != PS_OK) return fail(st, err);
    }
    if (n_samples != prog.n_samples)
        return fail(PS_E_INVALID_ARG, "n_samples (" + std::to_string(n_samples) + ") differs from the sequence's " +
                                          std::to_string(prog.n_samples));
    if (n_samples > 0 && !signal) return fail(PS_E_INVALID_ARG, "signal is NULL");
    for (int64_t e = 0; e < seq->n_events; ++e)
        if (seq->events[e].flags & PS_EV_TRAJECTORY)
            return fail(PS_E_INVALID_ARG, "event " + std::to_string(e) +
                                              ": trajectory readouts are not supported by the K-t engine");
    if (n_samples == 0) return PS_OK;

    // ---- populations per tissue, and the configurations populated at every sample
    std::unordered_map<PairKey, int64_t, PairKeyHash> pair_of;
    std::vector<int32_t> pair_tissue;
    std::vector<int64_t> pair_key;
    std::vector<RawEntry> raw;
    {   // at least one populated order per tissue and sample in most sequences
        int32_t with_spins = 0;
        for (int32_t c = 0; c < obj->n_tissues; ++c) with_spins += obj->tissue_begin[c + 1] > obj->tissue_begin[c];
        const size_t guess = (size_t)std::min<int64_t>(n_samples * (int64_t)with_spins, int64_t(1) << 24);
        pair_of.reserve(guess);
        pair_tissue.reserve(guess);
        pair_key.reserve(guess);
        raw.reserve(guess);
    }
    for (int32_t c = 0; c < obj->n_tissues; ++c) {
        if (obj->tissue_begin[c + 1] == obj->tissue_begin[c]) continue;   // no spins: no signal
        const KtTissue tis{1.0 / obj->t1[c], 1.0 / obj->t2[c], obj->dw[c]};
        KtPopulations pop;
        int64_t sample = 0;
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
                    pop.interval(sh.tau, q, tis);
                }
            }
            pop.pulse(ev.rf_alpha, ev.rf_phase);
            const int64_t n = (int64_t)ev.n_adc, K = n > 0 ? n : 1;
            const double mu[3] = {ev.m[0] / (double)K, ev.m[1] / (double)K, ev.m[2] / (double)K};
            int64_t q[3];
            if (!kt_lattice(mu, dk, q))
                return fail(PS_E_INVALID_ARG, "event " + std::to_string(e) +
                                                  ": (per-sample) moment is not a multiple of dk");
            for (int64_t s = 0; s < K; ++s) {
                pop.interval(ev.dt / (double)K, q, tis);
                if (pop.n_transverse() > kMaxConfigs || pop.Z.size() > kMaxConfigs)
                    return fail(PS_E_TOO_LARGE, "tissue " + std::to_string(c) + ": more than 2^22 configurations");
                if (n == 0) continue;
                pop.each_F([&](int64_t order, cplx f) {
                    if (std::abs(f) <= kKtPopFloor) return;
                    const PairKey pk{c, order};
                    auto it = pair_of.find(pk);
                    int64_t u;
                    if (it == pair_of.end()) {
                        u = (int64_t)pair_tissue.size();
                        pair_of.emplace(pk, u);
                        pair_tissue.push_back(c);
                        pair_key.push_back(order);
                    } else {
                        u = it->second;
                    }
                    // voxel spectrum at the configuration's position
                    double w = 1.0;
                    for (int d = 0; d < 3; ++d) w *= sinc_pi((double)kt_axis(order, d) * dk[d] * vox[d]);
                    raw.push_back(RawEntry{sample, u, w * f.real(), w * f.imag()});
                });
                if ((int64_t)raw.size() > kMaxEntries)
                    return fail(PS_E_TOO_LARGE, "more than 2^28 (sample, configuration) entries");
                ++sample;
            }
            if (ev.flags & PS_EV_SPOIL) pop.spoil();
        }
    }

    // ---- tables: entries by sample, pairs by tissue in blocks, work items
    std::vector<int64_t> offsets((size_t)n_samples + 1, 0);
    for (const RawEntry& r : raw) ++offsets[(size_t)r.sample + 1];
    for (int64_t n = 0; n < n_samples; ++n) offsets[n + 1] += offsets[n];
    std::vector<KtEntry> entries(raw.size());
    {
        std::vector<int64_t> fill(offsets.begin(), offsets.end() - 1);
        for (const RawEntry& r : raw) {          // stable: tissues in order within a sample
            KtEntry& q = entries[(size_t)fill[(size_t)r.sample]++];
            q.a_re = r.re;
            q.a_im = r.im;
            q.pair = r.pair;
            q.pad = 0;
        }
    }
    const int64_t n_pairs_raw = (int64_t)pair_tissue.size();
    // pairs reordered tissue by tissue (stable), so that every block of
    // kKtPairs holds one tissue's pairs
    std::vector<int64_t> order((size_t)n_pairs_raw), rank((size_t)n_pairs_raw);
    for (int64_t u = 0; u < n_pairs_raw; ++u) order[u] = u;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return pair_tissue[a] < pair_tissue[b]; });
    for (int64_t i = 0; i < n_pairs_raw; ++i) rank[order[i]] = i;
    for (KtEntry& q : entries) q.pair = rank[q.pair];
    std::vector<double> pair_k((size_t)n_pairs_raw * 3);
    std::vector<KtPairSum> pair_sums((size_t)n_pairs_raw);
    std::vector<KtItem> items;
    for (int64_t i = 0; i < n_pairs_raw;) {
        const int32_t c = pair_tissue[order[i]];
        int64_t j = i;
        while (j < n_pairs_raw && pair_tissue[order[j]] == c) ++j;
        const int64_t s0 = obj->tissue_begin[c], ns = obj->tissue_begin[c + 1] - s0;
        const int64_t n_tiles = (ns + kKtTile - 1) / kKtTile;
        for (int64_t b = i; b < j; b += kKtPairs) {
            const int32_t np = (int32_t)std::min<int64_t>(kKtPairs, j - b);
            const int64_t item0 = (int64_t)items.size();
            for (int64_t t = 0; t < n_tiles; ++t)
                items.push_back(KtItem{s0 + t * kKtTile, b, (int32_t)std::min<int64_t>(kKtTile, ns - t * kKtTile), np});
            for (int32_t p = 0; p < np; ++p) {
                pair_sums[b + p] = KtPairSum{item0, (int32_t)n_tiles, p};
                const int64_t key = pair_key[order[b + p]];
                for (int d = 0; d < 3; ++d) pair_k[3 * (b + p) + d] = (double)kt_axis(key, d) * dk[d];
            }
        }
        i = j;
    }
    const int64_t n_items = (int64_t)items.size();
    if (n_items > 0x7fffffffll) return fail(PS_E_TOO_LARGE, "too many spectrum work items");

    // ---- device buffers (a buffer set of the context) and launches
    const size_t real_bytes = ctx->cfg.precision == 64 ? 8 : 4;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_items = up(items.size() * sizeof(KtItem)), b_pk = up(pair_k.size() * sizeof(double));
    const size_t b_ps = up(pair_sums.size() * sizeof(KtPairSum)), b_en = up(entries.size() * sizeof(KtEntry));
    const size_t b_off = up(offsets.size() * sizeof(int64_t));
    const size_t tables = b_items + b_pk + b_ps + b_en + b_off;
    BufSet* set = nullptr;
    ps_status st;
    if ((st = acquire_set(ctx, &set)) != PS_OK) return st;
    if ((st = set->ops.reserve(tables)) != PS_OK) return st;
    if ((st = set->partial.reserve(std::max<size_t>(1, (size_t)n_items * 64 * real_bytes))) != PS_OK) return st;
    if ((st = set->fin_scratch.reserve(std::max<size_t>(1, (size_t)n_pairs_raw * 2 * sizeof(double)))) != PS_OK)
        return st;
    if ((st = set->staging.reserve(tables)) != PS_OK) return st;
    unsigned char* h = reinterpret_cast<unsigned char*>(set->staging.ptr);
    std::memset(h, 0, tables);
    size_t off = 0;
    auto place = [&](const void* src, size_t bytes, size_t slot) {
        if (bytes) std::memcpy(h + off, src, bytes);
        const size_t at = off;
        off += slot;
        return at;
    };
    const size_t o_items = place(items.data(), items.size() * sizeof(KtItem), b_items);
    const size_t o_pk = place(pair_k.data(), pair_k.size() * sizeof(double), b_pk);
    const size_t o_ps = place(pair_sums.data(), pair_sums.size() * sizeof(KtPairSum), b_ps);
    const size_t o_en = place(entries.data(), entries.size() * sizeof(KtEntry), b_en);
    const size_t o_off = place(offsets.data(), offsets.size() * sizeof(int64_t), b_off);
    unsigned char* d = reinterpret_cast<unsigned char*>(set->ops.ptr);
    hipError_t e = hipMemcpyAsync(d, h, tables, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = launch_kt(reinterpret_cast<const KtItem*>(d + o_items), n_items, reinterpret_cast<const double*>(d + o_pk),
                      reinterpret_cast<const KtPairSum*>(d + o_ps), n_pairs_raw,
                      reinterpret_cast<const KtEntry*>(d + o_en), reinterpret_cast<const int64_t*>(d + o_off),
                      n_samples, obj->x, obj->y, obj->z, obj->m0, set->partial.ptr,
                      reinterpret_cast<double*>(set->fin_scratch.ptr), signal, ctx->cfg.precision, stream);
    // the set's staging may be in a copy on `stream` even after a failure
    const ps_status rel = release_set_after(set, stream);
    if (e != hipSuccess) return hip_fail(e, "K-t launch");
    return rel;
}
