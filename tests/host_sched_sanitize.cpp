// The served loop's host code under ThreadSanitizer (or AddressSanitizer +
// UndefinedBehaviorSanitizer): a scheduler-test context (no device) driven
// from several threads at once -- submissions, polls, waits with and
// without time-outs, cancellations, request records, server counters --
// while its scheduler thread admits, batches, retires and fails requests
// (one injected device error).  Every finished request's stand-in pattern
// is checked.  Built by tests/test_host_sanitizers.py.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../include/parspin.h"

static std::atomic<int> g_bad{0};

struct Req {
    std::vector<ps_event> ev;
    std::vector<float> arr;          // stand-in object arrays (never read)
    std::vector<double> signal;
    int64_t n_spins = 0, n_samples = 0;
    uint64_t ticket = 0;
};

static void make(Req& r, std::mt19937_64& rng) {
    const int n_pe = 1 + (int)(rng() % 40), n_read = 1 + (int)(rng() % 100);
    for (int j = 0; j < n_pe; ++j) {
        ps_event a{}, b{}, c{};
        a.dt = 2e-3; a.m[1] = j; a.rf_alpha = 0.5; a.rf_shape = -1;
        b.dt = 1e-3; b.m[0] = n_read; b.n_adc = (uint32_t)n_read; b.rf_shape = -1;
        c.dt = 5e-3; c.flags = PS_EV_SPOIL; c.rf_shape = -1;
        r.ev.push_back(a); r.ev.push_back(b); r.ev.push_back(c);
    }
    r.n_spins = (rng() % 9 == 0) ? 0 : 1 + (int64_t)(rng() % 5000);
    r.n_samples = (int64_t)n_pe * n_read;
    r.arr.assign(8, 0.f);
    r.signal.assign((size_t)(2 * r.n_samples), NAN);
}

static bool pattern_ok(const Req& r) {
    for (int64_t n = 0; n < r.n_samples; ++n) {
        const double re = r.signal[2 * n], im = r.signal[2 * n + 1];
        if (r.n_spins == 0) {
            if (re != 0.0 || im != 0.0) return false;
        } else if (re != (double)(r.n_spins + n) || !(im >= 0) || (n > 0 && im < r.signal[2 * n - 1])) {
            return false;
        }
    }
    return true;
}

int main() {
    ps_config cfg;
    ps_config_default(&cfg);
    cfg.max_slice_steps = 300;
    ps_test_backend tb{0.0002, 25};
    ps_ctx* ctx = nullptr;
    if (ps_create_scheduler_test(&ctx, &cfg, &tb) != PS_OK) { std::fprintf(stderr, "create\n"); return 2; }
    std::atomic<bool> stop{false};
    std::thread watcher([&] {                // server counters while everything runs
        ps_server_stats_t st;
        while (!stop.load()) {
            if (ps_server_stats(ctx, &st) != PS_OK) ++g_bad;
            std::this_thread::yield();
        }
    });
    std::vector<std::thread> workers;
    std::atomic<int> done{0}, cancelled{0}, failed{0};
    for (int w = 0; w < 4; ++w) {
        workers.emplace_back([&, w] {
            std::mt19937_64 rng(1000 + w);
            std::vector<Req> reqs(30);
            for (Req& r : reqs) {
                make(r, rng);
                ps_object o{r.n_spins, r.arr.data(), r.arr.data(), r.arr.data(), r.arr.data(), r.arr.data(),
                            r.arr.data(), r.arr.data()};
                ps_sequence s{(int64_t)r.ev.size(), r.ev.data(), 0, 0, nullptr, nullptr};
                if (ps_submit(ctx, &o, &s, r.signal.data(), r.n_samples, &r.ticket) != PS_OK) ++g_bad;
                if ((&r - reqs.data()) % 7 == 3) ps_cancel(ctx, r.ticket);   // queued, running or done
            }
            for (size_t i = 0; i < reqs.size(); ++i) {
                Req& r = reqs[i];
                if (i % 11 == 5) ps_cancel(ctx, r.ticket);
                int32_t d = 0;
                ps_poll(ctx, r.ticket, &d);
                ps_request_info_t info;
                ps_request_info(ctx, r.ticket, &info);
                ps_wait(ctx, r.ticket, 0.0);               // a time-out or the result
                const ps_status st = ps_wait(ctx, r.ticket, -1.0);
                double q, k, e;
                if (ps_stats(ctx, r.ticket, &q, &k, &e) != PS_OK || !(e >= 0)) ++g_bad;
                if (st == PS_OK) {
                    ++done;
                    if (!pattern_ok(r)) { std::fprintf(stderr, "pattern of a finished request\n"); ++g_bad; }
                } else if (st == PS_E_CANCELLED) {
                    ++cancelled;
                } else if (st == PS_E_DEVICE) {
                    ++failed;
                } else {
                    ++g_bad;
                }
                ps_release(ctx, r.ticket);
            }
        });
    }
    for (std::thread& t : workers) t.join();
    stop = true;
    watcher.join();
    ps_destroy(ctx);
    std::printf("host-sched-sanitize: %d done, %d cancelled, %d failed by the injected error, %d problems\n",
                done.load(), cancelled.load(), failed.load(), g_bad.load());
    return g_bad.load() == 0 && failed.load() > 0 && done.load() > 0 ? 0 : 1;
}
