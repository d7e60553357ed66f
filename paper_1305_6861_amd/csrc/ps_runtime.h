// Host runtime internals shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/parspin.h"
#include "compile.h"

namespace ps {

ps_status fail(ps_status st, const std::string& msg);
ps_status hip_fail(hipError_t e, const char* what);
void clear_error();

class DeviceGuard {
public:
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
private:
    int prev_ = -1, dev_ = 0;
};

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    ps_status reserve(size_t n);   // grows, never shrinks; contents not kept
    void release();
};

struct HostBuf {                   // pinned
    void* ptr = nullptr;
    size_t bytes = 0;
    ps_status reserve(size_t n);
    void release();
};

struct Server;                     // served / batched mode (server.cpp)

// Device tables and work buffers of one stream-ordered call (ps_simulate*,
// ps_simulate_batch), with the pinned staging its tables are uploaded from.
// A context rotates through kBufSets of them: a call takes a set whose last
// call has completed, so two calls in flight (on one stream or on two) never
// wait on the host; only a third call waits for the oldest set.
struct BufSet {
    DevBuf ops, rows, traj, partial, state, fin_scratch;
    DevBuf batch_tables, batch_records;   // ps_simulate_batch
    HostBuf staging, staging2;
    hipEvent_t done = nullptr;     // completion of the last call that used the set
    bool pending = false;
    void release();
};
constexpr int kBufSets = 2;

// How a request is tiled: spins per lane (S) and how its readouts are split
// over workgroup replicas when its tiles leave compute units idle.
enum ReplicaMode : int32_t {
    REPLICAS_NONE = 0,    // one workgroup per tile
    REPLICAS_RULE = 1,    // replicas_for_load's rule
    REPLICAS_DOUBLE = 2,  // twice the rule's count (within the tile's bound)
};
struct Tiling {
    int S = 1;
    int32_t replicas = REPLICAS_RULE;
    bool tuned = false;   // taken from the autotuner's table
};

// Class of requests the autotuner keeps one tiling for: precision, object
// size, readout length, shaped pulses or not, receive coils (tune.cpp).
struct TuneKey {
    int32_t precision = 32;
    int32_t spins_log2 = 0;     // floor(log2(n_spins)), -1 for none
    int32_t readout_log2 = -1;  // floor(log2(longest readout in samples)), -1 without readouts
    int32_t shaped = 0;         // any shaped pulse
    int32_t coils_log2 = 0;     // ceil(log2(n_coils)), 0 for one homogeneous coil
    bool operator<(const TuneKey& o) const {
        return std::tie(precision, spins_log2, readout_log2, shaped, coils_log2) <
               std::tie(o.precision, o.spins_log2, o.readout_log2, o.shaped, o.coils_log2);
    }
};
struct TuneEntry {
    Tiling tiling;
    double best_ms = 0.0;       // the winner's time on the probe
    double rule_ms = 0.0;       // the threshold rule's tiling on the same probe
};

struct Ctx {
    ps_config cfg{};
    int n_cu = 256;
    std::mutex mu;                 // serialises calls on one context
    BufSet sets[kBufSets];
    int next_set = 0;              // round-robin position (the oldest set)
    // kernel timing (PS_CFG_KERNEL_TIMING): event pairs around launches
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> step_marks, fin_marks;
    // set once by the first ps_submit (under mu) and read without mu by the
    // served-request calls of other threads
    std::atomic<Server*> server{nullptr};
    std::map<TuneKey, TuneEntry> tuned;   // autotuner table (guarded by mu)
    // allocation-free entry point: the device's static scratch array, and
    // pinned staging for its table uploads (both set up by ps_create)
    void* noalloc_base = nullptr;
    HostBuf noalloc_staging;
    hipEvent_t noalloc_done = nullptr;    // the last upload from the staging has completed
    bool noalloc_pending = false;
    // scheduler-test context (ps_create_scheduler_test): no device; the
    // served loop runs against a stand-in that writes a fixed pattern
    bool scheduler_test = false;
    ps_test_backend test_backend{};
};
// Pinned staging a context sets aside for the allocation-free entry point's
// table uploads (bounds the tables of a request it accepts).
constexpr size_t kNoAllocStagingBytes = size_t(8) << 20;

// The fixed threshold rule: 2 spins per lane once the object fills the
// device twice over at that size, else 1 (or the configured value); 1 for
// an FP32 sequence (when given) whose readouts take the matrix cores.
int threshold_spins_per_lane(const Ctx* ctx, int64_t n_spins, const ps_sequence* seq = nullptr);
// Tuner class of a request (seq must be valid; n_coils 0 = one homogeneous coil).
TuneKey tune_key(const Ctx* ctx, int64_t n_spins, const ps_sequence* seq, int n_coils);
// The tiling a request gets: the configured spins per lane if set, else the
// autotuner's entry for its class, else the threshold rule (with the
// readout-replica rule, or no replicas under PS_CFG_NO_READOUT_SPLIT).
Tiling choose_tiling(const Ctx* ctx, int64_t n_spins, const ps_sequence* seq, int n_coils);
// With PS_CFG_AUTOTUNE: tune the request's class first if the table has no
// entry for it (synchronous; the probe runs after the work already queued
// on `after`).  A no-op otherwise.
ps_status autotune_if_new(Ctx* ctx, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                          hipStream_t after);
hipEvent_t timing_event(Ctx* ctx);  // from the pool (timing-enabled contexts)
ps_status validate_object(const ps_object* obj);
// max_partial_bytes > 0 overrides the context's bound on the partial rows.
ps_status prepare(const Ctx* ctx, const ps_sequence* seq, int64_t n_rows, int S, Program* prog, int n_coils = 0,
                  bool snapshots = false, int64_t max_partial_bytes = 0);
// Propagator cache slots a request tiled with S spins per lane may use.
int shape_cache_slots(const Ctx* ctx, int S, const Program& prog);
// A buffer set for the next call: one whose last call has completed, or
// else the oldest, after waiting for it.
ps_status acquire_set(Ctx* ctx, BufSet** out);
// Mark the set in use until the work enqueued on `stream` so far completes.
ps_status release_set_after(BufSet* set, hipStream_t stream);
ps_status validate_receive(const ps_receive* rx, const ps_object* obj);
// Readout replicas (see the step kernel) a tile of a program can use: at
// most `hard` (one per readout of its busiest slice, at most 64); replicas
// that share a CU with others are worth it only up to `work`, where their
// repeated RF and shaped-pulse stepping reaches the readout work they
// split.  replicas_for_load gives the number to launch for n_tiles tiles.
struct ReplicaBound {
    int hard = 1;
    int work = 1;
    double other_share = 0.0;   // estimated share of a tile's work outside its readouts
};
ReplicaBound replica_bound(const Program& p, int n_out);
int replicas_for_load(const Ctx* ctx, int64_t n_tiles, ReplicaBound bound, int32_t mode = REPLICAS_RULE);
// A single request's launch: tiles 0 .. n_whole - 1 whole, the rest in
// `replicas` readout replicas each (replicas_for_load's count with
// n_whole = 0 when that is above one; else the tiles past the last whole
// round of slots, the workgroups the device holds at once, split over the
// slots that round leaves free, when there are at most four whole rounds).
struct ReplicaSplit {
    int replicas = 1;
    int64_t n_whole = 0;
};
ReplicaSplit replica_split(const Ctx* ctx, int64_t n_tiles, ReplicaBound bound, int32_t mode, int64_t slots);
// Workgroups of the step kernel that runs p at S spins per lane resident on
// the whole device at once.
int64_t device_slots(const Ctx* ctx, int S, const Program& p);

// One request compiled for a context: program, tiling and buffer sizes.
struct Single {
    Program prog;
    int S = 1, n_coils = 0, n_out = 1;
    int32_t replica_mode = REPLICAS_RULE;
    int n_replicas = 1;            // readout replicas per tile from tile n_whole on
    int64_t n_whole = 0;           // tiles that run whole (see ReplicaSplit)
    int64_t n_blocks = 0, n_rows = 0, coil_stride = 0, row_stride = 0;
    bool any_snaps = false;
    ps_object obj{};
    ps_receive rx{};
    double* signal = nullptr;
    int64_t n_samples = 0;
    void* snaps = nullptr;
    size_t partial_bytes = 0, fin_bytes = 0, state_bytes = 0;
    bool empty() const;            // nothing for the step kernel to do
};
// Device tables and work buffers one request's launches use.
struct SingleBuffers {
    const void* ops = nullptr;
    const void* rows = nullptr;
    const void* traj = nullptr;
    void* partial = nullptr;
    void* state = nullptr;
    double* fin_scratch = nullptr;
};
// force: a tiling to use instead of choose_tiling's (NULL: choose).
ps_status plan_single(Ctx* ctx, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                      double* signal, int64_t n_samples, void* snaps, int64_t n_snapshots, const Tiling* force,
                      Single* r, int64_t max_partial_bytes = 0);
// Stream-ordered launches of a planned request (tables already resident in
// b); kernel timing events go to timing_ctx when it is not NULL.
ps_status enqueue_single(const Ctx* ctx, const Single& r, const SingleBuffers& b, hipStream_t stream,
                         Ctx* timing_ctx);
ps_status run_request(Ctx* ctx, const ps_object* obj, const ps_sequence* seq, double* signal,
                      int64_t n_samples, hipStream_t stream, const Tiling* force, const ps_receive* rx,
                      void* snaps = nullptr, int64_t n_snapshots = -1);
void destroy_runtime(Ctx* ctx);    // stops the server if one runs

}  // namespace ps
