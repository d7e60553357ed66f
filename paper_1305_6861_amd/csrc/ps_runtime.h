// Host runtime internals shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime_api.h>

#include <mutex>
#include <string>
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

struct Ctx {
    ps_config cfg{};
    int n_cu = 256;
    std::mutex mu;                 // serialises calls on one context
    BufSet sets[kBufSets];
    int next_set = 0;              // round-robin position (the oldest set)
    // kernel timing (PS_CFG_KERNEL_TIMING): event pairs around launches
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> step_marks, fin_marks;
    Server* server = nullptr;
};

int choose_spins_per_lane(const Ctx* ctx, int64_t n_spins);
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
};
ReplicaBound replica_bound(const Program& p, int n_out);
int replicas_for_load(const Ctx* ctx, int64_t n_tiles, ReplicaBound bound);

// One request compiled for a context: program, tiling and buffer sizes.
struct Single {
    Program prog;
    int S = 1, n_coils = 0, n_out = 1;
    int n_replicas = 1;            // readout replicas per tile
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
ps_status plan_single(Ctx* ctx, const ps_object* obj, const ps_sequence* seq, const ps_receive* rx,
                      double* signal, int64_t n_samples, void* snaps, int64_t n_snapshots, int S_override,
                      Single* r, int64_t max_partial_bytes = 0);
// Stream-ordered launches of a planned request (tables already resident in
// b); kernel timing events go to timing_ctx when it is not NULL.
ps_status enqueue_single(const Ctx* ctx, const Single& r, const SingleBuffers& b, hipStream_t stream,
                         Ctx* timing_ctx);
ps_status run_request(Ctx* ctx, const ps_object* obj, const ps_sequence* seq, double* signal,
                      int64_t n_samples, hipStream_t stream, int S_override, const ps_receive* rx,
                      void* snaps = nullptr, int64_t n_snapshots = -1);
void destroy_runtime(Ctx* ctx);    // stops the server if one runs

}  // namespace ps
