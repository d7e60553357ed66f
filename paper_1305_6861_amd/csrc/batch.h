// Batched / served execution internals (batch.cpp, server.cpp).
#pragma once
#include <hip/hip_runtime_api.h>

#include <vector>

#include "../../include/parspin.h"
#include "compile.h"
#include "ps_kernels.h"
#include "ps_runtime.h"

namespace ps {

// One request compiled for its own tiling and slicing.
struct ReqPlan {
    ps_object obj{};
    double* signal = nullptr;
    Program prog;
    int S = 1;
    int32_t replica_mode = REPLICAS_RULE;
    ReplicaBound max_replicas;         // readout replicas one tile can use
    int64_t n_blocks = 0, n_rows = 0, row_stride = 0, n_groups = 0;
    size_t bytes_partial = 0, bytes_state = 0, bytes_mid = 0, bytes_ops = 0, bytes_rows = 0, bytes_traj = 0;
    // device placement (bind)
    void* d_partial = nullptr;
    void* d_state = nullptr;
    double* d_mid = nullptr;
    Op* d_ops = nullptr;
    double* d_rows = nullptr;
    double* d_traj = nullptr;

    size_t device_bytes() const;       // library buffers of this request
    size_t table_bytes() const;        // op, rotation and trajectory tables (uploaded)
    size_t footprint() const;          // + object arrays + output (admission)
    void bind(unsigned char* base);    // place the buffers at base (256-aligned)
    void bind_tables(unsigned char* t);   // the tables alone at t (256-aligned)
    void bind_work(unsigned char* w);     // partial rows, slice state, finalize scratch at w
    StepArgs args_for_slice(size_t k, int n_replicas = 1) const;
};

// Validate, compile and slice one request (max_slice_steps > 0 additionally
// bounds the intervals per spin in one slice).
ps_status plan_request(const Ctx* ctx, const ps_object* obj, const ps_sequence* seq, int64_t n_samples,
                       double* signal, int64_t max_slice_steps, ReqPlan* p);

// Stream-ordered upload of the requests' op and rotation tables.
ps_status upload_tables(std::vector<ReqPlan*>& plans, HostBuf& staging, size_t staging_off, hipStream_t stream);
// The same for requests whose tables were bound back to back (bind_tables)
// from device address dev: one host image, one copy.
ps_status upload_tables_contiguous(std::vector<ReqPlan*>& plans, void* dev, HostBuf& staging, hipStream_t stream);

// Host image of one round's launch records, laid out for a single upload:
// per spins-per-lane class its request records and queue counter (zero),
// then the round's finalize records.
struct RoundImage {
    struct Class {                      // one kernel: spins per lane and variant
        int S;
        int variant;                    // step-kernel variant of its requests (step_variant)
        size_t items_off;               // offset of its BatchItem array in the image
        size_t counter_off;             // offset of its queue counter
        int32_t n_req;
        int64_t total;
        size_t dyn_lds;                 // largest dynamic LDS of its requests
    };
    std::vector<Class> classes;
    size_t fin_off = 0;
    int32_t n_fin = 0;
    int64_t tiles1 = 0, tiles2 = 0;
};
// Records of slices first[i] .. first[i] + count[i] - 1 of every plan, one
// slice per round, all rounds in one host image (no device work).
ps_status build_rounds(const Ctx* ctx, std::vector<ReqPlan*>& plans, const std::vector<size_t>& first,
                       const std::vector<size_t>& count, std::vector<unsigned char>* img,
                       std::vector<RoundImage>* rounds);
// The launches of one round whose image sits at device address dev: one
// persistent step kernel per spins-per-lane class, then the batched
// finalize passes, appended to *nodes.
ps_status round_nodes(const Ctx* ctx, const RoundImage& round, unsigned char* dev, std::vector<KernelNode>* nodes);
// build_rounds, one upload of the image through arena/staging, and every
// round's launches, stream-ordered.
ps_status run_rounds(Ctx* ctx, std::vector<ReqPlan*>& plans, const std::vector<size_t>& first,
                     const std::vector<size_t>& count, hipStream_t stream, DevBuf& arena, HostBuf& staging);

}  // namespace ps
