// Kernel arguments and launchers (host side of kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <vector>

#include "ps_ops.h"

namespace ps {

struct StepArgs {
    const float *x, *y, *z, *m0, *t1, *t2, *dw;  // device SoA object
    int64_t n_spins;
    const Op* ops;           // device, this time slice's operations
    int32_t n_ops;
    int32_t n_shape_rows;    // shaped-pulse rotation rows (9 doubles each)
    const void* rows;        // device, n_shape_rows * 9 doubles (rotation deltas)
    void* partial;           // device, gridDim.x * rows_per_block rows of row_stride reals
    int64_t row_stride;      // reals per workgroup row (2 per sample of the slice)
    void* state;             // device, (6 + 12 * slots) * n_spins reals, SoA: two buffers of
                             // anchors (Mxy_a re, im, Mz_a), then kShapeCacheReals entries
                             // per kept propagator slot
    int32_t load_state;      // resume from anchor buffer anchor_parity ^ 1 instead of equilibrium
    int32_t save_state;      // write the anchors to buffer anchor_parity at the end
    int32_t anchor_parity;   // slice index & 1: a slice reads the buffer the previous one wrote
                             // and writes the other, so a readout replica that starts after
                             // replica 0 of its tile has finished still reads the slice's start
    int32_t n_cache_slots;   // shaped-pulse propagator slots the slice's ops use
    uint32_t cache_load;     // slots read from the state at the start (bit per slot)
    uint32_t cache_save;     // slots written to the state at the end (bit per slot)
    int32_t n_coils;         // receive coils (0: one homogeneous coil, no weights)
    const float *s_x, *s_y;  // device, n_coils * n_spins transverse sensitivities
    int64_t coil_stride;     // reals between coils' sample blocks inside a row
    void* snaps;             // device, n_snapshots * 3 * n_spins reals (OP_SNAP targets)
    const double* traj;      // device, trajectory rows (K + k_s, txy + t_s), 4 doubles each
    int32_t n_replicas;      // readout replicas per tile (>= 1) from tile n_whole on
    int64_t n_tiles;         // workgroup tiles of the object (set by launch_step)
    int64_t n_whole;         // launch_step: tiles 0 .. n_whole - 1 run whole (one replica);
                             // the batched kernel splits every tile (n_whole = 0)
    double mx_mu[3];         // matrix-only kernel: the per-sample step (mu, tau) that every
    double mx_tau;           // readout of the program shares
};

// One request of a persistent batched launch: its arguments and the number
// of the first of its tiles in the launch's item sequence.
struct alignas(16) BatchItem {
    StepArgs args;
    int64_t item_begin;
    int64_t n_items;
};

// One request of a batched finalize.
struct alignas(16) FinDesc {
    const void* partial;     // n_rows rows of row_stride reals
    int64_t n_rows, row_stride, n_vals;
    int64_t n_groups;        // row groups (pass 2 needed when > 1)
    double* out;             // n_vals doubles
    double* mid;             // n_groups * n_vals doubles when n_groups > 1
    int64_t tile_begin1;     // first pass-1 block (n_groups * finalize_tiles(n_vals) blocks)
    int64_t tile_begin2;     // first pass-2 block (ceil(n_vals/256) blocks if n_groups > 1, else 0)
};

// Spins handled by one workgroup for a given spins-per-lane choice.
int64_t spins_per_block_of(int spins_per_lane);
// Partial-sum rows one workgroup writes (one per wave group).
int64_t rows_per_block_of(int spins_per_lane);

// Step-kernel variants at FP32 and one spin per lane (elsewhere there is
// only the general kernel):
//   STEP_GENERAL      both readout paths; the matrix-core tables are built
//                     when a readout needs them (two waves per SIMD);
//   STEP_MATRIX_ONLY  a program whose readouts are all marked OPF_MATRIX,
//                     none tabulated, and share one per-sample step (given
//                     in StepArgs::mx_mu / mx_tau): built without the vector
//                     and trajectory readouts, it builds the tables once,
//                     before its operations, so they stay in the same
//                     registers throughout (three waves per SIMD);
//   STEP_VECTOR_ONLY  a program with no OPF_MATRIX readout: built without
//                     the matrix-core readout, so its registers allow three
//                     waves per SIMD.
enum StepVariant : int { STEP_GENERAL = 0, STEP_MATRIX_ONLY = 1, STEP_VECTOR_ONLY = 2 };
// The variant that runs a program (Program::matrix_only, ::any_matrix).
inline int step_variant(int precision, int spins_per_lane, bool matrix_only, bool any_matrix) {
    if (precision == 64 || spins_per_lane != 1) return STEP_GENERAL;
    return matrix_only ? STEP_MATRIX_ONLY : any_matrix ? STEP_GENERAL : STEP_VECTOR_ONLY;
}

// Launches a.n_whole + (n_blocks - a.n_whole) * a.n_replicas workgroups:
// the first n_whole tiles whole, every later tile once per readout replica
// (replicas split the slice's readouts), with the kernel variant given
// (step_variant; ignored where only the general kernel exists).
hipError_t launch_step(const StepArgs& a, int precision, int spins_per_lane, int64_t n_blocks,
                       hipStream_t st, int variant = STEP_GENERAL);
// Dynamic LDS of a step workgroup: shaped-pulse rows (not in the
// matrix-only kernel, which reads them through the scalar cache) and
// propagator slots.
size_t step_dyn_lds_bytes(int precision, int spins_per_lane, int32_t n_shape_rows, int32_t n_cache_slots,
                          int variant = STEP_GENERAL);
// Step workgroups resident per CU (occupancy of the kernel the arguments
// select, with dyn_lds bytes of dynamic LDS).
int step_workgroups_per_cu(int precision, int spins_per_lane, int variant, size_t dyn_lds);
// Propagator slots (at most kShapeSlots) that fit a step workgroup's LDS
// budget next to n_shape_rows shaped-pulse rows.
int shape_cache_slots_fitting(int precision, int spins_per_lane, int32_t n_shape_rows, int variant = STEP_GENERAL);
// Finalize pass 1: each thread sums kFinVals consecutive values, so partial
// rows and the coil blocks inside them are padded to a multiple of kFinVals
// values; finalize_tiles(n) workgroups of 256 threads cover n values.
constexpr int64_t kFinVals = 4;
constexpr int64_t finalize_tiles(int64_t n_vals) { return (n_vals + 256 * kFinVals - 1) / (256 * kFinVals); }
constexpr int64_t pad_fin(int64_t n_vals) { return (n_vals + kFinVals - 1) / kFinVals * kFinVals; }
// Doubles of scratch launch_finalize needs for n_rows rows of n_vals values.
int64_t finalize_scratch_doubles(int64_t n_rows, int64_t n_vals);
// row_stride and the partial base must be multiples of kFinVals values.
hipError_t launch_finalize(const void* partial, int precision, int64_t n_rows, int64_t row_stride,
                           int64_t n_vals, double* out, double* scratch, hipStream_t st);
hipError_t launch_fill_zero(double* out, int64_t n, hipStream_t st);
// Persistent launch over total items of the n_req requests in reqs (device);
// counter (device) must hold 0; dyn_lds covers every request's
// step_dyn_lds_bytes.
hipError_t launch_batch_step(const BatchItem* reqs, int32_t n_req, int64_t total, unsigned long long* counter,
                             size_t dyn_lds, int precision, int spins_per_lane, int n_cu, hipStream_t st,
                             int variant = STEP_GENERAL);
hipError_t launch_batch_finalize(const FinDesc* d, int32_t n, int64_t tiles1, int64_t tiles2, int precision,
                                 hipStream_t st);

// A kernel launch described for a HIP graph kernel node or a direct launch:
// the kernel, its grid and the argument values (at most four; argv points
// into this object, so set it up again with params() after a copy).
struct KernelNode {
    const void* func = nullptr;
    dim3 grid{1, 1, 1}, block{256, 1, 1};
    size_t shmem = 0;
    int n_args = 0;
    const void* a0 = nullptr;
    int32_t a1 = 0;
    int64_t a2 = 0;
    void* a3 = nullptr;
    void* argv[4] = {nullptr, nullptr, nullptr, nullptr};
    hipKernelNodeParams params();
    hipError_t launch(hipStream_t st);
};
// The launches launch_batch_step / launch_batch_finalize would make, as
// nodes appended to *out (none when there is nothing to run).
hipError_t batch_step_nodes(const BatchItem* reqs, int32_t n_req, int64_t total, unsigned long long* counter,
                            size_t dyn_lds, int precision, int spins_per_lane, int n_cu, std::vector<KernelNode>* out,
                            int variant = STEP_GENERAL);
hipError_t batch_finalize_nodes(const FinDesc* d, int32_t n, int64_t tiles1, int64_t tiles2, int precision,
                                std::vector<KernelNode>* out);
int64_t row_group_size();

// K-t simulation (kt_engine.cpp): work items of the spectrum kernel, the
// tile-sum description of every (tissue, lattice point) pair, and the
// per-sample entries a_e (population times voxel weight) of eq. 4.19.
constexpr int kKtPairs = 32;               // pairs per work item (64 reduced values)
constexpr int kKtSpl = 4;                  // spins per lane
constexpr int64_t kKtTile = 256 * kKtSpl;  // spins per work item
struct alignas(16) KtItem {
    int64_t spin_begin;      // first spin of the tile
    int64_t pair_begin;      // first pair of the block (pair_k rows)
    int32_t n_spins;         // spins of the tile (<= kKtTile)
    int32_t n_pairs;         // pairs of the block (<= kKtPairs)
};
struct alignas(16) KtPairSum {
    int64_t item0;           // work item of the pair's block and the tissue's first tile
    int32_t n_tiles;         // tiles of the tissue (items item0 .. item0 + n_tiles - 1)
    int32_t slot;            // position of the pair in its block
};
struct alignas(16) KtEntry {
    double a_re, a_im;       // population times voxel weight
    int64_t pair;
    int64_t pad;
};
// Spectrum over (tissue, pair block, tile) items into partial (n_items x 64
// reals of the precision), tile sums per pair into spec (2 n_pairs doubles),
// then signal (2 n_samples doubles) from the entries.
hipError_t launch_kt(const KtItem* items, int64_t n_items, const double* pair_k, const KtPairSum* pair_sums,
                     int64_t n_pairs, const KtEntry* entries, const int64_t* offsets, int64_t n_samples,
                     const float* x, const float* y, const float* z, const float* m0, void* partial, double* spec,
                     double* signal, int precision, hipStream_t st);

// Bytes of the static device array behind the allocation-free entry point.
constexpr int64_t kNoAllocScratchBytes = int64_t(256) << 20;
constexpr int kMaxDevices = 64;
// Device address of that array on `device`, which must be the current
// device the first time it is asked for (hipGetSymbolAddress, cached per
// device afterwards).
hipError_t noalloc_scratch(int device, void** ptr);

}  // namespace ps
