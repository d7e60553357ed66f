// Host-side sequence compiler: elementary sequences -> device operations.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/parspin.h"
#include "ps_ops.h"

namespace ps {

struct Slice {
    int64_t op_begin = 0, op_end = 0;  // operation range of the slice
    int64_t sample_begin = 0;          // index of the slice's first sample
    int64_t n_samples = 0;
    int32_t n_cache_slots = 0;         // shaped-pulse propagator slots its ops use
    uint32_t cache_load = 0;           // slots whose propagators it reads from the slice state
    uint32_t cache_save = 0;           // slots whose propagators it writes to the slice state
};

struct Program {
    std::vector<Op> ops;               // rotation deltas R - I in FP64 (r64)
    std::vector<double> rows;          // shaped-pulse rotation deltas, 9 per sub-step
    std::vector<double> traj;          // trajectory sample rows: K + k_s (3), txy + t_s
    int64_t n_samples = 0;
    int64_t n_steps = 0;               // intervals per spin (see ps_count)
    int64_t n_rf = 0, n_shape_substeps = 0, n_adc_ops = 0;
    int64_t n_snapshots = 0;           // events flagged PS_EV_SNAPSHOT
    int32_t n_state_slots = 0;         // propagator slots kept in the slice state between slices
    bool any_matrix = false;           // some readout marked OPF_MATRIX
    bool matrix_only = false;          // every readout marked OPF_MATRIX, none tabulated (OP_ADCT),
    double matrix_mu[3] = {0, 0, 0};   // and all with this per-sample step (mu, tau)
    double matrix_tau = 0;
    std::vector<Slice> slices;
};

// Eq. 3.19: rotation matrix of a hard pulse (alpha, phi), row-major.
void rf_matrix(double alpha, double phi, double r[9]);
// The same rotation minus the identity, R - I, formed without cancellation.
// Device tables hold these deltas: M <- M + (R - I) M keeps small pulses
// exact to FP32 relative precision of their deviation from the identity.
void rf_delta(double alpha, double phi, double d[9]);

// Validate and compile; on failure returns an error status and sets *err.
// With snapshots, events flagged PS_EV_SNAPSHOT become OP_SNAP operations;
// without, the flag is only counted.
ps_status compile_sequence(const ps_sequence* seq, Program* out, std::string* err, bool snapshots = false);

// Cut the program into time slices of at most max_samples samples each,
// setting every ADC op's offset inside its slice.  max_samples >= 1.  A
// readout that does not fit the rest of a slice starts the next one when it
// fits a slice of its own (readouts stay whole, so each keeps its readout
// path); only readouts longer than max_samples are split, exactly.  A
// Cartesian readout is also cut into runs of near-equal length, at most
// kAdcRun samples: each run starts from its own FP64 phase, which bounds
// the FP32 recurrence a readout accumulates (its anchor advances one
// multiply per wave group's 32 G samples, and the rounding of that factor
// adds up linearly along the run).
constexpr int64_t kAdcRun = 8192;
void plan_slices(Program* p, int64_t max_samples);

// Give every shape that occurs often (at least five times) in the program a
// propagator cache slot (at most max_slots <= kShapeSlots, the most frequent
// shapes first): its first occurrence fills the slot, later ones apply it.
// A slot filled in one time slice and used in a later one is written to the
// slice state at the end of the slice that filled it and read back by the
// slices that use it (Slice::cache_save / cache_load), so a shape is stepped
// sub-step by sub-step once per request.  Other SHAPE ops (all of them when
// max_slots is 0) step their sub-steps directly.  Run after the slices are
// final.
void assign_shape_slots(Program* p, int max_slots);

// Copy of the ops with rotations narrowed to FP32 (precision 32 tables).
void narrow_rotations(std::vector<Op>* ops);
// Flag OPF_MATRIX on the readouts of at least kMatrixMinSamples samples whose
// per-sample step (mu, tau) equals that of the readout before or after them:
// the matrix-core path builds per-spin tables for a step once and keeps them
// while the step stays the same, so it pays off for runs of such readouts.
// Sets p->any_matrix when it flags one, and p->matrix_only (and matrix_mu /
// matrix_tau) when that covers every readout, none is tabulated and all
// share one step.
void mark_matrix_readouts(Program* p);

}  // namespace ps
