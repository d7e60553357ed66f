// Device-side sequence table shared by the host compiler and the kernels.
//
// The host compiles the caller's elementary sequences into a short list of
// operations that only appear where a spin's state changes in a way that is
// not a pure precession/relaxation: hard RF pulses, shaped pulses, ADC
// readouts and spoilers.  Free-precession intervals between them cost
// nothing on the device: precession about z and relaxation over consecutive
// intervals compose in closed form (eq. 3.5 / 3.14: phases and times add),
// so the compiler only accumulates, per operation,
//   k   = gradient moment since the transverse anchor (cycles/m, FP64),
//   txy = time since the transverse anchor (s, FP64),
//   tz  = time since the longitudinal anchor (s, FP64),
// and every spin keeps its magnetisation at its anchors ("lazy anchors"):
//   Mxy(t) = Mxy_a * exp(-txy/T2) * exp(-j 2 pi (k.x + dw/(2 pi) txy))
//   Mz(t)  = M0 + (Mz_a - M0) * exp(-tz/T1).
// An RF pulse or shaped pulse evaluates both, rotates, and resets both
// anchors; a spoiler zeroes Mxy_a and resets only the transverse anchor.
#pragma once
#include <stdint.h>

namespace ps {

enum OpKind : uint32_t {
    OP_RF = 1,     // hard pulse: evaluate, rotate by r (eq. 3.19), re-anchor
    OP_ADC = 2,    // n samples at k, k + mu, ...; txy, txy + tau, ...
    OP_SPOIL = 3,  // Mxy_a := 0 (transverse anchor reset)
    OP_SHAPE = 4,  // shaped pulse: evaluate, then n_sub sub-steps (eq. 3.23)
    OP_SNAP = 5,   // evaluate and store every spin's M as snapshot aux
    OP_ADCT = 6,   // n samples at tabulated (k, t): rows u.tab.row ... of the
                   // trajectory table hold (K + k_s, txy + t_s), absolute
};

enum OpFlags : uint32_t {
    OPF_MXY_ZERO = 1u,  // Mxy_a is known to be 0 for every spin (after init/spoil)
    OPF_EVEN_T = 2u,    // ADCT: sample instants equally spaced by u.tab.dt
    OPF_MATRIX = 4u,    // ADC: sum over the spins on the matrix cores (FP32,
                        // one spin per lane; other tilings ignore it)
};

// Matrix-core readouts: tiles of kMatrixTile samples; the host marks a
// readout for them from kMatrixMinSamples samples on.
constexpr int kMatrixTile = 128;
constexpr int kMatrixMinSamples = 64;

// 128-byte operation record.
struct alignas(16) Op {
    double k[3];   // moment since the transverse anchor, at the op (RF/SHAPE)
                   // or at sample 0 (ADC), cycles/m
    double txy;    // time since the transverse anchor, same instant, s
    double tz;     // time since the longitudinal anchor (RF/SHAPE), s
    union {
        double r64[9];                           // RF rotation, FP64 tables
        float r32[9];                            // RF rotation, FP32 tables
        struct { double mu[3]; double tau; } adc;  // ADC: per-sample moment and
                                                   // dwell
        struct { uint64_t row; double dt; } tab; // ADCT: first row of its samples;
                                                 // spacing of the instants (OPF_EVEN_T)
        struct {
            double mu[3];       // per-sub-step moment (same place as adc.mu)
            double tau;         // sub-step duration (same place as adc.tau)
            double rot[2];      // cos, sin of the event's RF phase
            int32_t slot;       // propagator cache slot, or -1 (step directly)
            uint32_t mode;      // ShapeMode
            int32_t shape_id;   // index of the shape in the sequence
        } shape;
    } u;
    uint32_t kind;
    uint32_t flags;
    uint32_t n;    // ADC: samples; SHAPE: sub-steps
    uint32_t aux;  // ADC: first sample's offset inside the time slice;
                   // SHAPE: first sub-step index in the shape rotation table;
                   // SNAP: snapshot index
};
static_assert(sizeof(Op) == 128, "Op must be 128 bytes");

// A SHAPE op keeps the shape's sub-step duration and per-sub-step moment in
// u.shape (mu, tau).  Its sub-step rotations live in a separate table of 9
// reals per sub-step, one block of rows per shape, built with the shape's own
// sub-pulse phases.  The event's RF phase phi enters as a conjugation: adding
// phi to every sub-pulse phase turns each sub-pulse rotation R into
// Rz(phi) R Rz(-phi) (eq. 3.19), and precession about z and relaxation
// commute with Rz, so the whole pulse maps M to Rz(phi) P(Rz(-phi) M), P
// being the pulse at the shape's own phases.  Phase-cycled sequences thus
// share one block of rows.
constexpr int kMaxShapeRows = 512;

// Propagator cache for repeated shaped pulses.  For a given spin a shaped
// pulse (its sub-pulses, its slab gradient, the spin's off-resonance and
// relaxation over the sub-steps) is one fixed affine map M -> A M + b, since
// every sub-step of eq. 3.23 is affine in M.  The first occurrence of the
// shape in a launch builds (A, b) per spin and keeps it in LDS; later
// occurrences apply it, each with its own phase conjugation as above.
enum ShapeMode : uint32_t {
    SHAPE_DIRECT = 0,  // step the sub-steps (no cache)
    SHAPE_FILL = 1,    // build the slot's map, then apply it
    SHAPE_APPLY = 2,   // apply the slot's map (rot gives the phase offset)
};
constexpr int kShapeSlots = 2;
constexpr int kShapeCacheReals = 12;  // A (3 x 3, row-major) then b (3)

// Slice state per spin, in reals (SoA rows of n_spins): two buffers of
// anchors (Mxy_a re, im, Mz_a) that alternate between slices, then the
// propagator slots kept across slices.  A slot is written once, by the
// slice that fills it, and only read afterwards, so it needs one buffer.
constexpr int kStateSlot0 = 6;
constexpr int64_t state_reals_per_spin(int n_state_slots) {
    return kStateSlot0 + (int64_t)kShapeCacheReals * n_state_slots;
}

}  // namespace ps
