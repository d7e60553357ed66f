/*
 * parspin.h -- C ABI of the MI355X spin-stepping Bloch simulator.
 *
 * The library steps every spin (isochromat) of a discretised object through
 * a pulse sequence with analytic solutions of the Bloch equation and sums
 * the rotating-frame transverse magnetisation of all spins into complex
 * receive-signal samples (section 5.1.1, spin-based simulation procedure;
 * section 3.5.2 for the signal).  The work is data-parallel over spins
 * (section 5.3.2, domain decomposition).
 *
 * Conventions shared by every call:
 *  - No C++ exceptions cross this boundary; every call returns ps_status.
 *    On failure the thread-local message of ps_last_error() says why.
 *  - Device pointers are HIP device addresses on the context's device.  The
 *    caller owns them and keeps them valid until the work that uses them has
 *    completed on the given stream (for ps_submit: until ps_poll/ps_wait
 *    report completion or ps_cancel returns).
 *  - Host pointers are read during the call only; the library copies what it
 *    needs (the sequence is compiled and uploaded during the call).
 *  - Streams are hipStream_t passed as void*; NULL is the null stream.
 */
#ifndef PARSPIN_H
#define PARSPIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ps_status {
    PS_OK = 0,
    PS_E_INVALID_ARG = 1,  /* a pointer, size, count or value is out of range   */
    PS_E_NO_MEMORY = 2,    /* host or device allocation failed                  */
    PS_E_DEVICE = 3,       /* a HIP call failed; ps_last_error() has its text   */
    PS_E_TOO_LARGE = 4,    /* the request's device footprint exceeds the cap    */
    PS_E_NOT_READY = 5,    /* ps_wait timed out / result not yet available      */
    PS_E_CANCELLED = 6,    /* the request was cancelled                         */
    PS_E_NO_DEVICE = 7     /* no usable gfx950 device                           */
} ps_status;

/* ps_event.flags: transverse magnetisation is set to zero at the end of the
 * interval.  An idealised spoiler; the paper has no such primitive. */
#define PS_EV_SPOIL 1u
/* ps_event.flags: record the magnetisation (Mx, My, Mz) of every spin at the
 * end of the interval, after a spoiler (section 7.2: magnetisation instead of
 * echo data).  Honoured by ps_simulate_ex; the other entry points ignore it. */
#define PS_EV_SNAPSHOT 2u
/* ps_event.flags: the event's n_adc samples follow the trajectory table
 * ps_sequence.trajectories[ps_event.trajectory] instead of the n_adc equal
 * sub-steps: sample s is taken t[s] after the interval start, when the
 * moment accumulated since the start is k[s]; the interval still ends after
 * dt with total moment m.  Without this flag ps_event.trajectory must be 0. */
#define PS_EV_TRAJECTORY 4u

typedef struct ps_ctx ps_ctx;  /* opaque; one per device */

/* ps_config.flags: bracket every step-kernel and finalize-kernel launch with
 * HIP events on its stream so that ps_kernel_times() can report durations. */
#define PS_CFG_KERNEL_TIMING 1u
/* ps_config.flags: step every shaped pulse sub-step by sub-step.  By default a
 * shaped pulse that recurs in a request is stepped once per spin into the
 * affine map it applies (every sub-step of eq. 3.23 is affine in M; the map
 * is kept across time slices), and later occurrences apply that map,
 * rotated by their RF phase offset.  Both
 * give the same signal within FP32 rounding; this flag exists to measure and
 * test the sub-step path on sequences with repeated shapes. */
#define PS_CFG_NO_SHAPE_CACHE 2u
/* ps_config.flags: never split readouts across workgroups.  By default an
 * object too small to fill the device runs each workgroup tile as several
 * replicas that repeat the tile's RF and shaped-pulse stepping and share its
 * readouts (a readout changes no spin state); every sample is still computed
 * once, by the same arithmetic, so the signal is bitwise the same. */
#define PS_CFG_NO_READOUT_SPLIT 4u
/* ps_config.flags: tune on first use.  ps_simulate, ps_simulate_rx,
 * ps_simulate_ex, ps_plan_create and ps_simulate_batch first run ps_tune for
 * every request whose class (see ps_tune) has no entry in the context's
 * tiling table yet: a synchronous probe of a few ms per candidate tiling,
 * on a private stream ordered after the work already queued on the call's
 * stream.  ps_submit only reads the table.  Ignored when spins_per_lane is
 * set. */
#define PS_CFG_AUTOTUNE 8u
/* ps_config.flags: the served loop runs one iteration at a time, launching
 * its kernels one by one, instead of replaying them from a HIP graph with
 * short iterations launched ahead (the results are the same; for
 * measurement). */
#define PS_CFG_SERVE_DIRECT 16u
/* ps_config.flags: FP32 readouts on the vector ALUs only.  By default, at one
 * spin per lane, a readout of at least 64 samples whose per-sample step
 * (moment and dwell) it shares with the neighbouring readout is summed over
 * the spins on the matrix cores: the superposition of eq. 3.32 over a tile of
 * 128 samples is a complex matrix product, (sample block) x (spin) times
 * (spin) x (sample in block).  Both give the signal within FP32 rounding;
 * this flag exists to measure and test the vector path. */
#define PS_CFG_NO_MATRIX_READOUT 32u

typedef struct ps_config {
    int32_t device;              /* HIP device ordinal                                 */
    int32_t precision;           /* 32: FP32 stepping (FP64 phases and cross-block
                                    sums); 64: FP64 throughout                         */
    int32_t spins_per_lane;      /* 0 = the tiling table's entry for the request's
                                    class (ps_tune), else the threshold rule of
                                    ps_tile; or fixed: 1, 2, 4, 8 (FP64: 1 or 2)       */
    int32_t flags;               /* PS_CFG_* bits                                      */
    int64_t max_partial_bytes;   /* bound on the per-block partial-sum buffer; longer
                                    sequences run in time slices (0 = default 2 GiB)   */
    int64_t max_footprint_bytes; /* admission cap for served requests (0 = 64 GiB)     */
    int64_t max_slice_steps;     /* served requests: at most this many elementary
                                    intervals per spin in one scheduler iteration, so
                                    that long requests yield the device regularly and
                                    new ones join between their slices (0 = 65,536)    */
} ps_config;

/* Spins as structure-of-arrays, n_spins entries each, FP32, DEVICE memory
 * (section 6.1.1: position, rest magnetisation M0, T1, T2 and the
 * rotating-frame off-resonance of eq. 6.1 / 6.2). */
typedef struct ps_object {
    int64_t n_spins;             /* >= 0                                               */
    const float *x, *y, *z;      /* position, m                                        */
    const float *m0;             /* rest magnetisation (isochromat weight)             */
    const float *t1, *t2;        /* s, > 0; +INF means no relaxation of that kind      */
    const float *dw;             /* rad/s off-resonance (chemical shift + B0 + suscep.)*/
} ps_object;

/* One elementary sequence (section 4.1, eq. 4.1): a hard RF pulse at the
 * start (eq. 3.19), then precession and relaxation over dt under a gradient
 * given by its moment m = (gamma / 2 pi) * integral G dt (eq. 3.16), in
 * cycles/m.  With n_adc = N > 0 the interval is cut into N equal sub-steps
 * and one sample is taken after each (section 5.1.1).  With rf_shape >= 0
 * the shape's sub-steps run first, then the hard pulse, then the interval. */
typedef struct ps_event {
    double   dt;                 /* s, finite, >= 0                                    */
    double   m[3];               /* cycles/m over the whole interval                   */
    double   rf_alpha;           /* rad; 0 = no pulse                                  */
    double   rf_phase;           /* rad; rotation axis (cos, sin, 0) in x'y'; also
                                    added to every sub-pulse phase of rf_shape         */
    int32_t  rf_shape;           /* -1, or index into ps_sequence.shapes               */
    uint32_t n_adc;              /* 0, or number of samples (< 2^31)                   */
    uint32_t flags;              /* PS_EV_SPOIL | PS_EV_SNAPSHOT | PS_EV_TRAJECTORY    */
    uint32_t trajectory;         /* with PS_EV_TRAJECTORY: index into
                                    ps_sequence.trajectories; else 0                   */
} ps_event;

/* A shaped pulse in the hard-pulse approximation (eq. 3.23): n_sub equal
 * sub-steps of length tau, each a hard sub-pulse (alpha[i], phase[i]) at its
 * start followed by precession and relaxation under the moment m_sub. */
typedef struct ps_rf_shape {
    int32_t       n_sub;         /* >= 1                                               */
    int32_t       reserved;
    double        tau;           /* s per sub-step, finite, >= 0                       */
    double        m_sub[3];      /* cycles/m per sub-step                              */
    const double *alpha;         /* HOST, n_sub flip angles, rad (signed)              */
    const double *phase;         /* HOST, n_sub phases, rad                            */
} ps_rf_shape;

/* Sample instants of a non-uniform readout (spirals, curved or variable-rate
 * trajectories played as piecewise-constant gradients): n samples; k[3 s ..
 * 3 s + 2] is the moment (cycles/m) accumulated from the interval start to
 * sample s, t[s] its time after the interval start (s, 0 <= t[0] <= t[1] ...
 * <= dt of every event that uses it). */
typedef struct ps_trajectory {
    int64_t       n;
    const double *k;             /* HOST, 3 n                                          */
    const double *t;             /* HOST, n                                            */
} ps_trajectory;

typedef struct ps_sequence {
    int64_t              n_events;
    const ps_event      *events;        /* HOST                                        */
    int32_t              n_shapes;
    int32_t              n_trajectories;
    const ps_rf_shape   *shapes;        /* HOST                                        */
    const ps_trajectory *trajectories;  /* HOST, may be NULL when n_trajectories = 0   */
} ps_sequence;

/* Fill *cfg with the defaults (device 0, precision 32, tiles from the tiling
 * table or the threshold rule). */
ps_status ps_config_default(ps_config *cfg);

/* Create a context on cfg->device (NULL = defaults).  Fails with
 * PS_E_NO_DEVICE when the device is absent or is not gfx950. */
ps_status ps_create(ps_ctx **out, const ps_config *cfg);

/* Wait for the context's outstanding work and free everything it owns. */
void ps_destroy(ps_ctx *ctx);

/* Message describing the last failure on the calling thread ("" if none). */
const char *ps_last_error(void);

/* Number of ADC samples (the signal length) and the number of elementary
 * intervals each spin is stepped through after cutting ADC intervals into
 * their samples and shaped pulses into their sub-pulses (section 5.1.1: an
 * ADC elementary sequence is divided into as many steps as it has samples;
 * eq. 3.23: a shaped pulse is a list of hard-pulse elementary sequences).
 * Validates the sequence (PS_E_INVALID_ARG with the offending event or
 * shape named by ps_last_error()); needs no device.  Either output pointer
 * may be NULL. */
ps_status ps_count(const ps_sequence *seq, int64_t *n_samples, int64_t *n_steps_per_spin);

/* Simulate one request, stream-ordered on `stream`.
 * signal: DEVICE, 2 * n_samples doubles, interleaved (re, im), samples in
 * event order and by sample index inside an event; it receives
 * sum over spins of (Mx + j My) at every sample (eq. 3.30 - 3.32).
 * n_samples must equal ps_count's value.  The result is bitwise
 * reproducible for a given context configuration and n_spins. */
ps_status ps_simulate(ps_ctx *ctx, const ps_object *obj, const ps_sequence *seq,
                      double *signal, int64_t n_samples, void *stream);

/* Receive coils with inhomogeneous sensitivity (section 3.5.1).  The
 * sensitivity of a coil is S = B1 / i (eq. 3.24); only its transverse
 * components reach the demodulated signal.  Taking eq. 3.25 through the
 * demodulation of eq. 3.28 - 3.31 with both transverse components, coil c
 * receives at every sample
 *     sum over spins of (S_x - j S_y) (Mx + j My),
 * S at the spin, M in the rotating frame, the constant omega_0 / 2 dropped.
 * The homogeneous coil S = (1, 0, 0) gives ps_simulate's signal.
 * s_x, s_y: DEVICE, FP32, n_coils * n_spins each, coil-major (coil c, spin i
 * at [c * n_spins + i]); owned by the caller, read during the call's kernels. */
typedef struct ps_receive {
    int32_t      n_coils;        /* >= 1                                               */
    int32_t      reserved;       /* 0                                                  */
    const float *s_x;            /* DEVICE                                             */
    const float *s_y;            /* DEVICE                                             */
} ps_receive;

/* ps_simulate with receive coils: signal (DEVICE) holds rx->n_coils blocks of
 * 2 * n_samples doubles, coil c's block at signal + 2 * n_samples * c, each
 * laid out as ps_simulate's.  rx == NULL is ps_simulate.  The spins are
 * stepped once for all coils; readouts cost one pass per coil.
 * PS_E_INVALID_ARG for n_coils < 1, a nonzero reserved field or NULL arrays. */
ps_status ps_simulate_rx(ps_ctx *ctx, const ps_object *obj, const ps_sequence *seq, const ps_receive *rx,
                         double *signal, int64_t n_samples, void *stream);

/* Number of events flagged PS_EV_SNAPSHOT (validates the sequence). */
ps_status ps_count_snapshots(const ps_sequence *seq, int64_t *n_snapshots);

/* ps_simulate_rx that also records snapshots: after every event flagged
 * PS_EV_SNAPSHOT, in event order, the magnetisation of every spin in the
 * rotating frame.  snapshots: DEVICE, n_snapshots * 3 * n_spins reals of the
 * stepping precision (float for precision 32, double for 64), laid out
 * [snapshot][component Mx, My, Mz][spin]; n_snapshots must equal
 * ps_count_snapshots (snapshots may be NULL when it is 0).  rx may be NULL
 * (one homogeneous coil).  The signal is bitwise that of ps_simulate_rx. */
ps_status ps_simulate_ex(ps_ctx *ctx, const ps_object *obj, const ps_sequence *seq, const ps_receive *rx,
                         double *signal, int64_t n_samples, void *snapshots, int64_t n_snapshots,
                         void *stream);

/* Spin spacing a sequence needs (section 5.2), from the K-t formalism
 * (section 4.2; host computation, no device).  Every gradient moment of seq
 * (per ADC sample inside readouts, per sub-step inside shapes) must be an
 * integer multiple of dk[d] cycles/m on each axis d (dk[d] = 0: no moment on
 * that axis).  The configuration populations of one reference tissue
 * (t1, t2 in s, > 0, +inf allowed) are tracked through the sequence; then
 *   grey_step == 0: k_max[d] = the largest |k_d| of any configuration with a
 *                   population above 1e-12 M0 at any instant (eq. 5.1);
 *   grey_step > 0:  at every ADC sample the outer transverse configurations
 *                   whose populations add up to at most grey_step / 2 of the
 *                   largest one are left out (eq. 5.4 / 5.5, grey_step being
 *                   the grey-value step, e.g. 1/256);
 * k_max in cycles/m, and dx_max[d] = 1 / (2 k_max[d]) m, the largest spin
 * spacing free of aliasing (eq. 5.2 with k in cycles/m; +inf where k_max is
 * 0).  extent (HOST, may be NULL): the object's size per axis in m (0 on an
 * axis it does not span); then *n_spins_min receives the isochromats one
 * tissue class needs to cover it at that spacing, the product over the axes
 * with extent > 0 and a finite dx_max of ceil(extent / dx_max) (1 when no
 * axis counts).  n_spins_min may be NULL, and must be when extent is.
 * *n_configs_peak (may be NULL): the most transverse configurations
 * populated at once.  PS_E_INVALID_ARG for a moment off the lattice, an
 * invalid sequence or a negative / non-finite extent; PS_E_TOO_LARGE past
 * 2^22 configurations or a spin count beyond 2^62. */
ps_status ps_kt_extent(const ps_sequence *seq, const double dk[3], double t1, double t2, double grey_step,
                       const double extent[3], double k_max[3], double dx_max[3], int64_t *n_spins_min,
                       int64_t *n_configs_peak);

/* ---- K-t simulation ------------------------------------------------------
 * A second engine for the signal, after the K-t formalism (sections 4.2 -
 * 4.4) and its simulation procedure (section 5.1.2): when every gradient
 * moment of the sequence is an integer multiple of a lattice step dk per
 * axis (per ADC sample inside readouts, per sub-step inside shapes), the
 * magnetisation of a tissue with uniform T1, T2 and off-resonance is a
 * finite series of configurations whose populations do not depend on
 * position (eq. 4.7 - 4.11).  The host tracks them per tissue through the
 * sequence (hard pulses eq. 4.14, relaxation eq. 4.15 / 4.16, gradients
 * eq. 4.17, the off-resonance as a turn exp(-j dw t) of every transverse
 * population); the device evaluates every tissue's spatial-frequency
 * function at the configurations' lattice positions and superposes them
 * at each sample (eq. 4.19):
 *   s[n] = sum over tissues c and transverse orders q populated at sample n
 *          of F_c(q) W(q) S_c(q dk),
 *   S_c(k) = sum over the tissue's spins i of m0_i exp(-2 pi j k . x_i),
 *   W(q) = prod over the axes d of sinc(q_d dk_d voxel_d), sinc(u) =
 *          sin(pi u) / (pi u): the spectrum of a box voxel centred on each
 *          spin (the signal integrated over the voxel, section 5.2), 1 for
 *          point spins (voxel = 0).
 * With point spins this equals ps_simulate of the same spins given their
 * tissue's T1, T2 and off-resonance, for every lattice sequence.  Readings
 * (operator order, sample instants, PS_EV_SPOIL) are ps_simulate's. */
typedef struct ps_kt_object {
    int32_t        n_tissues;    /* >= 1                                               */
    int32_t        reserved;     /* 0                                                  */
    const double  *t1, *t2;      /* HOST, n_tissues: s, > 0, +INF allowed              */
    const double  *dw;           /* HOST, n_tissues: rad/s, uniform over the tissue    */
    const int64_t *tissue_begin; /* HOST, n_tissues + 1: tissue c holds spins
                                    tissue_begin[c] .. tissue_begin[c + 1] - 1;
                                    tissue_begin[0] = 0, [n_tissues] = n_spins        */
    int64_t        n_spins;      /* >= 0                                               */
    const float   *x, *y, *z;    /* DEVICE, n_spins: voxel centres, m                  */
    const float   *m0;           /* DEVICE, n_spins: M0 of the voxel (density x volume)*/
    double         voxel[3];     /* box size per axis, m (0: point spins on that axis) */
} ps_kt_object;
/* Signal of obj under seq by the K-t engine, stream-ordered on `stream`.
 * dk: HOST, lattice step per axis in cycles/m (0 on an axis with no
 * moment).  signal: DEVICE, 2 * n_samples doubles as for ps_simulate; the
 * spectrum is summed in the context's precision (FP32 or FP64 sine and
 * cosine of FP64 phases), tiles and configurations in FP64.  The population
 * tracking runs on the host during the call.  PS_E_INVALID_ARG for a moment
 * off the lattice, trajectory readouts, tissue arrays that do not cover the
 * spins, or the arguments ps_simulate refuses; PS_E_TOO_LARGE past 2^22
 * configurations of a tissue or 2^28 (sample, configuration) pairs. */
ps_status ps_kt_simulate(ps_ctx *ctx, const ps_kt_object *obj, const ps_sequence *seq, const double dk[3],
                         double *signal, int64_t n_samples, void *stream);

/* Compiled plans: one request compiled once and its kernel launches captured
 * in a HIP graph, for callers that simulate the same (object layout,
 * sequence, coils) many times, e.g. parameter sweeps that rewrite the object
 * arrays in place.  The plan owns its device tables and work buffers; the
 * pointers in obj, rx and signal are captured and must stay valid while the
 * plan exists (their contents may change between replays).  Arguments and
 * errors as for ps_simulate_rx (rx may be NULL).  Snapshots are not captured. */
typedef struct ps_plan ps_plan;
ps_status ps_plan_create(ps_ctx *ctx, const ps_object *obj, const ps_sequence *seq, const ps_receive *rx,
                         double *signal, int64_t n_samples, ps_plan **plan);
/* Replay the plan, stream-ordered on `stream`: one graph launch; the result
 * is bitwise that of ps_simulate_rx on the same context.  Replays of one plan
 * share its buffers: launch them on one stream (they then run in order). */
ps_status ps_plan_launch(ps_plan *plan, void *stream);
/* Wait for the plan's last replay, then free it. */
void ps_plan_destroy(ps_plan *plan);

/* ps_simulate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the call allocates nothing -- no hipMalloc, hipFree or pinned allocation,
 * no allocating library routine.  Its tables, partial-sum rows, finalize
 * sums and slice state live in a static device array of 256 MiB
 * (kNoAllocScratchBytes) that every GPU the library runs on holds from
 * load to process end; its tables are uploaded from 8 MiB of pinned staging
 * the context set aside at ps_create.  Arguments, output and errors as for
 * ps_simulate; additionally PS_E_TOO_LARGE, with nothing launched, when the
 * request does not fit: the tables exceed the staging, or the slice state
 * (up to 30 reals per spin) plus the partial rows of its smallest time
 * slices exceed the array.  When the context's partial-row bound would
 * overflow the array the request runs in shorter time slices (the result
 * then matches ps_simulate within FP32 rounding instead of bitwise).
 * Nothing in the array has to start at zero: every value a launch reads was
 * written earlier in the same call.  All calls on one GPU share the array
 * (across contexts): calls on one stream run in order, calls that overlap
 * on the device -- on different streams or from different contexts -- race
 * and give undefined results.  The tiling is the table's or the rule's
 * (PS_CFG_AUTOTUNE does not tune here, since tuning allocates).  A call
 * waits on the host for the previous call's table upload before it reuses
 * the staging. */
ps_status ps_simulate_noalloc(ps_ctx *ctx, const ps_object *obj, const ps_sequence *seq, double *signal,
                              int64_t n_samples, void *stream);

/* Simulate n_requests independent requests together, stream-ordered on
 * `stream`.  All workgroup tiles of all requests form one work queue that a
 * persistent kernel drains (one launch per spins-per-lane class and time
 * slice round), after the paper's dynamic assignment of more spin blocks than
 * compute nodes (section 5.3.2).  objs[i], seqs[i], signals[i] and
 * n_samples[i] are as for ps_simulate.  Each request keeps the tiling and
 * time slicing it would get alone, so signals[i] is bitwise identical to
 * ps_simulate on the same context.  On failure no request has been started;
 * ps_last_error() names the offending request. */
ps_status ps_simulate_batch(ps_ctx *ctx, int32_t n_requests, const ps_object *objs, const ps_sequence *seqs,
                            double *const *signals, const int64_t *n_samples, void *stream);

/* ---- served execution ------------------------------------------------
 * A scheduler thread (started by the first ps_submit on a context) admits
 * queued requests in submission order while the sum of their device
 * footprints stays under ps_config.max_footprint_bytes (a request of at least
 * 2.5e10 spin-steps waits while another such request runs, letting smaller
 * ones behind it through), and advances every
 * admitted request by one time slice per iteration in one batched round, so
 * requests that arrive while others run join at the next iteration
 * (continuous batching; after the master / compute-node / superposition
 * roles of sections 5.3.2 and 6.3).  An iteration's kernels are replayed
 * from a HIP graph (kernel nodes only, their arguments updated per
 * iteration; PS_CFG_SERVE_DIRECT launches them one by one instead).  While
 * iterations are short (at most 1e10 spin-steps) the next one is planned
 * and launched before the previous completes, two in flight, and the host
 * waits on the device only to retire completed iterations (the master learns
 * of a finished block after its superposition, section 7.3.1).  Spin state
 * stays in device memory between slices.  A request's result is bitwise the same alone or in any
 * mix.  The object arrays must hold their data when ps_submit is called (no
 * ordering with the caller's streams); signal must not be read before
 * ps_poll / ps_wait report completion. */

typedef enum ps_request_state {
    PS_REQ_QUEUED = 0, PS_REQ_RUNNING = 1, PS_REQ_DONE = 2, PS_REQ_FAILED = 3, PS_REQ_CANCELLED = 4
} ps_request_state;

typedef struct ps_request_info_t {
    int32_t state;               /* ps_request_state                                   */
    int32_t status;              /* final ps_status (PS_OK while not finished)         */
    double  t_submit, t_admit, t_done;  /* s since the scheduler started; -1 = not yet */
    int64_t n_slices;            /* time slices the request runs as                    */
    int64_t footprint_bytes;     /* counted against the admission cap                  */
    int64_t n_spins, n_steps_per_spin;
    double  t_kernel;            /* s of device time of the iterations it ran in (see
                                    ps_stats)                                          */
} ps_request_info_t;

typedef struct ps_server_stats_t {
    int64_t iterations, queued, running, footprint_in_use;
    double  now;                 /* s since the scheduler started                      */
} ps_server_stats_t;

/* Queue one request; arguments as for ps_simulate.  Validates and compiles
 * on the calling thread.  PS_E_TOO_LARGE when the request alone exceeds the
 * admission cap.  *ticket identifies it in the calls below.  Thread-safe. */
ps_status ps_submit(ps_ctx *ctx, const ps_object *obj, const ps_sequence *seq, double *signal,
                    int64_t n_samples, uint64_t *ticket);
/* *done = 1 once the request has finished (completed, failed or cancelled). */
ps_status ps_poll(ps_ctx *ctx, uint64_t ticket, int32_t *done);
/* Block until the request finishes (timeout_s < 0: no limit).  Returns its
 * final status, or PS_E_NOT_READY on timeout. */
ps_status ps_wait(ps_ctx *ctx, uint64_t ticket, double timeout_s);
/* Cancel: a queued request is dropped, a running one at the next iteration
 * boundary (its signal is then undefined).  Other requests are unaffected. */
ps_status ps_cancel(ps_ctx *ctx, uint64_t ticket);
/* State, status and timing of a request. */
ps_status ps_request_info(ps_ctx *ctx, uint64_t ticket, ps_request_info_t *out);
/* Timing of a served request (the bookkeeping of the paper's master, section
 * 6.3, and the simulation time of eq. 7.1), in seconds:
 *   t_queue  from ps_submit to admission (waiting for the footprint cap or
 *            for a large request ahead of it);
 *   t_kernel device time of the scheduler iterations the request ran in:
 *            for each, the span from the start of its first kernel to the end
 *            of its last one, measured with HIP events.  Requests admitted
 *            together share an iteration's kernels, so each is charged the
 *            whole span (the time the device spent with it in flight);
 *   t_e2e    from ps_submit to completion.
 * Values not known yet (a request still queued or running) are -1; any
 * output pointer may be NULL.  PS_E_INVALID_ARG for an unknown ticket. */
ps_status ps_stats(ps_ctx *ctx, uint64_t ticket, double *t_queue, double *t_kernel, double *t_e2e);
/* ---- scheduler test support -----------------------------------------------
 * A context whose served loop (ps_submit and the calls below) runs without a
 * device, for testing admission, continuous batching, cancellation, failure
 * handling and the timing bookkeeping on a CPU.  It computes no
 * magnetisation: every served iteration "runs" each member's time slice by
 * writing into the request's signal, which must be HOST memory here, the
 * pattern (re, im) = (n_spins + sample index, slice index) for every sample
 * of the slice (zeros for an object without spins), and "takes"
 * iteration_seconds of stand-in device time; the object arrays are never
 * read.  The iteration numbered fail_iteration (0-based, -1: none) reports
 * a device error: the requests with a slice in it fail with PS_E_DEVICE,
 * the others go on.  Only ps_submit, ps_poll, ps_wait, ps_cancel,
 * ps_request_info, ps_stats, ps_release, ps_server_stats and ps_destroy
 * accept such a context; every other call returns PS_E_INVALID_ARG. */
typedef struct ps_test_backend {
    double  iteration_seconds;   /* >= 0                                               */
    int64_t fail_iteration;      /* -1 or the iteration that fails                     */
} ps_test_backend;
ps_status ps_create_scheduler_test(ps_ctx **out, const ps_config *cfg, const ps_test_backend *backend);

/* Forget a finished request's record (PS_E_NOT_READY while in flight). */
ps_status ps_release(ps_ctx *ctx, uint64_t ticket);
/* Scheduler counters (all zero before the first ps_submit). */
ps_status ps_server_stats(ps_ctx *ctx, ps_server_stats_t *out);

/* The threshold rule's tiling for an object of n_spins spins on this
 * context (what a request gets when the tiling table has no entry for its
 * class): spins held per lane -- the configured value, else 2 once the
 * object gives every SIMD two waves at 2 spins per lane, else 1 -- and
 * spins per workgroup (4 waves of 64 lanes).  A request whose FP32 readouts
 * take the matrix cores (PS_CFG_NO_MATRIX_READOUT) gets 1 whatever its
 * size; this call, which sees no sequence, gives the size rule. */
ps_status ps_tile(ps_ctx *ctx, int64_t n_spins, int32_t *spins_per_lane, int64_t *spins_per_block);

/* ---- tiling autotuner -------------------------------------------------
 * The paper sizes its spin blocks so that every compute node gets one and
 * hands out more blocks than nodes so that their speeds level out (section
 * 5.3.2).  Here a block is a workgroup tile of 256 S spins, S spins per
 * lane; readout replicas split a small object's readouts over idle compute
 * units.  ps_tune times the candidate tilings of a request on the device
 * and records the fastest for the request's class in the context's tiling
 * table; every later request of that class, on every entry point, uses it.
 * A class is: precision, floor(log2 n_spins), floor(log2 of the longest
 * readout in samples) (none without readouts), shaped pulses or not,
 * ceil(log2 n_coils).  Candidates: S = 1, 2, 4, 8 (FP64: 1, 2) with the
 * readout-replica rule, plus no replicas and twice the rule's count where
 * the rule gives replicas.  Each is timed on a probe -- the request's object
 * with the longest prefix of its sequence of about 6e10 spin-steps (at least
 * through its first readout; the whole sequence when shorter) -- by the
 * device time of its kernels, in rounds over all candidates (one warm-up
 * round, then five timed rounds; median of each candidate's five).  The
 * threshold rule's tiling is kept unless a candidate is more than 3 % faster
 * (for a request whose probe takes under 1 ms, 15 % for another
 * spins-per-lane value: such requests share batched rounds, which run one
 * kernel per spins-per-lane class).
 * The result of a request depends on its tiling (bitwise; within the FP32
 * tolerance across tilings), so a request run after its class was tuned may
 * differ in the last bits from one run before. */
#define PS_TUNE_MAX_CANDIDATES 12
/* ps_tune flags: time the candidates again even if the class has an entry. */
#define PS_TUNE_FORCE 1u
typedef struct ps_tune_result {
    int32_t spins_per_lane;      /* the class's tiling                                 */
    int32_t replicas;            /* 0: no readout replicas, 1: the rule, 2: twice it   */
    int32_t from_table;          /* 1: the class had an entry; nothing was timed       */
    int32_t n_candidates;        /* candidates timed (0 with from_table)               */
    double  best_ms;             /* the chosen tiling's median probe time              */
    double  rule_ms;             /* the threshold rule's tiling on the same probe      */
    int64_t probe_events;        /* events of the sequence prefix the probe ran        */
    int32_t cand_spins_per_lane[PS_TUNE_MAX_CANDIDATES];
    int32_t cand_replicas[PS_TUNE_MAX_CANDIDATES];
    double  cand_ms[PS_TUNE_MAX_CANDIDATES];
} ps_tune_result;
/* Tune the request's class (arguments as for ps_simulate_rx; rx may be NULL;
 * the object arrays must hold their data: the probe runs on a private stream
 * after work queued on the null stream).  Synchronous; allocates a probe
 * signal buffer for the call.  out may be NULL.  PS_E_INVALID_ARG for an
 * invalid request, an object without spins or a context whose
 * spins_per_lane is fixed. */
ps_status ps_tune(ps_ctx *ctx, const ps_object *obj, const ps_sequence *seq, const ps_receive *rx, uint32_t flags,
                  ps_tune_result *out);
/* The tiling a request of n_spins spins, this sequence and n_coils coils (0:
 * one homogeneous coil) gets on this context, and whether it comes from the
 * tiling table (*tuned = 1) or the threshold rule.  Any output may be NULL. */
ps_status ps_tile_for(ps_ctx *ctx, int64_t n_spins, const ps_sequence *seq, int32_t n_coils,
                      int32_t *spins_per_lane, int32_t *replicas, int32_t *tuned);
/* How the readouts of a request (n_spins spins, this sequence, n_coils coils
 * with 0 for one homogeneous coil) are summed at spins_per_lane (1, 2, 4 or
 * 8) on this context, planned as ps_simulate_rx plans it: *n_readouts ADC
 * intervals (after time slicing and cutting at 8,192 samples), *n_matrix of
 * them on the matrix cores, *matrix_only = 1 when that is all of them with
 * one per-sample step, so that the kernel built without the vector readout
 * runs the request (see PS_CFG_NO_MATRIX_READOUT), and *n_slices time
 * slices.  Any output may be NULL.  PS_E_INVALID_ARG for an invalid
 * sequence, n_spins < 0 or n_coils < 0.  Host only
 * (no device work); measurement support, not part of the simulation. */
ps_status ps_readout_path(ps_ctx *ctx, int64_t n_spins, const ps_sequence *seq, int32_t n_coils,
                          int32_t spins_per_lane, int64_t *n_readouts, int64_t *n_matrix, int32_t *matrix_only,
                          int64_t *n_slices);
/* Write the tiling table to a text file, headed by the device model, its
 * compute-unit count and a hash of this library's sources. */
ps_status ps_tune_save(ps_ctx *ctx, const char *path);
/* Add the entries of a file written by ps_tune_save for this precision to
 * the table (*n_loaded: how many; may be NULL).  PS_E_INVALID_ARG when the
 * file is unreadable, malformed, or written for another device model or
 * library build (nothing is loaded then). */
ps_status ps_tune_load(ps_ctx *ctx, const char *path, int32_t *n_loaded);
/* Empty the tiling table. */
ps_status ps_tune_clear(ps_ctx *ctx);

/* Durations in ms of the kernels launched since the previous call (contexts
 * created with PS_CFG_KERNEL_TIMING only): the step kernels in launch order
 * into step_ms[0 .. min(capacity, *n_step) - 1] (step_ms may be NULL when
 * capacity is 0), their count into *n_step, and the summed finalize-kernel
 * time into *finalize_ms.  Waits for those kernels to finish, then forgets
 * them.  Measurement support, not part of the simulation. */
ps_status ps_kernel_times(ps_ctx *ctx, double *step_ms, int64_t capacity, int64_t *n_step,
                          double *finalize_ms);

/* The vector FMA rate, in TFLOP/s (an FMA counted as 2 flops), that code
 * built like this library's kernels attains on the context's device:
 * 8,192 workgroups of 256 lanes run 8 independent FMA chains of 4,096 steps
 * per lane in FP32 (precision 32; packed FP32 disabled, as for the kernels)
 * or FP64 (precision 64); the best of 5 timed launches after one warm-up.
 * Allocates 16 bytes of device memory for the call; synchronous.
 * PS_E_INVALID_ARG for a NULL argument or another precision, PS_E_DEVICE on
 * a HIP error.  Measurement support, not part of the simulation. */
ps_status ps_valu_peak(ps_ctx *ctx, int32_t precision, double *tflops);

#ifdef __cplusplus
}
#endif

#endif /* PARSPIN_H */
