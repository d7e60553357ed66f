/*
 * FP64 CPU oracle of spin-based Bloch simulation.  TEST INFRASTRUCTURE ONLY:
 * it exists so that tests, the smoke check and the benchmark's CPU baseline
 * can check the GPU library against an independent, plain, slow and
 * obviously correct implementation.  Nothing in the product path may load it.
 *
 * What it computes (section 5.1.1, the course of a spin-based simulation):
 * every spin starts at thermal equilibrium M = (0, 0, M0).  The elementary
 * sequences are applied in order (eq. 4.1): a hard RF rotation at the start
 * of the interval (eq. 3.19), then precession about z by the gradient phase
 * and the off-resonance phase together with T1/T2 relaxation over the
 * interval (eq. 3.5 / 3.12 / 3.14 in the rotating frame, eq. 3.8).  An
 * interval with N ADC samples is cut into N equal sub-steps and the
 * magnetisation is recorded after each one; the signal of a sample is the
 * sum over all spins of the rotating-frame transverse magnetisation
 * Mx + j My (eq. 3.30 - 3.32 and the conclusion of section 3.5.2).
 * A shaped pulse is its own list of n_sub elementary sequences, each a hard
 * sub-pulse followed by precession and relaxation (eq. 3.23).
 *
 * Readings where the paper leaves a choice:
 *  - the gradient is given by its moment m = (gamma/2pi) integral G dt in
 *    cycles/m (eq. 3.16); its phase over a sub-step is 2 pi (m_sub . x);
 *  - off-resonance dw (rad/s) precesses in the same sense as a positive
 *    gradient phase: theta = 2 pi (m_sub . x) + dw * tau, and
 *    (Mx, My) <- E2 [[cos, sin], [-sin, cos]] (Mx, My)  (eq. 3.5 matrix);
 *  - an event with a shape runs the shape's sub-steps first (each sub-pulse
 *    phase is offset by the event's RF phase), then the event's own hard
 *    pulse, then its interval;
 *  - SPOIL sets Mx = My = 0 at the end of the interval (an idealised
 *    spoiler; the paper has no such primitive);
 *  - an event with a trajectory takes its samples at the listed instants t_s
 *    after the interval start, where the moment accumulated since the start
 *    is k_s: the interval is cut at those instants (precession and relaxation
 *    over each piece with its own moment), the magnetisation recorded at
 *    each, and the last piece runs to dt with the remaining moment m - k_last;
 *  - SNAPSHOT records every spin's (Mx, My, Mz) at the end of the interval,
 *    after the spoiler if both are set (the magnetisation output of section
 *    7.2, the state the next elementary sequence starts from);
 *  - T1 or T2 = +inf means no relaxation of that kind (exp(-t/inf) = 1).
 *
 * Receive coils (section 3.5.1, eq. 3.24 / 3.25): with an inhomogeneous
 * receive sensitivity S(x) every spin's magnetisation is weighted before the
 * superposition.  Taking eq. 3.25 through the same steps as eq. 3.28 - 3.31
 * (laboratory-frame precession at the carrier, time derivative, quadrature
 * demodulation and low-pass filtering) for a sensitivity with both
 * transverse components gives, with the constant omega_0 / 2 dropped as for
 * the homogeneous coil,
 *     real part  = sum_i  S_x Mx + S_y My       (in-plane dot product)
 *     imag part  = sum_i  S_x My - S_y Mx       (z component of S x M)
 * with S at the spin and M in the rotating frame.  S_z does not contribute:
 * it multiplies the slowly varying Mz, which the demodulation removes.
 * Without coils S = (1, 0, 0), which gives the sum of Mx + j My.
 *
 * Every spin is independent.  Threads take contiguous spin ranges and keep
 * private FP64 signal buffers that are summed in thread order at the end.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_SPOIL 1u
#define ORACLE_SNAPSHOT 2u

typedef struct {
    /* spins */
    const double *x, *y, *z, *m0, *t1, *t2, *dw;
    /* events */
    int64_t n_events;
    const double *ev_dt, *ev_m, *ev_alpha, *ev_phase;
    const int32_t *ev_shape;
    const int64_t *ev_nadc;
    const uint32_t *ev_flags;
    /* shapes */
    int32_t n_shapes;
    const int64_t *sh_nsub, *sh_offset;
    const double *sh_tau, *sh_m, *sh_alpha, *sh_phase;
    int64_t n_samples;
    /* receive coils: transverse sensitivity of each coil at each spin,
     * coil-major (s_x[c * n_spins + i]); n_coils == 0: one coil S = (1, 0, 0) */
    int32_t n_coils;
    int64_t n_spins;
    const double *s_x, *s_y;
    /* snapshots: [snapshot][component][spin], may be NULL */
    double *snap;
    /* trajectories: event e uses trajectory ev_traj[e] (-1: equal sub-steps);
     * trajectory j has tr_n[j] samples at rows tr_off[j] .. of tr_k (3 per
     * row) and tr_t */
    const int32_t *ev_traj;
    const int64_t *tr_n, *tr_off;
    const double *tr_k, *tr_t;
} problem_t;

typedef struct {
    const problem_t *pb;
    int64_t begin, end;
    double *signal;   /* 2 * n_samples per coil, private to the thread */
    double *final_m;  /* 3 * n_spins, shared, disjoint ranges, may be NULL */
} job_t;

/* Hard RF pulse, eq. 3.19: rotation by flip alpha about the axis in the
 * x'y' plane at phase phi, written out element by element as printed. */
static void rf_pulse(double M[3], double alpha, double phi)
{
    double ca = cos(alpha), sa = sin(alpha);
    double cp = cos(phi), sp = sin(phi);
    double r00 = cp * cp + sp * sp * ca, r01 = sp * cp * (1.0 - ca), r02 = -sp * sa;
    double r10 = sp * cp * (1.0 - ca),   r11 = sp * sp + cp * cp * ca, r12 = cp * sa;
    double r20 = sp * sa,                r21 = -cp * sa,               r22 = ca;
    double mx = M[0], my = M[1], mz = M[2];
    M[0] = r00 * mx + r01 * my + r02 * mz;
    M[1] = r10 * mx + r11 * my + r12 * mz;
    M[2] = r20 * mx + r21 * my + r22 * mz;
}

/* Free precession and relaxation over tau under a gradient of moment mu
 * (cycles/m) and off-resonance dw: eq. 3.14 with the off-resonance term of
 * eq. 3.12 folded into the rotation angle, T_Relax * T_grad * M + T_Relax,z. */
static void precess_relax(double M[3], double tau, const double mu[3],
                          double x, double y, double z, double dw,
                          double m0, double t1, double t2)
{
    const double two_pi = 6.283185307179586476925286766559;
    double theta = two_pi * (mu[0] * x + mu[1] * y + mu[2] * z) + dw * tau;
    double c = cos(theta), s = sin(theta);
    double e1 = exp(-tau / t1), e2 = exp(-tau / t2);
    double mx = M[0], my = M[1];
    M[0] = e2 * (c * mx + s * my);
    M[1] = e2 * (-s * mx + c * my);
    M[2] = e1 * M[2] + m0 * (1.0 - e1);
}

/* Add spin i's magnetisation M to sample `sample` of every coil's signal. */
static void record(const problem_t *pb, int64_t i, double *signal, int64_t sample, const double M[3])
{
    if (pb->n_coils == 0) {
        signal[2 * sample] += M[0];
        signal[2 * sample + 1] += M[1];
        return;
    }
    for (int32_t c = 0; c < pb->n_coils; ++c) {
        double sx = pb->s_x[c * pb->n_spins + i], sy = pb->s_y[c * pb->n_spins + i];
        double *sc = signal + 2 * pb->n_samples * c;
        sc[2 * sample] += sx * M[0] + sy * M[1];
        sc[2 * sample + 1] += sx * M[1] - sy * M[0];
    }
}

static void run_spin(const problem_t *pb, int64_t i, double *signal, double *final_m)
{
    double x = pb->x[i], y = pb->y[i], z = pb->z[i];
    double m0 = pb->m0[i], t1 = pb->t1[i], t2 = pb->t2[i], dw = pb->dw[i];
    double M[3] = {0.0, 0.0, m0};
    int64_t sample = 0;
    int64_t snap = 0;

    for (int64_t e = 0; e < pb->n_events; ++e) {
        int32_t sh = pb->ev_shape[e];
        if (sh >= 0) {
            /* shaped pulse: n_sub elementary sequences (eq. 3.23) */
            int64_t n_sub = pb->sh_nsub[sh], off = pb->sh_offset[sh];
            double tau = pb->sh_tau[sh];
            const double *mu = pb->sh_m + 3 * sh;
            for (int64_t k = 0; k < n_sub; ++k) {
                double a = pb->sh_alpha[off + k];
                if (a != 0.0)
                    rf_pulse(M, a, pb->sh_phase[off + k] + pb->ev_phase[e]);
                precess_relax(M, tau, mu, x, y, z, dw, m0, t1, t2);
            }
        }
        if (pb->ev_alpha[e] != 0.0)
            rf_pulse(M, pb->ev_alpha[e], pb->ev_phase[e]);

        int64_t n_adc = pb->ev_nadc[e];
        int32_t tj = pb->ev_traj ? pb->ev_traj[e] : -1;
        if (tj >= 0) {
            /* samples at the trajectory's instants, then the rest of the interval */
            double t_prev = 0.0, k_prev[3] = {0.0, 0.0, 0.0};
            const double *tk = pb->tr_k + 3 * pb->tr_off[tj], *tt = pb->tr_t + pb->tr_off[tj];
            for (int64_t q = 0; q < n_adc; ++q) {
                double mu[3] = {tk[3 * q] - k_prev[0], tk[3 * q + 1] - k_prev[1], tk[3 * q + 2] - k_prev[2]};
                precess_relax(M, tt[q] - t_prev, mu, x, y, z, dw, m0, t1, t2);
                record(pb, i, signal, sample, M);
                ++sample;
                t_prev = tt[q];
                k_prev[0] = tk[3 * q]; k_prev[1] = tk[3 * q + 1]; k_prev[2] = tk[3 * q + 2];
            }
            double mu[3] = {pb->ev_m[3 * e] - k_prev[0], pb->ev_m[3 * e + 1] - k_prev[1],
                            pb->ev_m[3 * e + 2] - k_prev[2]};
            precess_relax(M, pb->ev_dt[e] - t_prev, mu, x, y, z, dw, m0, t1, t2);
        } else {
            int64_t K = n_adc > 0 ? n_adc : 1;
            double tau = pb->ev_dt[e] / (double)K;
            double mu[3] = {pb->ev_m[3 * e] / (double)K, pb->ev_m[3 * e + 1] / (double)K,
                            pb->ev_m[3 * e + 2] / (double)K};
            for (int64_t k = 0; k < K; ++k) {
                precess_relax(M, tau, mu, x, y, z, dw, m0, t1, t2);
                if (n_adc > 0) {
                    record(pb, i, signal, sample, M);
                    ++sample;
                }
            }
        }
        if (pb->ev_flags[e] & ORACLE_SPOIL) {
            M[0] = 0.0;
            M[1] = 0.0;
        }
        if (pb->ev_flags[e] & ORACLE_SNAPSHOT) {
            if (pb->snap)
                for (int c = 0; c < 3; ++c)
                    pb->snap[(3 * snap + c) * pb->n_spins + i] = M[c];
            ++snap;
        }
    }
    if (final_m) {
        final_m[3 * i] = M[0];
        final_m[3 * i + 1] = M[1];
        final_m[3 * i + 2] = M[2];
    }
}

static void *worker(void *arg)
{
    job_t *j = (job_t *)arg;
    for (int64_t i = j->begin; i < j->end; ++i)
        run_spin(j->pb, i, j->signal, j->final_m);
    return NULL;
}

/* Returns 0 on success, -1 on an invalid argument, -2 on allocation failure.
 * All arrays are host arrays.  out_snap (may be NULL) receives one block of
 * 3 * n_spins doubles per event flagged SNAPSHOT, in event order, laid out
 * [component][spin].  n_coils == 0: one homogeneous coil, out_signal
 * holds 2 * n_samples doubles (interleaved re/im); n_coils >= 1: s_x and
 * s_y hold n_coils * n_spins transverse sensitivities (coil-major) and
 * out_signal holds n_coils blocks of 2 * n_samples.  out_signal and out_final_m (3 * n_spins)
 * may each be NULL. */
int oracle_simulate_traj(int64_t n_spins,
                          const double *x, const double *y, const double *z, const double *m0,
                          const double *t1, const double *t2, const double *dw,
                          int64_t n_events, const double *ev_dt, const double *ev_m,
                          const double *ev_alpha, const double *ev_phase, const int32_t *ev_shape,
                          const int64_t *ev_nadc, const uint32_t *ev_flags,
                          int32_t n_shapes, const int64_t *sh_nsub, const double *sh_tau,
                          const double *sh_m, const int64_t *sh_offset, const double *sh_alpha,
                          const double *sh_phase,
                          int32_t n_coils, const double *s_x, const double *s_y, double *out_snap,
                          const int32_t *ev_traj, int32_t n_traj, const int64_t *tr_n, const int64_t *tr_off,
                          const double *tr_k, const double *tr_t,
                          int n_threads, int64_t n_samples, double *out_signal, double *out_final_m)
{
    if (n_spins < 0 || n_events < 0 || n_samples < 0 || n_threads < 1 || n_coils < 0 || n_traj < 0)
        return -1;
    if (ev_traj)
        for (int64_t e = 0; e < n_events; ++e) {
            if (ev_traj[e] >= n_traj || ev_traj[e] < -1)
                return -1;
            if (ev_traj[e] >= 0) {
                int64_t n = tr_n[ev_traj[e]], off = tr_off[ev_traj[e]];
                if (n != ev_nadc[e])
                    return -1;
                double tp = 0.0;
                for (int64_t q = 0; q < n; ++q) {
                    if (!(tr_t[off + q] >= tp))
                        return -1;
                    tp = tr_t[off + q];
                }
                if (!(ev_dt[e] >= tp))
                    return -1;
            }
        }
    if (n_coils > 0 && n_spins > 0 && (!s_x || !s_y))
        return -1;
    int64_t total = 0;
    for (int64_t e = 0; e < n_events; ++e) {
        if (ev_nadc[e] < 0 || !(ev_dt[e] >= 0.0))
            return -1;
        if (ev_shape[e] >= n_shapes)
            return -1;
        total += ev_nadc[e];
    }
    if (total != n_samples)
        return -1;

    problem_t pb = {x, y, z, m0, t1, t2, dw, n_events, ev_dt, ev_m, ev_alpha, ev_phase,
                    ev_shape, ev_nadc, ev_flags, n_shapes, sh_nsub, sh_offset, sh_tau, sh_m,
                    sh_alpha, sh_phase, n_samples, n_coils, n_spins, s_x, s_y, out_snap,
                    ev_traj, tr_n, tr_off, tr_k, tr_t};
    const int64_t n_vals = 2 * n_samples * (n_coils > 0 ? n_coils : 1);

    if (n_threads > n_spins && n_spins > 0)
        n_threads = (int)n_spins;
    if (n_spins == 0)
        n_threads = 1;
    job_t *jobs = (job_t *)calloc((size_t)n_threads, sizeof(job_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs); free(tid);
        return -2;
    }
    int rc = 0;
    for (int t = 0; t < n_threads; ++t) {
        jobs[t].pb = &pb;
        jobs[t].begin = n_spins * t / n_threads;
        jobs[t].end = n_spins * (t + 1) / n_threads;
        jobs[t].final_m = out_final_m;
        jobs[t].signal = (double *)calloc((size_t)(n_vals + 1), sizeof(double));
        if (!jobs[t].signal)
            rc = -2;
    }
    if (rc == 0) {
        char *started = (char *)calloc((size_t)n_threads, 1);
        for (int t = 1; t < n_threads; ++t) {
            if (started && pthread_create(&tid[t], NULL, worker, &jobs[t]) == 0)
                started[t] = 1;
            else
                worker(&jobs[t]);   /* no thread: run the range here */
        }
        worker(&jobs[0]);
        for (int t = 1; t < n_threads; ++t)
            if (started && started[t])
                pthread_join(tid[t], NULL);
        free(started);
        if (out_signal) {
            memset(out_signal, 0, (size_t)n_vals * sizeof(double));
            for (int t = 0; t < n_threads; ++t)
                for (int64_t s = 0; s < n_vals; ++s)
                    out_signal[s] += jobs[t].signal[s];
        }
    }
    for (int t = 0; t < n_threads; ++t)
        free(jobs[t].signal);
    free(jobs);
    free(tid);
    return rc;
}

/* Without trajectories; see oracle_simulate_traj. */
int oracle_simulate_full(int64_t n_spins,
                         const double *x, const double *y, const double *z, const double *m0,
                         const double *t1, const double *t2, const double *dw,
                         int64_t n_events, const double *ev_dt, const double *ev_m,
                         const double *ev_alpha, const double *ev_phase, const int32_t *ev_shape,
                         const int64_t *ev_nadc, const uint32_t *ev_flags,
                         int32_t n_shapes, const int64_t *sh_nsub, const double *sh_tau,
                         const double *sh_m, const int64_t *sh_offset, const double *sh_alpha,
                         const double *sh_phase,
                         int32_t n_coils, const double *s_x, const double *s_y, double *out_snap,
                         int n_threads, int64_t n_samples, double *out_signal, double *out_final_m)
{
    return oracle_simulate_traj(n_spins, x, y, z, m0, t1, t2, dw, n_events, ev_dt, ev_m, ev_alpha,
                                ev_phase, ev_shape, ev_nadc, ev_flags, n_shapes, sh_nsub, sh_tau,
                                sh_m, sh_offset, sh_alpha, sh_phase, n_coils, s_x, s_y, out_snap,
                                NULL, 0, NULL, NULL, NULL, NULL, n_threads, n_samples, out_signal,
                                out_final_m);
}

/* Signals of receive coils, no snapshots; see oracle_simulate_traj. */
int oracle_simulate_coils(int64_t n_spins,
                          const double *x, const double *y, const double *z, const double *m0,
                          const double *t1, const double *t2, const double *dw,
                          int64_t n_events, const double *ev_dt, const double *ev_m,
                          const double *ev_alpha, const double *ev_phase, const int32_t *ev_shape,
                          const int64_t *ev_nadc, const uint32_t *ev_flags,
                          int32_t n_shapes, const int64_t *sh_nsub, const double *sh_tau,
                          const double *sh_m, const int64_t *sh_offset, const double *sh_alpha,
                          const double *sh_phase,
                          int32_t n_coils, const double *s_x, const double *s_y,
                          int n_threads, int64_t n_samples, double *out_signal, double *out_final_m)
{
    return oracle_simulate_full(n_spins, x, y, z, m0, t1, t2, dw, n_events, ev_dt, ev_m, ev_alpha,
                                ev_phase, ev_shape, ev_nadc, ev_flags, n_shapes, sh_nsub, sh_tau,
                                sh_m, sh_offset, sh_alpha, sh_phase, n_coils, s_x, s_y, NULL,
                                n_threads, n_samples, out_signal, out_final_m);
}

/* The signal of one homogeneous coil, S = (1, 0, 0); see oracle_simulate_full. */
int oracle_simulate(int64_t n_spins,
                    const double *x, const double *y, const double *z, const double *m0,
                    const double *t1, const double *t2, const double *dw,
                    int64_t n_events, const double *ev_dt, const double *ev_m,
                    const double *ev_alpha, const double *ev_phase, const int32_t *ev_shape,
                    const int64_t *ev_nadc, const uint32_t *ev_flags,
                    int32_t n_shapes, const int64_t *sh_nsub, const double *sh_tau,
                    const double *sh_m, const int64_t *sh_offset, const double *sh_alpha,
                    const double *sh_phase,
                    int n_threads, int64_t n_samples, double *out_signal, double *out_final_m)
{
    return oracle_simulate_coils(n_spins, x, y, z, m0, t1, t2, dw, n_events, ev_dt, ev_m, ev_alpha,
                                 ev_phase, ev_shape, ev_nadc, ev_flags, n_shapes, sh_nsub, sh_tau,
                                 sh_m, sh_offset, sh_alpha, sh_phase, 0, NULL, NULL, n_threads,
                                 n_samples, out_signal, out_final_m);
}

/* Single hard pulse applied to one vector, exposed so that tests can compare
 * eq. 3.19 as implemented here with independent rotation formulas. */
void oracle_rf_pulse(double *M, double alpha, double phi)
{
    rf_pulse(M, alpha, phi);
}

/* One free-precession/relaxation interval applied to one vector. */
void oracle_precess_relax(double *M, double tau, const double *mu, double x, double y, double z,
                          double dw, double m0, double t1, double t2)
{
    precess_relax(M, tau, mu, x, y, z, dw, m0, t1, t2);
}
