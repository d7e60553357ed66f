"""Pins of the oracle's per-sample trajectory tables: samples at listed
instants t_s and moments k_s inside an interval (the rest of the interval
runs to dt with the remaining moment).  Fixed by: the equal sub-steps of
section 5.1.1 as a special table, the NUDFT closed form of a spiral after a
90 deg pulse with and without relaxation and off-resonance, and the state
at the interval end seen by a following readout."""
import math

import numpy as np

import oracle
from workloads import Sequence, Trajectory, configs as C
from workloads.phantom import random_spins


def _f64(a):
    return np.asarray(a, np.float32).astype(np.float64)


def spiral(n, k_max, turns, dur):
    """Archimedean spiral, sampled at n instants over dur seconds."""
    u = (np.arange(n) + 1) / n
    r = k_max * u
    th = 2 * math.pi * turns * u
    k = np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n)], axis=1)
    return Trajectory(k=k, t=u * dur)


def test_equal_sub_steps_as_a_table():
    obj = random_spins(200, seed=3, dw_sigma_hz=40.0)
    seq0 = C.spoiled_gre_2d(16, 5)
    seq1 = Sequence("as-table")
    for e in range(seq0.n_events):
        n = int(seq0.n_adc[e])
        tr = -1
        if n:
            s = (np.arange(n) + 1) / n
            tr = seq1.add_trajectory(Trajectory(k=np.outer(s, seq0.m[e]), t=s * seq0.dt[e]))
        seq1.add(seq0.dt[e], m=seq0.m[e], alpha=seq0.rf_alpha[e], phase=seq0.rf_phase[e], n_adc=n,
                 flags=int(seq0.flags[e]), trajectory=tr)
    a, b = oracle.simulate(obj, seq0), oracle.simulate(obj, seq1)
    assert oracle.rel_l2(b, a) < 1e-13


def test_spiral_nudft_closed_form():
    obj = random_spins(300, seed=4)
    n, dur = 400, 8e-3
    tr = spiral(n, 60.0, 5.0, dur)
    for relax in (False, True):
        o = obj.take(np.arange(obj.n_spins))
        if not relax:
            o.t1[:] = np.inf; o.t2[:] = np.inf; o.dw[:] = 0.0
        seq = Sequence("spiral")
        j = seq.add_trajectory(tr)
        seq.add(dur + 1e-3, m=(0, 0, 0), alpha=math.pi / 2, n_adc=n, trajectory=j)
        got = oracle.simulate(o, seq)
        x = np.stack([_f64(o.x), _f64(o.y), _f64(o.z)], axis=1)
        ph = np.exp(-2j * math.pi * (tr.k @ x.T))
        dec = np.exp(-np.outer(tr.t, 1 / _f64(o.t2))) * np.exp(-1j * np.outer(tr.t, _f64(o.dw)))
        want = 1j * np.sum(_f64(o.m0)[None, :] * ph * dec, axis=1)
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())


def test_interval_end_state_after_a_table():
    """A trajectory readout followed by an ordinary readout: the second one
    only sees the end state, which must be that of an interval of the same
    dt and total moment."""
    obj = random_spins(150, seed=5, dw_sigma_hz=30.0)
    tr = spiral(50, 40.0, 2.0, 3e-3)
    m_tot = (12.0, -7.0, 3.0)
    seqs = []
    for use_table in (True, False):
        seq = Sequence("t")
        j = seq.add_trajectory(tr)
        seq.add(5e-3, m=m_tot, alpha=1.0, n_adc=50 if use_table else 0, trajectory=j if use_table else -1)
        seq.add(2e-3, m=(20.0, 0, 0), n_adc=16)
        seqs.append(seq)
    a = oracle.simulate(obj, seqs[0])[50:]
    b = oracle.simulate(obj, seqs[1])
    assert oracle.rel_l2(a, b) < 1e-12
