"""Pins of the oracle's magnetisation snapshots (section 7.2): the state of
every spin at the end of each event flagged SNAPSHOT, after a spoiler,
laid out (snapshot, component, spin).  Fixed by closed forms and by the
received signal, which is the spin sum of the same transverse state."""
import math

import numpy as np

import oracle
from workloads import Sequence, SNAPSHOT, SPOIL, configs as C
from workloads.phantom import random_spins


def _f64(a):
    return np.asarray(a, np.float32).astype(np.float64)


def test_free_precession_after_a_90x_pulse():
    """After 90x: M = (0, M0, 0); then Mxy(t) = j M0 e^{-t/T2} e^{-j dw t}
    and Mz(t) = M0 (1 - e^{-t/T1}), at two instants."""
    obj = random_spins(50, seed=5, dw_sigma_hz=60.0)
    seq = Sequence("fid-snap")
    seq.add(1.3e-3, alpha=math.pi / 2, flags=SNAPSHOT)
    seq.add(2.2e-3, flags=SNAPSHOT)
    sig, snap = oracle.simulate(obj, seq, snapshots=True)
    assert sig.size == 0 and snap.shape == (2, 3, 50)
    m0, t1, t2, dw = _f64(obj.m0), _f64(obj.t1), _f64(obj.t2), _f64(obj.dw)
    for k, t in enumerate((1.3e-3, 3.5e-3)):
        mxy = 1j * m0 * np.exp(-t / t2) * np.exp(-1j * dw * t)
        np.testing.assert_allclose(snap[k, 0], mxy.real, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(snap[k, 1], mxy.imag, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(snap[k, 2], m0 * (1 - np.exp(-t / t1)), rtol=1e-12, atol=1e-14)


def test_snapshot_follows_the_spoiler_and_inversion_recovery():
    """180 then TI with SPOIL: Mxy = 0 exactly, Mz = M0 (1 - 2 e^{-TI/T1})."""
    obj = random_spins(40, seed=6)
    ti = 0.4
    seq = Sequence("ir-snap")
    seq.add(ti, alpha=math.pi, flags=SPOIL | SNAPSHOT)
    _, snap = oracle.simulate(obj, seq, snapshots=True)
    m0, t1 = _f64(obj.m0), _f64(obj.t1)
    assert np.all(snap[0, 0] == 0.0) and np.all(snap[0, 1] == 0.0)
    np.testing.assert_allclose(snap[0, 2], m0 * (1 - 2 * np.exp(-ti / t1)), rtol=1e-12, atol=1e-14)


def test_ernst_approach_in_snapshots():
    """Spoiled GRE without gradients: Mz just before the m-th pulse is
    Mz_ss + (M0 - Mz_ss)(E1 cos a)^m (snapshot at the end of each TR)."""
    obj = random_spins(30, seed=7)
    a, tr, te, n_tr = 0.5, 0.02, 0.005, 6
    seq = Sequence("gre-snap")
    for _ in range(n_tr):
        seq.add(te, alpha=a, n_adc=1)
        seq.add(tr - te, flags=SPOIL | SNAPSHOT)
    _, snap = oracle.simulate(obj, seq, snapshots=True)
    m0, t1 = _f64(obj.m0), _f64(obj.t1)
    e1 = np.exp(-tr / t1)
    mss = m0 * (1 - e1) / (1 - e1 * math.cos(a))
    for m in range(n_tr):
        want = mss + (m0 - mss) * (e1 * math.cos(a)) ** (m + 1)
        np.testing.assert_allclose(snap[m, 2], want, rtol=1e-12)


def test_snapshot_sum_is_the_last_sample_of_its_readout():
    """A snapshot at the end of a readout interval holds the state whose spin
    sum is that interval's last sample (the sample is taken after the last
    sub-step), on a full imaging sequence with gradients and shapes."""
    obj, _ = C.c3(8)
    seq = C.gre_3d_sinc(8, 2, 2)
    ev_flags = seq.flags.copy()
    adc = np.nonzero(seq.n_adc > 0)[0]
    seq2 = Sequence("snap-at-adc")
    for sh in seq.shapes:
        seq2.add_shape(sh)
    for e in range(seq.n_events):
        seq2.add(seq.dt[e], m=seq.m[e], alpha=seq.rf_alpha[e], phase=seq.rf_phase[e], shape=int(seq.rf_shape[e]),
                 n_adc=int(seq.n_adc[e]), flags=int(ev_flags[e]) | (SNAPSHOT if e in set(adc) else 0))
    sig, snap = oracle.simulate(obj, seq2, snapshots=True)
    np.testing.assert_array_equal(sig, oracle.simulate(obj, seq))
    ends = np.cumsum(seq.n_adc[adc]) - 1
    for k, n_end in enumerate(ends):
        s = snap[k, 0].sum() + 1j * snap[k, 1].sum()
        assert abs(s - sig[n_end]) <= 1e-12 * max(abs(sig[n_end]), 1e-300) + 1e-15 * obj.m0.sum()


def test_final_snapshot_equals_final_state():
    obj, seq = C.c2(8)
    seq.add(0.01, flags=SNAPSHOT)
    sig, fm, snap = oracle.simulate(obj, seq, final_m=True, snapshots=True)
    np.testing.assert_array_equal(snap[-1].T, fm)
