"""Pins of the K-t configuration oracle (section 4.2) and of the spin-spacing
rules built on it (section 5.2).

The K-t oracle shares no code with the isochromat oracle: it never steps a
spin.  It is pinned by the printed worked example eq. 4.6 (populations term
by term), by exact agreement with the isochromat oracle on random lattice
sequences (the two formulations of the same physics, eq. 4.19), by the
stimulated-echo amplitude, and by the k-space extent of standard
sequences, whose largest configuration orders are known by construction."""
import math

import numpy as np
import pytest

import oracle
from oracle import kt
from workloads import Sequence, Shape, SPOIL, configs as C
from workloads.phantom import SpinObject, random_spins
from tests.test_oracle_pins import _load_eq46, _factor


@pytest.mark.parametrize("a1,a2", [(0.5, 1.1), (np.pi / 2, np.pi / 2), (1.3, -0.7)])
def test_populations_of_the_worked_example_eq_4_6(a1, a2):
    dk = 40.0
    seq = Sequence("eq46")
    seq.add(1e-3, m=(dk, 0, 0), alpha=a1)
    seq.add(1e-3, m=(dk, 0, 0), alpha=a2)
    st = kt.run(seq, (dk, 0, 0), math.inf, math.inf)
    want_f, want_z = {}, {}
    for comp, order, coef, facs in _load_eq46():
        w = coef * np.prod([_factor(t, a1, a2) for t in facs])
        if comp == "Mxy":
            want_f[order] = want_f.get(order, 0) + w
        elif comp == "Mz":
            want_z[order] = want_z.get(order, 0) + w
        else:                                   # Mxy*: order -k holds conj(F(k))
            want_f.setdefault(-order, 0)
            assert abs(np.conj(st.F.get((-order, 0, 0), 0j)) - w) < 1e-12
    for k, w in want_f.items():
        assert abs(st.F.get((k, 0, 0), 0j) - w) < 1e-12, (k, st.F.get((k, 0, 0)), w)
    for k, w in want_z.items():
        assert abs(st.Z.get((k, 0, 0), 0j) - w) < 1e-12
    assert all(abs(v) < 1e-12 for k, v in st.F.items() if k[0] not in want_f)
    assert all(abs(v) < 1e-12 for k, v in st.Z.items() if k[0] not in want_z)


def _random_lattice_sequence(rng, dk, n_events=10):
    seq = Sequence("lattice")
    q_shape = rng.integers(-2, 3, 3) * (np.asarray(dk) > 0)
    seq.add_shape(Shape(tau=2e-5, m_sub=tuple(q_shape * np.asarray(dk)), alpha=rng.uniform(-0.3, 0.3, 6),
                        phase=rng.uniform(-1, 1, 6)))
    for e in range(n_events):
        n_adc = int(rng.choice([0, 0, 3, 8]))
        q = rng.integers(-3, 4, 3) * (np.asarray(dk) > 0)
        if n_adc:
            q = q * n_adc                            # every sample a lattice step
        seq.add(float(rng.uniform(1e-4, 3e-3)), m=tuple(q * np.asarray(dk)),
                alpha=float(rng.choice([0.0, rng.uniform(0.1, 3.0)])), phase=float(rng.uniform(-3, 3)),
                shape=0 if rng.uniform() < 0.2 else -1, n_adc=n_adc,
                flags=SPOIL if rng.uniform() < 0.15 else 0)
    seq.add(1e-3, alpha=0.7, n_adc=4)
    return seq


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_agrees_with_the_isochromat_oracle(seed):
    """Same tissue for every spin, arbitrary positions and weights: the
    configuration series (eq. 4.19) and the spin-by-spin stepping give the
    same signal."""
    rng = np.random.default_rng(seed)
    dk = (37.0, 23.0, 0.0 if seed % 2 else 11.0)
    seq = _random_lattice_sequence(rng, dk)
    n = 40
    # tissue values as the object stores them (float32)
    t1, t2, dw = (float(np.float32(v)) for v in (0.8, 0.09, rng.normal(0, 200.0)))
    base = random_spins(n, seed=seed)
    obj = SpinObject(x=base.x, y=base.y, z=base.z if dk[2] else np.zeros(n), m0=base.m0,
                     t1=np.full(n, t1), t2=np.full(n, t2), dw=np.full(n, dw))
    got = kt.signal(obj, seq, dk, t1, t2, dw)
    ref = oracle.simulate(obj, seq)
    assert got.shape == ref.shape and ref.size > 0
    assert oracle.rel_l2(got, ref) < 1e-11


def test_stimulated_echo_amplitude():
    """Three pulses a1, a2, a3 with gradient dk before and after the middle
    interval: the stimulated echo at order 0 after the third interval has
    |F(0)| = 1/2 sin a1 sin a2 sin a3 E2(tau1) E1(tau2) E2(tau3), tau3 = tau1."""
    a = (1.1, 0.8, 1.4)
    t1, t2 = 0.9, 0.07
    tau1, tau2 = 4e-3, 30e-3
    seq = Sequence("ste")
    seq.add(tau1, m=(1.0, 0, 0), alpha=a[0])
    seq.add(tau2, alpha=a[1], flags=SPOIL)
    seq.add(tau1, m=(1.0, 0, 0), alpha=a[2])
    st = kt.run(seq, (1.0, 0, 0), t1, t2)
    want = 0.5 * math.sin(a[0]) * math.sin(a[1]) * math.sin(a[2]) * math.exp(-2 * tau1 / t2) * math.exp(-tau2 / t1)
    assert abs(abs(st.F.get((0, 0, 0), 0j)) - want) < 1e-13


def test_extent_of_standard_sequences():
    """Cartesian GRE / SE with Delta k = 1/FOV: the prephaser reaches
    -(N/2 + 1) in x and the encodes reach -n_pe/2 in y; SPOIL before every
    pulse keeps Z at order 0."""
    fov = C.FOV
    for seq in (C.spoiled_gre_2d(32, 12), C.spin_echo_2d(32, 12)):
        k = kt.extent(seq, (1 / fov, 1 / fov, 0.0), 1.0, 0.1)
        np.testing.assert_allclose(k, [17 / fov, 6 / fov, 0.0])
        np.testing.assert_allclose(kt.max_spacing(k)[:2], [fov / 34, fov / 12])
        assert np.isinf(kt.max_spacing(k)[2])


def test_extent_grows_without_spoiling_and_pruning_bounds_it():
    """A gradient-spoiled steady-state GRE (section 5.2.4): every TR moves
    all configurations one step further, so the unpruned K_max grows with
    the number of TRs, while the populations of the outer ones decay; with
    eq. 5.4 / 5.5 (Delta rho = 1/256) the pruned extent stays small."""
    seq = Sequence("ssfp-like")
    for _ in range(60):
        seq.add(2e-3, alpha=0.3, n_adc=1)
        seq.add(6e-3, m=(1.0, 0, 0))
    full = kt.extent(seq, (1.0, 0, 0), 0.5, 0.02)
    pruned = kt.extent(seq, (1.0, 0, 0), 0.5, 0.02, grey_step=1 / 256)
    finer = kt.extent(seq, (1.0, 0, 0), 0.5, 0.02, grey_step=1 / 4096)
    assert full[0] == 60
    assert 1 <= pruned[0] < finer[0] < 40
