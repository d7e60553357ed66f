"""Pins of the oracle's receive-coil weighting (section 3.5.1, eq. 3.25) and
of the coil-sensitivity generator.

The weighting follows from eq. 3.25 taken through the steps of eq. 3.28 -
3.31 for a sensitivity with two transverse components: coil c receives
sum_i (S_x Mx + S_y My) + j (S_x My - S_y Mx).  What fixes it here:
  - the homogeneous x coil of section 3.5.2 reproduces the plain sum of
    Mx + j My bit for bit (so the weighting reduces to eq. 3.30 / 3.31);
  - a coil turned by b about z sees every spin turned by -b: its signal is
    exp(-j b) times the x coil's (a y coil: -j times);
  - on the axis of a loop whose normal is z, the sensitivity is parallel to
    the longitudinal magnetisation and nothing is received (the dark regions
    discussed in section 7.1.6);
  - superposition: a multi-coil signal is the per-spin single-spin signals
    summed with each spin's own weights, spin by spin and coil by coil
    (brute force), which pins the indexing of spins and coils;
  - a closed-form FID under an inhomogeneous coil.
"""
import numpy as np
import pytest

import oracle
from workloads import Sequence, coils, configs as C
from workloads.phantom import random_spins


def test_loop_generator_matches_on_axis_closed_form():
    d = np.linspace(-0.3, 0.3, 31)
    for nrm, pos in (([0, 0, 1], lambda t: (0 * t, 0 * t, t)), ([1, 0, 0], lambda t: (t, 0 * t, 0 * t))):
        x, y, z = pos(d)
        s = coils.loop_sensitivity(x, y, z, center=[0, 0, 0], normal=nrm, radius=0.075, n_seg=1024)
        axial = s[int(np.argmax(np.abs(nrm)))]
        np.testing.assert_allclose(axial, coils.loop_on_axis(d, 0.075), rtol=2e-5, atol=1e-9)
        off = [s[k] for k in range(3) if nrm[k] == 0]
        assert max(np.max(np.abs(o)) for o in off) < 1e-12


def test_homogeneous_x_coil_is_the_plain_signal_bitwise():
    obj, seq = C.c2(12)
    plain = oracle.simulate(obj, seq)
    got = oracle.simulate(obj, seq, coils=coils.homogeneous(obj))
    assert got.shape == (1, plain.size)
    np.testing.assert_array_equal(got[0], plain)


def test_turned_coil_turns_the_signal():
    obj = random_spins(300, seed=3, dw_sigma_hz=40.0)
    seq = C.spoiled_gre_2d(16, 4)
    plain = oracle.simulate(obj, seq)
    b = np.array([0.0, np.pi / 2, 0.7, -2.1])
    sx, sy = coils.homogeneous(obj, 4, b)
    sx[1], sy[1] = 0.0, 1.0                                      # exactly the y coil
    got = oracle.simulate(obj, seq, coils=(sx, sy))
    np.testing.assert_array_equal(got[1], -1j * plain)          # y coil: exactly -j
    for c in range(4):
        bb = np.float64(sx[c, 0]) - 1j * np.float64(sy[c, 0])
        np.testing.assert_allclose(got[c], bb * plain, rtol=1e-13, atol=1e-13 * np.abs(plain).max())


def test_spins_on_the_axis_of_a_z_loop_are_not_received():
    n = 64
    rng = np.random.default_rng(9)
    obj = random_spins(n, seed=9)
    obj.x[:] = 0.0
    obj.y[:] = 0.0
    obj.z[:] = rng.uniform(-0.1, 0.1, n).astype(np.float32)
    sx, sy = coils.surface_loop(obj, center=[0, 0, 0.15], normal=[0, 0, 1])
    assert np.max(np.abs(sx)) < 1e-10 and np.max(np.abs(sy)) < 1e-10
    got = oracle.simulate(obj, C.fid(np.pi / 2, 16, 1e-4), coils=(sx, sy))
    assert np.max(np.abs(got)) < 1e-9 * n


def test_superposition_over_spins_and_coils_brute_force():
    obj = random_spins(7, seed=13, dw_sigma_hz=30.0)
    seq = C.spin_echo_2d(8, 3)
    sx, sy = coils.loop_ring(obj, 3, ring_radius=0.2, coil_radius=0.06)
    got = oracle.simulate(obj, seq, coils=(sx, sy))
    want = np.zeros_like(got)
    for i in range(obj.n_spins):
        single = oracle.simulate(obj.take(np.array([i])), seq)
        for c in range(3):
            wx, wy = np.float64(sx[c, i]), np.float64(sy[c, i])
            want[c] += (wx * single.real + wy * single.imag) + 1j * (wx * single.imag - wy * single.real)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_fid_under_a_surface_loop_closed_form():
    """90x then free decay: each spin's Mxy = j m0 e^{-t/T2} e^{-j dw t}, so
    coil c receives sum_i (S_x - j S_y)_i j m0_i e^{-t/T2_i} e^{-j dw_i t}."""
    obj = random_spins(200, seed=17, dw_sigma_hz=25.0)
    n, dwell = 20, 2e-4
    sx, sy = coils.surface_loop(obj, center=[0.0, 0.2, 0.0], normal=[0, 1, 0])
    got = oracle.simulate(obj, C.fid(np.pi / 2, n, dwell), coils=(sx, sy))[0]
    t = dwell * np.arange(1, n + 1)
    m0, t2, dw = (obj.m0.astype(float), obj.t2.astype(float), obj.dw.astype(float))
    w = sx[0].astype(float) - 1j * sy[0].astype(float)
    want = (w[None, :] * 1j * m0 * np.exp(-t[:, None] / t2) * np.exp(-1j * dw * t[:, None])).sum(axis=1)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_coil_shape_errors():
    obj = random_spins(10, seed=1)
    with pytest.raises(ValueError):
        oracle.simulate(obj, C.fid(1.0, 4, 1e-4), coils=(np.ones((2, 9)), np.ones((2, 9))))
