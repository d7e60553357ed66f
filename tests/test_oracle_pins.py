"""Pins of the FP64 oracle against facts that do not come from the oracle:
printed results of the paper, closed forms of MR physics, library routines
(matrix exponential, FFT, Bessel function, rotation library), invariants and
brute force on tiny inputs.  A plausible slip in the oracle (a dropped term,
a wrong sign, a swapped index, a transposed matrix) fails at least one of
these.  CPU only.
"""
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.spatial.transform import Rotation
from scipy.special import j1

import oracle
from workloads import Sequence, Shape, SPOIL, configs as C
from workloads.phantom import SpinObject, grid2d, single_spin, uniform_disc, random_spins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EXACT = 1e-12


def _rand_vec(rng, n=3):
    return rng.normal(size=n)


# --------------------------------------------------------------------------
# RF operator, eq. 3.19
# --------------------------------------------------------------------------
def test_rf_equals_rotation_by_minus_alpha_about_phase_axis():
    """eq. 3.19 is a rotation by -alpha (clockwise) about (cos phi, sin phi, 0):
    compared with scipy's independent rotation-vector implementation."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        a = rng.uniform(-2 * np.pi, 2 * np.pi)
        p = rng.uniform(-np.pi, np.pi)
        M = _rand_vec(rng)
        axis = np.array([math.cos(p), math.sin(p), 0.0])
        ref = Rotation.from_rotvec(-a * axis).apply(M)
        np.testing.assert_allclose(oracle.rf_pulse(M, a, p), ref, rtol=0, atol=EXACT)


def test_rf_equals_expm_of_rotating_frame_generator():
    """On resonance and without relaxation, eq. A.14/A.12 give
    dM'/dt = G M' with G = gamma B1 [[0,0,-sin phi],[0,0,cos phi],
    [sin phi,-cos phi,0]]; its flow over alpha/(gamma B1) is eq. 3.19."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        a = rng.uniform(0, 2 * np.pi)
        p = rng.uniform(-np.pi, np.pi)
        sp, cp = math.sin(p), math.cos(p)
        G = np.array([[0, 0, -sp], [0, 0, cp], [sp, -cp, 0]])
        R = expm(a * G)
        M = _rand_vec(rng)
        np.testing.assert_allclose(oracle.rf_pulse(M, a, p), R @ M, rtol=0, atol=EXACT)


def test_rf_special_cases_and_invariants():
    # 90 deg about x' tips +z onto +y: Mxy = +j M0 (rotation sense of eq. 3.19)
    np.testing.assert_allclose(oracle.rf_pulse([0, 0, 1], np.pi / 2, 0.0), [0, 1, 0], atol=EXACT)
    # 180 deg about y' maps (Mx, My, Mz) -> (-Mx, My, -Mz)
    M = np.array([0.3, -0.7, 0.2])
    np.testing.assert_allclose(oracle.rf_pulse(M, np.pi, np.pi / 2), [-M[0], M[1], -M[2]], atol=EXACT)
    # full turn is the identity; same-axis pulses add; |M| is preserved
    rng = np.random.default_rng(3)
    for _ in range(50):
        M = _rand_vec(rng)
        p = rng.uniform(-np.pi, np.pi)
        a, b = rng.uniform(-3, 3, 2)
        np.testing.assert_allclose(oracle.rf_pulse(M, 2 * np.pi, p), M, atol=EXACT)
        np.testing.assert_allclose(oracle.rf_pulse(oracle.rf_pulse(M, a, p), b, p),
                                   oracle.rf_pulse(M, a + b, p), atol=EXACT)
        assert abs(np.linalg.norm(oracle.rf_pulse(M, a, p)) - np.linalg.norm(M)) < EXACT


def test_rf_complex_form_eq_4_2():
    """The complex-magnetisation operator of eq. 4.2 acting on
    (Mxy, Mxy*, Mz) agrees with the real operator of eq. 3.19."""
    rng = np.random.default_rng(4)
    for _ in range(100):
        a = rng.uniform(-3, 3)
        p = rng.uniform(-np.pi, np.pi)
        c2, s2 = math.cos(a / 2) ** 2, math.sin(a / 2) ** 2
        T = np.array([
            [c2, s2 * np.exp(2j * p), math.sin(a) * np.exp(1j * (p + np.pi / 2))],
            [s2 * np.exp(-2j * p), c2, math.sin(a) * np.exp(-1j * (p + np.pi / 2))],
            [math.sin(a) / 2 * np.exp(-1j * (p - np.pi / 2)),
             math.sin(a) / 2 * np.exp(1j * (p - np.pi / 2)), math.cos(a)]])
        M = _rand_vec(rng)
        mxy = M[0] + 1j * M[1]
        out = T @ np.array([mxy, np.conj(mxy), M[2]])
        got = oracle.rf_pulse(M, a, p)
        assert abs(out[0] - (got[0] + 1j * got[1])) < EXACT
        assert abs(out[1] - (got[0] - 1j * got[1])) < EXACT
        assert abs(out[2] - got[2]) < EXACT


# --------------------------------------------------------------------------
# free precession + relaxation, eq. 3.5 / 3.14, against eq. A.2-A.4
# --------------------------------------------------------------------------
def test_interval_equals_expm_of_augmented_bloch_generator():
    """The interval operator solves dM/dt = A M + f (eq. A.2) with A from
    eq. A.3 for a pure z field (B = (0, 0, Bz), gamma Bz tau = theta) and
    f = (0, 0, M0/T1) (eq. A.4): compared with expm of the 4x4 augmented
    generator [[A, f], [0, 0]]."""
    rng = np.random.default_rng(5)
    for _ in range(100):
        tau = rng.uniform(1e-5, 0.05)
        t1 = rng.uniform(0.05, 3.0)
        t2 = rng.uniform(0.01, 1.0)
        m0 = rng.uniform(0.1, 2.0)
        mu = rng.normal(scale=50.0, size=3)
        x, y, z = rng.uniform(-0.1, 0.1, 3)
        dw = rng.normal(scale=300.0)
        theta = 2 * np.pi * (mu[0] * x + mu[1] * y + mu[2] * z) + dw * tau
        gbz = theta / tau
        A = np.array([[-1 / t2, gbz, 0.0], [-gbz, -1 / t2, 0.0], [0.0, 0.0, -1 / t1]])
        aug = np.zeros((4, 4))
        aug[:3, :3] = A
        aug[2, 3] = m0 / t1
        M = _rand_vec(rng)
        ref = (expm(aug * tau) @ np.append(M, 1.0))[:3]
        got = oracle.precess_relax(M, tau, mu, x, y, z, dw, m0, t1, t2)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_interval_without_relaxation_matches_eq_3_26():
    """T1 = T2 = inf: pure clockwise precession (eq. 3.26/3.27)."""
    rng = np.random.default_rng(6)
    M = _rand_vec(rng)
    dw, tau = 123.0, 0.01
    got = oracle.precess_relax(M, tau, [0, 0, 0], 0, 0, 0, dw, 1.0, np.inf, np.inf)
    w = dw * tau
    ref = [M[0] * math.cos(w) + M[1] * math.sin(w), -M[0] * math.sin(w) + M[1] * math.cos(w), M[2]]
    np.testing.assert_allclose(got, ref, atol=EXACT)


# --------------------------------------------------------------------------
# the printed worked example, eq. 4.6
# --------------------------------------------------------------------------
def _load_eq46():
    rows = []
    with open(os.path.join(GOLDEN, "eq4_6_two_pulse.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            comp, order, coef = parts[0], int(parts[1]), complex(parts[2])
            rows.append((comp, order, coef, parts[3:]))
    return rows


def _factor(tok, a1, a2):
    power = 1
    if tok.endswith("^2"):
        tok, power = tok[:-2], 2
    table = {"sin(a1)": math.sin(a1), "cos(a1)": math.cos(a1), "sin(a2)": math.sin(a2),
             "cos(a2)": math.cos(a2), "sin(a2/2)": math.sin(a2 / 2), "cos(a2/2)": math.cos(a2 / 2)}
    return table[tok] ** power


@pytest.mark.parametrize("a1,a2", [(0.5, 1.1), (np.pi / 2, np.pi / 2), (1.3, -0.7), (2.5, 0.2)])
def test_worked_example_eq_4_6(a1, a2):
    rows = _load_eq46()
    assert len(rows) == 9
    dk = 40.0                       # cycles/m per gradient interval
    xs = np.linspace(-0.05, 0.05, 11)
    seq = Sequence("eq46")
    seq.add(1e-3, m=(dk, 0, 0), alpha=a1, phase=0.0)
    seq.add(1e-3, m=(dk, 0, 0), alpha=a2, phase=0.0)
    obj = SpinObject(x=xs, y=np.zeros(11), z=np.zeros(11), m0=np.ones(11),
                     t1=np.full(11, np.inf), t2=np.full(11, np.inf), dw=np.zeros(11))
    _, fm = oracle.simulate(obj, seq, final_m=True)
    xs32 = obj.x.astype(np.float64)
    for i, x in enumerate(xs32):
        comp = {"Mxy": 0j, "Mxy*": 0j, "Mz": 0j}
        for name, order, coef, factors in rows:
            w = coef
            for tok in factors:
                w *= _factor(tok, a1, a2)
            comp[name] += w * np.exp(-order * 2j * np.pi * dk * x)
        mxy = fm[i, 0] + 1j * fm[i, 1]
        assert abs(comp["Mxy"] - mxy) < 1e-12
        assert abs(comp["Mxy*"] - np.conj(mxy)) < 1e-12
        assert abs(comp["Mz"] - fm[i, 2]) < 1e-12


# --------------------------------------------------------------------------
# closed forms of whole sequences
# --------------------------------------------------------------------------
def test_fid_decay_and_off_resonance_phase():
    """After 90x: s(t) = j m0 exp(-t/T2) exp(-j dw t), samples at the end of
    each sub-step (section 5.1.1); pins the sign of dw."""
    obj = random_spins(37, seed=7)
    n, dwell = 50, 1e-3
    seq = C.fid(np.pi / 2, n, dwell)
    sig = oracle.simulate(obj, seq)
    t = (np.arange(n) + 1) * dwell
    m0, t2, dw = (obj.m0.astype(float), obj.t2.astype(float), obj.dw.astype(float))
    ref = (1j * m0[None, :] * np.exp(-t[:, None] / t2[None, :]) *
           np.exp(-1j * dw[None, :] * t[:, None])).sum(axis=1)
    np.testing.assert_allclose(sig, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_readout_gradient_phase_sign():
    """A readout gradient of moment mu per sample gives s_n = j m0 exp(-2 pi j k_n x),
    k_n = (n+1) mu (eq. 3.17 / 3.33 sign)."""
    x = np.array([0.013, -0.041, 0.002])
    obj = SpinObject(x=x, y=np.zeros(3), z=np.zeros(3), m0=np.ones(3), t1=np.full(3, np.inf),
                     t2=np.full(3, np.inf), dw=np.zeros(3))
    n, mu = 32, 7.5
    seq = Sequence("ro")
    seq.add(n * 1e-5, m=(n * mu, 0, 0), alpha=np.pi / 2, n_adc=n)
    sig = oracle.simulate(obj, seq)
    k = (np.arange(n) + 1) * mu
    ref = (1j * np.exp(-2j * np.pi * k[:, None] * obj.x.astype(float)[None, :])).sum(axis=1)
    np.testing.assert_allclose(sig, ref, atol=1e-12)


def test_spin_echo_amplitude_independent_of_off_resonance():
    """90x - TE/2 - 180y - TE/2: echo = j m0 exp(-TE/T2) for every dw."""
    rng = np.random.default_rng(8)
    te, n, dwell = 40e-3, 16, 1e-4
    seq = C.spin_echo_single(te, n, dwell)
    for _ in range(5):
        dw = rng.normal(scale=2 * np.pi * 100)
        t2 = rng.uniform(0.02, 0.3)
        obj = single_spin(m0=0.8, t1=1.0, t2=t2, dw=dw)
        sig = oracle.simulate(obj, seq)
        echo = sig[n // 2]
        ref = 1j * float(obj.m0[0]) * math.exp(-te / float(obj.t2[0]))
        assert abs(echo - ref) < 1e-12


def test_spin_echo_repeated_with_spoiling():
    """TR >= 2 of spoiled SE: echo = j m0 [1 - 2 E1(TR - TE/2) + E1(TR)] E2(TE)."""
    te, tr, n, dwell = 30e-3, 300e-3, 8, 1e-4
    seq = C.spin_echo_single(te, n, dwell, tr=tr, n_tr=4)
    obj = single_spin(m0=1.0, t1=0.7, t2=0.1, dw=2 * np.pi * 37)
    sig = oracle.simulate(obj, seq).reshape(4, n)
    t1, t2 = float(obj.t1[0]), float(obj.t2[0])
    assert abs(sig[0, n // 2] - 1j * math.exp(-te / t2)) < 1e-12
    ss = 1 - 2 * math.exp(-(tr - te / 2) / t1) + math.exp(-tr / t1)
    for r in range(1, 4):
        assert abs(sig[r, n // 2] - 1j * ss * math.exp(-te / t2)) < 1e-12


def test_spoiled_gre_ernst_approach_to_steady_state():
    """Mz before pulse m: Mz_ss + (m0 - Mz_ss)(E1 cos a)^m with
    Mz_ss = m0 (1 - E1) / (1 - E1 cos a); signal j sin a Mz_m E2(TE) e^{-j dw TE}."""
    a, tr, te, n_tr = 0.4, 12e-3, 4e-3, 60
    seq = C.spoiled_gre_probe(a, tr, te, n_tr)
    obj = single_spin(m0=0.9, t1=0.8, t2=0.05, dw=2 * np.pi * 13)
    sig = oracle.simulate(obj, seq)
    m0, t1, t2, dw = (float(obj.m0[0]), float(obj.t1[0]), float(obj.t2[0]), float(obj.dw[0]))
    e1 = math.exp(-tr / t1)
    mss = m0 * (1 - e1) / (1 - e1 * math.cos(a))
    m = np.arange(n_tr)
    mz = mss + (m0 - mss) * (e1 * math.cos(a)) ** m
    ref = 1j * math.sin(a) * mz * math.exp(-te / t2) * np.exp(-1j * dw * te)
    np.testing.assert_allclose(sig, ref, rtol=0, atol=1e-12)


def _widen(obj):
    return tuple(np.asarray(a, dtype=float) for a in (obj.x, obj.y, obj.m0, obj.t1, obj.t2, obj.dw))


def test_whole_c1_output_closed_form():
    """Every sample of the c1 workload (64^2 spins, 64 spoiled-GRE
    repetitions of 64 samples) in closed form: before pulse m,
    Mz_{m+1} = m0 + (cos a Mz_m - m0) E1(TR) (spoiled, so Mxy starts at zero);
    sample n of repetition m is j sin a Mz_m E2(t_n) e^{-j(2 pi k.x + dw t_n)}
    with t_n = TE + (n - N/2) dwell and k = ((n - N/2) / FOV, (m - M/2) / FOV)
    (eq. 3.19 as a rotation by -a about x, eq. 3.5 / 3.14 / 3.33).  Built from
    the recipe's parameters, not from its event list."""
    obj, seq = C.c1()
    md = seq.meta
    n_ro, n_pe, fov, tr, te, dwell, a = (md["n_read"], md["n_pe"], md["fov"], md["tr"], md["te"],
                                         md["dwell"], md["alpha"])
    x, y, m0, t1, t2, dw = _widen(obj)
    sig = oracle.simulate(obj, seq).reshape(n_pe, n_ro)
    t = te + (np.arange(n_ro) - n_ro // 2) * dwell
    kx = (np.arange(n_ro) - n_ro // 2) / fov
    e2 = np.exp(-t[:, None] / t2[None, :])
    mz = m0.copy()
    worst = 0.0
    for m in range(n_pe):
        ky = (m - n_pe // 2) / fov
        ph = 2 * np.pi * (kx[:, None] * x[None, :] + ky * y[None, :]) + dw[None, :] * t[:, None]
        ref = (1j * math.sin(a) * mz[None, :] * e2 * np.exp(-1j * ph)).sum(axis=1)
        worst = max(worst, np.abs(sig[m] - ref).max() / np.abs(ref).max())
        mz = m0 + (math.cos(a) * mz - m0) * np.exp(-tr / t1)
    assert worst < EXACT, worst


def test_whole_c2_recipe_output_closed_form():
    """Every sample of the c2 recipe at 64^2 x 4 jittered isochromats with
    off-resonance: 90x makes j Mz_m; TE/2 of free precession; 180y turns
    Mxy into -conj(Mxy), so Mxy = j Mz_m E2(TE/2) e^{+j dw TE/2}; sample n
    then lies t_n = TE/2 + (n - N/2) dwell after the 180 with
    k = ((n - N/2) / FOV, (m - M/2) / FOV).  Mz before the 90 is m0 for the
    first repetition and m0 [1 - 2 E1(TR - TE/2) + E1(TR)] after it."""
    obj, seq = C.c2(64)
    md = seq.meta
    n_ro, n_pe, fov, tr, te, dwell = (md["n_read"], md["n_pe"], md["fov"], md["tr"], md["te"], md["dwell"])
    x, y, m0, t1, t2, dw = _widen(obj)
    sig = oracle.simulate(obj, seq).reshape(n_pe, n_ro)
    t = te / 2 + (np.arange(n_ro) - n_ro // 2) * dwell
    kx = (np.arange(n_ro) - n_ro // 2) / fov
    before = np.exp(-(te / 2) / t2) * np.exp(1j * dw * te / 2)
    decay = np.exp(-t[:, None] / t2[None, :])
    mz_ss = m0 * (1 - 2 * np.exp(-(tr - te / 2) / t1) + np.exp(-tr / t1))
    worst = 0.0
    for m in range(n_pe):
        mz = m0 if m == 0 else mz_ss
        ky = (m - n_pe // 2) / fov
        ph = 2 * np.pi * (kx[:, None] * x[None, :] + ky * y[None, :]) + dw[None, :] * t[:, None]
        ref = (1j * (mz * before)[None, :] * decay * np.exp(-1j * ph)).sum(axis=1)
        worst = max(worst, np.abs(sig[m] - ref).max() / np.abs(ref).max())
    assert worst < EXACT, worst


def test_inversion_recovery_null_at_t1_ln2():
    t1 = 0.9
    for ti, expect in [(t1 * math.log(2), 0.0), (0.3, None), (2.0, None)]:
        obj = single_spin(m0=1.0, t1=t1, t2=0.1)
        sig = oracle.simulate(obj, C.inversion_recovery(ti))
        ref = 1.0 - 2 * math.exp(-ti / float(obj.t1[0]))
        assert abs(sig[0] - 1j * ref) < 1e-12
        if expect is not None:
            assert abs(sig[0]) < 1e-7


def test_cartesian_encoding_is_exactly_the_shifted_fft():
    """T2 = inf, dw = 0, full recovery each TR, 90 deg spoiled GRE on a voxel-
    centre grid: s(ky_m, kx_n) = j sum m0 exp(-2 pi j k.x) (eq. 3.33), which on
    these grids is fftshift(fft2(ifftshift(rho)))."""
    n = 16
    obj = grid2d(n, C.FOV, 1, seed=11)
    obj.t1[:] = 1e-9          # full recovery within every TR
    obj.t2[:] = np.inf
    seq = C.spoiled_gre_2d(n, n, alpha_deg=90.0)
    sig = oracle.simulate(obj, seq).reshape(n, n)
    rho = obj.m0.astype(np.float64).reshape(n, n)
    ref = 1j * np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(rho)))
    np.testing.assert_allclose(sig, ref, rtol=0, atol=1e-10)


def test_uniform_disc_approaches_jinc():
    """Continuum limit: a uniform disc of radius R (rho = 1, spins on a grid of
    spacing d with m0 = d^2) excited by 90x gives s(k) -> j R J1(2 pi k R) / k
    (k in cycles/m).  Staircase error is O(d / R); tolerance 2e-2 of pi R^2."""
    R, d = 0.05, 0.05 / 64
    obj = uniform_disc(R, d)
    n, kmax = 64, 8 / R
    seq = Sequence("disc")
    mu = kmax / n
    seq.add(n * 1e-6, m=(n * mu, 0, 0), alpha=np.pi / 2, n_adc=n)
    sig = oracle.simulate(obj, seq)
    k = (np.arange(n) + 1) * mu
    ref = 1j * R * j1(2 * np.pi * k * R) / k
    err = np.max(np.abs(sig - ref)) / (np.pi * R * R)
    assert err < 2e-2, err


@pytest.mark.parametrize("n_iso,expect_echo", [(1, False), (2, False), (3, True), (4, True), (7, True)])
def test_two_pulse_echo_and_spatial_sampling_criterion(n_iso, expect_echo):
    """Two 90x pulses each followed by a gradient of moment dk: the echo at
    the end is -j/2 N m0 when N isochromats sample one period 1/dk finely
    enough (N >= 3, criterion eq. 5.2), and collapses to 0 for N <= 2."""
    dk = 25.0
    x = np.arange(n_iso) / (n_iso * dk)
    obj = SpinObject(x=x, y=np.zeros(n_iso), z=np.zeros(n_iso), m0=np.ones(n_iso),
                     t1=np.full(n_iso, np.inf), t2=np.full(n_iso, np.inf), dw=np.zeros(n_iso))
    seq = Sequence("hahn")
    seq.add(1e-3, m=(dk, 0, 0), alpha=np.pi / 2)
    seq.add(1e-3, m=(dk, 0, 0), alpha=np.pi / 2, n_adc=1)
    xs = obj.x.astype(np.float64)
    sig = oracle.simulate(obj, seq)[0]
    # brute-force reference from the configuration sum (eq. 4.6 at 90/90)
    brute = np.sum(0.5j * np.exp(-2j * 2 * np.pi * dk * xs) - 0.5j)
    assert abs(sig - brute) < 1e-12
    if expect_echo:
        assert abs(sig - (-0.5j * n_iso)) < 1e-5
    else:
        assert abs(sig) < 1e-12 or abs(sig - (-0.5j * n_iso)) > 0.1


def test_shaped_pulse_on_resonance_composes_to_one_rotation():
    """No gradient, dw = 0, no relaxation, constant phase: the sub-pulses of
    eq. 3.23 add up to one hard pulse of the summed flip angle."""
    rng = np.random.default_rng(12)
    alpha = rng.uniform(-0.2, 0.4, 40)
    p0 = 0.7
    shp = Shape(tau=1e-5, m_sub=(0, 0, 0), alpha=alpha, phase=np.zeros(40))
    seq = Sequence("shape")
    sid = seq.add_shape(shp)
    seq.add(0.0, shape=sid, phase=p0)
    M = np.array([0.2, -0.5, 0.8])
    obj = single_spin()
    # start from equilibrium: compare M0 = (0, 0, 1)
    _, fm = oracle.simulate(obj, seq, final_m=True)
    ref = Rotation.from_rotvec(-alpha.sum() * np.array([math.cos(p0), math.sin(p0), 0])).apply([0, 0, 1])
    np.testing.assert_allclose(fm[0], ref, atol=1e-12)
    del M


def test_small_tip_slab_profile_is_fourier_transform_of_envelope():
    """Small flip (5 deg) sinc with slab gradient and rephaser: the excited
    Mxy(z) follows eq. 3.22, here j sum_i alpha_i exp(-2 pi j ((N-1)/2 - i) mu z),
    up to O(alpha^3)."""
    n_rf, tau = 64, 20e-6
    shp = C.sinc_shape(n_rf, tau, 5 * C.DEG, 4.0, 0.1)
    mu = shp.m_sub[2]
    seq = Sequence("slab")
    sid = seq.add_shape(shp)
    seq.add(0.0, m=(0, 0, -(n_rf - (n_rf - 1) / 2) * mu), shape=sid)
    zs = np.linspace(-0.12, 0.12, 97)
    nz = zs.size
    obj = SpinObject(x=np.zeros(nz), y=np.zeros(nz), z=zs, m0=np.ones(nz),
                     t1=np.full(nz, np.inf), t2=np.full(nz, np.inf), dw=np.zeros(nz))
    _, fm = oracle.simulate(obj, seq, final_m=True)
    mxy = fm[:, 0] + 1j * fm[:, 1]
    i = np.arange(n_rf)
    z32 = obj.z.astype(np.float64)
    ref = 1j * (shp.alpha[None, :] * np.exp(-2j * np.pi * ((n_rf - 1) / 2 - i)[None, :] * mu
                                            * z32[:, None])).sum(axis=1)
    assert np.max(np.abs(mxy - ref)) < 1e-2 * 5 * C.DEG
    # at z = 0 the slab gradient adds no phase: the sub-pulses compose exactly
    i0 = int(np.argmin(np.abs(z32)))
    assert z32[i0] == 0.0
    assert abs(mxy[i0] - 1j * math.sin(shp.alpha.sum())) < 1e-12
    # well outside the slab almost nothing is excited
    assert np.max(np.abs(mxy[np.abs(z32) > 0.09])) < 0.2 * math.sin(5 * C.DEG)


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------
def test_superposition_linearity_and_permutation():
    obj = random_spins(301, seed=13)
    _, seq = C.c1()
    seq = seq.truncated(12)
    s_all = oracle.simulate(obj, seq, n_threads=3)
    a = obj.take(np.arange(0, 150)); b = obj.take(np.arange(150, 301))
    s_ab = oracle.simulate(a, seq) + oracle.simulate(b, seq)
    np.testing.assert_allclose(s_all, s_ab, rtol=0, atol=1e-12 * np.abs(s_all).max())
    perm = np.random.default_rng(0).permutation(301)
    s_p = oracle.simulate(obj.take(perm), seq, n_threads=5)
    np.testing.assert_allclose(s_all, s_p, rtol=0, atol=1e-12 * np.abs(s_all).max())
    obj2 = obj.take(np.arange(301)); obj2.m0 = (obj2.m0 * 2).astype(np.float32)
    np.testing.assert_allclose(oracle.simulate(obj2, seq), 2 * s_all, rtol=0,
                               atol=1e-12 * np.abs(s_all).max())


def test_spoil_flag_clears_transverse_only():
    obj = single_spin(m0=1.0, t1=0.5, t2=0.2)
    seq = Sequence("sp")
    seq.add(0.01, alpha=0.6, flags=SPOIL)
    _, fm = oracle.simulate(obj, seq, final_m=True)
    e1 = math.exp(-0.01 / float(obj.t1[0]))
    assert fm[0, 0] == 0.0 and fm[0, 1] == 0.0
    assert abs(fm[0, 2] - (e1 * math.cos(0.6) + 1 - e1)) < 1e-12


def test_empty_inputs():
    obj = random_spins(5, seed=1)
    assert oracle.simulate(obj, Sequence("empty")).shape == (0,)
    empty = obj.take(np.arange(0))
    sig = oracle.simulate(empty, C.fid(1.0, 4, 1e-3))
    assert sig.shape == (4,) and np.all(sig == 0)


def test_regression_metric_matches_paper_definition():
    """Noise distance (section 5.4.2) is 20 log10 of the relative L2 error."""
    ref = np.array([1 + 1j, 2 - 1j, 0.5j])
    test = ref + np.array([1e-5, -2e-5j, 1e-5])
    de = oracle.stoerabstand_db(test, ref)
    direct = 10 * math.log10(np.sum(np.abs(ref - test) ** 2) / np.sum(np.abs(ref) ** 2))
    assert abs(de - direct) < 1e-9
    assert oracle.count_over_threshold(test, ref, 1e-4) == 0
    assert oracle.count_over_threshold(test, ref, 1e-6) >= 1
