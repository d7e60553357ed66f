"""Checks of the synthetic workload generators (CPU only): sample counts,
k-space position and time of every sample obtained by integrating the
moments of the event table, TE placement, the RF sampling condition
(eq. B.5) of the sinc pulse, and determinism of the seeded draws."""
import math

import numpy as np
import pytest

from workloads import configs as C, SPOIL
from workloads.phantom import grid2d, grid3d_two_species


def _sample_k_and_t(seq):
    """Integrate moments and durations: k (cycles/m) and time of each sample,
    k reset to 0 by every excitation (hard pulse of any angle or shape)."""
    ks, ts = [], []
    k = np.zeros(3)
    t = 0.0
    t_exc = 0.0
    for e in range(seq.n_events):
        sh = int(seq.rf_shape[e])
        if sh >= 0:
            shp = seq.shapes[sh]
            t_exc = t + (shp.n_sub - 1) * shp.tau / 2      # pulse centre
            k = shp.m_sub * (shp.n_sub - (shp.n_sub - 1) / 2)
            t += shp.n_sub * shp.tau
        a = seq.rf_alpha[e]
        if abs(a - math.pi / 2) < 1e-12 or (0 < abs(a) < math.pi - 1e-9):
            k = np.zeros(3); t_exc = t
        elif abs(a - math.pi) < 1e-12:
            k = -k
        n = int(seq.n_adc[e])
        K = max(n, 1)
        for j in range(K):
            k = k + seq.m[e] / K
            t += seq.dt[e] / K
            if n:
                ks.append(k.copy()); ts.append(t - t_exc)
        if seq.flags[e] & SPOIL:
            k = np.zeros(3)
    return np.array(ks), np.array(ts)


def test_c1_counts_kspace_and_te():
    obj, seq = C.c1()
    assert obj.n_spins == 4096
    assert seq.n_events == 192 and seq.n_samples == 4096 and seq.n_steps_per_spin == 4224
    k, t = _sample_k_and_t(seq)
    k = k.reshape(64, 64, 3)
    n = np.arange(64)
    np.testing.assert_allclose(k[:, :, 0], np.broadcast_to((n - 32) / C.FOV, (64, 64)), atol=1e-9)
    np.testing.assert_allclose(k[:, :, 1], np.broadcast_to(((n - 32) / C.FOV)[:, None], (64, 64)), atol=1e-9)
    np.testing.assert_allclose(t.reshape(64, 64)[:, 32], 5e-3, atol=1e-12)
    assert abs(seq.dt.reshape(64, 3).sum(axis=1) - 10e-3).max() < 1e-12


def test_c2_counts_kspace_and_te():
    obj, seq = C.c2()
    assert obj.n_spins == 262144
    assert seq.n_events == 1024 and seq.n_samples == 65536 and seq.n_steps_per_spin == 66304
    k, t = _sample_k_and_t(seq)
    k = k.reshape(256, 256, 3)
    n = np.arange(256)
    np.testing.assert_allclose(k[0, :, 0], (n - 128) / C.FOV, atol=1e-9)
    np.testing.assert_allclose(k[:, 0, 1], (n - 128) / C.FOV, atol=1e-9)
    np.testing.assert_allclose(t.reshape(256, 256)[:, 128], 20e-3, atol=1e-12)
    assert abs(seq.dt.reshape(256, 4).sum(axis=1) - 0.5).max() < 1e-12
    # m0 = rho / 4 per isochromat, jitter within half a voxel
    d = C.FOV / 256
    xc = np.repeat((np.arange(256 * 256) % 256 - 128) * d, 4)
    assert np.all(np.abs(obj.x - xc) <= d / 2 + 1e-7)


def test_c3_counts_kspace_te_and_rf_sampling_condition():
    seq = C.gre_3d_sinc(128, 4, 3)          # a few encodes of the full recipe
    full_steps = 4227072
    assert seq.n_steps_per_spin * (128 * 128) // 12 == full_steps
    k, t = _sample_k_and_t(seq)
    k = k.reshape(3, 4, 128, 3)
    n = np.arange(128)
    np.testing.assert_allclose(k[0, 0, :, 0], (n - 64) / C.FOV, atol=1e-9)
    np.testing.assert_allclose(k[:, 0, 0, 2], (np.arange(3) - 1) / C.FOV, atol=1e-9)
    np.testing.assert_allclose(k[0, :, 0, 1], (np.arange(4) - 2) / C.FOV, atol=1e-9)
    np.testing.assert_allclose(t.reshape(12, 128)[:, 64], 5e-3, atol=1e-12)
    shp = seq.shapes[0]
    assert shp.n_sub == 128 and abs(shp.alpha.sum() - 30 * C.DEG) < 1e-12
    # eq. B.4 / B.5: tau < pi / (w_max + dw/2), w_max = gamma Gz FOV/2 (rad/s),
    # dw = pulse bandwidth (rad/s); gamma Gz / 2pi = m_sub_z / tau.
    gz_hz_per_m = shp.m_sub[2] / shp.tau
    w_max = 2 * math.pi * gz_hz_per_m * C.FOV / 2
    dw = 2 * math.pi * 4.0 / (shp.n_sub * shp.tau)
    assert shp.tau < math.pi / (w_max + dw / 2)
    # slab: bandwidth / gradient = 0.15 m
    assert abs((4.0 / (shp.n_sub * shp.tau)) / gz_hz_per_m - 0.15) < 1e-12


def test_c3_object_species_and_b0():
    obj = grid3d_two_species(8, seed=1003)
    nv = 8 ** 3
    assert obj.n_spins == 2 * nv
    np.testing.assert_array_equal(obj.x[:nv], obj.x[nv:])
    np.testing.assert_allclose(obj.m0[:nv] / 0.8, obj.m0[nv:] / 0.2, rtol=1e-6)
    b0_w = obj.dw[:nv] / (2 * np.pi)
    b0_f = obj.dw[nv:] / (2 * np.pi)
    np.testing.assert_allclose(b0_f - b0_w, -440.0, atol=2e-3)
    assert abs(np.max(np.abs(b0_w)) - 50.0) < 1e-3


def test_c4_requests_are_seeded_and_in_range():
    a = C.c4(8)
    b = C.c4(8)
    for (o1, s1), (o2, s2) in zip(a, b):
        np.testing.assert_array_equal(o1.m0, o2.m0)
        assert s1.n_samples == s2.n_samples
        n = int(round(math.sqrt(o1.n_spins)))
        assert 16 <= n <= 256
        assert s1.meta["n_read"] == n and 32 <= s1.meta["n_pe"] <= 256


def test_c5_stream_rate_and_mix():
    st = C.c5_stream()
    assert len(st) == 2000
    t = np.array([a for a, _, _ in st])
    assert np.all(np.diff(t) >= 0)
    rate = (len(t) - 1) / (t[-1] - t[0])
    assert 45 < rate < 55
    frac3d = np.mean([k == "3d" for _, k, _ in st])
    assert 0.07 < frac3d < 0.13


def test_grid_is_seeded():
    a = grid2d(16, seed=3, iso_per_voxel=4, jitter=True, dw_sigma_hz=20)
    b = grid2d(16, seed=3, iso_per_voxel=4, jitter=True, dw_sigma_hz=20)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.dw, b.dw)


def test_legendre_polynomial_matches_scipy():
    from scipy.special import eval_legendre
    from workloads.phantom import legendre_p
    x = np.linspace(-1, 1, 401)
    for l in (0, 1, 2, 5, 12):
        np.testing.assert_allclose(legendre_p(l, x), eval_legendre(l, x), rtol=1e-12, atol=1e-13)


def test_legendre_b0_field_eq_6_3():
    """On the z axis P_12(1) = 1, so dB0 = -C (r/R)^12; in the z = 0 plane
    P_12(0) = 231/1024 (a positive constant); zero field at the centre."""
    from workloads.phantom import legendre_b0_tesla
    r = np.linspace(0, 0.3, 13)
    np.testing.assert_allclose(legendre_b0_tesla(0 * r, 0 * r, r, 2e-5, 0.2), -2e-5 * (r / 0.2) ** 12, rtol=1e-12)
    np.testing.assert_allclose(legendre_b0_tesla(r, 0 * r, 0 * r, 2e-5, 0.2),
                               -2e-5 * (r / 0.2) ** 12 * 231 / 1024, rtol=1e-12, atol=1e-30)
    assert legendre_b0_tesla(0.0, 0.0, 0.0, 1.0, 0.2) == 0.0


def test_table78_workloads():
    from workloads import configs as C
    sizes = {}
    for k in C.TABLE78:
        obj, seq = C.table78(k)
        sizes[k] = (obj.n_spins, seq.n_samples)
        assert np.all(np.isfinite(obj.dw))
    assert sizes["tse"] == sizes["radial"] == sizes["epi"] == (10000, 128 * 128)
    assert sizes["se3d"] == (56 ** 3, 128 * 128 * 64)
    # the radial spokes cross the k-space centre at sample n/2
    seq = C.radial_2d(16, 8)
    m = seq.m
    for p in range(8):
        pre, ro = m[3 * p], m[3 * p + 1]
        k_mid = pre + ro * (16 // 2 + 1) / 16
        np.testing.assert_allclose(k_mid, 0.0, atol=1e-9)
