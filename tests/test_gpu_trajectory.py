"""GPU: readouts at tabulated instants (per-sample trajectory tables,
PS_EV_TRAJECTORY) against the FP64 oracle -- multi-shot spirals with
relaxation and off-resonance, equal sub-steps written as a table, the
interval-end state, receive coils, snapshots, time slicing, every tiling,
the readout split, batched and served execution, and argument errors."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import Sequence, SNAPSHOT, Trajectory, coils, configs as C
from workloads.phantom import random_spins

pytestmark = pytest.mark.gpu
TOL32, TOL64 = 1e-5, 1e-12


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


def run(ps, obj, seq, rx=None, **kw):
    import torch
    with ps.Context(**kw) as ctx:
        out = ctx.simulate(obj, seq, coils=rx)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def check(label, got, ref, tol):
    within(got, ref, tol, f"trajectory {label}")


def test_spiral_against_the_oracle(ps):
    obj = random_spins(3000, seed=61, dw_sigma_hz=60.0)
    seq = C.spiral_2d(4, 300, res=64)
    ref = oracle.simulate(obj, seq)
    check("spiral 4x300 fp32", run(ps, obj, seq), ref, TOL32)
    check("spiral 4x300 fp64", run(ps, obj, seq, precision=64), ref, TOL64)


def test_equal_sub_steps_as_a_table(ps):
    obj = random_spins(2000, seed=62, dw_sigma_hz=40.0)
    seq0 = C.spoiled_gre_2d(40, 6)
    seq1 = Sequence("as-table")
    for e in range(seq0.n_events):
        n = int(seq0.n_adc[e])
        j = -1
        if n:
            s = (np.arange(n) + 1) / n
            j = seq1.add_trajectory(Trajectory(k=np.outer(s, seq0.m[e]), t=s * seq0.dt[e]))
        seq1.add(seq0.dt[e], m=seq0.m[e], alpha=seq0.rf_alpha[e], n_adc=n, flags=int(seq0.flags[e]), trajectory=j)
    a, b = run(ps, obj, seq0), run(ps, obj, seq1)
    check("table vs sub-steps", b, a, 3e-6)
    check("table vs oracle", b, oracle.simulate(obj, seq1), TOL32)


def test_interval_end_state(ps):
    obj = random_spins(1500, seed=63, dw_sigma_hz=30.0)
    u = (np.arange(50) + 1) / 50
    tr = Trajectory(k=np.stack([40 * u * np.cos(9 * u), 40 * u * np.sin(9 * u), 5 * u], axis=1), t=u * 3e-3)
    seq = Sequence("t")
    j = seq.add_trajectory(tr)
    seq.add(5e-3, m=(12.0, -7.0, 3.0), alpha=1.0, n_adc=50, trajectory=j)
    seq.add(2e-3, m=(20.0, 0, 0), n_adc=16)
    check("table + readout", run(ps, obj, seq), oracle.simulate(obj, seq), TOL32)


def test_coils_snapshots_and_time_slices(ps):
    obj = random_spins(1800, seed=64, dw_sigma_hz=50.0)
    seq0 = C.spiral_2d(3, 200, res=48)
    seq = Sequence("spiral+snap")
    for t in seq0.trajectories:
        seq.add_trajectory(t)
    for e in range(seq0.n_events):
        seq.add(seq0.dt[e], m=seq0.m[e], alpha=seq0.rf_alpha[e], n_adc=int(seq0.n_adc[e]),
                flags=int(seq0.flags[e]) | (SNAPSHOT if seq0.n_adc[e] else 0), trajectory=int(seq0.trajectory[e]))
    rx = coils.loop_ring(obj, 2, ring_radius=0.2, coil_radius=0.06)
    ref_sig, ref_snap = oracle.simulate(obj, seq, coils=rx, snapshots=True)
    import torch
    # 1800 spins at S = 1: 8 workgroups x 1 row; 2 coils; 64 samples per slice
    for kw in ({}, {"spins_per_lane": 1, "max_partial_bytes": 8 * 2 * 4 * 2 * 64}):
        with ps.Context(**kw) as ctx:
            sig, snap = ctx.simulate(obj, seq, coils=rx, snapshots=True)
            torch.cuda.synchronize()
            sig, snap = sig.cpu().numpy(), snap.cpu().numpy().astype(np.float64)
        for c in range(2):
            check(f"coil {c} {kw}", sig[c], ref_sig[c], TOL32)
        check(f"snapshots {kw}", snap, ref_snap, TOL32)


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_every_tiling(ps, S):
    obj = random_spins(2600, seed=65 + S, dw_sigma_hz=40.0)
    seq = C.spiral_2d(2, 150, res=40)
    check(f"spiral S={S}", run(ps, obj, seq, spins_per_lane=S), oracle.simulate(obj, seq), TOL32)


def _spiral_table(n, t_end, power):
    """A spiral whose instants are t_end (s / n)^power: an equal raster for
    power 1, uneven (variable density) otherwise."""
    u = (np.arange(n) + 1) / n
    th = 2 * np.pi * 6 * u
    k = np.stack([300 * u * np.cos(th), 300 * u * np.sin(th), 20 * u], axis=1)
    return Trajectory(k=k, t=t_end * u ** power)


@pytest.mark.parametrize("S", [1, 2, 4])
@pytest.mark.parametrize("power", [1.0, 1.3])
def test_even_and_uneven_instants_with_fast_decay(ps, S, power):
    """Instants on an equal raster (the decay stepped by one factor per
    sample) and uneven instants (the decay evaluated at every sample), with
    T2 down to 1.5 ms so that the decay inside an 8-sample block matters,
    on the tilings whose wave groups share their spins."""
    obj = random_spins(2300, seed=80 + S, dw_sigma_hz=40.0)
    obj.t2[:] = obj.t2 / 20.0
    seq = Sequence("even" if power == 1.0 else "uneven")
    for i in range(3):
        j = seq.add_trajectory(_spiral_table(150 + 13 * i, 1.5e-3, power))
        seq.add(1e-3, alpha=0.6 + 0.2 * i, phase=0.4 * i)
        seq.add(2e-3, m=(3.0, -2.0, 1.0), n_adc=150 + 13 * i, trajectory=j)
    check(f"instants^{power} S={S}", run(ps, obj, seq, spins_per_lane=S), oracle.simulate(obj, seq), TOL32)


def test_split_batch_and_serve_bitwise(ps):
    import torch
    obj = random_spins(900, seed=70, dw_sigma_hz=40.0)
    seq = C.spiral_2d(4, 120, res=40)
    a = run(ps, obj, seq)
    np.testing.assert_array_equal(a, run(ps, obj, seq, readout_split=False))
    with ps.Context() as ctx:
        b = ctx.simulate_batch([obj, obj], [seq, seq])
        c = ctx.submit(obj, seq).wait(60.0)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(b[0].cpu().numpy(), a)
        np.testing.assert_array_equal(b[1].cpu().numpy(), a)
        np.testing.assert_array_equal(c.cpu().numpy(), a)


def test_errors(ps):
    u = (np.arange(8) + 1) / 8
    tr = Trajectory(k=np.zeros((8, 3)), t=u * 1e-3)
    for bad in ("count", "late", "index", "decreasing"):
        seq = Sequence("bad")
        j = seq.add_trajectory(Trajectory(k=np.zeros((8, 3)), t=(u[::-1] if bad == "decreasing" else u) * 1e-3))
        seq.add(1e-3 if bad != "late" else 0.5e-3, alpha=1.0, n_adc=7 if bad == "count" else 8,
                trajectory=j + (1 if bad == "index" else 0))
        with pytest.raises(ps.PsError) as ei:
            ps.count(seq)
        assert ei.value.status == 1, bad
