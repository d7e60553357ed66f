"""GPU parity of the matrix-core readout (FP32, one spin per lane).

A readout of at least 64 samples whose per-sample step it shares with a
neighbouring readout is summed over the spins as a complex matrix product on
the matrix cores (eq. 3.32 over tiles of 128 samples).  Each case runs with
that path and with the vector path (PS_CFG_NO_MATRIX_READOUT), checks both
against the FP64 oracle by the two measures of section 5.4.2, and checks
that the two results are not bitwise equal, i.e. that the matrix path did
run.  Cases: tile-ragged readout lengths and spin counts, a readout long
enough to re-anchor from the FP64 phase, receive coils, readout replicas,
time slices that cut readouts, and sequences whose per-sample step changes
between runs of readouts (tables rebuilt) or from readout to readout (the
vector path), mixed with trajectory and short readouts.
"""
import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import Sequence, SPOIL, Trajectory, configs as C
from workloads.phantom import random_spins, subset

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


def run(ps, obj, seq, coils=None, **kw):
    import torch
    with ps.Context(precision=32, spins_per_lane=1, **kw) as ctx:
        out = ctx.simulate(obj, seq, coils=coils) if coils is not None else ctx.simulate(obj, seq)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def both_paths(ps, obj, seq, label, ref=None, coils=None, **kw):
    """Matrix and vector path against the oracle; they must differ in rounding."""
    if ref is None:
        ref = oracle.simulate(obj, seq, coils=coils) if coils is not None else oracle.simulate(obj, seq)
    mat = run(ps, obj, seq, coils=coils, **kw)
    vec = run(ps, obj, seq, coils=coils, matrix_readout=False, **kw)
    within(mat, ref, TOL32, f"{label} matrix")
    within(vec, ref, TOL32, f"{label} vector")
    assert not np.array_equal(mat, vec), f"{label}: the matrix path did not run"
    return mat, vec, ref


def cartesian(n_adc, n_rep, ky_step=3.0, kz=0.4, alpha=0.5, dwell=1e-5):
    """Repetitions of one readout step (mu, tau) with a varying phase encode."""
    seq = Sequence(f"cart{n_adc}")
    for r in range(n_rep):
        seq.add(1e-3, m=(-(n_adc // 2 + 1) * 1.3, ky_step * (r - n_rep // 2), kz), alpha=alpha, phase=0.3 * r)
        seq.add(n_adc * dwell, m=(n_adc * 1.3, 0.0, 0.2), n_adc=n_adc, flags=SPOIL)
    return seq


@pytest.mark.parametrize("n_adc", [64, 100, 128, 129, 200, 256, 300])
def test_readout_lengths_and_ragged_spins(ps, n_adc):
    """Tiles of 128 samples with a ragged last tile; 1,000 spins fill three
    workgroup tiles and part of a fourth (padding spins contribute zero)."""
    obj = random_spins(1000, seed=100 + n_adc, dw_sigma_hz=40.0)
    both_paths(ps, obj, cartesian(n_adc, 6), f"n_adc={n_adc}")


def test_long_readout_reanchors(ps):
    """A 2,500-sample readout (20 tiles): m is stepped by z^128 from tile to
    tile and taken again from the FP64 phase every 8 tiles."""
    obj = random_spins(777, seed=7, dw_sigma_hz=60.0, t_inf_frac=0.3)
    both_paths(ps, obj, cartesian(2500, 3, dwell=4e-6), "2500 samples")


def test_c2_recipe(ps):
    """The 2-D spin echo recipe at 64^2 x 4 isochromats (64-sample readouts)."""
    obj, seq = C.c2(64)
    both_paths(ps, obj, seq, "c2[64]")


def test_c2_full_sequence_spin_subset(ps):
    """Every 64th spin of the full 256^2 x 4 object through all 256
    repetitions: 256-sample readouts, two tiles each."""
    obj, seq = C.c2()
    both_paths(ps, subset(obj, 64, 3), seq, "c2 subset/64")


@pytest.mark.parametrize("shape_cache", [True, False])
def test_c3_recipe_reduced(ps, shape_cache):
    """3-D GRE with the sinc at 16^3 x 2 species, 128-sample readouts: the
    matrix-only kernel, which reads the sinc's sub-pulse rotations from
    memory instead of LDS, with the cached propagator and stepping the
    sub-steps directly."""
    obj, _ = C.c3(16)
    seq = C.gre_3d_sinc(128, 8, 3)
    both_paths(ps, obj, seq, f"c3 16^3 128-sample readouts shape_cache={shape_cache}", shape_cache=shape_cache)


@pytest.mark.parametrize("n_coils", [1, 3])
def test_receive_coils(ps, n_coils):
    """Each coil's pass weights m by (S_x - j S_y) of the coil at the spin."""
    obj = random_spins(900, seed=11, dw_sigma_hz=20.0)
    rng = np.random.default_rng(12)
    sx = rng.normal(size=(n_coils, obj.n_spins)).astype(np.float32)
    sy = rng.normal(size=(n_coils, obj.n_spins)).astype(np.float32)
    both_paths(ps, obj, cartesian(192, 5), f"{n_coils} coils", coils=(sx, sy))


def test_replicas_and_time_slices(ps):
    """Readout replicas (a small object, split readouts) and time slices that
    cut the sequence inside a readout (a partial buffer of 4 rows x 200
    samples): every piece of a cut readout keeps its step, so it stays on the
    matrix path."""
    obj = random_spins(1000, seed=21, dw_sigma_hz=30.0)
    seq = cartesian(160, 9)
    ref = oracle.simulate(obj, seq)
    for kw in ({"readout_split": True}, {"readout_split": False},
               {"readout_split": True, "max_partial_bytes": 4 * 2 * 4 * 200}):
        both_paths(ps, obj, seq, f"replicas/slices {kw}", ref=ref, **kw)


def test_step_changes_and_mixed_readouts(ps):
    """Runs of readouts with one step, then another (tables rebuilt), an
    isolated readout with a step of its own and readouts of fewer than 64
    samples (both on the vector path), and a trajectory readout in between."""
    obj = random_spins(1300, seed=31, dw_sigma_hz=45.0, t_inf_frac=0.2)
    seq = Sequence("mixed")
    traj = seq.add_trajectory(Trajectory(k=np.linspace(0, 1, 3 * 80).reshape(80, 3) * 40.0,
                                         t=np.linspace(1e-5, 8e-4, 80)))
    for r, (n_adc, gx, gy) in enumerate([(128, 1.3, 0.0)] * 3 + [(96, 0.0, 1.7)] * 3 + [(128, 1.3, 0.0)] * 2 +
                                        [(150, 0.9, 0.9)] + [(40, 1.3, 0.0)] * 2 + [(128, 1.3, 0.0)] * 2):
        seq.add(1e-3, m=(-(n_adc // 2) * gx, -(n_adc // 2) * gy + 2.0 * r, 0.3), alpha=0.6, phase=0.2 * r)
        seq.add(n_adc * 1e-5, m=(n_adc * gx, n_adc * gy, 0.0), n_adc=n_adc, flags=SPOIL)
        if r == 4:
            seq.add(1e-3, alpha=0.3)
            seq.add(1e-3, m=(40.0, 40.0, 40.0), n_adc=80, trajectory=traj, flags=SPOIL)
    both_paths(ps, obj, seq, "mixed steps")


def test_batch_at_one_spin_per_lane(ps):
    """Requests in one persistent launch take the matrix path per request and
    give the same bits as alone."""
    import torch
    objs = [random_spins(n, seed=40 + n, dw_sigma_hz=25.0) for n in (300, 1000, 2600)]
    seqs = [cartesian(n_adc, 4) for n_adc in (64, 200, 130)]
    with ps.Context(precision=32, spins_per_lane=1) as ctx:
        batch = [o.cpu().numpy() for o in ctx.simulate_batch(objs, seqs)]
        alone = []
        for o, s in zip(objs, seqs):
            alone.append(ctx.simulate(o, s).cpu().numpy())
        torch.cuda.synchronize()
    for b, a, o, s in zip(batch, alone, objs, seqs):
        np.testing.assert_array_equal(b, a)
        within(b, oracle.simulate(o, s), TOL32, f"batch {o.n_spins} spins")
