"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
identical seeded inputs.

Bars: FP32 stepping rel-L2 <= 1e-5, FP64 stepping rel-L2 <= 1e-12 over all
samples of a request (rel-L2 = 10^(dE/20) with the noise distance dE of
section 5.4.2).  Full-size configurations are checked on sampled outputs
the oracle can compute (the first repetitions of the full object) and on
fixed spin subsets over the whole sequence (superposition makes subset
parity exact up to summation order).
"""
import math

import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import Sequence, Shape, SPOIL, configs as C
from workloads.phantom import SpinObject, grid2d, grid3d_two_species, random_spins, subset

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


@pytest.fixture(scope="module")
def ctx32(ps):
    return ps.Context(precision=32)


@pytest.fixture(scope="module")
def ctx64(ps):
    return ps.Context(precision=64)


def gpu(ctx, obj, seq):
    import torch
    out = ctx.simulate(obj, seq)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(ctx, obj, seq, tol, ref=None, label=""):
    ref = oracle.simulate(obj, seq) if ref is None else ref
    got = gpu(ctx, obj, seq)
    err = within(got, ref, tol, f"{label or seq.name} spins={obj.n_spins}")
    return got, ref, err


# --------------------------------------------------------------------------
# whole configurations at oracle-friendly sizes
# --------------------------------------------------------------------------
def test_c1_full_fp32(ctx32):
    obj, seq = C.c1()
    check(ctx32, obj, seq, TOL32, label="c1")


def test_c1_full_fp64(ctx64):
    obj, seq = C.c1()
    check(ctx64, obj, seq, TOL64, label="c1/fp64")


@pytest.mark.parametrize("n", [32, 64])
def test_c2_recipe_reduced(ctx32, ctx64, n):
    obj, seq = C.c2(n)
    ref = oracle.simulate(obj, seq)
    check(ctx32, obj, seq, TOL32, ref=ref, label=f"c2[{n}]")
    check(ctx64, obj, seq, TOL64, ref=ref, label=f"c2[{n}]/fp64")


def test_c3_recipe_reduced(ctx32, ctx64):
    obj, _ = C.c3(16)
    seq = C.gre_3d_sinc(16, 4, 3)
    ref = oracle.simulate(obj, seq)
    check(ctx32, obj, seq, TOL32, ref=ref, label="c3[16]")
    check(ctx64, obj, seq, TOL64, ref=ref, label="c3[16]/fp64")


# --------------------------------------------------------------------------
# full sizes in the benchmark's launch configuration
# --------------------------------------------------------------------------
def test_c2_full_size_first_repetitions(ctx32):
    """The full 256^2 x 4-isochromat object through the whole sequence; the
    oracle computes the first two repetitions' 512 samples exactly."""
    obj, seq = C.c2()
    got = gpu(ctx32, obj, seq)
    ref = oracle.simulate(obj, seq.truncated(8))
    within(got[:ref.size], ref, TOL32, "c2 full, first 2 TRs")


def test_c2_full_sequence_spin_subset(ctx32):
    """Every 64th spin of the full object through all 256 repetitions."""
    obj, seq = C.c2()
    check(ctx32, subset(obj, 64), seq, TOL32, label="c2 subset/64")


def test_c3_full_object_subset_truncated(ctx32):
    """Every 4096th spin of the full 2 x 128^3 object, first 48 repetitions
    of the full recipe (sinc 128 sub-steps, 128 samples)."""
    obj, seq = C.c3()
    check(ctx32, subset(obj, 4096, 7), seq.truncated(3 * 48), TOL32, label="c3 subset/4096")


def test_c3_full_sequence_spin_subset_sliced(ps):
    """Every 1024th spin of the full 2 x 128^3 object (4,096 spins) through
    all 16,384 repetitions, with the partial-sum buffer held to 4 MiB.  At 2
    spins per lane the 2,097,152 samples run as 32 time slices of 65,536: the
    sinc propagator cached in the first slice is written to the slice state
    and read back by all 31 later slices at S = 2, and the spin anchors pass
    through the alternating anchor buffers.  Without readout replicas (the
    tiling the full object gets), and with them (8 tiles, so replicas share
    every slice's 512 readouts).  At 1 spin per lane (64 slices) every
    readout is summed on the matrix cores."""
    obj, seq = C.c3()
    sub = subset(obj, 1024, 5)
    ref = oracle.simulate(sub, seq)
    for S, split in ((2, False), (2, True), (1, False), (1, True)):
        with ps.Context(precision=32, spins_per_lane=S, readout_split=split, max_partial_bytes=4 << 20) as ctx:
            within(gpu(ctx, sub, seq), ref, TOL32, f"c3 subset/1024 full sequence S={S}, sliced, split={split}")


def test_replicas_across_many_slices_fp64(ps):
    """Readout replicas of a tile all start from the slice's anchors, while
    replica 0 writes the next slice's anchors at its end.  With 150 tiles and
    4 replicas (600 workgroups of one per CU in FP64) later replicas start
    after replica 0 of their tile has finished; the anchors alternate between
    two buffers, so they still read the slice's start.  Five slices of eight
    64-sample readouts; bitwise equal to the unsplit launch and within the
    FP64 bar of the oracle."""
    obj = random_spins(150 * 256, seed=31, dw_sigma_hz=25.0)
    seq = C.spoiled_gre_2d(64, 40, alpha_deg=40.0)
    part = 150 * 2 * 8 * 64 * 8                        # rows x re/im x FP64 x 8 readouts of 64 samples
    res = {}
    for split in (True, False):
        with ps.Context(precision=64, spins_per_lane=1, readout_split=split, max_partial_bytes=part) as ctx:
            res[split] = gpu(ctx, obj, seq)
    np.testing.assert_array_equal(res[True], res[False])
    within(res[True], oracle.simulate(obj, seq), TOL64, "replicas across 5 slices fp64")


def test_two_streams_without_host_sync(ps):
    """Two requests on two streams, the second issued while the first still
    runs: each call takes its own buffer set, so the second returns without
    waiting for the first, and both match the oracle.  The first is a
    2^22-sample readout of 1,000 spins kept on 4 workgroups (no readout
    replicas), tens of ms of device time."""
    import torch
    long_obj = random_spins(1000, seed=41, dw_sigma_hz=10.0, t_inf_frac=0.5)
    n = 1 << 22
    long_seq = Sequence("long")
    long_seq.add(1e-3, alpha=np.pi / 2)
    long_seq.add(n * 2e-7, m=(0.002 * n, 0.0, 0.0), n_adc=n)
    short_obj, short_seq = C.c2(32)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with ps.Context(precision=32, readout_split=False) as ctx:
        torch.cuda.synchronize()
        a = ctx.simulate(long_obj, long_seq, stream=s1)
        b = ctx.simulate(short_obj, short_seq, stream=s2)
        first_busy = not s1.query()
        torch.cuda.synchronize()
    print(f"[parity] two streams: first request still running after the second call returned: {first_busy}",
          flush=True)
    assert first_busy
    within(b.cpu().numpy(), oracle.simulate(short_obj, short_seq), TOL32, "two streams, short request")
    within(a.cpu().numpy(), oracle.simulate(long_obj, long_seq), TOL32, "two streams, 2^22-sample request")


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------
def test_empty_object_gives_zeros(ctx32):
    obj = random_spins(4, seed=1).take(np.arange(0))
    got = gpu(ctx32, obj, C.fid(1.0, 10, 1e-3))
    assert got.shape == (10,) and np.all(got == 0)


def test_sequence_without_samples(ctx32):
    got = gpu(ctx32, random_spins(100, seed=2), Sequence("none").add(1e-3, alpha=1.0))
    assert got.shape == (0,)


@pytest.mark.parametrize("n_spins", [1, 63, 257, 1000, 4097])
def test_ragged_spin_counts(ctx32, n_spins):
    obj = random_spins(n_spins, seed=n_spins, t_inf_frac=0.2)
    _, seq = C.c1()
    check(ctx32, obj, seq.truncated(9), TOL32, label=f"ragged{n_spins}")


@pytest.mark.parametrize("n_adc", [1, 17, 31, 32, 33, 95, 1000])
def test_ragged_sample_counts(ctx32, ctx64, n_adc):
    obj = random_spins(700, seed=3)
    seq = Sequence(f"adc{n_adc}")
    seq.add(2e-3, m=(-40, 10, 5), alpha=0.5, phase=0.3)
    seq.add(n_adc * 1e-5, m=(n_adc * 1.5, 0, 0), n_adc=n_adc)
    seq.add(1e-3, m=(3, 0, 0), alpha=1.2, phase=-0.4)
    seq.add(n_adc * 2e-5, m=(0, n_adc * 0.7, 0), n_adc=n_adc, flags=SPOIL)
    seq.add(1e-3, alpha=0.4, n_adc=3)
    ref = oracle.simulate(obj, seq)
    check(ctx32, obj, seq, TOL32, ref=ref, label=f"adc{n_adc}")
    check(ctx64, obj, seq, TOL64, ref=ref, label=f"adc{n_adc}/fp64")


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_short_readouts_every_tiling(ps, S):
    """Readouts of 1, 2 and 3 chunks of 32 samples (one chunk ragged): with
    fewer chunks than a wave group has waves, the waves share each chunk's
    spins and add their sums in LDS; wave groups of 4, 4, 2 and 1 waves."""
    obj = random_spins(1500, seed=5)
    seq = Sequence("short")
    for n_adc in (20, 64, 70):
        seq.add(1e-3, m=(-n_adc / 2, 3, 0), alpha=0.6, phase=0.2)
        seq.add(n_adc * 1e-5, m=(n_adc * 1.1, 0, 0), n_adc=n_adc, flags=SPOIL)
    with ps.Context(precision=32, spins_per_lane=S) as ctx:
        check(ctx, obj, seq, TOL32, label=f"short readouts S={S}")


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_readouts_with_a_partial_last_round(ps, S):
    """Readouts of 5, 6, 7 and 10 chunks of 32 samples (the last ragged):
    the waves of a wave group run different numbers of chunks, each from its
    own anchor advanced by W = z^(32 G) per round; FP64 on the tilings it
    has."""
    obj = random_spins(2100, seed=6 + S, dw_sigma_hz=35.0)
    seq = Sequence("rounds")
    for n_adc in (150, 180, 220, 300):
        seq.add(1e-3, m=(-n_adc / 3, 2, 1), alpha=0.8, phase=0.1)
        seq.add(n_adc * 1e-5, m=(n_adc * 0.9, 0, 0.2), n_adc=n_adc, flags=SPOIL)
    with ps.Context(precision=32, spins_per_lane=S) as ctx:
        check(ctx, obj, seq, TOL32, label=f"partial last round S={S}")
    if S <= 2:
        with ps.Context(precision=64, spins_per_lane=S) as ctx:
            check(ctx, obj, seq, TOL64, label=f"partial last round fp64 S={S}")


def test_long_readout_and_time_slicing(ps):
    """A 5000-sample readout forced through many time slices (small partial
    buffer).  A slice boundary inside a readout re-anchors the recurrence from
    the FP64 phase, so the sliced run agrees with the unsliced one to rounding
    (not bit for bit); both match the oracle."""
    obj = random_spins(3000, seed=4)
    seq = Sequence("long")
    seq.add(1e-3, alpha=1.0)
    seq.add(5000 * 4e-6, m=(2000, 0, 0), n_adc=5000)
    seq.add(1e-3, alpha=2.0, phase=1.0, n_adc=7, flags=SPOIL)
    seq.add(1e-3, alpha=0.7, n_adc=300)
    with ps.Context(precision=32, spins_per_lane=1) as big, \
            ps.Context(precision=32, spins_per_lane=1, max_partial_bytes=12 * 8 * 256) as small:
        a = gpu(big, obj, seq)
        b = gpu(small, obj, seq)
    within(b, a, 5e-6)
    ref = oracle.simulate(obj, seq)
    print(f"[parity] long readout unsliced {oracle.rel_l2(a, ref):.3e} sliced {oracle.rel_l2(b, ref):.3e}",
          flush=True)
    within(a, ref, TOL32)
    within(b, ref, TOL32)


def test_readout_of_a_million_samples(ctx32, ctx64):
    """One readout of 2^20 samples (1 us dwell) on spins without relaxation,
    so the last samples weigh as much as the first: the recurrence is cut
    into runs that each start from their own FP64 phase, so its rounding
    does not build up along the readout (one unbroken FP32 run was 2.4e-4
    off here).  The FP32 signal is checked against the oracle; the FP64 one
    against the closed form j m0 exp(-j (2 pi k_n.x + dw t_n)) at the first
    and last 4096 samples, since the oracle's own 2^20 sequential FP64
    sub-steps carry ~1e-11 of rounding."""
    obj = random_spins(600, seed=9, dw_sigma_hz=30.0, t_inf_frac=1.0)
    n, tau, pre = 1 << 20, 1e-6, 1e-3
    m = np.array([0.01, -0.004, 0.002]) * n
    seq = Sequence("long1M")
    seq.add(pre, alpha=np.pi / 2)
    seq.add(n * tau, m=tuple(m), n_adc=n)
    ref = oracle.simulate(obj, seq)
    idx = np.r_[0:4096, n - 4096:n]
    pos = np.stack([obj.x, obj.y, obj.z]).astype(np.float64)
    k = np.outer(idx + 1, m / n)                                        # cycles/m at sample idx
    t = pre + (idx + 1) * tau
    ph = 2 * np.pi * (k @ pos) + t[:, None] * obj.dw.astype(np.float64)[None, :]
    closed = (1j * obj.m0.astype(np.float64)[None, :] * np.exp(-1j * ph)).sum(axis=1)
    got32 = gpu(ctx32, obj, seq)
    got64 = gpu(ctx64, obj, seq)
    print(f"[parity] 2^20-sample readout: oracle vs closed form {oracle.rel_l2(ref[idx], closed):.3e}", flush=True)
    within(got32, ref, TOL32, "2^20-sample readout fp32")
    within(got32[-4096:], ref[-4096:], TOL32, "2^20-sample readout fp32, last 4096")
    within(got64[idx], closed, TOL64, "2^20-sample readout fp64 vs closed form")


def test_shaped_pulses_with_phase_offsets_and_hard_pulse(ctx32, ctx64):
    obj = random_spins(900, seed=5, dw_sigma_hz=200.0)
    rng = np.random.default_rng(5)
    seq = Sequence("shapes")
    s0 = seq.add_shape(Shape(tau=1e-5, m_sub=(0, 0, 4.0), alpha=rng.uniform(-0.1, 0.2, 50),
                             phase=rng.uniform(-1, 1, 50)))
    s1 = seq.add_shape(C.sinc_shape(64, 2e-5, 0.8, 4.0, 0.1))
    seq.add(1e-3, m=(0, 0, -100), shape=s0, phase=0.3, n_adc=20)
    seq.add(2e-3, m=(30, -20, 0), shape=s1, alpha=0.4, phase=1.1, n_adc=40)
    seq.add(1e-3, shape=s0, phase=0.3, flags=SPOIL)
    seq.add(1e-3, shape=s1, phase=-2.0, n_adc=33)
    ref = oracle.simulate(obj, seq)
    check(ctx32, obj, seq, TOL32, ref=ref, label="shapes")
    check(ctx64, obj, seq, TOL64, ref=ref, label="shapes/fp64")


def test_closed_form_spin_echo_on_gpu(ctx64):
    """GPU FP64 against the closed form directly (echo = j m0 e^{-TE/T2})."""
    te, n = 40e-3, 16
    obj = random_spins(333, seed=6, dw_sigma_hz=80.0)
    got = gpu(ctx64, obj, C.spin_echo_single(te, n, 1e-4))
    ref = 1j * np.sum(obj.m0.astype(float) * np.exp(-te / obj.t2.astype(float)))
    assert abs(got[n // 2] - ref) <= 1e-12 * abs(ref)


# --------------------------------------------------------------------------
# determinism and tiling
# --------------------------------------------------------------------------
def test_bitwise_repeatable(ctx32):
    obj, seq = C.c2(48)
    a = gpu(ctx32, obj, seq)
    b = gpu(ctx32, obj, seq)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_every_tiling_matches_oracle(ps, S):
    obj, seq = C.c2(40)
    with ps.Context(precision=32, spins_per_lane=S) as ctx:
        check(ctx, obj, seq, TOL32, label=f"c2[40] S={S}")


def test_spin_permutation_and_superposition(ctx32):
    obj, seq = C.c2(32)
    a = gpu(ctx32, obj, seq)
    perm = np.random.default_rng(0).permutation(obj.n_spins)
    b = gpu(ctx32, obj.take(perm), seq)
    within(b, a, TOL32)
    half = obj.n_spins // 2
    c = gpu(ctx32, obj.take(np.arange(half)), seq) + gpu(ctx32, obj.take(np.arange(half, obj.n_spins)), seq)
    within(c, a, TOL32)
