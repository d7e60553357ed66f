"""GPU: receive coils with inhomogeneous sensitivity (ps_simulate_rx) against
the FP64 oracle (section 3.5.1, eq. 3.25: coil c receives the sum over spins
of (S_x - j S_y)(Mx + j My)).  The spins are stepped once for all coils; each
coil has its own readout pass and its own partial sums."""
import ctypes

import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import SPOIL, Sequence, coils, configs as C
from workloads.phantom import random_spins

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12


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


def per_coil(label, got, ref, tol):
    assert got.shape == ref.shape
    errs = [within(got[c], ref[c], tol, f"{label} coil {c}") for c in range(ref.shape[0])]
    print(f"[coils] {label} worst rel_l2={max(errs):.3e} over {len(errs)} coils", flush=True)


def test_loop_ring_on_2d_spin_echo(ps):
    obj, seq = C.c2(24)
    rx = coils.loop_ring(obj, 4, ring_radius=0.2, coil_radius=0.07)
    ref = oracle.simulate(obj, seq, coils=rx)
    per_coil("c2[24] 4 loops", run(ps, obj, seq, rx), ref, TOL32)
    per_coil("c2[24] 4 loops/fp64", run(ps, obj, seq, rx, precision=64), ref, TOL64)


def test_homogeneous_x_coil_equals_plain_simulate_bitwise(ps):
    obj, seq = C.c2(20)
    plain = run(ps, obj, seq)
    got = run(ps, obj, seq, coils.homogeneous(obj))
    np.testing.assert_array_equal(got[0], plain)


def test_turned_homogeneous_coils(ps):
    obj = random_spins(1500, seed=31, dw_sigma_hz=50.0)
    seq = C.spoiled_gre_2d(32, 6)
    sx, sy = coils.homogeneous(obj, 3, [0.0, 0.9, -2.4])
    sx[1], sy[1] = 0.0, 1.0                                       # the y coil
    got = run(ps, obj, seq, (sx, sy))
    plain = oracle.simulate(obj, seq)
    within(got[1], -1j * plain, TOL32)
    per_coil("turned coils", got, oracle.simulate(obj, seq, coils=(sx, sy)), TOL32)


def test_surface_loop_with_shaped_pulses_and_cache(ps):
    obj, _ = C.c3(14)
    seq = C.gre_3d_sinc(14, 3, 3)
    rx = coils.loop_ring(obj, 3, ring_radius=0.18, coil_radius=0.05)
    ref = oracle.simulate(obj, seq, coils=rx)
    per_coil("c3[14] 3 loops", run(ps, obj, seq, rx), ref, TOL32)
    per_coil("c3[14] 3 loops direct", run(ps, obj, seq, rx, shape_cache=False), ref, TOL32)


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_coils_on_every_tiling(ps, S):
    obj = random_spins(2900, seed=32 + S, dw_sigma_hz=30.0)
    seq = C.spin_echo_2d(24, 5)
    rx = coils.loop_ring(obj, 2, ring_radius=0.25, coil_radius=0.1)
    per_coil(f"S={S} 2 loops", run(ps, obj, seq, rx, spins_per_lane=S), oracle.simulate(obj, seq, coils=rx), TOL32)


@pytest.mark.parametrize("S", [1, 2, 4])
def test_coils_on_short_readouts(ps, S):
    """Readouts of 1, 2 and 3 chunks of 32 samples (the last ragged) with
    three coils: where a readout has fewer chunks than the wave group has
    waves, the waves split the group's spins and add their sums in LDS, once
    per coil pass."""
    obj = random_spins(1700, seed=50 + S, dw_sigma_hz=25.0)
    seq = Sequence("short")
    for n_adc in (20, 64, 70):
        seq.add(1e-3, m=(-n_adc / 2, 2, 0), alpha=0.7, phase=0.3)
        seq.add(n_adc * 1e-5, m=(n_adc * 1.1, 0, 0), n_adc=n_adc, flags=SPOIL)
    rx = coils.loop_ring(obj, 3, ring_radius=0.2, coil_radius=0.08)
    per_coil(f"short readouts S={S} 3 loops", run(ps, obj, seq, rx, spins_per_lane=S),
             oracle.simulate(obj, seq, coils=rx), TOL32)


@pytest.mark.parametrize("precision", [32, 64])
def test_odd_sample_counts_row_groups_coils_and_slices(ps, precision):
    """Odd sample counts (rows and coil blocks padded for the finalize's
    four-value loads), more than one row group of partial rows (the
    two-pass cross-workgroup sum), three coils and several time slices, for
    one call and for the batched path."""
    import torch
    obj = random_spins(20000, seed=60, dw_sigma_hz=30.0)     # 79 workgroups at S = 1: two row groups
    seq = Sequence("odd")
    for i in range(5):
        n_adc = 21 + 2 * i
        seq.add(2e-3, m=(-n_adc / 2, i - 2, 0), alpha=0.5 + 0.1 * i, phase=0.2 * i)
        seq.add(n_adc * 1e-5, m=(n_adc * 1.1, 0, 0), n_adc=n_adc, flags=SPOIL)
    rx = coils.loop_ring(obj, 3, ring_radius=0.2, coil_radius=0.08)
    ref = oracle.simulate(obj, seq, coils=rx)
    tol = TOL32 if precision == 32 else TOL64
    # 79 rows x 3 coils x 2 x 64 samples per slice: the 125 samples take two slices
    sliced = run(ps, obj, seq, rx, precision=precision, spins_per_lane=1,
                 max_partial_bytes=79 * 3 * 2 * (precision // 8) * 64)
    whole = run(ps, obj, seq, rx, precision=precision, spins_per_lane=1)
    per_coil(f"odd samples sliced fp{precision}", sliced, ref, tol)
    per_coil(f"odd samples whole fp{precision}", whole, ref, tol)
    plain_ref = oracle.simulate(obj, seq)
    with ps.Context(precision=precision, spins_per_lane=1) as ctx:
        batched = ctx.simulate_batch([obj, obj.take(np.arange(777))], [seq, seq])
        torch.cuda.synchronize()
        b0, b1 = (t.cpu().numpy() for t in batched)
    within(b0, plain_ref, tol)
    within(b1, oracle.simulate(obj.take(np.arange(777)), seq), tol)


def test_many_coils_and_time_slices(ps):
    """16 coils and a partial buffer small enough to force several slices:
    every coil keeps its own block of samples in each row."""
    obj = random_spins(1200, seed=40, dw_sigma_hz=40.0)
    seq = C.spoiled_gre_2d(40, 8)
    rx = coils.loop_ring(obj, 16, ring_radius=0.22, coil_radius=0.05)
    ref = oracle.simulate(obj, seq, coils=rx)
    # 1200 spins at S = 1: 5 workgroups x 1 row; 64 samples x 16 coils per slice
    sliced = run(ps, obj, seq, rx, spins_per_lane=1, max_partial_bytes=5 * 2 * 4 * 16 * 64)
    whole = run(ps, obj, seq, rx, spins_per_lane=1)
    per_coil("16 coils sliced", sliced, ref, TOL32)
    per_coil("16 coils whole", whole, ref, TOL32)


def test_empty_object_and_invalid_receive(ps):
    import torch
    obj = random_spins(5, seed=1).take(np.arange(0))
    seq = C.fid(1.0, 10, 1e-4)
    z = run(ps, obj, seq, (np.zeros((3, 0), np.float32), np.zeros((3, 0), np.float32)))
    assert z.shape == (3, 10) and np.all(z == 0)
    obj = random_spins(40, seed=2)
    with ps.Context() as ctx:
        with pytest.raises(ps.PsError) as ei:
            ctx.simulate(obj, seq, coils=(np.zeros((0, 40), np.float32), np.zeros((0, 40), np.float32)))
        assert ei.value.status == 1
        # reserved field must be zero (raw C ABI call)
        from paper_1305_6861_amd import _binding as b
        dev = ps.to_device(obj)
        sx = torch.ones(40, dtype=torch.float32, device="cuda")
        rx = b.ps_receive(1, 7, sx.data_ptr(), sx.data_ptr())
        out = torch.empty(20, dtype=torch.float64, device="cuda")
        pk = ps.pack_sequence(seq)
        o = ps._object_struct(dev)
        st = b.lib.ps_simulate_rx(ctx._h, ctypes.byref(o), ctypes.byref(pk.struct), ctypes.byref(rx),
                                  ctypes.c_void_p(out.data_ptr()), 10, None)
        assert st == 1
