"""GPU: magnetisation snapshots (ps_simulate_ex, section 7.2) against the FP64
oracle.  Snapshots are compared over the whole (snapshot, component, spin)
array by relative L2 error; the signal of a run with snapshots is bitwise
that of the same run without them."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import Sequence, SNAPSHOT, SPOIL, coils, configs as C
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
        sig, snap = ctx.simulate(obj, seq, coils=rx, snapshots=True)
        torch.cuda.synchronize()
        return sig.cpu().numpy(), snap.cpu().numpy().astype(np.float64)


def plain(ps, obj, seq, rx=None, **kw):
    import torch
    with ps.Context(**kw) as ctx:
        sig = ctx.simulate(obj, seq, coils=rx)
        torch.cuda.synchronize()
        return sig.cpu().numpy()


def with_snapshots(seq, every_tr_event=None):
    """Copy of seq with SNAPSHOT on events whose index satisfies the predicate."""
    out = Sequence(seq.name + "+snap")
    for sh in seq.shapes:
        out.add_shape(sh)
    for e in range(seq.n_events):
        f = int(seq.flags[e]) | (SNAPSHOT if every_tr_event(e) else 0)
        out.add(seq.dt[e], m=seq.m[e], alpha=seq.rf_alpha[e], phase=seq.rf_phase[e], shape=int(seq.rf_shape[e]),
                n_adc=int(seq.n_adc[e]), flags=f)
    return out


def check(label, got, ref, tol):
    within(got, ref, tol, f"snapshots {label} shape={ref.shape}")


def test_free_precession_and_recovery(ps):
    obj = random_spins(777, seed=51, dw_sigma_hz=80.0)
    seq = Sequence("fid-snap")
    seq.add(1.3e-3, alpha=math.pi / 2, flags=SNAPSHOT)
    seq.add(2.2e-3, m=(40.0, -10.0, 5.0), flags=SNAPSHOT)
    seq.add(0.3, alpha=math.pi, phase=0.4, flags=SPOIL | SNAPSHOT)
    _, ref = oracle.simulate(obj, seq, snapshots=True)
    for prec, tol in ((32, TOL32), (64, TOL64)):
        sig, snap = run(ps, obj, seq, precision=prec)
        assert sig.size == 0
        check(f"fid/ir fp{prec}", snap, ref, tol)


def test_spin_echo_snapshots_every_repetition(ps):
    obj, seq0 = C.c2(20)
    tr_ends = set(np.nonzero(seq0.flags & SPOIL)[0].tolist())
    seq = with_snapshots(seq0, lambda e: e in tr_ends)
    ref_sig, ref = oracle.simulate(obj, seq, snapshots=True)
    for prec, tol in ((32, TOL32), (64, TOL64)):
        sig, snap = run(ps, obj, seq, precision=prec)
        check(f"c2[20] fp{prec}", snap, ref, tol)
        np.testing.assert_array_equal(sig, plain(ps, obj, seq0, precision=prec))


def test_snapshots_with_shapes_coils_slices_and_ragged_spins(ps):
    obj, _ = C.c3(10)
    obj = obj.take(np.arange(obj.n_spins - 37))                 # ragged tail
    seq0 = C.gre_3d_sinc(10, 3, 3)
    adc = set(np.nonzero(seq0.n_adc > 0)[0].tolist())
    seq = with_snapshots(seq0, lambda e: e in adc or e == 0)
    rx = coils.loop_ring(obj, 2, ring_radius=0.2, coil_radius=0.06)
    ref_sig, ref = oracle.simulate(obj, seq, coils=rx, snapshots=True)
    for kw in ({}, {"shape_cache": False}, {"spins_per_lane": 1, "max_partial_bytes": 8 * 2 * 4 * 2 * 64}):
        sig, snap = run(ps, obj, seq, rx, **kw)
        check(f"c3[10] {kw}", snap, ref, TOL32)
        for c in range(2):
            within(sig[c], ref_sig[c], TOL32)
        np.testing.assert_array_equal(sig, plain(ps, obj, seq0, rx, **kw))


def test_empty_object_and_count_mismatch(ps):
    import torch
    seq = Sequence("s")
    seq.add(1e-3, alpha=1.0, n_adc=4, flags=SNAPSHOT)
    empty = random_spins(3, seed=1).take(np.arange(0))
    sig, snap = run(ps, empty, seq)
    assert snap.shape == (1, 3, 0) and sig.shape == (4,) and np.all(sig == 0)
    obj = random_spins(100, seed=2)
    with ps.Context() as ctx:
        from paper_1305_6861_amd import _binding as b
        dev = ps.to_device(obj)
        pk = ps.pack_sequence(seq)
        assert pk.count_snapshots() == 1
        out = torch.empty(8, dtype=torch.float64, device="cuda")
        buf = torch.empty(3 * 100 * 2, dtype=torch.float32, device="cuda")
        o = ps._object_struct(dev)
        st = b.lib.ps_simulate_ex(ctx._h, ctypes.byref(o), ctypes.byref(pk.struct), None,
                                  ctypes.c_void_p(out.data_ptr()), 4, ctypes.c_void_p(buf.data_ptr()), 2, None)
        assert st == 1                                            # n_snapshots differs
        st = b.lib.ps_simulate_ex(ctx._h, ctypes.byref(o), ctypes.byref(pk.struct), None,
                                  ctypes.c_void_p(out.data_ptr()), 4, None, 1, None)
        assert st == 1                                            # NULL buffer
