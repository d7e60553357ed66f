"""GPU K-t engine (ps_kt_simulate, sections 4.2 - 4.4 and 5.1.2, eq. 4.19)
against the two oracles: the isochromat oracle on the same spins given
their tissue's T1, T2 and off-resonance (for lattice sequences the two
methods give the same signal), and the K-t oracle (configuration
populations in plain Python, eq. 4.19 summed per tissue).  Box voxels are
pinned by the continuum limit: isochromats on m x m sub-cells of each voxel
sum to the voxel's spectrum times a Dirichlet kernel, which tends to the
sinc with an error series in 1 / m^2, so a Richardson combination of m = 16
and m = 32 matches the engine's voxel-integrated signal."""
import math

import numpy as np
import pytest

import oracle
from oracle import kt as ktor
from tests.parity import within
from workloads import Sequence, Shape, SPOIL, configs as C
from workloads.phantom import kt_phantom_2d

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12
FOV = 0.25


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


def _kt(ctx, ph, seq, dk, voxel=(0.0, 0.0, 0.0)):
    import torch
    obj, begin, t1, t2, dw, _ = ph
    out = ctx.kt_simulate(obj, begin, t1, t2, dw, seq, dk, voxel=voxel)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_spoiled_gre_against_both_oracles(ps):
    ph = kt_phantom_2d(32, FOV)
    obj, begin, t1, t2, dw, _ = ph
    seq = C.spoiled_gre_2d(32, 32, FOV)
    dk = (1 / FOV, 1 / FOV, 0.0)
    ref = oracle.simulate(obj, seq)
    kt_ref = sum(ktor.signal(obj.take(np.arange(begin[c], begin[c + 1])), seq, dk, t1[c], t2[c], dw[c])
                 for c in range(len(t1)))
    within(kt_ref, ref, 1e-12, "K-t oracle vs isochromat oracle", precision=64)
    with ps.Context(precision=32) as c32:
        within(_kt(c32, ph, seq, dk), ref, TOL32, "kt gre32 fp32")
    with ps.Context(precision=64) as c64:
        within(_kt(c64, ph, seq, dk), ref, TOL64, "kt gre32 fp64")


def test_spin_echo_off_resonance_and_shaped_pulse(ps):
    """Spin echo with per-tissue off-resonance, then the same object under a
    non-selective shaped excitation (sub-steps with a lattice moment on z)."""
    ph = kt_phantom_2d(24, FOV)
    obj = ph[0]
    se = C.spin_echo_2d(24, 24, FOV)
    dk = (1 / FOV, 1 / FOV, 0.0)
    with ps.Context() as ctx:
        within(_kt(ctx, ph, se, dk), oracle.simulate(obj, se), TOL32, "kt se24")
        seq = Sequence("shaped")
        u = (np.arange(16) + 0.5) / 16 - 0.5
        a = np.sinc(3 * u)
        sid = seq.add_shape(Shape(tau=20e-6, m_sub=(0.0, 0.0, 2.0), alpha=0.5 * a / a.sum(),
                                  phase=np.linspace(0, 0.3, 16)))
        for j in range(12):
            seq.add(2e-3, m=(-7 / FOV, (j - 6) / FOV, -16.0), shape=sid, phase=0.4 * j)
            seq.add(12 * 10e-6, m=(12 / FOV, 0.0, 0.0), n_adc=12)
            seq.add(5e-3, flags=SPOIL)
        dk3 = (1 / FOV, 1 / FOV, 2.0)
        within(_kt(ctx, ph, seq, dk3), oracle.simulate(obj, seq), TOL32, "kt shaped")


def test_unspoiled_sequence_with_many_configurations(ps):
    """Three pulses without spoiling and gradients between them: stimulated
    and secondary echoes, many configurations per sample."""
    ph = kt_phantom_2d(24, FOV)
    obj = ph[0]
    seq = Sequence("multi_echo")
    for r in range(4):
        seq.add(3e-3, m=(5 / FOV, 2 / FOV, 0.0), alpha=math.radians(90 - 15 * r), phase=0.7 * r)
        seq.add(32 * 10e-6, m=(32 / FOV, -32 / FOV, 0.0), n_adc=32)
        seq.add(2e-3, m=(-9 / FOV, 3 / FOV, 0.0))
    dk = (1 / FOV, 1 / FOV, 0.0)
    ref = oracle.simulate(obj, seq)
    with ps.Context() as ctx:
        within(_kt(ctx, ph, seq, dk), ref, TOL32, "kt unspoiled")
    with ps.Context(precision=64) as ctx:
        within(_kt(ctx, ph, seq, dk), ref, TOL64, "kt unspoiled fp64")


def test_box_voxels_match_the_continuum_limit(ps):
    """8 x 8 voxels of the FOV / 8 box: the engine's voxel-integrated signal
    (sinc weights) against (4 s_32 - s_16) / 3 of isochromat sums on 32 x 32
    and 16 x 16 sub-cells per voxel (both from the oracle, FP64)."""
    seq = C.spoiled_gre_2d(16, 16, FOV)
    dk = (1 / FOV, 1 / FOV, 0.0)
    s = {}
    for m in (16, 32):
        s[m] = oracle.simulate(kt_phantom_2d(8, FOV, iso_per_axis=m)[0], seq)
    extrap = (4 * s[32] - s[16]) / 3
    ph = kt_phantom_2d(8, FOV)
    d = ph[5]
    with ps.Context(precision=64) as ctx:
        got = _kt(ctx, ph, seq, dk, voxel=(d, d, 0.0))
        point = _kt(ctx, ph, seq, dk)
    err_point = oracle.rel_l2(point, extrap)
    print(f"[kt] voxel-integrated vs the continuum limit; point spins are {err_point:.2e} off", flush=True)
    within(got, extrap, 2e-5, "kt box voxels vs Richardson limit", precision=64)
    assert err_point > 100 * oracle.rel_l2(got, extrap)


def test_full_size_object_against_the_isochromat_path(ps):
    """256 x 256 grid of tissue classes under the c2-size spoiled GRE (41,689
    spins, 65,536 samples): the K-t engine against the oracle over the whole
    request, and against the GPU isochromat stepper on the same spins."""
    import time
    import torch
    ph = kt_phantom_2d(256, FOV)
    obj = ph[0]
    seq = C.spoiled_gre_2d(256, 256, FOV, dwell=10e-6)
    dk = (1 / FOV, 1 / FOV, 0.0)
    with ps.Context() as ctx:
        iso = ctx.simulate(obj, seq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        got = _kt(ctx, ph, seq, dk)
        dt = time.perf_counter() - t0
        iso = iso.cpu().numpy()
    print(f"[kt] {obj.n_spins} spins, {seq.n_samples} samples: {dt * 1e3:.1f} ms", flush=True)
    ref = oracle.simulate(obj, seq)
    within(got, ref, TOL32, "kt 256^2 GRE vs oracle")
    within(iso, ref, TOL32, "isochromat GPU 256^2 GRE vs oracle")
    within(got, iso, TOL32, "kt vs isochromat GPU, 256^2 GRE")


def test_errors_and_edges(ps):
    import torch
    ph = kt_phantom_2d(16, FOV)
    obj, begin, t1, t2, dw, _ = ph
    seq = C.spoiled_gre_2d(16, 8, FOV)
    with ps.Context() as ctx:
        with pytest.raises(ps.PsError) as ei:                 # moments off the lattice
            ctx.kt_simulate(obj, begin, t1, t2, dw, seq, (0.7 / FOV, 1 / FOV, 0.0))
        assert ei.value.status == 1
        with pytest.raises(ps.PsError):                       # ranges that do not cover the spins
            ctx.kt_simulate(obj, begin - np.array([0, 1, 1, 1, 1]), t1, t2, dw, seq, (1 / FOV, 1 / FOV, 0.0))
        with pytest.raises(ps.PsError):                       # t2 <= 0
            ctx.kt_simulate(obj, begin, t1, -t2, dw, seq, (1 / FOV, 1 / FOV, 0.0))
        tr = C.spiral_2d(2, 64, FOV, res=16)
        with pytest.raises(ps.PsError):                       # trajectory readouts
            ctx.kt_simulate(obj, begin, t1, t2, dw, tr, (1 / FOV, 1 / FOV, 0.0))
        empty = obj.take(np.arange(0))
        z = ctx.kt_simulate(empty, np.zeros(5, np.int64), t1, t2, dw, seq, (1 / FOV, 1 / FOV, 0.0))
        torch.cuda.synchronize()
        assert z.numel() == seq.n_samples and float(z.abs().max()) == 0.0
        none = Sequence("no samples").add(1e-3, alpha=1.0)
        assert ctx.kt_simulate(obj, begin, t1, t2, dw, none, (1 / FOV, 1 / FOV, 0.0)).numel() == 0
