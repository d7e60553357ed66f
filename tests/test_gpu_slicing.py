"""Time slicing does not change a result (GPU).

A request whose partial rows exceed the context's bound runs as several
time slices; a slice hands the spins' anchors (and any propagator slot) to
the next through the slice state in the stepping precision, exactly the
values the registers held, and readouts that fit a slice of their own are
never cut.  So the signal of a request is bitwise the same in one slice and
in many, on the matrix-core readout (FP32, one spin per lane), the vector
readout and FP64 alike (the per-sample readout of each ADC interval,
section 5.1.1, summed over the spins, eq. 3.32).  Each case also matches
the FP64 oracle by the measures of section 5.4.2.
"""
import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import Sequence, SPOIL, configs as C
from workloads.phantom import random_spins

pytestmark = pytest.mark.gpu

TOL = {32: 1e-5, 64: 1e-12}


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


def run(ps, obj, seq, precision, max_partial_bytes, **kw):
    import torch
    with ps.Context(precision=precision, max_partial_bytes=max_partial_bytes, **kw) as ctx:
        n_slices = ctx.readout_path(obj.n_spins, seq, kw.get("spins_per_lane", 1))["slices"]
        out = ctx.simulate(obj, seq)
        torch.cuda.synchronize()
        return out.cpu().numpy(), n_slices


def spin_echo(n_adc, n_rep):
    """Spin echoes of n_adc-sample readouts with a varying phase encode."""
    seq = Sequence(f"se{n_adc}")
    for r in range(n_rep):
        seq.add(2e-3, alpha=np.pi / 2)
        seq.add(1e-3, m=(-(n_adc // 2 + 1) * 1.1, 2.5 * (r - n_rep // 2), 0.3), alpha=np.pi, phase=np.pi / 2)
        seq.add(n_adc * 1e-5, m=(n_adc * 1.1, 0.0, 0.0), n_adc=n_adc)
        seq.add(5e-3, flags=SPOIL)
    return seq


@pytest.mark.parametrize("precision,kw", [(32, {}), (32, {"matrix_readout": False}), (64, {})],
                         ids=["matrix", "vector", "fp64"])
def test_slices_leave_the_signal_bitwise_unchanged(ps, precision, kw):
    # 1,000 spins (4 tiles at one spin per lane), 100-sample readouts, and
    # a partial-row bound of 350 samples per slice: slices close after three
    # readouts instead of cutting the fourth
    obj = random_spins(1000, seed=71)
    seq = spin_echo(100, 24)
    real = 4 if precision == 32 else 8
    rows = 4                                     # one row per 256-spin tile at one spin per lane
    per_sample = rows * 2 * real
    small = 350 * per_sample                     # 350 samples per slice: 3 readouts
    whole, n1 = run(ps, obj, seq, precision, 1 << 30, spins_per_lane=1, **kw)
    sliced, n2 = run(ps, obj, seq, precision, small, spins_per_lane=1, **kw)
    assert n1 == 1 and n2 == 8, (n1, n2)
    assert np.array_equal(whole, sliced), "slicing changed the signal"
    within(whole, oracle.simulate(obj, seq), TOL[precision], f"{precision} {kw} sliced")


def test_slices_with_a_cached_shaped_pulse(ps):
    """The c3 recipe at 2 x 16^3 spins with 128-sample readouts (the
    matrix-only kernel): the sinc's propagator, filled in the first slice,
    reaches the later ones through the slice state."""
    obj, _ = C.c3(16)
    seq = C.gre_3d_sinc(128, 8, 3)
    rows = (obj.n_spins + 255) // 256            # one row per 256-spin tile
    small = 3 * 128 * rows * 2 * 4               # three readouts per slice
    whole, n1 = run(ps, obj, seq, 32, 1 << 30, spins_per_lane=1)
    sliced, n2 = run(ps, obj, seq, 32, small, spins_per_lane=1)
    assert n1 == 1 and n2 == 8, (n1, n2)
    assert np.array_equal(whole, sliced), "slicing changed the signal"
    within(whole, oracle.simulate(obj, seq), TOL[32], "c3 recipe sliced")
