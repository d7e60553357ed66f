"""GPU: readout replicas for objects too small to fill the device.

A tile's replicas repeat its RF / shaped-pulse stepping and share its
readouts; every sample is computed once by the same arithmetic, so the
signal (and every snapshot) is bitwise that of the unsplit launch.  Checked
on small requests of every kind, plus the oracle bar."""
import numpy as np
import pytest

import oracle
from tests.parity import within
from workloads import SNAPSHOT, coils, configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


@pytest.mark.parametrize("case", ["c2", "epi", "tse", "radial", "c3", "c1"])
def test_split_is_bitwise_unsplit(ps, case):
    if case == "c2":
        obj, seq = C.c2(28)
    elif case == "c3":
        obj, _ = C.c3(10)
        seq = C.gre_3d_sinc(10, 3, 3)
    elif case == "c1":
        obj, seq = C.c1()
    else:
        obj, seq = C.table78(case, scale=4)
    res = {}
    for split in (True, False):
        for prec in (32, 64):
            with ps.Context(readout_split=split, precision=prec) as ctx:
                res[split, prec] = ctx.simulate(obj, seq).cpu().numpy()
    for prec in (32, 64):
        np.testing.assert_array_equal(res[True, prec], res[False, prec])
    ref = oracle.simulate(obj, seq)
    within(res[True, 32], ref, 1e-5, f"split {case} spins={obj.n_spins}")
    within(res[True, 64], ref, 1e-12, f"split {case} spins={obj.n_spins} fp64")


def test_split_with_coils_snapshots_and_slices(ps):
    obj, _ = C.c3(10)
    seq0 = C.gre_3d_sinc(10, 3, 3)
    from tests.test_gpu_snapshots import with_snapshots
    adc = set(np.nonzero(seq0.n_adc > 0)[0].tolist())
    seq = with_snapshots(seq0, lambda e: e in adc)
    rx = coils.loop_ring(obj, 2, ring_radius=0.2, coil_radius=0.06)
    res = {}
    for split in (True, False):
        with ps.Context(readout_split=split, spins_per_lane=1, max_partial_bytes=8 * 2 * 4 * 2 * 64) as ctx:
            sig, snap = ctx.simulate(obj, seq, coils=rx, snapshots=True)
            res[split] = (sig.cpu().numpy(), snap.cpu().numpy())
    np.testing.assert_array_equal(res[True][0], res[False][0])
    np.testing.assert_array_equal(res[True][1], res[False][1])


def test_tail_split_of_a_large_object(ps):
    """More tiles than the device holds workgroups at once: the tiles of the
    whole rounds run whole and only the rest (which would leave the last
    round part-empty) are split into replicas.  1,000 tiles at one spin per
    lane (256,000 spins) with 12 readouts of 160 samples, in FP32 and FP64,
    in one launch and in five time slices; bitwise equal to the unsplit
    launch and within the oracle bars."""
    from workloads.phantom import random_spins
    from tests.test_gpu_matrix_readout import cartesian
    obj = random_spins(256000, seed=77, dw_sigma_hz=30.0)
    seq = cartesian(160, 12)
    ref = oracle.simulate(obj, seq)
    for prec, tol in ((32, 1e-5), (64, 1e-12)):
        # whole, and in five time slices of 400 samples: the split tiles'
        # replicas then start from the anchors that replica 0 of the
        # previous slice wrote to the other anchor buffer
        rows = 1000
        for part in (0, rows * 2 * (prec // 8) * 400):
            res = {}
            for split in (True, False):
                with ps.Context(readout_split=split, spins_per_lane=1, precision=prec,
                                max_partial_bytes=part) as ctx:
                    res[split] = ctx.simulate(obj, seq).cpu().numpy()
            np.testing.assert_array_equal(res[True], res[False])
            within(res[True], ref, tol, f"tail split 1000 tiles fp{prec} partial={part}")
