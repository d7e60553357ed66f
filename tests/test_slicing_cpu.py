"""Time slicing and the readout path, planned on the host (no device): a
scheduler-test context plans a request exactly as a simulate call does, and
ps_readout_path reports the plan.  Readouts that fit a time slice of their
own stay whole (a slice closes early instead of cutting one), so a sliced
Cartesian request keeps every readout on the matrix cores and runs the
matrix-only kernel; readouts longer than the 8,192-sample run limit are cut
into near-equal runs, none short enough to leave that path (section 5.1.1:
the per-sample readout of each ADC interval, here summed over the spins as
a matrix product)."""
import math

import pytest

from workloads import Sequence, configs as C

PARTIAL_BYTES = 2 << 30          # the default bound on a slice's partial rows (ps_config)


@pytest.fixture(scope="module")
def ctx():
    import paper_1305_6861_amd as ps
    with ps.SchedulerTest() as c:
        yield c


def _samples_per_slice(n_spins: int, coils: int = 0) -> int:
    """FP32 partial rows at one spin per lane: one row per 256-spin tile (the
    four waves share each readout)."""
    rows = math.ceil(n_spins / 256)
    return PARTIAL_BYTES // (rows * 2 * 4 * max(coils, 1))


def _gre(n_read: int, n_pe: int) -> Sequence:
    """Spoiled GRE with a 1 us dwell and TE, TR stretched to fit the readout."""
    return C.spoiled_gre_2d(n_read, n_pe, dwell=1e-6, te=0.5e-6 * n_read + 1e-3, tr=1e-6 * n_read + 5e-3)


def test_slice_boundary_inside_a_readout_keeps_the_matrix_path(ctx):
    """The 3-D spin echo of Table 7.8 (56^3 spins, 128-sample readouts):
    391,290 samples per slice is not a whole number of readouts."""
    seq = C.se_3d(128, 128, 64)
    n = 56 ** 3
    per_slice = _samples_per_slice(n)
    assert per_slice % 128 != 0
    path = ctx.readout_path(n, seq, 1)
    assert path["slices"] == math.ceil(8192 / (per_slice // 128))
    assert path == {"readouts": 8192, "matrix": 8192, "matrix_only": True, "slices": path["slices"]}
    assert path["slices"] > 1


@pytest.mark.parametrize("n_read,runs", [(8192, 1), (8200, 2), (10000, 2), (20000, 3)])
def test_long_readouts_cut_into_near_equal_runs(ctx, n_read, runs):
    """Runs of at most 8,192 samples and near-equal length: an 8,200-sample
    readout is two runs of 4,100, not 8,192 and a short 8."""
    seq = _gre(n_read, 4)
    path = ctx.readout_path(4096, seq, 1)
    assert path["slices"] == 1
    assert path["readouts"] == 4 * runs
    assert path["matrix"] == 4 * runs and path["matrix_only"]


def test_readouts_longer_than_a_slice_are_still_cut(ctx):
    """A slice of 1,024 samples (2^26 spins) and 5,000-sample readouts:
    the readouts are cut at slice boundaries (the only way to bound the
    partial rows), and the pieces (1,024 samples and less) remain readouts
    of the sequence's step, all on the matrix cores here."""
    n = 1 << 26
    assert _samples_per_slice(n) == 1024
    seq = _gre(5000, 2)
    path = ctx.readout_path(n, seq, 1)
    assert path["slices"] == math.ceil(2 * 5000 / 1024)
    assert path["readouts"] >= 2 * 5
    assert path["matrix"] == path["readouts"] and path["matrix_only"]


def test_whole_readouts_start_new_slices(ctx):
    """Readouts of 300 samples into slices of 1,024 samples: three per slice
    (900 samples), never a cut one, so ceil(n / 3) slices."""
    n = 1 << 26
    seq = _gre(300, 10)
    path = ctx.readout_path(n, seq, 1)
    assert path["readouts"] == 10
    assert path["slices"] == 4
    assert path["matrix_only"]


def test_other_tilings_and_precision_report_no_matrix_readouts():
    import paper_1305_6861_amd as ps
    seq = C.se_3d(128, 8, 2)
    with ps.SchedulerTest() as c32:
        p2 = c32.readout_path(56 ** 3, seq, 2)
        assert p2["matrix"] == 0 and not p2["matrix_only"] and p2["readouts"] == 16
    with ps.SchedulerTest(precision=64) as c64:
        p1 = c64.readout_path(56 ** 3, seq, 1)
        assert p1["matrix"] == 0 and not p1["matrix_only"]
