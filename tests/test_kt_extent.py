"""Host logic (CPU): the library's spin-spacing calculator ps_kt_extent
(section 5.2, K-t formalism of section 4.2) against the K-t oracle, which
is an independent implementation of the same configuration stepping."""
import math

import numpy as np
import pytest

from oracle import kt
from workloads import Sequence, configs as C
from tests.test_oracle_kt import _random_lattice_sequence


@pytest.fixture(scope="module")
def ps():
    import paper_1305_6861_amd as ps
    return ps


FOV = C.FOV
D2 = (1 / FOV, 1 / FOV, 0.0)


def _ssfp(n_tr):
    seq = Sequence("ssfp-like")
    for _ in range(n_tr):
        seq.add(2e-3, alpha=0.3, n_adc=1)
        seq.add(6e-3, m=(1.0, 0, 0))
    return seq


CASES = {
    "gre": (lambda: C.spoiled_gre_2d(32, 12), D2, 1.0, 0.1),
    "se": (lambda: C.spin_echo_2d(32, 12), D2, 1.0, 0.1),
    "tse": (lambda: C.tse_2d(32, 8), D2, 1.2, 0.08),
    "epi": (lambda: C.epi_2d(16), D2, 1.0, 0.05),
    "ssfp": (lambda: _ssfp(60), (1.0, 0.0, 0.0), 0.5, 0.02),
    "se3d": (lambda: C.se_3d(16, 8, 4), (1 / FOV, 1 / FOV, 1 / FOV), 0.9, 0.1),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("grey", [0.0, 1 / 256, 1 / 4096])
def test_matches_the_kt_oracle(ps, name, grey):
    make, dk, t1, t2 = CASES[name]
    seq = make()
    got = ps.kt_extent(seq, dk, t1, t2, grey_step=grey)
    want = kt.extent(seq, dk, t1, t2, grey_step=grey if grey > 0 else None)
    np.testing.assert_allclose(got["k_max"], want, rtol=0, atol=1e-9)
    np.testing.assert_allclose(got["dx_max"], kt.max_spacing(want))
    assert got["n_configs_peak"] >= 1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_lattice_sequences(ps, seed):
    rng = np.random.default_rng(seed)
    dk = (37.0, 23.0, 11.0)
    seq = _random_lattice_sequence(rng, dk)
    for grey in (0.0, 1 / 256):
        got = ps.kt_extent(seq, dk, 0.8, 0.09, grey_step=grey)
        want = kt.extent(seq, dk, 0.8, 0.09, grey_step=grey if grey > 0 else None)
        np.testing.assert_allclose(got["k_max"], want, rtol=0, atol=1e-9)


def test_known_extents_and_spin_counts(ps):
    r = ps.kt_extent(C.spoiled_gre_2d(32, 12), D2, 1.0, 0.1)
    np.testing.assert_allclose(r["k_max"], [17 / FOV, 6 / FOV, 0.0])
    assert math.isinf(r["dx_max"][2])
    assert ps.min_spins((FOV, FOV, 0.0), r["dx_max"]) == 34 * 12


def test_errors(ps):
    with pytest.raises(ps.PsError) as ei:                 # radial spokes leave the lattice
        ps.kt_extent(C.radial_2d(16, 8), D2, 1.0, 0.1)
    assert ei.value.status == 1
    with pytest.raises(ps.PsError):
        ps.kt_extent(C.spoiled_gre_2d(16, 4), (1 / FOV, 0.0, 0.0), 1.0, 0.1)   # y moments, no y step
    with pytest.raises(ps.PsError):
        ps.kt_extent(C.spoiled_gre_2d(16, 4), D2, 0.0, 0.1)
    with pytest.raises(ps.PsError):
        ps.kt_extent(C.spoiled_gre_2d(16, 4), D2, 1.0, 0.1, grey_step=-1.0)
