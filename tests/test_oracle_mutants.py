"""Mutation check of the oracle's pins (CPU only).

Each case copies the oracle's C source, plants one plausible slip (a wrong
sign, a transposed entry, a dropped term, swapped relaxation times, an
off-by-one in the ADC sub-step, an ignored flag ...), compiles the copy into
a temporary directory and runs the pin suite against it.  At least one pin
must fail for every mutant; the unmodified source must pass them all.  The
planted mistakes live only in the temporary copies.
"""
import os
import tempfile

import pytest

import oracle
from oracle import build as obuild
import tests.test_oracle_coils as coil_pins
import tests.test_oracle_pins as pins
import tests.test_oracle_snapshots as snapshot_pins
import tests.test_oracle_trajectory as trajectory_pins

PIN_MODULES = (pins, coil_pins, snapshot_pins, trajectory_pins)

MUTANTS = {
    "rf_sign_r02": ("r02 = -sp * sa", "r02 = sp * sa"),
    "rf_transposed_row": ("M[2] = r20 * mx + r21 * my + r22 * mz;",
                          "M[2] = r02 * mx + r12 * my + r22 * mz;"),
    "rf_cos_sin_swapped": ("double ca = cos(alpha), sa = sin(alpha);",
                           "double ca = sin(alpha), sa = cos(alpha);"),
    "precession_sense": ("M[0] = e2 * (c * mx + s * my);", "M[0] = e2 * (c * mx - s * my);"),
    "no_t1_recovery": ("M[2] = e1 * M[2] + m0 * (1.0 - e1);", "M[2] = e1 * M[2];"),
    "t1_t2_swapped": ("double e1 = exp(-tau / t1), e2 = exp(-tau / t2);",
                      "double e1 = exp(-tau / t2), e2 = exp(-tau / t1);"),
    "e2_on_one_component": ("M[1] = e2 * (-s * mx + c * my);", "M[1] = (-s * mx + c * my);"),
    "missing_two_pi": ("double theta = two_pi * (", "double theta = ("),
    "dw_sign": ("+ dw * tau;", "- dw * tau;"),
    "y_z_swapped": ("mu[1] * y + mu[2] * z", "mu[1] * z + mu[2] * y"),
    "adc_substep_off_by_one": ("double tau = pb->ev_dt[e] / (double)K;",
                               "double tau = pb->ev_dt[e] / (double)(K + 1);"),
    "spoil_ignored": ("if (pb->ev_flags[e] & ORACLE_SPOIL) {", "if (0) {"),
    "shape_phase_offset_dropped": ("pb->sh_phase[off + k] + pb->ev_phase[e]", "pb->sh_phase[off + k]"),
    "sample_records_mz": ("signal[2 * sample + 1] += M[1];", "signal[2 * sample + 1] += M[2];"),
    "coil_imag_sign": ("sc[2 * sample + 1] += sx * M[1] - sy * M[0];",
                       "sc[2 * sample + 1] += sx * M[1] + sy * M[0];"),
    "coil_real_drops_sy": ("sc[2 * sample] += sx * M[0] + sy * M[1];", "sc[2 * sample] += sx * M[0];"),
    "coil_sx_sy_swapped": ("double sx = pb->s_x[c * pb->n_spins + i], sy = pb->s_y[c * pb->n_spins + i];",
                           "double sx = pb->s_y[c * pb->n_spins + i], sy = pb->s_x[c * pb->n_spins + i];"),
    "coil_index_ignores_coil": ("double sx = pb->s_x[c * pb->n_spins + i], sy = pb->s_y[c * pb->n_spins + i];",
                                "double sx = pb->s_x[i], sy = pb->s_y[i];"),
    "coil_block_offset": ("double *sc = signal + 2 * pb->n_samples * c;",
                          "double *sc = signal + pb->n_samples * c;"),
    "snapshot_components_reversed": ("pb->snap[(3 * snap + c) * pb->n_spins + i] = M[c];",
                                     "pb->snap[(3 * snap + c) * pb->n_spins + i] = M[2 - c];"),
    "snapshot_index_stuck": ("            ++snap;\n", "\n"),
    "traj_last_piece_dropped": ("precess_relax(M, pb->ev_dt[e] - t_prev, mu, x, y, z, dw, m0, t1, t2);", ""),
    "traj_moment_not_differenced": (
        "double mu[3] = {tk[3 * q] - k_prev[0], tk[3 * q + 1] - k_prev[1], tk[3 * q + 2] - k_prev[2]};",
        "double mu[3] = {tk[3 * q], tk[3 * q + 1], tk[3 * q + 2]};"),
    "traj_time_not_differenced": ("precess_relax(M, tt[q] - t_prev, mu", "precess_relax(M, tt[q], mu"),
    "snapshot_spin_major": ("pb->snap[(3 * snap + c) * pb->n_spins + i] = M[c];",
                            "pb->snap[3 * snap * pb->n_spins + 3 * i + c] = M[c];"),
}


def _pin_functions():
    out = []
    for mod in PIN_MODULES:
        out.extend(_module_pins(mod))
    return out


def _module_pins(mod):
    out = []
    for name in dir(mod):
        if not name.startswith("test_"):
            continue
        fn = getattr(mod, name)
        params = getattr(fn, "pytestmark", [])
        cases = [()]
        for mark in params:
            if mark.name == "parametrize":
                cases = [tuple(c) if isinstance(c, (tuple, list)) else (c,) for c in mark.args[1]]
        out.extend((name, fn, c) for c in cases)
    return out


def _run_pins():
    """Names of pins that fail with the currently loaded oracle library."""
    failed = []
    for name, fn, case in _pin_functions():
        try:
            fn(*case)
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(name)
    return failed


@pytest.fixture(scope="module")
def workdir():
    with tempfile.TemporaryDirectory(prefix="oracle_mut_") as d:
        yield d


def _with_lib(path):
    saved = oracle._lib
    oracle._lib = oracle.load_library(path)
    try:
        return _run_pins()
    finally:
        oracle._lib = saved


def test_unmodified_oracle_passes_every_pin(workdir):
    with open(obuild.SRC) as f:
        src = f.read()
    p = os.path.join(workdir, "clean.c")
    with open(p, "w") as f:
        f.write(src)
    lib = obuild.build(src=p, out=os.path.join(workdir, "clean.so"))
    assert _with_lib(lib) == []


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_every_planted_mistake_is_caught(mutant, workdir):
    old, new = MUTANTS[mutant]
    with open(obuild.SRC) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation anchor not found once: {old!r}"
    p = os.path.join(workdir, mutant + ".c")
    with open(p, "w") as f:
        f.write(src.replace(old, new))
    lib = obuild.build(src=p, out=os.path.join(workdir, mutant + ".so"))
    failed = _with_lib(lib)
    assert failed, f"no pin detects mutant {mutant}"
