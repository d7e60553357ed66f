"""Mutation check of the K-t oracle's pins (CPU only): each case plants one
plausible slip in a copy of oracle/kt.py, loads the copy as a module of its
own, and runs the K-t pins against it; at least one must fail.  The
unmodified source must pass them all.  (Leaving the longitudinal
configurations out of the unpruned extent is not a mutant: a longitudinal
configuration only ever sits at an order some transverse one held first.)"""
import importlib.util
import os
import tempfile

import pytest

import tests.test_oracle_kt as pins
from oracle import kt as kt_real

SRC = os.path.join(os.path.dirname(kt_real.__file__), "kt.py")

MUTANTS = {
    "shift_sign": ("(k[0] + q[0], k[1] + q[1], k[2] + q[2])", "(k[0] - q[0], k[1] - q[1], k[2] - q[2])"),
    "missing_conj": ("v = np.conj(self.F.get(mk, 0j))", "v = self.F.get(mk, 0j)"),
    "z_relaxes_with_t2": ("Z = {k: z * e1 for k, z in self.Z.items()}", "Z = {k: z * e2 for k, z in self.Z.items()}"),
    "off_resonance_sign": ("ph = complex(math.cos(self.dw * tau), -math.sin(self.dw * tau))",
                           "ph = complex(math.cos(self.dw * tau), math.sin(self.dw * tau))"),
    "rotation_transposed": ("T = _C @ _rotation(alpha, phi) @ _CI", "T = _C @ _rotation(alpha, phi).T @ _CI"),
    "pruning_keeps_everything": ("budget = 0.5 * grey_step * ref", "budget = 0.0"),
}


def _load(text, name, d):
    path = os.path.join(d, name + ".py")
    with open(path, "w") as f:
        f.write(text)
    spec = importlib.util.spec_from_file_location("kt_" + name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _failures(mod):
    saved = pins.kt
    pins.kt = mod
    failed = []
    try:
        for name in dir(pins):
            if not name.startswith("test_"):
                continue
            fn = getattr(pins, name)
            cases = [()]
            for mark in getattr(fn, "pytestmark", []):
                if mark.name == "parametrize":
                    cases = [tuple(c) if isinstance(c, (tuple, list)) else (c,) for c in mark.args[1]]
            for c in cases:
                try:
                    fn(*c)
                except (AssertionError, ValueError, KeyError, ZeroDivisionError):
                    failed.append(name)
    finally:
        pins.kt = saved
    return failed


def test_clean_kt_oracle_passes_every_pin():
    with tempfile.TemporaryDirectory() as d:
        assert _failures(_load(open(SRC).read(), "clean", d)) == []


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_every_planted_kt_mistake_is_caught(mutant):
    old, new = MUTANTS[mutant]
    src = open(SRC).read()
    assert src.count(old) == 1, f"anchor not found once: {old!r}"
    with tempfile.TemporaryDirectory() as d:
        assert _failures(_load(src.replace(old, new), mutant, d)), f"no pin detects {mutant}"
