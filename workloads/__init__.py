"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds *inputs only*: spin objects (positions, rho/T1/T2 and
off-resonance arrays) and pulse sequences expressed as lists of elementary
sequences.  It contains none of the Bloch arithmetic of the method itself, so
that the FP64 oracle and the GPU path can both consume it without sharing any
code that computes a result.

Object model (section 6.1.1): every spin has a position, a rest magnetisation
M0, relaxation times T1 and T2, and an off-resonance angular frequency that
collects chemical shift, B0 inhomogeneity and susceptibility (eq. 6.1 / 6.2).

Sequence model (section 4.1, section 6.1.2): a sequence is a list of elementary
sequences.  Each has a hard RF pulse at its start (flip alpha, phase phi), a
gradient whose time integral over the interval is given as a moment in
cycles/m, a duration dt >= 0, and optionally N ADC samples taken after each
of N equal sub-steps (section 5.1.1).  A shaped pulse is a reusable list of
equal-length elementary sequences (hard-pulse approximation, eq. 3.23).

Receive coils (section 3.5.1): sensitivity maps S = B1 / i of circular
loops (coils.py), inputs for multi-coil signals.
"""
from .sequence import Sequence, Shape, Trajectory, SPOIL, SNAPSHOT, concat
from .phantom import SpinObject, grid2d, grid3d_two_species, subset
from . import coils, configs

__all__ = [
    "Sequence", "Shape", "Trajectory", "SPOIL", "SNAPSHOT", "concat",
    "SpinObject", "grid2d", "grid3d_two_species", "subset",
    "coils", "configs",
]
