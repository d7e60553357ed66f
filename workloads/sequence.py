"""Pulse sequences as lists of elementary sequences (section 4.1).

An elementary sequence ("Elementarsequenz", section 4.1, eq. 4.1) is an
interval of length dt >= 0 that starts with a hard RF pulse and carries a
gradient of fixed functional form; data may be acquired during it.  The
gradient enters the Bloch solution only through its time integral
(eq. 3.14-3.17), so each interval stores its gradient moment directly, in
cycles/m: m = (gamma / 2 pi) * integral of G over the interval (eq. 3.16).

Field layout (one entry per elementary sequence):

  dt        float64  seconds, >= 0
  m         float64  (n, 3) gradient moment over the whole interval, cycles/m
  rf_alpha  float64  flip angle of the hard pulse at the interval start, rad
  rf_phase  float64  phase of that pulse's rotation axis in the x'y' plane, rad
  rf_shape  int32    -1, or index of a Shape that runs before the hard pulse
  n_adc     int64    0, or N: the interval is cut into N equal sub-steps and
                     one sample is taken after each (section 5.1.1)
  flags     uint32   SPOIL: transverse magnetisation is set to zero at the
                     end of the interval (an idealised spoiler; an extension,
                     the paper has no such primitive)
                     SNAPSHOT: the magnetisation of every spin is recorded at
                     the end of the interval, after a spoiler (section 7.2)

A Shape (eq. 3.23, hard-pulse approximation of a modulated pulse) is n_sub
equal sub-steps of length tau, each a hard pulse (alpha_i, phase_i + the
event's rf_phase) followed by precession under the per-sub-step moment m_sub.

A Trajectory replaces the equal ADC sub-steps of an interval by explicit
sample instants: sample s is taken t[s] seconds after the interval start,
when the gradient moment accumulated since the start is k[s] (cycles/m);
the interval still ends after dt with total moment m.  An event refers to
one with trajectory = index (n_adc must equal its length); -1 means the
equal sub-steps of section 5.1.1.  Piecewise-constant gradients sampled on
any raster (spirals, curved or variable-rate readouts) fit this form.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence as _Seq

import numpy as np

SPOIL = 1
SNAPSHOT = 2


@dataclasses.dataclass
class Shape:
    tau: float                       # s per sub-step
    m_sub: np.ndarray                # (3,) cycles/m per sub-step
    alpha: np.ndarray                # (n_sub,) rad, signed
    phase: np.ndarray                # (n_sub,) rad

    def __post_init__(self):
        self.m_sub = np.asarray(self.m_sub, dtype=np.float64).reshape(3)
        self.alpha = np.ascontiguousarray(self.alpha, dtype=np.float64)
        self.phase = np.ascontiguousarray(self.phase, dtype=np.float64)
        if self.alpha.shape != self.phase.shape or self.alpha.ndim != 1:
            raise ValueError("shape alpha/phase must be 1-D arrays of equal length")

    @property
    def n_sub(self) -> int:
        return int(self.alpha.shape[0])


@dataclasses.dataclass
class Trajectory:
    k: np.ndarray                    # (n, 3) cycles/m accumulated since the interval start
    t: np.ndarray                    # (n,) s since the interval start, increasing

    def __post_init__(self):
        self.k = np.ascontiguousarray(self.k, dtype=np.float64).reshape(-1, 3)
        self.t = np.ascontiguousarray(self.t, dtype=np.float64).reshape(-1)
        if self.k.shape[0] != self.t.shape[0] or self.t.shape[0] < 1:
            raise ValueError("trajectory k must be (n, 3) and t (n,), n >= 1")

    @property
    def n(self) -> int:
        return int(self.t.shape[0])


class Sequence:
    """Growable list of elementary sequences plus shape and trajectory libraries."""

    def __init__(self, name: str = "seq"):
        self.name = name
        self._rows: List[tuple] = []
        self.shapes: List[Shape] = []
        self.trajectories: List[Trajectory] = []
        self.meta: dict = {}
        self._frozen = None

    # -- building -----------------------------------------------------------
    def add(self, dt: float, m=(0.0, 0.0, 0.0), alpha: float = 0.0, phase: float = 0.0,
            shape: int = -1, n_adc: int = 0, flags: int = 0, trajectory: int = -1) -> "Sequence":
        m = tuple(float(v) for v in m)
        if len(m) != 3:
            raise ValueError("moment must have 3 components")
        self._rows.append((float(dt), m, float(alpha), float(phase), int(shape),
                           int(n_adc), int(flags), int(trajectory)))
        self._frozen = None
        return self

    def add_shape(self, shape: Shape) -> int:
        self.shapes.append(shape)
        self._frozen = None
        return len(self.shapes) - 1

    def add_trajectory(self, traj: Trajectory) -> int:
        self.trajectories.append(traj)
        self._frozen = None
        return len(self.trajectories) - 1

    # -- array views ----------------------------------------------------------
    def _freeze(self):
        if self._frozen is None:
            n = len(self._rows)
            dt = np.empty(n, np.float64)
            m = np.empty((n, 3), np.float64)
            a = np.empty(n, np.float64)
            p = np.empty(n, np.float64)
            s = np.empty(n, np.int32)
            na = np.empty(n, np.int64)
            fl = np.empty(n, np.uint32)
            tr = np.empty(n, np.int32)
            for i, (dti, mi, ai, pi, si, ni, fi, ti) in enumerate(self._rows):
                dt[i] = dti; m[i] = mi; a[i] = ai; p[i] = pi
                s[i] = si; na[i] = ni; fl[i] = fi; tr[i] = ti
            self._frozen = dict(dt=dt, m=m, rf_alpha=a, rf_phase=p, rf_shape=s,
                                n_adc=na, flags=fl, trajectory=tr)
        return self._frozen

    @property
    def n_events(self) -> int:
        return len(self._rows)

    @property
    def dt(self) -> np.ndarray: return self._freeze()["dt"]
    @property
    def m(self) -> np.ndarray: return self._freeze()["m"]
    @property
    def rf_alpha(self) -> np.ndarray: return self._freeze()["rf_alpha"]
    @property
    def rf_phase(self) -> np.ndarray: return self._freeze()["rf_phase"]
    @property
    def rf_shape(self) -> np.ndarray: return self._freeze()["rf_shape"]
    @property
    def n_adc(self) -> np.ndarray: return self._freeze()["n_adc"]
    @property
    def flags(self) -> np.ndarray: return self._freeze()["flags"]
    @property
    def trajectory(self) -> np.ndarray: return self._freeze()["trajectory"]

    @property
    def n_samples(self) -> int:
        return int(self.n_adc.sum()) if self.n_events else 0

    @property
    def n_steps_per_spin(self) -> int:
        """Intervals per spin after cutting ADC intervals into their sample
        sub-steps and shaped pulses into their sub-pulses."""
        if not self.n_events:
            return 0
        steps = int(np.maximum(self.n_adc, 1).sum())
        for s in self.rf_shape:
            if s >= 0:
                steps += self.shapes[int(s)].n_sub
        for e, j in enumerate(self.trajectory):       # the piece after a table's last sample
            if j >= 0 and self.trajectories[int(j)].t[-1] < self.dt[e]:
                steps += 1
        return steps

    def truncated(self, n_events: int) -> "Sequence":
        """The first n_events elementary sequences (same shape library)."""
        out = Sequence(self.name + f"[:{n_events}]")
        out._rows = list(self._rows[:n_events])
        out.shapes = list(self.shapes)
        out.trajectories = list(self.trajectories)
        out.meta = dict(self.meta)
        return out

    def __repr__(self):
        return (f"Sequence({self.name!r}, events={self.n_events}, samples={self.n_samples}, "
                f"shapes={len(self.shapes)})")


def concat(seqs: _Seq[Sequence], name: Optional[str] = None) -> Sequence:
    """Sequences played back to back (shape indices are remapped)."""
    out = Sequence(name or "+".join(s.name for s in seqs))
    for s in seqs:
        base = len(out.shapes)
        tbase = len(out.trajectories)
        out.shapes.extend(s.shapes)
        out.trajectories.extend(s.trajectories)
        for (dt, m, a, p, sh, na, fl, tr) in s._rows:
            out._rows.append((dt, m, a, p, sh + base if sh >= 0 else -1, na, fl, tr + tbase if tr >= 0 else -1))
    return out
