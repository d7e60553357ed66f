"""FP64 CPU oracle of spin-based Bloch simulation -- TEST INFRASTRUCTURE.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library: the stepping is plain
C (bloch_oracle.c) following section 5.1.1 with eq. 3.19 for hard pulses,
eq. 3.5 / 3.12 / 3.14 for precession and relaxation, eq. 3.23 for shaped
pulses, eq. 3.30 - 3.32 for the received signal, eq. 3.25 for receive
coils with an inhomogeneous sensitivity, and per-sample trajectory tables
(samples at listed instants and moments inside an interval).

Inputs are duck-typed: a spin object exposes float32 arrays x, y, z, m0,
t1, t2, dw (widened exactly to float64 here), a sequence exposes the
elementary-sequence arrays dt, m, rf_alpha, rf_phase, rf_shape, n_adc,
flags and a list of shapes with tau, m_sub, alpha, phase.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import build as _build

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def _configure(lib):
    lib.oracle_simulate.restype = ctypes.c_int
    lib.oracle_simulate.argtypes = (
        [ctypes.c_int64] + [_dp] * 7 +
        [ctypes.c_int64, _dp, _dp, _dp, _dp, _i32p, _i64p, _u32p] +
        [ctypes.c_int32, _i64p, _dp, _dp, _i64p, _dp, _dp] +
        [ctypes.c_int, ctypes.c_int64, _dp, _dp])
    lib.oracle_simulate_coils.restype = ctypes.c_int
    lib.oracle_simulate_coils.argtypes = (
        [ctypes.c_int64] + [_dp] * 7 +
        [ctypes.c_int64, _dp, _dp, _dp, _dp, _i32p, _i64p, _u32p] +
        [ctypes.c_int32, _i64p, _dp, _dp, _i64p, _dp, _dp] +
        [ctypes.c_int32, _dp, _dp] +
        [ctypes.c_int, ctypes.c_int64, _dp, _dp])
    lib.oracle_simulate_full.restype = ctypes.c_int
    lib.oracle_simulate_full.argtypes = (
        [ctypes.c_int64] + [_dp] * 7 +
        [ctypes.c_int64, _dp, _dp, _dp, _dp, _i32p, _i64p, _u32p] +
        [ctypes.c_int32, _i64p, _dp, _dp, _i64p, _dp, _dp] +
        [ctypes.c_int32, _dp, _dp, _dp] +
        [ctypes.c_int, ctypes.c_int64, _dp, _dp])
    lib.oracle_simulate_traj.restype = ctypes.c_int
    lib.oracle_simulate_traj.argtypes = (
        [ctypes.c_int64] + [_dp] * 7 +
        [ctypes.c_int64, _dp, _dp, _dp, _dp, _i32p, _i64p, _u32p] +
        [ctypes.c_int32, _i64p, _dp, _dp, _i64p, _dp, _dp] +
        [ctypes.c_int32, _dp, _dp, _dp] +
        [_i32p, ctypes.c_int32, _i64p, _i64p, _dp, _dp] +
        [ctypes.c_int, ctypes.c_int64, _dp, _dp])
    lib.oracle_rf_pulse.restype = None
    lib.oracle_rf_pulse.argtypes = [_dp, ctypes.c_double, ctypes.c_double]
    lib.oracle_precess_relax.restype = None
    lib.oracle_precess_relax.argtypes = [_dp, ctypes.c_double, _dp] + [ctypes.c_double] * 7
    return lib


def load_library(path: str):
    """Load an oracle build from an explicit path (used by the mutation
    tests, which compile deliberately broken copies of the source)."""
    return _configure(ctypes.CDLL(path))


def _load():
    """The oracle library: PS_ORACLE_LIB names another build of the same
    source (the sanitizer test's); else the in-tree one, built if missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("PS_ORACLE_LIB")
    if not path:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
    _lib = _configure(ctypes.CDLL(path))
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


SNAPSHOT = 2     # event flag: record every spin's magnetisation at the end of the interval


def simulate(obj, seq, n_threads: Optional[int] = None, final_m: bool = False, coils=None,
             snapshots: bool = False):
    """Signal (complex128, one entry per ADC sample in event order) and,
    when final_m is set, the final magnetisation (n_spins, 3) float64.

    coils: optional receive sensitivities, a pair (s_x, s_y) of arrays of
    shape (n_coils, n_spins) holding the transverse components of each
    coil's sensitivity at each spin (section 3.5.1, eq. 3.24), float32 as
    the GPU library receives them; the signal is then (n_coils, n_samples),
    coil c receiving sum_i (S_x Mx + S_y My) + j (S_x My - S_y Mx).

    snapshots: also return the magnetisation of every spin at the end of
    every event flagged SNAPSHOT (section 7.2), float64 of shape
    (n_snapshots, 3, n_spins), as the last element of a tuple."""
    lib = _load()
    n = int(np.asarray(obj.x).shape[0])
    sp = [np.ascontiguousarray(np.asarray(getattr(obj, f), dtype=np.float32), dtype=np.float64)
          for f in ("x", "y", "z", "m0", "t1", "t2", "dw")]
    ne = int(seq.n_events)
    dt = np.ascontiguousarray(seq.dt, np.float64) if ne else np.zeros(0)
    m = np.ascontiguousarray(seq.m, np.float64).reshape(-1) if ne else np.zeros(0)
    al = np.ascontiguousarray(seq.rf_alpha, np.float64) if ne else np.zeros(0)
    ph = np.ascontiguousarray(seq.rf_phase, np.float64) if ne else np.zeros(0)
    sh = np.ascontiguousarray(seq.rf_shape, np.int32) if ne else np.zeros(0, np.int32)
    na = np.ascontiguousarray(seq.n_adc, np.int64) if ne else np.zeros(0, np.int64)
    fl = np.ascontiguousarray(seq.flags, np.uint32) if ne else np.zeros(0, np.uint32)
    shapes = list(seq.shapes)
    ns = len(shapes)
    sh_nsub = np.array([s.n_sub for s in shapes] or [0], np.int64)
    sh_tau = np.array([s.tau for s in shapes] or [0.0], np.float64)
    sh_m = np.array([list(s.m_sub) for s in shapes] or [[0.0, 0.0, 0.0]], np.float64).reshape(-1)
    offs = np.zeros(max(ns, 1), np.int64)
    if ns:
        offs[1:ns] = np.cumsum(sh_nsub[:ns])[:-1]
    sh_alpha = np.concatenate([s.alpha for s in shapes] + [np.zeros(1)]).astype(np.float64)
    sh_phase = np.concatenate([s.phase for s in shapes] + [np.zeros(1)]).astype(np.float64)
    n_samples = int(na.sum())
    if coils is None:
        n_coils = 0
        s_x = s_y = np.zeros(1, np.float64)
    else:
        s_x, s_y = (np.asarray(np.asarray(c, dtype=np.float32), dtype=np.float64) for c in coils)
        if s_x.ndim != 2 or s_x.shape != s_y.shape or s_x.shape[1] != n:
            raise ValueError(f"coil sensitivities must have shape (n_coils, {n})")
        n_coils = int(s_x.shape[0])
        s_x = np.ascontiguousarray(s_x).reshape(-1)
        s_y = np.ascontiguousarray(s_y).reshape(-1)
        if s_x.size == 0:
            s_x = s_y = np.zeros(1, np.float64)
    out = np.zeros(2 * n_samples * max(n_coils, 1) + 1, np.float64)
    fm = np.zeros(3 * n + 1, np.float64) if final_m else None
    n_snap = int(np.count_nonzero(fl & SNAPSHOT))
    snap = np.zeros(3 * n * n_snap + 1, np.float64) if snapshots else None
    trajs = list(getattr(seq, "trajectories", []))
    ev_tr = (np.ascontiguousarray(seq.trajectory, np.int32) if ne and hasattr(seq, "trajectory")
             else np.full(max(ne, 1), -1, np.int32))
    tr_n = np.array([t.n for t in trajs] or [0], np.int64)
    tr_off = np.zeros(max(len(trajs), 1), np.int64)
    if trajs:
        tr_off[1:len(trajs)] = np.cumsum(tr_n[:len(trajs)])[:-1]
    tr_k = np.concatenate([t.k.reshape(-1) for t in trajs] + [np.zeros(3)]).astype(np.float64)
    tr_t = np.concatenate([t.t for t in trajs] + [np.zeros(1)]).astype(np.float64)
    nt = int(n_threads or default_threads())
    rc = lib.oracle_simulate_traj(
        n, *[_ptr(a, _dp) for a in sp],
        ne, _ptr(dt, _dp), _ptr(m, _dp), _ptr(al, _dp), _ptr(ph, _dp), _ptr(sh, _i32p),
        _ptr(na, _i64p), _ptr(fl, _u32p),
        ns, _ptr(sh_nsub, _i64p), _ptr(sh_tau, _dp), _ptr(sh_m, _dp), _ptr(offs, _i64p),
        _ptr(sh_alpha, _dp), _ptr(sh_phase, _dp),
        n_coils, _ptr(s_x, _dp), _ptr(s_y, _dp), _ptr(snap, _dp) if snap is not None else None,
        _ptr(ev_tr, _i32p), len(trajs), _ptr(tr_n, _i64p), _ptr(tr_off, _i64p), _ptr(tr_k, _dp), _ptr(tr_t, _dp),
        nt, n_samples, _ptr(out, _dp), _ptr(fm, _dp) if fm is not None else None)
    if rc != 0:
        raise ValueError(f"oracle_simulate failed with code {rc}")
    sig = out[:2 * n_samples * max(n_coils, 1)].view(np.complex128).copy()
    if coils is not None:
        sig = sig.reshape(n_coils, n_samples)
    res = [sig]
    if final_m:
        res.append(fm[:3 * n].reshape(n, 3).copy())
    if snapshots:
        res.append(snap[:3 * n * n_snap].reshape(n_snap, 3, n).copy())
    return res[0] if len(res) == 1 else tuple(res)


def rf_pulse(M, alpha: float, phase: float) -> np.ndarray:
    """eq. 3.19 applied to one vector, as implemented by the oracle."""
    v = np.array(M, dtype=np.float64).copy()
    _load().oracle_rf_pulse(_ptr(v, _dp), float(alpha), float(phase))
    return v


def precess_relax(M, tau, mu, x, y, z, dw, m0, t1, t2) -> np.ndarray:
    """One precession/relaxation interval (eq. 3.14 with eq. 3.12) on one vector."""
    v = np.array(M, dtype=np.float64).copy()
    mu = np.ascontiguousarray(mu, np.float64)
    _load().oracle_precess_relax(_ptr(v, _dp), float(tau), _ptr(mu, _dp), float(x), float(y),
                                 float(z), float(dw), float(m0), float(t1), float(t2))
    return v


def rel_l2(test, ref) -> float:
    """Relative L2 error ||test - ref|| / ||ref||; equals 10^(dE/20) for the
    noise-distance measure dE of section 5.4.2 (absolute norm when ref is 0)."""
    test = np.asarray(test); ref = np.asarray(ref)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(test - ref)
    return float(num / den) if den > 0 else float(num)


def stoerabstand_db(test, ref) -> float:
    """Noise distance of section 5.4.2: 10 dB log10(sum|ref-test|^2 / sum|ref|^2)."""
    r = rel_l2(test, ref)
    return float(20.0 * np.log10(r)) if r > 0 else float("-inf")


def count_over_threshold(test, ref, rel_threshold: float, eps_scale: float = 1e3, eps: Optional[float] = None) -> int:
    """Number of sample components whose relative error exceeds rel_threshold,
    skipping components whose reference magnitude lies within
    eps_scale * eps of the largest (section 5.4.2); eps is the machine
    epsilon of the arithmetic under test (default FP64)."""
    t = np.asarray(test); r = np.asarray(ref)
    comps_t = np.concatenate([t.real.ravel(), t.imag.ravel()])
    comps_r = np.concatenate([r.real.ravel(), r.imag.ravel()])
    eps = float(np.finfo(np.float64).eps) if eps is None else float(eps)
    floor = eps_scale * eps * max(np.max(np.abs(comps_r)), 1e-300)
    sel = np.abs(comps_r) > floor
    rel = np.abs(comps_t[sel] - comps_r[sel]) / np.abs(comps_r[sel])
    return int(np.count_nonzero(rel > rel_threshold))
