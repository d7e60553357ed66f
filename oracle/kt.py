"""K-t (configuration) oracle -- TEST INFRASTRUCTURE.

A second, independent oracle for the signal of the spin-based method,
following the K-t formalism of section 4.2.  When every gradient moment of a
sequence is an integer multiple of a lattice step dk (per axis), the
magnetisation of a spin at x is a finite series over lattice orders k
(eq. 4.7 - 4.11):

    Mxy(x) = sum_k F(k) exp(-2 pi j (k dk) . x)
    Mz(x)  = sum_k Z(k) exp(-2 pi j (k dk) . x),     Z(-k) = conj(Z(k)),

whose populations F, Z depend only on the RF pulses and the relaxation
(and a spatially uniform off-resonance) of one tissue, never on x.  The
operators act on them as in eq. 4.12 - 4.17:

  * a hard pulse mixes, at every order k, the triplet (F(k), conj(F(-k)),
    Z(k)) with the complex form of the eq. 3.19 rotation (eq. 4.14);
  * relaxation scales F by E2 and Z by E1, and adds M0 (1 - E1) to Z(0)
    only (eq. 4.15 / 4.16);
  * a gradient of moment q dk moves every transverse population from order
    k to k + q and leaves Z alone (eq. 4.17);
  * a spatially uniform off-resonance dw multiplies F by exp(-j dw tau).

The signal of spins x_i with weights m0_i sharing one tissue is then
sum_k F(k) S(k) with S(k) = sum_i m0_i exp(-2 pi j (k dk) . x_i) (eq. 4.19):
the same sum the isochromat oracle forms spin by spin, computed without
stepping any spin.  Sequences use the workloads Sequence model; readings
(operator order, sample instants, rotation sense, SPOIL) are those of the
isochromat oracle.  Plain Python dictionaries over lattice points; meant for
small cases.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence as _Seq, Tuple

import numpy as np

Order = Tuple[int, int, int]

SPOIL = 1


def _lattice(m, dk, what: str) -> Order:
    """Integer lattice vector q with m = q * dk per axis (axes with dk = 0
    must carry no moment)."""
    q = []
    for d in range(3):
        if dk[d] == 0.0:
            if abs(m[d]) > 1e-9:
                raise ValueError(f"{what}: moment {m[d]} on axis {d} without a lattice step")
            q.append(0)
            continue
        r = m[d] / dk[d]
        n = int(round(r))
        if abs(r - n) > 1e-6 * max(1.0, abs(r)):
            raise ValueError(f"{what}: moment {m[d]} on axis {d} is not a multiple of {dk[d]}")
        q.append(n)
    return (q[0], q[1], q[2])


def _rotation(alpha: float, phi: float) -> np.ndarray:
    """eq. 3.19 for one hard pulse (flip alpha about the axis at phase phi in
    the x'y' plane)."""
    ca, sa, cp, sp = math.cos(alpha), math.sin(alpha), math.cos(phi), math.sin(phi)
    return np.array([[cp * cp + sp * sp * ca, sp * cp * (1 - ca), -sp * sa],
                     [sp * cp * (1 - ca), sp * sp + cp * cp * ca, cp * sa],
                     [sp * sa, -cp * sa, ca]])


# (Mx, My, Mz) -> (Mx + j My, Mx - j My, Mz) and back
_C = np.array([[1, 1j, 0], [1, -1j, 0], [0, 0, 1]], dtype=complex)
_CI = np.linalg.inv(_C)


class KtState:
    """Configuration populations of one tissue (per unit M0)."""

    def __init__(self, t1: float, t2: float, dw: float = 0.0):
        self.t1, self.t2, self.dw = float(t1), float(t2), float(dw)
        self.F: Dict[Order, complex] = {}
        self.Z: Dict[Order, complex] = {(0, 0, 0): 1.0 + 0j}

    def rf(self, alpha: float, phi: float):
        """eq. 4.14: the complex form T = C R C^-1 of eq. 3.19, order by order."""
        if alpha == 0.0:
            return
        T = _C @ _rotation(alpha, phi) @ _CI
        keys = set(self.F) | {(-a, -b, -c) for a, b, c in self.F} | set(self.Z)
        F, Z = {}, {}
        for k in keys:
            mk = (-k[0], -k[1], -k[2])
            u = self.F.get(k, 0j)
            v = np.conj(self.F.get(mk, 0j))
            w = self.Z.get(k, 0j)
            fu = T[0, 0] * u + T[0, 1] * v + T[0, 2] * w
            zw = T[2, 0] * u + T[2, 1] * v + T[2, 2] * w
            if fu != 0:
                F[k] = complex(fu)
            if zw != 0:
                Z[k] = complex(zw)
        self.F, self.Z = F, Z

    def interval(self, tau: float, q: Order):
        """Precession over tau under a gradient of lattice moment q, with
        relaxation (eq. 4.15 - 4.17) and the uniform off-resonance."""
        e1 = math.exp(-tau / self.t1)
        e2 = math.exp(-tau / self.t2)
        ph = complex(math.cos(self.dw * tau), -math.sin(self.dw * tau))
        self.F = {(k[0] + q[0], k[1] + q[1], k[2] + q[2]): f * e2 * ph for k, f in self.F.items()}
        Z = {k: z * e1 for k, z in self.Z.items()}
        Z[(0, 0, 0)] = Z.get((0, 0, 0), 0j) + (1.0 - e1)
        self.Z = Z

    def spoil(self):
        self.F = {}

    def max_order(self, transverse: bool = True, longitudinal: bool = True, tol: float = 0.0) -> np.ndarray:
        """Largest |k| per axis over the populations above tol."""
        out = np.zeros(3, dtype=np.int64)
        for src, use in ((self.F, transverse), (self.Z, longitudinal)):
            if not use:
                continue
            for k, a in src.items():
                if abs(a) > tol:
                    out = np.maximum(out, np.abs(np.array(k)))
        return out


def run(seq, dk, t1: float, t2: float, dw: float = 0.0, on_sample=None, on_step=None) -> KtState:
    """Step one tissue's populations through seq (section 5.1.1 order: shape
    sub-steps, the event's hard pulse, K = max(n_adc, 1) sub-steps, SPOIL).
    on_sample(state) is called after every ADC sub-step, on_step(state)
    after every interval sub-step and pulse."""
    st = KtState(t1, t2, dw)
    dk = [float(v) for v in dk]
    shapes = list(seq.shapes)
    for e in range(seq.n_events):
        sh = int(seq.rf_shape[e])
        if sh >= 0:
            shape = shapes[sh]
            qs = _lattice(shape.m_sub, dk, f"shape {sh}")
            for a, p in zip(shape.alpha, shape.phase):
                st.rf(float(a), float(p) + float(seq.rf_phase[e]))
                if on_step:
                    on_step(st)
                st.interval(float(shape.tau), qs)
                if on_step:
                    on_step(st)
        st.rf(float(seq.rf_alpha[e]), float(seq.rf_phase[e]))
        if on_step:
            on_step(st)
        n = int(seq.n_adc[e])
        K = max(n, 1)
        m = np.asarray(seq.m[e], np.float64) / K
        q = _lattice(m, dk, f"event {e}")
        for _ in range(K):
            st.interval(float(seq.dt[e]) / K, q)
            if on_step:
                on_step(st)
            if n > 0 and on_sample:
                on_sample(st)
        if int(seq.flags[e]) & SPOIL:
            st.spoil()
            if on_step:
                on_step(st)
    return st


def signal(obj, seq, dk, t1: float, t2: float, dw: float = 0.0) -> np.ndarray:
    """eq. 4.19: the signal of spins obj.x/y/z with weights obj.m0 that all
    share the tissue (t1, t2, dw), from the populations alone."""
    x = np.stack([np.asarray(obj.x, np.float32).astype(np.float64), np.asarray(obj.y, np.float32).astype(np.float64),
                  np.asarray(obj.z, np.float32).astype(np.float64)], axis=1)
    m0 = np.asarray(obj.m0, np.float32).astype(np.float64)
    dkv = np.asarray(dk, np.float64)
    cache: Dict[Order, complex] = {}
    out: List[complex] = []

    def S(k: Order) -> complex:
        if k not in cache:
            kv = np.array(k, np.float64) * dkv
            cache[k] = complex(np.sum(m0 * np.exp(-2j * np.pi * (x @ kv))))
        return cache[k]

    def on_sample(st: KtState):
        out.append(sum(f * S(k) for k, f in st.F.items()))

    run(seq, dk, t1, t2, dw, on_sample=on_sample)
    return np.array(out, dtype=np.complex128)


def extent(seq, dk, t1: float, t2: float, grey_step: Optional[float] = None) -> np.ndarray:
    """K_max per axis in cycles/m (eq. 5.1).

    Without grey_step: the largest |k| of any transverse or longitudinal
    configuration with a population above 1e-12 M0 (rounding left by
    cancelling terms does not count) at any instant (section 5.2.2 / 5.2.3).  With grey_step = Delta rho (eq. 5.5): at every ADC sample the
    outer transverse configurations whose populations sum to at most
    Delta rho / 2 of the largest transverse population (eq. 5.4) are left
    out, and only transverse configurations at samples count (section
    5.2.4)."""
    dkv = np.abs(np.asarray(dk, np.float64))
    kmax = np.zeros(3, dtype=np.int64)

    if grey_step is None:
        def on_step(st: KtState):
            nonlocal kmax
            kmax = np.maximum(kmax, st.max_order(tol=1e-12))
        run(seq, dk, t1, t2, on_step=on_step)
        return kmax * dkv

    def on_sample(st: KtState):
        nonlocal kmax
        if not st.F:
            return
        ref = max(abs(a) for a in st.F.values())
        budget = 0.5 * grey_step * ref
        for d in range(3):
            pops = sorted(((abs(k[d]), abs(a)) for k, a in st.F.items()), reverse=True)
            cut = 0.0
            K = 0
            for i, (kk, a) in enumerate(pops):
                if cut + a > budget:
                    K = kk
                    break
                cut += a
            kmax[d] = max(kmax[d], K)
    run(seq, dk, t1, t2, on_sample=on_sample)
    return kmax * dkv


def max_spacing(kmax) -> np.ndarray:
    """eq. 5.2 with k in cycles/m: spins closer than 1 / (2 K_max) per axis
    (pi / K_max with K in rad/m); +inf on axes with K_max = 0."""
    k = np.asarray(kmax, np.float64)
    with np.errstate(divide="ignore"):
        return np.where(k > 0, 0.5 / np.where(k > 0, k, 1.0), np.inf)
