"""Receive-coil sensitivity maps (seeded-free, deterministic input generators).

Section 3.5.1 characterises a receive coil by its sensitivity S = B1 / i
(eq. 3.24): the flux density the coil would produce per unit current, in
laboratory coordinates.  Section 7.1.6 simulates a circular surface coil
of diameter 150 mm.  These helpers compute S for circular loops by the
Biot-Savart law (the loop cut into straight segments), in units of mu_0 / (4
pi) and scaled so that the field at the loop centre is 1; they only produce
inputs -- how S enters the signal is the simulator's business.
"""
from __future__ import annotations

from typing import Sequence as _Seq, Tuple

import numpy as np


def _unit(v) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def loop_sensitivity(x, y, z, center, normal, radius: float, n_seg: int = 512,
                     chunk: int = 1 << 14) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Sensitivity (S_x, S_y, S_z) of a circular loop (centre, unit normal,
    radius in m) at the points (x, y, z), float64.  Units: mu_0 i / (4 pi)
    per unit current, divided by the centre field 2 pi / radius."""
    pts = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64), np.asarray(z, np.float64)], axis=1)
    n = _unit(normal)
    a = np.cross(n, [1.0, 0.0, 0.0])
    if np.linalg.norm(a) < 1e-6:
        a = np.cross(n, [0.0, 1.0, 0.0])
    u = _unit(a)
    v = np.cross(n, u)
    phi = np.linspace(0.0, 2.0 * np.pi, n_seg + 1)
    ring = np.asarray(center, np.float64)[None, :] + radius * (np.cos(phi)[:, None] * u + np.sin(phi)[:, None] * v)
    mid = 0.5 * (ring[1:] + ring[:-1])            # segment midpoints
    dl = ring[1:] - ring[:-1]                     # segment vectors (current sense: right-handed about n)
    out = np.empty_like(pts)
    for b in range(0, pts.shape[0], chunk):
        r = pts[b:b + chunk, None, :] - mid[None, :, :]
        d3 = np.linalg.norm(r, axis=2) ** 3
        out[b:b + chunk] = np.sum(np.cross(dl[None, :, :], r) / d3[:, :, None], axis=1)
    out *= radius / (2.0 * np.pi)
    return out[:, 0], out[:, 1], out[:, 2]


def loop_on_axis(dist, radius: float) -> np.ndarray:
    """Closed form of the same normalised field on the loop's axis at
    distance dist from its centre: radius^3 / (radius^2 + dist^2)^(3/2)."""
    d = np.asarray(dist, np.float64)
    return radius ** 3 / (radius ** 2 + d ** 2) ** 1.5


def loop_ring(obj, n_coils: int, ring_radius: float, coil_radius: float, z0: float = 0.0,
              n_seg: int = 256) -> Tuple[np.ndarray, np.ndarray]:
    """An array of n_coils equal loops on a ring of radius ring_radius about
    the z axis (the B0 direction), each facing the centre; returns the
    transverse sensitivities (s_x, s_y), float32, shape (n_coils, n_spins)."""
    sx = np.empty((n_coils, obj.n_spins), np.float32)
    sy = np.empty((n_coils, obj.n_spins), np.float32)
    for c in range(n_coils):
        t = 2.0 * np.pi * c / n_coils
        nrm = np.array([np.cos(t), np.sin(t), 0.0])
        cx, cy, _ = loop_sensitivity(obj.x, obj.y, obj.z, center=ring_radius * nrm + [0.0, 0.0, z0],
                                     normal=-nrm, radius=coil_radius, n_seg=n_seg)
        sx[c] = cx
        sy[c] = cy
    return sx, sy


def surface_loop(obj, center, normal, diameter: float = 0.15, n_seg: int = 256):
    """One surface loop (section 7.1.6 uses a 150 mm loop): (s_x, s_y),
    float32, shape (1, n_spins)."""
    cx, cy, _ = loop_sensitivity(obj.x, obj.y, obj.z, center=center, normal=normal, radius=diameter / 2,
                                 n_seg=n_seg)
    return cx.astype(np.float32)[None, :], cy.astype(np.float32)[None, :]


def homogeneous(obj, n_coils: int = 1, angles: _Seq[float] = None):
    """Spatially constant transverse sensitivities (cos b, sin b), one per
    coil (default b = 0, the homogeneous coil of section 3.5.2)."""
    b = np.zeros(n_coils) if angles is None else np.asarray(angles, np.float64)
    sx = np.repeat(np.cos(b)[:, None], obj.n_spins, axis=1).astype(np.float32)
    sy = np.repeat(np.sin(b)[:, None], obj.n_spins, axis=1).astype(np.float32)
    return sx, sy
