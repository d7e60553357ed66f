"""The synthetic workloads: sequences and objects of the five configurations,
plus the small sequences the closed-form tests use.

k-space convention: samples of a readout of N points sit at
k_n = (n - N/2) / FOV cycles/m (FFT order), so with one isochromat per voxel
centre at (i - N/2) * FOV / N the encoding matrix is exactly a shifted DFT
(eq. 3.33).  A sample is taken at the *end* of each of the N equal
sub-steps of an ADC interval (section 5.1.1), so the prephaser is
-(N/2 + 1) / FOV and sample N/2 falls on k = 0.  Receive bandwidth follows
the usual Delta k = 1 / FOV (eq. B.3 form).

Configurations (FOV = 0.25 m throughout):
  c1  2-D 64^2, 1 isochromat/voxel, dw = 0; spoiled GRE, 30 deg, TR 10 ms,
      TE 5 ms, 64 phase encodes x 64 samples (dwell 20 us)
  c2  2-D 256^2, 4 jittered isochromats/voxel, dw ~ N(0, (2 pi 20 Hz)^2);
      spin echo 90x/180y, TE 20 ms, TR 500 ms, 256 x 256 (dwell 10 us)
  c3  3-D 128^3 x two species (4,194,304 spins), quadratic B0 +-50 Hz,
      fat at -440 Hz; GRE with a 128-sub-step TBW-4 sinc (30 deg), 0.15 m
      slab, TE 5 ms from the pulse centre, TR 10 ms, 128 x 128 phase
      encodes (kz outer) x 128 samples (dwell 10 us)
  c4  64 requests, 2-D N^2 with N log-uniform in [16, 256], GRE or SE,
      phase encodes U{32..256}, N samples per readout
  c5  2000 requests arriving as a Poisson stream at 50 req/s: 90 % c4-type,
      10 % 3-D 64^3 two-species c3-recipe jobs (64 x 64 encodes x 64 samples)
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from .sequence import Sequence, Shape, Trajectory, SPOIL
from .phantom import SpinObject, grid2d, grid3d_two_species

FOV = 0.25
DEG = math.pi / 180.0


# --------------------------------------------------------------------------
# sequence recipes
# --------------------------------------------------------------------------
def spoiled_gre_2d(n_read: int, n_pe: int, fov: float = FOV, alpha_deg: float = 30.0,
                   tr: float = 10e-3, te: float = 5e-3, dwell: float = 20e-6,
                   name: str = "gre2d") -> Sequence:
    """Cartesian spoiled gradient echo, linear phase order.

    Per TR: [RF alpha_x, prephase + phase encode] [ADC n_read] [rest, SPOIL].
    """
    seq = Sequence(name)
    t_pre = te - (n_read // 2 + 1) * dwell
    t_adc = n_read * dwell
    t_rest = tr - t_pre - t_adc
    if t_pre < 0 or t_rest < 0:
        raise ValueError("TE/TR too short for this readout")
    for j in range(n_pe):
        ky = (j - n_pe // 2) / fov
        seq.add(t_pre, m=(-(n_read // 2 + 1) / fov, ky, 0.0), alpha=alpha_deg * DEG, phase=0.0)
        seq.add(t_adc, m=(n_read / fov, 0.0, 0.0), n_adc=n_read)
        seq.add(t_rest, flags=SPOIL)
    seq.meta.update(kind="gre2d", n_read=n_read, n_pe=n_pe, fov=fov, tr=tr, te=te,
                    dwell=dwell, alpha=alpha_deg * DEG)
    return seq


def spin_echo_2d(n_read: int, n_pe: int, fov: float = FOV, te: float = 20e-3,
                 tr: float = 500e-3, dwell: float = 10e-6, name: str = "se2d") -> Sequence:
    """Cartesian spin echo: [90x, TE/2] [180y, prephase + encode]
    [ADC n_read] [rest, SPOIL].  The echo (sample n_read/2) is at TE."""
    seq = Sequence(name)
    t_pre = te / 2 - (n_read // 2 + 1) * dwell
    t_adc = n_read * dwell
    t_rest = tr - te / 2 - t_pre - t_adc
    if t_pre < 0 or t_rest < 0:
        raise ValueError("TE/TR too short for this readout")
    for j in range(n_pe):
        ky = (j - n_pe // 2) / fov
        seq.add(te / 2, alpha=math.pi / 2, phase=0.0)
        seq.add(t_pre, m=(-(n_read // 2 + 1) / fov, ky, 0.0), alpha=math.pi, phase=math.pi / 2)
        seq.add(t_adc, m=(n_read / fov, 0.0, 0.0), n_adc=n_read)
        seq.add(t_rest, flags=SPOIL)
    seq.meta.update(kind="se2d", n_read=n_read, n_pe=n_pe, fov=fov, tr=tr, te=te, dwell=dwell)
    return seq


def sinc_shape(n_sub: int, tau: float, flip: float, tbw: float, slab: float) -> Shape:
    """Rect-windowed sinc (section 7.2.1) cut into n_sub hard sub-pulses at
    the start of each sub-step (eq. 3.23).  Envelope a(u) = sinc(tbw * u) on
    u_i = (i + 1/2) / n_sub - 1/2; sub-flips alpha_i = flip * a_i / sum(a)
    are signed.  The slab gradient's moment per sub-step is
    (tbw / (n_sub * tau)) * tau / slab cycles/m, so the pulse bandwidth
    tbw / (n_sub tau) spans the slab thickness."""
    u = (np.arange(n_sub) + 0.5) / n_sub - 0.5
    a = np.sinc(tbw * u)
    alpha = flip * a / a.sum()
    bw = tbw / (n_sub * tau)
    mz = bw * tau / slab
    return Shape(tau=tau, m_sub=(0.0, 0.0, mz), alpha=alpha, phase=np.zeros(n_sub))


def gre_3d_sinc(n_read: int, n_pe_y: int, n_pe_z: int, fov: float = FOV,
                alpha_deg: float = 30.0, tr: float = 10e-3, te: float = 5e-3,
                dwell: float = 10e-6, n_rf: int = 128, rf_tau: float = 20e-6,
                tbw: float = 4.0, slab: float = 0.15, name: str = "gre3d") -> Sequence:
    """3-D spoiled GRE with a slab-selective sinc excitation, kz outer loop.

    Per TR: [sinc pulse (n_rf sub-steps); then rephase + prephase + (ky, kz)
    encode] [ADC n_read] [rest, SPOIL].  The pulse centre lies at
    (n_rf - 1) * rf_tau / 2 after its start (hard sub-pulse at the start of
    each sub-step), TE is counted from there, and the slab rephaser is
    -(n_rf - (n_rf - 1) / 2) * m_sub_z."""
    seq = Sequence(name)
    shp = sinc_shape(n_rf, rf_tau, alpha_deg * DEG, tbw, slab)
    sid = seq.add_shape(shp)
    t_rf = n_rf * rf_tau
    t_centre = (n_rf - 1) * rf_tau / 2
    t_adc_start = t_centre + te - (n_read // 2 + 1) * dwell
    t_pre = t_adc_start - t_rf
    t_adc = n_read * dwell
    t_rest = tr - t_adc_start - t_adc
    if t_pre < 0 or t_rest < 0:
        raise ValueError("TE/TR too short for this readout")
    rephase_z = -(n_rf - (n_rf - 1) / 2) * shp.m_sub[2]
    for jz in range(n_pe_z):
        kz = (jz - n_pe_z // 2) / fov
        for jy in range(n_pe_y):
            ky = (jy - n_pe_y // 2) / fov
            seq.add(t_pre, m=(-(n_read // 2 + 1) / fov, ky, kz + rephase_z), shape=sid)
            seq.add(t_adc, m=(n_read / fov, 0.0, 0.0), n_adc=n_read)
            seq.add(t_rest, flags=SPOIL)
    seq.meta.update(kind="gre3d", n_read=n_read, n_pe_y=n_pe_y, n_pe_z=n_pe_z, fov=fov, tr=tr,
                    te=te, dwell=dwell, alpha=alpha_deg * DEG, n_rf=n_rf, rf_tau=rf_tau, tbw=tbw,
                    slab=slab)
    return seq


# --------------------------------------------------------------------------
# the configurations
# --------------------------------------------------------------------------
def c1() -> Tuple[SpinObject, Sequence]:
    return grid2d(64, FOV, 1, seed=1001), spoiled_gre_2d(64, 64, name="c1_gre64")


def c2(n: int = 256, n_pe: int = None) -> Tuple[SpinObject, Sequence]:
    """n defaults to the full 256; smaller n gives the same recipe shrunk."""
    n_pe = n if n_pe is None else n_pe
    obj = grid2d(n, FOV, 4, jitter=True, dw_sigma_hz=20.0, seed=1002)
    return obj, spin_echo_2d(n, n_pe, name=f"c2_se{n}")


def c3(n: int = 128, n_pe_y: int = None, n_pe_z: int = None) -> Tuple[SpinObject, Sequence]:
    n_pe_y = n if n_pe_y is None else n_pe_y
    n_pe_z = n if n_pe_z is None else n_pe_z
    obj = grid3d_two_species(n, FOV, seed=1003)
    return obj, gre_3d_sinc(n, n_pe_y, n_pe_z, name=f"c3_gre3d{n}")


def c4_request(r: int) -> Tuple[SpinObject, Sequence]:
    """Request r (seed 4000 + r) of the batched configuration."""
    rng = np.random.default_rng(4000 + r)
    n = int(round(math.exp(rng.uniform(math.log(16), math.log(256)))))
    kind = "gre" if rng.uniform() < 0.5 else "se"
    n_pe = int(rng.integers(32, 257))
    if kind == "gre":
        obj = grid2d(n, FOV, 1, seed=4000 + r)
        seq = spoiled_gre_2d(n, n_pe, name=f"c4_{r}_gre{n}")
    else:
        obj = grid2d(n, FOV, 1, dw_sigma_hz=20.0, seed=4000 + r)
        seq = spin_echo_2d(n, n_pe, name=f"c4_{r}_se{n}")
    return obj, seq


def c4(n_requests: int = 64) -> List[Tuple[SpinObject, Sequence]]:
    return [c4_request(r) for r in range(n_requests)]


def c5_stream(n_requests: int = 2000, rate_hz: float = 50.0, frac_3d: float = 0.1,
              seed: int = 5000):
    """Arrival schedule of the served configuration: a list of
    (arrival_time_s, kind, param) with kind 'c4' (param = request index into
    an independent c4-style draw) or '3d' (param = 3-D job index)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    kinds = rng.uniform(size=n_requests) < frac_3d
    out = []
    n2 = n3 = 0
    for i in range(n_requests):
        if kinds[i]:
            out.append((float(t[i]), "3d", n3)); n3 += 1
        else:
            out.append((float(t[i]), "c4", 10000 + n2)); n2 += 1
    return out


def c5_request(kind: str, param: int) -> Tuple[SpinObject, Sequence]:
    if kind == "c4":
        return c4_request(param)
    obj = grid3d_two_species(64, FOV, seed=5000 + 7919 * (param + 1))
    return obj, gre_3d_sinc(64, 64, 64, name=f"c5_3d_{param}")


# --------------------------------------------------------------------------
# small closed-form sequences
# --------------------------------------------------------------------------
def fid(alpha: float, n_adc: int, dwell: float, phase: float = 0.0) -> Sequence:
    seq = Sequence("fid")
    seq.add(n_adc * dwell, alpha=alpha, phase=phase, n_adc=n_adc)
    return seq


def spin_echo_single(te: float, n_adc: int, dwell: float, tr: float = None,
                     n_tr: int = 1) -> Sequence:
    """90x - TE/2 - 180y - (TE/2 - (n_adc/2 + 1) dwell) - ADC whose sample
    n_adc/2 falls exactly on TE, optionally repeated with SPOIL and a rest
    interval up to TR."""
    seq = Sequence("se1")
    half = n_adc // 2
    t2 = te / 2 - (half + 1) * dwell
    for _ in range(n_tr):
        seq.add(te / 2, alpha=math.pi / 2)
        seq.add(t2, alpha=math.pi, phase=math.pi / 2)
        seq.add(n_adc * dwell, n_adc=n_adc)
        if tr is not None:
            seq.add(tr - te / 2 - t2 - n_adc * dwell, flags=SPOIL)
    return seq


def spoiled_gre_probe(alpha: float, tr: float, te: float, n_tr: int) -> Sequence:
    """One sample exactly at TE each TR, no gradients, SPOIL at TR end."""
    seq = Sequence("gre_probe")
    for _ in range(n_tr):
        seq.add(te, alpha=alpha, n_adc=1)
        seq.add(tr - te, flags=SPOIL)
    return seq


def inversion_recovery(ti: float, read_delay: float = 0.0) -> Sequence:
    seq = Sequence("ir")
    seq.add(ti, alpha=math.pi, flags=SPOIL)
    seq.add(read_delay, alpha=math.pi / 2, n_adc=1)
    return seq


# --------------------------------------------------------------------------
# the experiments of Table 7.8 (section 7.3.2) on synthetic objects
# --------------------------------------------------------------------------
# The paper times a 2-D turbo spin echo, a 2-D radial and a 2-D EPI
# acquisition (128^2 matrix, 10,000 spins) and a 3-D spin echo (128^2 x 64,
# 176,000 spins), with its Shepp-Logan phantom and the Legendre B0 field of
# eq. 6.3.  Here the objects are tissue-recipe grids of the same spin counts
# (100^2 and 56^3) with the eq. 6.3 field; the sequences are standard forms
# of the four acquisitions built from elementary sequences.  The event counts
# need not equal the paper's (its event granularity is not given).
LEGENDRE_C_TESLA = 1e-5      # C of eq. 6.3 (free constant, 1 tesla dimension)
LEGENDRE_RADIUS = 0.2        # radius of the sphere of homogeneity, m


def tse_2d(n: int, etl: int, fov: float = FOV, esp: float = 10e-3, tr: float = 2.0,
           dwell: float = 10e-6, name: str = "tse2d") -> Sequence:
    """Turbo spin echo (CPMG): per TR a 90x pulse, then etl echoes, each
    [180y, read prephase + phase encode] [ADC n] [rewind]; the echo (sample
    n/2) sits midway between refocusing pulses, and k returns to the origin
    before every 180.  Line order: echo j of TR t takes line j * n_tr + t."""
    if n % etl:
        raise ValueError("etl must divide n")
    n_tr = n // etl
    seq = Sequence(name)
    half = n // 2
    t_pre = esp / 2 - (half + 1) * dwell
    t_rew = esp / 2 - (n - half - 1) * dwell
    if t_pre < 0 or t_rew < 0:
        raise ValueError("echo spacing too short for this readout")
    for t in range(n_tr):
        seq.add(esp / 2, alpha=math.pi / 2, phase=0.0)
        for j in range(etl):
            ky = (j * n_tr + t - half) / fov
            seq.add(t_pre, m=(-(half + 1) / fov, ky, 0.0), alpha=math.pi, phase=math.pi / 2)
            seq.add(n * dwell, m=(n / fov, 0.0, 0.0), n_adc=n)
            seq.add(t_rew, m=(-(n - half - 1) / fov, -ky, 0.0))
        seq.add(tr - esp / 2 - etl * esp, flags=SPOIL)
    seq.meta.update(kind="tse2d", n=n, etl=etl, fov=fov, esp=esp, tr=tr, dwell=dwell)
    return seq


def radial_2d(n: int, n_proj: int, fov: float = FOV, alpha_deg: float = 30.0, tr: float = 10e-3,
              te: float = 4e-3, dwell: float = 10e-6, name: str = "radial2d") -> Sequence:
    """Radial spoiled gradient echo: projection p reads a full spoke through
    the k-space centre at angle pi p / n_proj, with prephaser and readout
    along (cos, sin) of that angle."""
    seq = Sequence(name)
    half = n // 2
    t_pre = te - (half + 1) * dwell
    t_rest = tr - t_pre - n * dwell
    if t_pre < 0 or t_rest < 0:
        raise ValueError("TE/TR too short for this readout")
    for p in range(n_proj):
        th = math.pi * p / n_proj
        d = (math.cos(th), math.sin(th), 0.0)
        seq.add(t_pre, m=tuple(-(half + 1) / fov * c for c in d), alpha=alpha_deg * DEG)
        seq.add(n * dwell, m=tuple(n / fov * c for c in d), n_adc=n)
        seq.add(t_rest, flags=SPOIL)
    seq.meta.update(kind="radial2d", n=n, n_proj=n_proj, fov=fov, tr=tr, te=te, dwell=dwell)
    return seq


def epi_2d(n: int, fov: float = FOV, dwell: float = 4e-6, blip: float = 40e-6, t_pre: float = 5e-3,
           name: str = "epi2d") -> Sequence:
    """Single-shot gradient-echo EPI: 90x with prephasers to the k-space
    corner, then n readout lines of alternating polarity with a ky blip of
    1/fov between lines, and a final spoiled interval."""
    seq = Sequence(name)
    half = n // 2
    seq.add(t_pre, m=(-(half + 1) / fov, -half / fov, 0.0), alpha=math.pi / 2)
    for line in range(n):
        sgn = 1.0 if line % 2 == 0 else -1.0
        seq.add(n * dwell, m=(sgn * n / fov, 0.0, 0.0), n_adc=n)
        if line + 1 < n:
            seq.add(blip, m=(0.0, 1.0 / fov, 0.0))
    seq.add(1e-3, flags=SPOIL)
    seq.meta.update(kind="epi2d", n=n, fov=fov, dwell=dwell, blip=blip)
    return seq


def se_3d(n: int, n_pe_y: int, n_pe_z: int, fov: float = FOV, te: float = 20e-3, tr: float = 0.5,
          dwell: float = 10e-6, name: str = "se3d") -> Sequence:
    """3-D spin echo: per TR [90x, TE/2] [180y, read prephase + (ky, kz)
    encode] [ADC n] [rest, SPOIL]; kz outer loop."""
    seq = Sequence(name)
    half = n // 2
    t_pre = te / 2 - (half + 1) * dwell
    t_rest = tr - te / 2 - t_pre - n * dwell
    if t_pre < 0 or t_rest < 0:
        raise ValueError("TE/TR too short for this readout")
    for jz in range(n_pe_z):
        kz = (jz - n_pe_z // 2) / fov
        for jy in range(n_pe_y):
            ky = (jy - n_pe_y // 2) / fov
            seq.add(te / 2, alpha=math.pi / 2)
            seq.add(t_pre, m=(-(half + 1) / fov, ky, kz), alpha=math.pi, phase=math.pi / 2)
            seq.add(n * dwell, m=(n / fov, 0.0, 0.0), n_adc=n)
            seq.add(t_rest, flags=SPOIL)
    seq.meta.update(kind="se3d", n=n, n_pe_y=n_pe_y, n_pe_z=n_pe_z, fov=fov, te=te, tr=tr, dwell=dwell)
    return seq


TABLE78 = ("tse", "radial", "epi", "se3d")


def table78(kind: str, scale: int = 1) -> Tuple[SpinObject, Sequence]:
    """One experiment of Table 7.8: scale = 1 is the paper's size (128^2
    matrix, 10,000 spins; 3-D: 128^2 x 64, 175,616 spins); scale = s divides
    the matrix and the object side by s (for oracle-sized tests)."""
    from .phantom import grid2d_legendre, grid3d_legendre
    n = 128 // scale
    if kind == "se3d":
        obj = grid3d_legendre(max(56 // scale, 2), FOV, seed=7804, c_tesla=LEGENDRE_C_TESLA,
                              radius=LEGENDRE_RADIUS)
        return obj, se_3d(n, n, max(64 // scale, 1))
    obj = grid2d_legendre(max(100 // scale, 2), FOV, seed={"tse": 7801, "radial": 7802, "epi": 7803}[kind],
                          c_tesla=LEGENDRE_C_TESLA, radius=LEGENDRE_RADIUS)
    if kind == "tse":
        return obj, tse_2d(n, max(16 // scale, 2))
    if kind == "radial":
        return obj, radial_2d(n, n)
    if kind == "epi":
        return obj, epi_2d(n)
    raise ValueError(f"unknown Table 7.8 experiment {kind!r}")


def spiral_2d(n_interleaves: int, n_samples: int, fov: float = FOV, res: int = 128, alpha_deg: float = 30.0,
              tr: float = 20e-3, te: float = 2e-3, dwell: float = 4e-6, name: str = "spiral2d") -> Sequence:
    """Multi-shot spiral spoiled GRE: each TR a pulse, a wait to TE, then a
    constant-angular-velocity Archimedean spiral out to k_max = res / (2 fov)
    sampled on the dwell raster (a per-sample trajectory table), and a
    spoiled rest.  Interleave i is rotated by 2 pi i / n_interleaves."""
    seq = Sequence(name)
    k_max = res / (2.0 * fov)
    turns = res / (2.0 * n_interleaves)
    u = (np.arange(n_samples) + 1) / n_samples
    t = u * n_samples * dwell
    t_adc = n_samples * dwell + dwell
    for i in range(n_interleaves):
        th = 2 * math.pi * turns * u + 2 * math.pi * i / n_interleaves
        k = np.stack([k_max * u * np.cos(th), k_max * u * np.sin(th), np.zeros(n_samples)], axis=1)
        j = seq.add_trajectory(Trajectory(k=k, t=t))
        seq.add(te, alpha=alpha_deg * DEG)
        seq.add(t_adc, m=tuple(k[-1]), n_adc=n_samples, trajectory=j)
        seq.add(tr - te - t_adc, flags=SPOIL)
    seq.meta.update(kind="spiral2d", n_interleaves=n_interleaves, n_samples=n_samples, fov=fov, res=res)
    return seq
