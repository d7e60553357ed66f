"""Seeded synthetic spin objects (section 6.1.1 object model).

A spin ("isochromat") carries a position, M0, T1, T2 and a rotating-frame
off-resonance dw in rad/s (eq. 6.1 / 6.2).  Arrays are float32 structure-of-
arrays; the oracle widens them exactly to float64, the GPU path reads them as
stored, so both consume identical values.

Tissue draws follow one recipe everywhere: rho ~ U[0, 1), T1 ~ U[0.3, 2) s,
T2 ~ U[0.03, 0.3) s, drawn per voxel with numpy's PCG64 in that order.  The
paper's own phantom (Shepp-Logan ellipses with the parameters of Table 7.1)
is not reproduced: its ellipse geometry is given only by reference, so these
random-tissue grids stand in for it.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

FIELDS = ("x", "y", "z", "m0", "t1", "t2", "dw")


@dataclasses.dataclass
class SpinObject:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m0: np.ndarray
    t1: np.ndarray
    t2: np.ndarray
    dw: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)

    def __post_init__(self):
        n = None
        for f in FIELDS:
            a = np.ascontiguousarray(getattr(self, f), dtype=np.float32).reshape(-1)
            setattr(self, f, a)
            if n is None:
                n = a.shape[0]
            elif a.shape[0] != n:
                raise ValueError(f"field {f} has {a.shape[0]} entries, expected {n}")

    @property
    def n_spins(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return {f: getattr(self, f) for f in FIELDS}

    def take(self, idx) -> "SpinObject":
        idx = np.asarray(idx)
        return SpinObject(**{f: getattr(self, f)[idx] for f in FIELDS}, meta=dict(self.meta))


def subset(obj: SpinObject, stride: int, offset: int = 0) -> SpinObject:
    """Every stride-th spin starting at offset (a fixed, seed-free subset)."""
    return obj.take(np.arange(offset, obj.n_spins, stride))


def _tissue(rng: np.random.Generator, n: int):
    rho = rng.uniform(0.0, 1.0, n)
    t1 = rng.uniform(0.3, 2.0, n)
    t2 = rng.uniform(0.03, 0.3, n)
    return rho, t1, t2


def grid_positions(n: int, fov: float) -> np.ndarray:
    """Voxel centres (i - n/2) * fov / n, i = 0 .. n-1 (FFT convention)."""
    return (np.arange(n, dtype=np.float64) - n // 2) * (fov / n)


def grid2d(n: int, fov: float = 0.25, iso_per_voxel: int = 1, jitter: bool = False,
           dw_sigma_hz: float = 0.0, seed: int = 0) -> SpinObject:
    """2-D n x n voxel grid at z = 0.

    iso_per_voxel isochromats share their voxel's rho/T1/T2 with
    m0 = rho / iso_per_voxel.  The first isochromat of a voxel sits at the
    voxel centre, the others (when jitter is set) at the centre plus a
    uniform offset in (-d/2, d/2) per axis.  dw ~ N(0, (2 pi dw_sigma_hz)^2)
    per isochromat.  Spin order: voxel-major (row y, column x), then
    isochromat.
    """
    rng = np.random.default_rng(seed)
    nv = n * n
    rho, t1, t2 = _tissue(rng, nv)
    d = fov / n
    c = grid_positions(n, fov)
    yy, xx = np.meshgrid(c, c, indexing="ij")
    xx = xx.reshape(-1); yy = yy.reshape(-1)
    k = iso_per_voxel
    x = np.repeat(xx, k); y = np.repeat(yy, k)
    if jitter and k > 1:
        off = rng.uniform(-d / 2, d / 2, size=(nv, k, 2))
        off[:, 0, :] = 0.0
        x = x + off[:, :, 0].reshape(-1)
        y = y + off[:, :, 1].reshape(-1)
    m0 = np.repeat(rho / k, k)
    T1 = np.repeat(t1, k); T2 = np.repeat(t2, k)
    if dw_sigma_hz > 0:
        dw = rng.normal(0.0, 2 * np.pi * dw_sigma_hz, nv * k)
    else:
        dw = np.zeros(nv * k)
    obj = SpinObject(x=x, y=y, z=np.zeros_like(x), m0=m0, t1=T1, t2=T2, dw=dw)
    obj.meta.update(kind="grid2d", n=n, fov=fov, iso_per_voxel=k, seed=seed,
                    rho=rho.reshape(n, n))
    return obj


def quadratic_b0_hz(xh, yh, zh, coef, peak_hz: float):
    """Smooth B0 offset map in Hz: a full degree-2 polynomial in normalised
    coordinates, scaled so that its largest magnitude on the given points is
    peak_hz.  coef holds the 10 coefficients of
    1, x, y, z, x^2, y^2, z^2, xy, xz, yz."""
    q = (coef[0] + coef[1] * xh + coef[2] * yh + coef[3] * zh
         + coef[4] * xh * xh + coef[5] * yh * yh + coef[6] * zh * zh
         + coef[7] * xh * yh + coef[8] * xh * zh + coef[9] * yh * zh)
    return peak_hz * q / np.max(np.abs(q))


def grid3d_two_species(n: int, fov: float = 0.25, fat_shift_hz: float = -440.0,
                       b0_peak_hz: float = 50.0, split=(0.8, 0.2), seed: int = 0) -> SpinObject:
    """3-D n^3 voxel grid holding two co-located species per voxel.

    The two species are superposed spin sets at the same positions (the
    paper's superposition of cuboids, section 6.1.1): water with
    m0 = split[0] * rho and fat with m0 = split[1] * rho, each with its own
    T1/T2 draw, fat shifted by fat_shift_hz.  Both see the same smooth B0
    map (quadratic_b0_hz, +-b0_peak_hz).  Spin order: species-major (all
    water spins, then all fat spins), voxel order z, y, x.
    """
    rng = np.random.default_rng(seed)
    nv = n ** 3
    rho = rng.uniform(0.0, 1.0, nv)
    t1w = rng.uniform(0.3, 2.0, nv); t2w = rng.uniform(0.03, 0.3, nv)
    t1f = rng.uniform(0.3, 2.0, nv); t2f = rng.uniform(0.03, 0.3, nv)
    coef = rng.normal(0.0, 1.0, 10)
    c = grid_positions(n, fov)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    xx = xx.reshape(-1); yy = yy.reshape(-1); zz = zz.reshape(-1)
    h = fov / 2
    b0 = quadratic_b0_hz(xx / h, yy / h, zz / h, coef, b0_peak_hz)
    dw_w = 2 * np.pi * b0
    dw_f = 2 * np.pi * (b0 + fat_shift_hz)
    obj = SpinObject(
        x=np.concatenate([xx, xx]), y=np.concatenate([yy, yy]), z=np.concatenate([zz, zz]),
        m0=np.concatenate([split[0] * rho, split[1] * rho]),
        t1=np.concatenate([t1w, t1f]), t2=np.concatenate([t2w, t2f]),
        dw=np.concatenate([dw_w, dw_f]))
    obj.meta.update(kind="grid3d_two_species", n=n, fov=fov, seed=seed, b0_coef=coef)
    return obj


def uniform_disc(radius: float, spacing: float, rho: float = 1.0) -> SpinObject:
    """Spins on a square grid of the given spacing inside a disc, with
    m0 = rho * spacing^2 (area weight), T1 = T2 = +inf and dw = 0."""
    nmax = int(np.ceil(radius / spacing)) + 1
    c = (np.arange(-nmax, nmax + 1) + 0.5) * spacing
    yy, xx = np.meshgrid(c, c, indexing="ij")
    inside = xx ** 2 + yy ** 2 <= radius ** 2
    x = xx[inside]; y = yy[inside]
    n = x.size
    return SpinObject(x=x, y=y, z=np.zeros(n), m0=np.full(n, rho * spacing ** 2),
                      t1=np.full(n, np.inf), t2=np.full(n, np.inf), dw=np.zeros(n))


def single_spin(x=0.0, y=0.0, z=0.0, m0=1.0, t1=np.inf, t2=np.inf, dw=0.0) -> SpinObject:
    return SpinObject(x=[x], y=[y], z=[z], m0=[m0], t1=[t1], t2=[t2], dw=[dw])


def random_spins(n: int, seed: int, fov: float = 0.25, dw_sigma_hz: float = 30.0,
                 t_inf_frac: float = 0.0) -> SpinObject:
    """Unstructured random spins (positions uniform in the FOV cube, tissue
    recipe as above); a fraction t_inf_frac gets T1 = T2 = +inf."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-fov / 2, fov / 2, size=(3, n))
    rho, t1, t2 = _tissue(rng, n)
    dw = rng.normal(0.0, 2 * np.pi * dw_sigma_hz, n)
    if t_inf_frac > 0:
        sel = rng.uniform(size=n) < t_inf_frac
        t1 = np.where(sel, np.inf, t1); t2 = np.where(sel, np.inf, t2)
    return SpinObject(x=pos[0], y=pos[1], z=pos[2], m0=rho, t1=t1, t2=t2, dw=dw)


GAMMA_RAD = 2.0 * np.pi * 42.577478e6     # 1H gyromagnetic ratio, rad/(s T)


def legendre_p(l: int, x) -> np.ndarray:
    """Legendre polynomial P_l(x) by Bonnet's recursion
    (k + 1) P_{k+1} = (2k + 1) x P_k - k P_{k-1}."""
    x = np.asarray(x, np.float64)
    p0, p1 = np.ones_like(x), x.copy()
    if l == 0:
        return p0
    for k in range(1, l):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    return p1


def legendre_b0_tesla(x, y, z, c_tesla: float, radius: float, order: int = 12) -> np.ndarray:
    """Main-field deviation of a whole-body magnet outside its sphere of
    homogeneity (eq. 6.3): dB0 = -C (r / R)^12 P_12(cos theta), r = |x|,
    theta the angle to the z axis.  Returns tesla, float64."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64); z = np.asarray(z, np.float64)
    r = np.sqrt(x * x + y * y + z * z)
    cos_t = np.divide(z, r, out=np.ones_like(r), where=r > 0)
    return -c_tesla * (r / radius) ** order * legendre_p(order, cos_t)


def grid2d_legendre(n_side: int, fov: float, seed: int, c_tesla: float, radius: float,
                    gamma: float = GAMMA_RAD) -> SpinObject:
    """n_side^2 spins on a grid in the z = 0 plane with the tissue recipe and
    the eq. 6.3 field deviation as off-resonance dw = gamma dB0 (rad/s)."""
    rng = np.random.default_rng(seed)
    c = grid_positions(n_side, fov)
    yy, xx = np.meshgrid(c, c, indexing="ij")
    xx = xx.reshape(-1); yy = yy.reshape(-1)
    rho, t1, t2 = _tissue(rng, xx.size)
    dw = gamma * legendre_b0_tesla(xx, yy, np.zeros_like(xx), c_tesla, radius)
    obj = SpinObject(x=xx, y=yy, z=np.zeros_like(xx), m0=rho, t1=t1, t2=t2, dw=dw)
    obj.meta.update(kind="grid2d_legendre", n=n_side, fov=fov, seed=seed, c_tesla=c_tesla, radius=radius)
    return obj


def grid3d_legendre(n_side: int, fov: float, seed: int, c_tesla: float, radius: float,
                    gamma: float = GAMMA_RAD) -> SpinObject:
    """n_side^3 spins on a grid with the tissue recipe and the eq. 6.3 field."""
    rng = np.random.default_rng(seed)
    c = grid_positions(n_side, fov)
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    xx = xx.reshape(-1); yy = yy.reshape(-1); zz = zz.reshape(-1)
    rho, t1, t2 = _tissue(rng, xx.size)
    dw = gamma * legendre_b0_tesla(xx, yy, zz, c_tesla, radius)
    obj = SpinObject(x=xx, y=yy, z=zz, m0=rho, t1=t1, t2=t2, dw=dw)
    obj.meta.update(kind="grid3d_legendre", n=n_side, fov=fov, seed=seed, c_tesla=c_tesla, radius=radius)
    return obj


# Tissue classes of the K-t phantom: (rho, T1 s, T2 s, off-resonance Hz).
# Illustrative values of the usual brain-like ordering; uniform per class.
KT_TISSUES = (
    (0.9, 0.30, 0.080, -50.0),   # outer ring ("fat-like", shifted)
    (0.7, 0.80, 0.070, 0.0),     # "white matter"
    (0.8, 1.30, 0.100, 10.0),    # "grey matter"
    (1.0, 4.00, 2.000, 0.0),     # "fluid"
)


def kt_phantom_2d(n: int, fov: float = 0.25, iso_per_axis: int = 1):
    """2-D n x n voxel grid at z = 0 made of the KT_TISSUES classes in nested
    discs (radii 0.45, 0.36, 0.24, 0.10 of the FOV; voxels outside hold no
    spins), ordered tissue by tissue.  With iso_per_axis = m every voxel
    holds m x m isochromats at the centres of its m x m sub-cells, each with
    m0 = rho / m^2 (a sampling of the voxel's uniform density).

    Returns (SpinObject with each spin's tissue T1, T2 and dw,
    tissue_begin offsets, t1, t2, dw per tissue (dw in rad/s; the float32
    values the spins hold, widened), voxel size).
    """
    d = fov / n
    c = grid_positions(n, fov)
    yy, xx = np.meshgrid(c, c, indexing="ij")
    r = np.hypot(xx, yy).reshape(-1) / fov
    radii = (0.45, 0.36, 0.24, 0.10)
    cls = np.full(r.shape, -1)
    for t, rad in enumerate(radii):
        cls[r <= rad] = t
    m = iso_per_axis
    sub = (np.arange(m) + 0.5) * (d / m) - d / 2
    sy, sx = np.meshgrid(sub, sub, indexing="ij")
    xs, ys, m0, t1, t2, dw, begin = [], [], [], [], [], [], [0]
    for t, (rho, T1, T2, f) in enumerate(KT_TISSUES):
        sel = np.nonzero(cls == t)[0]
        px = (xx.reshape(-1)[sel][:, None] + sx.reshape(-1)[None, :]).reshape(-1)
        py = (yy.reshape(-1)[sel][:, None] + sy.reshape(-1)[None, :]).reshape(-1)
        xs.append(px); ys.append(py)
        m0.append(np.full(px.shape, rho / (m * m)))
        t1.append(np.full(px.shape, T1)); t2.append(np.full(px.shape, T2))
        dw.append(np.full(px.shape, 2 * np.pi * f))
        begin.append(begin[-1] + px.size)
    x = np.concatenate(xs); y = np.concatenate(ys)
    obj = SpinObject(x=x, y=y, z=np.zeros_like(x), m0=np.concatenate(m0), t1=np.concatenate(t1),
                     t2=np.concatenate(t2), dw=np.concatenate(dw))
    obj.meta.update(kind="kt_phantom_2d", n=n, fov=fov, iso_per_axis=m)
    # per-tissue values as the spins store them (float32), widened exactly
    tis = np.array(KT_TISSUES, dtype=np.float64)
    w32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    return (obj, np.array(begin, dtype=np.int64), w32(tis[:, 1]), w32(tis[:, 2]), w32(2 * np.pi * tis[:, 3]), d)
