"""Seeded synthetic inputs: Hamiltonian presets, spin textures, directions.

This module generates inputs only.  It holds none of the method's arithmetic
(no energy, gradient, Hessian, eigen-solve or step) and imports neither the
HIP binding nor the oracle, so both sides can be fed identical inputs from it.

Workloads follow the paper's atomistic-spin testbeds: Neel skyrmions and
antiskyrmions (Q = +1 / -1) and biskyrmions (Q = 2) on a periodic triangular
monolayer with exchange shells, interfacial DMI, uniaxial anisotropy and a
field along z (Results, Pd/Fe/Ir(111) networks; Methods, spin Hamiltonian).
The reduced-unit presets below have J1 = 1; `ham_pdfeir` carries the
Pd/Fe/Ir(111) exchange of the paper's Supplementary Note 4 (Table S1, 35
shells) with the stand-ins it states for what the paper does not give.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

SQ3 = np.sqrt(3.0)


@dataclass
class HamParams:
    """Plain parameter record: periodic rhombic Lx x Ly triangular lattice,
    exchange J[s] and DMI D[s] per neighbour shell s, uniaxial K (axis e_z),
    Zeeman field B."""

    Lx: int
    Ly: int
    J: List[float]
    D: List[float] = field(default_factory=list)
    K: float = 0.0
    B: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    def with_size(self, Lx: int, Ly: int) -> "HamParams":
        return HamParams(Lx, Ly, list(self.J), list(self.D), self.K, tuple(self.B))

    def asdict(self):
        return dict(Lx=self.Lx, Ly=self.Ly, J=list(self.J), D=list(self.D), K=self.K, B=tuple(self.B))


# ---------------------------------------------------------------------------
# Hamiltonian presets
# ---------------------------------------------------------------------------
def ham_nn(L: int = 16, Ly: int = None) -> HamParams:
    """Nearest-neighbour model: J = 1, D = 0.3, K = 0.05, B = 0.02 z."""
    return HamParams(L, Ly or L, [1.0], [0.3], 0.05, (0.0, 0.0, 0.02))


def three_shell_J(seed: int = 2509) -> Tuple[float, float]:
    """J2, J3 drawn once from U[-0.3, 0.1] with numpy PCG64 default_rng(seed)."""
    j2, j3 = np.random.default_rng(seed).uniform(-0.3, 0.1, 2)
    return float(j2), float(j3)


def ham_3shell(L: int = 128, Ly: int = None, seed: int = 2509) -> HamParams:
    """Three exchange shells J = (1, J2, J3), NN DMI D = 0.25, K = 0.04,
    B = 0.03 z."""
    j2, j3 = three_shell_J(seed)
    return HamParams(L, Ly or L, [1.0, j2, j3], [0.25, 0.0, 0.0], 0.04, (0.0, 0.0, 0.03))


# Exchange of the Pd/Fe/Ir(111) monolayer, Supplementary Note 4, Table S1
# (mRy, shells by increasing |r_ij|, 6/12/18/24 bonds each).  The table prints
# one value per bond; within a shell the printed values agree except for the
# last digit of a few far shells (and the two orbits at |r|^2 = 49 NN units),
# so each shell takes the mean of its printed values.
PDFEIR_J = [
    8.324670e-01, -7.340000e-03, -1.573290e-01, -2.045300e-02, -1.547800e-02,
    1.283500e-02, -2.734000e-03, 6.973000e-03, -7.460000e-04, 2.388000e-03,
    7.600000e-04, 6.770000e-04, -1.129000e-03, 5.720000e-04, -3.130000e-04,
    -3.700000e-05, -4.000000e-05, 2.700000e-05, 4.300000e-05, -2.266667e-05,
    4.200000e-05, 8.600000e-05, 3.700000e-05, 5.000000e-06, 2.800000e-05,
    1.800000e-05, 5.000000e-06, -5.000000e-07, -2.300000e-05, 9.333333e-06,
    2.333333e-05, -2.116667e-05, -6.750000e-06, -1.166667e-05, -2.333333e-06,
]
# In-plane magnitude of the nearest-neighbour DMI vectors of Table S2 (mRy).
# Which bond each printed vector belongs to is not stated, so only this
# magnitude is used, in the interfacial form D (z x dhat); the out-of-plane
# components and the longer-range DMI are left out.
PDFEIR_D1 = 0.040657


def ham_pdfeir(L: int = 64, Ly: int = None, n_shells: int = 35, K: float = 0.05,
               bz: float = 0.02) -> HamParams:
    """Pd/Fe/Ir(111): the first n_shells exchange shells of Table S1 and the
    NN DMI magnitude of Table S2 (mRy).  The paper gives neither the
    anisotropy nor the moment: K = 0.05 mRy (easy axis z) and a field term
    mu B = 0.02 mRy along z are stand-ins of the right order."""
    return HamParams(L, Ly or L, list(PDFEIR_J[:n_shells]), [PDFEIR_D1] + [0.0] * (n_shells - 1), K,
                     (0.0, 0.0, bz))


def ham_sw(L: int = 8, b: float = 0.02, K: float = 0.05, J: float = 1.0) -> HamParams:
    """Coherent-rotation (Stoner-Wohlfarth) test: NN exchange, no DMI, easy
    axis z, field along x."""
    return HamParams(L, L, [J], [0.0], K, (b, 0.0, 0.0))


# ---------------------------------------------------------------------------
# Geometry helpers (positions only)
# ---------------------------------------------------------------------------
def positions(Lx: int, Ly: int):
    """Cartesian positions of the sites s = x + Lx*y (a1 = (1,0), a2 = (1/2, sqrt3/2))."""
    y, x = np.divmod(np.arange(Lx * Ly), Lx)
    return x + 0.5 * y, 0.5 * SQ3 * y


def min_image(Lx: int, Ly: int, cx: float, cy: float):
    """Displacement (rx, ry) of every site from the point given in lattice
    coordinates (cx, cy), minimum image over the periodic rhombic cell."""
    y, x = np.divmod(np.arange(Lx * Ly), Lx)
    # wrap lattice coordinates into [-L/2, L/2), then try the neighbouring images
    dx0 = np.mod(x - cx + 0.5 * Lx, Lx) - 0.5 * Lx
    dy0 = np.mod(y - cy + 0.5 * Ly, Ly) - 0.5 * Ly
    best = None
    for ix in (-1, 0, 1):
        for iy in (-1, 0, 1):
            dx = dx0 + ix * Lx
            dy = dy0 + iy * Ly
            rx = dx + 0.5 * dy
            ry = 0.5 * SQ3 * dy
            r2 = rx * rx + ry * ry
            if best is None:
                best = (r2, rx, ry)
            else:
                sel = r2 < best[0]
                best = (np.where(sel, r2, best[0]), np.where(sel, rx, best[1]), np.where(sel, ry, best[2]))
    return best[1], best[2]


# ---------------------------------------------------------------------------
# Textures
# ---------------------------------------------------------------------------
def neel_profile(rx, ry, R: float, helicity: float = -1.0, vorticity: int = 1, w: float = 1.0,
                 stretch: float = 1.0, axis_angle: float = 0.0):
    """Neel (anti)skyrmion ansatz around the origin: polar angle
    theta(r) = 2 atan(exp((R - r)/w)) (core down, m_z = 0 at r = R), azimuth
    vorticity*phi, in-plane part scaled by the helicity sign c.  An elliptic
    stretch elongates the texture along axis_angle."""
    if stretch != 1.0:
        ca, sa = np.cos(axis_angle), np.sin(axis_angle)
        u = rx * ca + ry * sa
        v = -rx * sa + ry * ca
        u = u / stretch
        rx, ry = u * ca - v * sa, u * sa + v * ca
    r = np.sqrt(rx * rx + ry * ry)
    th = 2.0 * np.arctan(np.exp((R - r) / w))
    ph = np.arctan2(ry, rx)
    return np.stack([helicity * np.sin(th) * np.cos(vorticity * ph),
                     helicity * np.sin(th) * np.sin(vorticity * ph),
                     np.cos(th)])


def skyrmion(Lx: int, Ly: int, R: float = 3.0, center=None, helicity: float = -1.0,
             vorticity: int = 1, **kw) -> np.ndarray:
    """Single Neel skyrmion (vorticity +1, Q = +1) or antiskyrmion
    (vorticity -1, Q = -1) in a +z background, shape (3, N)."""
    cx, cy = center if center is not None else (Lx / 2.0, Ly / 2.0)
    rx, ry = min_image(Lx, Ly, cx, cy)
    return neel_profile(rx, ry, R, helicity, vorticity, **kw)


def multi_skyrmion(Lx: int, Ly: int, centers: Sequence[Tuple[float, float]], R: float,
                   helicity: float = -1.0, vorticity: int = 1, **kw) -> np.ndarray:
    """Several cores; every site takes the profile of its nearest core."""
    best_r2 = None
    out = None
    for (cx, cy) in centers:
        rx, ry = min_image(Lx, Ly, cx, cy)
        prof = neel_profile(rx, ry, R, helicity, vorticity, **kw)
        r2 = rx * rx + ry * ry
        if out is None:
            out, best_r2 = prof, r2
        else:
            sel = r2 < best_r2
            out = np.where(sel, prof, out)
            best_r2 = np.where(sel, r2, best_r2)
    return out


def biskyrmion(Lx: int, Ly: int, R: float = 3.0, center=None, **kw) -> np.ndarray:
    """Two skyrmion cores 2.5 R apart along a1 (Q = 2)."""
    cx, cy = center if center is not None else (Lx / 2.0, Ly / 2.0)
    d = 1.25 * R
    return multi_skyrmion(Lx, Ly, [(cx - d, cy), (cx + d, cy)], R, **kw)


def uniform(N: int, direction=(0.0, 0.0, 1.0)) -> np.ndarray:
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    return np.repeat(d[:, None], N, axis=1)


def random_texture(N: int, rng: np.random.Generator) -> np.ndarray:
    """Unit spins drawn as normalised N(0, I3) samples."""
    m = rng.standard_normal((3, N))
    return m / np.sqrt((m * m).sum(0))


def add_tilt_noise(m: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian tilt noise: a tangent Gaussian displacement with standard
    deviation sigma (rad) per tangent component, followed by renormalisation."""
    xi = rng.standard_normal(m.shape) * sigma
    xi = xi - (xi * m).sum(0) * m
    out = m + xi
    return out / np.sqrt((out * out).sum(0))


def random_tangent(m: np.ndarray, n: int, rng: np.random.Generator) -> np.ndarray:
    """n random tangent directions at m, shape (n, 3, N)."""
    v = rng.standard_normal((n,) + m.shape)
    return v - (v * m[None]).sum(1, keepdims=True) * m[None]


def random_mask_disc(Lx: int, Ly: int, radius: float, center=None) -> np.ndarray:
    """uint8 mask of the sites within `radius` of a point (the masked
    perturbation subspace Omega of the explorer)."""
    cx, cy = center if center is not None else (Lx / 2.0, Ly / 2.0)
    rx, ry = min_image(Lx, Ly, cx, cy)
    return (rx * rx + ry * ry <= radius * radius).astype(np.uint8)


# ---------------------------------------------------------------------------
# Workload recipes
# ---------------------------------------------------------------------------
def nn_start(seed: int, L: int = 16, R: float = 3.0, sigma: float = 0.05) -> np.ndarray:
    """16x16 NN-model start: Neel skyrmion of radius R (helicity -1) at the
    centre plus tilt noise sigma, seeded."""
    rng = np.random.default_rng(seed)
    return add_tilt_noise(skyrmion(L, L, R), sigma, rng)


def three_shell_start(L: int, seed: int, kind: str = "skyrmion", R: float = 3.0,
                      sigma: float = 0.05) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "skyrmion":
        m = skyrmion(L, L, R)
    elif kind == "antiskyrmion":
        m = skyrmion(L, L, R, vorticity=-1)
    elif kind == "biskyrmion":
        m = biskyrmion(L, L, R)
    else:
        raise ValueError(kind)
    return add_tilt_noise(m, sigma, rng)


def two_skyrmions(L: int = 512, R: float = 4.0, seed: int = 0, sigma: float = 0.05) -> np.ndarray:
    """Two Neel skyrmions at (L/4, L/2) and (3L/4, L/2) in lattice coordinates (Q = 2)."""
    rng = np.random.default_rng(seed)
    m = multi_skyrmion(L, L, [(L / 4.0, L / 2.0), (3 * L / 4.0, L / 2.0)], R)
    return add_tilt_noise(m, sigma, rng)


@dataclass
class BatchSpec:
    L: List[int]
    kinds: List[str]
    R: List[float]
    stretch: List[float]
    angle: List[float]
    seeds: List[int]


def ragged_batch_spec(n: int = 256, seed: int = 26269, Lmin: int = 32, Lmax: int = 96) -> BatchSpec:
    """Uneven square lattices L ~ U{Lmin..Lmax}; start kind cycling
    skyrmion / antiskyrmion / biskyrmion; R ~ U[1, 3]; elliptic stretch
    ~ U[1, 1.5] along a random in-plane axis; per-member noise seeds."""
    rng = np.random.default_rng(seed)
    L = rng.integers(Lmin, Lmax + 1, n).tolist()
    kinds = [("skyrmion", "antiskyrmion", "biskyrmion")[i % 3] for i in range(n)]
    R = rng.uniform(1.0, 3.0, n).tolist()
    st = rng.uniform(1.0, 1.5, n).tolist()
    ang = rng.uniform(0.0, np.pi, n).tolist()
    seeds = rng.integers(0, 2**31 - 1, n).tolist()
    return BatchSpec(L, kinds, R, st, ang, seeds)


def fixed_size_spec(n: int, L: int, seed: int = 128) -> BatchSpec:
    """Same start rules as ragged_batch_spec on n lattices of one size L."""
    spec = ragged_batch_spec(n, seed, L, L)
    spec.L = [L] * n
    return spec


def batch_member(spec: BatchSpec, i: int, sigma: float = 0.05) -> np.ndarray:
    L = spec.L[i]
    kind = spec.kinds[i]
    kw = dict(stretch=spec.stretch[i], axis_angle=spec.angle[i])
    if kind == "skyrmion":
        m = skyrmion(L, L, spec.R[i], **kw)
    elif kind == "antiskyrmion":
        m = skyrmion(L, L, spec.R[i], vorticity=-1, **kw)
    else:
        m = biskyrmion(L, L, spec.R[i], **kw)
    return add_tilt_noise(m, sigma, np.random.default_rng(spec.seeds[i]))
