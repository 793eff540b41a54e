"""Seed shapes for the phase field phi on the node grid.

Node (i, j, k) sits at (i h, j h, k h); arrays have shape (nx, ny, nz), z fastest.
x and z are periodic (period nx h, nz h); the walls are the planes j = 0 and
j = ny - 1, so the channel height is H = (ny - 1) h. A body is centred at
(nx h / 2, H / 2, nz h / 2) unless a centre is given, distances use the minimum
image in x and z, and the polar axis of the spherical coordinates is z (the flow
direction).

Every shape is a radial tanh profile phi = tanh((R(theta, varphi) - r) / w),
+1 inside and -1 outside. The width w is sqrt(2) eps for a membrane and
sqrt(2 sigma) for a Cahn-Hilliard droplet, the one-dimensional equilibrium
profile of the supplementary matched-asymptotics section, eq. (10).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.special


@dataclass(frozen=True)
class GridSpec:
    nx: int
    ny: int
    nz: int
    h: float = 1.0

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    @property
    def H(self):
        return (self.ny - 1) * self.h


def alm_coefficients(seed: int, sigma: float = 0.02, lmax: int = 3) -> np.ndarray:
    """Random shape coefficients a_lm ~ N(0, sigma^2), l = 0..lmax, lexicographic (l, m)."""
    n = (lmax + 1) ** 2
    return np.random.default_rng(seed).normal(0.0, sigma, n)


def real_sph_harm(l: int, m: int, theta, varphi):
    """Real orthonormal spherical harmonic; theta polar (from +z), varphi azimuth.

    m > 0: sqrt(2) Re Y_l^m, m < 0: sqrt(2) Im Y_l^|m|, m = 0: Y_l^0, with scipy's
    complex orthonormal Y_l^m (Condon-Shortley phase included).
    """
    y = scipy.special.sph_harm_y(l, abs(m), theta, varphi)
    if m > 0:
        return math.sqrt(2.0) * y.real
    if m < 0:
        return math.sqrt(2.0) * y.imag
    return y.real


def _coords(g: GridSpec, center=None):
    cx, cy, cz = center if center is not None else (g.nx * g.h / 2, g.H / 2, g.nz * g.h / 2)
    x = np.arange(g.nx) * g.h - cx
    y = np.arange(g.ny) * g.h - cy
    z = np.arange(g.nz) * g.h - cz
    Lx, Lz = g.nx * g.h, g.nz * g.h
    x = x - Lx * np.round(x / Lx)
    z = z - Lz * np.round(z / Lz)
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    theta = np.arccos(np.clip(np.divide(Z, r, out=np.ones_like(r), where=r > 0), -1.0, 1.0))
    varphi = np.arctan2(Y, X)
    return r, theta, varphi


def phi_sh_vesicle(g: GridSpec, R0: float, alm: np.ndarray, width: float, center=None) -> np.ndarray:
    """phi = tanh((R0 (1 + sum a_lm Y_lm) - r) / width), l up to sqrt(len(alm)) - 1."""
    r, theta, varphi = _coords(g, center)
    lmax = int(round(math.sqrt(len(alm)))) - 1
    s = np.zeros_like(r)
    idx = 0
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            s += alm[idx] * real_sph_harm(l, m, theta, varphi)
            idx += 1
    R = R0 * (1.0 + s)
    return np.tanh((R - r) / width)


def phi_sphere(g: GridSpec, R: float, width: float, center=None) -> np.ndarray:
    r, _, _ = _coords(g, center)
    return np.tanh((R - r) / width)


def phi_prolate_sh(g: GridSpec, a: float, b: float, alm: np.ndarray, width: float,
                   center=None) -> np.ndarray:
    """Spheroid (semi-axis a along z, b in x, y) with a spherical-harmonic perturbation:
    R(theta, varphi) = R_spheroid(theta) (1 + sum a_lm Y_lm)."""
    r, theta, varphi = _coords(g, center)
    Rs = 1.0 / np.sqrt(np.cos(theta) ** 2 / a**2 + np.sin(theta) ** 2 / b**2)
    lmax = int(round(math.sqrt(len(alm)))) - 1
    s = np.zeros_like(r)
    idx = 0
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            s += alm[idx] * real_sph_harm(l, m, theta, varphi)
            idx += 1
    return np.tanh((Rs * (1.0 + s) - r) / width)


def phi_prolate(g: GridSpec, a: float, b: float, width: float, center=None) -> np.ndarray:
    """Spheroid with semi-axis a along z and b in x, y: R(theta) = (cos^2/a^2 + sin^2/b^2)^(-1/2)."""
    r, theta, _ = _coords(g, center)
    R = 1.0 / np.sqrt(np.cos(theta) ** 2 / a**2 + np.sin(theta) ** 2 / b**2)
    return np.tanh((R - r) / width)


def prolate_area(a: float, b: float) -> float:
    """Surface area of a prolate spheroid (a >= b): 2 pi b^2 (1 + a asin(e) / (b e))."""
    if a <= b * (1 + 1e-14):
        return 4.0 * math.pi * b * b
    e = math.sqrt(1.0 - (b * b) / (a * a))
    return 2.0 * math.pi * b * b * (1.0 + a * math.asin(e) / (b * e))


def prolate_axes(R_area: float, reduced_volume: float) -> tuple[float, float]:
    """Semi-axes (a, b) of the prolate spheroid with area 4 pi R_area^2 and the given
    reduced volume V / ((4/3) pi (A / 4 pi)^(3/2)) (supplementary eq. (40)), by bisection
    on the aspect ratio a / b."""
    A = 4.0 * math.pi * R_area**2

    def vr(t):
        b = math.sqrt(A / prolate_area(t, 1.0))
        return t * b**3 / R_area**3, b

    lo, hi = 1.0, 50.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        v, _ = vr(mid)
        if v > reduced_volume:
            lo = mid
        else:
            hi = mid
    t = 0.5 * (lo + hi)
    _, b = vr(t)
    return t * b, b
