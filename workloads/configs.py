"""Named synthetic workloads: grid, channel flow, physical parameters, time step and seed shape.

All lengths are in lattice units (h = 1) unless a grid says otherwise. The flow is
along +z, the walls are normal to y, x and z are periodic.

  vesicle32   : 32^3, plane Poiseuille (centreline 0.05), membrane kappa = 1, no
                surface tension, seeded l <= 3 shape perturbation of radius 8,
                5 steps of dt = 1e-3, Poisson relative residual 1e-10.
  vesicle128  : 128^3, plane Poiseuille (centreline 0.05), prolate membrane of
                area-equivalent radius 24 and reduced volume 0.8, kappa in
                {0.5, 1, 2}, volume/area penalties on, 200 steps of dt = 5e-4.
  droplet256  : 128 x 128 x 256 (256 along the flow), plane Couette with walls at
                -0.05 / +0.05, Cahn-Hilliard droplet R = 20, sigma = 1, 500 steps of
                dt = 1e-3.
  adjoint96   : 96^3, plane Poiseuille (centreline 0.05), membrane kappa = 1 with a
                seeded l <= 3 shape perturbation of radius 16, 50 steps of dt = 5e-4; the
                differentiation workload (loss ||phi^50 - phi_target||^2, the target from
                kappa = 1.5 and 1.2 times the wall speed, checkpoints every 10 steps).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from .shapes import (GridSpec, alm_coefficients, phi_prolate, phi_prolate_sh, phi_sh_vesicle,
                     phi_sphere, prolate_axes)

BENDING = "bending"
CAHN_HILLIARD = "cahn_hilliard"
POISEUILLE = "poiseuille"
COUETTE = "couette"


@dataclass(frozen=True)
class Workload:
    name: str
    grid: GridSpec
    wall_kind: str
    u0: float
    u1: float
    model: str
    eta: float = 1.0
    mobility: float = 1.0
    eps: float = 1.0
    kappa: float = 1.0
    sigma: float = 1.0
    gamma0: float = 0.0
    rate_V: float = 0.0
    k_A: float = 0.0
    bend_scale: float = 1.0
    rtol: float = 1e-10
    max_cycles: int = 3
    rho: float = 0.0             # fluid density of the inertial variant; 0 = Stokes flow
    dt: float = 1e-3
    nsteps: int = 5
    shape: str = "sh"            # "sh" | "prolate" | "sphere"
    R0: float = 8.0
    seed: int = 0
    prolate_Vr: float = 0.8
    center: tuple | None = None
    extra: dict = field(default_factory=dict)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)

    @property
    def width(self) -> float:
        if self.model == CAHN_HILLIARD:
            return math.sqrt(2.0 * self.sigma)
        return math.sqrt(2.0) * self.eps

    def phi0(self) -> np.ndarray:
        g = self.grid
        if self.shape == "sh":
            return phi_sh_vesicle(g, self.R0, alm_coefficients(self.seed), self.width, self.center)
        if self.shape == "prolate":
            a, b = prolate_axes(self.R0, self.prolate_Vr)
            return phi_prolate(g, a, b, self.width, self.center)
        if self.shape == "sphere":
            return phi_sphere(g, self.R0, self.width, self.center)
        if self.shape == "prolate_sh":
            a, b = prolate_axes(self.R0, self.prolate_Vr)
            return phi_prolate_sh(g, a, b, np.asarray(self.extra["alm"]), self.width, self.center)
        raise ValueError(self.shape)

    def params(self) -> dict:
        return dict(model=self.model, eta=self.eta, mobility=self.mobility, eps=self.eps,
                    kappa=self.kappa, sigma=self.sigma, gamma0=self.gamma0, rate_V=self.rate_V,
                    k_A=self.k_A, bend_scale=self.bend_scale, rtol=self.rtol,
                    max_cycles=self.max_cycles, rho=self.rho)

    def walls(self) -> dict:
        return dict(kind=self.wall_kind, u0=self.u0, u1=self.u1)


WORKLOADS = {
    "vesicle32": Workload(
        name="vesicle32", grid=GridSpec(32, 32, 32), wall_kind=POISEUILLE, u0=0.05, u1=0.0,
        model=BENDING, kappa=1.0, gamma0=0.0, dt=1e-3, nsteps=5, shape="sh", R0=8.0, seed=0),
    "vesicle128": Workload(
        name="vesicle128", grid=GridSpec(128, 128, 128), wall_kind=POISEUILLE, u0=0.05, u1=0.0,
        model=BENDING, kappa=1.0, rate_V=10.0, k_A=1.0, dt=5e-4, nsteps=200, shape="prolate",
        R0=24.0, prolate_Vr=0.8),
    "droplet256": Workload(
        name="droplet256", grid=GridSpec(128, 128, 256), wall_kind=COUETTE, u0=-0.05, u1=0.05,
        model=CAHN_HILLIARD, sigma=1.0, dt=1e-3, nsteps=500, shape="sphere", R0=20.0),
    "adjoint96": Workload(
        name="adjoint96", grid=GridSpec(96, 96, 96), wall_kind=POISEUILLE, u0=0.05, u1=0.0,
        model=BENDING, kappa=1.0, dt=5e-4, nsteps=50, shape="sh", R0=16.0, seed=0),
}


def batch_instances(count: int = 64, seed_base: int = 1000) -> list[Workload]:
    """The batched workload: instance i draws from default_rng(seed_base + i) a cubic grid
    from {48, 64, 96, 128}, a plane Poiseuille (centreline 0.05) or Couette (-/+0.05) channel
    by coin flip, an area-equivalent vesicle radius U(0.15, 0.25) of the channel width,
    kappa ~ U(0.5, 2), reduced volume ~ U(0.7, 0.95) and l <= 3 shape coefficients
    N(0, 0.02^2); membrane with volume/area penalties, dt = 5e-4."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed_base + i)
        n = int(rng.choice([48, 64, 96, 128]))
        couette = bool(rng.integers(0, 2))
        frac = float(rng.uniform(0.15, 0.25))
        kappa = float(rng.uniform(0.5, 2.0))
        vr = float(rng.uniform(0.7, 0.95))
        alm = rng.normal(0.0, 0.02, 16)
        g = GridSpec(n, n, n)
        out.append(Workload(
            name=f"batch{i}", grid=g, wall_kind=COUETTE if couette else POISEUILLE,
            u0=-0.05 if couette else 0.05, u1=0.05 if couette else 0.0, model=BENDING,
            kappa=kappa, rate_V=10.0, k_A=1.0, dt=5e-4, nsteps=100, shape="prolate_sh",
            R0=frac * g.H, prolate_Vr=vr, seed=seed_base + i, extra={"alm": alm.tolist()}))
    return out


def workload(name: str, **overrides) -> Workload:
    return WORKLOADS[name].with_(**overrides)
