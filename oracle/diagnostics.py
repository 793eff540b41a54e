"""Paper diagnostics of a state, plain FP64 numpy.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the HIP product path.

  * in-plane shear stress ("In plane shear"): sigma_ij = eta (d_j v_i + d_i v_j) and its
    intensity sigma_t = sqrt(sigma_xy^2 + sigma_yz^2 + sigma_xz^2), with v on every node as
    the step uses it (curl psi inside, the wall speed on the walls) and central differences;
    reading R20: sigma_t is evaluated on the interior rows, where every central difference has
    both neighbours, and is 0 on the wall rows (the interface never reaches the walls);
  * the flow observables of the results section (the integrals of the squared fluctuations
    of omega and psi about the no-body fields omega_0, psi_0), trapezoid rule in y (R4);
  * the free energy: bending, SM eq. (30) without the area term (``vsref.bending_energy``), or
    Cahn-Hilliard, eq. F_CH: int 1/4 (phi^2 - 1)^2 + (sigma/2) |grad phi|^2;
  * two checks of a run's health: the gauge defect int (div psi)^2 over the interior rows
    (the Coulomb gauge div psi = 0 is assumed, not imposed: main text after eq. (7), reading
    R14), with central differences, and the largest speed |v| over the nodes;
  * time-dependent walls (SM "Time-dependency and inertial flow": only the boundary data
    change): ``set_walls`` replaces the wall speeds and re-solves omega and psi from the
    current phi and mu with the new walls.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from .vsref import (
    BENDING,
    Grid,
    Params,
    State,
    Walls,
    bending_energy,
    grad_mirror,
    no_body_fields,
    solve_flow,
    velocity,
)


def shear_stress(psi: np.ndarray, grid: Grid, walls: Walls, eta: float) -> np.ndarray:
    """sigma_t on every node (0 on the wall rows, R20)."""
    v = velocity(psi, grid, walls)
    h = grid.h

    def d(f, axis):
        # central difference on the interior rows (true neighbours in y)
        if axis == 1:
            return (f[:, 2:, :] - f[:, :-2, :]) / (2.0 * h)
        c = f[:, 1:-1, :]
        return (np.roll(c, -1, axis) - np.roll(c, 1, axis)) / (2.0 * h)

    vx, vy, vz = v
    sxy = eta * (d(vx, 1) + d(vy, 0))
    syz = eta * (d(vy, 2) + d(vz, 1))
    sxz = eta * (d(vx, 2) + d(vz, 0))
    out = np.zeros(grid.shape)
    out[:, 1:-1, :] = np.sqrt(sxy * sxy + syz * syz + sxz * sxz)
    return out


def observables(omega: np.ndarray, psi: np.ndarray, grid: Grid, walls: Walls):
    """(int |omega - omega_0|^2, int |psi - psi_0|^2) over the domain, trapezoid weights."""
    om0, ps0 = no_body_fields(grid, walls)
    w = grid.weights()
    h3 = grid.h**3
    oo = h3 * float(np.sum(w * np.sum((omega - om0) ** 2, axis=0)))
    op = h3 * float(np.sum(w * np.sum((psi - ps0) ** 2, axis=0)))
    return oo, op


def gauge_defect(psi: np.ndarray, grid: Grid) -> float:
    """h^3 sum over the interior rows of (D_x psi_x + D_y psi_y + D_z psi_z)^2."""
    h = grid.h
    px, py, pz = psi
    dx = (np.roll(px, -1, 0) - np.roll(px, 1, 0))[:, 1:-1, :] / (2.0 * h)
    dy = (py[:, 2:, :] - py[:, :-2, :]) / (2.0 * h)
    dz = (np.roll(pz, -1, 2) - np.roll(pz, 1, 2))[:, 1:-1, :] / (2.0 * h)
    div = dx + dy + dz
    return grid.h**3 * float(np.sum(div * div))


def max_speed(psi: np.ndarray, grid: Grid, walls: Walls) -> float:
    """max |v| over the nodes, v as the step uses it."""
    v = velocity(psi, grid, walls)
    return float(np.sqrt(np.max(np.sum(v * v, axis=0))))


def ch_energy(phi: np.ndarray, grid: Grid, sigma: float) -> float:
    """F_CH = int 1/4 (phi^2 - 1)^2 + (sigma/2) |D phi|^2, trapezoid weights, mirror ghosts."""
    dx, dy, dz = grad_mirror(phi, grid.h)
    dens = 0.25 * (phi * phi - 1.0) ** 2 + 0.5 * sigma * (dx * dx + dy * dy + dz * dz)
    return grid.h**3 * float(np.sum(grid.weights() * dens))


def free_energy(phi: np.ndarray, grid: Grid, params: Params) -> float:
    if params.model == BENDING:
        return bending_energy(phi, grid, params)
    return ch_energy(phi, grid, params.sigma)


def set_walls(s: State, grid: Grid, walls: Walls, params: Params) -> State:
    """The state with new wall speeds: omega, psi re-solved from its phi and mu."""
    omega, psi = solve_flow(s.phi, s.mu, grid, walls, params)
    return replace(s, omega=omega, psi=psi)


def no_body_state_fields(grid: Grid, walls: Walls):
    """(omega_0, psi_0) on every node: the reference of the observables."""
    return no_body_fields(grid, walls)
