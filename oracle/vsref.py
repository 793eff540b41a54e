"""Plain FP64 CPU oracle of one finite-difference time step of the vorticity-stream-vector
phase-field method (Gallen, Munoz Biosca, Castro, Hernandez-Machado, arXiv 2601.05031).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg
of the benchmark, never by the HIP product path.

What is computed (paper references by section and equation):
  * phase-field evolution  d(phi)/dt = M (lap mu + lambda_V) - (curl psi) . grad phi
    (main text system eq. (5a); supplementary eq. (29a), (33), (38)), forward Euler
    ("Numerical implementation");
  * vorticity Poisson problem  lap omega = (1/eta) grad phi x grad mu  (eq. (5b), SM (29b));
  * stream-vector Poisson problem  lap psi = -omega  (eq. (5c), SM (29c)), Coulomb gauge
    assumed, not imposed (eq. (7) and the gauge sentence after it);
  * velocity v = curl psi (eq. (3)); vorticity omega = curl v (eq. (4)), used for the walls;
  * chemical potential of the phase-field bending energy, SM eq. (35) (energy SM (30)), or
    of the Cahn-Hilliard energy (eq. F_CH, SM (31)): mu = phi^3 - phi - sigma lap phi;
  * area and volume functionals SM (32) and (37), penalty multipliers (SM "Lagrange
    multipliers" section, eq. (38));
  * wall values of psi and omega from the no-body channel flow ("Boundary conditions").

Discretisation ("Numerical implementation": fixed cubic grid, equal spacing h, forward Euler,
segregated order phi -> omega -> psi inside one step). The readings where the paper is silent
or inconsistent are listed here and in the design notes:
  R1 nodes at (i h, j h, k h), arrays (nx, ny, nz), z fastest; x, z periodic; walls are the
     node planes j = 0 and j = ny - 1, H = (ny - 1) h.
  R2 second-order operators: 7-point Laplacian L_h, central differences D_a.
  R3 phi, g and mu use mirror ghosts in y (u[-1] = u[1], u[ny] = u[ny-2]): no-flux walls.
  R4 trapezoid weights w_j = 1/2 on wall rows, 1 elsewhere; |Omega| = nx nz (ny-1) h^3.
  R5 C_b = bend_scale * 3 sqrt(2) kappa / (8 eps^3); bend_scale = 1 is SM eq. (35).
  R6 area term of SM eq. (35) kept as -gamma_A lap phi, gamma_A = gamma0 + k_A (A - A0) / A0.
  R7 lambda_V = 2 rate_V (V0 - V) / (M |Omega|), so V relaxes to V0 at rate rate_V.
  R8 V = (|Omega| + h^3 sum_w phi) / 2 (SM (37) with its V_0 read as the domain volume).
  R9 mu, lambda_V, gamma_A are functions of the current phi: at level n+1 they use A, V of
     phi^{n+1}. The step is: advance phi with mu^n, lambda_V^n, psi^n; then V, A, lambda_V,
     gamma_A and mu from phi^{n+1}; then omega^{n+1}; then psi^{n+1}.
  R10 wall nodes move with the wall: v = (0, 0, v_wall) there, not curl psi.
  R11 wall tables re-derived from v (the printed Couette forms fail lap psi = -omega):
      Poiseuille (centreline U): v_z = 4U y(H-y)/H^2, psi_x = -(4U/H^2)(H y^2/2 - y^3/3),
      omega_x = (4U/H^2)(H - 2y); Couette (u0 at y = 0, u1 at y = H): v_z = u0 + (u1-u0) y/H,
      psi_x = -(u0 y + (u1-u0) y^2/(2H)), omega_x = (u1-u0)/H; other components 0.
  R12 each Poisson problem is the exact solution of the discrete 7-point system on the
      interior nodes with Dirichlet wall values (here by the eigen-decomposition of L_h:
      DFT in x and z, sine transform in y).
  R23 inertial variant (SM "Time-dependency and inertial flow", eq. (36)): with density
      rho > 0 the vorticity obeys (rho/eta) d(omega)/dt - lap omega = -(1/eta) grad phi x
      grad mu. The time derivative is taken backward (implicit) in the same segregated
      step: (L_h - a) omega^{n+1} = S^{n+1} - a omega^n, a = rho / (eta dt), with the same
      Dirichlet wall values; psi then from eq. (5c) as before. rho = 0 is eq. (5b).
  R24 the initial omega^0 of an inertial run is the quasi-steady one of eq. (5b).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np
import scipy.fft

BENDING = "bending"
CAHN_HILLIARD = "cahn_hilliard"
POISEUILLE = "poiseuille"
COUETTE = "couette"


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    h: float = 1.0

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def H(self) -> float:
        return (self.ny - 1) * self.h

    @property
    def domain_volume(self) -> float:
        return self.nx * self.nz * (self.ny - 1) * self.h**3

    def weights(self) -> np.ndarray:
        """Trapezoid weights in y as a (1, ny, 1) array (R4)."""
        w = np.ones(self.ny)
        w[0] = w[-1] = 0.5
        return w[None, :, None]

    def y(self) -> np.ndarray:
        return np.arange(self.ny) * self.h


@dataclass(frozen=True)
class Walls:
    kind: str          # POISEUILLE or COUETTE; flow along +z
    u0: float          # Poiseuille: centreline speed; Couette: speed of the wall y = 0
    u1: float = 0.0    # Couette: speed of the wall y = H


@dataclass(frozen=True)
class Params:
    model: str = BENDING
    eta: float = 1.0
    mobility: float = 1.0
    eps: float = 1.0
    kappa: float = 1.0
    sigma: float = 1.0
    gamma0: float = 0.0
    rate_V: float = 0.0
    k_A: float = 0.0
    bend_scale: float = 1.0
    rho: float = 0.0      # fluid density of the inertial variant (R23); 0 = eq. (5b)

    @property
    def C_b(self) -> float:
        return self.bend_scale * 3.0 * math.sqrt(2.0) * self.kappa / (8.0 * self.eps**3)


@dataclass
class State:
    phi: np.ndarray
    mu: np.ndarray
    omega: np.ndarray     # (3, nx, ny, nz)
    psi: np.ndarray       # (3, nx, ny, nz)
    V0: float
    A0: float
    V: float
    A: float
    lam_V: float
    gamma_A: float
    step: int = 0


# ----------------------------------------------------------------------------- operators
def _pad_y_mirror(u: np.ndarray) -> np.ndarray:
    """u with one mirror ghost row on each wall (R3)."""
    return np.concatenate([u[:, 1:2, :], u, u[:, -2:-1, :]], axis=1)


def lap_mirror(u: np.ndarray, h: float) -> np.ndarray:
    """7-point Laplacian at every node, periodic in x, z, mirror ghosts in y (R2, R3)."""
    p = _pad_y_mirror(u)
    s = (np.roll(u, 1, 0) + np.roll(u, -1, 0)
         + p[:, 2:, :] + p[:, :-2, :]
         + np.roll(u, 1, 2) + np.roll(u, -1, 2))
    return (s - 6.0 * u) / (h * h)


def grad_mirror(u: np.ndarray, h: float):
    """Central differences (D_x u, D_y u, D_z u) at every node, mirror ghosts in y."""
    p = _pad_y_mirror(u)
    dx = (np.roll(u, -1, 0) - np.roll(u, 1, 0)) / (2.0 * h)
    dy = (p[:, 2:, :] - p[:, :-2, :]) / (2.0 * h)
    dz = (np.roll(u, -1, 2) - np.roll(u, 1, 2)) / (2.0 * h)
    return dx, dy, dz


def lap_interior(u: np.ndarray, h: float) -> np.ndarray:
    """7-point Laplacian on the interior rows j = 1..ny-2, using the stored wall rows."""
    c = u[:, 1:-1, :]
    s = (np.roll(c, 1, 0) + np.roll(c, -1, 0)
         + u[:, 2:, :] + u[:, :-2, :]
         + np.roll(c, 1, 2) + np.roll(c, -1, 2))
    return (s - 6.0 * c) / (h * h)


def curl_interior(psi: np.ndarray, h: float) -> np.ndarray:
    """v = curl psi (main text eq. (3)) by central differences on the interior rows."""
    def d(f, axis):
        if axis == 1:
            return (f[:, 2:, :] - f[:, :-2, :]) / (2.0 * h)
        c = f[:, 1:-1, :]
        return (np.roll(c, -1, axis) - np.roll(c, 1, axis)) / (2.0 * h)

    px, py, pz = psi
    return np.stack([d(pz, 1) - d(py, 2),
                     d(px, 2) - d(pz, 0),
                     d(py, 0) - d(px, 1)])


# ------------------------------------------------------------------ walls ("Boundary conditions")
def wall_profiles(grid: Grid, walls: Walls):
    """No-body channel flow as functions of y at the node rows: (v_z, psi_x, omega_x) (R11).

    psi_x = -int_0^y v_z makes v = curl psi = (0, 0, v_z); omega_x = dv_z/dy is curl v;
    then d^2 psi_x / dy^2 = -omega_x, the stream-vector problem without a body.
    """
    y = grid.y()
    H = grid.H
    if walls.kind == POISEUILLE:
        U = walls.u0
        vz = 4.0 * U * y * (H - y) / H**2
        psix = -(4.0 * U / H**2) * (H * y**2 / 2.0 - y**3 / 3.0)
        omx = (4.0 * U / H**2) * (H - 2.0 * y)
    elif walls.kind == COUETTE:
        u0, u1 = walls.u0, walls.u1
        vz = u0 + (u1 - u0) * y / H
        psix = -(u0 * y + (u1 - u0) * y**2 / (2.0 * H))
        omx = np.full_like(y, (u1 - u0) / H)
    else:
        raise ValueError(walls.kind)
    return vz, psix, omx


def no_body_fields(grid: Grid, walls: Walls):
    """(omega, psi) of the channel without a body, on every node."""
    _, psix, omx = wall_profiles(grid, walls)
    omega = np.zeros((3,) + grid.shape)
    psi = np.zeros((3,) + grid.shape)
    omega[0] += omx[None, :, None]
    psi[0] += psix[None, :, None]
    return omega, psi


# ------------------------------------------------------------- free energy and chemical potential
def chemical_potential(phi: np.ndarray, grid: Grid, params: Params, gamma_A: float) -> np.ndarray:
    """mu = delta F / delta phi on every node.

    Bending (SM eq. (35)): g = phi^3 - phi - eps^2 lap phi,
        mu = C_b [ (3 phi^2 - 1) g - eps^2 lap g ] - gamma_A lap phi.
    Cahn-Hilliard (eq. F_CH, SM (31); SM (1c) with sigma for eps^2): mu = phi^3 - phi - sigma lap phi.
    """
    h = grid.h
    lphi = lap_mirror(phi, h)
    if params.model == CAHN_HILLIARD:
        return phi**3 - phi - params.sigma * lphi
    eps2 = params.eps**2
    g = phi**3 - phi - eps2 * lphi
    return params.C_b * ((3.0 * phi**2 - 1.0) * g - eps2 * lap_mirror(g, h)) - gamma_A * lphi


def bending_energy(phi: np.ndarray, grid: Grid, params: Params) -> float:
    """Discrete SM eq. (30) without the area term: 3 sqrt(2) kappa/(8 eps^3) h^3 sum_w g^2."""
    g = phi**3 - phi - params.eps**2 * lap_mirror(phi, grid.h)
    cF = 3.0 * math.sqrt(2.0) * params.kappa / (8.0 * params.eps**3)
    return cF * grid.h**3 * float(np.sum(grid.weights() * g * g))


# ------------------------------------------------------------------------------- functionals
def volume(phi: np.ndarray, grid: Grid) -> float:
    """V = (|Omega| + int phi) / 2, SM eq. (37) (R8), trapezoid rule in y."""
    return 0.5 * (grid.domain_volume + grid.h**3 * float(np.sum(grid.weights() * phi)))


def area(phi: np.ndarray, grid: Grid, eps: float) -> float:
    """A = 3/(2 sqrt 2) int (eps/2)|grad phi|^2 + (phi^2-1)^2/(4 eps), SM eq. (32)."""
    dx, dy, dz = grad_mirror(phi, grid.h)
    dens = 0.5 * eps * (dx * dx + dy * dy + dz * dz) + (phi * phi - 1.0) ** 2 / (4.0 * eps)
    return 3.0 / (2.0 * math.sqrt(2.0)) * grid.h**3 * float(np.sum(grid.weights() * dens))


def multipliers(V: float, A: float, V0: float, A0: float, grid: Grid, params: Params):
    """(lambda_V, gamma_A) by the penalty method (R6, R7). With no interface (A0 = 0) or
    k_A = 0 the area penalty is off."""
    lam_V = 2.0 * params.rate_V * (V0 - V) / (params.mobility * grid.domain_volume)
    gamma_A = params.gamma0
    if params.k_A != 0.0 and A0 > 0.0:
        gamma_A += params.k_A * (A - A0) / A0
    return lam_V, gamma_A


# ------------------------------------------------------------------------------ time stepping
def velocity(psi: np.ndarray, grid: Grid, walls: Walls) -> np.ndarray:
    """v on every node: curl psi inside, the wall velocity on the walls (R10)."""
    vz, _, _ = wall_profiles(grid, walls)
    v = np.zeros((3,) + grid.shape)
    v[:, :, 1:-1, :] = curl_interior(psi, grid.h)
    v[2, :, 0, :] = vz[0]
    v[2, :, -1, :] = vz[-1]
    return v


def advance_phi(phi, mu, v, lam_V, dt, grid: Grid, params: Params) -> np.ndarray:
    """phi^{n+1} = phi^n + dt [ M (lap mu^n + lambda_V^n) - v^n . grad phi^n ] on every node."""
    dx, dy, dz = grad_mirror(phi, grid.h)
    adv = v[0] * dx + v[1] * dy + v[2] * dz
    return phi + dt * (params.mobility * (lap_mirror(mu, grid.h) + lam_V) - adv)


def vorticity_source(phi, mu, grid: Grid, eta: float) -> np.ndarray:
    """S = (1/eta) grad phi x grad mu on the interior rows (main text eq. (5b))."""
    fx, fy, fz = (a[:, 1:-1, :] for a in grad_mirror(phi, grid.h))
    mx, my, mz = (a[:, 1:-1, :] for a in grad_mirror(mu, grid.h))
    return np.stack([fy * mz - fz * my, fz * mx - fx * mz, fx * my - fy * mx]) / eta


def poisson_solve(b_int: np.ndarray, u_lo: np.ndarray, u_hi: np.ndarray, grid: Grid,
                  shift: float = 0.0) -> np.ndarray:
    """Exact solution of (L_h - shift) u = b on the interior rows with Dirichlet walls (R12;
    shift > 0 is the implicit inertial vorticity problem of R23).

    b_int: (nx, ny-2, nz) right-hand side on j = 1..ny-2. u_lo, u_hi: (nx, nz) wall values
    at j = 0 and j = ny-1. The wall values are moved to the right-hand side, then L_h with
    homogeneous Dirichlet walls is inverted through its eigenvectors: discrete Fourier modes
    in x and z (eigenvalue (2 cos(2 pi p/n) - 2)/h^2) and sine modes sin(pi m j/(ny-1)) in y
    (eigenvalue (2 cos(pi m/(ny-1)) - 2)/h^2, m = 1..ny-2); the shift moves every eigenvalue
    by -shift.
    """
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    M = ny - 2
    bt = np.array(b_int, dtype=np.float64, copy=True)
    bt[:, 0, :] -= u_lo / h**2
    bt[:, -1, :] -= u_hi / h**2
    lx = (2.0 * np.cos(2.0 * np.pi * np.arange(nx) / nx) - 2.0) / h**2
    ly = (2.0 * np.cos(np.pi * np.arange(1, M + 1) / (M + 1)) - 2.0) / h**2
    lz = (2.0 * np.cos(2.0 * np.pi * np.arange(nz // 2 + 1) / nz) - 2.0) / h**2
    bh = scipy.fft.dst(bt, type=1, axis=1)
    bh = scipy.fft.rfft(bh, axis=2)
    bh = scipy.fft.fft(bh, axis=0)
    uh = bh / (lx[:, None, None] + ly[None, :, None] + lz[None, None, :] - shift)
    u = scipy.fft.ifft(uh, axis=0)
    u = scipy.fft.irfft(u, n=nz, axis=2)
    return scipy.fft.idst(u, type=1, axis=1)


def solve_flow(phi, mu, grid: Grid, walls: Walls, params: Params, omega_prev=None,
               dt: float | None = None):
    """omega from eq. (5b), then psi from eq. (5c) (segregated order), walls from R11. With
    params.rho > 0 and the previous vorticity and dt given, omega from the implicit inertial
    problem of R23 instead."""
    omega, psi = no_body_fields(grid, walls)
    S = vorticity_source(phi, mu, grid, params.eta)
    shift = 0.0
    if params.rho > 0.0 and omega_prev is not None:
        shift = params.rho / (params.eta * dt)
        S = S - shift * omega_prev[:, :, 1:-1, :]
    for c in range(3):
        omega[c, :, 1:-1, :] = poisson_solve(S[c], omega[c, :, 0, :], omega[c, :, -1, :], grid,
                                             shift)
    for c in range(3):
        psi[c, :, 1:-1, :] = poisson_solve(-omega[c, :, 1:-1, :], psi[c, :, 0, :], psi[c, :, -1, :], grid)
    return omega, psi


def init_state(grid: Grid, walls: Walls, params: Params, phi0: np.ndarray, flow: bool = True) -> State:
    """Initial state: V0 = V[phi0], A0 = A[phi0], lambda_V = 0, gamma_A = gamma0, mu from phi0,
    omega and psi solved from phi0."""
    phi = np.array(phi0, dtype=np.float64, copy=True)
    V0 = volume(phi, grid)
    A0 = area(phi, grid, params.eps)
    lam_V, gamma_A = multipliers(V0, A0, V0, A0, grid, params)
    mu = chemical_potential(phi, grid, params, gamma_A)
    if flow:
        omega, psi = solve_flow(phi, mu, grid, walls, params)
    else:
        omega = np.zeros((3,) + grid.shape)
        psi = np.zeros((3,) + grid.shape)
    return State(phi, mu, omega, psi, V0, A0, V0, A0, lam_V, gamma_A, 0)


def step(s: State, dt: float, grid: Grid, walls: Walls, params: Params, flow: bool = True) -> State:
    """One time step n -> n+1 in the paper's segregated order (R9)."""
    v = velocity(s.psi, grid, walls) if flow else np.zeros((3,) + grid.shape)
    phi = advance_phi(s.phi, s.mu, v, s.lam_V, dt, grid, params)
    V = volume(phi, grid)
    A = area(phi, grid, params.eps)
    lam_V, gamma_A = multipliers(V, A, s.V0, s.A0, grid, params)
    mu = chemical_potential(phi, grid, params, gamma_A)
    if flow:
        omega, psi = solve_flow(phi, mu, grid, walls, params, s.omega, dt)
    else:
        omega, psi = s.omega, s.psi
    return replace(s, phi=phi, mu=mu, omega=omega, psi=psi, V=V, A=A, lam_V=lam_V,
                   gamma_A=gamma_A, step=s.step + 1)


def run(grid: Grid, walls: Walls, params: Params, phi0: np.ndarray, dt: float, nsteps: int,
        flow: bool = True) -> State:
    s = init_state(grid, walls, params, phi0, flow)
    for _ in range(nsteps):
        s = step(s, dt, grid, walls, params, flow)
    return s
