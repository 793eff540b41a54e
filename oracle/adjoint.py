"""Reverse mode (discrete adjoint) of one oracle time step, in plain FP64 numpy.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the HIP product path.

The forward step (``vsref.step``) maps phi^n to phi^{n+1}; every other quantity it uses at
level n (mu^n, omega^n, psi^n, V, A, lambda_V^n, gamma_A^n) is a function of phi^n and of the
parameters (reading R9), with V0 and A0 fixed by the initial state. For a loss L, one reverse
step takes a = dL/dphi^{n+1} and returns

    dL/dphi^n  = (d phi^{n+1} / d phi^n)^T a          (V0, A0 held fixed),
    dL/dkappa  : this step's term a^T d phi^{n+1} / d kappa,
    dL/ds      : this step's term a^T d phi^{n+1} / d s, where s scales both wall speeds
                 (u0, u1) -> (s u0, s u1) at s = 1. Every wall table (v_z, psi, omega on the
                 walls; "Boundary conditions", R11) is linear in the wall speeds, so its
                 s-derivative at s = 1 is the table itself.

The derivative is written operator by operator from the forward step, each transpose taken
from the operator's definition:

  * L_h with mirror ghosts is symmetric in the trapezoid-weighted inner product (R3, R4), so
    L_h^T u = w L_h (u / w);
  * the central difference D_c: periodic in x, z, so D^T = -D; in y the mirrored difference
    vanishes on the wall rows, so (D_y^T u)_j = (u_{j-1} - u_{j+1}) / 2h with u kept on the
    interior rows only;
  * the interior Laplacian with Dirichlet walls is symmetric, so each adjoint Poisson problem
    is the same solve with homogeneous walls; the wall values enter the interior rows 1 and
    ny-2 with weight 1/h^2, which gives their adjoint;
  * V (SM (37), R8), A (SM (32)), lambda_V (R7) and gamma_A (R6) are differentiated directly.
"""
from __future__ import annotations

import math
from dataclasses import replace

import numpy as np

from .vsref import (
    BENDING,
    Grid,
    Params,
    State,
    Walls,
    grad_mirror,
    init_state,
    lap_mirror,
    poisson_solve,
    step,
    velocity,
    wall_profiles,
)


def lap_mirror_T(u: np.ndarray, grid: Grid) -> np.ndarray:
    """Transpose of lap_mirror: w L_h (u / w) (W L_h is symmetric)."""
    w = grid.weights()
    return w * lap_mirror(u / w, grid.h)


def grad_mirror_T(u: np.ndarray, axis: int, h: float) -> np.ndarray:
    """Transpose of one component of grad_mirror."""
    if axis != 1:
        return (np.roll(u, 1, axis) - np.roll(u, -1, axis)) / (2.0 * h)
    r = np.zeros_like(u)
    r[:, 1:-1, :] = u[:, 1:-1, :]
    out = np.zeros_like(u)
    out[:, 1:, :] += r[:, :-1, :]
    out[:, :-1, :] -= r[:, 1:, :]
    return out / (2.0 * h)


def curl_interior_T(b: np.ndarray, h: float, ny: int) -> np.ndarray:
    """Transpose of curl_interior: b has shape (3, nx, ny-2, nz) (values on the interior rows);
    returns (3, nx, ny, nz), wall rows included."""
    nx, _, nz = b.shape[1:]

    def dT(f, axis):
        out = np.zeros((nx, ny, nz))
        if axis == 1:
            out[:, 2:, :] += f / (2.0 * h)
            out[:, :-2, :] -= f / (2.0 * h)
        else:
            out[:, 1:-1, :] = (np.roll(f, 1, axis) - np.roll(f, -1, axis)) / (2.0 * h)
        return out

    bx, by, bz = b
    # v_x = D_y psi_z - D_z psi_y, v_y = D_z psi_x - D_x psi_z, v_z = D_x psi_y - D_y psi_x
    return np.stack([dT(by, 2) - dT(bz, 1),
                     dT(bz, 0) - dT(bx, 2),
                     dT(bx, 1) - dT(by, 0)])


def poisson_adjoint(ubar_int: np.ndarray, grid: Grid):
    """Adjoint of u_int = poisson_solve(b_int, u_lo, u_hi): returns (b_bar, lo_bar, hi_bar)."""
    z = np.zeros((grid.nx, grid.nz))
    bbar = poisson_solve(ubar_int, z, z, grid)
    h2 = grid.h * grid.h
    return bbar, -bbar[:, 0, :] / h2, -bbar[:, -1, :] / h2


def area_gradient(phi: np.ndarray, grid: Grid, eps: float) -> np.ndarray:
    """dA/dphi of vsref.area (SM eq. (32), trapezoid weights)."""
    w = grid.weights()
    h = grid.h
    d = grad_mirror(phi, h)
    s = sum(grad_mirror_T(w * d[c], c, h) for c in range(3))
    return 3.0 / (2.0 * math.sqrt(2.0)) * h**3 * (eps * s + w * (phi * phi - 1.0) * phi / eps)


def grad_step(s: State, a: np.ndarray, dt: float, grid: Grid, walls: Walls, params: Params):
    """One reverse step at level n: returns (dL/dphi^n, dL/dkappa term, dL/ds term)."""
    h = grid.h
    w = grid.weights()
    Mob = params.mobility
    phi, mu, psi, omega = s.phi, s.mu, s.psi, s.omega
    v = velocity(psi, grid, walls)
    Dphi = grad_mirror(phi, h)

    # phi^{n+1} = phi + dt [ M (L_h mu + lambda_V) - v . D phi ]
    phibar = np.array(a, dtype=np.float64, copy=True)
    for c in range(3):
        phibar -= dt * grad_mirror_T(a * v[c], c, h)
    # v through psi on the interior rows, through the wall speed on the walls
    b = np.stack([-dt * a[:, 1:-1, :] * Dphi[c][:, 1:-1, :] for c in range(3)])
    psibar = curl_interior_T(b, h, grid.ny)
    vz_wall = wall_profiles(grid, walls)[0]
    sbar = 0.0
    for j in (0, grid.ny - 1):
        sbar += -dt * vz_wall[j] * float(np.sum(a[:, j, :] * Dphi[2][:, j, :]))
    mubar = dt * Mob * lap_mirror_T(a, grid)
    lambar = dt * Mob * float(np.sum(a))
    # lambda_V = 2 rate_V (V0 - V) / (M |Omega|), V = (|Omega| + h^3 sum_w phi) / 2
    phibar += lambar * (-params.rate_V * h**3 * w / (Mob * grid.domain_volume))

    # psi_int = P(-omega_int; psi walls), omega_int = P(S; omega walls)
    ombar_int = np.zeros((3, grid.nx, grid.ny - 2, grid.nz))
    for c in range(3):
        fbar, lo, hi = poisson_adjoint(psibar[c][:, 1:-1, :], grid)
        ombar_int[c] = -fbar
        sbar += float(np.sum((psibar[c][:, 0, :] + lo) * psi[c][:, 0, :]))
        sbar += float(np.sum((psibar[c][:, -1, :] + hi) * psi[c][:, -1, :]))
    Sbar = np.zeros_like(ombar_int)
    for c in range(3):
        fbar, lo, hi = poisson_adjoint(ombar_int[c], grid)
        Sbar[c] = fbar
        sbar += float(np.sum(lo * omega[c][:, 0, :])) + float(np.sum(hi * omega[c][:, -1, :]))

    # S = (1/eta) D phi x D mu on the interior rows
    A_ = np.stack([d[:, 1:-1, :] for d in Dphi])
    B_ = np.stack([d[:, 1:-1, :] for d in grad_mirror(mu, h)])
    abar = np.cross(B_, Sbar, axis=0) / params.eta      # d/d(D phi)
    bbar = np.cross(Sbar, A_, axis=0) / params.eta      # d/d(D mu)
    for c in range(3):
        fa = np.zeros(grid.shape)
        fb = np.zeros(grid.shape)
        fa[:, 1:-1, :] = abar[c]
        fb[:, 1:-1, :] = bbar[c]
        phibar += grad_mirror_T(fa, c, h)
        mubar += grad_mirror_T(fb, c, h)

    # mu(phi) (SM eq. (35) or F_CH)
    lphi = lap_mirror(phi, h)
    kbar = 0.0
    if params.model == BENDING:
        eps2 = params.eps**2
        Cb = params.C_b
        g = phi**3 - phi - eps2 * lphi
        gbar = Cb * ((3.0 * phi**2 - 1.0) * mubar - eps2 * lap_mirror_T(mubar, grid))
        phibar += (6.0 * Cb * phi * g * mubar - s.gamma_A * lap_mirror_T(mubar, grid)
                   + (3.0 * phi**2 - 1.0) * gbar - eps2 * lap_mirror_T(gbar, grid))
        if params.kappa != 0.0:
            dmu_dk = (Cb / params.kappa) * ((3.0 * phi**2 - 1.0) * g - eps2 * lap_mirror(g, h))
            kbar = float(np.sum(mubar * dmu_dk))
        gambar = -float(np.sum(mubar * lphi))
        if params.k_A != 0.0 and s.A0 > 0.0:
            phibar += gambar * params.k_A / s.A0 * area_gradient(phi, grid, params.eps)
    else:
        phibar += (3.0 * phi**2 - 1.0) * mubar - params.sigma * lap_mirror_T(mubar, grid)
    return phibar, kbar, sbar


def scaled_walls(walls: Walls, s: float) -> Walls:
    return replace(walls, u0=s * walls.u0, u1=s * walls.u1)


def rollout_gradient(grid: Grid, walls: Walls, params: Params, phi0: np.ndarray, dt: float,
                     nsteps: int, phi_target: np.ndarray, checkpoint_every: int = 0):
    """L = ||phi^N - phi_target||^2 (sum over nodes) and (dL/dkappa, dL/ds, dL/dphi^0 with
    V0, A0 fixed). With checkpoint_every > 0 only every checkpoint_every-th state is kept and
    the others are recomputed forward from the nearest checkpoint during the reverse sweep."""
    s0 = init_state(grid, walls, params, phi0)
    keep = {0: s0}
    s = s0
    for n in range(nsteps):
        s = step(s, dt, grid, walls, params)
        if checkpoint_every <= 0 or (n + 1) % checkpoint_every == 0:
            keep[n + 1] = s
    r = s.phi - phi_target
    L = float(np.sum(r * r))
    a = 2.0 * r
    kb = sb = 0.0
    for n in range(nsteps - 1, -1, -1):
        if n in keep:
            sn = keep[n]
        else:
            base = max(k for k in keep if k < n)
            sn = keep[base]
            for _ in range(n - base):
                sn = step(sn, dt, grid, walls, params)
        a, dk, ds = grad_step(sn, a, dt, grid, walls, params)
        kb += dk
        sb += ds
    return L, kb, sb, a
