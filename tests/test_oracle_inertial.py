"""Pins of the oracle's inertial variant (SM "Time-dependency and inertial flow", eq. (36)):
the implicit vorticity problem (L_h - a) omega^{n+1} = S - a omega^n, a = rho/(eta dt).

The shifted solve is checked against a dense matrix assembled node by node; the time
discretisation against the closed-form decay of one eigenmode of L_h in a no-body channel
(S = 0): omega^{n+1} - omega_0 = a/(a - lambda) (omega^n - omega_0); and the two limits
rho -> 0 (eq. (5b)) and rho -> infinity (omega frozen).
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import brute

RNG = np.random.default_rng(36)


def test_shifted_poisson_matches_dense_assembly():
    g = O.Grid(4, 6, 5, h=0.8)
    b = RNG.standard_normal(g.shape)
    ulo = RNG.standard_normal((g.nx, g.nz))
    uhi = RNG.standard_normal((g.nx, g.nz))
    for shift in (0.0, 0.37, 25.0):
        u = O.poisson_solve(b[:, 1:-1, :], ulo, uhi, g, shift)
        ref = brute.poisson_dense(b, ulo, uhi, g.h, shift)
        assert np.allclose(u, ref[:, 1:-1, :], rtol=1e-12, atol=1e-12), shift


def _mode(g, p, m, q):
    i, j, k = np.meshgrid(np.arange(g.nx), np.arange(g.ny), np.arange(g.nz), indexing="ij")
    u = (np.cos(2 * np.pi * p * i / g.nx + 0.2) * np.sin(np.pi * m * j / (g.ny - 1))
         * np.cos(2 * np.pi * q * k / g.nz - 0.4))
    lam = ((2 * math.cos(2 * math.pi * p / g.nx) - 2) + (2 * math.cos(math.pi * m / (g.ny - 1)) - 2)
           + (2 * math.cos(2 * math.pi * q / g.nz) - 2)) / g.h**2
    return u, lam


@pytest.mark.parametrize("model", [O.BENDING, O.CAHN_HILLIARD])
def test_single_mode_decays_by_the_backward_euler_factor(model):
    """No body (phi = -1 everywhere, so mu = 0, S = 0 and phi stays): the vorticity relaxes
    to the no-body profile mode by mode with factor a/(a - lambda); psi follows eq. (5c)."""
    g = O.Grid(8, 9, 10, h=0.9)
    walls = O.Walls(O.POISEUILLE, 0.05)
    rho, eta, dt = 2.0, 1.3, 0.01
    p = O.Params(model=model, eta=eta, rho=rho)
    s = O.init_state(g, walls, p, -np.ones(g.shape))
    om0, ps0 = O.no_body_fields(g, walls)
    assert np.allclose(s.omega, om0, atol=1e-14)
    pert = np.zeros((3,) + g.shape)
    lams = []
    for c, (pp, m, q) in enumerate([(1, 1, 2), (2, 3, 0), (0, 5, 1)]):
        u, lam = _mode(g, pp, m, q)
        pert[c] = (0.01 * (c + 1)) * u
        lams.append(lam)
    s.omega = om0 + pert
    s2 = O.step(s, dt, g, walls, p)
    a = rho / (eta * dt)
    assert np.array_equal(s2.phi, s.phi)
    for c in range(3):
        expect = om0[c] + a / (a - lams[c]) * pert[c]
        assert np.allclose(s2.omega[c], expect, rtol=1e-12, atol=1e-14), c
    res = O.lap_interior(s2.psi[0], g.h) + s2.omega[0][:, 1:-1, :]
    assert np.max(np.abs(res)) < 1e-12


def test_zero_density_is_the_poisson_step_and_large_density_freezes_omega():
    g = O.Grid(12, 11, 10)
    walls = O.Walls(O.COUETTE, -0.03, 0.05)
    from workloads.shapes import GridSpec, phi_sphere
    phi0 = phi_sphere(GridSpec(12, 11, 10), 3.0, math.sqrt(2.0))
    base = O.Params(model=O.CAHN_HILLIARD, sigma=1.0)
    dt = 1e-3
    s0 = O.init_state(g, walls, base, phi0)
    ref = O.step(s0, dt, g, walls, base)
    tiny = O.step(s0, dt, g, walls, O.Params(model=O.CAHN_HILLIARD, sigma=1.0, rho=1e-13))
    assert np.allclose(tiny.omega, ref.omega, rtol=1e-8, atol=1e-12)
    assert np.array_equal(tiny.phi, ref.phi)
    big = O.step(s0, dt, g, walls, O.Params(model=O.CAHN_HILLIARD, sigma=1.0, rho=1e9))
    # (L_h - a) w = S - a omega^n: w = omega^n + O(1/a)
    assert np.max(np.abs(big.omega - s0.omega)) < 1e-7 * max(1.0, np.max(np.abs(s0.omega)))
    assert np.max(np.abs(ref.omega - s0.omega)) > 1e-6   # the Poisson step does move omega
