"""Pins of the oracle diagnostics (oracle/diagnostics.py): closed-form shear stresses of
channel and shear flows, exact observables of shifted fields, the Cahn-Hilliard surface
tension of a planar interface (SM eq. (15)), and the re-solved flow after a wall change."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import diagnostics as D


def _grid():
    return O.Grid(8, 21, 10, h=0.5)


def test_shear_stress_of_poiseuille_flow():
    g = _grid()
    U, eta = 0.07, 1.3
    walls = O.Walls(O.POISEUILLE, U)
    _, psi = O.no_body_fields(g, walls)
    st = D.shear_stress(psi, g, walls, eta)
    y = g.y()
    exact = eta * np.abs(4.0 * U * (g.H - 2.0 * y) / g.H**2)
    # rows 2..ny-3: every difference sees interior velocities (the cubic psi makes the discrete
    # v_z a constant offset of the exact one, which the y difference removes)
    assert np.allclose(st[:, 2:-2, :], exact[None, 2:-2, None], rtol=1e-12, atol=1e-15)
    assert np.all(st[:, 0, :] == 0.0) and np.all(st[:, -1, :] == 0.0)


def test_shear_stress_of_couette_flow():
    g = _grid()
    walls = O.Walls(O.COUETTE, -0.03, 0.05)
    _, psi = O.no_body_fields(g, walls)
    st = D.shear_stress(psi, g, walls, 0.8)
    assert np.allclose(st[:, 1:-1, :], 0.8 * 0.08 / g.H, rtol=1e-12)


def test_shear_stress_of_a_transverse_shear():
    """psi_z = -a y^2 / 2 gives v = (-a y, 0, 0) inside, so sigma_xy = -eta a."""
    g = _grid()
    a, eta = 0.3, 1.7
    psi = np.zeros((3,) + g.shape)
    psi[2] = -0.5 * a * (g.y() ** 2)[None, :, None]
    walls = O.Walls(O.COUETTE, 0.0, 0.0)
    st = D.shear_stress(psi, g, walls, eta)
    assert np.allclose(st[:, 2:-2, :], eta * a, rtol=1e-12)


def test_observables_of_shifted_fields():
    g = _grid()
    walls = O.Walls(O.POISEUILLE, 0.05)
    om0, ps0 = O.no_body_fields(g, walls)
    assert D.observables(om0, ps0, g, walls) == (0.0, 0.0)
    om = om0.copy()
    om[1] += 0.2
    ps = ps0.copy()
    ps[2] -= 0.1
    ps[0] += 0.3
    oo, op = D.observables(om, ps, g, walls)
    assert oo == pytest.approx(0.04 * g.domain_volume, rel=1e-13)
    assert op == pytest.approx(0.1 * g.domain_volume, rel=1e-13)


def test_cahn_hilliard_energy_of_a_planar_interface_pair():
    """Two flat interfaces normal to x: F_CH = 2 gamma (area), gamma = 2 sqrt(2 sigma)/3."""
    sigma = 1.0
    g = O.Grid(160, 5, 4, h=0.25)
    x = np.arange(g.nx) * g.h
    L = g.nx * g.h
    prof = np.tanh((L / 4.0 - np.abs(x - L / 2.0)) / math.sqrt(2.0 * sigma))
    phi = np.broadcast_to(prof[:, None, None], g.shape).copy()
    F = D.ch_energy(phi, g, sigma)
    area = g.H * g.nz * g.h
    gamma = 2.0 * math.sqrt(2.0 * sigma) / 3.0
    assert F == pytest.approx(2.0 * gamma * area, rel=5e-3)


def test_set_walls_re_solves_the_flow_and_shifts_by_the_no_body_difference():
    g = O.Grid(12, 11, 10)
    p = O.Params(kappa=1.0)
    from workloads.shapes import GridSpec, phi_sphere
    phi0 = phi_sphere(GridSpec(12, 11, 10), 3.0, math.sqrt(2.0))
    w1 = O.Walls(O.POISEUILLE, 0.05)
    w2 = O.Walls(O.POISEUILLE, -0.02)
    s1 = O.init_state(g, w1, p, phi0)
    s2 = D.set_walls(s1, g, w2, p)
    om2, ps2 = O.no_body_fields(g, w2)
    om1, ps1 = O.no_body_fields(g, w1)
    # walls now hold the new tables, and the interior solves the Poisson problems
    assert np.allclose(s2.psi[:, :, [0, -1], :], ps2[:, :, [0, -1], :], atol=1e-15)
    res = O.lap_interior(s2.psi[0], g.h) + s2.omega[0][:, 1:-1, :]
    assert np.max(np.abs(res)) < 1e-12
    # the Poisson problems are linear in the wall data and the no-body fields solve them
    # exactly, so the change is the difference of the no-body fields
    assert np.allclose(s2.omega - s1.omega, om2 - om1, atol=1e-13)
    assert np.allclose(s2.psi - s1.psi, ps2 - ps1, atol=1e-13)


def test_gauge_defect_closed_forms():
    g = O.Grid(12, 9, 10, h=0.7)
    walls = O.Walls(O.POISEUILLE, 0.05)
    _, ps0 = O.no_body_fields(g, walls)
    assert D.gauge_defect(ps0, g) == 0.0
    psi = np.zeros((3,) + g.shape)
    i = np.arange(g.nx)
    psi[0] = np.sin(2.0 * math.pi * i / g.nx)[:, None, None]
    M = g.ny - 2
    exact = g.h * g.nz * M * (g.nx / 2.0) * math.sin(2.0 * math.pi / g.nx) ** 2
    assert D.gauge_defect(psi, g) == pytest.approx(exact, rel=1e-12)


def test_max_speed_of_channel_flows():
    g = O.Grid(6, 21, 8, h=0.5)          # ny odd: a node on the centreline
    U = 0.07
    walls = O.Walls(O.POISEUILLE, U)
    _, psi = O.no_body_fields(g, walls)
    # the central difference of the cubic psi_x offsets v_z by -4 U h^2 / (3 H^2)
    assert D.max_speed(psi, g, walls) == pytest.approx(U * (1.0 - 4.0 * g.h**2 / (3.0 * g.H**2)), rel=1e-12)
    walls = O.Walls(O.COUETTE, -0.03, 0.05)
    _, psi = O.no_body_fields(g, walls)
    assert D.max_speed(psi, g, walls) == pytest.approx(0.05, rel=1e-12)
