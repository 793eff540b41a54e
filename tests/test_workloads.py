"""Checks of the seeded input generators (they carry none of the method's arithmetic)."""
import math

import numpy as np
import pytest

from workloads import WORKLOADS, alm_coefficients, prolate_area, prolate_axes, real_sph_harm, workload


def test_prolate_axes_area_and_reduced_volume():
    """Area-equivalent radius 24 and reduced volume 0.8 (SM eq. (40)) give a ~ 44.17, b ~ 15.82."""
    a, b = prolate_axes(24.0, 0.8)
    A = prolate_area(a, b)
    V = 4.0 / 3.0 * math.pi * a * b * b
    assert A == pytest.approx(4 * math.pi * 24.0**2, rel=1e-12)
    assert V / (4.0 / 3.0 * math.pi * (A / (4 * math.pi)) ** 1.5) == pytest.approx(0.8, rel=1e-12)
    assert a == pytest.approx(44.169, abs=2e-3) and b == pytest.approx(15.823, abs=2e-3)


def test_prolate_area_sphere_limit():
    assert prolate_area(3.0, 3.0) == pytest.approx(4 * math.pi * 9.0)
    assert prolate_area(3.0 * (1 + 1e-7), 3.0) == pytest.approx(4 * math.pi * 9.0, rel=1e-6)


def test_real_sph_harm_orthonormal():
    """Gauss-Legendre x uniform quadrature of Y_lm Y_l'm' over the sphere is the identity."""
    xg, wg = np.polynomial.legendre.leggauss(24)
    theta = np.arccos(xg)
    ph = np.linspace(0, 2 * np.pi, 48, endpoint=False)
    T, P = np.meshgrid(theta, ph, indexing="ij")
    W = wg[:, None] * (2 * np.pi / 48)
    Y = [real_sph_harm(l, m, T, P) for l in range(4) for m in range(-l, l + 1)]
    G = np.array([[np.sum(W * a * b) for b in Y] for a in Y])
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_alm_seeded_and_sized():
    a = alm_coefficients(0)
    assert a.shape == (16,)
    assert np.array_equal(a, np.random.default_rng(0).normal(0, 0.02, 16))


@pytest.mark.parametrize("name", ["vesicle32"])
def test_phi0_range_and_inside_positive(name):
    w = workload(name)
    phi = w.phi0()
    assert phi.shape == w.grid.shape
    assert phi.max() <= 1 and phi.min() >= -1
    nx, ny, nz = w.grid.shape
    assert phi[nx // 2, (ny - 1) // 2, nz // 2] > 0.99
    assert phi[0, 0, 0] < -0.99


def test_workload_table():
    assert set(WORKLOADS) >= {"vesicle32", "vesicle128", "droplet256"}
    assert WORKLOADS["vesicle128"].grid.shape == (128, 128, 128)
