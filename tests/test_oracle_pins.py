"""Pins of the CPU oracle against mathematics the paper and the discretisation fix.

Each test names the part it pins and what would break it. Grids are tiny or small so the
whole file runs in seconds on the CPU.
"""
import math
from dataclasses import replace

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

import oracle as O
from tests import brute

RNG = np.random.default_rng(1234)


def _eig1(n, p, h, periodic=True):
    if periodic:
        return (2 * math.cos(2 * math.pi * p / n) - 2) / h**2
    return (2 * math.cos(math.pi * p / (n - 1)) - 2) / h**2


# --------------------------------------------------------------------------- operators (P1)
def test_lap_mirror_eigenfunction():
    """cos modes (periodic x, z) times cos(pi m j/(ny-1)) (even about both walls) are exact
    eigenfunctions of the mirror-ghost 7-point Laplacian. Pins the ghost rule, the roll
    directions and the 1/h^2 scale."""
    g = O.Grid(8, 7, 6, h=0.7)
    i, j, k = np.meshgrid(np.arange(8), np.arange(7), np.arange(6), indexing="ij")
    for (p, m, q) in [(1, 1, 1), (2, 3, 0), (3, 5, 2), (0, 6, 3)]:
        u = (np.cos(2 * np.pi * p * i / 8 + 0.3) * np.cos(np.pi * m * j / 6)
             * np.sin(2 * np.pi * q * k / 6 + 0.1))
        lam = _eig1(8, p, g.h) + _eig1(7, m, g.h, periodic=False) + _eig1(6, q, g.h)
        assert np.allclose(O.lap_mirror(u, g.h), lam * u, atol=1e-12)


def test_lap_mirror_weighted_sum_zero():
    """sum_w L_h u = 0 for any u with mirror ghosts and trapezoid weights (no-flux walls)."""
    g = O.Grid(5, 6, 4)
    u = RNG.standard_normal(g.shape)
    assert abs(np.sum(g.weights() * O.lap_mirror(u, g.h))) < 1e-12


def test_operators_match_node_loops():
    g = O.Grid(5, 6, 4, h=0.9)
    u = RNG.standard_normal(g.shape)
    assert np.allclose(O.lap_mirror(u, g.h), brute.lap_m(u, g.h), atol=1e-12)
    assert np.allclose(np.stack(O.grad_mirror(u, g.h)), brute.grad_m(u, g.h), atol=1e-12)


def test_central_difference_closed_form():
    """D_x sin(2 pi p i/n) = sin(2 pi p/n)/h cos(2 pi p i/n); D_y of the even wall mode is
    -sin(pi m/(ny-1))/h sin(pi m j/(ny-1)), zero on the walls."""
    g = O.Grid(8, 9, 6, h=0.5)
    i, j, k = np.meshgrid(np.arange(8), np.arange(9), np.arange(6), indexing="ij")
    u = np.sin(2 * np.pi * 3 * i / 8) * np.cos(np.pi * 2 * j / 8) * np.cos(2 * np.pi * k / 6)
    dx, dy, dz = O.grad_mirror(u, g.h)
    ex = (math.sin(2 * math.pi * 3 / 8) / g.h * np.cos(2 * np.pi * 3 * i / 8)
          * np.cos(np.pi * 2 * j / 8) * np.cos(2 * np.pi * k / 6))
    ey = (-math.sin(math.pi * 2 / 8) / g.h * np.sin(2 * np.pi * 3 * i / 8)
          * np.sin(np.pi * 2 * j / 8) * np.cos(2 * np.pi * k / 6))
    ez = (-math.sin(2 * math.pi / 6) / g.h * np.sin(2 * np.pi * 3 * i / 8)
          * np.cos(np.pi * 2 * j / 8) * np.sin(2 * np.pi * k / 6))
    assert np.allclose(dx, ex, atol=1e-12)
    assert np.allclose(dy, ey, atol=1e-12)
    assert np.allclose(dz, ez, atol=1e-12)
    assert np.all(dy[:, 0, :] == 0) and np.all(dy[:, -1, :] == 0)


def test_vorticity_source_closed_form():
    """S = (1/eta) grad phi x grad mu (main text eq. (5b)) on the interior rows, by central
    differences: phi varying along x only and mu along z only give S = (0, -phi_x mu_z, 0)/eta;
    phi along y (an even wall mode) and mu along x give S = (0, 0, -phi_y mu_x)/eta. Swapping
    the factors of the cross product flips both signs; dropping 1/eta scales them."""
    eta = 1.7
    g = O.Grid(8, 9, 6, h=0.5)
    i, j, k = np.meshgrid(np.arange(8), np.arange(9), np.arange(6), indexing="ij")
    cx, cz, cy = 2 * math.pi * 3 / 8, 2 * math.pi * 1 / 6, math.pi * 2 / 8
    phi = np.sin(cx * i) + 0.0 * j
    mu = np.sin(cz * k) + 0.0 * j
    S = O.vorticity_source(phi, mu, g, eta)
    fx = math.sin(cx) / g.h * np.cos(cx * i)
    mz = math.sin(cz) / g.h * np.cos(cz * k)
    assert S.shape == (3, 8, 7, 6)
    assert np.allclose(S[0], 0.0, atol=1e-13) and np.allclose(S[2], 0.0, atol=1e-13)
    assert np.allclose(S[1], (-fx * mz / eta)[:, 1:-1, :], atol=1e-12)
    phi = np.cos(cy * j) + 0.0 * i
    mu = np.sin(cx * i) + 0.0 * k
    S = O.vorticity_source(phi, mu, g, eta)
    fy = -math.sin(cy) / g.h * np.sin(cy * j)
    mx = math.sin(cx) / g.h * np.cos(cx * i)
    assert np.allclose(S[0], 0.0, atol=1e-13) and np.allclose(S[1], 0.0, atol=1e-13)
    assert np.allclose(S[2], (-fy * mx / eta)[:, 1:-1, :], atol=1e-12)


def test_curl_closed_form_and_divergence_free():
    """curl (0, 0, sin(2 pi i/nx)) = (0, -sin(2 pi/nx)/h cos(2 pi i/nx), 0); and the discrete
    divergence of a central-difference curl vanishes (central differences commute)."""
    g = O.Grid(8, 7, 6, h=1.0)
    i = np.arange(8)[:, None, None] * np.ones(g.shape)
    psi = np.zeros((3,) + g.shape)
    psi[2] = np.sin(2 * np.pi * i / 8)
    v = O.curl_interior(psi, g.h)
    assert np.allclose(v[0], 0) and np.allclose(v[2], 0)
    assert np.allclose(v[1], -math.sin(2 * math.pi / 8) * np.cos(2 * np.pi * i[:, 1:-1, :] / 8))
    psi = RNG.standard_normal((3,) + g.shape)
    v = O.curl_interior(psi, g.h)  # rows 1..ny-2
    # divergence at rows 2..ny-3 uses only rows 1..ny-2 of v
    div = ((np.roll(v[0], -1, 0) - np.roll(v[0], 1, 0))[:, 1:-1, :]
           + (v[1][:, 2:, :] - v[1][:, :-2, :])
           + (np.roll(v[2], -1, 2) - np.roll(v[2], 1, 2))[:, 1:-1, :])
    assert np.max(np.abs(div)) < 1e-12


# --------------------------------------------------------------------------- Poisson (P2)
def test_poisson_discrete_eigenfunction():
    """u = sin(pi m j/(ny-1)) e^{...} with zero walls solves L_h u = lambda u exactly."""
    g = O.Grid(8, 10, 6, h=0.8)
    i, j, k = np.meshgrid(np.arange(8), np.arange(10), np.arange(6), indexing="ij")
    u = np.sin(np.pi * 4 * j / 9) * np.cos(2 * np.pi * 3 * i / 8) * np.sin(2 * np.pi * 2 * k / 6 + 0.4)
    lam = _eig1(8, 3, g.h) + (2 * math.cos(math.pi * 4 / 9) - 2) / g.h**2 + _eig1(6, 2, g.h)
    z = np.zeros((8, 6))
    sol = O.poisson_solve(lam * u[:, 1:-1, :], z, z, g)
    assert np.max(np.abs(sol - u[:, 1:-1, :])) < 1e-13


@pytest.mark.parametrize("shape", [(4, 5, 4), (8, 9, 8), (6, 4, 9)])
def test_poisson_matches_sparse_direct(shape):
    """Against scipy's sparse LU of the matrix assembled from an explicit COO list."""
    g = O.Grid(*shape, h=1.3)
    nx, ny, nz = shape
    M = ny - 2
    b = RNG.standard_normal((nx, M, nz))
    lo = RNG.standard_normal((nx, nz))
    hi = RNG.standard_normal((nx, nz))
    rows, cols, vals = [], [], []
    rhs = b.reshape(-1).copy()

    def idx(i, j, k):
        return (i * M + j) * nz + k

    for i in range(nx):
        for j in range(M):
            for k in range(nz):
                r = idx(i, j, k)
                rows.append(r); cols.append(r); vals.append(-6.0 / g.h**2)
                for ii, kk in (((i + 1) % nx, k), ((i - 1) % nx, k), (i, (k + 1) % nz), (i, (k - 1) % nz)):
                    rows.append(r); cols.append(idx(ii, j, kk)); vals.append(1.0 / g.h**2)
                for jj in (j - 1, j + 1):
                    if jj < 0:
                        rhs[r] -= lo[i, k] / g.h**2
                    elif jj >= M:
                        rhs[r] -= hi[i, k] / g.h**2
                    else:
                        rows.append(r); cols.append(idx(i, jj, k)); vals.append(1.0 / g.h**2)
    A = scipy.sparse.coo_matrix((vals, (rows, cols)), shape=(rhs.size, rhs.size)).tocsc()
    ref = scipy.sparse.linalg.spsolve(A, rhs).reshape(nx, M, nz)
    sol = O.poisson_solve(b, lo, hi, g)
    assert np.max(np.abs(sol - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_poisson_dense_loops_agree():
    g = O.Grid(4, 5, 4)
    b = RNG.standard_normal(g.shape)
    lo = RNG.standard_normal((4, 4))
    hi = RNG.standard_normal((4, 4))
    ref = brute.poisson_dense(b, lo, hi, g.h)
    sol = O.poisson_solve(b[:, 1:-1, :], lo, hi, g)
    assert np.allclose(sol, ref[:, 1:-1, :], atol=1e-12)


def test_poisson_manufactured_second_order():
    """u = sin(2 pi x) cos(2 pi z) exp(y) on the unit box, walls from u, f = lap u (continuum):
    the discrete error falls by ~4 per halving of h (second order)."""
    errs = []
    for n in (8, 16, 32):
        h = 1.0 / n
        g = O.Grid(n, n + 1, n, h=h)
        x = np.arange(n) * h
        y = np.arange(n + 1) * h
        X, Y, Z = np.meshgrid(x, y, x, indexing="ij")
        u = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Z) * np.exp(Y)
        f = (1.0 - 8 * np.pi**2) * u
        sol = O.poisson_solve(f[:, 1:-1, :], u[:, 0, :], u[:, -1, :], g)
        errs.append(np.max(np.abs(sol - u[:, 1:-1, :])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.9 < r2 < 4.1, errs


# ----------------------------------------------------------------------- channel flow (P3, P4)
def _no_body(kind, u0, u1, shape=(8, 32, 8)):
    g = O.Grid(*shape)
    walls = O.Walls(kind, u0, u1)
    p = O.Params(kappa=1.0)
    phi = -np.ones(g.shape)
    s = O.init_state(g, walls, p, phi)
    return g, walls, s


def test_poiseuille_no_body_exact():
    """phi = -1: mu = 0, so omega_x is the linear wall profile and psi_x the cubic one, both
    exact discrete solutions (L_h is exact on cubics). The discrete centreline-type velocity
    is v_z = 4U y(H-y)/H^2 - (4/3) U h^2/H^2 in the interior (central difference of a cubic)."""
    U = 0.05
    g, walls, s = _no_body("poiseuille", U, 0.0)
    H = g.H
    y = g.y()
    assert np.max(np.abs(s.mu)) == 0.0
    om_ref = 4 * U / H**2 * (H - 2 * y)
    ps_ref = -(4 * U / H**2) * (H * y**2 / 2 - y**3 / 3)
    assert np.max(np.abs(s.omega[0] - om_ref[None, :, None])) < 1e-15
    assert np.max(np.abs(s.psi[0] - ps_ref[None, :, None])) < 1e-13
    assert np.max(np.abs(s.omega[1:])) == 0 and np.max(np.abs(s.psi[1:])) == 0
    v = O.velocity(s.psi, g, walls)
    vz_ref = 4 * U * y * (H - y) / H**2
    off = v[2, :, 1:-1, :] - vz_ref[None, 1:-1, None]
    assert np.allclose(off, -(4.0 / 3.0) * U * g.h**2 / H**2, atol=1e-14)
    assert v[2, 0, 0, 0] == 0 and v[2, 0, -1, 0] == 0
    # paper-scale check on the 32-node channel: offset 6.937e-5
    assert abs((4.0 / 3.0) * U / 31**2 - 6.9372e-5) < 1e-8


def test_couette_no_body_exact():
    u0, u1 = -0.05, 0.05
    g, walls, s = _no_body("couette", u0, u1)
    H = g.H
    y = g.y()
    ps_ref = -(u0 * y + (u1 - u0) * y**2 / (2 * H))
    assert np.max(np.abs(s.omega[0] - (u1 - u0) / H)) < 1e-15
    assert np.max(np.abs(s.psi[0] - ps_ref[None, :, None])) < 1e-13
    v = O.velocity(s.psi, g, walls)
    vz_ref = u0 + (u1 - u0) * y / H
    assert np.allclose(v[2], vz_ref[None, :, None], atol=1e-14)
    assert np.allclose(v[:2], 0.0, atol=1e-15)


def test_wall_profiles_are_curl_consistent():
    """omega_x = d v_z/dy and psi_x'' = -omega_x for both flows (continuum identities)."""
    g = O.Grid(4, 41, 4, h=0.25)
    for walls in (O.Walls("poiseuille", 0.3), O.Walls("couette", 0.2, -0.1)):
        vz, psx, omx = O.wall_profiles(g, walls)
        y = g.y()
        # exact polynomials: derivatives by finite differences of degree <= 3 are exact
        # up to the h^2/6 f''' term; use a 5-point derivative for the check
        dvz = np.gradient(vz, g.h, edge_order=2)
        assert np.allclose(dvz, omx, atol=1e-12)
        d2 = (psx[2:] - 2 * psx[1:-1] + psx[:-2]) / g.h**2
        assert np.allclose(d2, -omx[1:-1], atol=1e-12)
        assert np.allclose(-np.gradient(psx, g.h, edge_order=2), vz, atol=1e-3 * max(1, abs(vz).max()))
        del y


# -------------------------------------------------------------------- chemical potential (P6)
def _tanh_field(shape, seed=3):
    g = O.Grid(*shape, h=1.0)
    r = np.random.default_rng(seed)
    x = np.arange(shape[0])[:, None, None]
    y = np.arange(shape[1])[None, :, None]
    z = np.arange(shape[2])[None, None, :]
    d = np.sqrt((x - 2.5) ** 2 + (y - 3.0) ** 2 + (z - 2.5) ** 2)
    phi = np.tanh((2.2 - d) / math.sqrt(2)) + 0.05 * r.standard_normal(shape)
    return g, phi


@pytest.mark.parametrize("bend_scale", [1.0, 2.0])
def test_bending_mu_is_scaled_energy_gradient(bend_scale):
    """mu_i = (bend_scale/2) dF_h/dphi_i / (h^3 w_i) with F_h = c_F h^3 sum_w g^2 (SM eq. (30)
    discretised, gamma_A = 0). W L_h symmetric makes this exact; checked by central finite
    differences of F_h. bend_scale = 1 is SM eq. (35); 2 is the exact variational derivative."""
    g, phi = _tanh_field((6, 7, 6))
    p = O.Params(kappa=1.3, eps=0.9, bend_scale=bend_scale)
    mu = O.chemical_potential(phi, g, p, 0.0)
    w = g.weights() * np.ones(g.shape)
    hstep = 1e-6
    for idx in [(0, 0, 0), (2, 3, 2), (5, 6, 1), (3, 1, 4), (1, 5, 5)]:
        pp = phi.copy(); pp[idx] += hstep
        pm = phi.copy(); pm[idx] -= hstep
        dF = (O.bending_energy(pp, g, p) - O.bending_energy(pm, g, p)) / (2 * hstep)
        ref = 0.5 * bend_scale * dF / (g.h**3 * w[idx])
        assert abs(mu[idx] - ref) < 1e-7 * max(1.0, abs(ref)), (idx, mu[idx], ref)


def test_gradient_energy_edges_give_minus_laplacian():
    """d/dphi_i of (1/2) h^3 sum_edges w_e (dphi/h)^2 equals -h^3 w_i (L_h phi)_i: the
    surface-tension (-gamma_A lap phi) and Cahn-Hilliard (-sigma lap phi) terms are the
    gradients of a discrete Dirichlet energy, with the sign of a tension."""
    g, phi = _tanh_field((5, 6, 4))
    w = g.weights() * np.ones(g.shape)
    L = O.lap_mirror(phi, g.h)
    hstep = 1e-6
    for idx in [(0, 0, 0), (2, 3, 2), (4, 5, 3), (1, 1, 1)]:
        pp = phi.copy(); pp[idx] += hstep
        pm = phi.copy(); pm[idx] -= hstep
        dE = (brute.energy_grad_edges(pp, g.h) - brute.energy_grad_edges(pm, g.h)) / (2 * hstep)
        assert abs(dE - (-g.h**3 * w[idx] * L[idx])) < 1e-7


def test_surface_tension_and_cahn_hilliard_terms():
    """mu(gamma_A) - mu(0) = -gamma_A L_h phi (SM eq. (35)); CH mu = phi^3 - phi - sigma L_h phi
    is the gradient of h^3 sum_w (phi^2-1)^2/4 + sigma E_grad (SM eq. (31))."""
    g, phi = _tanh_field((5, 6, 4))
    p = O.Params(kappa=1.0)
    d = O.chemical_potential(phi, g, p, 0.7) - O.chemical_potential(phi, g, p, 0.0)
    assert np.allclose(d, -0.7 * O.lap_mirror(phi, g.h), atol=1e-12)
    pc = O.Params(model=O.CAHN_HILLIARD, sigma=0.8)
    mu = O.chemical_potential(phi, g, pc, 0.0)
    w = g.weights() * np.ones(g.shape)

    def F(ph):
        return (g.h**3 * np.sum(g.weights() * (ph**2 - 1) ** 2 / 4)
                + pc.sigma * brute.energy_grad_edges(ph, g.h))

    for idx in [(0, 0, 0), (2, 3, 2), (4, 5, 3)]:
        pp = phi.copy(); pp[idx] += 1e-6
        pm = phi.copy(); pm[idx] -= 1e-6
        ref = (F(pp) - F(pm)) / 2e-6 / (g.h**3 * w[idx])
        assert abs(mu[idx] - ref) < 1e-7


# ------------------------------------------------------------------- stationary interface (P5)
def _planar_slab(h, eps, L=80.0, ny=3):
    """Periodic slab |z - L/2| < L/4 with tanh interfaces; the |.| kinks sit L/4 away from both
    interfaces, where the profile is flat to ~1e-12, so they do not pollute the defect."""
    nz = int(round(L / h))
    g = O.Grid(2, ny, nz, h=h)
    z = np.arange(nz) * h
    prof = np.tanh((L / 4 - np.abs(z - L / 2)) / (math.sqrt(2) * eps))
    return g, np.broadcast_to(prof[None, None, :], g.shape).copy()


def test_planar_tanh_is_stationary_to_second_order():
    """The planar tanh profile has g = mu = 0 in the continuum (SM eq. (9)-(10) with
    sigma = eps^2); the discrete mu and the defect d(phi)/dt = M L_h mu fall ~4x per
    halving of h once h is well below eps."""
    eps = 1.0
    p = O.Params(kappa=1.0, eps=eps)
    mus, rates = [], []
    for h in (0.25, 0.125, 0.0625, 0.03125):
        g, phi = _planar_slab(h, eps)
        mu = O.chemical_potential(phi, g, p, 0.0)
        mus.append(np.max(np.abs(mu)))
        rates.append(np.max(np.abs(p.mobility * O.lap_mirror(mu, h))))
    assert all(a > b for a, b in zip(rates, rates[1:])), rates
    assert 3.85 < mus[-2] / mus[-1] < 4.1, mus
    assert 3.8 < rates[-2] / rates[-1] < 4.15, rates


# ----------------------------------------------------------------------------- area (P7)
def test_area_of_planar_interface_tends_to_one_per_unit_area():
    """SM eq. (32) on tanh(z/(sqrt2 eps)) is exactly 1 per unit interface area in the
    continuum; the discrete value converges to it at second order."""
    eps = 1.0
    vals = []
    for h in (1.0, 0.5, 0.25, 0.125, 0.0625):
        g, phi = _planar_slab(h, eps, ny=5)
        A = O.area(phi, g, eps)
        vals.append(A / (2 * g.nx * g.h * g.H))
    errs = [abs(v - 1.0) for v in vals]
    assert abs(vals[0] - 0.9444) < 1e-4      # h = eps = 1: the lattice-unit discretisation
    assert errs[-1] < 3e-4
    assert 3.4 < errs[0] / errs[1] < 3.6 and 3.95 < errs[-2] / errs[-1] < 4.05, vals


def test_volume_of_uniform_fields():
    g = O.Grid(6, 7, 5, h=0.5)
    assert O.volume(np.ones(g.shape), g) == pytest.approx(g.domain_volume, rel=1e-14)
    assert O.volume(-np.ones(g.shape), g) == pytest.approx(0.0, abs=1e-12)


# ------------------------------------------------------------------- conservation (P8)
def test_phi_integral_budget_each_step():
    """Delta(sum_w phi) = dt (M lambda_V W - sum_w v . D phi) exactly (sum_w L_h mu = 0),
    with the volume penalty on; and with the penalty off and the body far from the walls
    the change is only the advective term."""
    from workloads import workload
    w = workload("vesicle32")
    g = O.Grid(*w.grid.shape)
    walls = O.Walls(w.wall_kind, w.u0, w.u1)
    p = O.Params(kappa=1.0, rate_V=10.0, k_A=1.0)
    s = O.init_state(g, walls, p, w.phi0())
    W = float(np.sum(g.weights() * np.ones(g.shape)))
    for _ in range(3):
        v = O.velocity(s.psi, g, walls)
        dx, dy, dz = O.grad_mirror(s.phi, g.h)
        adv = float(np.sum(g.weights() * (v[0] * dx + v[1] * dy + v[2] * dz)))
        before = float(np.sum(g.weights() * s.phi))
        lam = s.lam_V
        s = O.step(s, w.dt, g, walls, p)
        after = float(np.sum(g.weights() * s.phi))
        pred = w.dt * (p.mobility * lam * W - adv)
        assert abs((after - before) - pred) < 1e-10 * max(1.0, abs(before))


# -------------------------------------------------------------------- dissipation (P9)
def test_bending_energy_decreases_without_flow():
    """Pure model-B relaxation (no flow, no penalties) of the bending energy: F_h never
    increases for dt at half the linear forward-Euler bound."""
    g = O.Grid(16, 16, 16)
    from workloads.shapes import GridSpec, phi_sh_vesicle, alm_coefficients
    phi0 = phi_sh_vesicle(GridSpec(16, 16, 16), 5.0, alm_coefficients(5, sigma=0.08), math.sqrt(2))
    p = O.Params(kappa=1.0)
    dt = 0.5 * 2.0 / (12 * p.C_b * (2 + 12) ** 2)
    s = O.init_state(g, O.Walls("poiseuille", 0.0), p, phi0, flow=False)
    E = [O.bending_energy(s.phi, g, p)]
    for _ in range(20):
        s = O.step(s, dt, g, O.Walls("poiseuille", 0.0), p, flow=False)
        E.append(O.bending_energy(s.phi, g, p))
    dE = np.diff(E)
    assert np.all(dE <= 1e-12 * E[0]), dE
    assert E[-1] < E[0]


# ----------------------------------------------------------------- one step by loops (P12)
@pytest.mark.parametrize("kind,u0,u1", [("poiseuille", 0.3, 0.0), ("couette", -0.2, 0.4)])
def test_step_matches_node_loops(kind, u0, u1):
    """One full oracle step against a node-by-node evaluation with a dense Poisson solver."""
    g = O.Grid(4, 5, 4, h=1.0)
    walls = O.Walls(kind, u0, u1)
    p = O.Params(kappa=0.8, eps=1.1, gamma0=0.3, rate_V=0.0, k_A=0.0)
    r = np.random.default_rng(7)
    phi0 = np.tanh(r.standard_normal(g.shape))
    s0 = O.init_state(g, walls, p, phi0)
    s0.lam_V = 0.01  # exercise the volume term in the update
    dt = 1e-3
    s1 = O.step(s0, dt, g, walls, p)
    ref = brute.step_loops(s0.phi, s0.mu, s0.psi, 0.01, dt, g.h, p.mobility, p.eta, p.eps,
                           p.C_b, 0.3, (kind, u0, u1))
    for a, b in zip((s1.phi, s1.mu, s1.omega, s1.psi), ref):
        assert np.allclose(a, b, atol=1e-11, rtol=1e-11)


# --------------------------------------------------------- penalty multipliers (SM (37)-(38))
# The multipliers are a reading of SM "Lagrange multipliers" (penalty form, lambda_V driving V
# to V0 at rate rate_V; gamma_A = gamma0 + k_A (A - A0)/A0). Two settings where the oracle's
# whole step reduces to a scalar recurrence that is derived here from the discrete operators,
# not from the oracle's code: a wrong sign, a lost factor 2, a missing mobility or domain
# volume, or A in place of A0 in the denominator each changes the recurrence.

def _volume_relaxation_error(mult=None, model=O.BENDING, h=1.0, mobility=1.0, steps=12):
    """No flow, V0 offset by delta from V[phi0]. sum_w L_h mu = 0 (mirror ghosts, trapezoid
    weights) and W h^3 = |Omega| make V^{n+1} = V^n + dt M lambda_V^n |Omega| / 2 exact, so
    under the penalty reading V^n - V0 = (1 - dt rate_V)^n (V^0 - V0). Returns the largest
    relative deviation from that geometric sequence (mult: a replacement multipliers()).
    """
    from workloads.shapes import GridSpec, alm_coefficients, phi_sh_vesicle
    n = 12
    g = O.Grid(n, n + 1, n, h=h)
    spec = GridSpec(n, n + 1, n, h=h)
    phi0 = phi_sh_vesicle(spec, 3.2 * h, alm_coefficients(2, sigma=0.05), math.sqrt(2) * h)
    if model == O.BENDING:
        p = O.Params(kappa=0.3, eps=h, mobility=mobility)
        rate = mobility * 12 / h**2 * p.C_b * (2 + 12) ** 2
    else:
        p = O.Params(model=O.CAHN_HILLIARD, sigma=0.5 * h * h, mobility=mobility)
        rate = mobility * 12 / h**2 * (2 + 12 * p.sigma / h**2)
    dt = 0.25 * 2.0 / rate
    rate_V = 0.15 / dt          # V relaxes by 15% of its offset per step
    p = replace(p, rate_V=rate_V)
    walls = O.Walls(O.POISEUILLE, 0.0)
    orig = O.vsref.multipliers
    if mult is not None:
        O.vsref.multipliers = mult
    try:
        s = O.init_state(g, walls, p, phi0, flow=False)
        delta = 0.01 * s.V0
        V0 = s.V0 + delta
        lam, gam = O.vsref.multipliers(s.V, s.A, V0, s.A0, g, p)
        mu = O.chemical_potential(s.phi, g, p, gam)
        s = replace(s, V0=V0, lam_V=lam, gamma_A=gam, mu=mu)
        worst = 0.0
        e0 = s.V - V0
        for m in range(1, steps + 1):
            s = O.step(s, dt, g, walls, p, flow=False)
            pred = (1.0 - dt * rate_V) ** m * e0
            worst = max(worst, abs((s.V - V0) - pred) / abs(e0))
    finally:
        O.vsref.multipliers = orig
    assert 0.05 < dt * rate_V < 1.0   # a visible relaxation per step, below overshoot
    return worst


@pytest.mark.parametrize("model,h,mob", [(O.BENDING, 1.0, 1.0), (O.BENDING, 1.0, 0.6),
                                         (O.CAHN_HILLIARD, 0.5, 1.7)])
def test_volume_penalty_relaxes_geometrically(model, h, mob):
    assert _volume_relaxation_error(model=model, h=h, mobility=mob) < 1e-10


def _area_mode_error(mult=None, h=1.0, mobility=1.0, steps=15):
    """kappa = 0, gamma0 = 0, no flow: mu = -gamma_A L_h phi. For phi = a cos(2 pi x/(6h))
    (constant in y, z), L_h phi = -lam phi with lam = (2 - 2 cos(pi/3))/h^2, so each step
    maps a -> a (1 - dt M gamma_A lam^2), and mu = gamma_A lam phi. The area of SM (32) for
    this field has a closed form (sums of cos^2, cos^4, sin^2 over a period of 6 nodes):
      A(a) = 3/(2 sqrt 2) h^3 W_yz [ (eps/2) a^2 (sin(pi/3)/h)^2 3 + (6 - 6 a^2 + 9 a^4/4)/(4 eps) ]
    with W_yz = nz (ny - 1) the trapezoid weight of one x-column. A0 is set 20% below
    A(a0), so gamma_A = k_A (A - A0)/A0 > 0 pulls the amplitude (and A) down. The first step
    is the identity (mu^0 = 0 from the initial gamma_A = 0). Returns the largest relative
    deviation of the oracle's amplitude and of its mu from the recurrence.
    """
    nx, ny, nz = 6, 4, 3
    g = O.Grid(nx, ny, nz, h=h)
    eps, k_A, a0 = 1.3 * h, 2.5, 0.9
    x = np.arange(nx)[:, None, None] * np.ones((1, ny, nz))
    mode = np.cos(2 * np.pi * x / nx)
    lam = (2.0 - 2.0 * math.cos(math.pi / 3)) / h**2
    Wyz = nz * (ny - 1)

    def area_closed(a):
        grad = 0.5 * eps * a * a * (math.sin(math.pi / 3) / h) ** 2 * 3.0
        well = (6.0 - 6.0 * a * a + 9.0 * a**4 / 4.0) / (4.0 * eps)
        return 3.0 / (2.0 * math.sqrt(2.0)) * h**3 * Wyz * (grad + well)

    p = O.Params(kappa=0.0, eps=eps, mobility=mobility, gamma0=0.0, k_A=k_A)
    # dt keeps every mode of the x line stable (largest lam^2 = (4/h^2)^2)
    dt = 0.2 / (mobility * 1.0 * (4.0 / h**2) ** 2)
    walls = O.Walls(O.POISEUILLE, 0.0)
    orig = O.vsref.multipliers
    if mult is not None:
        O.vsref.multipliers = mult
    try:
        s = O.init_state(g, walls, p, a0 * mode, flow=False)
        assert abs(s.A - area_closed(a0)) < 1e-12 * s.A
        A0 = 0.8 * area_closed(a0)
        s = replace(s, A0=A0)
        a = a0
        worst = 0.0
        for m in range(steps):
            gam_prev = k_A * (area_closed(a) - A0) / A0 if m > 0 else 0.0
            a = a * (1.0 - dt * mobility * gam_prev * lam * lam)
            s = O.step(s, dt, g, walls, p, flow=False)
            gam = k_A * (area_closed(a) - A0) / A0
            worst = max(worst, float(np.max(np.abs(s.phi - a * mode))) / a0,
                        float(np.max(np.abs(s.mu - gam * lam * a * mode))) / (a0 * lam))
    finally:
        O.vsref.multipliers = orig
    assert gam > 0.05 and a < 0.99 * a0   # the penalty acted
    return worst


@pytest.mark.parametrize("h,mob", [(1.0, 1.0), (0.5, 0.7)])
def test_area_penalty_single_mode_recurrence(h, mob):
    assert _area_mode_error(h=h, mobility=mob) < 1e-12


def _mutants():
    """Plausible mistakes in the multiplier formulas (planted on the CPU, in the oracle)."""
    def base(V, A, V0, A0, grid, params, sv=1.0, fv=2.0, mob=True, vol=True, sa=1.0, den0=True):
        lam = fv * sv * params.rate_V * (V0 - V) / ((params.mobility if mob else 1.0)
                                                    * (grid.domain_volume if vol else 1.0))
        gam = params.gamma0
        if params.k_A != 0.0 and A0 > 0.0:
            gam += sa * params.k_A * (A - A0) / (A0 if den0 else A)
        return lam, gam
    return {
        "lambda sign": lambda *a: base(*a, sv=-1.0),
        "lambda factor 1": lambda *a: base(*a, fv=1.0),
        "lambda factor 4": lambda *a: base(*a, fv=4.0),
        "lambda no mobility": lambda *a: base(*a, mob=False),
        "gamma sign": lambda *a: base(*a, sa=-1.0),
        "gamma factor 2": lambda *a: base(*a, sa=2.0),
        "gamma over A": lambda *a: base(*a, den0=False),
    }


@pytest.mark.parametrize("name", list(_mutants()))
def test_multiplier_pins_catch_planted_mistakes(name):
    """Each planted mistake in the penalty formulas fails at least one of the two pins (the
    volume pin at M = 0.6 for the mobility, the area pin at M = 1, h = 1)."""
    mut = _mutants()[name]
    ev = _volume_relaxation_error(mult=mut, mobility=0.6, steps=6)
    try:
        ea = _area_mode_error(mult=mut, steps=8)
    except AssertionError:
        ea = 1.0   # the penalty did not act as it must
    assert max(ev, ea) > 1e-6, (name, ev, ea)
