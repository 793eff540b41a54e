"""Per-node loop versions of the discrete operators and one time step, for tiny grids.

Written node by node from the definitions (7-point Laplacian, central differences, mirror
ghosts at the walls, Dirichlet walls for the Poisson problems assembled as an explicit
matrix) so that a vectorisation slip in the oracle (a rolled axis, a wrong ghost, a
transposed component) shows up as a mismatch. Tiny grids only: pure Python loops.
"""
import numpy as np


def _yg(j, ny):
    """Mirror ghost index in y."""
    if j < 0:
        return -j
    if j > ny - 1:
        return 2 * (ny - 1) - j
    return j


def lap_m(u, h):
    nx, ny, nz = u.shape
    out = np.zeros_like(u)
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                s = (u[(i + 1) % nx, j, k] + u[(i - 1) % nx, j, k]
                     + u[i, _yg(j + 1, ny), k] + u[i, _yg(j - 1, ny), k]
                     + u[i, j, (k + 1) % nz] + u[i, j, (k - 1) % nz])
                out[i, j, k] = (s - 6.0 * u[i, j, k]) / (h * h)
    return out


def grad_m(u, h):
    nx, ny, nz = u.shape
    d = np.zeros((3,) + u.shape)
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                d[0, i, j, k] = (u[(i + 1) % nx, j, k] - u[(i - 1) % nx, j, k]) / (2 * h)
                d[1, i, j, k] = (u[i, _yg(j + 1, ny), k] - u[i, _yg(j - 1, ny), k]) / (2 * h)
                d[2, i, j, k] = (u[i, j, (k + 1) % nz] - u[i, j, (k - 1) % nz]) / (2 * h)
    return d


def poisson_dense(b, ulo, uhi, h, shift=0.0):
    """Solve (L_h - shift) u = b on j = 1..ny-2 with u = ulo at j = 0, uhi at j = ny-1, by
    assembling the matrix entry by entry and calling a dense solver. b has the full
    (nx, ny, nz) shape; its wall rows are ignored. Returns the full field including the
    walls."""
    nx, ny, nz = b.shape
    M = ny - 2
    n = nx * M * nz

    def idx(i, j, k):
        return (i * M + (j - 1)) * nz + k

    A = np.zeros((n, n))
    rhs = np.zeros(n)
    for i in range(nx):
        for j in range(1, ny - 1):
            for k in range(nz):
                r = idx(i, j, k)
                A[r, r] += -6.0 / h**2 - shift
                rhs[r] = b[i, j, k]
                for (ii, jj, kk) in ((i + 1, j, k), (i - 1, j, k), (i, j, k + 1), (i, j, k - 1),
                                     (i, j + 1, k), (i, j - 1, k)):
                    ii %= nx
                    kk %= nz
                    if jj == 0:
                        rhs[r] -= ulo[ii, kk] / h**2
                    elif jj == ny - 1:
                        rhs[r] -= uhi[ii, kk] / h**2
                    else:
                        A[r, idx(ii, jj, kk)] += 1.0 / h**2
    x = np.linalg.solve(A, rhs)
    u = np.zeros_like(b)
    u[:, 0, :] = ulo
    u[:, -1, :] = uhi
    for i in range(nx):
        for j in range(1, ny - 1):
            for k in range(nz):
                u[i, j, k] = x[idx(i, j, k)]
    return u


def wall_vz(y, H, kind, u0, u1):
    if kind == "poiseuille":
        return 4 * u0 * y * (H - y) / H**2
    return u0 + (u1 - u0) * y / H


def step_loops(phi, mu, psi, lam_V, dt, h, M, eta, eps, C_b, gamma_A, walls):
    """One step, node by node: advance phi, then mu (with a fixed gamma_A), then omega, then
    psi. walls = (kind, u0, u1). Returns (phi1, mu1, omega1, psi1)."""
    kind, u0, u1 = walls
    nx, ny, nz = phi.shape
    H = (ny - 1) * h
    dphi = grad_m(phi, h)
    lmu = lap_m(mu, h)
    phi1 = np.zeros_like(phi)
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                if j == 0 or j == ny - 1:
                    v = (0.0, 0.0, wall_vz(j * h, H, kind, u0, u1))
                else:
                    def P(c, a, b_, cc):
                        return psi[c, a % nx, b_, cc % nz]
                    dyz = (P(2, i, j + 1, k) - P(2, i, j - 1, k)) / (2 * h)
                    dzy = (P(1, i, j, k + 1) - P(1, i, j, k - 1)) / (2 * h)
                    dzx = (P(0, i, j, k + 1) - P(0, i, j, k - 1)) / (2 * h)
                    dxz = (P(2, i + 1, j, k) - P(2, i - 1, j, k)) / (2 * h)
                    dxy = (P(1, i + 1, j, k) - P(1, i - 1, j, k)) / (2 * h)
                    dyx = (P(0, i, j + 1, k) - P(0, i, j - 1, k)) / (2 * h)
                    v = (dyz - dzy, dzx - dxz, dxy - dyx)
                adv = v[0] * dphi[0, i, j, k] + v[1] * dphi[1, i, j, k] + v[2] * dphi[2, i, j, k]
                phi1[i, j, k] = phi[i, j, k] + dt * (M * (lmu[i, j, k] + lam_V) - adv)
    lphi = lap_m(phi1, h)
    g = np.zeros_like(phi1)
    for idx3 in np.ndindex(phi1.shape):
        p = phi1[idx3]
        g[idx3] = p**3 - p - eps**2 * lphi[idx3]
    lg = lap_m(g, h)
    mu1 = np.zeros_like(phi1)
    for idx3 in np.ndindex(phi1.shape):
        p = phi1[idx3]
        mu1[idx3] = C_b * ((3 * p * p - 1) * g[idx3] - eps**2 * lg[idx3]) - gamma_A * lphi[idx3]
    dp = grad_m(phi1, h)
    dm = grad_m(mu1, h)
    S = np.zeros((3,) + phi.shape)
    for idx3 in np.ndindex(phi1.shape):
        a = dp[(slice(None),) + idx3]
        b = dm[(slice(None),) + idx3]
        S[(slice(None),) + idx3] = np.cross(a, b) / eta
    y = np.arange(ny) * h
    if kind == "poiseuille":
        U = u0
        omx = 4 * U / H**2 * (H - 2 * y)
        psx = -(4 * U / H**2) * (H * y**2 / 2 - y**3 / 3)
    else:
        omx = np.full(ny, (u1 - u0) / H)
        psx = -(u0 * y + (u1 - u0) * y**2 / (2 * H))
    omega = np.zeros((3,) + phi.shape)
    psi1 = np.zeros((3,) + phi.shape)
    for c in range(3):
        wlo = np.full((nx, nz), omx[0] if c == 0 else 0.0)
        whi = np.full((nx, nz), omx[-1] if c == 0 else 0.0)
        omega[c] = poisson_dense(S[c], wlo, whi, h)
    for c in range(3):
        plo = np.full((nx, nz), psx[0] if c == 0 else 0.0)
        phi_ = np.full((nx, nz), psx[-1] if c == 0 else 0.0)
        psi1[c] = poisson_dense(-omega[c], plo, phi_, h)
    return phi1, mu1, omega, psi1


def energy_grad_edges(phi, h):
    """E = (1/2) h^3 sum over grid edges of weight * ((phi_a - phi_b)/h)^2; x and z edges
    carry the trapezoid weight of their row, y edges weight 1."""
    nx, ny, nz = phi.shape
    E = 0.0
    for i in range(nx):
        for j in range(ny):
            wj = 0.5 if j in (0, ny - 1) else 1.0
            for k in range(nz):
                E += wj * ((phi[(i + 1) % nx, j, k] - phi[i, j, k]) / h) ** 2
                E += wj * ((phi[i, j, (k + 1) % nz] - phi[i, j, k]) / h) ** 2
                if j < ny - 1:
                    E += ((phi[i, j + 1, k] - phi[i, j, k]) / h) ** 2
    return 0.5 * h**3 * E

