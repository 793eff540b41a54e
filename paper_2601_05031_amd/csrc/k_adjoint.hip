// Reverse step of one time step (the discrete adjoint), FP64, gfx950.
//
// The forward step maps phi^n to phi^{n+1}; mu^n, psi^n, lambda_V^n, gamma_A^n are functions
// of phi^n (the state functions of the penalty method). For a = dL/dphi^{n+1} these kernels
// form (d phi^{n+1}/d phi^n)^T a term by term, each transpose taken from its forward stencil:
//   * L_h with mirror ghosts is symmetric in the trapezoid-weighted inner product, so
//     L_h^T u = w L_h (u / w) (w = 1/2 on the wall rows);
//   * a central difference transposes to (D^T u)_m = (u_{m-1} - u_{m+1}) / 2h, with u kept
//     where the forward difference is evaluated (all rows in x and z; the interior rows in y,
//     where the mirrored difference is non-zero);
//   * the Poisson problems are self-adjoint with homogeneous walls (solved by the host driver
//     with the forward solver); their wall values enter rows 1 and ny-2 with weight 1/h^2;
//   * V (SM eq. (37)), A (SM eq. (32)) and the penalty multipliers are differentiated directly.
// The node loops are plain one-node-per-lane stencils (the reverse step is off the timed path).
#include "stencil.h"

namespace vs {

namespace {

// Reverse of phi' = phi + dt [M (L_h mu + lambda_V) - v . D phi] with respect to phi (through
// D phi), mu, lambda_V and psi (through v = curl psi), and the wall speed. Each lane owns one
// (j, k) column and walks an x-slab: the quantities it needs at its own column in the planes
// i - 1 and i + 1 (a, a v_x, b_y, b_z with b_c = -dt a D_c phi on the interior rows, 0 on the
// walls) are computed once per plane and kept; those of the y and z neighbours are computed
// from the plane i through the cache. Two pieces of set-up of the reverse step ride along: the
// lanes of the wall rows zero those rows of up to six other fields (the spectral sets the
// adjoint solves write only inside), and block 0 clears the status words and residual scalars.
struct AdjZero {
    double* p[6];
};
__global__ __launch_bounds__(kBlock) void k_adj_advect(
    const double* __restrict__ a, const double* __restrict__ phi, Vel vel, Dims d, double dt,
    double mob, SlabGrid sg, double* __restrict__ phibar, double* __restrict__ mubar,
    double* __restrict__ qx, double* __restrict__ qy, double* __restrict__ qz,
    double* __restrict__ partials, AdjZero zw, double* scal, int* istat) {
    __shared__ double sh[3 * 16];
    double acc[3] = {0.0, 0.0, 0.0};
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[SC_RELRES_MAX] = 0.0;
        scal[SC_RELRES_LAST] = 0.0;
        istat[IS_FLAGS] = 0;
        istat[IS_CYCLES] = 0;
        istat[IS_CONV] = 0;
    }
    const SlabIter it = slab_iter(d, sg);
    if (it.ok && zw.p[0] && (it.j == 0 || it.j == d.ny - 1)) {
        for (int i = it.i0; i < it.i1; ++i) {
            const size_t c = (size_t)i * d.ny * d.nz + (size_t)it.j * d.nz + it.k;
#pragma unroll
            for (int f = 0; f < 6; ++f)
                if (zw.p[f]) zw.p[f][c] = 0.0;
        }
    }
    if (it.ok) {
        const int j = it.j, k = it.k, nz = d.nz;
        const size_t plane = (size_t)d.ny * nz;
        const double r2h = d.inv_2h;
        const int kp = wrap(k + 1, nz), km = wrap(k - 1, nz);
        const bool wall = (j == 0 || j == d.ny - 1);
        // neighbour rows: mirrored past the walls (the L_h^T stencil); the y-neighbour terms
        // of the advection and of b are taken only where that row is interior
        const int jm = (j == 0) ? 1 : j - 1, jp = (j == d.ny - 1) ? d.ny - 2 : j + 1;
        const bool in_m = j >= 2, in_p = j <= d.ny - 3;
        const int o = j * nz + k, okm = j * nz + km, okp = j * nz + kp;
        const int ojm = jm * nz + k, ojp = jp * nz + k;
        const double vw = j == 0 ? vel.vz_lo : vel.vz_hi;
        // a, a v_x, b_y, b_z at (ii, j, k)
        auto xnode = [&](int ii, double& av, double& ax, double& by, double& bz) {
            const size_t b = (size_t)ii * plane;
            av = a[b + o];
            ax = by = bz = 0.0;
            if (!wall) {
                const double vx = ((vel.pz[b + ojp] - vel.pz[b + ojm]) - (vel.py[b + okp] - vel.py[b + okm])) * r2h;
                ax = av * vx;
                by = -dt * av * ((phi[b + ojp] - phi[b + ojm]) * r2h);
                bz = -dt * av * ((phi[b + okp] - phi[b + okm]) * r2h);
            }
        };
        double a_m, ax_m, by_m, bz_m, a_0, ax_0, by_0, bz_0;
        xnode(wrap(it.i0 - 1, d.nx), a_m, ax_m, by_m, bz_m);
        xnode(it.i0, a_0, ax_0, by_0, bz_0);
        const double wj = wrow(d, j), rwm = 1.0 / wrow(d, jm), rwp = 1.0 / wrow(d, jp);
        for (int i = it.i0; i < it.i1; ++i) {
            const int ip = (i + 1 == d.nx) ? 0 : i + 1, im = (i == 0) ? d.nx - 1 : i - 1;
            double a_p, ax_p, by_p, bz_p;
            xnode(ip, a_p, ax_p, by_p, bz_p);
            const size_t b = (size_t)i * plane, bm = (size_t)im * plane, bp = (size_t)ip * plane;
            const size_t c = b + o;
            const double a_km = a[b + okm], a_kp = a[b + okp];
            const double a_jm = a[b + ojm], a_jp = a[b + ojp];
            // a v_z at k -/+ 1 (the wall speed on the walls)
            double vz_km = vw, vz_kp = vw;
            if (!wall) {
                vz_km = ((vel.py[bp + okm] - vel.py[bm + okm]) - (vel.px[b + jp * nz + km] - vel.px[b + jm * nz + km])) * r2h;
                vz_kp = ((vel.py[bp + okp] - vel.py[bm + okp]) - (vel.px[b + jp * nz + kp] - vel.px[b + jm * nz + kp])) * r2h;
            }
            // a v_y, b_x, b_z at j -/+ 1 (interior rows only)
            double ay_jm = 0.0, ay_jp = 0.0, bx_jm = 0.0, bx_jp = 0.0, bz_jm = 0.0, bz_jp = 0.0;
            if (in_m) {
                const int r = jm * nz;
                const double vy = ((vel.px[b + r + kp] - vel.px[b + r + km]) - (vel.pz[bp + ojm] - vel.pz[bm + ojm])) * r2h;
                ay_jm = a_jm * vy;
                bx_jm = -dt * a_jm * ((phi[bp + ojm] - phi[bm + ojm]) * r2h);
                bz_jm = -dt * a_jm * ((phi[b + r + kp] - phi[b + r + km]) * r2h);
            }
            if (in_p) {
                const int r = jp * nz;
                const double vy = ((vel.px[b + r + kp] - vel.px[b + r + km]) - (vel.pz[bp + ojp] - vel.pz[bm + ojp])) * r2h;
                ay_jp = a_jp * vy;
                bx_jp = -dt * a_jp * ((phi[bp + ojp] - phi[bm + ojp]) * r2h);
                bz_jp = -dt * a_jp * ((phi[b + r + kp] - phi[b + r + km]) * r2h);
            }
            // b_x, b_y at k -/+ 1 (row j, interior only)
            double bx_km = 0.0, bx_kp = 0.0, by_km = 0.0, by_kp = 0.0;
            if (!wall) {
                bx_km = -dt * a_km * ((phi[bp + okm] - phi[bm + okm]) * r2h);
                bx_kp = -dt * a_kp * ((phi[bp + okp] - phi[bm + okp]) * r2h);
                by_km = -dt * a_km * ((phi[b + jp * nz + km] - phi[b + jm * nz + km]) * r2h);
                by_kp = -dt * a_kp * ((phi[b + jp * nz + kp] - phi[b + jm * nz + kp]) * r2h);
            }
            // phibar = a - dt sum_c D_c^T (a v_c)
            double t = (ax_m - ax_p) + (a_km * vz_km - a_kp * vz_kp);
            t += ay_jm;
            t -= ay_jp;
            phibar[c] = a_0 - dt * t * r2h;
            // mubar = dt M L_h^T a
            const double xz = a_p + a_m + a_kp + a_km;
            mubar[c] = dt * mob * ((xz + wj * (a_jp * rwp + a_jm * rwm) - 6.0 * a_0) * d.inv_h2);
            // psibar = curl^T b
            const double sx = ((by_km - by_kp) - (bz_jm - bz_jp)) * r2h;
            const double sy = ((bz_m - bz_p) - (bx_km - bx_kp)) * r2h;
            const double sz = ((bx_jm - bx_jp) - (by_m - by_p)) * r2h;
            qx[c] = sx;
            qy[c] = sy;
            qz[c] = sz;
            acc[0] += a_0;
            if (wall) {
                const double dz = (phi[b + okp] - phi[b + okm]) * r2h;
                acc[1] += a_0 * vw * dz;
                acc[2] += sx * vel.px[c] + sy * vel.py[c] + sz * vel.pz[c];
            }
            a_m = a_0; ax_m = ax_0; by_m = by_0; bz_m = bz_0;
            a_0 = a_p; ax_0 = ax_p; by_0 = by_p; bz_0 = bz_p;
        }
    }
    block_sum<3>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) partials[q * kMaxPartialBlocks + blockIdx.x] = acc[q];
    }
}

// scal[dst + q] = sum_b partials[q][b] for q in [first, nslots), fixed order.
__global__ __launch_bounds__(1024) void k_adj_sum(const double* __restrict__ partials, int nblocks,
                                                  int first, int nslots, double* scal, int dst) {
    __shared__ double sh[4 * 16];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int q = first; q < nslots; ++q) acc[q] += partials[q * kMaxPartialBlocks + b];
    block_sum<4>(acc, sh);
    if (threadIdx.x == 0)
        for (int q = first; q < nslots; ++q) scal[dst + q] = acc[q];
}

// Wall coupling of an adjoint Poisson solve: the forward walls enter rows 1 and M with 1/h^2.
__global__ __launch_bounds__(kBlock) void k_adj_wall_couple(const double* __restrict__ u0,
                                                           const double* __restrict__ u1,
                                                           const double* __restrict__ u2,
                                                           const double* __restrict__ w0,
                                                           const double* __restrict__ w1,
                                                           const double* __restrict__ w2, Dims d,
                                                           double* __restrict__ partials) {
    __shared__ double sh[16];
    double acc[1] = {0.0};
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int plane = d.nx * d.nz;
    if (t < 3 * plane) {
        const int c = t / plane;
        const int r = t - c * plane;
        const int i = r / d.nz, k = r - (r / d.nz) * d.nz;
        const double* u = c == 0 ? u0 : (c == 1 ? u1 : u2);
        const double* w = c == 0 ? w0 : (c == 1 ? w1 : w2);
        acc[0] = -(u[node(d, i, 1, k)] * w[node(d, i, 0, k)] +
                   u[node(d, i, d.ny - 2, k)] * w[node(d, i, d.ny - 1, k)]) * d.inv_h2;
    }
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// Reverse of S = (1/eta) D phi x D mu on the interior rows: phibar -= D . abar and
// mubar -= D . bbar (central differences transposed), abar = (1/eta) D mu x Sbar,
// bbar = (1/eta) Sbar x D phi at each interior node (so the wall rows receive the y terms of
// rows 1 and M). Each lane owns one (j, k) column and walks an x-slab; the x components of
// abar, bbar at its column in the planes i -/+ 1 are kept from plane to plane, the y and z
// components at the neighbours are computed from the plane i. The
// wall couplings of the two adjoint solves ride along as block partials (slot 0: u1 on rows 1
// and M against the psi walls, skipped when u1 is NULL; slot 1: Sbar against the omega walls).
__global__ __launch_bounds__(kBlock) void k_adj_source(
    const double* __restrict__ phi, const double* __restrict__ mu, const double* __restrict__ s0,
    const double* __restrict__ s1, const double* __restrict__ s2, Dims d, double inv_eta,
    SlabGrid sg, double* __restrict__ phibar, double* __restrict__ mubar, WallPairs wp,
    double* __restrict__ partials) {
    __shared__ double sh[2 * 16];
    double acc[2] = {0.0, 0.0};
    const SlabIter it = slab_iter(d, sg);
    if (it.ok) {
        const int j = it.j, k = it.k, nz = d.nz;
        const bool inr = j >= 1 && j <= d.ny - 2;
        const size_t plane = (size_t)d.ny * nz;
        const double r2h = d.inv_2h;
        const int kp = wrap(k + 1, nz), km = wrap(k - 1, nz);
        const int o = j * nz + k, okm = j * nz + km, okp = j * nz + kp;
        const int ojm = (j - 1) * nz + k, ojp = (j + 1) * nz + k;
        const bool in_m = j >= 2, in_p = j <= d.ny - 3;   // rows j -/+ 1 interior
        // abar_x, bbar_x at (ii, j, k): D_y, D_z of mu and phi (0 on the wall rows)
        auto xnode = [&](int ii, double& ab, double& bb) {
            ab = bb = 0.0;
            if (!inr) return;
            const size_t b = (size_t)ii * plane;
            const double S1 = s1[b + o], S2 = s2[b + o];
            const double f1 = (phi[b + ojp] - phi[b + ojm]) * r2h, f2 = (phi[b + okp] - phi[b + okm]) * r2h;
            const double m1 = (mu[b + ojp] - mu[b + ojm]) * r2h, m2 = (mu[b + okp] - mu[b + okm]) * r2h;
            ab = (m1 * S2 - m2 * S1) * inv_eta;
            bb = (S1 * f2 - S2 * f1) * inv_eta;
        };
        double ab_m, bb_m, ab_0, bb_0;
        xnode(wrap(it.i0 - 1, d.nx), ab_m, bb_m);
        xnode(it.i0, ab_0, bb_0);
        for (int i = it.i0; i < it.i1; ++i) {
            const int ip = (i + 1 == d.nx) ? 0 : i + 1, im = (i == 0) ? d.nx - 1 : i - 1;
            double ab_p, bb_p;
            xnode(ip, ab_p, bb_p);
            const size_t b = (size_t)i * plane, bm = (size_t)im * plane, bp = (size_t)ip * plane;
            // abar_z, bbar_z at k -/+ 1: D_x, D_y
            double abz[2] = {0.0, 0.0}, bbz[2] = {0.0, 0.0};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (!inr) continue;
                const int kk = h ? kp : km;
                const int q = j * nz + kk;
                const double S0 = s0[b + q], S1 = s1[b + q];
                const double f0 = (phi[bp + q] - phi[bm + q]) * r2h;
                const double f1 = (phi[b + (j + 1) * nz + kk] - phi[b + (j - 1) * nz + kk]) * r2h;
                const double m0 = (mu[bp + q] - mu[bm + q]) * r2h;
                const double m1 = (mu[b + (j + 1) * nz + kk] - mu[b + (j - 1) * nz + kk]) * r2h;
                abz[h] = (m0 * S1 - m1 * S0) * inv_eta;
                bbz[h] = (S0 * f1 - S1 * f0) * inv_eta;
            }
            // abar_y, bbar_y at j -/+ 1 (interior rows only): D_z, D_x
            double aby[2] = {0.0, 0.0}, bby[2] = {0.0, 0.0};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h ? !in_p : !in_m) continue;
                const int r = (h ? j + 1 : j - 1) * nz;
                const int q = r + k;
                const double S0 = s0[b + q], S2 = s2[b + q];
                const double f0 = (phi[bp + q] - phi[bm + q]) * r2h;
                const double f2 = (phi[b + r + kp] - phi[b + r + km]) * r2h;
                const double m0 = (mu[bp + q] - mu[bm + q]) * r2h;
                const double m2 = (mu[b + r + kp] - mu[b + r + km]) * r2h;
                aby[h] = (m2 * S0 - m0 * S2) * inv_eta;
                bby[h] = (S2 * f0 - S0 * f2) * inv_eta;
            }
            const double tp = ((ab_m - ab_p) + (abz[0] - abz[1])) + (aby[0] - aby[1]);
            const double tm = ((bb_m - bb_p) + (bbz[0] - bbz[1])) + (bby[0] - bby[1]);
            const size_t c = b + o;
            phibar[c] += tp * r2h;
            mubar[c] += tm * r2h;
            // wall couplings: rows 1 and M against the wall planes 0 and ny - 1
            if (j == 1 || j == d.ny - 2) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    if (e == 0 ? j != 1 : j != d.ny - 2) continue;
                    const size_t w = b + (size_t)(e == 0 ? 0 : d.ny - 1) * nz + k;
                    if (wp.u[0])
                        acc[0] -= (wp.u[0][c] * wp.uw[0][w] + wp.u[1][c] * wp.uw[1][w] + wp.u[2][c] * wp.uw[2][w]) * d.inv_h2;
                    acc[1] -= (s0[c] * wp.sw[0][w] + s1[c] * wp.sw[1][w] + s2[c] * wp.sw[2][w]) * d.inv_h2;
                }
            }
            ab_m = ab_0; bb_m = bb_0;
            ab_0 = ab_p; bb_0 = bb_p;
        }
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        partials[0 * kMaxPartialBlocks + blockIdx.x] = acc[0];
        partials[1 * kMaxPartialBlocks + blockIdx.x] = acc[1];
    }
}

// Bending: gbar = C_b [(3 phi^2 - 1) mubar - eps^2 L_h^T mubar] (the transpose of
// mu = C_b [(3 phi^2 - 1) g - eps^2 L_h g], g = phi^3 - phi - eps^2 L_h phi), and the block
// partials of mubar . d mu/d kappa (slot 2) and of -mubar . L_h phi (slot 3). The first uses
// mubar . L_h g = g . L_h^T mubar (a transpose, exact), so g is needed at the node only:
// mubar . d mu/d kappa = (dC_b/d kappa) g [(3 phi^2 - 1) mubar - eps^2 L_h^T mubar].
__global__ __launch_bounds__(kBlock) void k_adj_mu1(const double* __restrict__ phi,
                                                   const double* __restrict__ mubar, Dims d,
                                                   double C_b, double dCb, double eps, SlabGrid sg,
                                                   double* __restrict__ gbar,
                                                   double* __restrict__ partials) {
    __shared__ double sh[2 * 16];
    double acc[2] = {0.0, 0.0};
    const SlabIter it = slab_iter(d, sg);
    const double eps2 = eps * eps;
    if (it.ok) {
        const int j = it.j, k = it.k;
        for (int i = it.i0; i < it.i1; ++i) {
            const Nbr n = neighbours_mirror(d, i, j, k);
            const double p = phi[n.c];
            const double mb = mubar[n.c];
            const double lphi = lap7(phi, n, d.inv_h2);
            const double gc = p * p * p - p - eps2 * lphi;
            const double core = (3.0 * p * p - 1.0) * mb - eps2 * lapT(mubar, d, i, j, k);
            gbar[n.c] = C_b * core;
            acc[0] += dCb * gc * core;
            acc[1] -= mb * lphi;
        }
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        partials[2 * kMaxPartialBlocks + blockIdx.x] = acc[0];
        partials[3 * kMaxPartialBlocks + blockIdx.x] = acc[1];
    }
}

// phibar += (d mu / d phi)^T mubar + lambda_bar d lambda_V/d phi + A_bar dA/d phi. Each lane
// owns one (j, k) column and walks an x-slab with phi of the planes i-2 .. i+2 and mubar, gbar
// of the planes i-1 .. i+1 in registers.
__global__ __launch_bounds__(kBlock) void k_adj_mu2(const double* __restrict__ phi,
                                                   const double* __restrict__ mubar,
                                                   const double* __restrict__ gbar,
                                                   const double* __restrict__ scal, Dims d,
                                                   int model, double C_b, double eps, double sigma,
                                                   double dt, double mob, double rate_V, double k_A,
                                                   SlabGrid sg, double* __restrict__ phibar) {
    const SlabIter it = slab_iter(d, sg);
    if (!it.ok) return;
    const int j = it.j, k = it.k, nz = d.nz;
    const size_t plane = (size_t)d.ny * nz;
    const bool ch = model == VS_CAHN_HILLIARD;
    const double w = wrow(d, j);
    const double h3 = d.h * d.h * d.h;
    const double vol = (double)d.nx * nz * (d.ny - 1) * h3;
    const double lam_bar = dt * mob * scal[SC_ADJ_SUM_A];
    const double r0 = lam_bar * (-rate_V * h3 * w / (mob * vol));
    const double eps2 = eps * eps;
    const double gam = scal[SC_GAMMA];
    const double A0 = scal[SC_A0];
    const bool area = !ch && k_A != 0.0 && A0 > 0.0;
    const double Abar = area ? scal[SC_ADJ_GAMMA] * k_A / A0 : 0.0;
    const int kp = wrap(k + 1, nz), km = wrap(k - 1, nz);
    const int kp2 = wrap(k + 2, nz), km2 = wrap(k - 2, nz);
    const int jm = (j == 0) ? 1 : j - 1, jp = (j == d.ny - 1) ? d.ny - 2 : j + 1;   // mirrored
    const int o = j * nz + k, okm = j * nz + km, okp = j * nz + kp;
    const int ojm = jm * nz + k, ojp = jp * nz + k;
    const double wj = wrow(d, j), rwm = 1.0 / wrow(d, jm), rwp = 1.0 / wrow(d, jp);
    const bool in_m = j >= 2, in_p = j <= d.ny - 3;   // rows j -/+ 1 interior
    // L_h^T u at the node from the x-neighbours xm, xp and the plane base b
    auto lapt = [&](const double* __restrict__ u, size_t b, double xm, double x0, double xp) {
        const double xz = xp + xm + u[b + okp] + u[b + okm];
        return (xz + wj * (u[b + ojp] * rwp + u[b + ojm] * rwm) - 6.0 * x0) * d.inv_h2;
    };
    auto ld = [&](const double* __restrict__ u, int ii) { return u[(size_t)ii * plane + o]; };
    const int i0 = it.i0;
    double pm2 = ld(phi, wrap(i0 - 2, d.nx)), pm1 = ld(phi, wrap(i0 - 1, d.nx)), p0 = ld(phi, i0);
    double pp1 = ld(phi, wrap(i0 + 1, d.nx));
    double mm = ld(mubar, wrap(i0 - 1, d.nx)), m0 = ld(mubar, i0);
    double gm = 0.0, g0 = 0.0;
    if (!ch) {
        gm = ld(gbar, wrap(i0 - 1, d.nx));
        g0 = ld(gbar, i0);
    }
    for (int i = i0; i < it.i1; ++i) {
        const int ip = (i + 1 == d.nx) ? 0 : i + 1;
        const double pp2 = ld(phi, wrap(i + 2, d.nx));
        const double mp = ld(mubar, ip);
        const double gp = ch ? 0.0 : ld(gbar, ip);
        const size_t b = (size_t)i * plane;
        const size_t c = b + o;
        const double p = p0;
        double r = r0;
        if (ch) {
            r += (3.0 * p * p - 1.0) * m0 - sigma * lapt(mubar, b, mm, m0, mp);
        } else {
            const double lphi = (pp1 + pm1 + phi[b + ojp] + phi[b + ojm] + phi[b + okp] + phi[b + okm] - 6.0 * p) * d.inv_h2;
            const double gc = p * p * p - p - eps2 * lphi;
            r += 6.0 * C_b * p * gc * m0 - gam * lapt(mubar, b, mm, m0, mp) +
                 (3.0 * p * p - 1.0) * g0 - eps2 * lapt(gbar, b, gm, g0, gp);
            if (area) {
                // dA/dphi = 3/(2 sqrt 2) h^3 [eps sum_c D_c^T (w D_c phi) + w (phi^2 - 1) phi / eps]
                const double dxm = (p - pm2) * d.inv_2h, dxp = (pp2 - p) * d.inv_2h;
                const double dzm = (p - phi[b + j * nz + km2]) * d.inv_2h;
                const double dzp = (phi[b + j * nz + kp2] - p) * d.inv_2h;
                double div = w * ((dxm - dxp) + (dzm - dzp));
                if (in_m) div += (p - phi[b + (j - 2) * nz + k]) * d.inv_2h;
                if (in_p) div -= (phi[b + (j + 2) * nz + k] - p) * d.inv_2h;
                const double dA = 3.0 / (2.0 * 1.4142135623730951) * h3 *
                                  (eps * div * d.inv_2h + w * (p * p - 1.0) * p / eps);
                r += Abar * dA;
            }
        }
        phibar[c] += r;
        pm2 = pm1; pm1 = p0; p0 = pp1; pp1 = pp2;
        mm = m0; m0 = mp;
        gm = g0; g0 = gp;
    }
}

}  // namespace

// x-slabs of about 8 planes for the marching reverse kernels (at most 512 blocks)
SlabGrid adj_slab_grid(const Dims& d) { return slab_grid(d.ny * d.nz, d.nx, 512); }

void launch_adj_advect(hipStream_t s, const Dims& d, const double* a, const double* phi,
                       const double* const psi[3], double dt, double mobility, double vz_lo,
                       double vz_hi, double* phibar, double* mubar, double* const psibar[3],
                       double* part, double* scal, int* istat, double* const zero_walls[6]) {
    const SlabGrid g = adj_slab_grid(d);
    const Vel vel{psi[0], psi[1], psi[2], vz_lo, vz_hi};
    const int nb = g.gx * g.gi;
    AdjZero zw{};
    for (int f = 0; f < 6; ++f) zw.p[f] = zero_walls ? zero_walls[f] : nullptr;
    launch_kernel(k_adj_advect, dim3(nb), dim3(kBlock), 0, s, a, phi, vel, d, dt, mobility, g,
                  phibar, mubar, psibar[0], psibar[1], psibar[2], part, zw, scal, istat);
    launch_kernel(k_adj_sum, dim3(1), dim3(1024), 0, s, (const double*)part, nb, 0, 3, scal,
                  (int)SC_ADJ_SUM_A);
}

void launch_adj_wall_couple(hipStream_t s, const Dims& d, double* const u[3],
                            double* const wall[3], double* part, double* scal, int slot) {
    const int nb = (3 * d.nx * d.nz + kBlock - 1) / kBlock;
    launch_kernel(k_adj_wall_couple, dim3(nb), dim3(kBlock), 0, s, u[0], u[1], u[2], wall[0],
                  wall[1], wall[2], d, part);
    launch_kernel(k_adj_sum, dim3(1), dim3(1024), 0, s, (const double*)part, nb, 0, 1, scal, slot);
}

void launch_adj_source(hipStream_t s, const Dims& d, const double* phi, const double* mu,
                       double* const sbar[3], double inv_eta, double* phibar, double* mubar,
                       const double* const u1[3], const double* const psi_walls[3],
                       const double* const om_walls[3], double* part) {
    const SlabGrid g = adj_slab_grid(d);
    WallPairs wp{};
    for (int c = 0; c < 3; ++c) {
        wp.u[c] = u1 ? u1[c] : nullptr;
        wp.uw[c] = psi_walls[c];
        wp.sw[c] = om_walls[c];
    }
    launch_kernel(k_adj_source, dim3(g.gx * g.gi), dim3(kBlock), 0, s, phi, mu,
                  (const double*)sbar[0], (const double*)sbar[1], (const double*)sbar[2], d, inv_eta,
                  g, phibar, mubar, wp, part);
}

void launch_adj_mu1(hipStream_t s, const Dims& d, const double* phi, const double* mubar,
                    double C_b, double dCb_dkappa, double eps, double* gbar, double* part) {
    const SlabGrid g = adj_slab_grid(d);
    launch_kernel(k_adj_mu1, dim3(g.gx * g.gi), dim3(kBlock), 0, s, phi, mubar, d, C_b, dCb_dkappa,
                  eps, g, gbar, part);
}

void launch_adj_sums(hipStream_t s, const Dims& d, const double* part, int first, int nslots,
                     double* scal) {
    const SlabGrid g = adj_slab_grid(d);
    static_assert(SC_ADJ_OMC == SC_ADJ_PSIC + 1 && SC_ADJ_KAPPA == SC_ADJ_PSIC + 2 &&
                      SC_ADJ_GAMMA == SC_ADJ_PSIC + 3,
                  "adjoint sums: slots 0-3 map onto consecutive scalars");
    launch_kernel(k_adj_sum, dim3(1), dim3(1024), 0, s, part, g.gx * g.gi, first, nslots, scal,
                  (int)SC_ADJ_PSIC);
}

void launch_adj_mu2(hipStream_t s, const Dims& d, const double* phi, const double* mubar,
                    const double* gbar, const double* scal, int model, double C_b, double eps,
                    double sigma, double dt, double mobility, double rate_V, double k_A,
                    double* phibar) {
    const SlabGrid g = adj_slab_grid(d);
    launch_kernel(k_adj_mu2, dim3(g.gx * g.gi), dim3(kBlock), 0, s, phi, mubar, gbar, scal, d, model,
                  C_b, eps, sigma, dt, mobility, rate_V, k_A, g, phibar);
}

}  // namespace vs
