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

// b_c = -dt a D_c phi at an interior node, 0 on the wall rows and outside the grid.
__device__ __forceinline__ double bcur(const double* __restrict__ a, const double* __restrict__ phi,
                                       const Dims& d, double dt, int c, int i, int j, int k) {
    if (j < 1 || j > d.ny - 2) return 0.0;
    return -dt * a[node(d, i, j, k)] * dcen(phi, d, c, i, j, k);
}

// Reverse of phi' = phi + dt [M (L_h mu + lambda_V) - v . D phi] with respect to phi (through
// D phi), mu, lambda_V and psi (through v = curl psi), and the wall speed.
__global__ __launch_bounds__(kBlock) void k_adj_advect(
    const double* __restrict__ a, const double* __restrict__ phi, Vel vel, Dims d, double dt,
    double mob, SlabGrid sg, double* __restrict__ phibar, double* __restrict__ mubar,
    double* __restrict__ qx, double* __restrict__ qy, double* __restrict__ qz,
    double* __restrict__ partials) {
    __shared__ double sh[3 * 16];
    double acc[3] = {0.0, 0.0, 0.0};
    const SlabIter it = slab_iter(d, sg);
    if (it.ok) {
        const int j = it.j, k = it.k;
        const int kp = wrap(k + 1, d.nz), km = wrap(k - 1, d.nz);
        const bool wall = (j == 0 || j == d.ny - 1);
        for (int i = it.i0; i < it.i1; ++i) {
            const int ip = wrap(i + 1, d.nx), im = wrap(i - 1, d.nx);
            const int c = node(d, i, j, k);
            const double am = a[c];
            // phibar = a - dt sum_c D_c^T (a v_c)
            double t = (a[node(d, im, j, k)] * vx_at(vel, d, im, j, k) -
                        a[node(d, ip, j, k)] * vx_at(vel, d, ip, j, k)) +
                       (a[node(d, i, j, km)] * vz_at(vel, d, i, j, km) -
                        a[node(d, i, j, kp)] * vz_at(vel, d, i, j, kp));
            if (j - 1 >= 0) t += a[node(d, i, j - 1, k)] * vy_at(vel, d, i, j - 1, k);
            if (j + 1 <= d.ny - 1) t -= a[node(d, i, j + 1, k)] * vy_at(vel, d, i, j + 1, k);
            phibar[c] = am - dt * t * d.inv_2h;
            mubar[c] = dt * mob * lapT(a, d, i, j, k);
            // psibar = curl^T b, b_c = -dt a D_c phi on the interior rows
            const double bx_jm = bcur(a, phi, d, dt, 0, i, j - 1, k), bx_jp = bcur(a, phi, d, dt, 0, i, j + 1, k);
            const double bz_jm = bcur(a, phi, d, dt, 2, i, j - 1, k), bz_jp = bcur(a, phi, d, dt, 2, i, j + 1, k);
            double by_km = 0.0, by_kp = 0.0, bz_im = 0.0, bz_ip = 0.0, bx_km = 0.0, bx_kp = 0.0,
                   by_im = 0.0, by_ip = 0.0;
            if (!wall) {
                by_km = bcur(a, phi, d, dt, 1, i, j, km);
                by_kp = bcur(a, phi, d, dt, 1, i, j, kp);
                bz_im = bcur(a, phi, d, dt, 2, im, j, k);
                bz_ip = bcur(a, phi, d, dt, 2, ip, j, k);
                bx_km = bcur(a, phi, d, dt, 0, i, j, km);
                bx_kp = bcur(a, phi, d, dt, 0, i, j, kp);
                by_im = bcur(a, phi, d, dt, 1, im, j, k);
                by_ip = bcur(a, phi, d, dt, 1, ip, j, k);
            }
            const double sx = ((by_km - by_kp) - (bz_jm - bz_jp)) * d.inv_2h;
            const double sy = ((bz_im - bz_ip) - (bx_km - bx_kp)) * d.inv_2h;
            const double sz = ((bx_jm - bx_jp) - (by_im - by_ip)) * d.inv_2h;
            qx[c] = sx;
            qy[c] = sy;
            qz[c] = sz;
            acc[0] += am;
            if (wall) {
                const double dz = (phi[node(d, i, j, kp)] - phi[node(d, i, j, km)]) * d.inv_2h;
                acc[1] += am * (j == 0 ? vel.vz_lo : vel.vz_hi) * dz;
                acc[2] += sx * vel.px[c] + sy * vel.py[c] + sz * vel.pz[c];
            }
        }
    }
    block_sum<3>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) partials[q * kMaxPartialBlocks + blockIdx.x] = acc[q];
    }
}

// scal[dst + q] = sum_b partials[q][b], fixed order.
__global__ __launch_bounds__(1024) void k_adj_sum(const double* __restrict__ partials, int nblocks,
                                                  int nslots, double* scal, int dst) {
    __shared__ double sh[4 * 16];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int q = 0; q < nslots; ++q) acc[q] += partials[q * kMaxPartialBlocks + b];
    block_sum<4>(acc, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < nslots; ++q) scal[dst + q] = acc[q];
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

// abar = (1/eta) D mu x Sbar and bbar = (1/eta) Sbar x D phi at an interior node.
__device__ __forceinline__ void cross_bars(const double* __restrict__ phi, const double* __restrict__ mu,
                                           const double* __restrict__ s0, const double* __restrict__ s1,
                                           const double* __restrict__ s2, const Dims& d, double inv_eta,
                                           int i, int j, int k, double* ab, double* bb) {
    const int c = node(d, i, j, k);
    const double S0 = s0[c], S1 = s1[c], S2 = s2[c];
    const double f0 = dcen(phi, d, 0, i, j, k), f1 = dcen(phi, d, 1, i, j, k), f2 = dcen(phi, d, 2, i, j, k);
    const double m0 = dcen(mu, d, 0, i, j, k), m1 = dcen(mu, d, 1, i, j, k), m2 = dcen(mu, d, 2, i, j, k);
    ab[0] = (m1 * S2 - m2 * S1) * inv_eta;
    ab[1] = (m2 * S0 - m0 * S2) * inv_eta;
    ab[2] = (m0 * S1 - m1 * S0) * inv_eta;
    bb[0] = (S1 * f2 - S2 * f1) * inv_eta;
    bb[1] = (S2 * f0 - S0 * f2) * inv_eta;
    bb[2] = (S0 * f1 - S1 * f0) * inv_eta;
}

__global__ __launch_bounds__(kBlock) void k_adj_source(const double* __restrict__ phi,
                                                      const double* __restrict__ mu,
                                                      const double* __restrict__ s0,
                                                      const double* __restrict__ s1,
                                                      const double* __restrict__ s2, Dims d,
                                                      double inv_eta, double* __restrict__ phibar,
                                                      double* __restrict__ mubar) {
    int i, j, k;
    bool ok;
    plane_index(d, i, j, k, ok);
    if (!ok) return;
    double ab[3], bb[3];
    double tp = 0.0, tm = 0.0;
    // x and z neighbours share row j: non-zero only on the interior rows
    if (interior(d, j)) {
        const int nb[4][3] = {{wrap(i - 1, d.nx), j, k}, {wrap(i + 1, d.nx), j, k},
                              {i, j, wrap(k - 1, d.nz)}, {i, j, wrap(k + 1, d.nz)}};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            cross_bars(phi, mu, s0, s1, s2, d, inv_eta, nb[q][0], nb[q][1], nb[q][2], ab, bb);
            const int ax = q < 2 ? 0 : 2;
            const double sg = (q & 1) ? -1.0 : 1.0;
            tp += sg * ab[ax];
            tm += sg * bb[ax];
        }
    }
    if (interior(d, j - 1)) {
        cross_bars(phi, mu, s0, s1, s2, d, inv_eta, i, j - 1, k, ab, bb);
        tp += ab[1];
        tm += bb[1];
    }
    if (interior(d, j + 1)) {
        cross_bars(phi, mu, s0, s1, s2, d, inv_eta, i, j + 1, k, ab, bb);
        tp -= ab[1];
        tm -= bb[1];
    }
    const int c = node(d, i, j, k);
    phibar[c] += tp * d.inv_2h;
    mubar[c] += tm * d.inv_2h;
}

// gbar = C_b [(3 phi^2 - 1) mubar - eps^2 L^T mubar]; partial sums of mubar d mu/d kappa
// and -mubar L_h phi.
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
            const int ip = wrap(i + 1, d.nx), im = wrap(i - 1, d.nx);
            const int jp = (j + 1 == d.ny) ? d.ny - 2 : j + 1;
            const int jm = (j == 0) ? 1 : j - 1;
            const int kp = wrap(k + 1, d.nz), km = wrap(k - 1, d.nz);
            const double gs = g_at(phi, d, ip, j, k, eps2) + g_at(phi, d, im, j, k, eps2) +
                              g_at(phi, d, i, jp, k, eps2) + g_at(phi, d, i, jm, k, eps2) +
                              g_at(phi, d, i, j, kp, eps2) + g_at(phi, d, i, j, km, eps2);
            const double lg = (gs - 6.0 * gc) * d.inv_h2;
            gbar[n.c] = C_b * ((3.0 * p * p - 1.0) * mb - eps2 * lapT(mubar, d, i, j, k));
            acc[0] += mb * dCb * ((3.0 * p * p - 1.0) * gc - eps2 * lg);
            acc[1] -= mb * lphi;
        }
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        partials[0 * kMaxPartialBlocks + blockIdx.x] = acc[0];
        partials[1 * kMaxPartialBlocks + blockIdx.x] = acc[1];
    }
}

// phibar += (d mu / d phi)^T mubar + lambda_bar d lambda_V/d phi + A_bar dA/d phi.
__global__ __launch_bounds__(kBlock) void k_adj_mu2(const double* __restrict__ phi,
                                                   const double* __restrict__ mubar,
                                                   const double* __restrict__ gbar,
                                                   const double* __restrict__ scal, Dims d,
                                                   int model, double C_b, double eps, double sigma,
                                                   double dt, double mob, double rate_V, double k_A,
                                                   double* __restrict__ phibar) {
    int i, j, k;
    bool ok;
    plane_index(d, i, j, k, ok);
    if (!ok) return;
    const Nbr n = neighbours_mirror(d, i, j, k);
    const double p = phi[n.c];
    const double mb = mubar[n.c];
    const double w = wrow(d, j);
    const double h3 = d.h * d.h * d.h;
    const double vol = (double)d.nx * d.nz * (d.ny - 1) * h3;
    const double lam_bar = dt * mob * scal[SC_ADJ_SUM_A];
    double r = lam_bar * (-rate_V * h3 * w / (mob * vol));
    if (model == VS_CAHN_HILLIARD) {
        r += (3.0 * p * p - 1.0) * mb - sigma * lapT(mubar, d, i, j, k);
        phibar[n.c] += r;
        return;
    }
    const double eps2 = eps * eps;
    const double gc = p * p * p - p - eps2 * lap7(phi, n, d.inv_h2);
    r += 6.0 * C_b * p * gc * mb - scal[SC_GAMMA] * lapT(mubar, d, i, j, k) +
         (3.0 * p * p - 1.0) * gbar[n.c] - eps2 * lapT(gbar, d, i, j, k);
    const double A0 = scal[SC_A0];
    if (k_A != 0.0 && A0 > 0.0) {
        const double Abar = scal[SC_ADJ_GAMMA] * k_A / A0;
        // dA/dphi = 3/(2 sqrt 2) h^3 [eps sum_c D_c^T (w D_c phi) + w (phi^2 - 1) phi / eps]
        const int ip = wrap(i + 1, d.nx), im = wrap(i - 1, d.nx);
        const int kp = wrap(k + 1, d.nz), km = wrap(k - 1, d.nz);
        double div = w * ((dcen(phi, d, 0, im, j, k) - dcen(phi, d, 0, ip, j, k)) +
                          (dcen(phi, d, 2, i, j, km) - dcen(phi, d, 2, i, j, kp)));
        if (interior(d, j - 1)) div += dcen(phi, d, 1, i, j - 1, k);
        if (interior(d, j + 1)) div -= dcen(phi, d, 1, i, j + 1, k);
        const double dA = 3.0 / (2.0 * 1.4142135623730951) * h3 *
                          (eps * div * d.inv_2h + w * (p * p - 1.0) * p / eps);
        r += Abar * dA;
    }
    phibar[n.c] += r;
}

}  // namespace

void launch_adj_advect(hipStream_t s, const Dims& d, const double* a, const double* phi,
                       const double* const psi[3], double dt, double mobility, double vz_lo,
                       double vz_hi, double* phibar, double* mubar, double* const psibar[3],
                       double* part, double* scal) {
    const SlabGrid g = slab_grid(d.ny * d.nz, d.nx, kMaxPartialBlocks);
    const Vel vel{psi[0], psi[1], psi[2], vz_lo, vz_hi};
    const int nb = g.gx * g.gi;
    launch_kernel(k_adj_advect, dim3(nb), dim3(kBlock), 0, s, a, phi, vel, d, dt, mobility, g,
                  phibar, mubar, psibar[0], psibar[1], psibar[2], part);
    launch_kernel(k_adj_sum, dim3(1), dim3(1024), 0, s, (const double*)part, nb, 3, scal,
                  (int)SC_ADJ_SUM_A);
}

void launch_adj_wall_couple(hipStream_t s, const Dims& d, double* const u[3],
                            double* const wall[3], double* part, double* scal, int slot) {
    const int nb = (3 * d.nx * d.nz + kBlock - 1) / kBlock;
    launch_kernel(k_adj_wall_couple, dim3(nb), dim3(kBlock), 0, s, u[0], u[1], u[2], wall[0],
                  wall[1], wall[2], d, part);
    launch_kernel(k_adj_sum, dim3(1), dim3(1024), 0, s, (const double*)part, nb, 1, scal, slot);
}

void launch_adj_source(hipStream_t s, const Dims& d, const double* phi, const double* mu,
                       double* const sbar[3], double inv_eta, double* phibar, double* mubar) {
    launch_kernel(k_adj_source, plane_grid(d), dim3(kBlock), 0, s, phi, mu, sbar[0], sbar[1],
                  sbar[2], d, inv_eta, phibar, mubar);
}

void launch_adj_mu1(hipStream_t s, const Dims& d, const double* phi, const double* mubar,
                    double C_b, double dCb_dkappa, double eps, double* gbar, double* part,
                    double* scal) {
    const SlabGrid g = slab_grid(d.ny * d.nz, d.nx, kMaxPartialBlocks);
    const int nb = g.gx * g.gi;
    launch_kernel(k_adj_mu1, dim3(nb), dim3(kBlock), 0, s, phi, mubar, d, C_b, dCb_dkappa, eps,
                  g, gbar, part);
    launch_kernel(k_adj_sum, dim3(1), dim3(1024), 0, s, (const double*)part, nb, 2, scal,
                  (int)SC_ADJ_KAPPA);
}

void launch_adj_mu2(hipStream_t s, const Dims& d, const double* phi, const double* mubar,
                    const double* gbar, const double* scal, int model, double C_b, double eps,
                    double sigma, double dt, double mobility, double rate_V, double k_A,
                    double* phibar) {
    launch_kernel(k_adj_mu2, plane_grid(d), dim3(kBlock), 0, s, phi, mubar, gbar, scal, d, model,
                  C_b, eps, sigma, dt, mobility, rate_V, k_A, phibar);
}

}  // namespace vs
