// Diagnostics of a state and the wall-speed change, FP64, gfx950.
//   * in-plane shear stress (main text "In plane shear"): sigma_ij = eta (d_j v_i + d_i v_j),
//     sigma_t = sqrt(sigma_xy^2 + sigma_yz^2 + sigma_xz^2), central differences of v (curl psi
//     inside, the wall speed on the walls), on the interior rows; 0 on the wall rows;
//   * the flow observables of the results section: int |omega - omega_0|^2 and
//     int |psi - psi_0|^2 about the no-body channel fields, trapezoid weights in y;
//   * the free-energy density: g^2 (bending, SM eq. (30) without the area term) or
//     1/4 (phi^2 - 1)^2 + (sigma/2) |D phi|^2 (Cahn-Hilliard, eq. F_CH);
//   * the gauge defect (D . psi)^2 on the interior rows (the Coulomb gauge is assumed, not
//     imposed) and the largest speed |v|;
//   * time-dependent walls (SM "Time-dependency and inertial flow"): the Poisson problems
//     are linear in the wall data and the no-body fields (polynomials of degree <= 3 in y)
//     solve them exactly, so a change of wall speeds adds the difference of the no-body fields
//     to omega_x and psi_x.
#include "stencil.h"

namespace vs {

namespace {

// The velocity on every node into three scratch fields (curl psi inside, the wall velocity on
// the walls), so that the shear stress reads each neighbour's velocity once instead of
// evaluating the curl there again.
__global__ __launch_bounds__(kBlock) void k_diag_vel(Vel vel, Dims d, double* __restrict__ v0,
                                                    double* __restrict__ v1,
                                                    double* __restrict__ v2) {
    int i, j, k;
    bool ok;
    plane_index(d, i, j, k, ok);
    if (!ok) return;
    const int c = node(d, i, j, k);
    v0[c] = vx_at(vel, d, i, j, k);
    v1[c] = vy_at(vel, d, i, j, k);
    v2[c] = vz_at(vel, d, i, j, k);
}

__global__ __launch_bounds__(kBlock) void k_diag(const double* __restrict__ phi,
                                                const double* __restrict__ o0,
                                                const double* __restrict__ o1,
                                                const double* __restrict__ o2, Vel vel,
                                                const double* __restrict__ V0,
                                                const double* __restrict__ V1,
                                                const double* __restrict__ V2,
                                                const double* __restrict__ prof, Dims d, double eta,
                                                int model, double eps, double sigma, SlabGrid sg,
                                                double* __restrict__ sigma_t,
                                                double* __restrict__ partials) {
    __shared__ double sh[4 * 16];
    __shared__ double shm[2 * 16];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double smax = 0.0, vmax = 0.0;
    const SlabIter it = slab_iter(d, sg);
    if (it.ok) {
        const int j = it.j, k = it.k;
        const double w = wrow(d, j);
        const double pw = prof[j], ow = prof[d.ny + j];
        const int kp = wrap(k + 1, d.nz), km = wrap(k - 1, d.nz);
        const double eps2 = eps * eps;
        for (int i = it.i0; i < it.i1; ++i) {
            const Nbr n = neighbours_mirror(d, i, j, k);
            const double a0 = o0[n.c] - ow, a1 = o1[n.c], a2 = o2[n.c];
            const double b0 = vel.px[n.c] - pw, b1 = vel.py[n.c], b2 = vel.pz[n.c];
            acc[0] += w * (a0 * a0 + a1 * a1 + a2 * a2);
            acc[1] += w * (b0 * b0 + b1 * b1 + b2 * b2);
            const double p = phi[n.c];
            if (model == VS_CAHN_HILLIARD) {
                const double dx = (phi[n.xp] - phi[n.xm]) * d.inv_2h;
                const double dy = (phi[n.yp] - phi[n.ym]) * d.inv_2h;
                const double dz = (phi[n.zp] - phi[n.zm]) * d.inv_2h;
                const double q = p * p - 1.0;
                acc[2] += w * (0.25 * q * q + 0.5 * sigma * (dx * dx + dy * dy + dz * dz));
            } else {
                const double g = p * p * p - p - eps2 * lap7(phi, n, d.inv_h2);
                acc[2] += w * g * g;
            }
            double st = 0.0;
            {
                const double vx = V0[n.c], vy = V1[n.c], vz = V2[n.c];
                vmax = fmax(vmax, sqrt(vx * vx + vy * vy + vz * vz));
            }
            if (interior(d, j)) {
                const int ip = wrap(i + 1, d.nx), im = wrap(i - 1, d.nx);
                const double dv = (vel.px[node(d, ip, j, k)] - vel.px[node(d, im, j, k)]) * d.inv_2h +
                                  (vel.py[node(d, i, j + 1, k)] - vel.py[node(d, i, j - 1, k)]) * d.inv_2h +
                                  (vel.pz[node(d, i, j, kp)] - vel.pz[node(d, i, j, km)]) * d.inv_2h;
                acc[3] += dv * dv;
                const int cjp = node(d, i, j + 1, k), cjm = node(d, i, j - 1, k);
                const int ckp = n.c - k + kp, ckm = n.c - k + km;
                const int cip = node(d, ip, j, k), cim = node(d, im, j, k);
                const double sxy = (V0[cjp] - V0[cjm]) + (V1[cip] - V1[cim]);
                const double syz = (V1[ckp] - V1[ckm]) + (V2[cjp] - V2[cjm]);
                const double sxz = (V0[ckp] - V0[ckm]) + (V2[cip] - V2[cim]);
                st = eta * d.inv_2h * sqrt(sxy * sxy + syz * syz + sxz * sxz);
            }
            if (sigma_t) sigma_t[n.c] = st;
            smax = fmax(smax, st);
        }
    }
    block_sum<4>(acc, sh);
    // block maxima, fixed order
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        smax = fmax(smax, __shfl_down(smax, off, 64));
        vmax = fmax(vmax, __shfl_down(vmax, off, 64));
    }
    if (lane == 0) {
        shm[wv] = smax;
        shm[16 + wv] = vmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0, mv = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            m = fmax(m, shm[q]);
            mv = fmax(mv, shm[16 + q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) partials[q * kMaxPartialBlocks + blockIdx.x] = acc[q];
        partials[4 * kMaxPartialBlocks + blockIdx.x] = m;
        partials[5 * kMaxPartialBlocks + blockIdx.x] = mv;
    }
}

__global__ __launch_bounds__(1024) void k_diag_finalize(const double* __restrict__ partials,
                                                       int nblocks, double* scal) {
    __shared__ double sh[4 * 16];
    __shared__ double shm[2 * 16];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double m = 0.0, mv = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += partials[q * kMaxPartialBlocks + b];
        m = fmax(m, partials[4 * kMaxPartialBlocks + b]);
        mv = fmax(mv, partials[5 * kMaxPartialBlocks + b]);
    }
    block_sum<4>(acc, sh);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        m = fmax(m, __shfl_down(m, off, 64));
        mv = fmax(mv, __shfl_down(mv, off, 64));
    }
    if (lane == 0) {
        shm[wv] = m;
        shm[16 + wv] = mv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = 0.0, mmv = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            mm = fmax(mm, shm[q]);
            mmv = fmax(mmv, shm[16 + q]);
        }
        scal[SC_DG_OMEGA] = acc[0];
        scal[SC_DG_PSI] = acc[1];
        scal[SC_DG_ENERGY] = acc[2];
        scal[SC_DG_GAUGE] = acc[3];
        scal[SC_DG_SMAX] = mm;
        scal[SC_DG_VMAX] = mmv;
    }
}

__global__ __launch_bounds__(kBlock) void k_shift_profiles(double* __restrict__ om,
                                                          double* __restrict__ ps, Dims d,
                                                          const double* __restrict__ dprof) {
    int i, j, k;
    bool ok;
    plane_index(d, i, j, k, ok);
    if (!ok) return;
    const int c = node(d, i, j, k);
    ps[c] += dprof[j];
    om[c] += dprof[d.ny + j];
}

}  // namespace

void launch_diagnostics(hipStream_t s, const Dims& d, const double* phi, double* const omega[3],
                        double* const psi[3], const double* prof, double vz_lo, double vz_hi,
                        double eta, int model, double eps, double sigma, double* sigma_t,
                        double* part, double* scal, double* const vscratch[3]) {
    const SlabGrid g = slab_grid(d.ny * d.nz, d.nx, kMaxPartialBlocks);
    const Vel vel{psi[0], psi[1], psi[2], vz_lo, vz_hi};
    const int nb = g.gx * g.gi;
    launch_kernel(k_diag_vel, plane_grid(d), dim3(kBlock), 0, s, vel, d, vscratch[0], vscratch[1],
                  vscratch[2]);
    launch_kernel(k_diag, dim3(nb), dim3(kBlock), 0, s, phi, (const double*)omega[0],
                  (const double*)omega[1], (const double*)omega[2], vel,
                  (const double*)vscratch[0], (const double*)vscratch[1],
                  (const double*)vscratch[2], prof, d, eta, model, eps, sigma, g, sigma_t, part);
    launch_kernel(k_diag_finalize, dim3(1), dim3(1024), 0, s, (const double*)part, nb, scal);
}

void launch_shift_profiles(hipStream_t s, const Dims& d, double* omega_x, double* psi_x,
                           const double* dprof) {
    launch_kernel(k_shift_profiles, plane_grid(d), dim3(kBlock), 0, s, omega_x, psi_x, d, dprof);
}

}  // namespace vs
