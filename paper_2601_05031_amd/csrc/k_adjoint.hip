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
#include "flow_check.h"
#include "stencil.h"

namespace vs {

namespace {

// Block layout of the tiled reverse kernels (see adj_tile_block).
struct AdjTile {
    int tj;      // rows per tile: max(1, 512 / nz), at most ny
    int ci;      // x-planes per slab
    int ntile;   // tiles per plane
    int nslab;   // slabs
};
// Block-partial slots of the reverse kernels: the wall couplings above the flow residual's
// twelve (which the source kernel's block 0 may still be reading), kappa and gamma_A below.
constexpr int kAdjSlotPsi = 12;
constexpr int kAdjSlotOm = 13;
constexpr int kAdjSlotKappa = 2;
constexpr int kAdjSlotGamma = 3;
constexpr int kAdjSlotAdv = 14;   // three slots: sum a, the wall-speed term, psibar . psi on the walls
static_assert(kAdjSlotAdv + 3 <= kPartialSlots, "partial slots");
static_assert(SC_ADJ_WALLV == SC_ADJ_SUM_A + 1 && SC_ADJ_PSIW == SC_ADJ_SUM_A + 2,
              "the advection sums map onto consecutive scalars");
// Work of block 0 of the source kernel before its tile: the sums of the advection kernel's
// partials (into SC_ADJ_SUM_A .. SC_ADJ_PSIW) and, if part is given, the check of the two
// adjoint solves from their residual partials.
struct AdjCheck {
    const double* part;   // residual partials of the two adjoint solves, or NULL: no check
    int nblocks;
    double rtol;
    double* scal;
    int* istat;
    const double* adv;    // partials of k_adj_advect (slots kAdjSlotAdv ..)
    int adv_nb;
};
inline AdjTile adj_tile(const Dims& d) {
    AdjTile t;
    t.tj = d.nz >= 512 ? 1 : 512 / d.nz;
    if (t.tj > d.ny) t.tj = d.ny;
    t.ntile = (d.ny + t.tj - 1) / t.tj;
    // slabs of four planes, longer where the block partials would not fit
    t.ci = 4;
    while (t.ntile * ((d.nx + t.ci - 1) / t.ci) > kMaxPartialBlocks && t.ci < d.nx) ++t.ci;
    t.nslab = (d.nx + t.ci - 1) / t.ci;
    return t;
}

// Tiles of the reverse node kernels: a block of kBlock lanes owns tj consecutive rows (all z)
// of an x-slab of ci planes and walks the slab. Per plane, every quantity a node's outputs take
// from its y and z neighbours is computed once per node of the tile and of its two halo rows and
// exchanged through LDS; the x neighbours' come from registers kept from plane to plane. A lane
// owns at most kAdjOwn nodes of the tile (tj nz <= kAdjOwn kBlock) and kAdjHalo halo nodes.
constexpr int kAdjOwn = 2;
constexpr int kAdjHalo = 4;

__device__ __forceinline__ void adj_tile_block(const Dims& d, const AdjTile& tl, int& j0, int& tjr,
                                               int& i0, int& i1) {
    const int nb = tl.ntile * tl.nslab;
    const int lb = xcd_block(blockIdx.x, nb);
    const int slab = lb / tl.ntile;
    const int tile = lb - slab * tl.ntile;
    j0 = tile * tl.tj;
    tjr = min(tl.tj, d.ny - j0);
    i0 = slab * tl.ci;
    i1 = min(d.nx, i0 + tl.ci);
}

// Reverse of phi' = phi + dt [M (L_h mu + lambda_V) - v . D phi] with respect to phi (through
// D phi), mu, lambda_V and psi (through v = curl psi), and the wall speed, on the tiles above.
// Per node: a, A = a v (v = curl psi on the interior rows, (0, 0, wall speed) on the walls) and
// b = -dt a D phi (0 on the walls); the outputs are phibar = a - dt sum_c D_c^T A_c,
// mubar = dt M L_h^T a and psibar = curl^T b. A lane keeps a, A_x, b_y, b_z of its nodes in
// the planes i - 1, i, i + 1 (the next plane's computed one step ahead); a, A_y, A_z, b_x, b_y,
// b_z of the plane i go through LDS. Two pieces of set-up of the reverse step ride along: the
// lanes of the wall rows zero those rows of up to six other fields (the spectral sets the
// adjoint solves write only inside), and block 0 clears the status words and residual scalars.
struct AdjZero {
    double* p[6];
};
__global__ __launch_bounds__(kBlock) void k_adj_advect(
    const double* __restrict__ a, const double* __restrict__ phi, Vel vel, Dims d, double dt,
    double mob, AdjTile tl, double* __restrict__ phibar, double* __restrict__ mubar,
    double* __restrict__ qx, double* __restrict__ qy, double* __restrict__ qz,
    double* __restrict__ partials, AdjZero zw, double* scal, int* istat) {
    extern __shared__ double lds[];
    __shared__ double sh[3 * 16];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[SC_RELRES_MAX] = 0.0;
        scal[SC_RELRES_LAST] = 0.0;
        istat[IS_FLAGS] = 0;
        istat[IS_CYCLES] = 0;
        istat[IS_CONV] = 0;
    }
    const int nz = d.nz;
    const size_t plane = (size_t)d.ny * nz;
    const double r2h = d.inv_2h;
    int j0, tjr, i0, i1;
    adj_tile_block(d, tl, j0, tjr, i0, i1);
    const int R = tl.tj + 2;   // LDS rows: halo, tile rows, halo
    double* sa = lds;
    double* say = sa + R * nz;
    double* sbx = say + R * nz;
    double* sbz = sbx + R * nz;
    double* saz = sbz + R * nz;
    double* sby = saz + R * nz;
    // own nodes
    bool ok[kAdjOwn];
    int oj[kAdjOwn], ok_[kAdjOwn], orow[kAdjOwn];
    double am[kAdjOwn], axm[kAdjOwn], bym[kAdjOwn], bzm[kAdjOwn];
    double a0[kAdjOwn], ax0[kAdjOwn], by0[kAdjOwn], bz0[kAdjOwn];
#pragma unroll
    for (int m = 0; m < kAdjOwn; ++m) {
        const int idx = threadIdx.x + m * kBlock;
        ok[m] = idx < tjr * nz;
        const int r = ok[m] ? idx / nz : 0;
        oj[m] = j0 + r;
        ok_[m] = ok[m] ? idx - r * nz : 0;
        orow[m] = r + 1;
    }
    // a, a v_x, b_y, b_z at node (j, k) of the plane base b
    auto xsub = [&](size_t b, int j, int k, double& av, double& ax, double& by, double& bz) {
        const int o = j * nz + k;
        av = a[b + o];
        ax = by = bz = 0.0;
        if (j >= 1 && j <= d.ny - 2) {
            const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
            const int okp = j * nz + kp, okm = j * nz + km;
            const double vx = ((vel.pz[b + o + nz] - vel.pz[b + o - nz]) - (vel.py[b + okp] - vel.py[b + okm])) * r2h;
            ax = av * vx;
            by = -dt * av * ((phi[b + o + nz] - phi[b + o - nz]) * r2h);
            bz = -dt * av * ((phi[b + okp] - phi[b + okm]) * r2h);
        }
    };
    double acc[3] = {0.0, 0.0, 0.0};
    if (i0 < i1) {
#pragma unroll
        for (int m = 0; m < kAdjOwn; ++m) {
            am[m] = axm[m] = bym[m] = bzm[m] = a0[m] = ax0[m] = by0[m] = bz0[m] = 0.0;
            if (!ok[m]) continue;
            xsub((size_t)wrap(i0 - 1, d.nx) * plane, oj[m], ok_[m], am[m], axm[m], bym[m], bzm[m]);
            xsub((size_t)i0 * plane, oj[m], ok_[m], a0[m], ax0[m], by0[m], bz0[m]);
        }
    }
    for (int i = i0; i < i1; ++i) {
        const int ip = (i + 1 == d.nx) ? 0 : i + 1, im = (i == 0) ? d.nx - 1 : i - 1;
        const size_t b = (size_t)i * plane, bm = (size_t)im * plane, bp = (size_t)ip * plane;
        double ap[kAdjOwn], axp[kAdjOwn], byp[kAdjOwn], bzp[kAdjOwn];
        // the next plane's x quantities, then the rest of this plane's into LDS
#pragma unroll
        for (int m = 0; m < kAdjOwn; ++m) {
            ap[m] = axp[m] = byp[m] = bzp[m] = 0.0;
            if (!ok[m]) continue;
            xsub(bp, oj[m], ok_[m], ap[m], axp[m], byp[m], bzp[m]);
            const int j = oj[m], k = ok_[m], o = j * nz + k;
            const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
            double Ay = 0.0, Az, bx = 0.0;
            if (j >= 1 && j <= d.ny - 2) {
                const double vy = ((vel.px[b + j * nz + kp] - vel.px[b + j * nz + km]) - (vel.pz[bp + o] - vel.pz[bm + o])) * r2h;
                const double vz = ((vel.py[bp + o] - vel.py[bm + o]) - (vel.px[b + o + nz] - vel.px[b + o - nz])) * r2h;
                Ay = a0[m] * vy;
                Az = a0[m] * vz;
                bx = -dt * a0[m] * ((phi[bp + o] - phi[bm + o]) * r2h);
            } else {
                Az = a0[m] * (j == 0 ? vel.vz_lo : vel.vz_hi);
            }
            const int q = orow[m] * nz + k;
            sa[q] = a0[m];
            say[q] = Ay;
            sbx[q] = bx;
            sbz[q] = bz0[m];
            saz[q] = Az;
            sby[q] = by0[m];
        }
        // halo rows j0 - 1 and j0 + tjr: a, A_y, b_x, b_z
#pragma unroll 1
        for (int h = 0; h < kAdjHalo; ++h) {
            const int idx = threadIdx.x + h * kBlock;
            if (idx >= 2 * nz) continue;
            const int side = idx / nz, k = idx - side * nz;
            const int j = side ? j0 + tjr : j0 - 1;
            if (j < 0 || j >= d.ny) continue;
            const int o = j * nz + k;
            const double av = a[b + o];
            double Ay = 0.0, bx = 0.0, bz = 0.0;
            if (j >= 1 && j <= d.ny - 2) {
                const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
                const double vy = ((vel.px[b + j * nz + kp] - vel.px[b + j * nz + km]) - (vel.pz[bp + o] - vel.pz[bm + o])) * r2h;
                Ay = av * vy;
                bx = -dt * av * ((phi[bp + o] - phi[bm + o]) * r2h);
                bz = -dt * av * ((phi[b + j * nz + kp] - phi[b + j * nz + km]) * r2h);
            }
            const int q = (side ? tjr + 1 : 0) * nz + k;
            sa[q] = av;
            say[q] = Ay;
            sbx[q] = bx;
            sbz[q] = bz;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kAdjOwn; ++m) {
            if (!ok[m]) continue;
            const int j = oj[m], k = ok_[m];
            const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
            const int rr = orow[m];
            const int qc = rr * nz + k, qkm = rr * nz + km, qkp = rr * nz + kp;
            const int qjm = qc - nz, qjp = qc + nz;   // rows j - 1, j + 1 (valid where they exist)
            const bool has_m = j >= 1, has_p = j <= d.ny - 2;
            const bool wall = (j == 0 || j == d.ny - 1);
            // phibar = a - dt sum_c D_c^T (a v_c)
            double t = (axm[m] - axp[m]) + (saz[qkm] - saz[qkp]);
            if (has_m) t += say[qjm];
            if (has_p) t -= say[qjp];
            const size_t c = b + (size_t)j * nz + k;
            phibar[c] = a0[m] - dt * t * r2h;
            // mubar = dt M L_h^T a (mirrored rows past the walls)
            const int jm_l = (j == 0) ? 1 : j - 1, jp_l = (j == d.ny - 1) ? d.ny - 2 : j + 1;
            const double xz = ap[m] + am[m] + sa[qkp] + sa[qkm];
            const double yy = sa[qc + (jp_l - j) * nz] / wrow(d, jp_l) + sa[qc + (jm_l - j) * nz] / wrow(d, jm_l);
            mubar[c] = dt * mob * ((xz + wrow(d, j) * yy - 6.0 * a0[m]) * d.inv_h2);
            // psibar = curl^T b
            const double bzjm = has_m ? sbz[qjm] : 0.0, bzjp = has_p ? sbz[qjp] : 0.0;
            const double bxjm = has_m ? sbx[qjm] : 0.0, bxjp = has_p ? sbx[qjp] : 0.0;
            const double sx = ((sby[qkm] - sby[qkp]) - (bzjm - bzjp)) * r2h;
            const double sy = ((bzm[m] - bzp[m]) - (sbx[qkm] - sbx[qkp])) * r2h;
            const double sz = ((bxjm - bxjp) - (bym[m] - byp[m])) * r2h;
            qx[c] = sx;
            qy[c] = sy;
            qz[c] = sz;
            acc[0] += a0[m];
            if (wall) {
                const double dz = (phi[b + (size_t)j * nz + kp] - phi[b + (size_t)j * nz + km]) * r2h;
                acc[1] += a0[m] * (j == 0 ? vel.vz_lo : vel.vz_hi) * dz;
                acc[2] += sx * vel.px[c] + sy * vel.py[c] + sz * vel.pz[c];
                if (zw.p[0]) {
#pragma unroll
                    for (int f = 0; f < 6; ++f)
                        if (zw.p[f]) zw.p[f][c] = 0.0;
                }
            }
            am[m] = a0[m]; axm[m] = ax0[m]; bym[m] = by0[m]; bzm[m] = bz0[m];
            a0[m] = ap[m]; ax0[m] = axp[m]; by0[m] = byp[m]; bz0[m] = bzp[m];
        }
        __syncthreads();
    }
    block_sum<3>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) partials[(kAdjSlotAdv + q) * kMaxPartialBlocks + blockIdx.x] = acc[q];
    }
}

// scal[dst + q] = sum_b partials[q][b] for q in [first, nslots), fixed order; slots below
// split have nb_lo blocks, the others nb_hi.
__global__ __launch_bounds__(1024) void k_adj_sum(const double* __restrict__ partials, int nb_lo,
                                                  int nb_hi, int split, int first, int nslots,
                                                  double* scal, int dst) {
    __shared__ double sh[4 * 16];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int nbmax = nb_lo > nb_hi ? nb_lo : nb_hi;
    for (int b = threadIdx.x; b < nbmax; b += blockDim.x)
        for (int q = first; q < nslots; ++q)
            if (b < (q < split ? nb_lo : nb_hi)) acc[q] += partials[q * kMaxPartialBlocks + b];
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
// bbar = (1/eta) Sbar x D phi at each interior node, 0 on the walls (so the wall rows receive
// the y terms of rows 1 and M). On the tiles of k_adj_advect: a lane keeps the x components of
// abar, bbar of its nodes in the planes i - 1 and i + 1 (with the y and z differences and Sbar
// of the next plane, computed one step ahead); the y and z components of the plane i go
// through LDS. The wall couplings of the two adjoint solves ride along as block partials
// (slot kAdjSlotPsi: u1 on rows 1 and M against the psi walls, skipped when u1 is NULL; slot
// kAdjSlotOm: Sbar against the omega walls), and, when chk.part is given, block 0 first takes
// the convergence check of the two adjoint solves from their residual partials (as
// k_check_flow does; the slots of this kernel lie above the residual's).
__global__ __launch_bounds__(kBlock) void k_adj_source(
    const double* __restrict__ phi, const double* __restrict__ mu, const double* __restrict__ s0,
    const double* __restrict__ s1, const double* __restrict__ s2, Dims d, double inv_eta,
    AdjTile tl, double* __restrict__ phibar, double* __restrict__ mubar, WallPairs wp,
    double* __restrict__ partials, AdjCheck chk) {
    extern __shared__ double lds[];
    __shared__ double sh[4 * 16];
    if (blockIdx.x == 0) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int b = threadIdx.x; b < chk.adv_nb; b += blockDim.x) {
#pragma unroll
            for (int q = 0; q < 3; ++q) v[q] += chk.adv[(kAdjSlotAdv + q) * kMaxPartialBlocks + b];
        }
        block_sum<3>(v, sh);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 0; q < 3; ++q) chk.scal[SC_ADJ_SUM_A + q] = v[q];
        }
        __syncthreads();
        if (chk.part) flow_check_block(chk.part, chk.nblocks, chk.rtol, chk.scal, chk.istat, sh, 1);
    }
    const int nz = d.nz;
    const size_t plane = (size_t)d.ny * nz;
    const double r2h = d.inv_2h;
    int j0, tjr, i0, i1;
    adj_tile_block(d, tl, j0, tjr, i0, i1);
    const int R = tl.tj + 2;
    double* sab_y = lds;
    double* sbb_y = sab_y + R * nz;
    double* sab_z = sbb_y + R * nz;
    double* sbb_z = sab_z + R * nz;
    bool ok[kAdjOwn], in[kAdjOwn];
    int oj[kAdjOwn], ok_[kAdjOwn], orow[kAdjOwn];
#pragma unroll
    for (int m = 0; m < kAdjOwn; ++m) {
        const int idx = threadIdx.x + m * kBlock;
        ok[m] = idx < tjr * nz;
        const int r = ok[m] ? idx / nz : 0;
        oj[m] = j0 + r;
        ok_[m] = ok[m] ? idx - r * nz : 0;
        orow[m] = r + 1;
        in[m] = ok[m] && oj[m] >= 1 && oj[m] <= d.ny - 2;
    }
    // y, z differences of phi and mu and Sbar_1, Sbar_2 at (j, k) of the plane base b (interior)
    struct Yz {
        double f1, f2, m1, m2, S1, S2;
    };
    auto yz = [&](size_t b, int j, int k) -> Yz {
        const int o = j * nz + k;
        const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
        Yz r;
        r.f1 = (phi[b + o + nz] - phi[b + o - nz]) * r2h;
        r.f2 = (phi[b + j * nz + kp] - phi[b + j * nz + km]) * r2h;
        r.m1 = (mu[b + o + nz] - mu[b + o - nz]) * r2h;
        r.m2 = (mu[b + j * nz + kp] - mu[b + j * nz + km]) * r2h;
        r.S1 = s1[b + o];
        r.S2 = s2[b + o];
        return r;
    };
    double abm[kAdjOwn], bbm[kAdjOwn], ab0[kAdjOwn], bb0[kAdjOwn];
    Yz y0[kAdjOwn];
    double acc[2] = {0.0, 0.0};
    if (i0 < i1) {
#pragma unroll
        for (int m = 0; m < kAdjOwn; ++m) {
            abm[m] = bbm[m] = ab0[m] = bb0[m] = 0.0;
            y0[m] = Yz{0, 0, 0, 0, 0, 0};
            if (!in[m]) continue;
            const Yz t = yz((size_t)wrap(i0 - 1, d.nx) * plane, oj[m], ok_[m]);
            abm[m] = (t.m1 * t.S2 - t.m2 * t.S1) * inv_eta;
            bbm[m] = (t.S1 * t.f2 - t.S2 * t.f1) * inv_eta;
            y0[m] = yz((size_t)i0 * plane, oj[m], ok_[m]);
            ab0[m] = (y0[m].m1 * y0[m].S2 - y0[m].m2 * y0[m].S1) * inv_eta;
            bb0[m] = (y0[m].S1 * y0[m].f2 - y0[m].S2 * y0[m].f1) * inv_eta;
        }
    }
    for (int i = i0; i < i1; ++i) {
        const int ip = (i + 1 == d.nx) ? 0 : i + 1, im = (i == 0) ? d.nx - 1 : i - 1;
        const size_t b = (size_t)i * plane, bm = (size_t)im * plane, bp = (size_t)ip * plane;
        double abp[kAdjOwn], bbp[kAdjOwn];
        Yz yp[kAdjOwn];
#pragma unroll
        for (int m = 0; m < kAdjOwn; ++m) {
            abp[m] = bbp[m] = 0.0;
            yp[m] = Yz{0, 0, 0, 0, 0, 0};
            if (!ok[m]) continue;
            double aby = 0.0, bby = 0.0, abz = 0.0, bbz = 0.0;
            if (in[m]) {
                yp[m] = yz(bp, oj[m], ok_[m]);
                abp[m] = (yp[m].m1 * yp[m].S2 - yp[m].m2 * yp[m].S1) * inv_eta;
                bbp[m] = (yp[m].S1 * yp[m].f2 - yp[m].S2 * yp[m].f1) * inv_eta;
                const int o = oj[m] * nz + ok_[m];
                const double f0 = (phi[bp + o] - phi[bm + o]) * r2h;
                const double m0 = (mu[bp + o] - mu[bm + o]) * r2h;
                const double S0 = s0[b + o];
                const Yz& t = y0[m];
                aby = (t.m2 * S0 - m0 * t.S2) * inv_eta;
                bby = (t.S2 * f0 - S0 * t.f2) * inv_eta;
                abz = (m0 * t.S1 - t.m1 * S0) * inv_eta;
                bbz = (S0 * t.f1 - t.S1 * f0) * inv_eta;
            }
            const int q = orow[m] * nz + ok_[m];
            sab_y[q] = aby;
            sbb_y[q] = bby;
            sab_z[q] = abz;
            sbb_z[q] = bbz;
        }
        // halo rows j0 - 1 and j0 + tjr: abar_y, bbar_y
#pragma unroll 1
        for (int h = 0; h < kAdjHalo; ++h) {
            const int idx = threadIdx.x + h * kBlock;
            if (idx >= 2 * nz) continue;
            const int side = idx / nz, k = idx - side * nz;
            const int j = side ? j0 + tjr : j0 - 1;
            if (j < 0 || j >= d.ny) continue;
            double aby = 0.0, bby = 0.0;
            if (j >= 1 && j <= d.ny - 2) {
                const int o = j * nz + k;
                const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
                const double f0 = (phi[bp + o] - phi[bm + o]) * r2h;
                const double m0 = (mu[bp + o] - mu[bm + o]) * r2h;
                const double f2 = (phi[b + j * nz + kp] - phi[b + j * nz + km]) * r2h;
                const double m2 = (mu[b + j * nz + kp] - mu[b + j * nz + km]) * r2h;
                const double S0 = s0[b + o], S2 = s2[b + o];
                aby = (m2 * S0 - m0 * S2) * inv_eta;
                bby = (S2 * f0 - S0 * f2) * inv_eta;
            }
            const int q = (side ? tjr + 1 : 0) * nz + k;
            sab_y[q] = aby;
            sbb_y[q] = bby;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kAdjOwn; ++m) {
            if (!ok[m]) continue;
            const int j = oj[m], k = ok_[m];
            const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
            const int rr = orow[m];
            const int qc = rr * nz + k, qkm = rr * nz + km, qkp = rr * nz + kp;
            const double abjm = j >= 1 ? sab_y[qc - nz] : 0.0, abjp = j <= d.ny - 2 ? sab_y[qc + nz] : 0.0;
            const double bbjm = j >= 1 ? sbb_y[qc - nz] : 0.0, bbjp = j <= d.ny - 2 ? sbb_y[qc + nz] : 0.0;
            const double tp = ((abm[m] - abp[m]) + (sab_z[qkm] - sab_z[qkp])) + (abjm - abjp);
            const double tm = ((bbm[m] - bbp[m]) + (sbb_z[qkm] - sbb_z[qkp])) + (bbjm - bbjp);
            const size_t c = b + (size_t)j * nz + k;
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
            abm[m] = ab0[m]; bbm[m] = bb0[m];
            ab0[m] = abp[m]; bb0[m] = bbp[m];
            y0[m] = yp[m];
        }
        __syncthreads();
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        partials[kAdjSlotPsi * kMaxPartialBlocks + blockIdx.x] = acc[0];
        partials[kAdjSlotOm * kMaxPartialBlocks + blockIdx.x] = acc[1];
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
        partials[kAdjSlotKappa * kMaxPartialBlocks + blockIdx.x] = acc[0];
        partials[kAdjSlotGamma * kMaxPartialBlocks + blockIdx.x] = acc[1];
    }
}

// phibar += (d mu / d phi)^T mubar + lambda_bar d lambda_V/d phi + A_bar dA/d phi. Each lane
// owns one (j, k) column and walks an x-slab with phi of the planes i-2 .. i+2 and mubar, gbar
// of the planes i-1 .. i+1 in registers.
// Sums of the reverse step's block partials (fixed order, the same in every block): nb_src
// blocks of k_adj_source, nb_mu1 of k_adj_mu1 (0: not launched).
struct AdjSums {
    const double* part;
    int nb_src, nb_mu1;
    int psi_on;       // the psi-wall coupling came from k_adj_source (else it is in scal already)
    double* scal;     // block 0 writes SC_ADJ_PSIC, SC_ADJ_OMC, SC_ADJ_KAPPA, SC_ADJ_GAMMA
};
__global__ __launch_bounds__(kBlock) void k_adj_mu2(const double* __restrict__ phi,
                                                   const double* __restrict__ mubar,
                                                   const double* __restrict__ gbar,
                                                   const double* __restrict__ scal, Dims d,
                                                   int model, double C_b, double eps, double sigma,
                                                   double dt, double mob, double rate_V, double k_A,
                                                   SlabGrid sg, double* __restrict__ phibar,
                                                   AdjSums sums) {
    // gamma_A's adjoint (needed by every block; a device-wide fence to let one block gather it
    // costs more here) and, in block 0, the step's other scalars
    __shared__ double sh[4 * 16];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const bool b0 = blockIdx.x == 0;
    for (int b = threadIdx.x; b < sums.nb_mu1; b += blockDim.x) {
        v[0] += sums.part[kAdjSlotGamma * kMaxPartialBlocks + b];
        if (b0) v[1] += sums.part[kAdjSlotKappa * kMaxPartialBlocks + b];
    }
    if (b0) {
        for (int b = threadIdx.x; b < sums.nb_src; b += blockDim.x) {
            if (sums.psi_on) v[2] += sums.part[kAdjSlotPsi * kMaxPartialBlocks + b];
            v[3] += sums.part[kAdjSlotOm * kMaxPartialBlocks + b];
        }
    }
    block_sum<4>(v, sh);
    if (threadIdx.x == 0) sh[4 * 16 - 1] = v[0];
    __syncthreads();
    const double gamma_bar = sh[4 * 16 - 1];
    if (b0 && threadIdx.x == 0) {
        sums.scal[SC_ADJ_GAMMA] = v[0];
        sums.scal[SC_ADJ_KAPPA] = v[1];
        if (sums.psi_on) sums.scal[SC_ADJ_PSIC] = v[2];
        sums.scal[SC_ADJ_OMC] = v[3];
    }
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
    const double Abar = area ? gamma_bar * k_A / A0 : 0.0;
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
    const AdjTile tl = adj_tile(d);
    const Vel vel{psi[0], psi[1], psi[2], vz_lo, vz_hi};
    const int nb = tl.ntile * tl.nslab;
    AdjZero zw{};
    for (int f = 0; f < 6; ++f) zw.p[f] = zero_walls ? zero_walls[f] : nullptr;
    const size_t lds = (size_t)6 * (tl.tj + 2) * d.nz * sizeof(double);
    launch_kernel(k_adj_advect, dim3(nb), dim3(kBlock), lds, s, a, phi, vel, d, dt, mobility, tl,
                  phibar, mubar, psibar[0], psibar[1], psibar[2], part, zw, scal, istat);
}

void launch_adj_wall_couple(hipStream_t s, const Dims& d, double* const u[3],
                            double* const wall[3], double* part, double* scal, int slot) {
    const int nb = (3 * d.nx * d.nz + kBlock - 1) / kBlock;
    launch_kernel(k_adj_wall_couple, dim3(nb), dim3(kBlock), 0, s, u[0], u[1], u[2], wall[0],
                  wall[1], wall[2], d, part);
    launch_kernel(k_adj_sum, dim3(1), dim3(1024), 0, s, (const double*)part, nb, nb, 0, 0, 1, scal, slot);
}

void launch_adj_source(hipStream_t s, const Dims& d, const double* phi, const double* mu,
                       double* const sbar[3], double inv_eta, double* phibar, double* mubar,
                       const double* const u1[3], const double* const psi_walls[3],
                       const double* const om_walls[3], double* part, const double* chk_part,
                       double rtol, double* scal, int* istat) {
    const AdjTile tl = adj_tile(d);
    AdjCheck chk{};
    if (chk_part) chk = AdjCheck{chk_part, resid_flow_blocks(d), rtol, scal, istat, nullptr, 0};
    chk.scal = scal;
    chk.adv = part;
    chk.adv_nb = tl.ntile * tl.nslab;   // the advection kernel's tiles are the same
    WallPairs wp{};
    for (int c = 0; c < 3; ++c) {
        wp.u[c] = u1 ? u1[c] : nullptr;
        wp.uw[c] = psi_walls[c];
        wp.sw[c] = om_walls[c];
    }
    const size_t lds = (size_t)4 * (tl.tj + 2) * d.nz * sizeof(double);
    launch_kernel(k_adj_source, dim3(tl.ntile * tl.nslab), dim3(kBlock), lds, s, phi, mu,
                  (const double*)sbar[0], (const double*)sbar[1], (const double*)sbar[2], d, inv_eta,
                  tl, phibar, mubar, wp, part, chk);
}

void launch_adj_mu1(hipStream_t s, const Dims& d, const double* phi, const double* mubar,
                    double C_b, double dCb_dkappa, double eps, double* gbar, double* part) {
    const SlabGrid g = adj_slab_grid(d);
    launch_kernel(k_adj_mu1, dim3(g.gx * g.gi), dim3(kBlock), 0, s, phi, mubar, d, C_b, dCb_dkappa,
                  eps, g, gbar, part);
}

void launch_adj_mu2(hipStream_t s, const Dims& d, const double* phi, const double* mubar,
                    const double* gbar, const double* scal, int model, double C_b, double eps,
                    double sigma, double dt, double mobility, double rate_V, double k_A,
                    double* phibar, double* part, bool mu1_ran, bool psi_from_source,
                    double* scal_out) {
    const AdjTile tl = adj_tile(d);
    const SlabGrid g1 = adj_slab_grid(d);
    const AdjSums sums{part, tl.ntile * tl.nslab, mu1_ran ? g1.gx * g1.gi : 0, psi_from_source ? 1 : 0,
                       scal_out};
    const SlabGrid g = adj_slab_grid(d);
    launch_kernel(k_adj_mu2, dim3(g.gx * g.gi), dim3(kBlock), 0, s, phi, mubar, gbar, scal, d, model,
                  C_b, eps, sigma, dt, mobility, rate_V, k_A, g, phibar, sums);
}

}  // namespace vs
