// Node-kernel helpers shared by the explicit and adjoint stencils (gfx950, FP64).
//
// Launch shape of the node kernels: block = 256 lanes (four 64-wide waves) over the
// contiguous (j, k) plane of one x-plane i = blockIdx.y, so a wave reads 64 consecutive z
// values; the x and y neighbours of a block are other rows of the same or adjacent blocks
// and are served by L2. Walls: mirror ghosts in y for phi, g and mu (no-flux walls).
#pragma once

#include "vs_internal.h"

namespace vs {
namespace {

constexpr int kBlock = 256;

// Node of this thread in a plane grid (blockIdx.x over the (j, k) plane, blockIdx.y = i),
// with the blocks ordered per XCD so that each XCD sweeps a contiguous range of x-planes.
__device__ __forceinline__ void plane_index(const Dims& d, int& i, int& j, int& k, bool& ok) {
    const int gx = gridDim.x;
    const int lb = xcd_block(blockIdx.x + gx * blockIdx.y, gx * gridDim.y);
    i = lb / gx;
    const int t = (lb - i * gx) * kBlock + threadIdx.x;
    ok = t < d.ny * d.nz;
    j = t / d.nz;
    k = t - j * d.nz;
}

struct Nbr {
    int c, xp, xm, yp, ym, zp, zm;
};

// Neighbour indices, periodic in x and z, mirror ghosts in y (u[-1] = u[1], u[ny] = u[ny-2]).
__device__ __forceinline__ Nbr neighbours_mirror(const Dims& d, int i, int j, int k) {
    const int ip = (i + 1 == d.nx) ? 0 : i + 1;
    const int im = (i == 0) ? d.nx - 1 : i - 1;
    const int jp = (j + 1 == d.ny) ? d.ny - 2 : j + 1;
    const int jm = (j == 0) ? 1 : j - 1;
    const int kp = (k + 1 == d.nz) ? 0 : k + 1;
    const int km = (k == 0) ? d.nz - 1 : k - 1;
    Nbr n;
    n.c = node(d, i, j, k);
    n.xp = node(d, ip, j, k);
    n.xm = node(d, im, j, k);
    n.yp = node(d, i, jp, k);
    n.ym = node(d, i, jm, k);
    n.zp = n.c - k + kp;
    n.zm = n.c - k + km;
    return n;
}

__device__ __forceinline__ double lap7(const double* __restrict__ u, const Nbr& n, double inv_h2) {
    return (u[n.xp] + u[n.xm] + u[n.yp] + u[n.ym] + u[n.zp] + u[n.zm] - 6.0 * u[n.c]) * inv_h2;
}

// g = phi^3 - phi - eps^2 L_h phi at node (i, j, k), mirror ghosts.
__device__ __forceinline__ double g_at(const double* __restrict__ phi, const Dims& d, int i, int j,
                                       int k, double eps2) {
    const Nbr n = neighbours_mirror(d, i, j, k);
    const double p = phi[n.c];
    return p * p * p - p - eps2 * lap7(phi, n, d.inv_h2);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block in a fixed order; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) sh[q * 16 + w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int i = 0; i < nw; ++i) s += sh[q * 16 + i];
            v[q] = s;
        }
    }
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Velocity components at a node: curl psi on the interior rows, the wall speed on the walls.
struct Vel {
    const double *px, *py, *pz;
    double vz_lo, vz_hi;
};

__device__ __forceinline__ double vx_at(const Vel& v, const Dims& d, int i, int j, int k) {
    if (j == 0 || j == d.ny - 1) return 0.0;
    const int kp = wrap(k + 1, d.nz), km = wrap(k - 1, d.nz);
    return ((v.pz[node(d, i, j + 1, k)] - v.pz[node(d, i, j - 1, k)]) -
            (v.py[node(d, i, j, kp)] - v.py[node(d, i, j, km)])) * d.inv_2h;
}
__device__ __forceinline__ double vy_at(const Vel& v, const Dims& d, int i, int j, int k) {
    if (j == 0 || j == d.ny - 1) return 0.0;
    const int ip = wrap(i + 1, d.nx), im = wrap(i - 1, d.nx);
    const int kp = wrap(k + 1, d.nz), km = wrap(k - 1, d.nz);
    return ((v.px[node(d, i, j, kp)] - v.px[node(d, i, j, km)]) -
            (v.pz[node(d, ip, j, k)] - v.pz[node(d, im, j, k)])) * d.inv_2h;
}
__device__ __forceinline__ double vz_at(const Vel& v, const Dims& d, int i, int j, int k) {
    if (j == 0) return v.vz_lo;
    if (j == d.ny - 1) return v.vz_hi;
    const int ip = wrap(i + 1, d.nx), im = wrap(i - 1, d.nx);
    return ((v.py[node(d, ip, j, k)] - v.py[node(d, im, j, k)]) -
            (v.px[node(d, i, j + 1, k)] - v.px[node(d, i, j - 1, k)])) * d.inv_2h;
}

__device__ __forceinline__ double wrow(const Dims& d, int j) {
    return (j == 0 || j == d.ny - 1) ? 0.5 : 1.0;
}

// (L_h^T u)_m = w_m (L_h (u / w))_m, mirror ghosts in y.
__device__ __forceinline__ double lapT(const double* __restrict__ u, const Dims& d, int i, int j,
                                       int k) {
    const int jp = (j + 1 == d.ny) ? d.ny - 2 : j + 1;
    const int jm = (j == 0) ? 1 : j - 1;
    const double xz = u[node(d, wrap(i + 1, d.nx), j, k)] + u[node(d, wrap(i - 1, d.nx), j, k)] +
                      u[node(d, i, j, wrap(k + 1, d.nz))] + u[node(d, i, j, wrap(k - 1, d.nz))];
    const double yy = u[node(d, i, jp, k)] / wrow(d, jp) + u[node(d, i, jm, k)] / wrow(d, jm);
    return (xz + wrow(d, j) * yy - 6.0 * u[node(d, i, j, k)]) * d.inv_h2;
}

// Central difference of u along axis c at an interior or any node (true neighbours in y; the
// callers use it on the rows where the forward difference is evaluated).
__device__ __forceinline__ double dcen(const double* __restrict__ u, const Dims& d, int c, int i,
                                       int j, int k) {
    if (c == 0) return (u[node(d, wrap(i + 1, d.nx), j, k)] - u[node(d, wrap(i - 1, d.nx), j, k)]) * d.inv_2h;
    if (c == 1) return (u[node(d, i, j + 1, k)] - u[node(d, i, j - 1, k)]) * d.inv_2h;
    return (u[node(d, i, j, wrap(k + 1, d.nz))] - u[node(d, i, j, wrap(k - 1, d.nz))]) * d.inv_2h;
}

__device__ __forceinline__ bool interior(const Dims& d, int j) { return j >= 1 && j <= d.ny - 2; }

// Walks a slab of x-planes per thread (the block-partial layout of the forward reductions).
struct SlabIter {
    int j, k, i0, i1;
    bool ok;
};
__device__ __forceinline__ SlabIter slab_iter(const Dims& d, const SlabGrid& sg) {
    const int nb = sg.gx * sg.gi;
    const int lb = xcd_block(blockIdx.x, nb);
    const int bi = lb / sg.gx;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    SlabIter it;
    it.ok = t < d.ny * d.nz;
    it.j = it.ok ? t / d.nz : 0;
    it.k = it.ok ? t - it.j * d.nz : 0;
    it.i0 = bi * sg.ci;
    it.i1 = min(d.nx, (bi + 1) * sg.ci);
    return it;
}

inline dim3 plane_grid(const Dims& d) {
    return dim3((unsigned)((d.ny * d.nz + kBlock - 1) / kBlock), (unsigned)d.nx, 1);
}

}  // namespace
}  // namespace vs
