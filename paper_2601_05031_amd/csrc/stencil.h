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

inline dim3 plane_grid(const Dims& d) {
    return dim3((unsigned)((d.ny * d.nz + kBlock - 1) / kBlock), (unsigned)d.nx, 1);
}

}  // namespace
}  // namespace vs
