// Direct solve of the discrete 7-point Poisson problems of the main text, eq. (5b) and (5c)
// (SM (29b), (29c)), on gfx950 in FP64: Dirichlet walls in y, periodic in x and z.
//
// The periodic second differences in x and z are diagonalised by the discrete Hartley
// transform H (H_pk = cos(2 pi p k/n) + sin(2 pi p k/n)): each column of H is an eigenvector
// with eigenvalue (2 cos(2 pi p/n) - 2)/h^2, and H H = n I. So L_h u = b becomes, for every
// Hartley mode (p, q), one symmetric tridiagonal system in y, solved by the Thomas
// algorithm with precomputed pivots. Everything stays real: no complex spectrum is stored.
//
// Pass structure for one vector solve (three components, each pass one launch):
//   rhs_dht_z : b~ (or the residual b - L_h u) on the interior rows, Hartley along z
//   dht_x     : Hartley along x, in place
//   tridiag_y : Thomas along y per mode, scaled by h^2/(nx nz), in place
//   dht_x     : Hartley along x, in place
//   dht_z_out : Hartley along z, write (or add to) u
//   resid_norm, check : ||b - L_h u||^2, ||b~||^2, relative residual, convergence flag
// A Hartley transform of a real line is computed by a complex FFT of two lines packed as
// (line a) + i (line b), then H_a(p) = Re A_p - Im A_p with A_p = (Z_p + conj Z_{n-p})/2,
// and likewise for b. The FFT is a Stockham autosort transform in LDS with radix-4/2/3
// passes (line lengths 2^a 3^b), twiddles from a table exp(-2 pi i m/n).
#include "vs_internal.h"

namespace vs {

namespace {

constexpr int kBlock = 256;

struct Ptr3 {
    double* p[3];
};
struct CPtr3 {
    const double* p[3];
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int R>
__device__ __forceinline__ void butterfly(double2 (&x)[R]);

template <>
__device__ __forceinline__ void butterfly<2>(double2 (&x)[2]) {
    const double2 a = x[0], b = x[1];
    x[0] = make_double2(a.x + b.x, a.y + b.y);
    x[1] = make_double2(a.x - b.x, a.y - b.y);
}

template <>
__device__ __forceinline__ void butterfly<4>(double2 (&x)[4]) {
    const double2 a = make_double2(x[0].x + x[2].x, x[0].y + x[2].y);
    const double2 b = make_double2(x[0].x - x[2].x, x[0].y - x[2].y);
    const double2 c = make_double2(x[1].x + x[3].x, x[1].y + x[3].y);
    const double2 e = make_double2(x[1].x - x[3].x, x[1].y - x[3].y);
    x[0] = make_double2(a.x + c.x, a.y + c.y);
    x[2] = make_double2(a.x - c.x, a.y - c.y);
    x[1] = make_double2(b.x + e.y, b.y - e.x);   // b - i e
    x[3] = make_double2(b.x - e.y, b.y + e.x);   // b + i e
}

template <>
__device__ __forceinline__ void butterfly<3>(double2 (&x)[3]) {
    const double c = 0.86602540378443864676;    // sqrt(3)/2
    const double2 s = make_double2(x[1].x + x[2].x, x[1].y + x[2].y);
    const double2 e = make_double2(x[1].x - x[2].x, x[1].y - x[2].y);
    const double2 m = make_double2(x[0].x - 0.5 * s.x, x[0].y - 0.5 * s.y);
    x[0] = make_double2(x[0].x + s.x, x[0].y + s.y);
    x[1] = make_double2(m.x + c * e.y, m.y - c * e.x);   // m - i c e
    x[2] = make_double2(m.x - c * e.y, m.y + c * e.x);   // m + i c e
}

// One radix-R Stockham pass over nlines lines of length n (line stride n), in -> out.
// p is the product of the radices already applied.
template <int R>
__device__ __forceinline__ void stockham_pass(const double2* in, double2* out, int n, int p,
                                              int nlines, const double2* __restrict__ tw) {
    const int T = n / R;
    const int ts = n / (p * R);
    for (int e = threadIdx.x; e < nlines * T; e += blockDim.x) {
        const int line = e / T;
        const int t = e - line * T;
        const double2* X = in + line * n;
        double2* Y = out + line * n;
        const int kk = t % p;
        double2 x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = X[t + r * T];
#pragma unroll
        for (int r = 1; r < R; ++r) x[r] = cmul(x[r], tw[r * kk * ts]);
        butterfly<R>(x);
        const int jo = (t - kk) * R + kk;
#pragma unroll
        for (int r = 0; r < R; ++r) Y[jo + r * p] = x[r];
    }
}

// Forward FFT of nlines lines held in A (B is scratch of the same size). Returns the buffer
// with the result. Ends with a barrier.
__device__ double2* fft_lines(double2* A, double2* B, const FftPlan& pl, int nlines,
                              const double2* __restrict__ tw) {
    int p = 1;
    for (int s = 0; s < pl.npass; ++s) {
        __syncthreads();
        const int R = pl.radix[s];
        if (R == 4)
            stockham_pass<4>(A, B, pl.n, p, nlines, tw);
        else if (R == 2)
            stockham_pass<2>(A, B, pl.n, p, nlines, tw);
        else
            stockham_pass<3>(A, B, pl.n, p, nlines, tw);
        p *= R;
        double2* t = A;
        A = B;
        B = t;
    }
    __syncthreads();
    return A;
}

// Hartley value of the real line packed in the real (part = 0) or imaginary (part = 1) slot.
__device__ __forceinline__ double hartley(const double2* Z, int n, int p, int part) {
    const double2 zp = Z[p];
    const double2 zm = Z[p == 0 ? 0 : n - p];
    return part ? 0.5 * (zp.x - zm.x + zp.y + zm.y) : 0.5 * (zp.x + zm.x - zp.y + zm.y);
}

__device__ __forceinline__ void set_part(double2* slot, int part, double v) {
    reinterpret_cast<double*>(slot)[part] = v;
}

// Right-hand side b at interior node (i, j, k), 1 <= j <= ny-2.
__device__ __forceinline__ void rhs_at(const RhsArgs& a, const Dims& d, int i, int j, int k,
                                       int ncomp, double (&b)[3]) {
    const int c0 = node(d, i, j, k);
    if (a.mode == RHS_VORT) {
        const int ip = (i + 1 == d.nx) ? 0 : i + 1;
        const int im = (i == 0) ? d.nx - 1 : i - 1;
        const int kp = (k + 1 == d.nz) ? 0 : k + 1;
        const int km = (k == 0) ? d.nz - 1 : k - 1;
        const int xp = node(d, ip, j, k), xm = node(d, im, j, k);
        const int yp = c0 + d.nz, ym = c0 - d.nz;
        const int zp = c0 - k + kp, zm = c0 - k + km;
        const double* f = a.phi;
        const double* m = a.mu;
        const double fx = (f[xp] - f[xm]) * d.inv_2h, fy = (f[yp] - f[ym]) * d.inv_2h,
                     fz = (f[zp] - f[zm]) * d.inv_2h;
        const double mx = (m[xp] - m[xm]) * d.inv_2h, my = (m[yp] - m[ym]) * d.inv_2h,
                     mz = (m[zp] - m[zm]) * d.inv_2h;
        b[0] = (fy * mz - fz * my) * a.inv_eta;
        b[1] = (fz * mx - fx * mz) * a.inv_eta;
        b[2] = (fx * my - fy * mx) * a.inv_eta;
        return;
    }
    const double sg = (a.mode == RHS_NEGW) ? -1.0 : 1.0;
    for (int c = 0; c < ncomp; ++c) b[c] = sg * a.f[c][c0];
}

// 7-point Laplacian at an interior node using the stored wall rows of u.
__device__ __forceinline__ double lap_interior(const double* __restrict__ u, const Dims& d, int i,
                                               int j, int k) {
    const int c0 = node(d, i, j, k);
    const int ip = (i + 1 == d.nx) ? 0 : i + 1;
    const int im = (i == 0) ? d.nx - 1 : i - 1;
    const int kp = (k + 1 == d.nz) ? 0 : k + 1;
    const int km = (k == 0) ? d.nz - 1 : k - 1;
    return (u[node(d, ip, j, k)] + u[node(d, im, j, k)] + u[c0 + d.nz] + u[c0 - d.nz] +
            u[c0 - k + kp] + u[c0 - k + km] - 6.0 * u[c0]) *
           d.inv_h2;
}

// Wall contribution of the Dirichlet values to row j (nonzero only for j = 1 and j = M).
__device__ __forceinline__ double wall_term(const double* __restrict__ u, const Dims& d, int i,
                                            int j, int k) {
    double w = 0.0;
    if (j == 1) w += u[node(d, i, 0, k)];
    if (j == d.M) w += u[node(d, i, d.ny - 1, k)];
    return w * d.inv_h2;
}

// ---------------------------------------------------------------------------------------
// rhs_dht_z: rows r = i*M + (j-1) of the interior, rpb rows per block, ncomp components.
// correct = 0: transform b - (wall terms); correct = 1: transform b - L_h u.
__global__ __launch_bounds__(kBlock) void k_rhs_dht_z(Dims d, FftPlan pz,
                                                     const double2* __restrict__ tw, RhsArgs rhs,
                                                     CPtr3 u, int ncomp, int correct, Ptr3 spec,
                                                     const int* gate, int rpb) {
    if (gate && *gate) return;
    extern __shared__ double2 lds[];
    const int n = d.nz;
    const int lpc = rpb >> 1;                 // complex lines per component
    const int nlines = ncomp * lpc;
    double2* A = lds;
    double2* B = lds + nlines * n;
    const int nrows = d.nx * d.M;
    const int r0 = blockIdx.x * rpb;
    for (int e = threadIdx.x; e < rpb * n; e += blockDim.x) {
        const int lr = e / n;
        const int k = e - lr * n;
        const int r = r0 + lr;
        double b[3] = {0.0, 0.0, 0.0};
        if (r < nrows) {
            const int i = r / d.M;
            const int j = 1 + (r - i * d.M);
            rhs_at(rhs, d, i, j, k, ncomp, b);
            for (int c = 0; c < ncomp; ++c)
                b[c] -= correct ? lap_interior(u.p[c], d, i, j, k) : wall_term(u.p[c], d, i, j, k);
        }
        for (int c = 0; c < ncomp; ++c) set_part(&A[(c * lpc + (lr >> 1)) * n + k], lr & 1, b[c]);
    }
    const double2* Z = fft_lines(A, B, pz, nlines, tw);
    for (int e = threadIdx.x; e < ncomp * rpb * n; e += blockDim.x) {
        const int c = e / (rpb * n);
        const int rem = e - c * rpb * n;
        const int lr = rem / n;
        const int p = rem - lr * n;
        const int r = r0 + lr;
        if (r >= nrows) continue;
        const int i = r / d.M;
        const int j = 1 + (r - i * d.M);
        spec.p[c][node(d, i, j, p)] = hartley(Z + (c * lpc + (lr >> 1)) * n, n, p, lr & 1);
    }
}

// dht_x: block = (component, interior row j, block of kb consecutive z-modes q).
__global__ __launch_bounds__(kBlock) void k_dht_x(Dims d, FftPlan px,
                                                 const double2* __restrict__ tw, Ptr3 spec,
                                                 const int* gate, int kb) {
    if (gate && *gate) return;
    extern __shared__ double2 lds[];
    const int n = d.nx;
    const int nlines = kb >> 1;
    double2* A = lds;
    double2* B = lds + nlines * n;
    const int c = blockIdx.z;
    const int j = 1 + blockIdx.y;
    const int q0 = blockIdx.x * kb;
    double* s = spec.p[c];
    for (int e = threadIdx.x; e < n * kb; e += blockDim.x) {
        const int i = e / kb;
        const int kk = e - i * kb;
        const int q = q0 + kk;
        const double v = (q < d.nz) ? s[node(d, i, j, q)] : 0.0;
        set_part(&A[(kk >> 1) * n + i], kk & 1, v);
    }
    const double2* Z = fft_lines(A, B, px, nlines, tw);
    for (int e = threadIdx.x; e < n * kb; e += blockDim.x) {
        const int p = e / kb;
        const int kk = e - p * kb;
        const int q = q0 + kk;
        if (q >= d.nz) continue;
        s[node(d, p, j, q)] = hartley(Z + (kk >> 1) * n, n, p, kk & 1);
    }
}

// tridiag_y: one thread per (component, p, q). Solves
//   U_{j-1} + beta U_j + U_{j+1} = scale * B_j,  j = 1..M,  U_0 = U_{M+1} = 0,
// beta = 2 cos(2 pi p/nx) + 2 cos(2 pi q/nz) - 6, with the forward-elimination pivots
// c'_j = 1/(beta - c'_{j-1}) read from a table indexed by the mode class
// (min(p, nx-p), min(q, nz-q)). In place; loads are issued in chunks of 8 rows.
__global__ __launch_bounds__(kBlock) void k_tridiag_y(Dims d, const double* __restrict__ tri,
                                                     Ptr3 spec, const int* gate, double scale) {
    if (gate && *gate) return;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= d.nx * d.nz) return;
    const int c = blockIdx.y;
    const int p = t / d.nz;
    const int q = t - p * d.nz;
    const int pc = min(p, d.nx - p);
    const int qc = min(q, d.nz - q);
    const double* cp = tri + (size_t)(pc * (d.nz / 2 + 1) + qc) * d.M;
    double* col = spec.p[c] + (size_t)p * d.ny * d.nz + q;
    const int sj = d.nz;
    const int M = d.M;
    constexpr int CH = 8;
    double dprev = 0.0;
    int j = 1;
    for (; j + CH - 1 <= M; j += CH) {
        double bv[CH], cv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            bv[u] = col[(size_t)(j + u) * sj];
            cv[u] = cp[j + u - 1];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            dprev = cv[u] * (scale * bv[u] - dprev);
            col[(size_t)(j + u) * sj] = dprev;
        }
    }
    for (; j <= M; ++j) {
        dprev = cp[j - 1] * (scale * col[(size_t)j * sj] - dprev);
        col[(size_t)j * sj] = dprev;
    }
    double unext = 0.0;
    j = M;
    for (; j - CH + 1 >= 1; j -= CH) {
        double dv[CH], cv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            dv[u] = col[(size_t)(j - u) * sj];
            cv[u] = cp[j - u - 1];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            unext = dv[u] - cv[u] * unext;
            col[(size_t)(j - u) * sj] = unext;
        }
    }
    for (; j >= 1; --j) {
        unext = col[(size_t)j * sj] - cp[j - 1] * unext;
        col[(size_t)j * sj] = unext;
    }
}

// dht_z_out: Hartley along z of the solved modes, then u = result (add = 0) or u += result.
__global__ __launch_bounds__(kBlock) void k_dht_z_out(Dims d, FftPlan pz,
                                                     const double2* __restrict__ tw, Ptr3 spec,
                                                     Ptr3 u, int ncomp, int add, const int* gate,
                                                     int rpb) {
    if (gate && *gate) return;
    extern __shared__ double2 lds[];
    const int n = d.nz;
    const int lpc = rpb >> 1;
    const int nlines = ncomp * lpc;
    double2* A = lds;
    double2* B = lds + nlines * n;
    const int nrows = d.nx * d.M;
    const int r0 = blockIdx.x * rpb;
    for (int e = threadIdx.x; e < ncomp * rpb * n; e += blockDim.x) {
        const int c = e / (rpb * n);
        const int rem = e - c * rpb * n;
        const int lr = rem / n;
        const int k = rem - lr * n;
        const int r = r0 + lr;
        double v = 0.0;
        if (r < nrows) {
            const int i = r / d.M;
            const int j = 1 + (r - i * d.M);
            v = spec.p[c][node(d, i, j, k)];
        }
        set_part(&A[(c * lpc + (lr >> 1)) * n + k], lr & 1, v);
    }
    const double2* Z = fft_lines(A, B, pz, nlines, tw);
    for (int e = threadIdx.x; e < ncomp * rpb * n; e += blockDim.x) {
        const int c = e / (rpb * n);
        const int rem = e - c * rpb * n;
        const int lr = rem / n;
        const int p = rem - lr * n;
        const int r = r0 + lr;
        if (r >= nrows) continue;
        const int i = r / d.M;
        const int j = 1 + (r - i * d.M);
        const double v = hartley(Z + (c * lpc + (lr >> 1)) * n, n, p, lr & 1);
        double* dst = u.p[c] + node(d, i, j, p);
        *dst = add ? *dst + v : v;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// resid_norm: block partials of sum (b - L_h u)_c^2 and sum b~_c^2 over the interior.
__global__ __launch_bounds__(kBlock) void k_resid_norm(Dims d, RhsArgs rhs, CPtr3 u, int ncomp,
                                                      double* __restrict__ partials,
                                                      const int* gate) {
    if (gate && *gate) return;
    __shared__ double sh[6 * 4];
    const int nint = d.nx * d.M * d.nz;
    const int plane = d.M * d.nz;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int t = blockIdx.x * kBlock + threadIdx.x; t < nint; t += gridDim.x * kBlock) {
        const int i = t / plane;
        const int rem = t - i * plane;
        const int jj = rem / d.nz;
        const int k = rem - jj * d.nz;
        const int j = jj + 1;
        double b[3] = {0.0, 0.0, 0.0};
        rhs_at(rhs, d, i, j, k, ncomp, b);
        for (int c = 0; c < ncomp; ++c) {
            const double r = b[c] - lap_interior(u.p[c], d, i, j, k);
            const double bt = b[c] - wall_term(u.p[c], d, i, j, k);
            acc[c] += r * r;
            acc[3 + c] += bt * bt;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) sh[q * 4 + w] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const double s = sh[threadIdx.x * 4 + 0] + sh[threadIdx.x * 4 + 1] +
                         sh[threadIdx.x * 4 + 2] + sh[threadIdx.x * 4 + 3];
        partials[blockIdx.x * kPartialStride + threadIdx.x] = s;
    }
}

// check: relative residual sqrt(sum_c r^2 / sum_c b~^2) in a fixed summation order; sets the
// convergence flag that gates the following cycles, counts the cycle and raises ST_NOCONV
// on the last allowed cycle, ST_NONFINITE on NaN/Inf.
__global__ __launch_bounds__(kBlock) void k_check(const double* __restrict__ partials,
                                                 int nblocks, double rtol, int last_cycle,
                                                 double* scal, int* istat, const int* gate) {
    if (gate && *gate) return;
    __shared__ double sh[2 * 4];
    double rr = 0.0, bb = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const double* pb = partials + b * kPartialStride;
        rr += pb[0] + pb[1] + pb[2];
        bb += pb[3] + pb[4] + pb[5];
    }
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[w] = rr;
        sh[4 + w] = bb;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    rr = sh[0] + sh[1] + sh[2] + sh[3];
    bb = sh[4] + sh[5] + sh[6] + sh[7];
    double rel;
    if (bb > 0.0)
        rel = sqrt(rr / bb);
    else
        rel = (rr > 0.0) ? INFINITY : 0.0;
    if (rr != rr || bb != bb) rel = NAN;
    const int conv = (rel <= rtol) ? 1 : 0;
    istat[IS_CONV] = conv;
    istat[IS_CYCLES] += 1;
    scal[SC_RELRES_LAST] = rel;
    if (conv || last_cycle) {
        const double prev = scal[SC_RELRES_MAX];
        scal[SC_RELRES_MAX] = (rel != rel || rel > prev) ? rel : prev;
    }
    if (!conv && last_cycle) istat[IS_FLAGS] |= ST_NOCONV;
    if (!isfinite(rr) || !isfinite(bb)) istat[IS_FLAGS] |= ST_NONFINITE;
}

int z_rows_per_block(const Dims& d, int ncomp) {
    int rpb = 2 * (1536 / (ncomp * d.nz));
    if (rpb < 2) rpb = 2;
    return rpb;
}

int x_modes_per_block(const Dims& d) {
    int kb = 4096 / d.nx;
    if (kb > 16) kb = 16;
    kb &= ~1;
    if (kb < 2) kb = 2;
    return kb;
}

}  // namespace

void launch_rhs_dht_z(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      const RhsArgs& rhs, const double* const u[3], int ncomp, int correct,
                      double* const spec[3], const int* gate) {
    const int rpb = z_rows_per_block(d, ncomp);
    const int nrows = d.nx * d.M;
    const size_t lds = 2ull * ncomp * (rpb / 2) * d.nz * sizeof(double2);
    CPtr3 uu{{u[0], ncomp > 1 ? u[1] : nullptr, ncomp > 2 ? u[2] : nullptr}};
    Ptr3 sp{{spec[0], ncomp > 1 ? spec[1] : nullptr, ncomp > 2 ? spec[2] : nullptr}};
    hipLaunchKernelGGL(k_rhs_dht_z, dim3((nrows + rpb - 1) / rpb), dim3(kBlock), lds, s, d, pz,
                       twz, rhs, uu, ncomp, correct, sp, gate, rpb);
}

void launch_dht_x(hipStream_t s, const Dims& d, const FftPlan& px, const double2* twx,
                  double* const spec[3], int ncomp, const int* gate) {
    const int kb = x_modes_per_block(d);
    const size_t lds = 2ull * (kb / 2) * d.nx * sizeof(double2);
    Ptr3 sp{{spec[0], ncomp > 1 ? spec[1] : nullptr, ncomp > 2 ? spec[2] : nullptr}};
    hipLaunchKernelGGL(k_dht_x, dim3((d.nz + kb - 1) / kb, d.M, ncomp), dim3(kBlock), lds, s, d,
                       px, twx, sp, gate, kb);
}

void launch_tridiag_y(hipStream_t s, const Dims& d, const double* tri, double* const spec[3],
                      int ncomp, const int* gate) {
    Ptr3 sp{{spec[0], ncomp > 1 ? spec[1] : nullptr, ncomp > 2 ? spec[2] : nullptr}};
    const double scale = d.h * d.h / ((double)d.nx * d.nz);
    hipLaunchKernelGGL(k_tridiag_y, dim3((d.nx * d.nz + kBlock - 1) / kBlock, ncomp),
                       dim3(kBlock), 0, s, d, tri, sp, gate, scale);
}

void launch_dht_z_out(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      double* const spec[3], double* const u[3], int ncomp, int add,
                      const int* gate) {
    const int rpb = z_rows_per_block(d, ncomp);
    const int nrows = d.nx * d.M;
    const size_t lds = 2ull * ncomp * (rpb / 2) * d.nz * sizeof(double2);
    Ptr3 sp{{spec[0], ncomp > 1 ? spec[1] : nullptr, ncomp > 2 ? spec[2] : nullptr}};
    Ptr3 uu{{u[0], ncomp > 1 ? u[1] : nullptr, ncomp > 2 ? u[2] : nullptr}};
    hipLaunchKernelGGL(k_dht_z_out, dim3((nrows + rpb - 1) / rpb), dim3(kBlock), lds, s, d, pz,
                       twz, sp, uu, ncomp, add, gate, rpb);
}

int resid_blocks(const Dims& d) {
    const long nint = (long)d.nx * d.M * d.nz;
    long b = (nint + kBlock - 1) / kBlock;
    if (b > kMaxPartialBlocks) b = kMaxPartialBlocks;
    return (int)b;
}

void launch_resid_norm(hipStream_t s, const Dims& d, const RhsArgs& rhs,
                       const double* const u[3], int ncomp, double* partials, int nblocks,
                       const int* gate) {
    CPtr3 uu{{u[0], ncomp > 1 ? u[1] : nullptr, ncomp > 2 ? u[2] : nullptr}};
    hipLaunchKernelGGL(k_resid_norm, dim3(nblocks), dim3(kBlock), 0, s, d, rhs, uu, ncomp,
                       partials, gate);
}

void launch_check(hipStream_t s, const double* partials, int nblocks, double rtol, int cycle,
                  int last_cycle, double* scal, int* istat, const int* gate) {
    (void)cycle;
    hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, partials, nblocks, rtol,
                       last_cycle, scal, istat, gate);
}

}  // namespace vs
