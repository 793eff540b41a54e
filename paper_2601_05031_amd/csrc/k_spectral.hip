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

// One radix-R Stockham pass, in place in LDS, over nlines lines of length n (line stride n).
// p is the product of the radices already applied. The tile holds at most 2 * R * blockDim
// elements per pass, so each thread stages at most two butterflies in registers: all reads,
// a barrier, then all writes.
template <int R>
__device__ __forceinline__ void stockham_pass(double2* A, int n, int p, int nlines,
                                              const double2* __restrict__ tw) {
    const int T = n / R;
    const int total = nlines * T;
    const int ts = n / (p * R);
    double2 x[2][R];
    int jo[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int e = threadIdx.x + b * blockDim.x;
        jo[b] = -1;
        if (e < total) {
            const int line = e / T;
            const int t = e - line * T;
            const int kk = t % p;
            const double2* X = A + line * n;
#pragma unroll
            for (int r = 0; r < R; ++r) x[b][r] = X[t + r * T];
#pragma unroll
            for (int r = 1; r < R; ++r) x[b][r] = cmul(x[b][r], tw[r * kk * ts]);
            butterfly<R>(x[b]);
            jo[b] = line * n + (t - kk) * R + kk;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        if (jo[b] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) A[jo[b] + r * p] = x[b][r];
        }
    }
    __syncthreads();
}

// Forward FFT, in place, of nlines lines held in A (nlines * n <= kTileElems). Starts and
// ends with a barrier.
__device__ void fft_tile(double2* A, const FftPlan& pl, int nlines, const double2* __restrict__ tw) {
    __syncthreads();
    int p = 1;
    for (int s = 0; s < pl.npass; ++s) {
        const int R = pl.radix[s];
        if (R == 4)
            stockham_pass<4>(A, pl.n, p, nlines, tw);
        else if (R == 2)
            stockham_pass<2>(A, pl.n, p, nlines, tw);
        else
            stockham_pass<3>(A, pl.n, p, nlines, tw);
        p *= R;
    }
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

// Component c of the right-hand side at interior node (i, j, k).
__device__ __forceinline__ double rhs_comp(const RhsArgs& a, const Dims& d, int i, int j, int k,
                                           int c) {
    const int c0 = node(d, i, j, k);
    if (a.mode == RHS_VORT) {
        const int ip = (i + 1 == d.nx) ? 0 : i + 1;
        const int im = (i == 0) ? d.nx - 1 : i - 1;
        const int kp = (k + 1 == d.nz) ? 0 : k + 1;
        const int km = (k == 0) ? d.nz - 1 : k - 1;
        const double* f = a.phi;
        const double* m = a.mu;
        // (D phi x D mu)_c needs the two derivative directions other than c
        double f1, f2, m1, m2;
        if (c == 0) {        // y, z
            f1 = f[c0 + d.nz] - f[c0 - d.nz]; m1 = m[c0 + d.nz] - m[c0 - d.nz];
            f2 = f[c0 - k + kp] - f[c0 - k + km]; m2 = m[c0 - k + kp] - m[c0 - k + km];
        } else if (c == 1) { // z, x
            f1 = f[c0 - k + kp] - f[c0 - k + km]; m1 = m[c0 - k + kp] - m[c0 - k + km];
            f2 = f[node(d, ip, j, k)] - f[node(d, im, j, k)];
            m2 = m[node(d, ip, j, k)] - m[node(d, im, j, k)];
        } else {             // x, y
            f1 = f[node(d, ip, j, k)] - f[node(d, im, j, k)];
            m1 = m[node(d, ip, j, k)] - m[node(d, im, j, k)];
            f2 = f[c0 + d.nz] - f[c0 - d.nz]; m2 = m[c0 + d.nz] - m[c0 - d.nz];
        }
        return ((f1 * d.inv_2h) * (m2 * d.inv_2h) - (f2 * d.inv_2h) * (m1 * d.inv_2h)) * a.inv_eta;
    }
    const double v = a.f[c][c0];
    return (a.mode == RHS_NEGW) ? -v : v;
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
// Tiles: every transform kernel holds at most kTileElems complex values (16 KB) in one LDS
// buffer, one component per block (blockIdx.y), so eight or more blocks fit on a CU.
constexpr int kTileElems = 1024;

// rhs_dht_z: block = (rows r0 .. r0+rpb-1 of the interior, r = i*M + (j-1); component c).
// correct = 0: transform b - (wall terms); correct = 1: transform b - L_h u.
__global__ __launch_bounds__(kBlock) void k_rhs_dht_z(Dims d, FftPlan pz,
                                                     const double2* __restrict__ tw, RhsArgs rhs,
                                                     CPtr3 u, int correct, Ptr3 spec,
                                                     const int* gate, int rpb) {
    if (gate && *gate) return;
    __shared__ double2 A[kTileElems];
    const int n = d.nz;
    const int nlines = rpb >> 1;
    const int c = blockIdx.y;
    const int nrows = d.nx * d.M;
    const int r0 = blockIdx.x * rpb;
    const double* uc = u.p[c];
    for (int e = threadIdx.x; e < rpb * n; e += blockDim.x) {
        const int lr = e / n;
        const int k = e - lr * n;
        const int r = r0 + lr;
        double b = 0.0;
        if (r < nrows) {
            const int i = r / d.M;
            const int j = 1 + (r - i * d.M);
            b = rhs_comp(rhs, d, i, j, k, c);
            b -= correct ? lap_interior(uc, d, i, j, k) : wall_term(uc, d, i, j, k);
        }
        set_part(&A[(lr >> 1) * n + k], lr & 1, b);
    }
    fft_tile(A, pz, nlines, tw);
    double* sc = spec.p[c];
    for (int e = threadIdx.x; e < rpb * n; e += blockDim.x) {
        const int lr = e / n;
        const int p = e - lr * n;
        const int r = r0 + lr;
        if (r >= nrows) continue;
        const int i = r / d.M;
        const int j = 1 + (r - i * d.M);
        sc[node(d, i, j, p)] = hartley(A + (lr >> 1) * n, n, p, lr & 1);
    }
}

// dht_x: block = (block of kb consecutive z-modes q, interior row j, component c).
__global__ __launch_bounds__(kBlock) void k_dht_x(Dims d, FftPlan px,
                                                 const double2* __restrict__ tw, Ptr3 spec,
                                                 const int* gate, int kb) {
    if (gate && *gate) return;
    __shared__ double2 A[kTileElems];
    const int n = d.nx;
    const int nlines = kb >> 1;
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
    fft_tile(A, px, nlines, tw);
    for (int e = threadIdx.x; e < n * kb; e += blockDim.x) {
        const int p = e / kb;
        const int kk = e - p * kb;
        const int q = q0 + kk;
        if (q >= d.nz) continue;
        s[node(d, p, j, q)] = hartley(A + (kk >> 1) * n, n, p, kk & 1);
    }
}

// tridiag_y: one thread per (p, q), component blockIdx.y. Solves
//   U_{j-1} + beta U_j + U_{j+1} = scale * B_j,  j = 1..M,  U_0 = U_{M+1} = 0,
// beta = 2 cos(2 pi p/nx) + 2 cos(2 pi q/nz) - 6, with the forward-elimination pivots
// c'_j = 1/(beta - c'_{j-1}) read from a table tri[(j-1) * nclass + class], class =
// min(p, nx-p) * (nz/2+1) + min(q, nz-q): lanes with consecutive q read consecutive (or
// reversed consecutive) entries. In place. Rows are processed in chunks of CH with the next
// chunk's loads issued before the current chunk's dependent recurrence runs.
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
    const size_t ncls = (size_t)(d.nx / 2 + 1) * (d.nz / 2 + 1);
    const double* cp = tri + (size_t)(pc * (d.nz / 2 + 1) + qc);
    double* col = spec.p[c] + (size_t)p * d.ny * d.nz + q;
    const size_t sj = d.nz;
    const int M = d.M;
    constexpr int CH = 8;
    double bv[CH], cv[CH];
    // forward elimination, rows 1..M
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const int j = 1 + u;
        bv[u] = (j <= M) ? col[j * sj] : 0.0;
        cv[u] = (j <= M) ? cp[(size_t)(j - 1) * ncls] : 0.0;
    }
    double dprev = 0.0;
    for (int j0 = 1; j0 <= M; j0 += CH) {
        double nb[CH], nc[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int j = j0 + CH + u;
            nb[u] = (j <= M) ? col[j * sj] : 0.0;
            nc[u] = (j <= M) ? cp[(size_t)(j - 1) * ncls] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int j = j0 + u;
            if (j <= M) {
                dprev = cv[u] * (scale * bv[u] - dprev);
                col[j * sj] = dprev;
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            bv[u] = nb[u];
            cv[u] = nc[u];
        }
    }
    // back substitution, rows M..1
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const int j = M - u;
        bv[u] = (j >= 1) ? col[j * sj] : 0.0;
        cv[u] = (j >= 1) ? cp[(size_t)(j - 1) * ncls] : 0.0;
    }
    double unext = 0.0;
    for (int j0 = M; j0 >= 1; j0 -= CH) {
        double nb[CH], nc[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int j = j0 - CH - u;
            nb[u] = (j >= 1) ? col[j * sj] : 0.0;
            nc[u] = (j >= 1) ? cp[(size_t)(j - 1) * ncls] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int j = j0 - u;
            if (j >= 1) {
                unext = bv[u] - cv[u] * unext;
                col[j * sj] = unext;
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            bv[u] = nb[u];
            cv[u] = nc[u];
        }
    }
}

// dht_z_out: Hartley along z of the solved modes, then u = result (add = 0) or u += result.
__global__ __launch_bounds__(kBlock) void k_dht_z_out(Dims d, FftPlan pz,
                                                     const double2* __restrict__ tw, Ptr3 spec,
                                                     Ptr3 u, int add, const int* gate, int rpb) {
    if (gate && *gate) return;
    __shared__ double2 A[kTileElems];
    const int n = d.nz;
    const int nlines = rpb >> 1;
    const int c = blockIdx.y;
    const int nrows = d.nx * d.M;
    const int r0 = blockIdx.x * rpb;
    const double* sc = spec.p[c];
    for (int e = threadIdx.x; e < rpb * n; e += blockDim.x) {
        const int lr = e / n;
        const int k = e - lr * n;
        const int r = r0 + lr;
        double v = 0.0;
        if (r < nrows) {
            const int i = r / d.M;
            const int j = 1 + (r - i * d.M);
            v = sc[node(d, i, j, k)];
        }
        set_part(&A[(lr >> 1) * n + k], lr & 1, v);
    }
    fft_tile(A, pz, nlines, tw);
    double* uc = u.p[c];
    for (int e = threadIdx.x; e < rpb * n; e += blockDim.x) {
        const int lr = e / n;
        const int p = e - lr * n;
        const int r = r0 + lr;
        if (r >= nrows) continue;
        const int i = r / d.M;
        const int j = 1 + (r - i * d.M);
        const double v = hartley(A + (lr >> 1) * n, n, p, lr & 1);
        double* dst = uc + node(d, i, j, p);
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
        partials[threadIdx.x * kMaxPartialBlocks + blockIdx.x] = s;
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
        const double* pb = partials + b;
        rr += pb[0 * kMaxPartialBlocks] + pb[1 * kMaxPartialBlocks] + pb[2 * kMaxPartialBlocks];
        bb += pb[3 * kMaxPartialBlocks] + pb[4 * kMaxPartialBlocks] + pb[5 * kMaxPartialBlocks];
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

// Rows per block of the z kernels: 2 * (kTileElems / nz), i.e. kTileElems / nz complex lines.
int z_rows_per_block(const Dims& d) {
    int lines = kTileElems / d.nz;
    if (lines < 1) lines = 1;
    return 2 * lines;
}

// z-modes per block of the x kernel: up to 32 consecutive q (256-byte runs), kb/2 lines of nx.
int x_modes_per_block(const Dims& d) {
    int kb = 2 * (kTileElems / d.nx);
    if (kb > 32) kb = 32;
    if (kb < 2) kb = 2;
    return kb;
}

}  // namespace

void launch_rhs_dht_z(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      const RhsArgs& rhs, const double* const u[3], int ncomp, int correct,
                      double* const spec[3], const int* gate) {
    const int rpb = z_rows_per_block(d);
    const int nrows = d.nx * d.M;
    CPtr3 uu{{u[0], ncomp > 1 ? u[1] : nullptr, ncomp > 2 ? u[2] : nullptr}};
    Ptr3 sp{{spec[0], ncomp > 1 ? spec[1] : nullptr, ncomp > 2 ? spec[2] : nullptr}};
    hipLaunchKernelGGL(k_rhs_dht_z, dim3((nrows + rpb - 1) / rpb, ncomp), dim3(kBlock), 0, s, d,
                       pz, twz, rhs, uu, correct, sp, gate, rpb);
}

void launch_dht_x(hipStream_t s, const Dims& d, const FftPlan& px, const double2* twx,
                  double* const spec[3], int ncomp, const int* gate) {
    const int kb = x_modes_per_block(d);
    Ptr3 sp{{spec[0], ncomp > 1 ? spec[1] : nullptr, ncomp > 2 ? spec[2] : nullptr}};
    hipLaunchKernelGGL(k_dht_x, dim3((d.nz + kb - 1) / kb, d.M, ncomp), dim3(kBlock), 0, s, d,
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
    const int rpb = z_rows_per_block(d);
    const int nrows = d.nx * d.M;
    Ptr3 sp{{spec[0], ncomp > 1 ? spec[1] : nullptr, ncomp > 2 ? spec[2] : nullptr}};
    Ptr3 uu{{u[0], ncomp > 1 ? u[1] : nullptr, ncomp > 2 ? u[2] : nullptr}};
    hipLaunchKernelGGL(k_dht_z_out, dim3((nrows + rpb - 1) / rpb, ncomp), dim3(kBlock), 0, s, d,
                       pz, twz, sp, uu, add, gate, rpb);
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
