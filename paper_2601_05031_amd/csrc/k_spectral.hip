// Direct solve of the discrete 7-point Poisson problems of the main text, eq. (5b) and (5c)
// (SM (29b), (29c)), on gfx950 in FP64: Dirichlet walls in y, periodic in x and z.
//
// The periodic second differences in x and z are diagonalised by the discrete Hartley
// transform H (H_pk = cos(2 pi p k/n) + sin(2 pi p k/n)): each column of H is an eigenvector
// with eigenvalue (2 cos(2 pi p/n) - 2)/h^2, and H H = n I. So L_h u = b becomes, for every
// Hartley mode (p, q), one symmetric tridiagonal system in y with precomputed pivots, solved
// in register segments (or by a two-ended elimination for very short or tall columns).
// Everything stays real: no complex spectrum is stored.
//
// Pass structure of the two flow solves of a step (each pass one launch):
//   z transform of S : Hartley along z of the vorticity source (the dht_z_out kernel)
//   dht_x            : Hartley along x, in place
//   tridiag_pair     : vorticity modes (walls in mode (0, 0)), then the stream-vector modes
//                      from them, scaled by h^2/(nx nz), into two spectral buffers
//   dht_x, dht_z_out : Hartley along x, then z, of both fields together (six components
//                      per launch)
//   resid_flow, check: ||b - L_h u||^2 and ||b~||^2 of both problems, relative residuals
// The inertial variant (SM eq. (36)) runs the same passes for (L_h - a) omega = S - a omega^n:
// its vorticity modes take the pivots of the shifted diagonal, its residual the shifted
// operator; the stream-vector problem is unchanged.
// The general form of one vector solve (vs_poisson_solve, refinement cycles) starts with
// rhs_dht_z (b~, or the residual b - L_h u, on the interior rows, Hartley along z) and runs
// dht_x, tridiag_y, dht_x, dht_z_out, resid_norm and check for each cycle.
// A Hartley transform of a real line is computed by a complex FFT of two lines packed as
// (line a) + i (line b), then H_a(p) = Re A_p - Im A_p with A_p = (Z_p + conj Z_{n-p})/2,
// and likewise for b. Line lengths n = B A (B in {8, 16}, A in {3, 4, 6, 8, 12, 16}) use a
// two-pass register FFT; other 2^a 3^b lengths a Stockham transform in LDS with radix-4/2/3
// passes. Twiddles come from a table exp(-2 pi i m/n).
#include "fft_reg.h"
#include "flow_check.h"
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
// Pointers to the spectral intermediates, stored as ST (double, or float in the refined mode).
template <class ST>
struct SPtr3 {
    ST* p[3];
};
// Up to six components for the two-pass transforms: the vorticity and stream-vector fields of
// a step go through one launch per direction.
template <class ST>
struct SPtr6 {
    ST* p[6];
};
struct Ptr6 {
    double* p[6];
};

// Loads widen to double and stores narrow from double: inside a kernel all arithmetic is FP64.
__device__ __forceinline__ double ld(const double* p) { return *p; }
__device__ __forceinline__ double ld(const float* p) { return (double)*p; }
__device__ __forceinline__ void st(double* p, double v) { *p = v; }
__device__ __forceinline__ void st(float* p, double v) { *p = (float)v; }
__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }
__device__ __forceinline__ double2 ld2(const float* p) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2(double* p, double a, double b) {
    *reinterpret_cast<double2*>(p) = make_double2(a, b);
}
__device__ __forceinline__ void st2(float* p, double a, double b) {
    *reinterpret_cast<float2*>(p) = make_float2((float)a, (float)b);
}

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

// Component c of the right-hand side b at an interior node offset c0.
__device__ __forceinline__ double rhs_val(const RhsArgs& a, int c, int c0) {
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
template <class ST>
__global__ __launch_bounds__(kBlock) void k_rhs_dht_z(Dims d, FftPlan pz,
                                                     const double2* __restrict__ tw, RhsArgs rhs,
                                                     CPtr3 u, int correct, SPtr3<ST> spec,
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
            b = rhs_val(rhs, c, node(d, i, j, k));
            b -= correct ? lap_interior(uc, d, i, j, k) : wall_term(uc, d, i, j, k);
        }
        set_part(&A[(lr >> 1) * n + k], lr & 1, b);
    }
    fft_tile(A, pz, nlines, tw);
    ST* sc = spec.p[c];
    for (int e = threadIdx.x; e < rpb * n; e += blockDim.x) {
        const int lr = e / n;
        const int p = e - lr * n;
        const int r = r0 + lr;
        if (r >= nrows) continue;
        const int i = r / d.M;
        const int j = 1 + (r - i * d.M);
        st(sc + node(d, i, j, p), hartley(A + (lr >> 1) * n, n, p, lr & 1));
    }
}

// dht_x: block = (block of kb consecutive z-modes q, interior row j, component c).
template <class ST>
__global__ __launch_bounds__(kBlock) void k_dht_x(Dims d, FftPlan px,
                                                 const double2* __restrict__ tw, SPtr3<ST> spec,
                                                 const int* gate, int kb) {
    if (gate && *gate) return;
    __shared__ double2 A[kTileElems];
    const int n = d.nx;
    const int nlines = kb >> 1;
    const int c = blockIdx.z;
    const int j = 1 + blockIdx.y;
    const int q0 = blockIdx.x * kb;
    ST* s = spec.p[c];
    for (int e = threadIdx.x; e < n * kb; e += blockDim.x) {
        const int i = e / kb;
        const int kk = e - i * kb;
        const int q = q0 + kk;
        const double v = (q < d.nz) ? ld(s + node(d, i, j, q)) : 0.0;
        set_part(&A[(kk >> 1) * n + i], kk & 1, v);
    }
    fft_tile(A, px, nlines, tw);
    for (int e = threadIdx.x; e < n * kb; e += blockDim.x) {
        const int p = e / kb;
        const int kk = e - p * kb;
        const int q = q0 + kk;
        if (q >= d.nz) continue;
        st(s + node(d, p, j, q), hartley(A + (kk >> 1) * n, n, p, kk & 1));
    }
}

// Twisted tridiagonal solve of
//   U_{j-1} + beta U_j + U_{j+1} = f_j,  j = 1..M,  U_0 = U_{M+1} = 0,
// beta = 2 cos(2 pi p/nx) + 2 cos(2 pi q/nz) - 6, shared by a lane pair: the even lane
// eliminates rows 1..m downwards (pivots c'_s = 1/(beta - c'_{s-1}), rows read as
// U_j + c'_j U_{j+1} = d'_j), the odd lane rows M..m+1 upwards with the same pivots counted
// from the bottom (the matrix is symmetric Toeplitz), the two meet in a 2x2 system at rows
// m, m+1 (values exchanged by a lane shuffle), then each back-substitutes away from the
// middle. f_j = rhs(j, v) with v the value read at row j of rd; d' and then U are written to
// wr (which may alias rd). Pivots come from cp[s * ncls]; loads run one chunk ahead. All lanes
// of the wave call this together; inactive lanes pass act = false.
// INPLACE: rd == wr (one pointer is used for both); otherwise rd and wr are distinct buffers.
template <bool INPLACE, class ST, class Rhs>
__device__ __forceinline__ void twisted_half(const ST* __restrict__ rd, ST* __restrict__ wr,
                                             long sj, int M, int half, bool act,
                                             const double* __restrict__ cp, size_t ncls, Rhs rhs) {
    const int m = (M + 1) / 2;
    const int nr = act ? (half ? M - m : m) : 0;      // rows eliminated by this lane
    const int j0 = half ? M : 1;                       // row of step 0 (the wall end)
    const int jd = half ? -1 : 1;
    const long dj = jd * sj;
    ST* wb = wr + (long)j0 * sj;
    const ST* rb = INPLACE ? wb : rd + (long)j0 * sj;
    constexpr int CH = 8;
    double fv[CH], cv[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        fv[u] = (u < nr) ? rhs(j0 + u * jd, ld(rb + u * dj)) : 0.0;
        cv[u] = (u < nr) ? cp[(size_t)u * ncls] : 0.0;
    }
    double acc = 0.0, clast = 0.0;
    for (int s0 = 0; s0 < nr; s0 += CH) {
        double nf[CH], nc[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int sn = s0 + CH + u;
            nf[u] = (sn < nr) ? rhs(j0 + sn * jd, ld(rb + sn * dj)) : 0.0;
            nc[u] = (sn < nr) ? cp[(size_t)sn * ncls] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (s0 + u < nr) {
                acc = cv[u] * (fv[u] - acc);
                clast = cv[u];
                st(wb + (s0 + u) * dj, acc);
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            fv[u] = nf[u];
            cv[u] = nc[u];
        }
    }
    // interface: top lane holds (d'_m, c'_m), bottom lane (g'_{m+1}, e'_{m+1}); a lane with no
    // rows contributes (0, 0), i.e. the wall value U = 0.
    const double oacc = __shfl_xor(acc, 1, 64);
    const double oc = __shfl_xor(clast, 1, 64);
    if (nr == 0) return;
    const double dm = half ? oacc : acc, cm = half ? oc : clast;
    const double gm = half ? acc : oacc, em = half ? clast : oc;
    const double Um = (dm - cm * gm) / (1.0 - cm * em);
    double unext = half ? (gm - em * Um) : Um;        // U at this lane's last row
    st(wb + (nr - 1) * dj, unext);
    // back substitution from step nr-2 towards the wall: U = d' - c' U_next
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const int sn = nr - 2 - u;
        fv[u] = (sn >= 0) ? ld(wb + sn * dj) : 0.0;
        cv[u] = (sn >= 0) ? cp[(size_t)(sn >= 0 ? sn : 0) * ncls] : 0.0;
    }
    for (int s0 = nr - 2; s0 >= 0; s0 -= CH) {
        double nf[CH], nc[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int sn = s0 - CH - u;
            nf[u] = (sn >= 0) ? ld(wb + sn * dj) : 0.0;
            nc[u] = (sn >= 0) ? cp[(size_t)(sn >= 0 ? sn : 0) * ncls] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (s0 - u >= 0) {
                unext = fv[u] - cv[u] * unext;
                st(wb + (s0 - u) * dj, unext);
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            fv[u] = nf[u];
            cv[u] = nc[u];
        }
    }
}

struct ModeLane {
    int p, q, half;
    bool act;
    const double* cp;
    size_t ncls;
    long off;   // offset of the (p, row 0, q) element
};

__device__ __forceinline__ ModeLane mode_lane(const Dims& d, const double* __restrict__ tri) {
    ModeLane ml;
    const int t = blockIdx.x * 64 + threadIdx.x;
    const int pair = t >> 1;
    ml.half = t & 1;
    ml.act = pair < d.nx * d.nz;
    const int pp = ml.act ? pair : 0;
    ml.p = pp / d.nz;
    ml.q = pp - ml.p * d.nz;
    const int pc = min(ml.p, d.nx - ml.p);
    const int qc = min(ml.q, d.nz - ml.q);
    ml.ncls = (size_t)(d.nx / 2 + 1) * (d.nz / 2 + 1);
    ml.cp = tri + (size_t)(pc * (d.nz / 2 + 1) + qc);
    ml.off = (long)ml.p * d.ny * d.nz + ml.q;
    return ml;
}

// tridiag_y: one Poisson problem per component blockIdx.y: f_j = scale * B_j (B = the 2D
// Hartley spectrum of the right-hand side, scale = h^2/(nx nz)), in place.
// wlo, whi: wall terms folded into mode (0, 0) (zero when the right-hand side holds them).
template <class ST>
__global__ __launch_bounds__(64) void k_tridiag_y(Dims d, const double* __restrict__ tri,
                                                 SPtr3<ST> spec, const int* gate, double scale,
                                                 double3 wlo, double3 whi) {
    if (gate && *gate) return;
    const ModeLane ml = mode_lane(d, tri);
    const int c = blockIdx.y;
    ST* col = spec.p[c] + ml.off;
    const bool m00 = (ml.p == 0 && ml.q == 0);
    const double a = c == 0 ? wlo.x : (c == 1 ? wlo.y : wlo.z);
    const double b = c == 0 ? whi.x : (c == 1 ? whi.y : whi.z);
    const int M = d.M;
    twisted_half<true, ST>(nullptr, col, d.nz, d.M, ml.half, ml.act, ml.cp, ml.ncls,
                           [&](int j, double v) {
                               double f = scale * v;
                               if (m00) {
                                   if (j == 1) f -= a;
                                   if (j == M) f -= b;
                               }
                               return f;
                           });
}

// tridiag_psi: the stream-vector problem lap psi = -w from the vorticity modes U_w = T w/(nx nz)
// left in spec by tridiag_y (T the 2D Hartley transform): its transformed right-hand side is
// -(nx nz) U_w minus the wall terms, whose transform for wall values constant over each wall
// plane lives only in mode (0, 0):
//   f_j = -h^2 U_w(j) - [p = q = 0] ([j = 1] psi_lo + [j = M] psi_hi);
// solved into spec2, leaving spec unchanged.
template <class ST>
__global__ __launch_bounds__(64) void k_tridiag_psi(Dims d, const double* __restrict__ tri,
                                                   SPtr3<ST> spec, SPtr3<ST> spec2, double3 plo,
                                                   double3 phi_) {
    const ModeLane ml = mode_lane(d, tri);
    const int c = blockIdx.y;
    const ST* col = spec.p[c] + ml.off;
    ST* col2 = spec2.p[c] + ml.off;
    const bool m00 = (ml.p == 0 && ml.q == 0);
    const double wlo = c == 0 ? plo.x : (c == 1 ? plo.y : plo.z);
    const double whi = c == 0 ? phi_.x : (c == 1 ? phi_.y : phi_.z);
    const double h2 = d.h * d.h;
    const int M = d.M;
    twisted_half<false, ST>(col, col2, d.nz, d.M, ml.half, ml.act, ml.cp, ml.ncls, [&](int j, double v) {
        double f = -h2 * v;
        if (m00) {
            if (j == 1) f -= wlo;
            if (j == M) f -= whi;
        }
        return f;
    });
}

// ---------------------------------------------------------------- segmented tridiagonal solve
// Partition solve of T x = f for one mode, T = tridiag(1, beta, 1) of size M with zero ends
// (the walls are folded into f). The column is cut into S consecutive segments, one lane each;
// a segment of L rows lives in registers. A 256-lane block owns 256/S consecutive modes, and
// its lanes are ordered mode-fastest, so each wave holds consecutive modes (consecutive q of
// one spectral row) of one or more segments and every row load or store covers whole runs.
// With G = T_L^{-1}, segment k obeys x_k = G (f_k - E_{k-1} e_1 - F_{k+1} e_L), where F_k, E_k
// are the first and last unknowns of segment k (E_{-1} = F_S = 0). Its ends give the coupled
// relations  F_k = p_k - g11 E_{k-1} - g1L F_{k+1},  E_k = q_k - g1L E_{k-1} - g11 F_{k+1}
// (p, q: ends of G f_k; g11 = G_11 = G_LL, g1L = G_1L = G_L1 since T_L is symmetric and
// persymmetric). A forward sweep over the segments, E_k = a_k - b_k F_{k+1},
// F_k = phi_k - chi_k F_{k+1}, and the back sweep both run redundantly in every lane of the
// mode, after the segment ends are exchanged through LDS. The segment is then finished from
// its forward-eliminated rows d'_j:
// the corrections of f enter d' as -E_{k-1} pi_j (pi = forward elimination of e_1) and
// -F_{k+1} c'_L at the last row. Pivots c'_j = 1/(beta - c'_{j-1}) come from the class table,
// so no lane divides in the row loops; beta itself is the table's last row.
//
// Segments have Lm rows (the first nlong of them) or Lm - 1 rows. Every lane walks Lm rows so
// that the row loops depend on wave-uniform values only; a short segment's extra last row is a
// phantom whose value is forced to zero by selects on the last two rows.
// Buffer-instruction access for the segmented solve (see seg_load).
typedef __amdgpu_buffer_rsrc_t BufRes;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ BufRes buf_res(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ double buf_ld(BufRes r, unsigned voff, unsigned soff, const double*) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ double buf_ld(BufRes r, unsigned voff, unsigned soff, const float*) {
    return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st(BufRes r, unsigned voff, unsigned soff, double v, double*) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_st(BufRes r, unsigned voff, unsigned soff, double v, float*) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)v), r, voff, soff, 0);
}

template <int LMAX>
struct SegCoef {
    double c[LMAX];
    double beta, g11l, g11s, g1ll, g1ls;   // G_11 and G_1L for Lm and Lm - 1 rows
};

template <int LMAX>
__device__ __forceinline__ void seg_coef(SegCoef<LMAX>& cf, const double* __restrict__ tri,
                                         unsigned cls, unsigned ncls, int M, int Lm) {
    const BufRes r = buf_res(tri, (unsigned)(M + 1) * ncls * 8u);
#pragma unroll
    for (int u = 0; u < LMAX; ++u) cf.c[u] = (u < Lm) ? buf_ld(r, cls * 8u, u * ncls * 8u, tri) : 0.0;
    cf.beta = buf_ld(r, cls * 8u, (unsigned)M * ncls * 8u, tri);
    // G_11(L) = c'_L; G_1L(L) = (-1)^(L-1) c'_1 ... c'_L
    double prod = 1.0;
    cf.g11l = cf.g11s = cf.g1ll = cf.g1ls = 0.0;
#pragma unroll
    for (int u = 0; u < LMAX; ++u) {
        if (u < Lm) {
            prod *= -cf.c[u];
            if (u == Lm - 2) {
                cf.g1ls = -prod;
                cf.g11s = cf.c[u];
            }
            if (u == Lm - 1) {
                cf.g1ll = -prod;
                cf.g11l = cf.c[u];
            }
        }
    }
}

// xch: 512 doubles of LDS for the exchange of the segment ends; every thread of the 256-thread
// block calls this (it holds two barriers).
template <int S, int LMAX>
__device__ __forceinline__ void seg_solve(double (&x)[LMAX], const SegCoef<LMAX>& cf, int k,
                                          bool shortl, int Lm, int nlong, double* xch) {
    const double* c = cf.c;
    // forward elimination in place; q = last d', piL = pi at the last row (phantom row zeroed)
    double acc = 0.0, pi = 0.0, q = 0.0, piL = 0.0;
#pragma unroll
    for (int u = 0; u < LMAX; ++u) {
        if (u < Lm) {
            acc = c[u] * (x[u] - acc);
            pi = (u == 0) ? c[0] : -c[u] * pi;
            if (u == Lm - 2) {
                q = acc;
                piL = pi;
            }
            if (u == Lm - 1) {
                q = shortl ? q : acc;
                piL = shortl ? piL : pi;
                x[u] = shortl ? 0.0 : acc;
            } else {
                x[u] = acc;
            }
        }
    }
    // p = first unknown of the zero-end segment solve (back substitution, nothing stored)
    double p = 0.0;
#pragma unroll
    for (int u = LMAX - 1; u >= 0; --u)
        if (u < Lm) p = x[u] - c[u] * p;
    // reduced system. Every segment's p and q are gathered first (through LDS: the S lanes of
    // a mode sit 256/S lanes apart); every lane then runs the forward sweep and the back
    // substitution of the whole reduced system itself, keeping phi and chi of every segment,
    // so no value has to travel between lanes after the gather.
    constexpr int NM = 256 / S;
    const int m = (int)threadIdx.x % NM;
    xch[threadIdx.x] = p;
    xch[256 + threadIdx.x] = q;
    __syncthreads();
    double P[S], Q[S];
#pragma unroll
    for (int kk = 0; kk < S; ++kk) {
        P[kk] = xch[kk * NM + m];
        Q[kk] = xch[256 + kk * NM + m];
    }
    __syncthreads();   // xch is free again
    double a = 0.0, b = 0.0, alp = 0.0, bep = 0.0;
    double PH[S], CH[S];
#pragma unroll
    for (int kk = 0; kk < S; ++kk) {
        const bool lng = nlong == 0 || kk < nlong;   // nlong = 0: all segments have Lm rows
        const double g11 = lng ? cf.g11l : cf.g11s;
        const double g1l = lng ? cf.g1ll : cf.g1ls;
        const double rden = 1.0 / (1.0 - g11 * b);
        const double ph = (P[kk] - g11 * a) * rden;
        const double ch = g1l * rden;
        const double an = Q[kk] - g1l * a + g1l * b * ph;
        const double bn = g11 + g1l * b * ch;
        PH[kk] = ph;
        CH[kk] = ch;
        if (kk == k - 1) {   // alpha, beta of the segment before this lane's
            alp = an;
            bep = bn;
        }
        a = an;
        b = bn;
    }
    // back substitution F_kk = phi_kk - chi_kk F_{kk+1} (F_S = 0); this lane keeps F_k, F_{k+1}
    double F = 0.0, Fk = 0.0, Fnext = 0.0;
#pragma unroll
    for (int kk = S - 1; kk >= 0; --kk) {
        if (kk == k) Fnext = F;
        F = PH[kk] - CH[kk] * F;
        if (kk == k) Fk = F;
    }
    // E_{k-1} = alpha_{k-1} - beta_{k-1} F_k
    const double Eprev = k > 0 ? alp - bep * Fk : 0.0;
    // finish the segment bottom up
    double xn = 0.0, pc = 0.0;
#pragma unroll
    for (int u = LMAX - 1; u >= 0; --u) {
        if (u < Lm) {
            double f;
            if (u == Lm - 1) {
                pc = shortl ? 0.0 : piL;
                f = shortl ? 0.0 : Fnext * c[u];
            } else if (u == Lm - 2) {
                pc = shortl ? piL : -pc * (cf.beta - c[u]);
                f = shortl ? Fnext * c[u] : 0.0;
            } else {
                pc = -pc * (cf.beta - c[u]);
                f = 0.0;
            }
            xn = (x[u] - Eprev * pc - f) - c[u] * xn;
            x[u] = xn;
        }
    }
}

template <int S>
struct SegLane {
    int p, q, k, Lm, nlong;
    int a;          // first interior row (0-based) of the lane's segment
    bool act, shortl;
    unsigned cls, ncls;
    unsigned off;   // offset of (p, first row of the segment, q); grids stay below 2^31 nodes
};

template <int S>
__device__ __forceinline__ SegLane<S> seg_lane(const Dims& d) {
    SegLane<S> sl;
    // a block owns 256/S consecutive modes; lane t of the block takes mode t % (256/S) and
    // segment t / (256/S), so the lanes of a wave hold consecutive modes (consecutive q) of
    // one or two segments, and a row's loads and stores cover whole runs of a spectral row
    constexpr int NM = 256 / S;
    const int mode = (int)blockIdx.x * NM + (int)threadIdx.x % NM;
    sl.k = (int)threadIdx.x / NM;
    sl.act = mode < d.nx * d.nz;
    const int mm = sl.act ? mode : 0;
    sl.p = mm / d.nz;
    sl.q = mm - sl.p * d.nz;
    const int base = d.M / S;
    sl.nlong = d.M - base * S;
    sl.Lm = base + (sl.nlong > 0);
    sl.shortl = sl.nlong > 0 && sl.k >= sl.nlong;
    const int a = sl.k * base + min(sl.k, sl.nlong);
    sl.a = a;
    const int pc = min(sl.p, d.nx - sl.p);
    const int qc = min(sl.q, d.nz - sl.q);
    sl.ncls = (unsigned)((d.nx / 2 + 1) * (d.nz / 2 + 1));
    sl.cls = (unsigned)(pc * (d.nz / 2 + 1) + qc);
    sl.off = (unsigned)(sl.p * d.ny * d.nz + (1 + a) * d.nz + sl.q);
    return sl;
}

// Segment rows go through buffer instructions: one buffer resource per array (wave-uniform),
// the lane's 32-bit byte offset in a VGPR and the row offset u * sj in an SGPR, so no lane
// keeps an address per row. Accesses beyond the array's extent read zero and drop stores.
// A short segment's phantom row reads the next segment's first row, or the wall row
// j = ny-1: in bounds, and zeroed by the solve.
template <int S, int LMAX, class ST>
__device__ __forceinline__ void seg_load(double (&x)[LMAX], const ST* base, unsigned nelem,
                                         unsigned off, unsigned sj, int Lm, double scale) {
    const BufRes r = buf_res(base, nelem * (unsigned)sizeof(ST));
    const unsigned vo = off * (unsigned)sizeof(ST);
#pragma unroll
    for (int u = 0; u < LMAX; ++u)
        x[u] = (u < Lm) ? scale * buf_ld(r, vo, u * sj * (unsigned)sizeof(ST), base) : 0.0;
}

template <int S, int LMAX, class ST>
__device__ __forceinline__ void seg_store(const double (&x)[LMAX], ST* base, unsigned nelem,
                                          unsigned sj, const SegLane<S>& sl) {
    const BufRes r = buf_res(base, nelem * (unsigned)sizeof(ST));
    const unsigned vo = sl.off * (unsigned)sizeof(ST);
    if (!sl.act) return;
#pragma unroll
    for (int u = 0; u < LMAX; ++u) {
        const unsigned so = u * sj * (unsigned)sizeof(ST);
        if (u < sl.Lm - 1) buf_st(r, vo, so, x[u], base);
        if (u == sl.Lm - 1 && !sl.shortl) buf_st(r, vo, so, x[u], base);
    }
}

// Segmented tridiag_y: f_j = scale * B_j per component blockIdx.y, solved in place.
// LMF, NLF: the segment length Lm and long-segment count nlong fixed at compile time for the
// common row counts (LMF = 0: taken from M at run time).
template <int S, int LMAX, class ST, int LMF, int NLF>
__global__ __launch_bounds__(256) void k_tridiag_seg(Dims d, const double* __restrict__ tri,
                                                    SPtr3<ST> spec, const int* gate, double scale) {
    if (gate && *gate) return;
    SegLane<S> sl = seg_lane<S>(d);
    if (LMF) {
        sl.Lm = LMF;
        sl.nlong = NLF;
        sl.shortl = NLF > 0 && sl.k >= NLF;
    }
    __shared__ double xch[512];
    SegCoef<LMAX> cf;
    seg_coef<LMAX>(cf, tri, sl.cls, sl.ncls, d.M, sl.Lm);
    ST* col = spec.p[blockIdx.y];
    const unsigned N = (unsigned)(d.nx * d.ny * d.nz);
    double x[LMAX];
    seg_load<S, LMAX, ST>(x, col, N, sl.off, d.nz, sl.Lm, scale);
    seg_solve<S, LMAX>(x, cf, sl.k, sl.shortl, sl.Lm, sl.nlong, xch);
    seg_store<S, LMAX, ST>(x, col, N, d.nz, sl);
}

// Segmented vorticity + stream-vector pair: the vorticity modes U_w (f = scale * B) are solved
// and stored in spec, then the stream-vector problem lap psi = -w is solved from them in
// registers, f_j = -h^2 U_w(j) - [p = q = 0]([j = 1] psi_lo + [j = M] psi_hi), into spec2.
// triw holds the vorticity's pivots: tri itself, or those of the shifted operator L_h - a of
// the inertial variant (SM eq. (36)).
template <int S, int LMAX, class ST, int LMF, int NLF>
__global__ __launch_bounds__(256) void k_tridiag_pair_seg(Dims d, const double* __restrict__ tri,
                                                         const double* __restrict__ triw,
                                                         SPtr3<ST> spec, SPtr3<ST> spec2,
                                                         double3 olo, double3 ohi, double3 plo,
                                                         double3 phi_, double scale) {
    SegLane<S> sl = seg_lane<S>(d);
    if (LMF) {
        sl.Lm = LMF;
        sl.nlong = NLF;
        sl.shortl = NLF > 0 && sl.k >= NLF;
    }
    const int c3 = blockIdx.y;
    __shared__ double xch[512];
    SegCoef<LMAX> cf;
    seg_coef<LMAX>(cf, triw, sl.cls, sl.ncls, d.M, sl.Lm);
    ST* col = spec.p[c3];
    const unsigned N = (unsigned)(d.nx * d.ny * d.nz);
    double x[LMAX];
    seg_load<S, LMAX, ST>(x, col, N, sl.off, d.nz, sl.Lm, scale);
    const bool m00 = sl.p == 0 && sl.q == 0;
    // the row j = M is the last real row of segment S - 1 (short if nlong > 0)
    const int ulast = sl.nlong > 0 ? sl.Lm - 2 : sl.Lm - 1;
    {
        // vorticity wall terms, constant over each wall plane: mode (0, 0) only
        const double a = c3 == 0 ? olo.x : (c3 == 1 ? olo.y : olo.z);
        const double b = c3 == 0 ? ohi.x : (c3 == 1 ? ohi.y : ohi.z);
#pragma unroll
        for (int u = 0; u < LMAX; ++u) {
            if (m00 && sl.k == 0 && u == 0) x[u] -= a;
            if (m00 && sl.k == S - 1 && u == ulast) x[u] -= b;
        }
    }
    seg_solve<S, LMAX>(x, cf, sl.k, sl.shortl, sl.Lm, sl.nlong, xch);
    seg_store<S, LMAX, ST>(x, col, N, d.nz, sl);
    // the stream-vector problem has no shift: its own pivots when the vorticity's differ
    if (triw != tri) seg_coef<LMAX>(cf, tri, sl.cls, sl.ncls, d.M, sl.Lm);
    const double h2 = d.h * d.h;
    const double wlo = c3 == 0 ? plo.x : (c3 == 1 ? plo.y : plo.z);
    const double whi = c3 == 0 ? phi_.x : (c3 == 1 ? phi_.y : phi_.z);
#pragma unroll
    for (int u = 0; u < LMAX; ++u) {
        double f = -h2 * x[u];
        if (m00 && sl.k == 0 && u == 0) f -= wlo;
        if (m00 && sl.k == S - 1 && u == ulast) f -= whi;
        x[u] = f;
    }
    seg_solve<S, LMAX>(x, cf, sl.k, sl.shortl, sl.Lm, sl.nlong, xch);
    seg_store<S, LMAX, ST>(x, spec2.p[c3], N, d.nz, sl);
}

// dht_z_out: Hartley along z of the solved modes, then u = result (add = 0) or u += result.
template <class ST>
__global__ __launch_bounds__(kBlock) void k_dht_z_out(Dims d, FftPlan pz,
                                                     const double2* __restrict__ tw, SPtr3<ST> spec,
                                                     Ptr3 u, int add, const int* gate, int rpb) {
    if (gate && *gate) return;
    __shared__ double2 A[kTileElems];
    const int n = d.nz;
    const int nlines = rpb >> 1;
    const int c = blockIdx.y;
    const int nrows = d.nx * d.M;
    const int r0 = blockIdx.x * rpb;
    const ST* sc = spec.p[c];
    for (int e = threadIdx.x; e < rpb * n; e += blockDim.x) {
        const int lr = e / n;
        const int k = e - lr * n;
        const int r = r0 + lr;
        double v = 0.0;
        if (r < nrows) {
            const int i = r / d.M;
            const int j = 1 + (r - i * d.M);
            v = ld(sc + node(d, i, j, k));
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

// ---------------------------------------------------------------------------------------
// Two-pass register transforms for line lengths n = B * A (B in {8, 16}; A in {3, 4, 6, 8,
// 12, 16}). One 64-lane wave per block handles L = 64 / A complex lines (2L real lines):
//  pass 1: item (line, k1), k1 < A: DFT_B over k2 of x[k1 + A k2] loaded from global memory,
//          twiddle exp(-2 pi i k1 p2 / n), store Y[line][p2][k1] in LDS (padded rows);
//  pass 2: item (line, s), s < B/2, owns the mode pair p2 = {s, B - s} ({0, B/2} for s = 0):
//          DFT_A over k1 for both, giving X[p2 + B p1]; every X_p and its partner X_{n-p}
//          sit in the same item, so both Hartley values are formed in registers and stored.
template <int B, int A>
struct TwoPass {
    static constexpr int N = B * A;
    static constexpr int L = (64 / A) > 0 ? (64 / A) : 1;
    static constexpr int RS = A + 1;             // padded row of Y
    static constexpr int LS = B * RS + 1;        // padded line of Y
    static constexpr int LDS = L * LS;           // double2 elements
};

// Prep: Pre prep(line) (per-line row offsets, computed once per item).
// Loader: double2 load(pre, k1, k2) -> (line a value, line b value) at position k1 + A k2.
// Storer: void store(pre, p, ha, hb).
template <int B, int A, bool LINE_FAST, class Prep, class Load, class Store>
__device__ __forceinline__ void two_pass_hartley(double2* Y, const double2* __restrict__ tw,
                                                 Prep prep, Load load, Store store) {
    using P = TwoPass<B, A>;
    constexpr int L = P::L;
#pragma unroll 1
    for (int it = threadIdx.x; it < L * A; it += 64) {
        const int line = LINE_FAST ? (it % L) : (it / A);
        const int k1 = LINE_FAST ? (it / L) : (it % A);
        const auto pre = prep(line);
        double2 x[B];
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) x[k2] = load(pre, k1, k2);
        fftr::DFT<B>::run(x);
#pragma unroll
        for (int p2 = 1; p2 < B; ++p2) x[p2] = cmul(x[p2], tw[k1 * p2]);
        double2* Yl = Y + line * P::LS + k1;
#pragma unroll
        for (int p2 = 0; p2 < B; ++p2) Yl[p2 * P::RS] = x[p2];
    }
    __syncthreads();
#pragma unroll 1
    for (int it = threadIdx.x; it < L * (B / 2); it += 64) {
        const int line = LINE_FAST ? (it % L) : (it / (B / 2));
        const int s = LINE_FAST ? (it / L) : (it % (B / 2));
        const auto pre = prep(line);
        const int pa = s;                          // s = 0 gives p2 = 0
        const int pb = (s == 0) ? B / 2 : B - s;
        double2* Ya = Y + line * P::LS + pa * P::RS;
        const double2* Yb = Y + line * P::LS + pb * P::RS;
        if constexpr (A >= 16) {
            // long lines: the a-line's transform goes back to its own LDS row (no other lane
            // reads it), so only one line of registers is live at a time
            double2 x[A];
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) x[k1] = Ya[k1];
            fftr::DFT<A>::run(x);
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) Ya[k1] = x[k1];
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) x[k1] = Yb[k1];
            fftr::DFT<A>::run(x);
#pragma unroll
            for (int p1 = 0; p1 < A; ++p1) {
                const double2 za = Ya[p1];
                const double2 ma = (s == 0) ? Ya[(A - p1) % A] : x[A - 1 - p1];
                store(pre, pa + B * p1, 0.5 * (za.x + ma.x - za.y + ma.y), 0.5 * (za.x - ma.x + za.y + ma.y));
                const double2 zb = x[p1];
                const double2 mb = (s == 0) ? x[A - 1 - p1] : Ya[A - 1 - p1];
                store(pre, pb + B * p1, 0.5 * (zb.x + mb.x - zb.y + mb.y), 0.5 * (zb.x - mb.x + zb.y + mb.y));
            }
        } else {
            double2 xa[A], xb[A];
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) {
                xa[k1] = Ya[k1];
                xb[k1] = Yb[k1];
            }
            fftr::DFT<A>::run(xa);
            fftr::DFT<A>::run(xb);
#pragma unroll
            for (int p1 = 0; p1 < A; ++p1) {
                const double2 za = xa[p1];
                const double2 ma = (s == 0) ? xa[(A - p1) % A] : xb[A - 1 - p1];
                store(pre, pa + B * p1, 0.5 * (za.x + ma.x - za.y + ma.y), 0.5 * (za.x - ma.x + za.y + ma.y));
                const double2 zb = xb[p1];
                const double2 mb = (s == 0) ? xb[A - 1 - p1] : xa[A - 1 - p1];
                store(pre, pb + B * p1, 0.5 * (zb.x + mb.x - zb.y + mb.y), 0.5 * (zb.x - mb.x + zb.y + mb.y));
            }
        }
    }
}

// Node offsets of the first z node of interior rows r and r+1 (r = i*M + j-1), -1 if past
// the last row.
struct RowPair {
    int a, b;
};
__device__ __forceinline__ int row_base(const Dims& d, int r, int nrows) {
    if (r >= nrows) return -1;
    const int i = r / d.M;
    return node(d, i, 1 + (r - i * d.M), 0);
}

// Component c of the right-hand side minus the wall terms (correct = 0) or minus L_h u
// (correct = 1), for the z index k of an interior row with node offset rb = node(i, j, 0) and
// x-neighbour row offsets xpb, xmb.
__device__ __forceinline__ double rhs_row(const RhsArgs& a, const Dims& d, const double* __restrict__ uc,
                                          int c, int correct, int rb, int xpb, int xmb, int j, int k) {
    const int c0 = rb + k;
    double b = rhs_val(a, c, c0);
    if (correct) {
        const int kp = (k + 1 == d.nz) ? 0 : k + 1;
        const int km = (k == 0) ? d.nz - 1 : k - 1;
        b -= (uc[xpb + k] + uc[xmb + k] + uc[c0 + d.nz] + uc[c0 - d.nz] + uc[rb + kp] + uc[rb + km] -
              6.0 * uc[c0]) * d.inv_h2;
    } else {
        double w = 0.0;
        if (j == 1) w += uc[c0 - d.nz];
        if (j == d.M) w += uc[c0 + d.nz];
        b -= w * d.inv_h2;
    }
    return b;
}

// rhs_dht_z, two-pass form: block = (2L consecutive interior rows, component c), blocks
// ordered per XCD. The right-hand side (a stencil for the vorticity source, the wall terms
// or the residual) is first evaluated with lane-consecutive z indices (coalesced) into the
// LDS tile, then pass 1 reads its strided inputs from there.
template <int B, int A, class ST>
__global__ __launch_bounds__(64) void k_rhs_hz(Dims d, const double2* __restrict__ tw,
                                              RhsArgs rhs, CPtr3 u, int correct, SPtr3<ST> spec,
                                              const int* gate) {
    if (gate && *gate) return;
    using P = TwoPass<B, A>;
    constexpr int N = P::N;
    constexpr int L = P::L;
    static_assert(L * N <= P::LDS, "input tile must fit in the exchange buffer");
    static_assert(L * A <= 64, "one pass-1 round per lane");
    __shared__ double2 Y[P::LDS];
    // Only the residual form (a stencil of u) benefits from XCD-ordered blocks; the pointwise
    // form keeps the hardware order (neighbouring rows stream together).
    const int gx = gridDim.x;
    const int lb = correct ? xcd_block(blockIdx.x + gx * blockIdx.y, gx * gridDim.y)
                           : (int)(blockIdx.x + gx * blockIdx.y);
    const int c = lb / gx;
    const int bx = lb - c * gx;
    const int nrows = d.nx * d.M;
    const int r0 = bx * 2 * L;
    const double* uc = u.p[c];
    ST* sc = spec.p[c];
    auto prep = [&](int ln) -> RowPair {
        return RowPair{row_base(d, r0 + 2 * ln, nrows), row_base(d, r0 + 2 * ln + 1, nrows)};
    };
    auto store = [&](const RowPair& rp, int p, double ha, double hb) {
        if (rp.a >= 0) st(sc + rp.a + p, ha);
        if (rp.b >= 0) st(sc + rp.b + p, hb);
    };
    if (!correct) {
        // b - wall terms: a pointwise read plus, on the first and last interior rows, the
        // wall row of u; pass 1 loads it directly. Per line: row offsets and wall flags
        // (bit 0: row j = 1 borders the y = 0 wall, bit 1: row j = M borders y = H).
        const double sg = (rhs.mode == RHS_NEGW) ? -1.0 : 1.0;
        const double* fc = rhs.f[c];
        auto prepw = [&](int ln) -> int4 {
            int4 o;
            const int ra = r0 + 2 * ln, rbb = ra + 1;
            o.x = row_base(d, ra, nrows);
            o.y = row_base(d, rbb, nrows);
            const int ja = 1 + (ra - (ra / d.M) * d.M), jb = 1 + (rbb - (rbb / d.M) * d.M);
            o.z = (ja == 1 ? 1 : 0) | (ja == d.M ? 2 : 0);
            o.w = (jb == 1 ? 1 : 0) | (jb == d.M ? 2 : 0);
            return o;
        };
        auto rowval = [&](int rb, int fl, int k) -> double {
            if (rb < 0) return 0.0;
            double b = sg * fc[rb + k];
            if (fl & 1) b -= uc[rb - d.nz + k] * d.inv_h2;
            if (fl & 2) b -= uc[rb + d.nz + k] * d.inv_h2;
            return b;
        };
        auto load = [&](const int4& o, int k1, int k2) -> double2 {
            const int k = k1 + A * k2;
            return make_double2(rowval(o.x, o.z, k), rowval(o.y, o.w, k));
        };
        auto storew = [&](const int4& o, int p, double ha, double hb) {
            if (o.x >= 0) st(sc + o.x + p, ha);
            if (o.y >= 0) st(sc + o.y + p, hb);
        };
        two_pass_hartley<B, A, false>(Y, tw, prepw, load, storew);
        return;
    }
#pragma unroll 4
    for (int lr = 0; lr < 2 * L; ++lr) {
        const int r = r0 + lr;
        double2* row = &Y[(lr >> 1) * N];
        if (r < nrows) {
            const int i = r / d.M;
            const int j = 1 + (r - i * d.M);
            const int ip = (i + 1 == d.nx) ? 0 : i + 1;
            const int im = (i == 0) ? d.nx - 1 : i - 1;
            const int rb = node(d, i, j, 0), xpb = node(d, ip, j, 0), xmb = node(d, im, j, 0);
#pragma unroll
            for (int k = threadIdx.x; k < N; k += 64)
                set_part(&row[k], lr & 1, rhs_row(rhs, d, uc, c, 1, rb, xpb, xmb, j, k));
        } else {
#pragma unroll
            for (int k = threadIdx.x; k < N; k += 64) set_part(&row[k], lr & 1, 0.0);
        }
    }
    __syncthreads();
    double2 xin[B];
    const int it = threadIdx.x;
    const bool act = it < L * A;
    const int line = act ? it / A : 0, k1 = act ? it % A : 0;
    if (act) {
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) xin[k2] = Y[line * N + k1 + A * k2];
    }
    __syncthreads();
    auto load = [&](const RowPair&, int, int k2) -> double2 { return xin[k2]; };
    two_pass_hartley<B, A, false>(Y, tw, prep, load, store);
}

// dht_x, two-pass form: block = (2L consecutive z-modes q, interior row j, component c);
// lines are the q-pairs (q, q+1), read and written as one 16-byte value.
// NC: the component count of the launch (3, or 6 for the vorticity and stream-vector fields
// together); the code is the same, the symbol tells the two launches apart in traces.
template <int B, int A, class ST, int NC>
__global__ __launch_bounds__(64) void k_hx(Dims d, const double2* __restrict__ tw, SPtr6<ST> spec,
                                          const int* gate) {
    if (gate && *gate) return;
    using P = TwoPass<B, A>;
    __shared__ double2 Y[P::LDS];
    const int c = blockIdx.z;
    const int j = 1 + blockIdx.y;
    const int q0 = blockIdx.x * 2 * P::L;
    ST* s = spec.p[c];
    const int pstride = d.ny * d.nz;
    auto prep = [&](int line) -> int {
        const int q = q0 + 2 * line;
        return q < d.nz ? j * d.nz + q : -1;
    };
    auto load = [&](int o, int k1, int k2) -> double2 {
        if (o < 0) return make_double2(0.0, 0.0);
        return ld2(s + o + (k1 + A * k2) * pstride);
    };
    auto store = [&](int o, int p, double ha, double hb) {
        if (o >= 0) st2(s + o + p * pstride, ha, hb);
    };
    two_pass_hartley<B, A, true>(Y, tw, prep, load, store);
}

// dht_z_out, two-pass form: block = (2L consecutive interior rows, component c).
// NC as for k_hx.
template <int B, int A, class ST, int NC>
__global__ __launch_bounds__(64) void k_hz_out(Dims d, const double2* __restrict__ tw, SPtr6<ST> spec,
                                              Ptr6 u, int add, const int* gate) {
    if (gate && *gate) return;
    using P = TwoPass<B, A>;
    __shared__ double2 Y[P::LDS];
    const int c = blockIdx.y;
    const int nrows = d.nx * d.M;
    const int r0 = blockIdx.x * 2 * P::L;
    const ST* sc = spec.p[c];
    double* uc = u.p[c];
    auto prep = [&](int line) -> RowPair {
        return RowPair{row_base(d, r0 + 2 * line, nrows), row_base(d, r0 + 2 * line + 1, nrows)};
    };
    auto load = [&](const RowPair& rp, int k1, int k2) -> double2 {
        const int k = k1 + A * k2;
        return make_double2(rp.a >= 0 ? ld(sc + rp.a + k) : 0.0, rp.b >= 0 ? ld(sc + rp.b + k) : 0.0);
    };
    auto store = [&](const RowPair& rp, int p, double ha, double hb) {
        if (rp.a >= 0) {
            double* dst = uc + rp.a + p;
            *dst = add ? *dst + ha : ha;
        }
        if (rp.b >= 0) {
            double* dst = uc + rp.b + p;
            *dst = add ? *dst + hb : hb;
        }
    };
    two_pass_hartley<B, A, false>(Y, tw, prep, load, store);
}

// Two-pass shape (B, A) for a line length, or (0, 0) if the LDS Stockham path is used.
void two_pass_shape(int n, int& B, int& A) {
    B = 16;
    switch (n) {
        case 32: B = 8; A = 4; return;
        case 48: A = 3; return;
        case 64: A = 4; return;
        case 96: A = 6; return;
        case 128: A = 8; return;
        case 192: A = 12; return;
        case 256: A = 16; return;
        default: B = 0; A = 0; return;
    }
}

#define VS_TWO_PASS_CASES(X) X(8, 4) X(16, 3) X(16, 4) X(16, 6) X(16, 8) X(16, 12) X(16, 16)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// resid_norm: block partials of sum (b - L_h u)_c^2 and sum b~_c^2 over the interior. A block
// owns one component c and a slab of ci consecutive x-planes; each thread owns one interior
// (j, k) and walks the slab with u_c at x-1 and x kept in registers, so one new centre value
// is read per plane. Blocks are ordered per XCD. Streaming a single component (u_c and b_c)
// per block keeps two arrays in flight per wave instead of six, which runs close to the copy
// rate where reading every component at each node does not.
__global__ __launch_bounds__(kBlock) void k_resid_norm(Dims d, RhsArgs rhs, CPtr3 u, int ncomp,
                                                      SlabGrid sg, double* __restrict__ partials,
                                                      const int* gate, int slot0) {
    if (gate && *gate) return;
    __shared__ double sh[2 * 4];
    const int nb = sg.gx * sg.gi;
    const int lb0 = xcd_block(blockIdx.x, ncomp * nb);
    const int c = lb0 / nb;
    const int lb = lb0 - c * nb;
    const int bi = lb / sg.gx;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    // block-uniform selects keep the pointer choice in scalar registers
    const double* uc = c == 0 ? u.p[0] : c == 1 ? u.p[1] : u.p[2];
    const double* fc = c == 0 ? rhs.f[0] : c == 1 ? rhs.f[1] : rhs.f[2];
    const double sgn = (rhs.mode == RHS_NEGW) ? -1.0 : 1.0;
    double rr = 0.0, bb = 0.0;
    if (t < d.M * d.nz) {
        const int jj = t / d.nz;
        const int k = t - jj * d.nz;
        const int j = jj + 1;
        const int plane = d.ny * d.nz;
        const int off = j * d.nz + k;
        const int kp = (k + 1 == d.nz) ? 0 : k + 1;
        const int km = (k == 0) ? d.nz - 1 : k - 1;
        const int i0 = bi * sg.ci;
        const int i1 = min(d.nx, i0 + sg.ci);
        const int im0 = (i0 == 0) ? d.nx - 1 : i0 - 1;
        double um = uc[im0 * plane + off];
        double ux = uc[i0 * plane + off];
#pragma unroll 2
        for (int i = i0; i < i1; ++i) {
            const int ip = (i + 1 == d.nx) ? 0 : i + 1;
            const int rb = i * plane + j * d.nz;
            const int c0 = rb + k;
            const double up = uc[ip * plane + off];
            const double b = sgn * fc[c0];
            const double ylo = uc[c0 - d.nz], yhi = uc[c0 + d.nz];
            const double w = (j == 1 ? ylo : 0.0) + (j == d.M ? yhi : 0.0);
            const double lap = (up + um + ylo + yhi + uc[rb + kp] + uc[rb + km] - 6.0 * ux) *
                               d.inv_h2;
            const double r = b - lap;
            const double bt = b - w * d.inv_h2;
            rr += r * r;
            bb += bt * bt;
            um = ux;
            ux = up;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    if (lane == 0) {
        sh[w] = rr;
        sh[4 + w] = bb;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int q = threadIdx.x;
        partials[(slot0 + 3 * q + c) * kMaxPartialBlocks + lb] =
            sh[4 * q + 0] + sh[4 * q + 1] + sh[4 * q + 2] + sh[4 * q + 3];
    } else if (c == 0 && threadIdx.x < 8) {
        // the check sums three components: the blocks of component 0 clear the absent ones
        const int q = (threadIdx.x - 2) / 3, cc = (threadIdx.x - 2) - 3 * q;
        if (cc >= ncomp) partials[(slot0 + 3 * q + cc) * kMaxPartialBlocks + lb] = 0.0;
    }
}

// resid_flow: both residual norms of the flow solve in one pass, in the layout of resid_norm
// (vorticity in slots 0-5, stream vector in slots 6-11). A block owns one component c and
// streams omega_c, S_c and psi_c: omega_c is read once for both problems (its stencil for
// eq. (5b), its centre as the right-hand side -omega_c of eq. (5c)). Sums are those of
// resid_norm, term for term.
// This one-z form serves n_z not a multiple of 32 (k_resid_flow2 below takes the others).
__global__ __launch_bounds__(kBlock) void k_resid_flow(Dims d, CPtr3 om, CPtr3 src, CPtr3 ps,
                                                      SlabGrid sg, double ashift,
                                                      double* __restrict__ partials) {
    __shared__ double sh[4 * 4];
    const int nb = sg.gx * sg.gi;
    const int lb0 = xcd_block(blockIdx.x, 3 * nb);
    const int c = lb0 / nb;
    const int lb = lb0 - c * nb;
    const int bi = lb / sg.gx;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    const double* wc = c == 0 ? om.p[0] : c == 1 ? om.p[1] : om.p[2];
    const double* sc = c == 0 ? src.p[0] : c == 1 ? src.p[1] : src.p[2];
    const double* pc = c == 0 ? ps.p[0] : c == 1 ? ps.p[1] : ps.p[2];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (t < d.M * d.nz) {
        const int jj = t / d.nz;
        const int k = t - jj * d.nz;
        const int j = jj + 1;
        const int plane = d.ny * d.nz;
        const int off = j * d.nz + k;
        const int kp = (k + 1 == d.nz) ? 0 : k + 1;
        const int km = (k == 0) ? d.nz - 1 : k - 1;
        // z neighbours of u at plane row rb
        auto zpair = [&](const double* u, int rb, double, double& zp, double& zm) {
            zp = u[rb + kp];
            zm = u[rb + km];
        };
        const int i0 = bi * sg.ci;
        const int i1 = min(d.nx, i0 + sg.ci);
        const int im0 = (i0 == 0) ? d.nx - 1 : i0 - 1;
        double wm = wc[im0 * plane + off], wx = wc[i0 * plane + off];
        double pm = pc[im0 * plane + off], px = pc[i0 * plane + off];
#pragma unroll 2
        for (int i = i0; i < i1; ++i) {
            const int ip = (i + 1 == d.nx) ? 0 : i + 1;
            const int rb = i * plane + j * d.nz;
            const int c0 = rb + k;
            const double wp = wc[ip * plane + off];
            const double pp = pc[ip * plane + off];
            {
                const double b = sc[c0];
                const double ylo = wc[c0 - d.nz], yhi = wc[c0 + d.nz];
                const double w = (j == 1 ? ylo : 0.0) + (j == d.M ? yhi : 0.0);
                double zp, zm;
                zpair(wc, rb, wx, zp, zm);
                const double lap = (wp + wm + ylo + yhi + zp + zm - 6.0 * wx) * d.inv_h2;
                // the inertial variant solves (L_h - a) omega = b
                const double r = b - (ashift != 0.0 ? lap - ashift * wx : lap);
                const double bt = b - w * d.inv_h2;
                a[0] += r * r;
                a[1] += bt * bt;
            }
            {
                const double b = -wx;
                const double ylo = pc[c0 - d.nz], yhi = pc[c0 + d.nz];
                const double w = (j == 1 ? ylo : 0.0) + (j == d.M ? yhi : 0.0);
                double zp, zm;
                zpair(pc, rb, px, zp, zm);
                const double lap = (pp + pm + ylo + yhi + zp + zm - 6.0 * px) * d.inv_h2;
                const double r = b - lap;
                const double bt = b - w * d.inv_h2;
                a[2] += r * r;
                a[3] += bt * bt;
            }
            wm = wx;
            wx = wp;
            pm = px;
            px = pp;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double v = wave_sum(a[q]);
        if (lane == 0) sh[4 * q + w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;   // 0: omega r, 1: omega b~, 2: psi r, 3: psi b~
        partials[(3 * q + c) * kMaxPartialBlocks + lb] =
            sh[4 * q + 0] + sh[4 * q + 1] + sh[4 * q + 2] + sh[4 * q + 3];
    }
}


// resid_flow with two consecutive z per lane: W lanes (64, 32 or 16) cover 2W consecutive z of
// one row, n_z a multiple of 2W. Every load moves 16 bytes, half the load instructions of the
// one-z form; the z neighbours inside the pair come from the pair itself, across lanes by
// width-W shuffles, and the segment's two edge values by one load each. The next plane's
// centres are loaded last (a scheduling barrier keeps them there), so they stay in flight
// while the current plane is summed. Same sums per node as k_resid_flow; a lane adds its two
// nodes' squares together.
template <int W>
__global__ __launch_bounds__(kBlock) void k_resid_flow2(Dims d, CPtr3 om, CPtr3 src, CPtr3 ps,
                                                       SlabGrid sg, double ashift,
                                                       double* __restrict__ partials) {
    __shared__ double sh[4 * 4];
    const int nb = sg.gx * sg.gi;
    const int lb0 = xcd_block(blockIdx.x, 3 * nb);
    const int c = lb0 / nb;
    const int lb = lb0 - c * nb;
    const int bi = lb / sg.gx;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    const double* wc = c == 0 ? om.p[0] : c == 1 ? om.p[1] : om.p[2];
    const double* sc = c == 0 ? src.p[0] : c == 1 ? src.p[1] : src.p[2];
    const double* pc = c == 0 ? ps.p[0] : c == 1 ? ps.p[1] : ps.p[2];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    const int hz = d.nz >> 1;
    if (t < d.M * hz) {
        const int jj = t / hz;
        const int k = 2 * (t - jj * hz);
        const int j = jj + 1;
        const int plane = d.ny * d.nz;
        const int off = j * d.nz + k;
        const int ln = threadIdx.x & (W - 1);
        const int k0 = k - 2 * ln;
        const int kpe = (k0 + 2 * W == d.nz) ? 0 : k0 + 2 * W;
        const int kme = (k0 == 0) ? d.nz - 1 : k0 - 1;
        auto ld2v = [](const double* q) { return *reinterpret_cast<const double2*>(q); };
        auto zn = [&](double2 v, double em, double ep, double& zm0, double& zp1) {
            const double prev = __shfl_up(v.y, 1, W), next = __shfl_down(v.x, 1, W);
            zm0 = ln == 0 ? em : prev;
            zp1 = ln == W - 1 ? ep : next;
        };
        const int i0 = bi * sg.ci;
        const int i1 = min(d.nx, i0 + sg.ci);
        const int im0 = (i0 == 0) ? d.nx - 1 : i0 - 1;
        double2 wm = ld2v(wc + im0 * plane + off), wx = ld2v(wc + i0 * plane + off);
        double2 pm = ld2v(pc + im0 * plane + off), px = ld2v(pc + i0 * plane + off);
        const bool lo = j == 1, hi = j == d.M;
#pragma unroll 2
        for (int i = i0; i < i1; ++i) {
            const int ip = (i + 1 == d.nx) ? 0 : i + 1;
            const int rb = i * plane + j * d.nz;
            const int c0 = rb + k;
            const double2 b = ld2v(sc + c0);
            const double2 ylo = ld2v(wc + c0 - d.nz), yhi = ld2v(wc + c0 + d.nz);
            const double2 qlo = ld2v(pc + c0 - d.nz), qhi = ld2v(pc + c0 + d.nz);
            const int ome = rb + kme, ope = rb + kpe;
            const double wem = wc[ome], wep = wc[ope], pem = pc[ome], pep = pc[ope];
            // the next plane's centres last: they stay in flight while this plane is summed
            const double2 wp = ld2v(wc + ip * plane + off);
            const double2 pp = ld2v(pc + ip * plane + off);
            __builtin_amdgcn_sched_barrier(0);
            {
                double zm0, zp1;
                zn(wx, wem, wep, zm0, zp1);
                const double l0 = (wp.x + wm.x + ylo.x + yhi.x + wx.y + zm0 - 6.0 * wx.x) * d.inv_h2;
                const double l1 = (wp.y + wm.y + ylo.y + yhi.y + zp1 + wx.x - 6.0 * wx.y) * d.inv_h2;
                const double r0 = b.x - (ashift != 0.0 ? l0 - ashift * wx.x : l0);
                const double r1 = b.y - (ashift != 0.0 ? l1 - ashift * wx.y : l1);
                const double t0 = b.x - ((lo ? ylo.x : 0.0) + (hi ? yhi.x : 0.0)) * d.inv_h2;
                const double t1 = b.y - ((lo ? ylo.y : 0.0) + (hi ? yhi.y : 0.0)) * d.inv_h2;
                a[0] += r0 * r0 + r1 * r1;
                a[1] += t0 * t0 + t1 * t1;
            }
            {
                const double2 ylo = qlo, yhi = qhi;
                double zm0, zp1;
                zn(px, pem, pep, zm0, zp1);
                const double l0 = (pp.x + pm.x + ylo.x + yhi.x + px.y + zm0 - 6.0 * px.x) * d.inv_h2;
                const double l1 = (pp.y + pm.y + ylo.y + yhi.y + zp1 + px.x - 6.0 * px.y) * d.inv_h2;
                const double r0 = -wx.x - l0, r1 = -wx.y - l1;
                const double t0 = -wx.x - ((lo ? ylo.x : 0.0) + (hi ? yhi.x : 0.0)) * d.inv_h2;
                const double t1 = -wx.y - ((lo ? ylo.y : 0.0) + (hi ? yhi.y : 0.0)) * d.inv_h2;
                a[2] += r0 * r0 + r1 * r1;
                a[3] += t0 * t0 + t1 * t1;
            }
            wm = wx;
            wx = wp;
            pm = px;
            px = pp;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double v = wave_sum(a[q]);
        if (lane == 0) sh[4 * q + w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        partials[(3 * q + c) * kMaxPartialBlocks + lb] =
            sh[4 * q + 0] + sh[4 * q + 1] + sh[4 * q + 2] + sh[4 * q + 3];
    }
}

// check: relative residual sqrt(sum_c r^2 / sum_c b~^2) in a fixed summation order; sets the
// convergence flag that gates the following cycles, counts the cycle and raises ST_NOCONV
// on the last allowed cycle, ST_NONFINITE on NaN/Inf.
__global__ __launch_bounds__(1024) void k_check(const double* __restrict__ partials,
                                               int nblocks, double rtol, int last_cycle,
                                               double* scal, int* istat, const int* gate,
                                               int slot0) {
    if (gate && *gate) return;
    __shared__ double sh[2 * 16];
    double rr = 0.0, bb = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const double* pb = partials + (size_t)slot0 * kMaxPartialBlocks + b;
        rr += pb[0 * kMaxPartialBlocks] + pb[1 * kMaxPartialBlocks] + pb[2 * kMaxPartialBlocks];
        bb += pb[3 * kMaxPartialBlocks] + pb[4 * kMaxPartialBlocks] + pb[5 * kMaxPartialBlocks];
    }
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
        sh[w] = rr;
        sh[16 + w] = bb;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    rr = 0.0;
    bb = 0.0;
    for (int i = 0; i < nw; ++i) {
        rr += sh[i];
        bb += sh[16 + i];
    }
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

// Convergence checks of the two flow solves of a step in one launch (flow_check.h).
__global__ __launch_bounds__(1024) void k_check_flow(const double* __restrict__ partials,
                                                    int nblocks, double rtol, double* scal,
                                                    int* istat) {
    __shared__ double sh[4 * 16];
    flow_check_block(partials, nblocks, rtol, scal, istat, sh);
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

template <class ST>
SPtr3<ST> sptr(void* const spec[3], int ncomp) {
    return SPtr3<ST>{{static_cast<ST*>(spec[0]), ncomp > 1 ? static_cast<ST*>(spec[1]) : nullptr,
                      ncomp > 2 ? static_cast<ST*>(spec[2]) : nullptr}};
}

template <class ST>
void rhs_dht_z_t(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                 const RhsArgs& rhs, const double* const u[3], int ncomp, int correct,
                 void* const spec[3], const int* gate) {
    const int nrows = d.nx * d.M;
    CPtr3 uu{{u[0], ncomp > 1 ? u[1] : nullptr, ncomp > 2 ? u[2] : nullptr}};
    const SPtr3<ST> sp = sptr<ST>(spec, ncomp);
    int B, A;
    two_pass_shape(d.nz, B, A);
#define VS_CASE(b, a)                                                                          \
    if (B == b && A == a) {                                                                    \
        const int rows = 2 * TwoPass<b, a>::L;                                                 \
        launch_kernel((k_rhs_hz<b, a, ST>), dim3((nrows + rows - 1) / rows, ncomp),       \
                           dim3(64), 0, s, d, twz, rhs, uu, correct, sp, gate);                \
        return;                                                                                \
    }
    VS_TWO_PASS_CASES(VS_CASE)
#undef VS_CASE
    const int rpb = z_rows_per_block(d);
    launch_kernel(k_rhs_dht_z<ST>, dim3((nrows + rpb - 1) / rpb, ncomp), dim3(kBlock), 0, s,
                       d, pz, twz, rhs, uu, correct, sp, gate, rpb);
}

template <class ST>
void dht_x_t(hipStream_t s, const Dims& d, const FftPlan& px, const double2* twx,
             void* const spec[], int ncomp, const int* gate) {
    SPtr6<ST> sp6{};
    for (int c = 0; c < ncomp; ++c) sp6.p[c] = static_cast<ST*>(spec[c]);
    int B, A;
    two_pass_shape(d.nx, B, A);
#define VS_CASE(b, a)                                                                          \
    if (B == b && A == a) {                                                                    \
        const int qs = 2 * TwoPass<b, a>::L;                                                   \
        const dim3 g((d.nz + qs - 1) / qs, d.M, ncomp);                                        \
        if (ncomp > 3)                                                                         \
            launch_kernel((k_hx<b, a, ST, 6>), g, dim3(64), 0, s, d, twx, sp6, gate);          \
        else                                                                                   \
            launch_kernel((k_hx<b, a, ST, 3>), g, dim3(64), 0, s, d, twx, sp6, gate);          \
        return;                                                                                \
    }
    VS_TWO_PASS_CASES(VS_CASE)
#undef VS_CASE
    const int kb = x_modes_per_block(d);
    for (int c0 = 0; c0 < ncomp; c0 += 3) {
        const int nc = ncomp - c0 < 3 ? ncomp - c0 : 3;
        launch_kernel(k_dht_x<ST>, dim3((d.nz + kb - 1) / kb, d.M, nc), dim3(kBlock), 0, s, d,
                      px, twx, sptr<ST>(spec + c0, nc), gate, kb);
    }
}

template <class ST>
void dht_z_out_t(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                 void* const spec[], double* const u[], int ncomp, int add, const int* gate) {
    const int nrows = d.nx * d.M;
    SPtr6<ST> sp6{};
    Ptr6 u6{};
    for (int c = 0; c < ncomp; ++c) {
        sp6.p[c] = static_cast<ST*>(spec[c]);
        u6.p[c] = u[c];
    }
    int B, A;
    two_pass_shape(d.nz, B, A);
#define VS_CASE(b, a)                                                                          \
    if (B == b && A == a) {                                                                    \
        const int rows = 2 * TwoPass<b, a>::L;                                                 \
        const dim3 g((nrows + rows - 1) / rows, ncomp);                                        \
        if (ncomp > 3)                                                                         \
            launch_kernel((k_hz_out<b, a, ST, 6>), g, dim3(64), 0, s, d, twz, sp6, u6, add,    \
                          gate);                                                               \
        else                                                                                   \
            launch_kernel((k_hz_out<b, a, ST, 3>), g, dim3(64), 0, s, d, twz, sp6, u6, add,    \
                          gate);                                                               \
        return;                                                                                \
    }
    VS_TWO_PASS_CASES(VS_CASE)
#undef VS_CASE
    const int rpb = z_rows_per_block(d);
    for (int c0 = 0; c0 < ncomp; c0 += 3) {
        const int nc = ncomp - c0 < 3 ? ncomp - c0 : 3;
        Ptr3 uu{{u[c0], nc > 1 ? u[c0 + 1] : nullptr, nc > 2 ? u[c0 + 2] : nullptr}};
        launch_kernel(k_dht_z_out<ST>, dim3((nrows + rpb - 1) / rpb, nc), dim3(kBlock), 0, s,
                      d, pz, twz, sptr<ST>(spec + c0, nc), uu, add, gate, rpb);
    }
}

}  // namespace

void launch_rhs_dht_z(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      const RhsArgs& rhs, const double* const u[3], int ncomp, int correct,
                      void* const spec[3], bool f32, const int* gate) {
    if (f32)
        rhs_dht_z_t<float>(s, d, pz, twz, rhs, u, ncomp, correct, spec, gate);
    else
        rhs_dht_z_t<double>(s, d, pz, twz, rhs, u, ncomp, correct, spec, gate);
}

void launch_dht_x(hipStream_t s, const Dims& d, const FftPlan& px, const double2* twx,
                  void* const spec[], int ncomp, bool f32, const int* gate) {
    if (f32)
        dht_x_t<float>(s, d, px, twx, spec, ncomp, gate);
    else
        dht_x_t<double>(s, d, px, twx, spec, ncomp, gate);
}

// Segment layout for M interior rows: S lanes per mode, at most LMAX rows per lane.
// 0 = the twisted two-lane solve (M < 4 or M > 256).
int seg_shape(int M) {
    if (M < 4 || M > 256) return 0;
    if (M <= 32) return 8;
    if (M <= 64) return 16;
    if (M <= 128) return 32;
    return 832;   // S = 8, LMAX = 32
}

// Launches the segmented solve with S lanes per mode; PAIR selects the vorticity +
// stream-vector kernel. Grids with ny = n in {32, 48, 64, 96, 128, 256} (M = n - 2) get
// their segment lengths as compile-time constants.
template <bool PAIR, int S, int LMAX, class ST, int LMF, int NLF>
void seg_launch(hipStream_t s, const Dims& d, const double* tri, const double* triw,
                void* const spec[3], void* const spec2[3], int ncomp, const int* gate,
                double3 olo, double3 ohi, double3 lo, double3 hi, double scale) {
    const dim3 grid((unsigned)(((long)d.nx * d.nz * S + 255) / 256), ncomp);
    if (PAIR)
        launch_kernel((k_tridiag_pair_seg<S, LMAX, ST, LMF, NLF>), grid, dim3(256), 0, s, d,
                      tri, triw, sptr<ST>(spec, 3), sptr<ST>(spec2, 3), olo, ohi, lo, hi, scale);
    else
        launch_kernel((k_tridiag_seg<S, LMAX, ST, LMF, NLF>), grid, dim3(256), 0, s, d, tri,
                           sptr<ST>(spec, ncomp), gate, scale);
}

template <bool PAIR, class ST>
bool seg_dispatch(hipStream_t s, const Dims& d, const double* tri, const double* triw,
                  void* const spec[3], void* const spec2[3], int ncomp, const int* gate,
                  double3 olo, double3 ohi, double3 lo, double3 hi) {
    const double scale = d.h * d.h / ((double)d.nx * d.nz);
#define VS_SEG(S_, LMAX_, LMF_, NLF_) \
    seg_launch<PAIR, S_, LMAX_, ST, LMF_, NLF_>(s, d, tri, triw, spec, spec2, ncomp, gate, olo, \
                                                ohi, lo, hi, scale)
    switch (d.M) {
    case 30: VS_SEG(4, 8, 8, 2); return true;
    case 46: VS_SEG(4, 16, 12, 2); return true;
    case 62: VS_SEG(4, 16, 16, 2); return true;
    case 94: VS_SEG(8, 16, 12, 6); return true;
    case 126: VS_SEG(8, 16, 16, 6); return true;
    case 254: VS_SEG(16, 16, 16, 14); return true;
    default: break;
    }
    switch (seg_shape(d.M)) {
    case 8: VS_SEG(4, 8, 0, 0); return true;
    case 16: VS_SEG(4, 16, 0, 0); return true;
    case 32: VS_SEG(4, 32, 0, 0); return true;
    case 832: VS_SEG(8, 32, 0, 0); return true;
    default: return false;
    }
#undef VS_SEG
}

template <class ST>
void tridiag_y_t(hipStream_t s, const Dims& d, const double* tri, void* const spec[3], int ncomp,
                 const int* gate) {
    const double3 z = make_double3(0.0, 0.0, 0.0);
    if (seg_dispatch<false, ST>(s, d, tri, tri, spec, nullptr, ncomp, gate, z, z, z, z)) return;
    const double scale = d.h * d.h / ((double)d.nx * d.nz);
    const dim3 grid((2 * d.nx * d.nz + 63) / 64, ncomp);
    launch_kernel(k_tridiag_y<ST>, grid, dim3(64), 0, s, d, tri, sptr<ST>(spec, ncomp), gate,
                  scale, z, z);
}

template <class ST>
void tridiag_pair_t(hipStream_t s, const Dims& d, const double* tri, const double* triw,
                    void* const spec[3], void* const spec2[3], double3 olo, double3 ohi,
                    double3 lo, double3 hi) {
    if (seg_dispatch<true, ST>(s, d, tri, triw, spec, spec2, 3, nullptr, olo, ohi, lo, hi)) return;
    const double scale = d.h * d.h / ((double)d.nx * d.nz);
    const dim3 grid((2 * d.nx * d.nz + 63) / 64, 3);
    launch_kernel(k_tridiag_y<ST>, grid, dim3(64), 0, s, d, triw, sptr<ST>(spec, 3),
                  (const int*)nullptr, scale, olo, ohi);
    launch_kernel(k_tridiag_psi<ST>, grid, dim3(64), 0, s, d, tri, sptr<ST>(spec, 3),
                       sptr<ST>(spec2, 3), lo, hi);
}

void launch_tridiag_y(hipStream_t s, const Dims& d, const double* tri, void* const spec[3],
                      int ncomp, bool f32, const int* gate) {
    if (f32)
        tridiag_y_t<float>(s, d, tri, spec, ncomp, gate);
    else
        tridiag_y_t<double>(s, d, tri, spec, ncomp, gate);
}

void launch_tridiag_pair(hipStream_t s, const Dims& d, const double* tri, const double* triw,
                         void* const spec[3], void* const spec2[3], const double om_lo[3],
                         const double om_hi[3], const double psi_lo[3], const double psi_hi[3],
                         bool f32) {
    const double3 olo = make_double3(om_lo[0], om_lo[1], om_lo[2]);
    const double3 ohi = make_double3(om_hi[0], om_hi[1], om_hi[2]);
    const double3 lo = make_double3(psi_lo[0], psi_lo[1], psi_lo[2]);
    const double3 hi = make_double3(psi_hi[0], psi_hi[1], psi_hi[2]);
    if (!triw) triw = tri;
    if (f32)
        tridiag_pair_t<float>(s, d, tri, triw, spec, spec2, olo, ohi, lo, hi);
    else
        tridiag_pair_t<double>(s, d, tri, triw, spec, spec2, olo, ohi, lo, hi);
}

void launch_dht_z_fwd(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      const double* const f[3], void* const spec[3], int ncomp) {
    // the z pass of the inverse computes the same Hartley sums (H is its own inverse up to
    // the scale, which the tridiagonal solve applies), from FP64 input to FP64 output
    void* const in[3] = {(void*)f[0], ncomp > 1 ? (void*)f[1] : nullptr, ncomp > 2 ? (void*)f[2] : nullptr};
    double* const out[3] = {(double*)spec[0], ncomp > 1 ? (double*)spec[1] : nullptr,
                            ncomp > 2 ? (double*)spec[2] : nullptr};
    dht_z_out_t<double>(s, d, pz, twz, in, out, ncomp, 0, nullptr);
}

void launch_dht_z_out(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      void* const spec[], double* const u[], int ncomp, int add, bool f32,
                      const int* gate) {
    if (f32)
        dht_z_out_t<float>(s, d, pz, twz, spec, u, ncomp, add, gate);
    else
        dht_z_out_t<double>(s, d, pz, twz, spec, u, ncomp, add, gate);
}

// Residual blocks per component: slabs of x-planes chosen so that about a thousand blocks
// cover one component (each component adds as many again).
static SlabGrid resid_grid(const Dims& d) { return slab_grid(d.M * d.nz, d.nx, 1024); }

int resid_blocks(const Dims& d) {
    const SlabGrid g = resid_grid(d);
    return g.gx * g.gi;
}

static SlabGrid resid_flow_grid(const Dims& d) {
    return d.nz % 32 == 0 ? slab_grid(d.M * d.nz / 2, d.nx, 1024) : resid_grid(d);
}

int resid_flow_blocks(const Dims& d) {
    const SlabGrid g = resid_flow_grid(d);
    return g.gx * g.gi;
}

void launch_resid_norm(hipStream_t s, const Dims& d, const RhsArgs& rhs,
                       const double* const u[3], int ncomp, double* partials, const int* gate,
                       int slot0) {
    CPtr3 uu{{u[0], ncomp > 1 ? u[1] : nullptr, ncomp > 2 ? u[2] : nullptr}};
    const SlabGrid g = resid_grid(d);
    launch_kernel(k_resid_norm, dim3(ncomp * g.gx * g.gi), dim3(kBlock), 0, s, d, rhs, uu, ncomp,
                  g, partials, gate, slot0);
}

void launch_resid_flow(hipStream_t s, const Dims& d, const double* const om[3],
                       const double* const src[3], const double* const ps[3], double ashift,
                       double* partials) {
    const CPtr3 o{{om[0], om[1], om[2]}}, f{{src[0], src[1], src[2]}}, p{{ps[0], ps[1], ps[2]}};
    const SlabGrid g = resid_flow_grid(d);
    if (d.nz % 128 == 0)
        launch_kernel(k_resid_flow2<64>, dim3(3 * g.gx * g.gi), dim3(kBlock), 0, s, d, o, f, p, g,
                      ashift, partials);
    else if (d.nz % 64 == 0)
        launch_kernel(k_resid_flow2<32>, dim3(3 * g.gx * g.gi), dim3(kBlock), 0, s, d, o, f, p, g,
                      ashift, partials);
    else if (d.nz % 32 == 0)
        launch_kernel(k_resid_flow2<16>, dim3(3 * g.gx * g.gi), dim3(kBlock), 0, s, d, o, f, p, g,
                      ashift, partials);
    else
        launch_kernel(k_resid_flow, dim3(3 * g.gx * g.gi), dim3(kBlock), 0, s, d, o, f, p, g,
                      ashift, partials);
}

void launch_check_flow(hipStream_t s, const Dims& d, const double* partials, double rtol,
                       double* scal, int* istat) {
    launch_kernel(k_check_flow, dim3(1), dim3(1024), 0, s, partials, resid_flow_blocks(d), rtol, scal,
                  istat);
}

void launch_check(hipStream_t s, const double* partials, int nblocks, double rtol, int cycle,
                  int last_cycle, double* scal, int* istat, const int* gate, int slot0) {
    (void)cycle;
    launch_kernel(k_check, dim3(1), dim3(1024), 0, s, partials, nblocks, rtol,
                       last_cycle, scal, istat, gate, slot0);
}

}  // namespace vs
