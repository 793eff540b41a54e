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
#include <type_traits>

#include "spectral.h"

namespace vs {

namespace {

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
// LM > 1: LM times the lines per block, so pass 1 takes LM rounds and pass 2 (B/2 items per
// line) fills more lanes (A = 16 leaves half the wave idle in pass 2 with LM = 1).
template <int B, int A, int LM = 1>
struct TwoPass {
    static constexpr int N = B * A;
    static constexpr int L = LM * ((64 / A) > 0 ? (64 / A) : 1);
    static constexpr int RS = A + 1;             // padded row of Y
    static constexpr int LS = B * RS + 1;        // padded line of Y
    static constexpr int LDS = L * LS;           // double2 elements
};

// Prep: Pre prep(line) (per-line row offsets, computed once per item).
// Loader: double2 load(pre, k1, k2) -> (line a value, line b value) at position k1 + A k2.
// Storer: void store(pre, p, ha, hb).
template <int B, int A, bool LINE_FAST, class T, int LM = 1, class Prep, class Load, class Store>
__device__ __forceinline__ void two_pass_hartley(C2<T>* Y, const double2* __restrict__ tw_,
                                                 Prep prep, Load load, Store store) {
    // the twiddle table is global memory (typed so, whatever the pointer's origin)
    const Gl<tw2v>* __restrict__ tw = (const Gl<tw2v>*)tw_;
    using P = TwoPass<B, A, LM>;
    using C = C2<T>;
    constexpr int L = P::L;
    const T half = (T)0.5;
#pragma unroll 1
    for (int it = threadIdx.x; it < L * A; it += 64) {
        const int line = LINE_FAST ? (it % L) : (it / A);
        const int k1 = LINE_FAST ? (it / L) : (it % A);
        const auto pre = prep(line);
        C x[B];
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) x[k2] = load(pre, k1, k2);
        fftr::DFT<B>::run(x);
#pragma unroll
        for (int p2 = 1; p2 < B; ++p2) x[p2] = cmul_tw<T>(x[p2], tw[k1 * p2]);
        C* Yl = Y + line * P::LS + k1;
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
        C* Ya = Y + line * P::LS + pa * P::RS;
        const C* Yb = Y + line * P::LS + pb * P::RS;
        if constexpr (A >= 16 && sizeof(T) == 8) {
            // long FP64 lines: the a-line's transform goes back to its own LDS row (no other
            // lane reads it), so only one line of registers is live at a time
            C x[A];
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
                const C za = Ya[p1];
                const C ma = (s == 0) ? Ya[(A - p1) % A] : x[A - 1 - p1];
                store(pre, pa + B * p1, half * (za.x + ma.x - za.y + ma.y), half * (za.x - ma.x + za.y + ma.y));
                const C zb = x[p1];
                const C mb = (s == 0) ? x[A - 1 - p1] : Ya[A - 1 - p1];
                store(pre, pb + B * p1, half * (zb.x + mb.x - zb.y + mb.y), half * (zb.x - mb.x + zb.y + mb.y));
            }
        } else {
            C xa[A], xb[A];
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) {
                xa[k1] = Ya[k1];
                xb[k1] = Yb[k1];
            }
            fftr::DFT<A>::run(xa);
            fftr::DFT<A>::run(xb);
#pragma unroll
            for (int p1 = 0; p1 < A; ++p1) {
                const C za = xa[p1];
                const C ma = (s == 0) ? xa[(A - p1) % A] : xb[A - 1 - p1];
                store(pre, pa + B * p1, half * (za.x + ma.x - za.y + ma.y), half * (za.x - ma.x + za.y + ma.y));
                const C zb = xb[p1];
                const C mb = (s == 0) ? xb[A - 1 - p1] : xa[A - 1 - p1];
                store(pre, pb + B * p1, half * (zb.x + mb.x - zb.y + mb.y), half * (zb.x - mb.x + zb.y + mb.y));
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
    using T = ST;
    using C = C2<T>;
    __shared__ C Y[P::LDS];
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
    auto store = [&](const RowPair& rp, int p, T ha, T hb) {
        if (rp.a >= 0) sc[rp.a + p] = (ST)ha;
        if (rp.b >= 0) sc[rp.b + p] = (ST)hb;
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
        auto load = [&](const int4& o, int k1, int k2) -> C {
            const int k = k1 + A * k2;
            return mkc<T>((T)rowval(o.x, o.z, k), (T)rowval(o.y, o.w, k));
        };
        auto storew = [&](const int4& o, int p, T ha, T hb) {
            if (o.x >= 0) sc[o.x + p] = (ST)ha;
            if (o.y >= 0) sc[o.y + p] = (ST)hb;
        };
        two_pass_hartley<B, A, false, T>(Y, tw, prepw, load, storew);
        return;
    }
#pragma unroll 4
    for (int lr = 0; lr < 2 * L; ++lr) {
        const int r = r0 + lr;
        C* row = &Y[(lr >> 1) * N];
        if (r < nrows) {
            const int i = r / d.M;
            const int j = 1 + (r - i * d.M);
            const int ip = (i + 1 == d.nx) ? 0 : i + 1;
            const int im = (i == 0) ? d.nx - 1 : i - 1;
            const int rb = node(d, i, j, 0), xpb = node(d, ip, j, 0), xmb = node(d, im, j, 0);
#pragma unroll
            for (int k = threadIdx.x; k < N; k += 64)
                reinterpret_cast<T*>(&row[k])[lr & 1] = (T)rhs_row(rhs, d, uc, c, 1, rb, xpb, xmb, j, k);
        } else {
#pragma unroll
            for (int k = threadIdx.x; k < N; k += 64) reinterpret_cast<T*>(&row[k])[lr & 1] = (T)0;
        }
    }
    __syncthreads();
    C xin[B];
    const int it = threadIdx.x;
    const bool act = it < L * A;
    const int line = act ? it / A : 0, k1 = act ? it % A : 0;
    if (act) {
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) xin[k2] = Y[line * N + k1 + A * k2];
    }
    __syncthreads();
    auto load = [&](const RowPair&, int, int k2) -> C { return xin[k2]; };
    two_pass_hartley<B, A, false, T>(Y, tw, prep, load, store);
}

// dht_x, two-pass form: block = (2L consecutive z-modes q, interior row j, component c);
// lines are the q-pairs (q, q+1), read and written as one 16-byte value.
// NC: the component count of the launch (3, or 6 for the vorticity and stream-vector fields
// together); the code is the same, the symbol tells the two launches apart in traces.
template <int B, int A, class ST, int NC, bool BATCH>
__global__ __launch_bounds__(64) void k_hx(Dims d, HxArgs one, const HxArgs* __restrict__ tab) {
    using P = TwoPass<B, A>;
    using T = ST;
    using C = C2<T>;
    const int inst = BATCH ? (int)blockIdx.z / NC : 0;
    const int c = (int)blockIdx.z - inst * NC;
    const HxArgs& a = inst_args<BATCH>(one, tab, inst);
    if (a.gate && *a.gate) return;
    __shared__ C Y[P::LDS];
    const int j = 1 + blockIdx.y;
    const int q0 = blockIdx.x * 2 * P::L;
    Gl<ST>* s = (Gl<ST>*)pick(a.spec, c);
    const int pstride = d.ny * d.nz;
    auto prep = [&](int line) -> int {
        const int q = q0 + 2 * line;
        return q < d.nz ? j * d.nz + q : -1;
    };
    auto load = [&](int o, int k1, int k2) -> C {
        if (o < 0) return mkc<T>((T)0, (T)0);
        return ldc<T>(s + o + (k1 + A * k2) * pstride);
    };
    auto store = [&](int o, int p, T ha, T hb) {
        if (o >= 0) stc<T>(s + o + p * pstride, ha, hb);
    };
    two_pass_hartley<B, A, true, T>(Y, a.tw, prep, load, store);
}

// Lines per block of the z output pass: doubled for FP32 256-long lines (see TwoPass).
template <int A, class ST>
constexpr int z_out_lm() { return (A == 16 && sizeof(ST) == 4) ? 2 : 1; }

// dht_z_out, two-pass form: block = (2L consecutive interior rows, component c).
// NC as for k_hx.
template <int B, int A, class ST, int NC, bool BATCH>
__global__ __launch_bounds__(64) void k_hz_out(Dims d, ZArgs one, const ZArgs* __restrict__ tab) {
    constexpr int LM = z_out_lm<A, ST>();
    using P = TwoPass<B, A, LM>;
    using T = ST;
    using C = C2<T>;
    const int inst = BATCH ? (int)blockIdx.y / NC : 0;
    const int c = (int)blockIdx.y - inst * NC;
    const ZArgs& a = inst_args<BATCH>(one, tab, inst);
    if (a.gate && *a.gate) return;
    __shared__ C Y[P::LDS];
    const int nrows = d.nx * d.M;
    const int r0 = blockIdx.x * 2 * P::L;
    const Gl<ST>* sc = (const Gl<ST>*)pick(a.spec, c);
    Gl<double>* uc = (Gl<double>*)pick(a.u, c);
    const int add = a.add;
    // the refined mode's time increments: h = -1 a later cycle (accumulate), 0..2 the first
    // cycle with that many increments held (the predictor of k_rhs_pred, same arithmetic)
    Gl<float>* __restrict__ ic = (Gl<float>*)pick(a.inc, c);
    const Gl<float>* __restrict__ pc = (const Gl<float>*)pick(a.pinc, c);
    const int h = a.hist ? *a.hist : -1;
    if (a.hist_out && blockIdx.x == 0 && c == 0 && threadIdx.x == 0) *a.hist_out = h < 2 ? h + 1 : 2;
    auto prep = [&](int line) -> RowPair {
        return RowPair{row_base(d, r0 + 2 * line, nrows), row_base(d, r0 + 2 * line + 1, nrows)};
    };
    auto load = [&](const RowPair& rp, int k1, int k2) -> C {
        const int k = k1 + A * k2;
        return mkc<T>(rp.a >= 0 ? ldt<T>(sc + rp.a + k) : (T)0, rp.b >= 0 ? ldt<T>(sc + rp.b + k) : (T)0);
    };
    // MODE 0: plain store or add; 1: a later cycle (u += e, inc += e); 2 + H: the first cycle
    // with H increments held; 5: the forward z pass in place (spec to spec)
    auto run = [&](auto mc) {
        constexpr int MODE = decltype(mc)::value;
        auto put = [&](int o, double e) {
            Gl<double>* dst = uc + o;
            if constexpr (MODE == 0) {
                *dst = add ? *dst + e : e;
            } else if constexpr (MODE == 1) {
                *dst = *dst + e;
                ic[o] = (float)((double)ic[o] + e);
            } else {
                double p = 0.0;
                if constexpr (MODE == 3) p = (double)pc[o];
                if constexpr (MODE == 4) p = 2.0 * (double)pc[o] - (double)ic[o];
                *dst = (*dst + p) + e;
                ic[o] = (float)(p + e);
            }
        };
        auto store = [&](const RowPair& rp, int p, T ha, T hb) {
            if constexpr (MODE == 5) {
                Gl<ST>* sw = const_cast<Gl<ST>*>(sc);
                if (rp.a >= 0) sw[rp.a + p] = (ST)ha;
                if (rp.b >= 0) sw[rp.b + p] = (ST)hb;
            } else {
                if (rp.a >= 0) put(rp.a + p, (double)ha);
                if (rp.b >= 0) put(rp.b + p, (double)hb);
            }
        };
        two_pass_hartley<B, A, false, T, LM>(Y, a.tw, prep, load, store);
    };
    if constexpr (std::is_same_v<ST, float> && NC == 6) {   // the refined mode's passes
        if (a.self) run(std::integral_constant<int, 5>{});
        else if (!add || !ic) run(std::integral_constant<int, 0>{});
        else if (h < 0) run(std::integral_constant<int, 1>{});
        else if (h == 0) run(std::integral_constant<int, 2>{});
        else if (h == 1) run(std::integral_constant<int, 3>{});
        else run(std::integral_constant<int, 4>{});
    } else {
        run(std::integral_constant<int, 0>{});
    }
}

// ---------------------------------------------------------------------------------------
// Both transform directions of one interior row in one pass: the whole (x, z) plane of row j
// and one component sits in LDS (n_x (n_z + 2) doubles, up to 135 KB at 128 x 128: one block
// per CU), so the spectral data crosses HBM once per direction instead of twice. Each 1D
// transform is the two-pass form above done in place in the plane: pass 1 overwrites the B
// inputs of its (line pair, k1) with their twiddled B-point DFT, pass 2 reads the A values of
// rows pa, pb, and after a barrier writes the Hartley values. z lines are pairs of x-rows
// (i, i+1), x lines pairs of z-columns (q, q+1) as in k_hx.
constexpr int kPlanePad = 2;
constexpr int kPlaneThreads = 512;

// One 1D Hartley transform of every line pair of the plane. ROWS: lines are x-rows (element m
// at P[row * RS + m]); otherwise z-columns (element m at P[m * RS + col]). T: the precision
// of the plane (FP64, or FP32 for the refined mode's corrections).
template <int B, int A, int NLP, int RS, bool ROWS, class T, int NT = kPlaneThreads>
__device__ __forceinline__ void plane_hartley(T* __restrict__ P, const tw2v* __restrict__ tw, int it) {
    using C = C2<T>;
    static_assert(NLP * A <= NT && NLP * (B / 2) <= NT, "one item per lane");
    auto ld = [&](int lp, int m) -> C {
        if constexpr (ROWS) return mkc<T>(P[(2 * lp) * RS + m], P[(2 * lp + 1) * RS + m]);
        else return *reinterpret_cast<const C*>(&P[m * RS + 2 * lp]);
    };
    auto st = [&](int lp, int m, T a, T b) {
        if constexpr (ROWS) {
            P[(2 * lp) * RS + m] = a;
            P[(2 * lp + 1) * RS + m] = b;
        } else {
            *reinterpret_cast<C*>(&P[m * RS + 2 * lp]) = mkc<T>(a, b);
        }
    };
    auto fma_t = [](T a, T b, T c) -> T {
        if constexpr (sizeof(T) == 8) return __builtin_fma(a, b, c);
        else return __builtin_fmaf(a, b, c);
    };
    // pass 1: B-point DFTs over k2, twiddled, back to the same positions k1 + A p2
    if (it < NLP * A) {
        const int lp = ROWS ? it / A : it % NLP;
        const int k1 = ROWS ? it % A : it / NLP;
        C x[B];
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) x[k2] = ld(lp, k1 + A * k2);
        fftr::DFT<B>::run(x);
#pragma unroll
        for (int p2 = 1; p2 < B; ++p2) x[p2] = cmul_tw<T>(x[p2], tw[k1 * p2]);
#pragma unroll
        for (int p2 = 0; p2 < B; ++p2) st(lp, k1 + A * p2, x[p2].x, x[p2].y);
    }
    __syncthreads();
    // pass 2: A-point DFTs of rows pa and pb, then the Hartley values of both lines
    const bool act = it < NLP * (B / 2);
    const int lp = act ? (ROWS ? it / (B / 2) : it % NLP) : 0;
    const int s = act ? (ROWS ? it % (B / 2) : it / NLP) : 0;
    const int pa = s, pb = (s == 0) ? B / 2 : B - s;
    // every lane computes (an idle one on line pair 0), so the arrays stay in registers
    C xa[A], xb[A];
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        xa[k1] = ld(lp, k1 + A * pa);
        xb[k1] = ld(lp, k1 + A * pb);
    }
    fftr::DFT<A>::run(xa);
    fftr::DFT<A>::run(xb);
    __syncthreads();
    if (act) {
        const T half = (T)0.5;
        // the partner Z_{n-p} comes from the lane's other row, except for s = 0 (rows 0 and
        // B/2, each its own partner); blended as f*u + (1-f)*v, exact for finite values (a
        // select here is turned into an indexed load from scratch memory)
        const T f = (s == 0) ? (T)1 : (T)0, g = (T)1 - f;
        auto blend = [&](const C& u, const C& v) -> C {
            return mkc<T>(fma_t(f, u.x, g * v.x), fma_t(f, u.y, g * v.y));
        };
#pragma unroll
        for (int p1 = 0; p1 < A; ++p1) {
            const C za = xa[p1];
            const C ma = blend(xa[(A - p1) % A], xb[A - 1 - p1]);
            st(lp, pa + B * p1, half * (za.x + ma.x - za.y + ma.y), half * (za.x - ma.x + za.y + ma.y));
            const C zb = xb[p1];
            const C mb = blend(xb[A - 1 - p1], xa[A - 1 - p1]);
            st(lp, pb + B * p1, half * (zb.x + mb.x - zb.y + mb.y), half * (zb.x - mb.x + zb.y + mb.y));
        }
    }
    __syncthreads();
}

// ZFIRST (the source's forward transform): z then x, from the field z.spec[c] (FP64, the
// interior rows) into the spectral buffer x.spec[c]. Otherwise (the inverse of the omega and
// psi modes): x then z, from x.spec[c] into the field z.u[c]. FP64 only; no gate, no
// accumulation. Persistent: block b takes the planes b, b + G, ... (G = gridDim.x; plane
// p = (instance * NC + component) * M + j - 1) and keeps the loads of its next plane in flight
// in registers while it works on the current one: the first half (NR1 values per lane) during
// the transforms, the rest during the stores (the whole plane beside a transform pass would
// not fit in the registers). The twiddles sit in LDS, so no global load inside the transforms
// waits behind the prefetch.
template <int BX, int AX, int BZ, int AZ, bool ZFIRST, int NC, bool BATCH>
__global__ __launch_bounds__(kPlaneThreads) void k_hxz_plane(Dims d, ZArgs zone,
                                                           const ZArgs* __restrict__ ztab,
                                                           HxArgs xone,
                                                           const HxArgs* __restrict__ xtab,
                                                           int nplanes) {
    constexpr int NX = BX * AX, NZ = BZ * AZ, RS = NZ + kPlanePad;
    constexpr int NT = kPlaneThreads;
    constexpr int NV = NX * NZ / 2;                          // double2 values of the plane
    constexpr int NR = (NV + NT - 1) / NT;
    __shared__ double P[NX * RS];
    __shared__ tw2v TWX[NX], TWZ[NZ];
    const size_t pstride = (size_t)d.ny * NZ;
    // twiddles of the two lengths (the same table for every instance)
    {
        const ZArgs& z0 = inst_args<BATCH>(zone, ztab, 0);
        const HxArgs& x0 = inst_args<BATCH>(xone, xtab, 0);
        const Gl<tw2v>* gz = (const Gl<tw2v>*)z0.tw;
        const Gl<tw2v>* gx = (const Gl<tw2v>*)x0.tw;
        for (int t = threadIdx.x; t < NX; t += NT) TWX[t] = gx[t];
        for (int t = threadIdx.x; t < NZ; t += NT) TWZ[t] = gz[t];
    }
    // the source and destination of plane p
    auto src_of = [&](int p) -> const Gl<double>* {
        const int cg = p / d.M;
        const int j = 1 + (p - cg * d.M);
        const int inst = BATCH ? cg / NC : 0;
        const int c = cg - inst * NC;
        const ZArgs& za = inst_args<BATCH>(zone, ztab, inst);
        const HxArgs& xa = inst_args<BATCH>(xone, xtab, inst);
        return (const Gl<double>*)(ZFIRST ? pick(za.spec, c) : pick(xa.spec, c)) + (size_t)j * NZ;
    };
    auto dst_of = [&](int p) -> Gl<double>* {
        const int cg = p / d.M;
        const int j = 1 + (p - cg * d.M);
        const int inst = BATCH ? cg / NC : 0;
        const int c = cg - inst * NC;
        const ZArgs& za = inst_args<BATCH>(zone, ztab, inst);
        const HxArgs& xa = inst_args<BATCH>(xone, xtab, inst);
        return (Gl<double>*)(ZFIRST ? pick(xa.spec, c) : pick(za.u, c)) + (size_t)j * NZ;
    };
    // x-row i of a plane at P[i * RS]; 16-byte values, NZ / 2 per row
    constexpr int NR1 = (NR + 1) / 2;
    double2 v[NR];
    auto load = [&](int p, int r0, int r1) {
        const Gl<double>* in = src_of(p);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r < r0 || r >= r1) continue;
            const int t = min((int)threadIdx.x + r * NT, NV - 1);
            const int i = t / (NZ / 2), k2 = t - i * (NZ / 2);
            v[r] = ldg2(in + i * pstride + 2 * k2);
        }
    };
    int p = blockIdx.x;
    if (p < nplanes) load(p, 0, NR);
    while (p < nplanes) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int t = threadIdx.x + r * NT;
            if (t < NV) {
                const int i = t / (NZ / 2), k2 = t - i * (NZ / 2);
                *reinterpret_cast<double2*>(&P[i * RS + 2 * k2]) = v[r];
            }
        }
        __syncthreads();
        const int pn = p + (int)gridDim.x;
        if (pn < nplanes) load(pn, 0, NR1);   // in flight while this plane is transformed
        // the lane index through an empty asm statement: the transforms' LDS offsets are then
        // recomputed in every round instead of held (and spilled) across the loop
        int it = threadIdx.x;
        asm volatile("" : "+v"(it));
        if constexpr (ZFIRST) {
            plane_hartley<BZ, AZ, NX / 2, RS, true>(P, TWZ, it);
            plane_hartley<BX, AX, NZ / 2, RS, false>(P, TWX, it);
        } else {
            plane_hartley<BX, AX, NZ / 2, RS, false>(P, TWX, it);
            plane_hartley<BZ, AZ, NX / 2, RS, true>(P, TWZ, it);
        }
        if (pn < nplanes) load(pn, NR1, NR);  // in flight while this plane is stored
        Gl<double>* out = dst_of(p);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int t = threadIdx.x + r * NT;
            if (t < NV) {
                const int i = t / (NZ / 2), k2 = t - i * (NZ / 2);
                const double2 w = *reinterpret_cast<const double2*>(&P[i * RS + 2 * k2]);
                stc<double>(out + i * pstride + 2 * k2, w.x, w.y);
            }
        }
        __syncthreads();   // the plane's LDS is read out before the next one is written
        p = pn;
    }
}

// The refined mode's plane passes: FP32 spectral data, the (x, z) plane of one interior row
// and component in LDS as floats (n_x (n_z + 2) floats: 66 KB at 128 x 128). ZFIRST: the forward transforms, z then x, of the FP32 residuals in place
// (z.spec[c], c < 6: vorticity then stream vector). Otherwise the inverse transforms, x then z,
// of the FP32 corrections (x.spec[c]) added to the FP64 fields (z.u[c]) as k_hz_out adds them:
// the time increments of the first cycle's update (z.inc, z.pinc, z.hist, z.hist_out) or of a
// later cycle (z.inc), or a plain add (z.add, the initial solve). Planes of an instance whose
// z.gate is set are skipped. Persistent, with the next plane's loads in flight, as k_hxz_plane.
template <int BX, int AX, int BZ, int AZ, bool ZFIRST, bool BATCH>
__global__ __launch_bounds__(kPlaneThreads) void k_plane32(Dims d, ZArgs zone,
                                                         const ZArgs* __restrict__ ztab,
                                                         HxArgs xone,
                                                         const HxArgs* __restrict__ xtab,
                                                         int nplanes) {
    constexpr int NC = 6;
    constexpr int NX = BX * AX, NZ = BZ * AZ, RS = NZ + kPlanePad;
    constexpr int NT = kPlaneThreads;
    constexpr int NV = NX * NZ / 2;                          // float pairs of the plane
    constexpr int NR = (NV + NT - 1) / NT;
    constexpr int NR1 = (NR + 1) / 2;
    // planes of more than 16 pairs per lane (128 x 256): transforms over halves of the lines
    // (one item per lane), and no prefetch (its registers would spill)
    constexpr bool PF = NR <= 16;
    constexpr int ZH = (NX / 2) * AZ > NT ? 2 : 1;
    constexpr int XH = (NZ / 2) * AX > NT ? 2 : 1;
    __shared__ float P[NX * RS];
    __shared__ tw2v TWX[NX], TWZ[NZ];
    const size_t pstride = (size_t)d.ny * NZ;
    {
        const ZArgs& z0 = inst_args<BATCH>(zone, ztab, 0);
        const HxArgs& x0 = inst_args<BATCH>(xone, xtab, 0);
        const Gl<tw2v>* gz = (const Gl<tw2v>*)z0.tw;
        const Gl<tw2v>* gx = (const Gl<tw2v>*)x0.tw;
        for (int t = threadIdx.x; t < NX; t += NT) TWX[t] = gx[t];
        for (int t = threadIdx.x; t < NZ; t += NT) TWZ[t] = gz[t];
    }
    struct Where {
        int inst, c, j;
    };
    auto where = [&](int p) -> Where {
        const int cg = p / d.M;
        const int inst = BATCH ? cg / NC : 0;
        return Where{inst, cg - inst * NC, 1 + (p - cg * d.M)};
    };
    auto live = [&](int q) {   // the next plane from q on (stride: the grid) not gated off
        while (q < nplanes) {
            const ZArgs& za = inst_args<BATCH>(zone, ztab, where(q).inst);
            if (!(za.gate && *(const Gl<int>*)za.gate)) break;
            q += (int)gridDim.x;
        }
        return q;
    };
    auto src_of = [&](int p) -> const Gl<float>* {
        const Where w = where(p);
        const ZArgs& za = inst_args<BATCH>(zone, ztab, w.inst);
        const HxArgs& xa = inst_args<BATCH>(xone, xtab, w.inst);
        return (const Gl<float>*)(ZFIRST ? pick(za.spec, w.c) : pick(xa.spec, w.c)) + (size_t)w.j * NZ;
    };
    float2 v[NR];
    auto load = [&](int p, int r0, int r1) {
        const Gl<float>* in = src_of(p);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r < r0 || r >= r1) continue;
            const int t = min((int)threadIdx.x + r * NT, NV - 1);
            const int i = t / (NZ / 2), k2 = t - i * (NZ / 2);
            const gf2v q = *reinterpret_cast<const Gl<gf2v>*>(in + i * pstride + 2 * k2);
            v[r] = make_float2(q.x, q.y);
        }
    };
    int p = live(blockIdx.x);
    if (PF && p < nplanes) load(p, 0, NR);
    while (p < nplanes) {
        if constexpr (PF) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int t = threadIdx.x + r * NT;
                if (t < NV) {
                    const int i = t / (NZ / 2), k2 = t - i * (NZ / 2);
                    *reinterpret_cast<float2*>(&P[i * RS + 2 * k2]) = v[r];
                }
            }
        } else {
            const Gl<float>* in = src_of(p);
#pragma unroll 8
            for (int r = 0; r < NR; ++r) {
                const int t = threadIdx.x + r * NT;
                const int i = t / (NZ / 2), k2 = t - i * (NZ / 2);
                const gf2v q = *reinterpret_cast<const Gl<gf2v>*>(in + i * pstride + 2 * k2);
                *reinterpret_cast<float2*>(&P[i * RS + 2 * k2]) = make_float2(q.x, q.y);
            }
        }
        __syncthreads();
        const int pn = live(p + (int)gridDim.x);
        if (PF && pn < nplanes) load(pn, 0, NR1);
        int it = threadIdx.x;
        asm volatile("" : "+v"(it));
        auto zpass = [&] {
#pragma unroll
            for (int q = 0; q < ZH; ++q)
                plane_hartley<BZ, AZ, NX / 2 / ZH, RS, true>(P + q * (NX / ZH) * RS, TWZ, it);
        };
        auto xpass = [&] {
#pragma unroll
            for (int q = 0; q < XH; ++q)
                plane_hartley<BX, AX, NZ / 2 / XH, RS, false>(P + q * (NZ / XH), TWX, it);
        };
        if constexpr (ZFIRST) {
            zpass();
            xpass();
        } else {
            xpass();
            zpass();
        }
        if (PF && pn < nplanes) load(pn, NR1, NR);
        const Where w = where(p);
        const ZArgs& za = inst_args<BATCH>(zone, ztab, w.inst);
        if constexpr (ZFIRST) {
            Gl<float>* out = (Gl<float>*)pick(za.spec, w.c) + (size_t)w.j * NZ;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int t = threadIdx.x + r * NT;
                if (t < NV) {
                    const int i = t / (NZ / 2), k2 = t - i * (NZ / 2);
                    const float2 e = *reinterpret_cast<const float2*>(&P[i * RS + 2 * k2]);
                    stc<float>(out + i * pstride + 2 * k2, e.x, e.y);
                }
            }
        } else {
            Gl<double>* uc = (Gl<double>*)pick(za.u, w.c) + (size_t)w.j * NZ;
            Gl<float>* __restrict__ ic = (Gl<float>*)pick(za.inc, w.c);
            const Gl<float>* __restrict__ pc = (const Gl<float>*)pick(za.pinc, w.c);
            if (ic) ic += (size_t)w.j * NZ;
            if (pc) pc += (size_t)w.j * NZ;
            const int h = za.hist ? *(const Gl<int>*)za.hist : -1;
            if (za.hist_out && w.c == 0 && w.j == 1 && threadIdx.x == 0)
                *(Gl<int>*)za.hist_out = h < 2 ? h + 1 : 2;
            const int add = za.add;
            // MODE as in k_hz_out: 0 plain store or add, 1 a later cycle, 2 + H the first cycle
            auto put = [&](auto mc) {
                constexpr int MODE = decltype(mc)::value;
#pragma unroll 4
                for (int r = 0; r < NR; ++r) {
                    const int t = threadIdx.x + r * NT;
                    if (t < NV) {
                        const int i = t / (NZ / 2), k2 = t - i * (NZ / 2);
                        const float2 ef = *reinterpret_cast<const float2*>(&P[i * RS + 2 * k2]);
                        const double e0 = (double)ef.x, e1 = (double)ef.y;
                        const size_t o = i * pstride + 2 * k2;
                        const double2 u = ldg2(uc + o);
                        if constexpr (MODE == 0) {
                            if (add) stc<double>(uc + o, u.x + e0, u.y + e1);
                            else stc<double>(uc + o, e0, e1);
                        } else if constexpr (MODE == 1) {
                            const double2 q = ldg2(ic + o);
                            stc<double>(uc + o, u.x + e0, u.y + e1);
                            stc<float>(ic + o, (float)(q.x + e0), (float)(q.y + e1));
                        } else {
                            double p0 = 0.0, p1 = 0.0;
                            if constexpr (MODE == 3) {
                                const double2 a = ldg2(pc + o);
                                p0 = a.x;
                                p1 = a.y;
                            } else if constexpr (MODE == 4) {
                                const double2 a = ldg2(pc + o), b = ldg2(ic + o);
                                p0 = 2.0 * a.x - b.x;
                                p1 = 2.0 * a.y - b.y;
                            }
                            stc<double>(uc + o, (u.x + p0) + e0, (u.y + p1) + e1);
                            stc<float>(ic + o, (float)(p0 + e0), (float)(p1 + e1));
                        }
                    }
                }
            };
            if (!add || !ic) put(std::integral_constant<int, 0>{});
            else if (h < 0) put(std::integral_constant<int, 1>{});
            else if (h == 0) put(std::integral_constant<int, 2>{});
            else if (h == 1) put(std::integral_constant<int, 3>{});
            else put(std::integral_constant<int, 4>{});
        }
        __syncthreads();   // the plane's LDS is read out before the next one is written
        p = pn;
    }
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
void dht_x_t(hipStream_t s, const Dims& d, const FftPlan& px, const Over<HxArgs>& a, int ncomp) {
    int B, A;
    two_pass_shape(d.nx, B, A);
    const unsigned ni = a.tab ? (unsigned)a.n : 1u;
#define VS_CASE(b, a_)                                                                         \
    if (B == b && A == a_) {                                                                   \
        const int qs = 2 * TwoPass<b, a_>::L;                                                  \
        const dim3 g((d.nz + qs - 1) / qs, d.M, ncomp * ni);                                   \
        if (ncomp > 3) {                                                                       \
            if (a.tab) launch_kernel((k_hx<b, a_, ST, 6, true>), g, dim3(64), 0, s, d, a.one, a.tab); \
            else launch_kernel((k_hx<b, a_, ST, 6, false>), g, dim3(64), 0, s, d, a.one, a.tab); \
        } else if (a.tab) {                                                                    \
            if constexpr (sizeof(ST) == 8)                                                     \
                launch_kernel((k_hx<b, a_, ST, 3, true>), g, dim3(64), 0, s, d, a.one, a.tab); \
        } else {                                                                               \
            launch_kernel((k_hx<b, a_, ST, 3, false>), g, dim3(64), 0, s, d, a.one, a.tab);    \
        }                                                                                      \
        return;                                                                                \
    }
    VS_TWO_PASS_CASES(VS_CASE)
#undef VS_CASE
    // general lengths: LDS Stockham transform, one instance, up to three components a launch
    const int kb = x_modes_per_block(d);
    for (int c0 = 0; c0 < ncomp; c0 += 3) {
        const int nc = ncomp - c0 < 3 ? ncomp - c0 : 3;
        SPtr3<ST> sp{{static_cast<ST*>(a.one.spec[c0]), nc > 1 ? static_cast<ST*>(a.one.spec[c0 + 1]) : nullptr,
                      nc > 2 ? static_cast<ST*>(a.one.spec[c0 + 2]) : nullptr}};
        launch_kernel(k_dht_x<ST>, dim3((d.nz + kb - 1) / kb, d.M, nc), dim3(kBlock), 0, s, d,
                      px, a.one.tw, sp, a.one.gate, kb);
    }
}

template <class ST>
void dht_z_out_t(hipStream_t s, const Dims& d, const FftPlan& pz, const Over<ZArgs>& a, int ncomp) {
    const int nrows = d.nx * d.M;
    int B, A;
    two_pass_shape(d.nz, B, A);
    const unsigned ni = a.tab ? (unsigned)a.n : 1u;
#define VS_CASE(b, a_)                                                                         \
    if (B == b && A == a_) {                                                                   \
        const int rows = 2 * TwoPass<b, a_, z_out_lm<a_, ST>()>::L;                            \
        const dim3 g((nrows + rows - 1) / rows, ncomp * ni);                                   \
        if (ncomp > 3) {                                                                       \
            if (a.tab) launch_kernel((k_hz_out<b, a_, ST, 6, true>), g, dim3(64), 0, s, d, a.one, a.tab); \
            else launch_kernel((k_hz_out<b, a_, ST, 6, false>), g, dim3(64), 0, s, d, a.one, a.tab); \
        } else if (a.tab) {                                                                    \
            if constexpr (sizeof(ST) == 8)                                                     \
                launch_kernel((k_hz_out<b, a_, ST, 3, true>), g, dim3(64), 0, s, d, a.one, a.tab); \
        } else {                                                                               \
            launch_kernel((k_hz_out<b, a_, ST, 3, false>), g, dim3(64), 0, s, d, a.one, a.tab); \
        }                                                                                      \
        return;                                                                                \
    }
    VS_TWO_PASS_CASES(VS_CASE)
#undef VS_CASE
    const int rpb = z_rows_per_block(d);
    for (int c0 = 0; c0 < ncomp; c0 += 3) {
        const int nc = ncomp - c0 < 3 ? ncomp - c0 : 3;
        Ptr3 uu{{a.one.u[c0], nc > 1 ? a.one.u[c0 + 1] : nullptr, nc > 2 ? a.one.u[c0 + 2] : nullptr}};
        SPtr3<ST> sp{{static_cast<ST*>(a.one.spec[c0]), nc > 1 ? static_cast<ST*>(a.one.spec[c0 + 1]) : nullptr,
                      nc > 2 ? static_cast<ST*>(a.one.spec[c0 + 2]) : nullptr}};
        launch_kernel(k_dht_z_out<ST>, dim3((nrows + rpb - 1) / rpb, nc), dim3(kBlock), 0, s,
                      d, pz, a.one.tw, sp, uu, a.one.add, a.one.gate, rpb);
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

void launch_hx(hipStream_t s, const Dims& d, const FftPlan& px, bool f32, int ncomp,
               const Over<HxArgs>& a) {
    if (f32)
        dht_x_t<float>(s, d, px, a, ncomp);
    else
        dht_x_t<double>(s, d, px, a, ncomp);
}

// Blocks of a persistent plane launch: the compute units of the current device.
int plane_blocks() {
    static int n = 0;
    if (n == 0) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            n = cus;
        else
            n = 256;
    }
    return n;
}

bool plane_fits(const Dims& d) {
    int bx, ax, bz, az;
    two_pass_shape(d.nx, bx, ax);
    two_pass_shape(d.nz, bz, az);
    return d.nx == d.nz && bx > 0 && bz > 0 && d.nx <= 128 && d.nx >= 32;
}

bool launch_plane(hipStream_t s, const Dims& d, bool zfirst, int ncomp, const Over<ZArgs>& z,
                  const Over<HxArgs>& x) {
    if (!plane_fits(d) || (ncomp != 3 && ncomp != 6)) return false;
    if (z.one.gate || z.one.add || x.one.gate) return false;
    const bool batch = z.tab != nullptr;
    if (batch != (x.tab != nullptr) || (batch && z.n != x.n)) return false;
    const int ni = batch ? z.n : 1;
    const int nplanes = d.M * ncomp * ni;
    // persistent: one block per CU (the plane takes most of the LDS) up to the plane count
    const dim3 g((unsigned)std::min(nplanes, plane_blocks()));
    const dim3 blk((unsigned)kPlaneThreads);   // the kernels' launch bound
    auto go = [&](auto kf3, auto kf6, auto kt3, auto kt6) {
        if (batch) {
            if (ncomp == 3) launch_kernel(kt3, g, blk, 0, s, d, z.one, z.tab, x.one, x.tab, nplanes);
            else launch_kernel(kt6, g, blk, 0, s, d, z.one, z.tab, x.one, x.tab, nplanes);
        } else {
            if (ncomp == 3) launch_kernel(kf3, g, blk, 0, s, d, z.one, z.tab, x.one, x.tab, nplanes);
            else launch_kernel(kf6, g, blk, 0, s, d, z.one, z.tab, x.one, x.tab, nplanes);
        }
    };
#define VS_PLANE(n, b, a_)                                                                       \
    if (d.nx == n) {                                                                             \
        if (zfirst)                                                                              \
            go(k_hxz_plane<b, a_, b, a_, true, 3, false>, k_hxz_plane<b, a_, b, a_, true, 6, false>, \
               k_hxz_plane<b, a_, b, a_, true, 3, true>, k_hxz_plane<b, a_, b, a_, true, 6, true>); \
        else                                                                                     \
            go(k_hxz_plane<b, a_, b, a_, false, 3, false>, k_hxz_plane<b, a_, b, a_, false, 6, false>, \
               k_hxz_plane<b, a_, b, a_, false, 3, true>, k_hxz_plane<b, a_, b, a_, false, 6, true>); \
        return true;                                                                             \
    }
    VS_PLANE(32, 8, 4)
    VS_PLANE(48, 16, 3)
    VS_PLANE(64, 16, 4)
    VS_PLANE(96, 16, 6)
    VS_PLANE(128, 16, 8)
#undef VS_PLANE
    return false;
}

// The refined mode's FP32 plane forms: square planes of n_x = n_z in {32, 48, 64, 96, 128}
// and the 128 x 256 plane (132 KB of floats).
bool plane32_fits(const Dims& d) {
    int bx, ax, bz, az;
    two_pass_shape(d.nx, bx, ax);
    two_pass_shape(d.nz, bz, az);
    if (!bx || !bz) return false;
    return (d.nx == d.nz && d.nx >= 32 && d.nx <= 128) || (d.nx == 128 && d.nz == 256);
}

bool launch_plane32(hipStream_t s, const Dims& d, bool zfirst, const Over<ZArgs>& z,
                    const Over<HxArgs>& x) {
    if (!plane32_fits(d)) return false;
    const bool batch = z.tab != nullptr;
    if (batch != (x.tab != nullptr) || (batch && z.n != x.n)) return false;
    const int ni = batch ? z.n : 1;
    const int nplanes = d.M * 6 * ni;
    // persistent: as many blocks as fit on the CUs at once (two per CU for planes up to
    // 80 KB of LDS)
    const size_t lds = (size_t)d.nx * (d.nz + kPlanePad) * sizeof(float) + (size_t)(d.nx + d.nz) * sizeof(tw2v);
    const int per_cu = lds <= 80 * 1024 ? 2 : 1;
    const dim3 g((unsigned)std::min(nplanes, per_cu * plane_blocks()));
    const dim3 blk((unsigned)kPlaneThreads);   // the kernels' launch bound
    auto go = [&](auto kf, auto kt) {
        if (batch) launch_kernel(kt, g, blk, 0, s, d, z.one, z.tab, x.one, x.tab, nplanes);
        else launch_kernel(kf, g, blk, 0, s, d, z.one, z.tab, x.one, x.tab, nplanes);
    };
#define VS_PLANE32(nx_, nz_, bx, ax, bz, az)                                                     \
    if (d.nx == nx_ && d.nz == nz_) {                                                            \
        if (zfirst)                                                                              \
            go(k_plane32<bx, ax, bz, az, true, false>, k_plane32<bx, ax, bz, az, true, true>);    \
        else                                                                                     \
            go(k_plane32<bx, ax, bz, az, false, false>, k_plane32<bx, ax, bz, az, false, true>);  \
        return true;                                                                             \
    }
    VS_PLANE32(32, 32, 8, 4, 8, 4)
    VS_PLANE32(48, 48, 16, 3, 16, 3)
    VS_PLANE32(64, 64, 16, 4, 16, 4)
    VS_PLANE32(96, 96, 16, 6, 16, 6)
    VS_PLANE32(128, 128, 16, 8, 16, 8)
    VS_PLANE32(128, 256, 16, 8, 16, 16)
#undef VS_PLANE32
    return false;
}

void launch_hz(hipStream_t s, const Dims& d, const FftPlan& pz, bool f32, int ncomp,
               const Over<ZArgs>& a) {
    if (f32)
        dht_z_out_t<float>(s, d, pz, a, ncomp);
    else
        dht_z_out_t<double>(s, d, pz, a, ncomp);
}

void launch_dht_x(hipStream_t s, const Dims& d, const FftPlan& px, const double2* twx,
                  void* const spec[], int ncomp, bool f32, const int* gate) {
    HxArgs h{};
    for (int c = 0; c < ncomp; ++c) h.spec[c] = spec[c];
    h.tw = twx;
    h.gate = gate;
    launch_hx(s, d, px, f32, ncomp, over_one(h));
}

void launch_dht_z_fwd(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      const double* const f[3], void* const spec[3], int ncomp) {
    // the z pass of the inverse computes the same Hartley sums (H is its own inverse up to
    // the scale, which the tridiagonal solve applies), from FP64 input to FP64 output
    ZArgs z{};
    for (int c = 0; c < ncomp; ++c) {
        z.spec[c] = (void*)f[c];
        z.u[c] = (double*)spec[c];
    }
    z.tw = twz;
    launch_hz(s, d, pz, false, ncomp, over_one(z));
}

void launch_dht_z_out(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      void* const spec[], double* const u[], int ncomp, int add, bool f32,
                      const int* gate) {
    ZArgs z{};
    for (int c = 0; c < ncomp; ++c) {
        z.spec[c] = spec[c];
        z.u[c] = u[c];
    }
    z.tw = twz;
    z.gate = gate;
    z.add = add;
    launch_hz(s, d, pz, f32, ncomp, over_one(z));
}

}  // namespace vs
