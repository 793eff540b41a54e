// Tridiagonal solves in y of the Poisson problems of the main text, eq. (5b) and (5c), per
// Hartley mode (the spectral transforms are in k_spectral.hip), and the residual norms and
// convergence checks that verify every solve on the device.
#include <type_traits>

#include "spectral.h"

namespace vs {

namespace {

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

// T: the arithmetic type of the solve (that of the spectral storage: FP64, or FP32 in the
// refined mode); the pivots come from the FP64 table, rounded to T.
template <int LMAX, class T>
struct SegCoef {
    T c[LMAX];
    T beta, g11l, g11s, g1ll, g1ls;   // G_11 and G_1L for Lm and Lm - 1 rows
};

template <int LMAX, class T>
__device__ __forceinline__ void seg_coef(SegCoef<LMAX, T>& cf, const double* __restrict__ tri,
                                         unsigned cls, unsigned ncls, int M, int Lm) {
    const BufRes r = buf_res(tri, (unsigned)(M + 1) * ncls * 8u);
#pragma unroll
    for (int u = 0; u < LMAX; ++u) cf.c[u] = (u < Lm) ? (T)buf_ld(r, cls * 8u, u * ncls * 8u, tri) : (T)0;
    cf.beta = (T)buf_ld(r, cls * 8u, (unsigned)M * ncls * 8u, tri);
    // G_11(L) = c'_L; G_1L(L) = (-1)^(L-1) c'_1 ... c'_L
    T prod = 1;
    cf.g11l = cf.g11s = cf.g1ll = cf.g1ls = 0;
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

// xch: 512 values of LDS for the exchange of the segment ends; every thread of the 256-thread
// block calls this (it holds two barriers).
template <int S, int LMAX, class T>
__device__ __forceinline__ void seg_solve(T (&x)[LMAX], const SegCoef<LMAX, T>& cf, int k,
                                          bool shortl, int Lm, int nlong, T* xch) {
    const T* c = cf.c;
    // forward elimination in place; q = last d', piL = pi at the last row (phantom row zeroed)
    T acc = 0, pi = 0, q = 0, piL = 0;
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
                x[u] = shortl ? (T)0 : acc;
            } else {
                x[u] = acc;
            }
        }
    }
    // p = first unknown of the zero-end segment solve (back substitution, nothing stored)
    T p = 0;
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
    T P[S], Q[S];
#pragma unroll
    for (int kk = 0; kk < S; ++kk) {
        P[kk] = xch[kk * NM + m];
        Q[kk] = xch[256 + kk * NM + m];
    }
    __syncthreads();   // xch is free again
    T a = 0, b = 0, alp = 0, bep = 0;
    T PH[S], CH[S];
#pragma unroll
    for (int kk = 0; kk < S; ++kk) {
        const bool lng = nlong == 0 || kk < nlong;   // nlong = 0: all segments have Lm rows
        const T g11 = lng ? cf.g11l : cf.g11s;
        const T g1l = lng ? cf.g1ll : cf.g1ls;
        const T rden = (T)1 / ((T)1 - g11 * b);
        const T ph = (P[kk] - g11 * a) * rden;
        const T ch = g1l * rden;
        const T an = Q[kk] - g1l * a + g1l * b * ph;
        const T bn = g11 + g1l * b * ch;
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
    T F = 0, Fk = 0, Fnext = 0;
#pragma unroll
    for (int kk = S - 1; kk >= 0; --kk) {
        if (kk == k) Fnext = F;
        F = PH[kk] - CH[kk] * F;
        if (kk == k) Fk = F;
    }
    // E_{k-1} = alpha_{k-1} - beta_{k-1} F_k
    const T Eprev = k > 0 ? alp - bep * Fk : (T)0;
    // finish the segment bottom up
    T xn = 0, pc = 0;
#pragma unroll
    for (int u = LMAX - 1; u >= 0; --u) {
        if (u < Lm) {
            T f;
            if (u == Lm - 1) {
                pc = shortl ? (T)0 : piL;
                f = shortl ? (T)0 : Fnext * c[u];
            } else if (u == Lm - 2) {
                pc = shortl ? piL : -pc * (cf.beta - c[u]);
                f = shortl ? Fnext * c[u] : (T)0;
            } else {
                pc = -pc * (cf.beta - c[u]);
                f = 0;
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
    const int mode = (int)blockIdx.x * NM + (int)threadIdx.x % NM;   // blockIdx.x: mode block
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
__device__ __forceinline__ void seg_load(ST (&x)[LMAX], const ST* base, unsigned nelem,
                                         unsigned off, unsigned sj, int Lm, ST scale) {
    const BufRes r = buf_res(base, nelem * (unsigned)sizeof(ST));
    const unsigned vo = off * (unsigned)sizeof(ST);
#pragma unroll
    for (int u = 0; u < LMAX; ++u)
        x[u] = (u < Lm) ? scale * (ST)buf_ld(r, vo, u * sj * (unsigned)sizeof(ST), base) : (ST)0;
}

template <int S, int LMAX, class ST>
__device__ __forceinline__ void seg_store(const ST (&x)[LMAX], ST* base, unsigned nelem,
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
    __shared__ ST xch[512];
    SegCoef<LMAX, ST> cf;
    seg_coef<LMAX, ST>(cf, tri, sl.cls, sl.ncls, d.M, sl.Lm);
    ST* col = spec.p[blockIdx.y];
    const unsigned N = (unsigned)(d.nx * d.ny * d.nz);
    ST x[LMAX];
    seg_load<S, LMAX, ST>(x, col, N, sl.off, d.nz, sl.Lm, (ST)scale);
    seg_solve<S, LMAX, ST>(x, cf, sl.k, sl.shortl, sl.Lm, sl.nlong, xch);
    seg_store<S, LMAX, ST>(x, col, N, d.nz, sl);
}

// Segmented vorticity + stream-vector pair: the vorticity modes U_w (f = scale * B) are solved
// and stored in spec, then the stream-vector problem lap psi = -w is solved from them in
// registers, f_j = -h^2 U_w(j) - [p = q = 0]([j = 1] psi_lo + [j = M] psi_hi), into spec2.
// triw holds the vorticity's pivots: tri itself, or those of the shifted operator L_h - a of
// the inertial variant (SM eq. (36)).
// CORR (the corrections of a defect-correction cycle, homogeneous walls): spec holds the
// transformed vorticity residual R_w and spec2 the stream-vector residual R_psi; the
// corrections are U_ew = T^{-1}(scale R_w) and U_epsi = T^{-1}(scale R_psi - h^2 U_ew), since the
// stream-vector correction solves L e_psi = r_psi - e_w.
// Grid: x = mode blocks, y = component (3) [x instances].
template <int S, int LMAX, class ST, int LMF, int NLF, bool CORR, bool BATCH>
__global__ __launch_bounds__(256) void k_tridiag_pair_seg(Dims d, TriArgs one,
                                                         const TriArgs* __restrict__ tab) {
    const int inst = BATCH ? (int)blockIdx.y / 3 : 0;
    const int c3 = (int)blockIdx.y - inst * 3;
    const TriArgs& ta = inst_args<BATCH>(one, tab, inst);
    if (ta.gate && *ta.gate) return;
    SegLane<S> sl = seg_lane<S>(d);
    if (LMF) {
        sl.Lm = LMF;
        sl.nlong = NLF;
        sl.shortl = NLF > 0 && sl.k >= NLF;
    }
    __shared__ ST xch[512];
    SegCoef<LMAX, ST> cf;
    seg_coef<LMAX, ST>(cf, ta.triw, sl.cls, sl.ncls, d.M, sl.Lm);
    ST* col = (ST*)pick(ta.spec, c3);
    ST* col2 = (ST*)pick(ta.spec2, c3);
    const unsigned N = (unsigned)(d.nx * d.ny * d.nz);
    const ST scale = (ST)(d.h * d.h / ((double)d.nx * d.nz));
    ST x[LMAX];
    seg_load<S, LMAX, ST>(x, col, N, sl.off, d.nz, sl.Lm, scale);
    ST y[LMAX];
    if (CORR) seg_load<S, LMAX, ST>(y, col2, N, sl.off, d.nz, sl.Lm, scale);
    const bool m00 = sl.p == 0 && sl.q == 0;
    // the row j = M is the last real row of segment S - 1 (short if nlong > 0)
    const int ulast = sl.nlong > 0 ? sl.Lm - 2 : sl.Lm - 1;
    if (!CORR) {
        // vorticity wall terms, constant over each wall plane: mode (0, 0) only
        const ST a = (ST)pick(ta.olo, c3);
        const ST b = (ST)pick(ta.ohi, c3);
#pragma unroll
        for (int u = 0; u < LMAX; ++u) {
            if (m00 && sl.k == 0 && u == 0) x[u] -= a;
            if (m00 && sl.k == S - 1 && u == ulast) x[u] -= b;
        }
    }
    seg_solve<S, LMAX, ST>(x, cf, sl.k, sl.shortl, sl.Lm, sl.nlong, xch);
    seg_store<S, LMAX, ST>(x, col, N, d.nz, sl);
    // the stream-vector problem has no shift: its own pivots when the vorticity's differ
    if (ta.triw != ta.tri) seg_coef<LMAX, ST>(cf, ta.tri, sl.cls, sl.ncls, d.M, sl.Lm);
    const ST h2 = (ST)(d.h * d.h);
    const ST wlo = CORR ? (ST)0 : (ST)pick(ta.plo, c3);
    const ST whi = CORR ? (ST)0 : (ST)pick(ta.phi, c3);
#pragma unroll
    for (int u = 0; u < LMAX; ++u) {
        ST f = CORR ? y[u] - h2 * x[u] : -h2 * x[u];
        if (m00 && sl.k == 0 && u == 0) f -= wlo;
        if (m00 && sl.k == S - 1 && u == ulast) f -= whi;
        x[u] = f;
    }
    seg_solve<S, LMAX, ST>(x, cf, sl.k, sl.shortl, sl.Lm, sl.nlong, xch);
    seg_store<S, LMAX, ST>(x, col2, N, d.nz, sl);
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
// The source S is stored as SS (double, or float in the refined mode); sums are FP64.
template <bool BATCH, class SS>
__global__ __launch_bounds__(kBlock) void k_resid_flow(Dims d, SlabGrid sg, ResArgs one,
                                                      const ResArgs* __restrict__ tab) {
    __shared__ double sh[4 * 4];
    const int nb = sg.gx * sg.gi;
    const int lbi = xcd_block(blockIdx.x, gridDim.x);
    const int inst = BATCH ? lbi / (3 * nb) : 0;
    const ResArgs& ra = inst_args<BATCH>(one, tab, inst);
    if (ra.gate && *ra.gate) return;
    const double ashift = ra.ashift;
    Gl<double>* __restrict__ partials = (Gl<double>*)ra.part;
    const int lb0 = lbi - inst * 3 * nb;
    const int c = lb0 / nb;
    const int lb = lb0 - c * nb;
    const int bi = lb / sg.gx;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    const Gl<double>* wc = (const Gl<double>*)(c == 0 ? ra.om[0] : c == 1 ? ra.om[1] : ra.om[2]);
    const Gl<SS>* sc = (const Gl<SS>*)(c == 0 ? ra.src[0] : c == 1 ? ra.src[1] : ra.src[2]);
    const Gl<double>* pc = (const Gl<double>*)(c == 0 ? ra.ps[0] : c == 1 ? ra.ps[1] : ra.ps[2]);
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
        auto zpair = [&](const Gl<double>* u, int rb, double, double& zp, double& zm) {
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
                const double b = (double)sc[c0];
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
template <int W, bool BATCH, class SS>
__global__ __launch_bounds__(kBlock) void k_resid_flow2(Dims d, SlabGrid sg, ResArgs one,
                                                       const ResArgs* __restrict__ tab) {
    __shared__ double sh[4 * 4];
    const int nb = sg.gx * sg.gi;
    const int lbi = xcd_block(blockIdx.x, gridDim.x);
    const int inst = BATCH ? lbi / (3 * nb) : 0;
    const ResArgs& ra = inst_args<BATCH>(one, tab, inst);
    if (ra.gate && *ra.gate) return;
    const double ashift = ra.ashift;
    Gl<double>* __restrict__ partials = (Gl<double>*)ra.part;
    const int lb0 = lbi - inst * 3 * nb;
    const int c = lb0 / nb;
    const int lb = lb0 - c * nb;
    const int bi = lb / sg.gx;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    const Gl<double>* wc = (const Gl<double>*)(c == 0 ? ra.om[0] : c == 1 ? ra.om[1] : ra.om[2]);
    const Gl<SS>* sc = (const Gl<SS>*)(c == 0 ? ra.src[0] : c == 1 ? ra.src[1] : ra.src[2]);
    const Gl<double>* pc = (const Gl<double>*)(c == 0 ? ra.ps[0] : c == 1 ? ra.ps[1] : ra.ps[2]);
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
        auto ld2v = [](const Gl<double>* q) { return ldg2(q); };
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
            const double2 b = ldg2(sc + c0);
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

// The first step of the refined mode's first correction cycle: both flow residuals at the
// predicted fields u* = u + p (p of order H: 0, the last increment i1, or 2 i1 - i2; the same
// arithmetic as the update of k_hz_out), r_w = S - L_h omega* (eq. (5b)) and
// r_psi = -omega* - L_h psi* (eq. (5c)), formed in FP64 and stored in FP32 at the node offsets of
// spec (vorticity) and spec2 (stream vector) for the z transform that follows. The walk of
// k_resid_flow2: a block owns one component, W lanes cover 2W consecutive z of one interior
// row, the slab marches along x with the x-neighbours in registers. Wall rows enter as stored
// (their increments are zero).
template <int W, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_rhs_pred(Dims d, SlabGrid sg, RhsFlowArgs one,
                                                    const RhsFlowArgs* __restrict__ tab) {
    const int nb = sg.gx * sg.gi;
    const int lbi = xcd_block(blockIdx.x, gridDim.x);
    const int inst = BATCH ? lbi / (3 * nb) : 0;
    const RhsFlowArgs& a = inst_args<BATCH>(one, tab, inst);
    if (a.gate && *a.gate) return;
    const int lb0 = lbi - inst * 3 * nb;
    const int c = lb0 / nb;
    const int lb = lb0 - c * nb;
    const int bi = lb / sg.gx;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    const int hz = d.nz >> 1;
    if (t >= d.M * hz) return;
    const Gl<double>* wc = (const Gl<double>*)pick(a.om, c);
    const Gl<double>* pc = (const Gl<double>*)pick(a.ps, c);
    const Gl<double>* sc = (const Gl<double>*)pick(a.src, c);
    const Gl<float>* w1 = (const Gl<float>*)pick(a.i1, c);
    const Gl<float>* w2 = (const Gl<float>*)pick(a.i2, c);
    const Gl<float>* p1 = (const Gl<float>*)pick(a.i1, 3 + c);
    const Gl<float>* p2 = (const Gl<float>*)pick(a.i2, 3 + c);
    Gl<float>* ow = (Gl<float>*)pick(a.spec, c);
    Gl<float>* op = (Gl<float>*)pick(a.spec2, c);
    const int h = a.hist ? *a.hist : 0;
    const int jj = t / hz;
    const int k = 2 * (t - jj * hz);
    const int j = jj + 1;
    const int plane = d.ny * d.nz;
    const int off = j * d.nz + k;
    const int ln = threadIdx.x & (W - 1);
    const int k0 = k - 2 * ln;
    const int kpe = (k0 + 2 * W == d.nz) ? 0 : k0 + 2 * W;
    const int kme = (k0 == 0) ? d.nz - 1 : k0 - 1;
    const int i0 = bi * sg.ci;
    const int i1 = min(d.nx, i0 + sg.ci);
    const int im0 = (i0 == 0) ? d.nx - 1 : i0 - 1;
    auto walk = [&](auto hc) {
        constexpr int H = decltype(hc)::value;
        // u* at a pair of nodes and at one node
        auto ld2 = [&](const Gl<double>* u, const Gl<float>* f1, const Gl<float>* f2, int o) -> double2 {
            double2 v = ldg2(u + o);
            if constexpr (H == 1) {
                const double2 e = ldg2(f1 + o);
                v.x = v.x + e.x;
                v.y = v.y + e.y;
            } else if constexpr (H == 2) {
                const double2 e1 = ldg2(f1 + o), e2 = ldg2(f2 + o);
                v.x = v.x + (2.0 * e1.x - e2.x);
                v.y = v.y + (2.0 * e1.y - e2.y);
            }
            return v;
        };
        auto ld1 = [&](const Gl<double>* u, const Gl<float>* f1, const Gl<float>* f2, int o) -> double {
            if constexpr (H == 0) return u[o];
            else if constexpr (H == 1) return u[o] + (double)f1[o];
            else return u[o] + (2.0 * (double)f1[o] - (double)f2[o]);
        };
        auto zn = [&](double2 v, double em, double ep, double& zm0, double& zp1) {
            const double prev = __shfl_up(v.y, 1, W), next = __shfl_down(v.x, 1, W);
            zm0 = ln == 0 ? em : prev;
            zp1 = ln == W - 1 ? ep : next;
        };
        double2 wm = ld2(wc, w1, w2, im0 * plane + off), wx = ld2(wc, w1, w2, i0 * plane + off);
        double2 pm = ld2(pc, p1, p2, im0 * plane + off), px = ld2(pc, p1, p2, i0 * plane + off);
#pragma unroll 2
        for (int i = i0; i < i1; ++i) {
            const int ip = (i + 1 == d.nx) ? 0 : i + 1;
            const int rb = i * plane + j * d.nz;
            const int c0 = rb + k;
            const double2 b = ldg2(sc + c0);
            const double2 ylo = ld2(wc, w1, w2, c0 - d.nz), yhi = ld2(wc, w1, w2, c0 + d.nz);
            const double2 qlo = ld2(pc, p1, p2, c0 - d.nz), qhi = ld2(pc, p1, p2, c0 + d.nz);
            const int ome = rb + kme, ope = rb + kpe;
            const double wem = ld1(wc, w1, w2, ome), wep = ld1(wc, w1, w2, ope);
            const double pem = ld1(pc, p1, p2, ome), pep = ld1(pc, p1, p2, ope);
            // the next plane's centres last: they stay in flight while this plane is formed
            const double2 wp = ld2(wc, w1, w2, ip * plane + off);
            const double2 pp = ld2(pc, p1, p2, ip * plane + off);
            __builtin_amdgcn_sched_barrier(0);
            {
                double zm0, zp1;
                zn(wx, wem, wep, zm0, zp1);
                const double l0 = (wp.x + wm.x + ylo.x + yhi.x + wx.y + zm0 - 6.0 * wx.x) * d.inv_h2;
                const double l1 = (wp.y + wm.y + ylo.y + yhi.y + zp1 + wx.x - 6.0 * wx.y) * d.inv_h2;
                stc<float>(ow + c0, (float)(b.x - l0), (float)(b.y - l1));
            }
            {
                double zm0, zp1;
                zn(px, pem, pep, zm0, zp1);
                const double l0 = (pp.x + pm.x + qlo.x + qhi.x + px.y + zm0 - 6.0 * px.x) * d.inv_h2;
                const double l1 = (pp.y + pm.y + qlo.y + qhi.y + zp1 + px.x - 6.0 * px.y) * d.inv_h2;
                stc<float>(op + c0, (float)(-wx.x - l0), (float)(-wx.y - l1));
            }
            wm = wx;
            wx = wp;
            pm = px;
            px = pp;
        }
    };
    if (h == 0) walk(std::integral_constant<int, 0>{});
    else if (h == 1) walk(std::integral_constant<int, 1>{});
    else walk(std::integral_constant<int, 2>{});
}

// check: relative residual sqrt(sum_c r^2 / sum_c b~^2) in a fixed summation order; sets the
// convergence flag that gates the following cycles, counts the cycle and raises ST_NOCONV
// on the last allowed cycle, ST_NONFINITE on NaN/Inf.
__global__ __launch_bounds__(1024) void k_check(const double* __restrict__ partials,
                                               int nblocks, double rtol, int last_cycle,
                                               double* scal, int* istat, const int* gate,
                                               int slot0, int role, double* log) {
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
        if (role == 1) scal[SC_RELRES_W] = rel;
        if (role == 2 && log) {   // the step's record (the per-step log; see flow_check.h)
            const double rw = scal[SC_RELRES_W];
            const int n = istat[IS_LOGN];
            double* r = log + (size_t)(n % kLogCap) * kLogFields;
            r[0] = (double)n;
            r[1] = (double)istat[IS_CYCLES];
            r[2] = (rw != rw || rw > rel) ? rw : rel;
            r[3] = scal[SC_V];
            r[4] = scal[SC_A];
            r[5] = scal[SC_LAMV];
            r[6] = scal[SC_GAMMA];
            r[7] = (double)((conv && rw <= rtol) ? 1 : 0);
            istat[IS_LOGN] = n + 1;
        }
    }
    if (!conv && last_cycle) istat[IS_FLAGS] |= ST_NOCONV;
    if (!isfinite(rr) || !isfinite(bb)) istat[IS_FLAGS] |= ST_NONFINITE;
}

// Convergence checks of the two flow solves of a step in one launch (flow_check.h); one block
// per instance.
template <bool BATCH>
__global__ __launch_bounds__(1024) void k_check_flow(int nblocks, int last_cycle, ChkArgs one,
                                                    const ChkArgs* __restrict__ tab) {
    const ChkArgs& a = inst_args<BATCH>(one, tab, (int)blockIdx.x);
    if (a.gate && *a.gate) return;
    __shared__ double sh[4 * 16];
    flow_check_block(a.part, nblocks, a.rtol, a.scal, a.istat, sh, last_cycle, a.log);
}

}  // namespace

// Segment layout for M interior rows: S lanes per mode, at most LMAX rows per lane.
// 0 = the twisted two-lane solve (M < 4 or M > 256).
int seg_shape(int M) {
    if (M < 4 || M > 256) return 0;
    if (M <= 32) return 8;
    if (M <= 64) return 16;
    if (M <= 128) return 32;
    return 832;   // S = 8, LMAX = 32
}

// Segmented solves. Grids with ny = n in {32, 48, 64, 96, 128, 256} (M = n - 2) get their
// segment lengths as compile-time constants; other M in [4, 256] a run-time length.
template <int S, int LMAX, class ST, int LMF, int NLF>
void seg_launch_single(hipStream_t s, const Dims& d, const double* tri, void* const spec[3],
                       int ncomp, const int* gate) {
    const double scale = d.h * d.h / ((double)d.nx * d.nz);
    const dim3 grid((unsigned)(((long)d.nx * d.nz * S + 255) / 256), ncomp);
    launch_kernel((k_tridiag_seg<S, LMAX, ST, LMF, NLF>), grid, dim3(256), 0, s, d, tri,
                  sptr<ST>(spec, ncomp), gate, scale);
}

template <int S, int LMAX, class ST, int LMF, int NLF>
void seg_launch_pair(hipStream_t s, const Dims& d, bool corr, const Over<TriArgs>& a) {
    const unsigned ni = a.tab ? (unsigned)a.n : 1u;
    const dim3 grid((unsigned)(((long)d.nx * d.nz * S + 255) / 256), 3 * ni);
    if constexpr (sizeof(ST) == 4) {   // the correction form serves the refined mode only
        if (corr) {
            if (a.tab) launch_kernel((k_tridiag_pair_seg<S, LMAX, ST, LMF, NLF, true, true>), grid, dim3(256), 0, s, d, a.one, a.tab);
            else launch_kernel((k_tridiag_pair_seg<S, LMAX, ST, LMF, NLF, true, false>), grid, dim3(256), 0, s, d, a.one, a.tab);
            return;
        }
    }
    {
        if (a.tab) launch_kernel((k_tridiag_pair_seg<S, LMAX, ST, LMF, NLF, false, true>), grid, dim3(256), 0, s, d, a.one, a.tab);
        else launch_kernel((k_tridiag_pair_seg<S, LMAX, ST, LMF, NLF, false, false>), grid, dim3(256), 0, s, d, a.one, a.tab);
    }
}

#define VS_SEG_SHAPES(X)                                                                       \
    switch (d.M) {                                                                             \
    case 30: X(4, 8, 8, 2); return true;                                                       \
    case 46: X(4, 16, 12, 2); return true;                                                     \
    case 62: X(4, 16, 16, 2); return true;                                                     \
    case 94: X(8, 16, 12, 6); return true;                                                     \
    case 126: X(8, 16, 16, 6); return true;                                                    \
    case 254: X(16, 16, 16, 14); return true;                                                  \
    default: break;                                                                            \
    }                                                                                          \
    switch (seg_shape(d.M)) {                                                                  \
    case 8: X(4, 8, 0, 0); return true;                                                        \
    case 16: X(4, 16, 0, 0); return true;                                                      \
    case 32: X(4, 32, 0, 0); return true;                                                      \
    case 832: X(8, 32, 0, 0); return true;                                                     \
    default: return false;                                                                     \
    }

template <class ST>
bool seg_single(hipStream_t s, const Dims& d, const double* tri, void* const spec[3], int ncomp,
                const int* gate) {
#define VS_X(S_, L_, F_, N_) seg_launch_single<S_, L_, ST, F_, N_>(s, d, tri, spec, ncomp, gate)
    VS_SEG_SHAPES(VS_X)
#undef VS_X
}

// The pair solves have a second layout for each compile-time row count, twice (or half) the
// lanes per mode, which the autotuner may pick (seg_alt).
template <class ST>
bool seg_pair(hipStream_t s, const Dims& d, bool corr, const Over<TriArgs>& a) {
#define VS_X(S_, L_, F_, N_) seg_launch_pair<S_, L_, ST, F_, N_>(s, d, corr, a)
    if (tuning_for(d).seg_alt) {
        switch (d.M) {
        case 30: VS_X(8, 4, 4, 6); return true;
        case 46: VS_X(8, 8, 6, 6); return true;
        case 62: VS_X(8, 8, 8, 6); return true;
        case 94: VS_X(16, 8, 6, 14); return true;
        case 126: VS_X(16, 8, 8, 14); return true;
        case 254: VS_X(8, 32, 32, 6); return true;
        default: break;
        }
    }
    VS_SEG_SHAPES(VS_X)
#undef VS_X
}

bool seg_has_alt(int M) {
    return M == 30 || M == 46 || M == 62 || M == 94 || M == 126 || M == 254;
}

template <class ST>
void tridiag_y_t(hipStream_t s, const Dims& d, const double* tri, void* const spec[3], int ncomp,
                 const int* gate) {
    const double3 z = make_double3(0.0, 0.0, 0.0);
    if (seg_single<ST>(s, d, tri, spec, ncomp, gate)) return;
    const double scale = d.h * d.h / ((double)d.nx * d.nz);
    const dim3 grid((2 * d.nx * d.nz + 63) / 64, ncomp);
    launch_kernel(k_tridiag_y<ST>, grid, dim3(64), 0, s, d, tri, sptr<ST>(spec, ncomp), gate,
                  scale, z, z);
}

void launch_tridiag_y(hipStream_t s, const Dims& d, const double* tri, void* const spec[3],
                      int ncomp, bool f32, const int* gate) {
    if (f32)
        tridiag_y_t<float>(s, d, tri, spec, ncomp, gate);
    else
        tridiag_y_t<double>(s, d, tri, spec, ncomp, gate);
}

void launch_tri_pair(hipStream_t s, const Dims& d, bool f32, bool corr, const Over<TriArgs>& a) {
    const bool done = f32 ? seg_pair<float>(s, d, corr, a) : seg_pair<double>(s, d, corr, a);
    if (done) return;
    // M < 4 or M > 256: the two-lane solves, one instance (no correction form)
    const TriArgs& t = a.one;
    const double scale = d.h * d.h / ((double)d.nx * d.nz);
    const dim3 grid((2 * d.nx * d.nz + 63) / 64, 3);
    const double3 olo = make_double3(t.olo[0], t.olo[1], t.olo[2]);
    const double3 ohi = make_double3(t.ohi[0], t.ohi[1], t.ohi[2]);
    const double3 lo = make_double3(t.plo[0], t.plo[1], t.plo[2]);
    const double3 hi = make_double3(t.phi[0], t.phi[1], t.phi[2]);
    void* const sp[3] = {t.spec[0], t.spec[1], t.spec[2]};
    void* const sp2[3] = {t.spec2[0], t.spec2[1], t.spec2[2]};
    if (f32) {
        launch_kernel(k_tridiag_y<float>, grid, dim3(64), 0, s, d, t.triw, sptr<float>(sp, 3),
                      (const int*)nullptr, scale, olo, ohi);
        launch_kernel(k_tridiag_psi<float>, grid, dim3(64), 0, s, d, t.tri, sptr<float>(sp, 3),
                      sptr<float>(sp2, 3), lo, hi);
    } else {
        launch_kernel(k_tridiag_y<double>, grid, dim3(64), 0, s, d, t.triw, sptr<double>(sp, 3),
                      (const int*)nullptr, scale, olo, ohi);
        launch_kernel(k_tridiag_psi<double>, grid, dim3(64), 0, s, d, t.tri, sptr<double>(sp, 3),
                      sptr<double>(sp2, 3), lo, hi);
    }
}

void launch_tridiag_pair(hipStream_t s, const Dims& d, const double* tri, const double* triw,
                         void* const spec[3], void* const spec2[3], const double om_lo[3],
                         const double om_hi[3], const double psi_lo[3], const double psi_hi[3],
                         bool f32) {
    TriArgs t{};
    t.tri = tri;
    t.triw = triw ? triw : tri;
    for (int c = 0; c < 3; ++c) {
        t.spec[c] = spec[c];
        t.spec2[c] = spec2[c];
        t.olo[c] = om_lo[c];
        t.ohi[c] = om_hi[c];
        t.plo[c] = psi_lo[c];
        t.phi[c] = psi_hi[c];
    }
    t.gate = nullptr;
    launch_tri_pair(s, d, f32, false, over_one(t));
}

bool fused_flow_ok(const Dims& d) {
    int B, A;
    two_pass_shape(d.nx, B, A);
    if (!B) return false;
    two_pass_shape(d.nz, B, A);
    if (!B) return false;
    return seg_shape(d.M) != 0;
}

// Residual blocks per component: slabs of x-planes chosen so that about a thousand blocks
// cover one component (each component adds as many again).
static SlabGrid resid_grid(const Dims& d) { return slab_grid(d.M * d.nz, d.nx, 1024); }

int resid_blocks(const Dims& d) {
    const SlabGrid g = resid_grid(d);
    return g.gx * g.gi;
}

// The block cap per component (tuned; 1024 by default).
static SlabGrid resid_flow_grid(const Dims& d) {
    const int maxb = tuning_for(d).res_maxb;
    return slab_grid(d.nz % 32 == 0 ? d.M * d.nz / 2 : d.M * d.nz, d.nx, maxb);
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

template <class SS>
static void resid_flow_t(hipStream_t s, const Dims& d, const Over<ResArgs>& a) {
    const SlabGrid g = resid_flow_grid(d);
    const unsigned ni = a.tab ? (unsigned)a.n : 1u;
    const dim3 gr(3 * g.gx * g.gi * ni);
    auto go = [&](auto kt, auto kf) {
        if (a.tab) launch_kernel(kt, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
        else launch_kernel(kf, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
    };
    if (d.nz % 128 == 0) go(k_resid_flow2<64, true, SS>, k_resid_flow2<64, false, SS>);
    else if (d.nz % 64 == 0) go(k_resid_flow2<32, true, SS>, k_resid_flow2<32, false, SS>);
    else if (d.nz % 32 == 0) go(k_resid_flow2<16, true, SS>, k_resid_flow2<16, false, SS>);
    else go(k_resid_flow<true, SS>, k_resid_flow<false, SS>);
}

void launch_resid_flow_over(hipStream_t s, const Dims& d, bool f32src, const Over<ResArgs>& a) {
    if (f32src)
        resid_flow_t<float>(s, d, a);
    else
        resid_flow_t<double>(s, d, a);
}

void launch_rhs_pred(hipStream_t s, const Dims& d, const Over<RhsFlowArgs>& a) {
    const SlabGrid g = slab_grid(d.M * (d.nz / 2), d.nx, tuning_for(d).res_maxb);
    const unsigned ni = a.tab ? (unsigned)a.n : 1u;
    const dim3 gr(3 * g.gx * g.gi * ni);
    auto go = [&](auto kt, auto kf) {
        if (a.tab) launch_kernel(kt, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
        else launch_kernel(kf, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
    };
    if (d.nz % 128 == 0) go(k_rhs_pred<64, true>, k_rhs_pred<64, false>);
    else if (d.nz % 64 == 0) go(k_rhs_pred<32, true>, k_rhs_pred<32, false>);
    else if (d.nz % 32 == 0) go(k_rhs_pred<16, true>, k_rhs_pred<16, false>);
    else go(k_rhs_pred<8, true>, k_rhs_pred<8, false>);
}

void launch_resid_flow(hipStream_t s, const Dims& d, const double* const om[3],
                       const double* const src[3], const double* const ps[3], double ashift,
                       double* partials) {
    ResArgs r{};
    for (int c = 0; c < 3; ++c) {
        r.om[c] = om[c];
        r.src[c] = src[c];
        r.ps[c] = ps[c];
    }
    r.part = partials;
    r.ashift = ashift;
    launch_resid_flow_over(s, d, false, over_one(r));
}

void launch_check_flow_over(hipStream_t s, const Dims& d, int last_cycle, const Over<ChkArgs>& a) {
    const unsigned ni = a.tab ? (unsigned)a.n : 1u;
    const int nb = resid_flow_blocks(d);
    if (a.tab)
        launch_kernel(k_check_flow<true>, dim3(ni), dim3(1024), 0, s, nb, last_cycle, a.one, a.tab);
    else
        launch_kernel(k_check_flow<false>, dim3(1), dim3(1024), 0, s, nb, last_cycle, a.one, a.tab);
}

void launch_check_flow(hipStream_t s, const Dims& d, const double* partials, double rtol,
                       double* scal, int* istat) {
    ChkArgs c{};
    c.part = partials;
    c.scal = scal;
    c.istat = istat;
    c.rtol = rtol;
    launch_check_flow_over(s, d, 1, over_one(c));
}

void launch_check(hipStream_t s, const double* partials, int nblocks, double rtol, int cycle,
                  int last_cycle, double* scal, int* istat, const int* gate, int slot0, int role,
                  double* log) {
    (void)cycle;
    launch_kernel(k_check, dim3(1), dim3(1024), 0, s, partials, nblocks, rtol,
                       last_cycle, scal, istat, gate, slot0, role, log);
}

}  // namespace vs
