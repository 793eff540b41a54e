// Explicit stencils of one time step on gfx950:
//   phi-update (main text eq. (5a), SM (29a)/(38)) with the velocity v = curl psi (eq. (3))
//   fused in registers; the chemical potential (SM eq. (35) bending, eq. F_CH / SM (31)
//   Cahn-Hilliard); the volume and area integrals (SM eq. (37), (32)) with the penalty
//   multipliers (SM "Lagrange multipliers"); the vorticity source of eq. (5b).
// Each kernel runs in FP64, or in the refined mode's precision (T = float: mu and S stored as
// float, the phi update and the source computed in FP32, phi kept in FP64), over one instance
// or over every instance of a grid class in one launch (BATCH: per-instance arguments from a
// device table; see Over in vs_internal.h). Launch shape and wall handling: stencil.h.
#include "flow_check.h"
#include "stencil.h"

namespace vs {

namespace {

// Pairs of two consecutive z values in the arithmetic type T.
template <class T>
struct P2;
template <>
struct P2<double> {
    using t = double2;
    typedef double v __attribute__((ext_vector_type(2)));   // the same pair for memory access
};
template <>
struct P2<float> {
    using t = float2;
    typedef float v __attribute__((ext_vector_type(2)));
};
// Objects in global memory. Pointers that a batched launch reads from its device table are
// generic; typing the accesses through them as global keeps them global loads and stores
// (flat ones would also count against the LDS counter).
template <class T>
using Gl = __attribute__((address_space(1))) T;

// An FP64 field's pair converted to T (identity in FP64).
template <class T>
__device__ __forceinline__ typename P2<T>::t cvt2(double2 v) {
    typename P2<T>::t r;
    r.x = (T)v.x;
    r.y = (T)v.y;
    return r;
}
template <class T>
__device__ __forceinline__ typename P2<T>::t ldt2(const Gl<T>* q) {
    const typename P2<T>::v m = *reinterpret_cast<const Gl<typename P2<T>::v>*>(q);
    typename P2<T>::t r;
    r.x = m.x;
    r.y = m.y;
    return r;
}
__device__ __forceinline__ double2 ldd2(const Gl<double>* q) { return ldt2<double>(q); }
template <class T>
__device__ __forceinline__ void stt2(Gl<T>* q, T a, T b) {
    typename P2<T>::v m;
    m.x = a;
    m.y = b;
    *reinterpret_cast<Gl<typename P2<T>::v>*>(q) = m;
}

// The instance of a block and its index inside the instance: logical blocks (after the XCD
// order over the whole grid) are split into runs of nb per instance.
template <bool BATCH>
__device__ __forceinline__ int split_block(int lb, int nb, int& inst) {
    if (!BATCH) {
        inst = 0;
        return lb;
    }
    inst = lb / nb;
    return lb - inst * nb;
}
template <bool BATCH, class A>
__device__ __forceinline__ A inst_args(const A& one, const A* __restrict__ tab, int inst) {
    if constexpr (BATCH)
        return tab[inst];
    else
        return one;
}

// phi_out = phi + dt [ M (L_h mu + lambda_V) - v . D phi ], v = curl psi (eq. (3)) on the
// interior rows and the wall speed on the walls; D is the central difference, L_h the
// 7-point Laplacian with mirror ghosts in y (phi[-1] = phi[1], phi[ny] = phi[ny-2]).
// Marching along x: each lane owns one (j, k) and walks a slab of consecutive x-planes (the
// tuned adv_slab, 4 by default),
// keeping phi, mu, psi_y and psi_z of the planes i-1, i, i+1 in registers, so the
// x-neighbours are not re-read; the y and z neighbours come through the cache. The increment
// is computed in T and added to the FP64 phi.

template <bool BATCH, class T>
__global__ __launch_bounds__(kBlock) void k_advance_x(Dims d, SlabGrid sg, AdvArgs one,
                                                      const AdvArgs* __restrict__ tab) {
    const int nb = sg.gx * sg.gi;
    int inst;
    const int lb = split_block<BATCH>(xcd_block(blockIdx.x, gridDim.x), nb, inst);
    const AdvArgs a = inst_args<BATCH>(one, tab, inst);
    if (a.ck_part && lb == 0) {
        // the previous step's flow check, off the critical path of this kernel's other blocks
        __shared__ double shc[4 * 16];
        flow_check_block(a.ck_part, a.ck_nb, a.ck_rtol, a.scal, a.ck_istat, shc, 1, a.ck_log);
    }
    const Gl<double>* __restrict__ phi = (const Gl<double>*)a.phi;
    const Gl<T>* __restrict__ mu = (const Gl<T>*)a.mu;
    const Gl<double>* __restrict__ px = (const Gl<double>*)a.ps[0];
    const Gl<double>* __restrict__ py = (const Gl<double>*)a.ps[1];
    const Gl<double>* __restrict__ pz = (const Gl<double>*)a.ps[2];
    Gl<double>* __restrict__ out = (Gl<double>*)a.out;
    const int bi = lb / sg.gx;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    if (t >= d.ny * d.nz) return;
    const int j = t / d.nz, k = t - (t / d.nz) * d.nz;
    const int i0 = bi * sg.ci, i1 = min(d.nx, i0 + sg.ci);
    const int plane = d.ny * d.nz;
    const int jp = (j + 1 == d.ny) ? d.ny - 2 : j + 1;   // mirror ghosts (phi, mu)
    const int jm = (j == 0) ? 1 : j - 1;
    const int kp = (k + 1 == d.nz) ? 0 : k + 1;
    const int km = (k == 0) ? d.nz - 1 : k - 1;
    const bool wall = (j == 0 || j == d.ny - 1);
    const int o = j * d.nz + k;                          // offset inside a plane
    const int oyp = jp * d.nz + k, oym = jm * d.nz + k, ozp = j * d.nz + kp, ozm = j * d.nz + km;
    const T lam = (T)a.scal[SC_LAMV];
    const T i2h = (T)d.inv_2h, ih2 = (T)d.inv_h2;
    auto pl = [&](int i) { return (size_t)((i + d.nx) % d.nx) * plane; };
    size_t b = pl(i0 - 1);
    double phm = phi[b + o];
    T mum = mu[b + o], pym = wall ? (T)0 : (T)py[b + o], pzm = wall ? (T)0 : (T)pz[b + o];
    b = pl(i0);
    double ph0 = phi[b + o];
    T mu0 = mu[b + o], py0 = wall ? (T)0 : (T)py[b + o], pz0 = wall ? (T)0 : (T)pz[b + o];
    for (int i = i0; i < i1; ++i) {
        const size_t bc = (size_t)i * plane, bn = pl(i + 1);
        const double php = phi[bn + o];
        const T mup = mu[bn + o];
        const T pyp = wall ? (T)0 : (T)py[bn + o], pzp = wall ? (T)0 : (T)pz[bn + o];
        const T lmu = (mup + mum + mu[bc + oyp] + mu[bc + oym] + mu[bc + ozp] + mu[bc + ozm] -
                       (T)6 * mu0) * ih2;
        const T dx = ((T)php - (T)phm) * i2h;
        const T dy = ((T)phi[bc + oyp] - (T)phi[bc + oym]) * i2h;
        const T dz = ((T)phi[bc + ozp] - (T)phi[bc + ozm]) * i2h;
        T vx = 0, vy = 0, vz;
        if (j == 0) {
            vz = (T)a.vz_lo;
        } else if (j == d.ny - 1) {
            vz = (T)a.vz_hi;
        } else {
            vx = (((T)pz[bc + oyp] - (T)pz[bc + oym]) - ((T)py[bc + ozp] - (T)py[bc + ozm])) * i2h;
            vy = (((T)px[bc + ozp] - (T)px[bc + ozm]) - (pzp - pzm)) * i2h;
            vz = ((pyp - pym) - ((T)px[bc + oyp] - (T)px[bc + oym])) * i2h;
        }
        const T inc = (T)a.dt * ((T)a.mob * (lmu + lam) - (vx * dx + vy * dy + vz * dz));
        out[bc + o] = ph0 + (double)inc;
        phm = ph0; ph0 = php;
        mum = mu0; mu0 = mup;
        pym = py0; py0 = pyp;
        pzm = pz0; pz0 = pzp;
    }
}

// k_advance_x with two consecutive z per lane. W lanes (64, 32 or 16) cover 2W consecutive z of
// one row, n_z a multiple of 2W: every FP64 field access moves 16 bytes, and the z neighbours
// inside the pair come from the pair itself, across lanes by width-W shuffles, and the
// segment's two edge values by one load each (the same address in every lane of a segment).
// The psi values of the wall rows are loaded too (in bounds, unused there), so that no branch
// guards a load, and the next plane's centres are loaded last (pinned by a scheduling
// barrier), so they stay in flight while the current plane is computed. Same arithmetic per
// node as k_advance_x, so the two forms agree bit for bit.

template <int W, bool BATCH, class T>
__global__ __launch_bounds__(kBlock) void k_advance_x2(Dims d, SlabGrid sg, AdvArgs one,
                                                       const AdvArgs* __restrict__ tab) {
    using V = typename P2<T>::t;
    const int nb = sg.gx * sg.gi;
    int inst;
    const int lb = split_block<BATCH>(xcd_block(blockIdx.x, gridDim.x), nb, inst);
    const AdvArgs a = inst_args<BATCH>(one, tab, inst);
    if (a.ck_part && lb == 0) {
        __shared__ double shc[4 * 16];
        flow_check_block(a.ck_part, a.ck_nb, a.ck_rtol, a.scal, a.ck_istat, shc, 1, a.ck_log);
    }
    const Gl<double>* __restrict__ phi = (const Gl<double>*)a.phi;
    const Gl<T>* __restrict__ mu = (const Gl<T>*)a.mu;
    const Gl<double>* __restrict__ px = (const Gl<double>*)a.ps[0];
    const Gl<double>* __restrict__ py = (const Gl<double>*)a.ps[1];
    const Gl<double>* __restrict__ pz = (const Gl<double>*)a.ps[2];
    Gl<double>* __restrict__ out = (Gl<double>*)a.out;
    const int bi = lb / sg.gx;
    const int hz = d.nz >> 1;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    if (t >= d.ny * hz) return;
    const int j = t / hz, k = 2 * (t - (t / hz) * hz);
    const int i0 = bi * sg.ci, i1 = min(d.nx, i0 + sg.ci);
    const int plane = d.ny * d.nz;
    const int jp = (j + 1 == d.ny) ? d.ny - 2 : j + 1;   // mirror ghosts (phi, mu)
    const int jm = (j == 0) ? 1 : j - 1;
    const int ln = threadIdx.x & (W - 1);
    const int k0 = k - 2 * ln;
    const int kpe = (k0 + 2 * W == d.nz) ? 0 : k0 + 2 * W;
    const int kme = (k0 == 0) ? d.nz - 1 : k0 - 1;
    const int o = j * d.nz + k;
    const int oyp = jp * d.nz + k, oym = jm * d.nz + k;
    const int re = j * d.nz;                             // row start inside a plane
    const T lam = (T)a.scal[SC_LAMV];
    const T i2h = (T)d.inv_2h, ih2 = (T)d.inv_h2;
    // z neighbours (zp, zm) of node k and of node k + 1 from the pair v; el, er: the values
    // just before the wave's first z and just after its last
    auto zn = [&](V v, T el, T er, T& zpa, T& zma, T& zpb, T& zmb) {
        const T prev = __shfl_up(v.y, 1, W), next = __shfl_down(v.x, 1, W);
        zpa = v.y;
        zma = ln == 0 ? el : prev;
        zpb = ln == W - 1 ? er : next;
        zmb = v.x;
    };
    auto pl = [&](int i) { return (size_t)((i + d.nx) % d.nx) * plane; };
    size_t b = pl(i0 - 1);
    double2 phm = ldd2(phi + b + o);
    V mum = ldt2<T>(mu + b + o), pym = cvt2<T>(ldd2(py + b + o)), pzm = cvt2<T>(ldd2(pz + b + o));
    b = pl(i0);
    double2 ph0 = ldd2(phi + b + o);
    V mu0 = ldt2<T>(mu + b + o), py0 = cvt2<T>(ldd2(py + b + o)), pz0 = cvt2<T>(ldd2(pz + b + o));
    for (int i = i0; i < i1; ++i) {
        const size_t bc = (size_t)i * plane, bn = pl(i + 1);
        const V myp = ldt2<T>(mu + bc + oyp), mym = ldt2<T>(mu + bc + oym);
        const V fyp = cvt2<T>(ldd2(phi + bc + oyp)), fym = cvt2<T>(ldd2(phi + bc + oym));
        const V zyp = cvt2<T>(ldd2(pz + bc + oyp)), zym = cvt2<T>(ldd2(pz + bc + oym));
        const V xyp = cvt2<T>(ldd2(px + bc + oyp)), xym = cvt2<T>(ldd2(px + bc + oym));
        const V pxc = cvt2<T>(ldd2(px + bc + o));
        const size_t ro = bc + re;
        const T mu_l = mu[ro + kme], mu_r = mu[ro + kpe];
        const T ph_l = (T)phi[ro + kme], ph_r = (T)phi[ro + kpe];
        const T py_l = (T)py[ro + kme], py_r = (T)py[ro + kpe];
        const T px_l = (T)px[ro + kme], px_r = (T)px[ro + kpe];
        // the next plane's centres last: they stay in flight while this plane is computed
        const double2 php = ldd2(phi + bn + o);
        const V mup = ldt2<T>(mu + bn + o);
        const V pyp = cvt2<T>(ldd2(py + bn + o)), pzp = cvt2<T>(ldd2(pz + bn + o));
        __builtin_amdgcn_sched_barrier(0);
        const V f0 = cvt2<T>(ph0), fp = cvt2<T>(php), fm = cvt2<T>(phm);
        T mzpa, mzma, mzpb, mzmb, fzpa, fzma, fzpb, fzmb;
        T yzpa, yzma, yzpb, yzmb, xzpa, xzma, xzpb, xzmb;
        zn(mu0, mu_l, mu_r, mzpa, mzma, mzpb, mzmb);
        zn(f0, ph_l, ph_r, fzpa, fzma, fzpb, fzmb);
        zn(py0, py_l, py_r, yzpa, yzma, yzpb, yzmb);
        zn(pxc, px_l, px_r, xzpa, xzma, xzpb, xzmb);
        double2 res;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const T c_mup = h ? mup.y : mup.x, c_mum = h ? mum.y : mum.x;
            const T c_mu0 = h ? mu0.y : mu0.x;
            const T c_php = h ? fp.y : fp.x, c_phm = h ? fm.y : fm.x;
            const double c_ph0 = h ? ph0.y : ph0.x;
            const T lmu = (c_mup + c_mum + (h ? myp.y : myp.x) + (h ? mym.y : mym.x) +
                           (h ? mzpb : mzpa) + (h ? mzmb : mzma) - (T)6 * c_mu0) * ih2;
            const T dx = (c_php - c_phm) * i2h;
            const T dy = ((h ? fyp.y : fyp.x) - (h ? fym.y : fym.x)) * i2h;
            const T dz = ((h ? fzpb : fzpa) - (h ? fzmb : fzma)) * i2h;
            T vx = 0, vy = 0, vz;
            if (j == 0) {
                vz = (T)a.vz_lo;
            } else if (j == d.ny - 1) {
                vz = (T)a.vz_hi;
            } else {
                vx = (((h ? zyp.y : zyp.x) - (h ? zym.y : zym.x)) -
                      ((h ? yzpb : yzpa) - (h ? yzmb : yzma))) * i2h;
                vy = (((h ? xzpb : xzpa) - (h ? xzmb : xzma)) -
                      ((h ? pzp.y : pzp.x) - (h ? pzm.y : pzm.x))) * i2h;
                vz = (((h ? pyp.y : pyp.x) - (h ? pym.y : pym.x)) -
                      ((h ? xyp.y : xyp.x) - (h ? xym.y : xym.x))) * i2h;
            }
            const T inc = (T)a.dt * ((T)a.mob * (lmu + lam) - (vx * dx + vy * dy + vz * dz));
            const double r = c_ph0 + (double)inc;
            if (h) res.y = r; else res.x = r;
        }
        stt2<double>(out + bc + o, res.x, res.y);
        phm = ph0; ph0 = php;
        mum = mu0; mu0 = mup;
        pym = py0; py0 = pyp;
        pzm = pz0; pz0 = pzp;
    }
}

// V = (|Omega| + h^3 sum_w phi)/2, A = 3/(2 sqrt 2) h^3 sum_w(...); then
// lambda_V = 2 rate_V (V0 - V)/(M |Omega|) and gamma_A = gamma0 + k_A (A - A0)/A0
// (off when k_A = 0 or A0 = 0); init also sets V0 = V, A0 = A. Every block of the calling
// kernel sums the block partials in the same fixed order and gets the same gamma_A; block 0
// writes the scalars. In three parts, so that the loads overlap other loads and the block
// sum rides on a barrier the caller has anyway:
//   va_load    each thread loads its kVaPer partials per slot (b = thread + u * blockDim);
//   va_reduce  per-thread sums in that order, wave sums into sh (before a barrier);
//   va_final   after the barrier: every thread adds the wave sums in order and finishes.
// More than kVaPer * blockDim partials (x-planes above 2^18 nodes) take a plain loop.
constexpr int kVaPer = 4;
struct VaLoads {
    double v[2][kVaPer];
};
__device__ __forceinline__ void va_load(const MuArgs& va, int nblocks, VaLoads& L) {
#pragma unroll
    for (int u = 0; u < kVaPer; ++u) {
        const int b = threadIdx.x + u * blockDim.x;
        const int bc = b < nblocks ? b : 0;
        L.v[0][u] = va.part[0 * kMaxPartialBlocks + bc];
        L.v[1][u] = va.part[1 * kMaxPartialBlocks + bc];
    }
}
__device__ __forceinline__ void va_reduce(const MuArgs& va, int nblocks, const VaLoads& L,
                                          double* sh) {
    double acc[2] = {0.0, 0.0};
    if (nblocks <= kVaPer * (int)blockDim.x) {
#pragma unroll
        for (int u = 0; u < kVaPer; ++u) {
            const bool ok = (int)(threadIdx.x + u * blockDim.x) < nblocks;
            acc[0] += ok ? L.v[0][u] : 0.0;
            acc[1] += ok ? L.v[1][u] : 0.0;
        }
    } else {
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
            acc[0] += va.part[0 * kMaxPartialBlocks + b];
            acc[1] += va.part[1 * kMaxPartialBlocks + b];
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) sh[q * 16 + w] = s;
    }
}
__device__ __forceinline__ double va_final(const MuArgs& va, const Dims& d, const double* sh,
                                           bool writer) {
    const int nw = blockDim.x >> 6;
    double acc[2] = {0.0, 0.0};
    for (int q = 0; q < 2; ++q)
        for (int i = 0; i < nw; ++i) acc[q] += sh[q * 16 + i];
    const double h3 = d.h * d.h * d.h;
    const double vol = (double)d.nx * d.nz * (d.ny - 1) * h3;
    const double V = 0.5 * (vol + h3 * acc[0]);
    const double A = 3.0 / (2.0 * 1.4142135623730951) * h3 * acc[1];
    const double V0 = va.init ? V : va.scal[SC_V0];
    const double A0 = va.init ? A : va.scal[SC_A0];
    double gamma = va.gamma0;
    if (va.k_A != 0.0 && A0 > 0.0) gamma += va.k_A * (A - A0) / A0;
    if (writer && threadIdx.x == 0) {
        if (va.init) {
            va.scal[SC_V0] = V;
            va.scal[SC_A0] = A;
        }
        va.scal[SC_V] = V;
        va.scal[SC_A] = A;
        va.scal[SC_LAMV] = 2.0 * va.rate_V * (V0 - V) / (va.mob * vol);
        va.scal[SC_GAMMA] = gamma;
        if (!isfinite(V) || !isfinite(A)) va.istat[IS_FLAGS] |= ST_NONFINITE;
    }
    return gamma;
}

// mu from phi. Bending (SM eq. (35)): g = phi^3 - phi - eps^2 L_h phi,
// mu = C_b [(3 phi^2 - 1) g - eps^2 L_h g] - gamma_A L_h phi. Cahn-Hilliard:
// mu = phi^3 - phi - sigma L_h phi. g never reaches HBM.
//
// mu by x-marching tiles. A block owns a kMuTY x kMuTZ tile of (j, k) and walks kMuNI
// consecutive x-planes: a 4-plane ring of phi (halo 2 in y and z) and a 3-plane ring of g
// (halo 1) live in LDS, the phi planes are prefetched into registers kMuD planes ahead of
// their use, and every x-neighbour comes from the rings instead of L2. Rows beyond the
// walls are filled with the mirror image (j -> -j, ny-1+m -> ny-1-m), so g computed there is
// the mirror ghost of g. Sums run in the order of lap7, so the result equals the plain
// stencil's bit for bit.
constexpr int kMuTY = 8, kMuTZ = 32, kMuNI = 8;
constexpr int kPY = kMuTY + 4, kPZ = kMuTZ + 4, kPN = kPY * kPZ;
constexpr int kGY = kMuTY + 2, kGZ = kMuTZ + 2, kGN = kGY * kGZ;
constexpr int kPre = (kPN + kBlock - 1) / kBlock;
// phi slot: every lane loads and stores (padded to whole blocks), one block more so that the
// padding elements of the g slot read inside it
constexpr int kPS = (kPre + 1) * kBlock;
constexpr int kGI = (kGN + kBlock - 1) / kBlock;
constexpr int kGS = kGI * kBlock;                // g slot, padded likewise
constexpr int kMuD = 2;                          // phi planes in flight ahead of their use
static_assert(((kGS - 1) / kGZ + 2) * kPZ + kGZ < kPS, "padded g nodes read inside the phi slot");

// Store through a buffer resource over one x-plane: a lane outside the grid passes an
// offset past the plane's extent and the hardware drops its store, so the store needs no
// branch (a branch around it would make the compiler wait for every load in flight).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void plane_store(double* plane_base, unsigned plane_bytes,
                                            unsigned byte_off, double v) {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(plane_base, 0, (int)plane_bytes, 0x00020000);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, byte_off, 0, 0);
}
__device__ __forceinline__ void plane_store(float* plane_base, unsigned plane_bytes,
                                            unsigned byte_off, double v) {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(plane_base, 0, (int)plane_bytes, 0x00020000);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)v), r, byte_off, 0, 0);
}

__device__ __forceinline__ int mirror_row(int j, int ny) {
    j = j < 0 ? -j : (j > ny - 1 ? 2 * (ny - 1) - j : j);
    return j < 0 ? 0 : (j > ny - 1 ? ny - 1 : j);   // only rows no output needs get clamped
}
__device__ __forceinline__ int wrap_mod(int k, int n) {
    k %= n;
    return k < 0 ? k + n : k;
}

// The plane loop is straight-line code: a fixed kMuNI steps, fully unrolled, no branch
// around a load or a store (planes past the slab end are computed on wrapped planes and
// their stores dropped; padding lanes load and store inside padded LDS slots). That keeps
// the compiler's memory-counter waits exact, so the kMuD planes in flight are really in
// flight while the block computes. Arithmetic is FP64; mu is stored as MT (double, or float
// in the refined mode).
template <bool BEND, bool BATCH, class MT>
__global__ __launch_bounds__(kBlock) void k_mu_tile(Dims d, int va_nb, MuArgs one,
                                                   const MuArgs* __restrict__ tab) {
    __shared__ double P[4][kPS];
    __shared__ double G[BEND ? 3 : 1][BEND ? kGS : 1];
    __shared__ double shv[2 * 16];
    const int tz_n = (d.nz + kMuTZ - 1) / kMuTZ;
    const int ty_n = (d.ny + kMuTY - 1) / kMuTY;
    const int nbi = ty_n * tz_n * ((d.nx + kMuNI - 1) / kMuNI);
    int inst;
    const int lb = split_block<BATCH>(xcd_block(blockIdx.x, gridDim.x), nbi, inst);
    const MuArgs va = inst_args<BATCH>(one, tab, inst);
    const Gl<double>* __restrict__ phi = (const Gl<double>*)va.phi;
    MT* __restrict__ mu = (MT*)va.mu;   // stored through a buffer resource
    const double C_b = va.C_b, eps = va.eps, sigma = va.sigma;
    const int ic = lb / (ty_n * tz_n);
    const int rem = lb - ic * ty_n * tz_n;
    const int j0 = (rem / tz_n) * kMuTY, k0 = (rem - (rem / tz_n) * tz_n) * kMuTZ;
    const int i0 = ic * kMuNI, i1 = min(d.nx, i0 + kMuNI);
    const int plane = d.ny * d.nz;
    // region element e -> node offset inside a plane (mirror rows, periodic z); padding
    // elements load node 0
    int roff[kPre];
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
        const int e = threadIdx.x + q * kBlock;
        const int r = e / kPZ, c = e - (e / kPZ) * kPZ;
        roff[q] = (e < kPN) ? mirror_row(j0 - 2 + r, d.ny) * d.nz + wrap_mod(k0 - 2 + c, d.nz) : 0;
    }
    auto fetch = [&](int i, double (&v)[kPre]) {
        const Gl<double>* src = phi + (size_t)wrap_mod(i, d.nx) * plane;
#pragma unroll
        for (int q = 0; q < kPre; ++q) v[q] = src[roff[q]];
    };
    auto put = [&](double* dst, const double (&v)[kPre]) {
#pragma unroll
        for (int q = 0; q < kPre; ++q) dst[threadIdx.x + q * kBlock] = v[q];
    };
    auto slot = [](int m) { return m & 3; };   // m >= -2 + 4 below
    const double eps2 = eps * eps;
    // g on the (kMuTY + 2) x (kMuTZ + 2) halo tile of plane m; the padding elements compute
    // on phi rows inside the padded slot and land in the g slot's padding
    auto make_g = [&](int m) {
        const double* pc = P[slot(m + 4)];
        const double* pm = P[slot(m + 3)];
        const double* pp = P[slot(m + 5)];
        double* g = G[BEND ? (m + 3) % 3 : 0];
#pragma unroll
        for (int q = 0; q < kGI; ++q) {
            const int e = threadIdx.x + q * kBlock;
            const int r = e / kGZ, c = e - (e / kGZ) * kGZ;
            const int x = (r + 1) * kPZ + (c + 1);
            const double p = pc[x];
            const double l = (pp[x] + pm[x] + pc[x + kPZ] + pc[x - kPZ] + pc[x + 1] + pc[x - 1] - 6.0 * p) * d.inv_h2;
            g[e] = p * p * p - p - eps2 * l;
        }
    };
    // prologue: phi planes i0-2 .. i0+1 (loads all in flight together), gamma_A from the
    // volume/area partials, g planes i0-1, i0
    {
        VaLoads vl;
        va_load(va, va_nb, vl);            // first, so their sums need not wait for phi
        double w0[kPre], w1[kPre], w2[kPre], w3[kPre];
        fetch(i0 - 2, w0);
        fetch(i0 - 1, w1);
        fetch(i0, w2);
        fetch(i0 + 1, w3);
        va_reduce(va, va_nb, vl, shv);
        put(P[slot(i0 + 2)], w0);
        put(P[slot(i0 + 3)], w1);
        put(P[slot(i0 + 4)], w2);
        put(P[slot(i0 + 5)], w3);
    }
    __syncthreads();
    const double gamma = va_final(va, d, shv, lb == 0);
    if (BEND) {
        make_g(i0 - 1);
        make_g(i0);
    }
    // phi(i0 + s + 2) is put at step s from register set s % kMuD, fetched kMuD steps earlier
    double v[kMuD][kPre];
#pragma unroll
    for (int s = 0; s < kMuD; ++s) fetch(i0 + 2 + s, v[s]);
    const int tj = threadIdx.x / kMuTZ, tk = threadIdx.x - (threadIdx.x / kMuTZ) * kMuTZ;
    const int j = j0 + tj, k = k0 + tk;
    const bool out = j < d.ny && k < d.nz;
    const unsigned pbytes = (unsigned)plane * (unsigned)sizeof(MT);
    const unsigned oofs = (unsigned)(j * d.nz + k) * (unsigned)sizeof(MT);
#pragma unroll
    for (int s = 0; s < kMuNI; ++s) {
        const int i = i0 + s;
        __syncthreads();                         // the slot of phi(i-2) and g(i-2) are free
        put(P[slot(i + 6)], v[s % kMuD]);        // phi(i+2)
        __syncthreads();
        fetch(i + 2 + kMuD, v[s % kMuD]);        // in flight during the next kMuD steps
        if (BEND) make_g(i + 1);
        __syncthreads();
        const double* pc = P[slot(i + 4)];
        const int x = (tj + 2) * kPZ + (tk + 2);
        const double p = pc[x];
        const double lphi = (P[slot(i + 5)][x] + P[slot(i + 3)][x] + pc[x + kPZ] + pc[x - kPZ] +
                             pc[x + 1] + pc[x - 1] - 6.0 * p) * d.inv_h2;
        double m;
        if (!BEND) {
            m = p * p * p - p - sigma * lphi;
        } else {
            const double* gc = G[(i + 3) % 3];
            const int y = (tj + 1) * kGZ + (tk + 1);
            const double g0 = gc[y];
            const double gs = G[(i + 4) % 3][y] + G[(i + 2) % 3][y] + gc[y + kGZ] + gc[y - kGZ] +
                              gc[y + 1] + gc[y - 1];
            const double lg = (gs - 6.0 * g0) * d.inv_h2;
            m = C_b * ((3.0 * p * p - 1.0) * g0 - eps2 * lg) - gamma * lphi;
        }
        // lanes outside the grid, and planes past the slab end, have their stores dropped
        const bool keep = out && i < i1;
        plane_store(mu + (size_t)(keep ? i : 0) * plane, pbytes, keep ? oofs : pbytes, m);
    }
}

// mu by register marching, for n_z = 64 ZPL (ZPL in {1, 2, 4}): one wave covers whole z rows,
// ZPL consecutive z per lane, so the periodic z neighbours come from the lane's own values and,
// at its ends, from the previous and next lane (a rotation across the whole wave). A wave owns
// RJ consecutive rows and walks ni consecutive x-planes; the phi planes i .. i+3 of the rows
// j0-2 .. j0+RJ+1 (mirror rows past the walls, so g there is the mirror ghost of g) and g of the
// planes i-1 .. i+1 stay in registers, and L_h phi of a plane is kept from the g computation
// of that plane. The phi plane three ahead is loaded first in each step, so it is in flight
// while the step computes. No LDS: the halo rows of a wave are read again by its neighbours
// through the cache. Same sums in the same order as k_mu_tile, so the two agree bit for bit.
// Four waves per block share the volume/area reduction.
template <bool BEND, bool BATCH, class MT, int ZPL, int RJ>
__global__ __launch_bounds__(kBlock) void k_mu_reg(Dims d, int va_nb, int ni, MuArgs one,
                                                  const MuArgs* __restrict__ tab) {
    constexpr int NR = RJ + 4;                    // phi rows j0-2 .. j0+RJ+1
    __shared__ double shv[2 * 16];
    const int ngr = (d.ny + 4 * RJ - 1) / (4 * RJ);   // groups of four waves' rows
    const int nsl = (d.nx + ni - 1) / ni;
    int inst;
    const int lb = split_block<BATCH>(xcd_block(blockIdx.x, gridDim.x), ngr * nsl, inst);
    const MuArgs va = inst_args<BATCH>(one, tab, inst);
    const Gl<double>* __restrict__ phi = (const Gl<double>*)va.phi;
    MT* __restrict__ mu = (MT*)va.mu;   // stored through a buffer resource
    const int sl = lb / ngr, gr = lb - sl * ngr;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j0 = (gr * 4 + wv) * RJ;
    const int i0 = sl * ni, i1 = min(d.nx, i0 + ni);
    const int plane = d.ny * d.nz;
    const int zo = lane * ZPL;
    const double eps2 = va.eps * va.eps, C_b = va.C_b, sigma = va.sigma;
    const int lprev = (lane + 63) & 63, lnext = (lane + 1) & 63;
    int roff[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) roff[r] = mirror_row(j0 - 2 + r, d.ny) * d.nz + zo;
    auto fetch = [&](int i, double (&v)[NR][ZPL]) {
        const Gl<double>* src = phi + (size_t)wrap_mod(i, d.nx) * plane;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if constexpr (ZPL == 1) {
                v[r][0] = src[roff[r]];
            } else {
#pragma unroll
                for (int q = 0; q < ZPL; q += 2) {
                    const double2 t = ldd2(src + roff[r] + q);
                    v[r][q] = t.x;
                    v[r][q + 1] = t.y;
                }
            }
        }
    };
    // z neighbours of value q of a row held as ZPL values per lane (periodic over the wave)
    auto zpair = [&](const double (&v)[ZPL], int q, double& zp, double& zm) {
        zm = q > 0 ? v[q > 0 ? q - 1 : 0] : __shfl(v[ZPL - 1], lprev, 64);
        zp = q < ZPL - 1 ? v[q < ZPL - 1 ? q + 1 : 0] : __shfl(v[0], lnext, 64);
    };
    // g and L_h phi of the plane held in b (x neighbours a, c) on the rows j0-1+r0 ..
    // j0-1+r0+n-1; rows are indexed from j0-2 in the phi arrays
    auto make_g = [&](const double (&a)[NR][ZPL], const double (&b)[NR][ZPL],
                      const double (&c)[NR][ZPL], double (&g)[RJ + 2][ZPL],
                      double (&lp)[RJ + 2][ZPL]) {
#pragma unroll
        for (int r = 0; r < RJ + 2; ++r) {
            const int R = r + 1;                  // phi row of g row j0-1+r
#pragma unroll
            for (int q = 0; q < ZPL; ++q) {
                double zp, zm;
                zpair(b[R], q, zp, zm);
                const double p = b[R][q];
                const double l = (c[R][q] + a[R][q] + b[R + 1][q] + b[R - 1][q] + zp + zm - 6.0 * p) * d.inv_h2;
                lp[r][q] = l;
                g[r][q] = p * p * p - p - eps2 * l;
            }
        }
    };
    // volume/area scalars and gamma_A, shared by the block (every block sums the partials)
    double gamma;
    {
        VaLoads vl;
        va_load(va, va_nb, vl);
        va_reduce(va, va_nb, vl, shv);
        __syncthreads();
        gamma = va_final(va, d, shv, lb == 0);
    }
    double A[NR][ZPL], B[NR][ZPL], C[NR][ZPL], D[NR][ZPL];
    double g0[RJ + 2][ZPL], g1[RJ + 2][ZPL], g2[RJ + 2][ZPL];
    double L1[RJ + 2][ZPL], L2[RJ + 2][ZPL];
    // warm-up: phi(i0-2 .. i0+2); g(i0-1) from phi(i0-2 .. i0), g(i0) from phi(i0-1 .. i0+1)
    fetch(i0 - 2, A);
    fetch(i0 - 1, B);
    fetch(i0, C);
    fetch(i0 + 1, D);
    if (BEND) make_g(A, B, C, g0, L1);           // g(i0-1) (L1 overwritten below)
    make_g(B, C, D, g1, L1);                      // g(i0), L_h phi(i0)
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int q = 0; q < ZPL; ++q) {
            A[r][q] = C[r][q];
            B[r][q] = D[r][q];
        }
    fetch(i0 + 2, C);                             // A = phi(i0), B = phi(i0+1), C = phi(i0+2)
    const unsigned pbytes = (unsigned)plane * (unsigned)sizeof(MT);
    for (int i = i0; i < i1; ++i) {
        fetch(i + 3, D);                          // in flight during this step
        if (BEND) make_g(A, B, C, g2, L2);        // g(i+1), L_h phi(i+1)
        else make_g(A, B, C, g2, L2);             // (CH: only L_h phi(i+1) is used)
#pragma unroll
        for (int r = 0; r < RJ; ++r) {
            const int j = j0 + r;
            const bool keep = j < d.ny;
#pragma unroll
            for (int q = 0; q < ZPL; ++q) {
                const double p = A[r + 2][q];
                const double lphi = L1[r + 1][q];
                double m;
                if (!BEND) {
                    m = p * p * p - p - sigma * lphi;
                } else {
                    double zp, zm;
                    zpair(g1[r + 1], q, zp, zm);
                    const double g = g1[r + 1][q];
                    const double gs = g2[r + 1][q] + g0[r + 1][q] + g1[r + 2][q] + g1[r][q] + zp + zm;
                    const double lg = (gs - 6.0 * g) * d.inv_h2;
                    m = C_b * ((3.0 * p * p - 1.0) * g - eps2 * lg) - gamma * lphi;
                }
                const unsigned off = (unsigned)(j * d.nz + zo + q) * (unsigned)sizeof(MT);
                plane_store(mu + (size_t)i * plane, pbytes, keep ? off : pbytes, m);
            }
        }
#pragma unroll
        for (int r = 0; r < RJ + 2; ++r)
#pragma unroll
            for (int q = 0; q < ZPL; ++q) {
                g0[r][q] = g1[r][q];
                g1[r][q] = g2[r][q];
                L1[r][q] = L2[r][q];
            }
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int q = 0; q < ZPL; ++q) {
                A[r][q] = B[r][q];
                B[r][q] = C[r][q];
                C[r][q] = D[r][q];
            }
    }
}

// Block partials of sum_w phi and sum_w [(eps/2)|D phi|^2 + (phi^2-1)^2/(4 eps)]
// (trapezoid weights w = 1/2 on the wall rows). Each thread owns one (j, k) and walks ci
// consecutive x-planes, keeping phi of the planes i-1, i, i+1 in registers; the partial of
// the instance's logical block b is written to slot b: fixed order, deterministic.
template <bool BATCH>
__global__ __launch_bounds__(kBlock) void k_va_partials(Dims d, SlabGrid sg, VaArgs one,
                                                       const VaArgs* __restrict__ tab) {
    __shared__ double sh[2 * 16];
    const int nb = sg.gx * sg.gi;
    int inst;
    const int lb = split_block<BATCH>(xcd_block(blockIdx.x, gridDim.x), nb, inst);
    const VaArgs va = inst_args<BATCH>(one, tab, inst);
    const Gl<double>* __restrict__ phi = (const Gl<double>*)va.phi;
    const double eps = va.eps;
    const int bi = lb / sg.gx;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (t < d.ny * d.nz) {
        const int j = t / d.nz;
        const int k = t - j * d.nz;
        const double w = (j == 0 || j == d.ny - 1) ? 0.5 : 1.0;
        const double inv4e = 0.25 / eps;
        const int i0 = bi * sg.ci, i1 = min(d.nx, (bi + 1) * sg.ci);
        // phi of the planes i-1, i, i+1 at (j, k) in registers; y, z neighbours via the cache
        const int plane = d.ny * d.nz;
        const int o = j * d.nz + k;
        const int oyp = ((j + 1 == d.ny) ? d.ny - 2 : j + 1) * d.nz + k;
        const int oym = ((j == 0) ? 1 : j - 1) * d.nz + k;
        const int ozp = j * d.nz + ((k + 1 == d.nz) ? 0 : k + 1);
        const int ozm = j * d.nz + ((k == 0) ? d.nz - 1 : k - 1);
        double pm = phi[(size_t)((i0 + d.nx - 1) % d.nx) * plane + o];
        double p0 = phi[(size_t)i0 * plane + o];
#pragma unroll 4
        for (int i = i0; i < i1; ++i) {
            const size_t bc = (size_t)i * plane;
            const double pp = phi[(size_t)((i + 1) % d.nx) * plane + o];
            const double p = p0;
            const double dx = (pp - pm) * d.inv_2h;
            const double dy = (phi[bc + oyp] - phi[bc + oym]) * d.inv_2h;
            const double dz = (phi[bc + ozp] - phi[bc + ozm]) * d.inv_2h;
            const double q = p * p - 1.0;
            acc[0] += w * p;
            acc[1] += w * (0.5 * eps * (dx * dx + dy * dy + dz * dz) + q * q * inv4e);
            pm = p0;
            p0 = pp;
        }
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        Gl<double>* part = (Gl<double>*)va.part;
        part[0 * kMaxPartialBlocks + lb] = acc[0];
        part[1 * kMaxPartialBlocks + lb] = acc[1];
    }
}


// k_va_partials with two consecutive z per lane (W-lane row segments, as k_advance_x2):
// 16-byte loads, z neighbours from the pair, shuffles and the wave's edge values.
template <int W, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_va_partials2(Dims d, SlabGrid sg, VaArgs one,
                                                        const VaArgs* __restrict__ tab) {
    __shared__ double sh[2 * 16];
    const int nb = sg.gx * sg.gi;
    int inst;
    const int lb = split_block<BATCH>(xcd_block(blockIdx.x, gridDim.x), nb, inst);
    const VaArgs va = inst_args<BATCH>(one, tab, inst);
    const Gl<double>* __restrict__ phi = (const Gl<double>*)va.phi;
    const double eps = va.eps;
    const int bi = lb / sg.gx;
    const int hz = d.nz >> 1;
    const int t = (lb - bi * sg.gx) * kBlock + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (t < d.ny * hz) {
        const int j = t / hz;
        const int k = 2 * (t - j * hz);
        const double w = (j == 0 || j == d.ny - 1) ? 0.5 : 1.0;
        const double inv4e = 0.25 / eps;
        const int i0 = bi * sg.ci, i1 = min(d.nx, (bi + 1) * sg.ci);
        const int plane = d.ny * d.nz;
        const int o = j * d.nz + k;
        const int oyp = ((j + 1 == d.ny) ? d.ny - 2 : j + 1) * d.nz + k;
        const int oym = ((j == 0) ? 1 : j - 1) * d.nz + k;
        const int ln = threadIdx.x & (W - 1);
        const int k0 = k - 2 * ln;
        const int kpe = (k0 + 2 * W == d.nz) ? 0 : k0 + 2 * W;
        const int kme = (k0 == 0) ? d.nz - 1 : k0 - 1;
        const int re = j * d.nz;
        auto ld2v = [](const Gl<double>* q) { return ldd2(q); };
        double2 pm = ld2v(phi + (size_t)((i0 + d.nx - 1) % d.nx) * plane + o);
        double2 p0 = ld2v(phi + (size_t)i0 * plane + o);
#pragma unroll 2
        for (int i = i0; i < i1; ++i) {
            const size_t bc = (size_t)i * plane;
            const int inx = (i + 1 == d.nx) ? 0 : i + 1;
            const double2 pp = ld2v(phi + (size_t)inx * plane + o);
            const double2 yp = ld2v(phi + bc + oyp), ym = ld2v(phi + bc + oym);
            const double em = phi[bc + re + kme], ep = phi[bc + re + kpe];
            const double prev = __shfl_up(p0.y, 1, W), next = __shfl_down(p0.x, 1, W);
            const double zma = ln == 0 ? em : prev, zpb = ln == W - 1 ? ep : next;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double p = h ? p0.y : p0.x;
                const double dx = ((h ? pp.y : pp.x) - (h ? pm.y : pm.x)) * d.inv_2h;
                const double dy = ((h ? yp.y : yp.x) - (h ? ym.y : ym.x)) * d.inv_2h;
                const double dz = ((h ? zpb : p0.y) - (h ? p0.x : zma)) * d.inv_2h;
                const double q = p * p - 1.0;
                acc[0] += w * p;
                acc[1] += w * (0.5 * eps * (dx * dx + dy * dy + dz * dz) + q * q * inv4e);
            }
            pm = p0;
            p0 = pp;
        }
    }
    block_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        Gl<double>* part = (Gl<double>*)va.part;
        part[0 * kMaxPartialBlocks + lb] = acc[0];
        part[1 * kMaxPartialBlocks + lb] = acc[1];
    }
}

// Vorticity source S = (1/eta) D phi x D mu (main text eq. (5b)) at the interior rows, stored
// so that the transform and the residual of the vorticity solve read it as a plain field. mu is
// read as T (double, or float in the refined mode); S is computed and stored in FP64 in both
// modes: the small components of psi respond to white noise in S far more than to S itself
// (their spectrum has little weight in the lowest modes, which the two inverse Laplacians
// amplify most), so FP32 rounding of S alone would cost them relative errors of order 1e-6.
// The inertial variant (SM eq. (36), implicit in time, FP64 only) stores S - a omega^n
// instead, the right-hand side of (L_h - a) omega^{n+1}, a = rho / (eta dt).
template <bool BATCH, class T>
__global__ __launch_bounds__(kBlock) void k_source(Dims d, SrcArgs one, const SrcArgs* __restrict__ tab) {
    const int gx = gridDim.x;
    const int lbg = xcd_block(blockIdx.x + gx * blockIdx.y, gx * gridDim.y);
    const int ig = lbg / gx;                      // instance * nx + i
    const int inst = BATCH ? ig / d.nx : 0;
    const int i = ig - inst * d.nx;
    const SrcArgs a = inst_args<BATCH>(one, tab, inst);
    const int t = (lbg - ig * gx) * kBlock + threadIdx.x;
    if (t >= d.ny * d.nz) return;
    const int j = t / d.nz, k = t - (t / d.nz) * d.nz;
    if (j == 0 || j == d.ny - 1) return;
    const Gl<double>* __restrict__ phi = (const Gl<double>*)a.phi;
    const Gl<T>* __restrict__ mu = (const Gl<T>*)a.mu;
    const Nbr n = neighbours_mirror(d, i, j, k);
    const double fx = (phi[n.xp] - phi[n.xm]) * d.inv_2h, fy = (phi[n.yp] - phi[n.ym]) * d.inv_2h,
                 fz = (phi[n.zp] - phi[n.zm]) * d.inv_2h;
    const double mx = ((double)mu[n.xp] - (double)mu[n.xm]) * d.inv_2h,
                 my = ((double)mu[n.yp] - (double)mu[n.ym]) * d.inv_2h,
                 mz = ((double)mu[n.zp] - (double)mu[n.zm]) * d.inv_2h;
    double s0 = (fy * mz - fz * my) * a.inv_eta;
    double s1 = (fz * mx - fx * mz) * a.inv_eta;
    double s2 = (fx * my - fy * mx) * a.inv_eta;
    if (a.a != 0.0) {
        s0 -= a.a * ((const Gl<double>*)a.om[0])[n.c];
        s1 -= a.a * ((const Gl<double>*)a.om[1])[n.c];
        s2 -= a.a * ((const Gl<double>*)a.om[2])[n.c];
    }
    ((Gl<double>*)a.src[0])[n.c] = s0;
    ((Gl<double>*)a.src[1])[n.c] = s1;
    ((Gl<double>*)a.src[2])[n.c] = s2;
}


// k_source with two consecutive z per lane (W-lane row segments, as k_advance_x2): 16-byte
// loads and stores of FP64 fields, z neighbours from the pair, shuffles and the wave's edge
// values. Same arithmetic per node as k_source.
template <int W, bool BATCH, class T>
__global__ __launch_bounds__(kBlock) void k_source2(Dims d, SrcArgs one, const SrcArgs* __restrict__ tab) {
    const int gx = gridDim.x;
    const int lbg = xcd_block(blockIdx.x + gx * blockIdx.y, gx * gridDim.y);
    const int ig = lbg / gx;                      // instance * nx + i
    const int inst = BATCH ? ig / d.nx : 0;
    const int i = ig - inst * d.nx;
    const SrcArgs a = inst_args<BATCH>(one, tab, inst);
    const int hz = d.nz >> 1;
    const int t = (lbg - ig * gx) * kBlock + threadIdx.x;
    if (t >= d.ny * hz) return;
    const int j = t / hz, k = 2 * (t - (t / hz) * hz);
    if (j == 0 || j == d.ny - 1) return;   // whole W-lane segments: each lies in one row
    const Gl<double>* __restrict__ phi = (const Gl<double>*)a.phi;
    const Gl<T>* __restrict__ mu = (const Gl<T>*)a.mu;
    const int plane = d.ny * d.nz;
    const int ip = (i + 1 == d.nx) ? 0 : i + 1;
    const int im = (i == 0) ? d.nx - 1 : i - 1;
    const int ln = threadIdx.x & (W - 1);
    const int k0 = k - 2 * ln;
    const int kpe = (k0 + 2 * W == d.nz) ? 0 : k0 + 2 * W;
    const int kme = (k0 == 0) ? d.nz - 1 : k0 - 1;
    const int rb = i * plane + j * d.nz;
    const int c = rb + k;
    auto ldm = [&](int q) {   // mu pair as FP64
        const typename P2<T>::t v = ldt2<T>(mu + q);
        return make_double2((double)v.x, (double)v.y);
    };
    const double2 fxp = ldd2(phi + ip * plane + j * d.nz + k), fxm = ldd2(phi + im * plane + j * d.nz + k);
    const double2 fyp = ldd2(phi + c + d.nz), fym = ldd2(phi + c - d.nz);
    const double2 mxp = ldm(ip * plane + j * d.nz + k), mxm = ldm(im * plane + j * d.nz + k);
    const double2 myp = ldm(c + d.nz), mym = ldm(c - d.nz);
    const double2 fc = ldd2(phi + c), mc = ldm(c);
    const double fem = phi[rb + kme], fep = phi[rb + kpe];
    const double mem = (double)mu[rb + kme], mep = (double)mu[rb + kpe];
    const double fprev = __shfl_up(fc.y, 1, W), fnext = __shfl_down(fc.x, 1, W);
    const double mprev = __shfl_up(mc.y, 1, W), mnext = __shfl_down(mc.x, 1, W);
    const double fzma = ln == 0 ? fem : fprev, fzpb = ln == W - 1 ? fep : fnext;
    const double mzma = ln == 0 ? mem : mprev, mzpb = ln == W - 1 ? mep : mnext;
    double r[3][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double fx = ((h ? fxp.y : fxp.x) - (h ? fxm.y : fxm.x)) * d.inv_2h;
        const double fy = ((h ? fyp.y : fyp.x) - (h ? fym.y : fym.x)) * d.inv_2h;
        const double fz = ((h ? fzpb : fc.y) - (h ? fc.x : fzma)) * d.inv_2h;
        const double mx = ((h ? mxp.y : mxp.x) - (h ? mxm.y : mxm.x)) * d.inv_2h;
        const double my = ((h ? myp.y : myp.x) - (h ? mym.y : mym.x)) * d.inv_2h;
        const double mz = ((h ? mzpb : mc.y) - (h ? mc.x : mzma)) * d.inv_2h;
        r[0][h] = (fy * mz - fz * my) * a.inv_eta;
        r[1][h] = (fz * mx - fx * mz) * a.inv_eta;
        r[2][h] = (fx * my - fy * mx) * a.inv_eta;
    }
    if (a.a != 0.0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double2 w = ldd2((const Gl<double>*)a.om[q] + c);
            r[q][0] -= a.a * w.x;
            r[q][1] -= a.a * w.y;
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) stt2<double>((Gl<double>*)a.src[q] + c, r[q][0], r[q][1]);
}

// dst[(i, j, k)] = prof[j]: the no-body channel fields as initial guesses and wall rows.
__global__ __launch_bounds__(kBlock) void k_fill_profile(double* __restrict__ dst, Dims d,
                                                        const double* __restrict__ prof) {
    int i, j, k;
    bool ok;
    plane_index(d, i, j, k, ok);
    if (!ok) return;
    dst[node(d, i, j, k)] = prof ? prof[j] : 0.0;
}

// Zero the two wall rows (j = 0 and j = ny-1) of up to six fields: homogeneous Dirichlet
// data for a solve whose interior the solve itself writes.
struct Fields6 {
    double* p[6];
};
__global__ __launch_bounds__(kBlock) void k_zero_walls(Fields6 f, Dims d) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    const int plane = d.nx * d.nz;
    if (e >= 2 * plane) return;
    const int wall = e / plane, r = e - wall * plane;
    const int i = r / d.nz, k = r - (r / d.nz) * d.nz;
    const int j = wall ? d.ny - 1 : 0;
    f.p[blockIdx.y][node(d, i, j, k)] = 0.0;
}

__global__ void k_reset_stats(double* scal, int* istat) {
    if (threadIdx.x == 0) {
        scal[SC_RELRES_MAX] = 0.0;
        scal[SC_RELRES_LAST] = 0.0;
        istat[IS_FLAGS] = 0;
        istat[IS_CYCLES] = 0;
        istat[IS_CONV] = 0;
    }
}


}  // namespace

// ------------------------------------------------------------------------------ launchers
// A launch over n instances multiplies the instance's grid by n (in x, or in y for the
// plane-indexed source kernel).
template <class A>
static unsigned nin(const Over<A>& o) { return (unsigned)(o.tab ? o.n : 1); }


template <class T>
static void advance_t(hipStream_t s, const Dims& d, const Over<AdvArgs>& a) {
    SlabGrid g;
    const int slab = tuning_for(d).adv_slab;
    if (d.nz % 32 == 0) {
        g.gx = (d.ny * d.nz / 2 + kBlock - 1) / kBlock;
        g.ci = slab;
        g.gi = (d.nx + slab - 1) / slab;
        const dim3 gr(g.gx * g.gi * nin(a));
        auto go = [&](auto kt, auto kf) {
            if (a.tab) launch_kernel(kt, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
            else launch_kernel(kf, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
        };
        if (d.nz % 128 == 0) go(k_advance_x2<64, true, T>, k_advance_x2<64, false, T>);
        else if (d.nz % 64 == 0) go(k_advance_x2<32, true, T>, k_advance_x2<32, false, T>);
        else go(k_advance_x2<16, true, T>, k_advance_x2<16, false, T>);
        return;
    }
    g.gx = (d.ny * d.nz + kBlock - 1) / kBlock;
    g.ci = slab;
    g.gi = (d.nx + slab - 1) / slab;
    const dim3 gr(g.gx * g.gi * nin(a));
    if (a.tab) launch_kernel(k_advance_x<true, T>, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
    else launch_kernel(k_advance_x<false, T>, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
}

void launch_advance(hipStream_t s, const Dims& d, Prec pr, const Over<AdvArgs>& a) {
    if (pr == P32)
        advance_t<float>(s, d, a);
    else
        advance_t<double>(s, d, a);
}

// n_z a multiple of 32: two z per lane (k_va_partials2). The block cap (tuned; 1024 by
// default) trades longer x-slabs per lane against a longer final sum.
static SlabGrid va_grid(const Dims& d) {
    return slab_grid(d.nz % 32 == 0 ? d.ny * d.nz / 2 : d.ny * d.nz, d.nx, tuning_for(d).va_maxb);
}

int va_partial_blocks(const Dims& d) {
    const SlabGrid g = va_grid(d);
    return g.gx * g.gi;
}

void launch_va_partials(hipStream_t s, const Dims& d, const Over<VaArgs>& a) {
    const SlabGrid g = va_grid(d);
    const dim3 gr(g.gx * g.gi * nin(a));
    auto go = [&](auto kt, auto kf) {
        if (a.tab) launch_kernel(kt, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
        else launch_kernel(kf, gr, dim3(kBlock), 0, s, d, g, a.one, a.tab);
    };
    if (d.nz % 128 == 0) go(k_va_partials2<64, true>, k_va_partials2<64, false>);
    else if (d.nz % 64 == 0) go(k_va_partials2<32, true>, k_va_partials2<32, false>);
    else if (d.nz % 32 == 0) go(k_va_partials2<16, true>, k_va_partials2<16, false>);
    else go(k_va_partials<true>, k_va_partials<false>);
}

// The chemical potential runs as x-marching LDS tiles (k_mu_tile, any grid) or, for n_z in
// {64, 128, 256}, by register marching (k_mu_reg) with RJ rows per wave and mu_ni planes per
// slab; the autotuner picks (mu_kind: 0 tiles, 1 or 2 register marching with RJ = 1 or 2).
template <bool BEND, class MT>
static void mu_t(hipStream_t s, const Dims& d, const Over<MuArgs>& a) {
    const unsigned ni_ = a.tab ? (unsigned)a.n : 1u;
    const int vnb = va_partial_blocks(d);
    const Tuning tu = tuning_for(d);
    const int zpl = d.nz / 64;
    if (tu.mu_kind > 0 && d.nz % 64 == 0 && (zpl == 1 || zpl == 2 || zpl == 4)) {
        const int RJ = tu.mu_kind;
        const int ni = tu.mu_ni > 0 ? tu.mu_ni : 8;
        const int nb = ((d.ny + 4 * RJ - 1) / (4 * RJ)) * ((d.nx + ni - 1) / ni);
        const dim3 gr(nb * ni_);
        auto go = [&](auto kt, auto kf) {
            if (a.tab) launch_kernel(kt, gr, dim3(kBlock), 0, s, d, vnb, ni, a.one, a.tab);
            else launch_kernel(kf, gr, dim3(kBlock), 0, s, d, vnb, ni, a.one, a.tab);
        };
#define VS_MUREG(Z, R) go(k_mu_reg<BEND, true, MT, Z, R>, k_mu_reg<BEND, false, MT, Z, R>)
        if (zpl == 1) { if (RJ == 1) VS_MUREG(1, 1); else VS_MUREG(1, 2); }
        else if (zpl == 2) { if (RJ == 1) VS_MUREG(2, 1); else VS_MUREG(2, 2); }
        else { if (RJ == 1) VS_MUREG(4, 1); else VS_MUREG(4, 2); }
#undef VS_MUREG
        return;
    }
    const int nb = ((d.ny + kMuTY - 1) / kMuTY) * ((d.nz + kMuTZ - 1) / kMuTZ) *
                   ((d.nx + kMuNI - 1) / kMuNI);
    const dim3 gr(nb * ni_);
    if (a.tab) launch_kernel(k_mu_tile<BEND, true, MT>, gr, dim3(kBlock), 0, s, d, vnb, a.one, a.tab);
    else launch_kernel(k_mu_tile<BEND, false, MT>, gr, dim3(kBlock), 0, s, d, vnb, a.one, a.tab);
}

void launch_mu(hipStream_t s, const Dims& d, int model, Prec pr, const Over<MuArgs>& a) {
    const bool ch = model == VS_CAHN_HILLIARD;
    if (pr == P32) {
        if (ch) mu_t<false, float>(s, d, a);
        else mu_t<true, float>(s, d, a);
    } else {
        if (ch) mu_t<false, double>(s, d, a);
        else mu_t<true, double>(s, d, a);
    }
}

void launch_zero_walls(hipStream_t s, const Dims& d, double* const f[], int nf) {
    if (nf < 1 || nf > 6) return;
    Fields6 ff{};
    for (int q = 0; q < nf; ++q) ff.p[q] = f[q];
    const int n = 2 * d.nx * d.nz;
    launch_kernel(k_zero_walls, dim3((n + kBlock - 1) / kBlock, nf), dim3(kBlock), 0, s, ff, d);
}

void launch_fill_profile(hipStream_t s, const Dims& d, double* dst, const double* prof) {
    launch_kernel(k_fill_profile, plane_grid(d), dim3(kBlock), 0, s, dst, d, prof);
}

template <class T>
static void source_t(hipStream_t s, const Dims& d, const Over<SrcArgs>& a) {
    auto go = [&](dim3 g, auto kt, auto kf) {
        if (a.tab) launch_kernel(kt, g, dim3(kBlock), 0, s, d, a.one, a.tab);
        else launch_kernel(kf, g, dim3(kBlock), 0, s, d, a.one, a.tab);
    };
    if (d.nz % 32 == 0) {
        const dim3 g((unsigned)((d.ny * d.nz / 2 + kBlock - 1) / kBlock), (unsigned)d.nx * nin(a), 1);
        if (d.nz % 128 == 0) go(g, k_source2<64, true, T>, k_source2<64, false, T>);
        else if (d.nz % 64 == 0) go(g, k_source2<32, true, T>, k_source2<32, false, T>);
        else go(g, k_source2<16, true, T>, k_source2<16, false, T>);
        return;
    }
    dim3 g = plane_grid(d);
    g.y *= nin(a);
    go(g, k_source<true, T>, k_source<false, T>);
}

void launch_source(hipStream_t s, const Dims& d, Prec pr, const Over<SrcArgs>& a) {
    if (pr == P32)
        source_t<float>(s, d, a);
    else
        source_t<double>(s, d, a);
}

void launch_reset_stats(hipStream_t s, double* scal, int* istat) {
    launch_kernel(k_reset_stats, dim3(1), dim3(64), 0, s, scal, istat);
}

}  // namespace vs
