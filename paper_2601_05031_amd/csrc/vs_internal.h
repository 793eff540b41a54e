// Internal declarations shared by the host driver and the kernel launchers of libvs.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vs.h"

namespace vs {

// Geometry passed by value to every kernel.
struct Dims {
    int nx, ny, nz;   // nodes; walls at j = 0 and j = ny-1
    int M;            // interior rows, ny - 2
    double h, inv_h2, inv_2h;
};

static inline __host__ __device__ int node(const Dims& d, int i, int j, int k) {
    return (i * d.ny + j) * d.nz + k;
}

// Blocks are handed to the 8 XCDs round-robin by linear block id. This maps a linear id to a
// logical block so that each XCD works through one contiguous range of logical blocks: the
// neighbouring x-planes a stencil reads are then produced and consumed in the same 4 MB L2.
// A bijection on [0, nblocks) for any nblocks.
static inline __device__ int xcd_block(int bid, int nblocks) {
    const int q = nblocks >> 3, rem = nblocks & 7;
    const int x = bid & 7, slot = bid >> 3;
    return x * q + (x < rem ? x : rem) + slot;
}

// Per-thread profiling probe. While `stop` is set, launch_kernel dispatches through
// hipExtLaunchKernelGGL so that the dispatch packet itself records `start` when the first
// kernel begins and `stop` when each kernel ends: the elapsed time covers the kernels alone,
// as a kernel tracer reports it, without the event packets' own dispatch latency.
struct LaunchProbe {
    hipEvent_t start = nullptr, stop = nullptr;
    int launches = 0;
};
LaunchProbe& launch_probe();

template <class... KArgs, class... Args>
inline void launch_kernel(void (*k)(KArgs...), dim3 grid, dim3 block, unsigned shmem,
                          hipStream_t s, Args&&... args) {
    LaunchProbe& p = launch_probe();
    if (p.stop) {
        hipExtLaunchKernelGGL(k, grid, block, shmem, s, p.launches == 0 ? p.start : nullptr,
                              p.stop, 0u, static_cast<KArgs>(args)...);
        ++p.launches;
    } else {
        hipLaunchKernelGGL(k, grid, block, shmem, s, static_cast<KArgs>(args)...);
    }
}

// Slots of the device scalar array (doubles).
enum {
    SC_V = 0, SC_A = 1, SC_V0 = 2, SC_A0 = 3, SC_LAMV = 4, SC_GAMMA = 5,
    SC_RELRES_MAX = 6,        // largest final relative residual since the last reset
    SC_RELRES_LAST = 7,       // relative residual of the last check
    // reverse step: sums gathered by its reduction kernels
    SC_ADJ_SUM_A = 8,         // sum a (the adjoint of lambda_V over dt M)
    SC_ADJ_WALLV = 9,         // sum over wall nodes of a v_wall D_z phi
    SC_ADJ_PSIW = 10,         // sum over wall rows of psi_bar . psi
    SC_ADJ_PSIC = 11,         // wall coupling of the first adjoint solve with the psi walls
    SC_ADJ_OMC = 12,          // wall coupling of the second adjoint solve with the omega walls
    SC_ADJ_KAPPA = 13,        // sum mu_bar d mu / d kappa
    SC_ADJ_GAMMA = 14,        // sum mu_bar d mu / d gamma_A = -sum mu_bar L_h phi
    SC_RELRES_W = 15,         // final relative residual of the step's vorticity solve (checks
                              // of one solve at a time: the stream-vector check logs the step)
    // diagnostics: sums over the nodes with trapezoid weights, and the largest sigma_t
    SC_DG_OMEGA = 16,         // sum_w |omega - omega_0|^2
    SC_DG_PSI = 17,           // sum_w |psi - psi_0|^2
    SC_DG_ENERGY = 18,        // sum_w of the free-energy density (g^2 for bending)
    SC_DG_SMAX = 19,          // max sigma_t
    SC_DG_GAUGE = 20,         // sum over the interior of (D . psi)^2
    SC_DG_VMAX = 21,          // max |v|
    SC_NSCAL = 24
};
// Slots of the device status array (ints).
enum {
    IS_FLAGS = 0,             // bit mask of ST_* below
    IS_CONV = 1,              // 1 once the running Poisson solve met rtol (gates later cycles)
    IS_CYCLES = 2,            // Poisson cycles run since the last reset
    IS_HIST = 3,              // refined mode: time increments of omega and psi the predictor
                              // holds (0, 1, 2), slots 3 and 4 by the parity of the step
    IS_LOGN = 5,              // records written to the per-step log since vs_init
    IS_NSTAT = 16
};
enum { ST_NOCONV = 1, ST_NONFINITE = 2 };
// The per-step log: a ring of kLogCap records of kLogFields doubles (VS_L_* in include/vs.h),
// one per time step (and one for the initial solve), written by the step's final flow check.
constexpr int kLogCap = VS_LOG_CAP;
constexpr int kLogFields = VS_LOG_FIELDS;

// Source of the right-hand side b of a Poisson solve.
enum RhsMode {
    RHS_FIELD = 0,   // b_c = f_c: explicit arrays, or the stored vorticity source of eq. (5b)
    RHS_NEGW = 2     // b_c = -omega_c, eq. (5c)
};

struct RhsArgs {
    int mode;
    const double* f[3];      // RHS_FIELD arrays, or omega for RHS_NEGW
};

// Plan of a length-n transform: radices applied in order (Stockham passes).
struct FftPlan {
    int n;
    int npass;
    int radix[12];
};

constexpr int kMaxPartialBlocks = 4096;

// Reduction grids: block (bx, bi) covers 256 consecutive nodes of a (j, k) plane for the ci
// consecutive x-planes [bi*ci, bi*ci + ci); gx * gi <= maxb <= kMaxPartialBlocks.
struct SlabGrid {
    int gx, ci, gi;
};
static inline SlabGrid slab_grid(int plane, int nx, int maxb) {
    SlabGrid g;
    g.gx = (plane + 255) / 256;
    g.ci = 1;
    while (g.gx * ((nx + g.ci - 1) / g.ci) > maxb && g.ci < nx) ++g.ci;
    g.gi = (nx + g.ci - 1) / g.ci;
    return g;
}
constexpr int kPartialSlots = 17;     // values per block; stored value-major: part[q * kMaxPartialBlocks + b]

// ---------------------------------------------------------------- tuned launch shapes
// Launch shapes that the autotuner (vs_autotune) picks per grid by timing the kernels on a
// state's own data; every launcher reads them at launch time. Defaults until a grid is tuned.
struct Tuning {
    int adv_slab;   // x-planes each lane of the phi update walks (2, 4 or 8)
    int va_maxb;    // block cap of the volume/area partials (sets their x-slab length)
    int res_maxb;   // block cap per component of the flow residual
    int seg_alt;    // 0: the default segment layout of the tridiagonal solves, 1: the other
    int mu_kind;    // chemical potential: 0 LDS tiles; 1, 2 register marching, rows per wave
    int mu_ni;      // x-planes per wave of the register-marching form
    int plane;      // 1: both transform directions of the FP64 flow pass in one plane pass
};
Tuning tuning_for(const Dims& d);
bool seg_has_alt(int M);   // the pair solves of M interior rows have a second layout

// ---------------------------------------------------------------- launches over instances
// Every kernel of a time step takes its per-instance arguments as one struct. A launch covers
// one instance (tab == nullptr: the struct is passed by value) or the n instances of one grid
// class (tab: device table of n structs, one per instance; the instance is read from the
// block index, so all instances run in one launch). Dims are those of the class.
template <class A>
struct Over {
    A one;
    const A* tab;   // device table of n entries, or nullptr
    int n;
};
template <class A>
inline Over<A> over_one(const A& a) {
    return Over<A>{a, nullptr, 1};
}

// ---------------------------------------------------------------- explicit stencils
// Precision of the explicit sweeps: FP64 (mu stored as double, FP64 arithmetic) or the refined
// mode's FP32 (mu stored as float; the phi update in FP32 arithmetic, added to the FP64 phi;
// the chemical potential in FP64 arithmetic, stored as float). The vorticity source is FP64
// in both.
enum Prec { P64 = 0, P32 = 1 };

// phi update (+ the previous step's flow check when ck_part is set)
struct AdvArgs {
    const double* phi;
    const void* mu;
    const double* ps[3];
    double* out;
    double* scal;
    double dt, mob, vz_lo, vz_hi;
    const double* ck_part;   // flow check of the previous step: its residual partials, or null
    int* ck_istat;
    double ck_rtol;
    int ck_nb;               // residual partial blocks of that check
    double* ck_log;          // the per-step log that check appends to
};
void launch_advance(hipStream_t s, const Dims& d, Prec pr, const Over<AdvArgs>& a);
int resid_flow_blocks(const Dims& d);

struct VaArgs {
    const double* phi;
    double* part;
    double eps;
};
void launch_va_partials(hipStream_t s, const Dims& d, const Over<VaArgs>& a);
int va_partial_blocks(const Dims& d);

// V, A and the penalty multipliers lambda_V, gamma_A (SM (32), (37), "Lagrange multipliers")
// from the volume/area block partials, then mu from phi with that gamma_A: every mu block
// reduces the partials itself (same fixed order in every block) and block 0 of the instance
// writes V, A, lambda_V, gamma_A (and V0, A0 when init) to scal.
struct MuArgs {
    const double* phi;
    void* mu;
    const double* part;
    double* scal;
    int* istat;
    double rate_V, k_A, gamma0, mob, C_b, eps, sigma;
    int init;
};
void launch_mu(hipStream_t s, const Dims& d, int model, Prec pr, const Over<MuArgs>& a);

// S = (1/eta) D phi x D mu on the interior rows (main text eq. (5b)); with a != 0 (the
// inertial variant, SM eq. (36)), S - a omega with om the previous vorticity (FP64 only).
struct SrcArgs {
    const double* phi;
    const void* mu;
    void* src[3];
    const double* om[3];
    double inv_eta, a;
};
void launch_source(hipStream_t s, const Dims& d, Prec pr, const Over<SrcArgs>& a);

void launch_fill_profile(hipStream_t s, const Dims& d, double* dst, const double* prof);
// Zero the wall rows j = 0, ny-1 of nf <= 6 fields in one launch.
void launch_zero_walls(hipStream_t s, const Dims& d, double* const f[], int nf);
void launch_reset_stats(hipStream_t s, double* scal, int* istat);

// ---------------------------------------------------------------- spectral Poisson
// Spectral pipeline. The spectral intermediates are stored as double, or as float in the
// refined mode; the two-pass transforms and the segmented tridiagonal solves compute in the
// precision of that storage (the general-length Stockham transforms and the two-lane solves
// of very short or tall columns compute in FP64 either way).

// z transforms (two-pass): spec[c] (ST) -> u[c] (FP64; add: u += result), c < ncomp <= 6.
// The forward transform of the vorticity source uses it with spec = S, u = FP64 modes.
struct ZArgs {
    void* spec[6];
    double* u[6];
    const double2* tw;
    const int* gate;     // skip when *gate != 0 (a converged defect-correction loop), or null
    int add;
    // refined mode (add = 1): the time increment of each field, FP32. With hist set (the first
    // cycle of a step): u <- u + p + e, inc <- p + e, where p is the predictor of the residual
    // pass (see RhsFlowArgs, read from pinc and inc) and e the correction; *hist_out gets
    // min(*hist + 1, 2). With hist null and inc set (a later cycle): u <- u + e, inc <- inc + e.
    float* inc[6];
    const float* pinc[6];
    const int* hist;
    int* hist_out;
    int self;            // refined mode: transform FP32 spec in place (the forward z pass)
};
// x transforms, in place on spec[c], c < ncomp <= 6.
struct HxArgs {
    void* spec[6];
    const double2* tw;
    const int* gate;
};
// Segmented vorticity + stream-vector tridiagonal solves (see k_tridiag_pair_seg).
struct TriArgs {
    const double* tri;
    const double* triw;
    void* spec[3];
    void* spec2[3];
    double olo[3], ohi[3], plo[3], phi[3];
    const int* gate;
};
// Both flow residuals (vorticity, eq. (5b): b = S; stream vector, eq. (5c): b = -omega) in
// one pass, into partial slots 0-5 and 6-11 as two resid_norm launches would write them.
// ashift != 0: the vorticity operator is L_h - ashift (the inertial variant).
struct ResArgs {
    const double* om[3];
    const void* src[3];
    const double* ps[3];
    double* part;
    double ashift;
    const int* gate;
};
struct ChkArgs {
    const double* part;
    double* scal;
    int* istat;
    double rtol;
    const int* gate;
    double* log;         // the per-step log (the step's final check appends a record), or null
};
// Residuals of both flow problems at the current (or predicted) fields, stored in FP32 for the
// refined mode's defect-correction cycle: vorticity into spec, stream vector into spec2.
struct RhsFlowArgs {
    const void* src[3];
    const double* om[3];
    const double* ps[3];
    void* spec[3];
    void* spec2[3];
    const double2* tw;
    const int* gate;
    // predictor of the first cycle of a step (refined mode), or hist null: the residual is
    // taken at u + p with p = 0, i1, 2 i1 - i2 for *hist = 0, 1, 2 held increments (i1 the
    // last step's increment u^n - u^{n-1}, i2 the one before; components 0-2 omega, 3-5 psi)
    const float* i1[6];
    const float* i2[6];
    const int* hist;
};
// The refined mode's first-cycle residuals at the predicted fields (k_rhs_pred), in FP32 at the
// node offsets of spec and spec2, for an in-place z pass (ZArgs::self) to transform.
void launch_rhs_pred(hipStream_t s, const Dims& d, const Over<RhsFlowArgs>& a);

// True when both periodic lengths have two-pass transforms and M a segmented solve: the forms
// the fused flow pass, the refined mode's fused cycle and batched launches use.
// The refined mode's cycle transforms as FP32 plane passes (k_plane32): forward in place on
// z.spec, or inverse from x.spec added to z.u with the increments of ZArgs; gated per instance.
// plane32_fits: n_x = n_z in {32, 48, 64, 96, 128}. Returns false (nothing launched) for other
// grids.
bool plane32_fits(const Dims& d);
bool launch_plane32(hipStream_t s, const Dims& d, bool zfirst, const Over<ZArgs>& z,
                    const Over<HxArgs>& x);
bool fused_flow_ok(const Dims& d);
// Both transform directions in one pass per (interior row, component), the (x, z) plane in
// LDS: zfirst, z then x from z.spec into x.spec (the source's forward transform); otherwise x
// then z from x.spec into z.u (the inverse of the omega and psi modes). FP64 spectral data,
// n_x = n_z in {32, 48, 64, 96, 128}, no gate or accumulation; returns false (nothing
// launched) otherwise.
bool plane_fits(const Dims& d);
bool launch_plane(hipStream_t s, const Dims& d, bool zfirst, int ncomp, const Over<ZArgs>& z,
                  const Over<HxArgs>& x);
void launch_hz(hipStream_t s, const Dims& d, const FftPlan& pz, bool f32, int ncomp,
               const Over<ZArgs>& a);
void launch_hx(hipStream_t s, const Dims& d, const FftPlan& px, bool f32, int ncomp,
               const Over<HxArgs>& a);
// corr: the correction form (homogeneous walls, stream-vector residual modes in spec2).
void launch_tri_pair(hipStream_t s, const Dims& d, bool f32, bool corr, const Over<TriArgs>& a);
// f32src: S stored as float (the refined mode).
void launch_resid_flow_over(hipStream_t s, const Dims& d, bool f32src, const Over<ResArgs>& a);
// last_cycle = 0: a defect-correction cycle that may be followed by another (gated).
void launch_check_flow_over(hipStream_t s, const Dims& d, int last_cycle, const Over<ChkArgs>& a);

// Single-instance forms of the same passes (vs_poisson_solve, refinement cycles, the reverse
// step).
// Forward: b~ (direct) or r = b - L_h u (correct) on interior rows, 2D Hartley in z then x.
void launch_rhs_dht_z(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      const RhsArgs& rhs, const double* const u[3], int ncomp, int correct,
                      void* const spec[3], bool f32, const int* gate);
// ncomp spectral fields spec[0 .. ncomp-1], ncomp <= 6.
void launch_dht_x(hipStream_t s, const Dims& d, const FftPlan& px, const double2* twx,
                  void* const spec[], int ncomp, bool f32, const int* gate);
// Hartley along z of FP64 fields on the interior rows into FP64 spectral storage (the direct
// vorticity transform of the source S, whose wall terms are folded into mode (0, 0)).
void launch_dht_z_fwd(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      const double* const f[3], void* const spec[3], int ncomp);
void launch_tridiag_y(hipStream_t s, const Dims& d, const double* tri, void* const spec[3],
                      int ncomp, bool f32, const int* gate);
// Vorticity modes solved in place in spec (as launch_tridiag_y), then the stream-vector modes
// into spec2 from them (psi wall values constant over each wall plane: psi_lo at j = 0,
// psi_hi at j = ny-1). The vorticity right-hand side's wall terms, om_lo at j = 0 and om_hi at
// j = ny-1 (constant over each wall plane), are added in mode (0, 0) (the transform read S
// alone). triw: the vorticity's pivot table (nullptr: tri; the inertial variant's shifted
// operator L_h - a has its own); the stream-vector problem always uses tri.
void launch_tridiag_pair(hipStream_t s, const Dims& d, const double* tri, const double* triw,
                         void* const spec[3], void* const spec2[3], const double om_lo[3],
                         const double om_hi[3], const double psi_lo[3], const double psi_hi[3],
                         bool f32);
// Hartley along z of spec[c] into u[c] (add: u[c] += result), c < ncomp <= 6.
void launch_dht_z_out(hipStream_t s, const Dims& d, const FftPlan& pz, const double2* twz,
                      void* const spec[], double* const u[], int ncomp, int add, bool f32,
                      const int* gate);
int resid_blocks(const Dims& d);
void launch_resid_flow(hipStream_t s, const Dims& d, const double* const om[3],
                       const double* const src[3], const double* const ps[3], double ashift,
                       double* partials);

// ---------------------------------------------------------------- reverse step (k_adjoint.hip)
// a = dL/dphi^{n+1}; writes phibar (dL/dphi^n, partial), mubar and psibar(3); block partials
// of SC_ADJ_SUM_A, SC_ADJ_WALLV, SC_ADJ_PSIW, which launch_adj_source sums. Also clears the
// status words and residual scalars (as launch_reset_stats) and, if zero_walls is given, the
// wall rows of those (non-NULL) fields.
void launch_adj_advect(hipStream_t s, const Dims& d, const double* a, const double* phi,
                       const double* const psi[3], double dt, double mobility, double vz_lo,
                       double vz_hi, double* phibar, double* mubar, double* const psibar[3],
                       double* part, double* scal, int* istat, double* const zero_walls[6]);
// scal[slot] = -(1/h^2) sum_c sum_{i,k} [u_c(i,1,k) wall_c(i,0,k) + u_c(i,M,k) wall_c(i,ny-1,k)]
void launch_adj_wall_couple(hipStream_t s, const Dims& d, double* const u[3],
                            double* const wall[3], double* part, double* scal, int slot);
// Wall couplings carried by the source's reverse kernel (u may be NULL: no slot-0 term).
struct WallPairs {
    const double* u[3];    // u1 of the first adjoint solve
    const double* uw[3];   // psi (its wall planes)
    const double* sw[3];   // omega (its wall planes), against Sbar
};
// phibar += sum_c D_c^T abar_c, mubar += sum_c D_c^T bbar_c with abar = (1/eta) D mu x Sbar,
// bbar = (1/eta) Sbar x D phi on the interior rows; block partials of the wall coupling of u1
// (if given) with the psi walls and of Sbar with the omega walls (each as
// launch_adj_wall_couple defines it). Block 0 first sums the advection kernel's partials into
// SC_ADJ_SUM_A .. SC_ADJ_PSIW and, with chk_part, checks the two adjoint solves from their
// residual partials (launch_check_flow).
void launch_adj_source(hipStream_t s, const Dims& d, const double* phi, const double* mu,
                       double* const sbar[3], double inv_eta, double* phibar, double* mubar,
                       const double* const u1[3], const double* const psi_walls[3],
                       const double* const om_walls[3], double* part, const double* chk_part,
                       double rtol, double* scal, int* istat);
// Bending: gbar = C_b [(3 phi^2 - 1) mubar - eps^2 L^T mubar]; block partials of the kappa and
// gamma_A terms.
void launch_adj_mu1(hipStream_t s, const Dims& d, const double* phi, const double* mubar,
                    double C_b, double dCb_dkappa, double eps, double* gbar, double* part);
int resid_flow_blocks(const Dims& d);
// Diagnostics (k_diag.hip): sigma_t (device field or NULL) and SC_DG_* sums; vscratch: three
// full fields the velocity is stored in first (scratch: overwritten).
void launch_diagnostics(hipStream_t s, const Dims& d, const double* phi, double* const omega[3],
                        double* const psi[3], const double* prof, double vz_lo, double vz_hi,
                        double eta, int model, double eps, double sigma, double* sigma_t,
                        double* part, double* scal, double* const vscratch[3]);
// omega_x += dprof[ny + j], psi_x += dprof[j] at every node (a wall-speed change).
void launch_shift_profiles(hipStream_t s, const Dims& d, double* omega_x, double* psi_x,
                           const double* dprof);
// phibar += (d mu/d phi)^T mubar + the volume and area multiplier terms. Every block sums the
// gamma_A partials of launch_adj_mu1 (if mu1_ran) itself; block 0 writes SC_ADJ_GAMMA,
// SC_ADJ_KAPPA, SC_ADJ_OMC and, if psi_from_source, SC_ADJ_PSIC of scal_out from the partials.
void launch_adj_mu2(hipStream_t s, const Dims& d, const double* phi, const double* mubar,
                    const double* gbar, const double* scal, int model, double C_b, double eps,
                    double sigma, double dt, double mobility, double rate_V, double k_A,
                    double* phibar, double* part, bool mu1_ran, bool psi_from_source,
                    double* scal_out);
// Residual-norm partials of a solve into slots slot0 .. slot0+5.
void launch_resid_norm(hipStream_t s, const Dims& d, const RhsArgs& rhs,
                       const double* const u[3], int ncomp, double* partials, const int* gate,
                       int slot0 = 0);
// The two single-cycle flow checks of a step in one launch (vorticity partials in slots 0-5,
// stream vector in 6-11).
void launch_check_flow(hipStream_t s, const Dims& d, const double* partials, double rtol,
                       double* scal, int* istat);
// role: 0 a lone solve; 1 the vorticity solve of a step (its final relres kept); 2 the
// stream-vector solve of a step (its final check appends the step's record to log).
void launch_check(hipStream_t s, const double* partials, int nblocks, double rtol, int cycle,
                  int last_cycle, double* scal, int* istat, const int* gate, int slot0 = 0,
                  int role = 0, double* log = nullptr);


}  // namespace vs
