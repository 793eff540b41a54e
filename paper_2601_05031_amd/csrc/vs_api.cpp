// Host driver and C ABI of libvs: argument checks, workspace carve-up, the step sequence of
// the segregated scheme ("Numerical implementation": advance phi, then the vorticity
// Poisson problem, then the stream-vector Poisson problem), status handling, checkpoints
// and per-kernel event timing. All device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "vs_internal.h"

using namespace vs;

namespace {

thread_local std::string g_err;

vs_status fail(vs_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(VS_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

// Kernel classes for the event timer.
enum KClass {
    K_ADVANCE, K_VA_PARTIALS, K_MU, K_SOURCE, K_RHS_Z_OMEGA, K_RHS_Z_PSI,
    K_RHS_Z_FIELD, K_DHT_X, K_TRIDIAG_Y, K_TRIDIAG_PAIR, K_DHT_Z_OUT, K_RESID_OMEGA, K_RESID_PSI,
    K_RESID_FIELD, K_CHECK, K_FILL, K_RESET, K_RESID_FLOW, K_DHT_X_PAIR, K_DHT_Z_OUT_PAIR,
    K_RHS_FLOW, K_ADJ_ADVECT, K_ADJ_WALLS, K_ADJ_SOURCE, K_ADJ_MU1, K_ADJ_MU2, K_ADJ_SUMS, K_DHT_ZX,
    K_DHT_XZ_PAIR, K_RHS_FLOW_Z, K_PLANE32_FWD, K_PLANE32_INV, K_NCLASS
};
const char* kClassNames[K_NCLASS] = {
    "advance", "va_partials", "mu", "source", "rhs_dht_z_omega", "rhs_dht_z_psi",
    "rhs_dht_z_field", "dht_x", "tridiag_y", "tridiag_pair", "dht_z_out", "resid_norm_omega",
    "resid_norm_psi", "resid_norm_field", "check", "fill_profile", "reset_stats",
    "resid_norm_flow", "dht_x_pair", "dht_z_out_pair", "rhs_flow", "adj_advect",
    "adj_wall_couple", "adj_source", "adj_mu1", "adj_mu2", "adj_sums", "dht_zx", "dht_xz_pair",
    "rhs_flow_z", "plane32_fwd", "plane32_inv"};
// Which solve a Poisson call belongs to (selects the timer classes).
enum SolveTag { TAG_OMEGA = 0, TAG_PSI = 1, TAG_FIELD = 2 };

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

bool fft_plan(int n, FftPlan* pl) {
    if (n < 4 || n > 512 || (n & 1)) return false;
    pl->n = n;
    pl->npass = 0;
    int m = n;
    while (m % 4 == 0) { pl->radix[pl->npass++] = 4; m /= 4; }
    while (m % 2 == 0) { pl->radix[pl->npass++] = 2; m /= 2; }
    while (m % 3 == 0) { pl->radix[pl->npass++] = 3; m /= 3; }
    return m == 1 && pl->npass <= 12;
}

struct Layout {
    size_t off_fields;      // 9 fields: phi(2), mu, omega(3), psi(3)
    size_t off_spec;        // 3 spectral scratch fields
    size_t off_src;         // 3 fields: the vorticity source S of the current step
    size_t off_spec2;       // 3 spectral fields: the stream-vector modes
    size_t off_twx, off_twz, off_tri, off_part, off_prof, off_scal, off_istat;
    size_t off_tri2;        // the shifted vorticity pivots of the inertial variant (or 0)
    size_t off_inc;         // refined mode: 2 x 6 FP32 fields, the last two time increments
                            // of omega and psi (or 0)
    size_t off_log;         // the per-step log: kLogCap records of kLogFields doubles
    size_t total;
};

Layout make_layout(const vs_grid& g, bool inertial, bool refined) {
    const size_t N = (size_t)g.nx * g.ny * g.nz;
    const size_t fb = align_up(N * sizeof(double));
    const size_t M = (size_t)g.ny - 2;
    Layout L;
    size_t o = 0;
    L.off_fields = o; o += 9 * fb;
    L.off_spec = o;   o += 3 * fb;
    L.off_src = o;    o += 3 * fb;
    L.off_spec2 = o;  o += 3 * fb;
    L.off_twx = o;    o += align_up((size_t)g.nx * sizeof(double2));
    L.off_twz = o;    o += align_up((size_t)g.nz * sizeof(double2));
    L.off_tri = o;    o += align_up((size_t)(g.nx / 2 + 1) * (g.nz / 2 + 1) * (M + 1) * sizeof(double));
    L.off_part = o;   o += align_up((size_t)kMaxPartialBlocks * kPartialSlots * sizeof(double));
    L.off_prof = o;   o += align_up(4 * (size_t)g.ny * sizeof(double));   // tables + a change
    L.off_scal = o;   o += align_up(SC_NSCAL * sizeof(double));
    L.off_istat = o;  o += align_up(IS_NSTAT * sizeof(int));
    L.off_log = o;    o += align_up((size_t)kLogCap * kLogFields * sizeof(double));
    L.off_tri2 = 0;
    if (inertial) {
        L.off_tri2 = o;
        o += align_up((size_t)(g.nx / 2 + 1) * (g.nz / 2 + 1) * (M + 1) * sizeof(double));
    }
    L.off_inc = 0;
    if (refined) {
        L.off_inc = o;
        o += 12 * align_up(N * sizeof(float));
    }
    L.total = o;
    return L;
}

// Pivots c'_j = 1/(beta - c'_{j-1}) of tridiag(1, beta, 1) per Hartley mode class (p, q) up
// to the conjugate pair, beta = 2 cos(2 pi p/nx) + 2 cos(2 pi q/nz) - 6 - shift_h2, and beta
// itself as row M. shift_h2 = a h^2 for the operator L_h - a (0: L_h).
std::vector<double> pivot_table(const vs_grid& g, double shift_h2) {
    const int M = g.ny - 2, hx = g.nx / 2 + 1, hz = g.nz / 2 + 1;
    std::vector<double> tri((size_t)hx * hz * (M + 1));
    for (int pc = 0; pc < hx; ++pc)
        for (int qc = 0; qc < hz; ++qc) {
            const long double PI = 3.14159265358979323846264338327950288L;
            const double beta = (double)(2.0L * cosl(2.0L * PI * pc / g.nx) +
                                         2.0L * cosl(2.0L * PI * qc / g.nz) - 6.0L -
                                         (long double)shift_h2);
            const size_t cls = (size_t)pc * hz + qc, ncls = (size_t)hx * hz;
            double prev = 0.0;
            for (int j = 0; j < M; ++j) {
                prev = 1.0 / (beta - prev);
                tri[(size_t)j * ncls + cls] = prev;
            }
            tri[(size_t)M * ncls + cls] = beta;
        }
    return tri;
}

// Twiddles exp(-2 pi i m/n), m < n, computed in long double.
std::vector<double2> twiddle_table(int n) {
    std::vector<double2> t(n);
    for (int m = 0; m < n; ++m) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * m / n;
        t[m] = make_double2((double)cosl(a), (double)(-sinl(a)));
    }
    return t;
}

vs_status check_grid(const vs_grid* g) {
    if (!g) return fail(VS_E_ARG, "grid is NULL");
    if (g->ny < 3) return fail(VS_E_ARG, "ny = %d: need at least 3 rows (two walls)", g->ny);
    if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(VS_E_ARG, "h must be > 0");
    FftPlan p;
    if (!fft_plan(g->nx, &p))
        return fail(VS_E_UNSUPPORTED, "nx = %d: need even 4 <= nx <= 512 of the form 2^a 3^b", g->nx);
    if (!fft_plan(g->nz, &p))
        return fail(VS_E_UNSUPPORTED, "nz = %d: need even 4 <= nz <= 512 of the form 2^a 3^b", g->nz);
    if ((long long)g->nx * g->ny * g->nz > (1ll << 30))
        return fail(VS_E_ARG, "grid too large");
    // reductions keep one partial per block of 256 plane nodes: at most kMaxPartialBlocks
    if ((long long)g->ny * g->nz > 256ll * kMaxPartialBlocks)
        return fail(VS_E_ARG, "ny * nz = %lld: at most %d nodes per x-plane",
                    (long long)g->ny * g->nz, 256 * kMaxPartialBlocks);
    return VS_OK;
}

vs_status check_params(const vs_params* p) {
    if (!p) return fail(VS_E_ARG, "params is NULL");
    if (p->model != VS_BENDING && p->model != VS_CAHN_HILLIARD)
        return fail(VS_E_ARG, "model must be VS_BENDING or VS_CAHN_HILLIARD");
    if (p->precision != VS_FP64 && p->precision != VS_FP32_REFINED)
        return fail(VS_E_ARG, "precision must be VS_FP64 or VS_FP32_REFINED");
    if (!(p->eta > 0.0)) return fail(VS_E_ARG, "eta must be > 0");
    if (!(p->mobility > 0.0)) return fail(VS_E_ARG, "mobility must be > 0");
    if (!(p->eps > 0.0)) return fail(VS_E_ARG, "eps must be > 0");
    if (!(p->kappa >= 0.0)) return fail(VS_E_ARG, "kappa must be >= 0");
    if (p->model == VS_CAHN_HILLIARD && !(p->sigma > 0.0))
        return fail(VS_E_ARG, "sigma must be > 0 for the Cahn-Hilliard model");
    if (!(p->poisson_rtol > 0.0)) return fail(VS_E_ARG, "poisson_rtol must be > 0");
    if (p->poisson_max_cycles < 1 || p->poisson_max_cycles > 16)
        return fail(VS_E_ARG, "poisson_max_cycles must be in [1, 16]");
    const double fin[] = {p->gamma0, p->rate_V, p->k_A, p->bend_scale};
    for (double v : fin)
        if (!std::isfinite(v)) return fail(VS_E_ARG, "non-finite parameter");
    if (p->rate_V < 0.0 || p->k_A < 0.0) return fail(VS_E_ARG, "penalties must be >= 0");
    if (!(p->rho >= 0.0) || !std::isfinite(p->rho)) return fail(VS_E_ARG, "rho must be >= 0");
    if (p->rho > 0.0 && (p->precision != VS_FP64 || p->poisson_max_cycles != 1))
        return fail(VS_E_UNSUPPORTED,
                    "the inertial variant (rho > 0) runs in VS_FP64 with poisson_max_cycles = 1");
    return VS_OK;
}

vs_status check_walls(const vs_walls* w) {
    if (!w) return fail(VS_E_ARG, "walls is NULL");
    if (w->kind != VS_POISEUILLE && w->kind != VS_COUETTE)
        return fail(VS_E_ARG, "walls.kind must be VS_POISEUILLE or VS_COUETTE");
    if (!std::isfinite(w->u0) || !std::isfinite(w->u1)) return fail(VS_E_ARG, "wall speed not finite");
    return VS_OK;
}

}  // namespace

struct vs_state {
    vs_grid g{};
    vs_walls w{};
    vs_params p{};
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout L{};
    Dims d{};
    FftPlan px{}, pz{};
    double* phi[2] = {nullptr, nullptr};
    int cur = 0;
    double* mu = nullptr;
    // the flow check of the last enqueued step is left to the next step's advance kernel
    // (set only between two steps of one vs_step call or one captured batch; never across
    // API calls)
    bool check_pending = false;
    double* om[3] = {};
    double* ps[3] = {};
    void* spec[3] = {};
    double* src[3] = {};
    void* spec2[3] = {};
    bool f32 = false;         // refined mode: spectral intermediates stored as float
    // refined mode: time increments of omega (0-2) and psi (3-5) in two FP32 buffers whose
    // roles alternate with the step parity (the predictor of the first correction cycle)
    float* inc[2][6] = {};
    double* log = nullptr;    // the per-step log (device ring, kLogCap records)
    long long log_shown = 0;  // records of it already printed (VS_LOG)
    double psi_wall_lo[3] = {0, 0, 0}, psi_wall_hi[3] = {0, 0, 0};
    double om_wall_lo[3] = {0, 0, 0}, om_wall_hi[3] = {0, 0, 0};
    double2* twx = nullptr;
    double2* twz = nullptr;
    double* tri = nullptr;
    double* tri2 = nullptr;    // inertial variant: pivots of L_h - a for the vorticity
    double tri2_dt = 0.0;      // the dt those pivots were made for (0: not yet)
    double* part = nullptr;
    double* prof = nullptr;   // [0, ny): psi_x profile, [ny, 2 ny): omega_x profile
    double* scal = nullptr;
    int* istat = nullptr;
    double vz_lo = 0.0, vz_hi = 0.0;
    std::vector<double> prof_host;   // the device wall tables prof[0, 2 ny), host copy
    long long walls_gen = 0;  // bumped on every wall change (a batch re-captures its graph)
    double gamma_host = 0.0;  // gamma_A as of the last synchronisation
    long long step = 0;
    double last_relres = 0.0;
    int last_cycles = 0;
    // event timer
    bool prof_on = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
    std::vector<hipEvent_t> ev_pool;
    // pinned host copy of the scalars and status words (one transfer per synchronisation)
    char* host_stat = nullptr;

    ~vs_state() {
        if (host_stat) (void)hipHostFree(host_stat);
    }

    double C_b() const { return p.bend_scale * 3.0 * std::sqrt(2.0) * p.kappa / (8.0 * p.eps * p.eps * p.eps); }
};

namespace {

hipEvent_t take_event(vs_state* S) {
    if (!S->ev_pool.empty()) {
        hipEvent_t e = S->ev_pool.back();
        S->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

LaunchProbe& vs::launch_probe() {
    static thread_local LaunchProbe probe;
    return probe;
}

// Tuned launch shapes per grid (nx, ny, nz), shared by every state of that grid.
namespace {
struct TuneKey {
    int nx, ny, nz;
    bool operator==(const TuneKey& o) const { return nx == o.nx && ny == o.ny && nz == o.nz; }
};
// One entry per grid; fp64 records that the FP64-only coordinate (the transform form) was
// tuned too: an FP32-refined state's tuning leaves it at its default.
struct TuneEntry {
    TuneKey k;
    Tuning t;
    bool fp64;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
constexpr Tuning kDefaultTuning{4, 1024, 1024, 0, 0, 8, 0};

void set_tuning(const Dims& d, const Tuning& t, bool fp64 = false) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const TuneKey k{d.nx, d.ny, d.nz};
    for (auto& e : g_tune)
        if (e.k == k) {
            e.t = t;
            e.fp64 = e.fp64 || fp64;
            return;
        }
    g_tune.push_back({k, t, fp64});
}
// Tuned for states of this precision (an FP64 state needs the FP64 coordinate tuned as well).
bool tuned(const Dims& d, bool f32) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& e : g_tune)
        if (e.k == TuneKey{d.nx, d.ny, d.nz}) return f32 || e.fp64;
    return false;
}
}  // namespace

Tuning vs::tuning_for(const Dims& d) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& e : g_tune)
        if (e.k == TuneKey{d.nx, d.ny, d.nz}) return e.t;
    return kDefaultTuning;
}

namespace {

// Run `launch` with its kernels timed by an event pair when the timer is on.
template <class F>
void timed(vs_state* S, int cls, F&& launch) {
    if (!S->prof_on) {
        launch();
        return;
    }
    hipEvent_t a = take_event(S), b = take_event(S);
    if (!a || !b) {
        launch();
        return;
    }
    LaunchProbe& p = vs::launch_probe();
    p.start = a;
    p.stop = b;
    p.launches = 0;
    launch();
    const int n = p.launches;
    p = LaunchProbe{};
    if (n > 0) S->ev_used.push_back({cls, {a, b}});
}

void release_events(vs_state* S) {
    for (auto& u : S->ev_used) {
        S->ev_pool.push_back(u.second.first);
        S->ev_pool.push_back(u.second.second);
    }
    S->ev_used.clear();
}

// Residual norms of the current u and the convergence check of cycle `cyc`.
void enqueue_verify(vs_state* S, const RhsArgs& rhs, double* const u[3], int ncomp, double rtol,
                    int cyc, int last, int tag, const int* gate) {
    const Dims& d = S->d;
    const double* const cu[3] = {u[0], u[1], u[2]};
    const int nb = resid_blocks(d);
    const int k_res = tag == TAG_OMEGA ? K_RESID_OMEGA : tag == TAG_PSI ? K_RESID_PSI : K_RESID_FIELD;
    timed(S, k_res, [&] { launch_resid_norm(S->stream, d, rhs, cu, ncomp, S->part, gate); });
    // the two solves of a time step (FP64, more than one cycle per solve): the stream-vector
    // check logs the step
    const int role = tag == TAG_OMEGA ? 1 : tag == TAG_PSI ? 2 : 0;
    timed(S, K_CHECK, [&] {
        launch_check(S->stream, S->part, nb, rtol, cyc, last, S->scal, S->istat, gate, 0, role,
                     S->log);
    });
}

// One transform cycle: cycle 0 (correct = 0) solves directly from b and the wall rows;
// a correction cycle solves for the correction of the residual and adds it to u.
void enqueue_cycle(vs_state* S, const RhsArgs& rhs, double* const u[3], int ncomp, int correct,
                   int tag, const int* gate) {
    const Dims& d = S->d;
    const double* const cu[3] = {u[0], u[1], u[2]};
    const int k_rhs = tag == TAG_OMEGA ? K_RHS_Z_OMEGA : tag == TAG_PSI ? K_RHS_Z_PSI : K_RHS_Z_FIELD;
    timed(S, k_rhs, [&] {
        launch_rhs_dht_z(S->stream, d, S->pz, S->twz, rhs, cu, ncomp, correct, S->spec, S->f32, gate);
    });
    timed(S, K_DHT_X, [&] { launch_dht_x(S->stream, d, S->px, S->twx, S->spec, ncomp, S->f32, gate); });
    timed(S, K_TRIDIAG_Y, [&] { launch_tridiag_y(S->stream, d, S->tri, S->spec, ncomp, S->f32, gate); });
    timed(S, K_DHT_X, [&] { launch_dht_x(S->stream, d, S->px, S->twx, S->spec, ncomp, S->f32, gate); });
    timed(S, K_DHT_Z_OUT, [&] {
        launch_dht_z_out(S->stream, d, S->pz, S->twz, S->spec, u, ncomp, correct, S->f32, gate);
    });
}

// Verified solve: cycle 0, then up to max_cycles-1 correction cycles gated on the device flag
// (a cycle runs only while the previous check missed rtol); each cycle ends with a check.
// warm = 1: cycle 0 too solves for the correction of the residual of the incoming u (the
// refined mode's defect correction from the previous time step's field).
void enqueue_solve(vs_state* S, const RhsArgs& rhs, double* const u[3], int ncomp, double rtol,
                   int max_cycles, int tag, int warm = 0) {
    for (int cyc = 0; cyc < max_cycles; ++cyc) {
        const int* gate = cyc == 0 ? nullptr : S->istat + IS_CONV;
        enqueue_cycle(S, rhs, u, ncomp, (cyc > 0 || warm) ? 1 : 0, tag, gate);
        enqueue_verify(S, rhs, u, ncomp, rtol, cyc, cyc == max_cycles - 1, tag, gate);
    }
}

// ------------------------------------------------------------------- one time step
// Everything one time step launches, as per-kernel argument structs: by value for one
// instance, or device tables for every instance of a batch class (Over in vs_internal.h).
// Index [g] of the refined mode's correction-cycle passes: 0 = the first cycle (always runs),
// 1 = later cycles (gated on the instance's convergence flag).
struct StepArgs {
    Over<AdvArgs> adv;
    Over<VaArgs> va;
    Over<MuArgs> mu;
    Over<SrcArgs> src;
    Over<ZArgs> zfwd;
    Over<HxArgs> hx3, hx6;
    Over<TriArgs> tri;
    Over<ZArgs> zout6;
    Over<ResArgs> res;
    Over<ChkArgs> chk;
    Over<RhsFlowArgs> rf[2];
    Over<ZArgs> zs[2];
    Over<HxArgs> hxc[2];
    Over<TriArgs> trc[2];
    Over<ZArgs> zadd[2];
    Over<ResArgs> resc[2];
    Over<ChkArgs> chkc[2];
};
#define VS_STEP_FIELDS(X)                                                                   \
    X(adv) X(va) X(mu) X(src) X(zfwd) X(hx3) X(hx6) X(tri) X(zout6) X(res) X(chk) X(rf[0])  \
    X(rf[1]) X(zs[0]) X(zs[1]) X(hxc[0]) X(hxc[1]) X(trc[0]) X(trc[1]) X(zadd[0]) X(zadd[1]) \
    X(resc[0]) X(resc[1]) X(chkc[0]) X(chkc[1])

// The fused refined-mode cycle and the fused FP64 pass need two-pass transform lengths and a
// segmented tridiagonal layout; the refined mode is offered only there.
bool refined_fused(const vs_state* S) { return S->f32 && fused_flow_ok(S->d); }

// Arguments of one step of S that reads phi[par] and writes phi[1 - par] (par = -1: the
// initial state, phi[0] read in place: no advance). with_ck: the advance takes the previous
// step's flow check. dt = 0: the initial solve.
StepArgs step_args(vs_state* S, int par, double dt, bool with_ck) {
    StepArgs A{};
    const double* phi_in = S->phi[par < 0 ? 0 : par];
    double* phi_new = par < 0 ? S->phi[0] : S->phi[1 - par];
    const double a = (S->p.rho > 0.0 && dt > 0.0) ? S->p.rho / (S->p.eta * dt) : 0.0;
    AdvArgs ad{};
    ad.phi = phi_in;
    ad.mu = S->mu;
    for (int c = 0; c < 3; ++c) ad.ps[c] = S->ps[c];
    ad.out = phi_new;
    ad.scal = S->scal;
    ad.dt = dt;
    ad.mob = S->p.mobility;
    ad.vz_lo = S->vz_lo;
    ad.vz_hi = S->vz_hi;
    if (with_ck) {
        ad.ck_part = S->part;
        ad.ck_istat = S->istat;
        ad.ck_rtol = S->p.poisson_rtol;
        ad.ck_nb = resid_flow_blocks(S->d);
        ad.ck_log = S->log;
    }
    A.adv = over_one(ad);
    A.va = over_one(VaArgs{phi_new, S->part, S->p.eps});
    MuArgs m{};
    m.phi = phi_new;
    m.mu = S->mu;
    m.part = S->part;
    m.scal = S->scal;
    m.istat = S->istat;
    m.rate_V = S->p.rate_V;
    m.k_A = S->p.k_A;
    m.gamma0 = S->p.gamma0;
    m.mob = S->p.mobility;
    m.C_b = S->C_b();
    m.eps = S->p.eps;
    m.sigma = S->p.sigma;
    m.init = par < 0 ? 1 : 0;
    A.mu = over_one(m);
    SrcArgs sr{};
    sr.phi = phi_new;
    sr.mu = S->mu;
    for (int c = 0; c < 3; ++c) {
        sr.src[c] = S->src[c];
        sr.om[c] = S->om[c];
    }
    sr.inv_eta = 1.0 / S->p.eta;
    sr.a = a;
    A.src = over_one(sr);
    ZArgs zf{};
    for (int c = 0; c < 3; ++c) {
        zf.spec[c] = S->src[c];
        zf.u[c] = (double*)S->spec[c];
    }
    zf.tw = S->twz;
    A.zfwd = over_one(zf);
    HxArgs h3{}, h6{};
    for (int c = 0; c < 3; ++c) {
        h3.spec[c] = S->spec[c];
        h6.spec[c] = S->spec[c];
        h6.spec[3 + c] = S->spec2[c];
    }
    h3.tw = h6.tw = S->twx;
    A.hx3 = over_one(h3);
    A.hx6 = over_one(h6);
    TriArgs t{};
    t.tri = S->tri;
    t.triw = a != 0.0 ? S->tri2 : S->tri;
    for (int c = 0; c < 3; ++c) {
        t.spec[c] = S->spec[c];
        t.spec2[c] = S->spec2[c];
        t.olo[c] = S->om_wall_lo[c];
        t.ohi[c] = S->om_wall_hi[c];
        t.plo[c] = S->psi_wall_lo[c];
        t.phi[c] = S->psi_wall_hi[c];
    }
    A.tri = over_one(t);
    ZArgs z6{};
    for (int c = 0; c < 3; ++c) {
        z6.spec[c] = S->spec[c];
        z6.spec[3 + c] = S->spec2[c];
        z6.u[c] = S->om[c];
        z6.u[3 + c] = S->ps[c];
    }
    z6.tw = S->twz;
    A.zout6 = over_one(z6);
    ResArgs r{};
    for (int c = 0; c < 3; ++c) {
        r.om[c] = S->om[c];
        r.src[c] = S->src[c];
        r.ps[c] = S->ps[c];
    }
    r.part = S->part;
    r.ashift = a;
    A.res = over_one(r);
    ChkArgs ck{};
    ck.part = S->part;
    ck.scal = S->scal;
    ck.istat = S->istat;
    ck.rtol = S->p.poisson_rtol;
    ck.log = S->log;
    A.chk = over_one(ck);
    // the refined mode's predictor (steps only, not the initial solve): increments i1 = inc[par]
    // (the last step's) and i2 = inc[1 - par] (the one before), which the first cycle's update
    // overwrites with this step's increment; the held count alternates between two slots
    const bool pred = S->f32 && par >= 0 && S->inc[0][0];
    const int q1 = par < 0 ? 0 : par, q2 = 1 - q1;
    for (int g = 0; g < 2; ++g) {
        const int* gate = g ? S->istat + IS_CONV : nullptr;
        RhsFlowArgs rf{};
        for (int c = 0; c < 3; ++c) {
            rf.src[c] = S->src[c];
            rf.om[c] = S->om[c];
            rf.ps[c] = S->ps[c];
            rf.spec[c] = S->spec[c];
            rf.spec2[c] = S->spec2[c];
        }
        rf.tw = S->twz;
        rf.gate = gate;
        if (pred && g == 0) {
            for (int q = 0; q < 6; ++q) {
                rf.i1[q] = S->inc[q1][q];
                rf.i2[q] = S->inc[q2][q];
            }
            rf.hist = S->istat + IS_HIST + q1;
        }
        A.rf[g] = over_one(rf);
        ZArgs zsf{};
        for (int c = 0; c < 3; ++c) {
            zsf.spec[c] = S->spec[c];
            zsf.spec[3 + c] = S->spec2[c];
        }
        zsf.tw = S->twz;
        zsf.gate = gate;
        zsf.self = 1;
        A.zs[g] = over_one(zsf);
        HxArgs hc = h6;
        hc.gate = gate;
        A.hxc[g] = over_one(hc);
        TriArgs tc = t;
        tc.triw = S->tri;
        tc.gate = gate;
        A.trc[g] = over_one(tc);
        ZArgs za = z6;
        za.add = 1;
        za.gate = gate;
        if (pred) {
            for (int q = 0; q < 6; ++q) za.inc[q] = S->inc[q2][q];
            if (g == 0) {
                for (int q = 0; q < 6; ++q) za.pinc[q] = S->inc[q1][q];
                za.hist = S->istat + IS_HIST + q1;
                za.hist_out = S->istat + IS_HIST + q2;
            }
        }
        A.zadd[g] = over_one(za);
        ResArgs rc = r;
        rc.gate = gate;
        A.resc[g] = over_one(rc);
        ChkArgs cc = ck;
        cc.gate = gate;
        A.chkc[g] = over_one(cc);
    }
    return A;
}

// What a step enqueue needs besides the arguments: the class's grid, plans and settings, the
// stream, and the state whose event timer (if on) times the launches.
struct StepCfg {
    hipStream_t st;
    Dims d;
    FftPlan px, pz;
    bool f32;
    int model, mc;
    double rtol;
    bool inertial;
    vs_state* timer;   // null: no timing
};

StepCfg step_cfg(vs_state* S) {
    return StepCfg{S->stream, S->d, S->px, S->pz, S->f32, S->p.model, S->p.poisson_max_cycles,
                   S->p.poisson_rtol, S->p.rho > 0.0, S->prof_on ? S : nullptr};
}

template <class F>
void timed_cfg(const StepCfg& c, int cls, F&& launch) {
    if (c.timer)
        timed(c.timer, cls, launch);
    else
        launch();
}

// V, A, the multipliers and mu from the new phi (SM (32), (37), "Lagrange multipliers", (35)).
void enqueue_va_mu_args(const StepCfg& c, const StepArgs& A) {
    timed_cfg(c, K_VA_PARTIALS, [&] { launch_va_partials(c.st, c.d, A.va); });
    timed_cfg(c, K_MU, [&] { launch_mu(c.st, c.d, c.model, c.f32 ? P32 : P64, A.mu); });
}

// The flow part of a step (main text eq. (5b), then (5c)) through the fused passes.
// FP64: one direct spectral pass (the vorticity modes after the tridiagonal solve are, up to
// -h^2, the transformed right-hand side of the stream-vector problem, so psi needs no forward
// transform), then both fields verified against their spatial residuals. Refined mode:
// defect-correction cycles from the incoming fields, each a residual pass in FP64 whose result
// is transformed and solved in FP32 and added to the FP64 fields, then verified; cycles after
// the first are gated on the device flag of the previous check.
// max_cycles > 1 in FP64: the verification is left to enqueue_fp64_corrections.
// Returns true when the final check was left to the next step's advance (defer).
bool enqueue_flow_args(const StepCfg& c, const StepArgs& A, bool defer, int max_cycles) {
    timed_cfg(c, K_SOURCE, [&] { launch_source(c.st, c.d, c.f32 ? P32 : P64, A.src); });
    if (c.f32) {
        // the transforms of a cycle as two FP32 plane passes where the plane fits in LDS
        const bool plane = plane32_fits(c.d);
        for (int cyc = 0; cyc < max_cycles; ++cyc) {
            const int g = cyc ? 1 : 0;
            timed_cfg(c, K_RHS_FLOW, [&] { launch_rhs_pred(c.st, c.d, A.rf[g]); });
            if (plane) {
                timed_cfg(c, K_PLANE32_FWD, [&] { launch_plane32(c.st, c.d, true, A.zs[g], A.hxc[g]); });
            } else {
                timed_cfg(c, K_RHS_FLOW_Z, [&] { launch_hz(c.st, c.d, c.pz, true, 6, A.zs[g]); });
                timed_cfg(c, K_DHT_X_PAIR, [&] { launch_hx(c.st, c.d, c.px, true, 6, A.hxc[g]); });
            }
            timed_cfg(c, K_TRIDIAG_PAIR, [&] { launch_tri_pair(c.st, c.d, true, true, A.trc[g]); });
            if (plane) {
                timed_cfg(c, K_PLANE32_INV, [&] { launch_plane32(c.st, c.d, false, A.zadd[g], A.hxc[g]); });
            } else {
                timed_cfg(c, K_DHT_X_PAIR, [&] { launch_hx(c.st, c.d, c.px, true, 6, A.hxc[g]); });
                timed_cfg(c, K_DHT_Z_OUT_PAIR, [&] { launch_hz(c.st, c.d, c.pz, true, 6, A.zadd[g]); });
            }
            timed_cfg(c, K_RESID_FLOW, [&] { launch_resid_flow_over(c.st, c.d, false, A.resc[g]); });
            if (max_cycles == 1 && defer) return true;
            timed_cfg(c, K_CHECK, [&] {
                launch_check_flow_over(c.st, c.d, cyc == max_cycles - 1 ? 1 : 0, A.chkc[g]);
            });
        }
        return false;
    }
    // The direct transform reads S alone: the omega wall terms go into mode (0, 0) of the
    // tridiagonal solve.
    // With the plane form (tuned, n_x = n_z up to 128) each direction is one pass.
    const bool plane = tuning_for(c.d).plane && plane_fits(c.d);
    if (plane) {
        timed_cfg(c, K_DHT_ZX, [&] { launch_plane(c.st, c.d, true, 3, A.zfwd, A.hx3); });
    } else {
        timed_cfg(c, K_RHS_Z_OMEGA, [&] { launch_hz(c.st, c.d, c.pz, false, 3, A.zfwd); });
        timed_cfg(c, K_DHT_X, [&] { launch_hx(c.st, c.d, c.px, false, 3, A.hx3); });
    }
    timed_cfg(c, K_TRIDIAG_PAIR, [&] { launch_tri_pair(c.st, c.d, false, false, A.tri); });
    // both fields back to physical space, six components per launch
    if (plane) {
        timed_cfg(c, K_DHT_XZ_PAIR, [&] { launch_plane(c.st, c.d, false, 6, A.zout6, A.hx6); });
    } else {
        timed_cfg(c, K_DHT_X_PAIR, [&] { launch_hx(c.st, c.d, c.px, false, 6, A.hx6); });
        timed_cfg(c, K_DHT_Z_OUT_PAIR, [&] { launch_hz(c.st, c.d, c.pz, false, 6, A.zout6); });
    }
    if (max_cycles > 1) return false;
    // both residuals in one pass, then both checks in one launch, or, when another step
    // follows in the same call, in the first block of its advance kernel
    timed_cfg(c, K_RESID_FLOW, [&] { launch_resid_flow_over(c.st, c.d, false, A.res); });
    if (defer) return true;
    timed_cfg(c, K_CHECK, [&] { launch_check_flow_over(c.st, c.d, 1, A.chk); });
    return false;
}

// FP64 correction cycles after the direct pass (poisson_max_cycles > 1), per solve, through
// the general verified path (normally never needed: the direct pass is exact).
void enqueue_fp64_corrections(vs_state* S) {
    const double rtol = S->p.poisson_rtol;
    const int mc = S->p.poisson_max_cycles;
    RhsArgs rv{};
    rv.mode = RHS_FIELD;
    for (int c = 0; c < 3; ++c) rv.f[c] = (const double*)S->src[c];
    RhsArgs rp{};
    rp.mode = RHS_NEGW;
    for (int c = 0; c < 3; ++c) rp.f[c] = S->om[c];
    enqueue_verify(S, rv, S->om, 3, rtol, 0, 0, TAG_OMEGA, nullptr);
    for (int cyc = 1; cyc < mc; ++cyc) {
        const int* gate = S->istat + IS_CONV;
        enqueue_cycle(S, rv, S->om, 3, 1, TAG_OMEGA, gate);
        enqueue_verify(S, rv, S->om, 3, rtol, cyc, cyc == mc - 1, TAG_OMEGA, gate);
    }
    enqueue_verify(S, rp, S->ps, 3, rtol, 0, 0, TAG_PSI, nullptr);
    for (int cyc = 1; cyc < mc; ++cyc) {
        const int* gate = S->istat + IS_CONV;
        enqueue_cycle(S, rp, S->ps, 3, 1, TAG_PSI, gate);
        enqueue_verify(S, rp, S->ps, 3, rtol, cyc, cyc == mc - 1, TAG_PSI, gate);
    }
}

// The initial state: V0, A0, mu^0, then omega^0 and psi^0 from the no-body fields. The refined
// mode starts from those fields with no step behind it, so it takes enough correction cycles
// for a full solve (its FP32 cycles each gain about six digits).
void enqueue_init(vs_state* S) {
    const StepCfg c = step_cfg(S);
    const StepArgs A = step_args(S, -1, 0.0, false);
    enqueue_va_mu_args(c, A);
    if (S->f32) {
        enqueue_flow_args(c, A, false, S->p.poisson_max_cycles > 4 ? S->p.poisson_max_cycles : 4);
        return;
    }
    enqueue_flow_args(c, A, false, S->p.poisson_max_cycles);
    if (S->p.poisson_max_cycles > 1) enqueue_fp64_corrections(S);
}

// One time step. more_follow: another step of the same call comes after this one, so its
// advance kernel can take this step's flow check.
void enqueue_step(vs_state* S, double dt, bool more_follow) {
    const StepCfg c = step_cfg(S);
    const StepArgs A = step_args(S, S->cur, dt, S->check_pending);
    S->check_pending = false;
    timed_cfg(c, K_ADVANCE, [&] { launch_advance(c.st, c.d, c.f32 ? P32 : P64, A.adv); });
    S->cur = 1 - S->cur;
    enqueue_va_mu_args(c, A);
    const int mc = S->p.poisson_max_cycles;
    if (S->f32) {
        S->check_pending = enqueue_flow_args(c, A, more_follow, mc);
        return;
    }
    S->check_pending = enqueue_flow_args(c, A, more_follow && mc == 1, mc);
    if (mc > 1) enqueue_fp64_corrections(S);
}

// The inertial variant's vorticity pivots depend on dt (a = rho/(eta dt)): made on the host
// when dt changes, before anything is enqueued. The device-wide wait covers a batch graph
// still replaying on its own streams with the old table.
vs_status ensure_inertial_table(vs_state* S, double dt) {
    if (!(S->p.rho > 0.0) || dt == S->tri2_dt) return VS_OK;
    const double a = S->p.rho / (S->p.eta * dt);
    const std::vector<double> t = pivot_table(S->g, a * S->g.h * S->g.h);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(S->tri2, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
    S->tri2_dt = dt;
    return VS_OK;
}

// No-body channel tables on the node rows (the wall data of "Boundary conditions", reading
// R11): prof[j] = psi_x(y_j), prof[ny + j] = omega_x(y_j).
std::vector<double> wall_tables(const vs_grid& g, const vs_walls& w) {
    const double H = (g.ny - 1) * g.h;
    std::vector<double> prof(2 * (size_t)g.ny);
    for (int j = 0; j < g.ny; ++j) {
        const double y = j * g.h;
        double psx, omx;
        if (w.kind == VS_POISEUILLE) {
            const double U = w.u0;
            psx = -(4.0 * U / (H * H)) * (H * y * y / 2.0 - y * y * y / 3.0);
            omx = (4.0 * U / (H * H)) * (H - 2.0 * y);
        } else {
            const double u0 = w.u0, u1 = w.u1;
            psx = -(u0 * y + (u1 - u0) * y * y / (2.0 * H));
            omx = (u1 - u0) / H;
        }
        prof[j] = psx;
        prof[g.ny + j] = omx;
    }
    return prof;
}

// Host-side wall state: the wall speeds the advection uses on the wall nodes and the psi wall
// values folded into mode (0, 0) of the stream-vector solve.
void set_wall_state(vs_state* S, const vs_walls& w, const std::vector<double>& prof) {
    S->w = w;
    S->prof_host = prof;
    S->psi_wall_lo[0] = prof[0];
    S->psi_wall_hi[0] = prof[S->g.ny - 1];
    S->om_wall_lo[0] = prof[S->g.ny];
    S->om_wall_hi[0] = prof[2 * S->g.ny - 1];
    if (w.kind == VS_POISEUILLE) {
        S->vz_lo = 0.0;
        S->vz_hi = 0.0;
    } else {
        S->vz_lo = w.u0;
        S->vz_hi = w.u1;
    }
    ++S->walls_gen;
}

// Reads the device status and scalars after a synchronisation; maps flags to a status.
// Waits for S's stream and copies the scalars and status words (adjacent in the workspace) to
// the host in one transfer through the pinned buffer.
vs_status read_status(vs_state* S, double* sc, int* ist) {
    const size_t ioff = (size_t)((char*)S->istat - (char*)S->scal);
    const size_t span = ioff + IS_NSTAT * sizeof(int);
    HIP_TRY(hipMemcpyAsync(S->host_stat, S->scal, span, hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    if (sc) std::memcpy(sc, S->host_stat, SC_NSCAL * sizeof(double));
    if (ist) std::memcpy(ist, S->host_stat + ioff, IS_NSTAT * sizeof(int));
    return VS_OK;
}

vs_status collect(vs_state* S, const char* what) {
    int ist[IS_NSTAT];
    double sc[SC_NSCAL];
    const vs_status rs = read_status(S, sc, ist);
    if (rs != VS_OK) return rs;
    S->gamma_host = sc[SC_GAMMA];
    S->last_relres = sc[SC_RELRES_MAX];
    S->last_cycles = ist[IS_CYCLES];
    if (ist[IS_FLAGS] & ST_NONFINITE)
        return fail(VS_E_NONFINITE, "%s: non-finite value in a residual norm or in V, A", what);
    if (ist[IS_FLAGS] & ST_NOCONV)
        return fail(VS_E_NOCONV, "%s: a Poisson solve missed rtol %.3g (relative residual %.3g)", what,
                    S->p.poisson_rtol, sc[SC_RELRES_MAX]);
    return VS_OK;
}

// The per-step log's records, oldest first (at most kLogCap), and the count written since
// vs_init. Synchronises.
vs_status read_log(vs_state* S, std::vector<double>& recs, long long& total) {
    int ist[IS_NSTAT];
    const vs_status rs = read_status(S, nullptr, ist);
    if (rs != VS_OK) return rs;
    total = ist[IS_LOGN];
    const long long kept = total < kLogCap ? total : kLogCap;
    std::vector<double> ring((size_t)kLogCap * kLogFields);
    HIP_TRY(hipMemcpy(ring.data(), S->log, ring.size() * sizeof(double), hipMemcpyDeviceToHost));
    recs.resize((size_t)kept * kLogFields);
    for (long long q = 0; q < kept; ++q) {
        const long long idx = total - kept + q;
        std::memcpy(&recs[(size_t)q * kLogFields], &ring[(size_t)(idx % kLogCap) * kLogFields],
                    kLogFields * sizeof(double));
    }
    return VS_OK;
}

// VS_LOG: the records of the steps just run, one line each, on stderr.
void print_log(vs_state* S) {
    static const bool on = std::getenv("VS_LOG") != nullptr;
    if (!on) return;
    std::vector<double> recs;
    long long total = 0;
    if (read_log(S, recs, total) != VS_OK) return;
    const long long kept = (long long)(recs.size() / kLogFields);
    for (long long q = 0; q < kept; ++q) {
        const double* r = &recs[(size_t)q * kLogFields];
        if ((long long)r[VS_L_INDEX] < S->log_shown) continue;
        std::fprintf(stderr, "vs step %lld: cycles %d relres %.3e V %.10g A %.10g lambda_V %.6g gamma_A %.6g%s\n",
                     (long long)r[VS_L_INDEX], (int)r[VS_L_CYCLES], r[VS_L_RELRES], r[VS_L_V], r[VS_L_A],
                     r[VS_L_LAMBDA_V], r[VS_L_GAMMA_A], r[VS_L_CONV] != 0.0 ? "" : " (not converged)");
    }
    S->log_shown = total;
}

double stability_rate(const vs_state* S) {
    const double h2 = S->g.h * S->g.h;
    const double lmax = 12.0 / h2;
    if (S->p.model == VS_CAHN_HILLIARD) return S->p.mobility * lmax * (2.0 + S->p.sigma * lmax);
    const double e2 = S->p.eps * S->p.eps;
    const double a = 2.0 + e2 * lmax;
    return S->p.mobility * lmax * (S->C_b() * a * a + std::fabs(S->gamma_host) * lmax);
}

}  // namespace

extern "C" {

const char* vs_last_error(void) { return g_err.c_str(); }

vs_status vs_workspace_bytes(const vs_grid* grid, const vs_params* params, size_t* bytes) {
    vs_status st = check_grid(grid);
    if (st != VS_OK) return st;
    if ((st = check_params(params)) != VS_OK) return st;
    if (!bytes) return fail(VS_E_ARG, "bytes is NULL");
    *bytes = make_layout(*grid, params->rho > 0.0, params->precision == VS_FP32_REFINED).total;
    return VS_OK;
}

vs_status vs_init(const vs_grid* grid, const vs_walls* walls, const vs_params* params,
                  const double* phi0, void* workspace, size_t bytes, void* stream,
                  vs_state** out) {
    vs_status st;
    if (!out) return fail(VS_E_ARG, "out is NULL");
    *out = nullptr;
    if ((st = check_grid(grid)) != VS_OK) return st;
    if ((st = check_walls(walls)) != VS_OK) return st;
    if ((st = check_params(params)) != VS_OK) return st;
    if (!phi0) return fail(VS_E_ARG, "phi0 is NULL");
    const Layout L = make_layout(*grid, params->rho > 0.0, params->precision == VS_FP32_REFINED);
    {
        Dims dd{grid->nx, grid->ny, grid->nz, grid->ny - 2, grid->h, 0.0, 0.0};
        if (params->precision == VS_FP32_REFINED && !fused_flow_ok(dd))
            return fail(VS_E_UNSUPPORTED,
                        "VS_FP32_REFINED needs nx, nz in {32, 48, 64, 96, 128, 192, 256} and "
                        "4 <= ny - 2 <= 256 (the fused transform and tridiagonal forms)");
    }
    if (!workspace) return fail(VS_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)workspace) & 255) return fail(VS_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < L.total) return fail(VS_E_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, L.total);

    vs_state* S = new vs_state();
    S->g = *grid;
    S->w = *walls;
    S->p = *params;
    S->stream = (hipStream_t)stream;
    S->ws = (char*)workspace;
    S->ws_bytes = bytes;
    S->L = L;
    S->d.nx = grid->nx;
    S->d.ny = grid->ny;
    S->d.nz = grid->nz;
    S->d.M = grid->ny - 2;
    S->d.h = grid->h;
    S->d.inv_h2 = 1.0 / (grid->h * grid->h);
    S->d.inv_2h = 0.5 / grid->h;
    fft_plan(grid->nx, &S->px);
    fft_plan(grid->nz, &S->pz);
    const size_t N = (size_t)grid->nx * grid->ny * grid->nz;
    const size_t fb = align_up(N * sizeof(double));
    double* f = (double*)(S->ws + L.off_fields);
    auto field = [&](int idx) { return (double*)((char*)f + idx * fb); };
    S->phi[0] = field(0);
    S->phi[1] = field(1);
    S->mu = field(2);
    for (int c = 0; c < 3; ++c) {
        S->om[c] = field(3 + c);
        S->ps[c] = field(6 + c);
        S->spec[c] = (void*)(S->ws + L.off_spec + c * fb);
        S->src[c] = (double*)(S->ws + L.off_src + c * fb);
        S->spec2[c] = (void*)(S->ws + L.off_spec2 + c * fb);
    }
    S->f32 = params->precision == VS_FP32_REFINED;
    S->twx = (double2*)(S->ws + L.off_twx);
    S->twz = (double2*)(S->ws + L.off_twz);
    S->tri = (double*)(S->ws + L.off_tri);
    S->tri2 = L.off_tri2 ? (double*)(S->ws + L.off_tri2) : nullptr;
    if (L.off_inc)
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 6; ++q)
                S->inc[b][q] = (float*)(S->ws + L.off_inc + (6 * b + q) * align_up(N * sizeof(float)));
    S->part = (double*)(S->ws + L.off_part);
    S->prof = (double*)(S->ws + L.off_prof);
    S->scal = (double*)(S->ws + L.off_scal);
    S->istat = (int*)(S->ws + L.off_istat);
    S->log = (double*)(S->ws + L.off_log);

    // Host tables: twiddles exp(-2 pi i m/n), Thomas pivots per Hartley mode class, and the
    // no-body channel profiles of psi_x and omega_x (main text "Boundary conditions").
    std::vector<double2> twx = twiddle_table(grid->nx), twz = twiddle_table(grid->nz);
    const std::vector<double> tri = pivot_table(*grid, 0.0);
    std::vector<double> prof = wall_tables(*grid, *walls);
    set_wall_state(S, *walls, prof);
    S->gamma_host = params->gamma0;

    auto bail = [&](vs_status s) {
        delete S;
        return s;
    };
#define INIT_TRY(expr)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return bail(fail(VS_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)));    \
    } while (0)
    INIT_TRY(hipHostMalloc((void**)&S->host_stat,
                           (size_t)((char*)S->istat - (char*)S->scal) + IS_NSTAT * sizeof(int),
                           hipHostMallocDefault));
    INIT_TRY(hipMemcpyAsync(S->twx, twx.data(), twx.size() * sizeof(double2), hipMemcpyHostToDevice, S->stream));
    INIT_TRY(hipMemcpyAsync(S->twz, twz.data(), twz.size() * sizeof(double2), hipMemcpyHostToDevice, S->stream));
    INIT_TRY(hipMemcpyAsync(S->tri, tri.data(), tri.size() * sizeof(double), hipMemcpyHostToDevice, S->stream));
    INIT_TRY(hipMemcpyAsync(S->prof, prof.data(), prof.size() * sizeof(double), hipMemcpyHostToDevice, S->stream));
    INIT_TRY(hipMemcpyAsync(S->phi[0], phi0, N * sizeof(double), hipMemcpyDeviceToDevice, S->stream));
    INIT_TRY(hipMemsetAsync(S->scal, 0, SC_NSCAL * sizeof(double), S->stream));
    INIT_TRY(hipMemsetAsync(S->istat, 0, IS_NSTAT * sizeof(int), S->stream));
    INIT_TRY(hipMemsetAsync(S->log, 0, (size_t)kLogCap * kLogFields * sizeof(double), S->stream));
    // the increments' wall rows are read (as zero) by the predictor and never written
    if (L.off_inc) INIT_TRY(hipMemsetAsync(S->ws + L.off_inc, 0, L.total - L.off_inc, S->stream));
    launch_fill_profile(S->stream, S->d, S->ps[0], S->prof);
    launch_fill_profile(S->stream, S->d, S->om[0], S->prof + grid->ny);
    for (int c = 1; c < 3; ++c) {
        launch_fill_profile(S->stream, S->d, S->ps[c], nullptr);
        launch_fill_profile(S->stream, S->d, S->om[c], nullptr);
    }
    INIT_TRY(hipGetLastError());
    enqueue_init(S);
    INIT_TRY(hipGetLastError());
    st = collect(S, "vs_init");
    if (st != VS_OK) return bail(st);
#undef INIT_TRY
    *out = S;
    return VS_OK;
}

vs_status vs_poisson_solve(vs_state* S, const double* f, double* u, double rtol, int32_t max_cycles,
                           int32_t* cycles_out, double* relres_out) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (!f || !u) return fail(VS_E_ARG, "f and u must be device pointers");
    if (!(rtol > 0.0)) return fail(VS_E_ARG, "rtol must be > 0");
    if (max_cycles < 1 || max_cycles > 16) return fail(VS_E_ARG, "max_cycles must be in [1, 16]");
    timed(S, K_RESET, [&] { launch_reset_stats(S->stream, S->scal, S->istat); });
    RhsArgs r{};
    r.mode = RHS_FIELD;
    r.f[0] = f;
    double* const uu[3] = {u, nullptr, nullptr};
    enqueue_solve(S, r, uu, 1, rtol, max_cycles, TAG_FIELD);
    HIP_TRY(hipGetLastError());
    int ist[IS_NSTAT];
    double sc[SC_NSCAL];
    const vs_status rs = read_status(S, sc, ist);
    if (rs != VS_OK) return rs;
    if (cycles_out) *cycles_out = ist[IS_CYCLES];
    if (relres_out) *relres_out = sc[SC_RELRES_LAST];
    if (ist[IS_FLAGS] & ST_NONFINITE) return fail(VS_E_NONFINITE, "vs_poisson_solve: non-finite residual");
    if (ist[IS_FLAGS] & ST_NOCONV)
        return fail(VS_E_NOCONV, "vs_poisson_solve: relative residual %.3g above rtol %.3g after %d cycles",
                    sc[SC_RELRES_LAST], rtol, ist[IS_CYCLES]);
    return VS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free solve
// vs_poisson_solve_noalloc keeps its scratch (one FP64 spectral field, the twiddle and
// pivot tables, the residual partials and the status words) in this file-scope device array
// instead of a caller workspace. Each device holds its own copy for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress returns on that device.
namespace {

constexpr size_t kNoAllocBytes = size_t(48) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {};
// grid whose twiddle and pivot tables the device's scratch holds (nx = 0: none yet)
vs_grid g_noalloc_tables[kNoAllocMaxDevices] = {};

struct NoAllocLayout {
    size_t off_spec, off_twx, off_twz, off_tri, off_part, off_scal, off_istat, total;
};

NoAllocLayout noalloc_layout(const vs_grid& g) {
    const size_t N = (size_t)g.nx * g.ny * g.nz;
    const size_t M = (size_t)g.ny - 2;
    NoAllocLayout L;
    size_t o = 0;
    L.off_spec = o;  o += align_up(N * sizeof(double));
    L.off_twx = o;   o += align_up((size_t)g.nx * sizeof(double2));
    L.off_twz = o;   o += align_up((size_t)g.nz * sizeof(double2));
    L.off_tri = o;   o += align_up((size_t)(g.nx / 2 + 1) * (g.nz / 2 + 1) * (M + 1) * sizeof(double));
    L.off_part = o;  o += align_up((size_t)kMaxPartialBlocks * kPartialSlots * sizeof(double));
    L.off_scal = o;  o += align_up(SC_NSCAL * sizeof(double));
    L.off_istat = o; o += align_up(IS_NSTAT * sizeof(int));
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

size_t vs_noalloc_scratch_bytes(void) { return kNoAllocBytes; }

vs_status vs_poisson_solve_noalloc(const vs_grid* grid, const double* f, double* u, double rtol,
                                   int32_t max_cycles, void* stream, int32_t* cycles_out,
                                   double* relres_out) {
    vs_status st = check_grid(grid);
    if (st != VS_OK) return st;
    if (!f || !u) return fail(VS_E_ARG, "f and u must be device pointers");
    if (!(rtol > 0.0)) return fail(VS_E_ARG, "rtol must be > 0");
    if (max_cycles < 1 || max_cycles > 16) return fail(VS_E_ARG, "max_cycles must be in [1, 16]");
    const NoAllocLayout L = noalloc_layout(*grid);
    if (L.total > kNoAllocBytes)
        return fail(VS_E_WORKSPACE,
                    "vs_poisson_solve_noalloc: the %d x %d x %d grid needs %zu bytes of scratch; "
                    "the static scratch holds %zu",
                    grid->nx, grid->ny, grid->nz, L.total, kNoAllocBytes);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return fail(VS_E_UNSUPPORTED, "vs_poisson_solve_noalloc: device %d out of range", dev);
    hipStream_t hs = (hipStream_t)stream;
    char* base = nullptr;
    bool tables = false;
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (!g_noalloc_ptr[dev]) {
            void* p = nullptr;
            HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            if (!p) return fail(VS_E_HIP, "hipGetSymbolAddress returned no address for the scratch");
            g_noalloc_ptr[dev] = p;
        }
        base = (char*)g_noalloc_ptr[dev];
        const vs_grid& t = g_noalloc_tables[dev];
        tables = t.nx == grid->nx && t.ny == grid->ny && t.nz == grid->nz && t.h == grid->h;
        g_noalloc_tables[dev] = *grid;
    }
    vs_state S;
    S.g = *grid;
    S.stream = hs;
    S.d.nx = grid->nx;
    S.d.ny = grid->ny;
    S.d.nz = grid->nz;
    S.d.M = grid->ny - 2;
    S.d.h = grid->h;
    S.d.inv_h2 = 1.0 / (grid->h * grid->h);
    S.d.inv_2h = 0.5 / grid->h;
    fft_plan(grid->nx, &S.px);
    fft_plan(grid->nz, &S.pz);
    S.spec[0] = base + L.off_spec;
    S.twx = (double2*)(base + L.off_twx);
    S.twz = (double2*)(base + L.off_twz);
    S.tri = (double*)(base + L.off_tri);
    S.part = (double*)(base + L.off_part);
    S.scal = (double*)(base + L.off_scal);
    S.istat = (int*)(base + L.off_istat);
    // host tables outlive their copies: the stream is synchronised before they go
    std::vector<double2> twx, twz;
    std::vector<double> tri;
    if (!tables) {
        twx = twiddle_table(grid->nx);
        twz = twiddle_table(grid->nz);
        tri = pivot_table(*grid, 0.0);
        hipError_t e = hipMemcpyAsync(S.twx, twx.data(), twx.size() * sizeof(double2),
                                      hipMemcpyHostToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S.twz, twz.data(), twz.size() * sizeof(double2),
                               hipMemcpyHostToDevice, hs);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S.tri, tri.data(), tri.size() * sizeof(double),
                               hipMemcpyHostToDevice, hs);
        if (e != hipSuccess) {
            std::lock_guard<std::mutex> lk(g_noalloc_mu);
            g_noalloc_tables[dev] = vs_grid{};
            return fail(VS_E_HIP, "vs_poisson_solve_noalloc: table upload failed: %s",
                        hipGetErrorString(e));
        }
    }
    // status words and residual scalars start from zero (a kernel, not a memset)
    launch_reset_stats(hs, S.scal, S.istat);
    RhsArgs r{};
    r.mode = RHS_FIELD;
    r.f[0] = f;
    double* const uu[3] = {u, nullptr, nullptr};
    enqueue_solve(&S, r, uu, 1, rtol, max_cycles, TAG_FIELD);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(hs));
    int ist[IS_NSTAT];
    double sc[SC_NSCAL];
    HIP_TRY(hipMemcpy(ist, S.istat, sizeof ist, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(sc, S.scal, sizeof sc, hipMemcpyDeviceToHost));
    if (cycles_out) *cycles_out = ist[IS_CYCLES];
    if (relres_out) *relres_out = sc[SC_RELRES_LAST];
    if (ist[IS_FLAGS] & ST_NONFINITE)
        return fail(VS_E_NONFINITE, "vs_poisson_solve_noalloc: non-finite residual");
    if (ist[IS_FLAGS] & ST_NOCONV)
        return fail(VS_E_NOCONV,
                    "vs_poisson_solve_noalloc: relative residual %.3g above rtol %.3g after %d cycles",
                    sc[SC_RELRES_LAST], rtol, ist[IS_CYCLES]);
    return VS_OK;
}

vs_status vs_step(vs_state* S, double dt, int32_t nsteps) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(VS_E_ARG, "dt must be > 0");
    if (nsteps < 1) return fail(VS_E_ARG, "nsteps must be >= 1");
    if (!(S->p.flags & VS_ALLOW_UNSTABLE)) {
        const double rate = stability_rate(S);
        if (dt * rate > 2.0)
            return fail(VS_E_UNSTABLE, "dt = %.4g exceeds the forward-Euler bound %.4g", dt, 2.0 / rate);
    }
    vs_status st = ensure_inertial_table(S, dt);
    if (st != VS_OK) return st;
    timed(S, K_RESET, [&] { launch_reset_stats(S->stream, S->scal, S->istat); });
    for (int s = 0; s < nsteps; ++s) enqueue_step(S, dt, s + 1 < nsteps);
    HIP_TRY(hipGetLastError());
    S->step += nsteps;
    const vs_status cs = collect(S, "vs_step");
    print_log(S);
    return cs;
}

vs_status vs_grad_step(vs_state* S, double dt, const double* adj_next, double* adj_prev,
                       double dparams[2]) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (!adj_next || !adj_prev || !dparams) return fail(VS_E_ARG, "adj_next, adj_prev and dparams are required");
    if (adj_next == adj_prev) return fail(VS_E_ARG, "adj_next and adj_prev must not alias");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(VS_E_ARG, "dt must be > 0");
    if (S->f32) return fail(VS_E_UNSUPPORTED, "vs_grad_step: the reverse step runs in the FP64 mode only");
    if (S->p.rho > 0.0)
        return fail(VS_E_UNSUPPORTED, "vs_grad_step: no reverse step for the inertial variant");
    const Dims& d = S->d;
    hipStream_t st = S->stream;
    const double rtol = S->p.poisson_rtol;
    const int mc = S->p.poisson_max_cycles;
    const double* phi = S->phi[S->cur];
    double* mubar = S->phi[1 - S->cur];     // free between steps
    double* const q[3] = {S->src[0], S->src[1], S->src[2]};
    double* const u1[3] = {(double*)S->spec2[0], (double*)S->spec2[1], (double*)S->spec2[2]};
    const double* const cps[3] = {S->ps[0], S->ps[1], S->ps[2]};
    // the one-pass solve below writes the two spectral sets inside only: their wall rows are
    // zeroed by the advection kernel, which also clears the status words
    double* const w6[6] = {(double*)S->spec[0], (double*)S->spec[1], (double*)S->spec[2],
                           (double*)S->spec2[0], (double*)S->spec2[1], (double*)S->spec2[2]};
    // advection, L_h mu and lambda_V terms; q = psi_bar
    timed(S, K_ADJ_ADVECT, [&] {
        launch_adj_advect(st, d, adj_next, phi, cps, dt, S->p.mobility, S->vz_lo, S->vz_hi,
                          adj_prev, mubar, q, S->part, S->scal, S->istat, mc == 1 ? w6 : nullptr);
    });
    // psi_int = P(-omega_int; psi walls): first adjoint solve, homogeneous walls;
    // omega_int = P(S; omega walls): second adjoint solve, of -u1, giving S_bar
    double* sb[3] = {q[0], q[1], q[2]};          // S_bar
    const double* u1w[3] = {nullptr, nullptr, nullptr};   // u1 for the source kernel's wall term
    if (mc == 1) {
        // one verified pass, as the forward flow solve: q transformed once, u1's modes solved
        // and S_bar's from them in the pair kernel (zero walls), both inverse-transformed in
        // place in the two spectral sets (u1 in spec, S_bar in spec2), then both residuals
        // against q and -u1 in one pass and one check
        double* const us[3] = {(double*)S->spec[0], (double*)S->spec[1], (double*)S->spec[2]};
        double* const ss[3] = {(double*)S->spec2[0], (double*)S->spec2[1], (double*)S->spec2[2]};
        const double* const qc[3] = {q[0], q[1], q[2]};
        // the transforms as in the forward flow pass: one plane pass per direction when tuned so
        const bool plane = tuning_for(d).plane && plane_fits(d);
        ZArgs zf{};
        HxArgs xf{};
        ZArgs zi{};
        HxArgs xi{};
        for (int c = 0; c < 3; ++c) {
            zf.spec[c] = (void*)q[c];
            zf.u[c] = (double*)S->spec[c];
            xf.spec[c] = S->spec[c];
        }
        for (int c = 0; c < 6; ++c) {
            void* sp = c < 3 ? S->spec[c] : S->spec2[c - 3];
            zi.spec[c] = sp;
            zi.u[c] = (double*)sp;
            xi.spec[c] = sp;
        }
        zf.tw = zi.tw = S->twz;
        xf.tw = xi.tw = S->twx;
        if (plane) {
            timed(S, K_DHT_ZX, [&] { launch_plane(st, d, true, 3, over_one(zf), over_one(xf)); });
        } else {
            timed(S, K_RHS_Z_FIELD, [&] { launch_dht_z_fwd(st, d, S->pz, S->twz, qc, S->spec, 3); });
            timed(S, K_DHT_X, [&] { launch_dht_x(st, d, S->px, S->twx, S->spec, 3, false, nullptr); });
        }
        const double zero[3] = {0.0, 0.0, 0.0};
        timed(S, K_TRIDIAG_PAIR, [&] {
            launch_tridiag_pair(st, d, S->tri, nullptr, S->spec, S->spec2, zero, zero, zero, zero, false);
        });
        void* const sp6[6] = {S->spec[0], S->spec[1], S->spec[2], S->spec2[0], S->spec2[1], S->spec2[2]};
        if (plane) {
            timed(S, K_DHT_XZ_PAIR, [&] { launch_plane(st, d, false, 6, over_one(zi), over_one(xi)); });
        } else {
            timed(S, K_DHT_X_PAIR, [&] { launch_dht_x(st, d, S->px, S->twx, sp6, 6, false, nullptr); });
            timed(S, K_DHT_Z_OUT_PAIR, [&] { launch_dht_z_out(st, d, S->pz, S->twz, sp6, w6, 6, 0, false, nullptr); });
        }
        const double* const cu[3] = {us[0], us[1], us[2]};
        const double* const cs[3] = {ss[0], ss[1], ss[2]};
        // both residuals in one pass; their check is taken by block 0 of the source kernel
        timed(S, K_RESID_FLOW, [&] { launch_resid_flow(st, d, cu, qc, cs, 0.0, S->part); });
        for (int c = 0; c < 3; ++c) {
            sb[c] = ss[c];
            u1w[c] = us[c];
        }
    } else {
        // the solve writes the interior; only the wall rows need zeros
        launch_zero_walls(st, d, u1, 3);
        RhsArgs r1{};
        r1.mode = RHS_FIELD;
        for (int c = 0; c < 3; ++c) r1.f[c] = q[c];
        enqueue_solve(S, r1, u1, 3, rtol, mc, TAG_FIELD);
        timed(S, K_ADJ_WALLS, [&] { launch_adj_wall_couple(st, d, u1, S->ps, S->part, S->scal, SC_ADJ_PSIC); });
        launch_zero_walls(st, d, q, 3);
        RhsArgs r2{};
        r2.mode = RHS_NEGW;
        for (int c = 0; c < 3; ++c) r2.f[c] = u1[c];
        enqueue_solve(S, r2, q, 3, rtol, mc, TAG_FIELD);
    }
    // S = (1/eta) D phi x D mu; the wall couplings of the adjoint solves as block partials
    const double* const cpsw[3] = {S->ps[0], S->ps[1], S->ps[2]};
    const double* const comw[3] = {S->om[0], S->om[1], S->om[2]};
    timed(S, K_ADJ_SOURCE, [&] {
        launch_adj_source(st, d, phi, S->mu, sb, 1.0 / S->p.eta, adj_prev, mubar,
                          u1w[0] ? u1w : nullptr, cpsw, comw, S->part,
                          mc == 1 ? S->part : nullptr, rtol, S->scal, S->istat);
    });
    // mu(phi)
    double* gbar = (double*)S->spec[0];
    const double dCb = S->p.bend_scale * 3.0 * std::sqrt(2.0) / (8.0 * S->p.eps * S->p.eps * S->p.eps);
    if (S->p.model == VS_BENDING)
        timed(S, K_ADJ_MU1, [&] {
            launch_adj_mu1(st, d, phi, mubar, S->C_b(), dCb, S->p.eps, gbar, S->part);
        });
    // the sums of the wall couplings (the psi one unless the general path summed it already)
    // and, for bending, of the kappa and gamma_A terms ride in the mu2 kernel
    timed(S, K_ADJ_MU2, [&] {
        launch_adj_mu2(st, d, phi, mubar, gbar, S->scal, S->p.model, S->C_b(), S->p.eps, S->p.sigma,
                       dt, S->p.mobility, S->p.rate_V, S->p.k_A, adj_prev, S->part,
                       S->p.model == VS_BENDING, u1w[0] != nullptr, S->scal);
    });
    HIP_TRY(hipGetLastError());
    int ist[IS_NSTAT];
    double sc[SC_NSCAL];
    const vs_status rs = read_status(S, sc, ist);
    if (rs != VS_OK) return rs;
    if (ist[IS_FLAGS] & ST_NONFINITE) return fail(VS_E_NONFINITE, "vs_grad_step: non-finite residual");
    if (ist[IS_FLAGS] & ST_NOCONV)
        return fail(VS_E_NOCONV, "vs_grad_step: an adjoint Poisson solve missed rtol %.3g", rtol);
    const double kbar = S->p.model == VS_BENDING ? sc[SC_ADJ_KAPPA] : 0.0;
    const double sbar = -dt * sc[SC_ADJ_WALLV] + sc[SC_ADJ_PSIW] + sc[SC_ADJ_PSIC] + sc[SC_ADJ_OMC];
    if (!std::isfinite(kbar) || !std::isfinite(sbar))
        return fail(VS_E_NONFINITE, "vs_grad_step: non-finite parameter gradient");
    dparams[0] += kbar;
    dparams[1] += sbar;
    return VS_OK;
}

vs_status vs_set_walls(vs_state* S, const vs_walls* walls) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    vs_status st = check_walls(walls);
    if (st != VS_OK) return st;
    if (walls->kind != S->w.kind) return fail(VS_E_ARG, "vs_set_walls: the wall kind cannot change");
    if (S->p.rho > 0.0)
        return fail(VS_E_UNSUPPORTED, "vs_set_walls: not for the inertial variant");
    const std::vector<double> prof = wall_tables(S->g, *walls);
    const int ny = S->g.ny;
    std::vector<double> dprof(2 * (size_t)ny);
    for (size_t q = 0; q < dprof.size(); ++q) dprof[q] = prof[q] - S->prof_host[q];
    HIP_TRY(hipMemcpyAsync(S->prof + 2 * ny, dprof.data(), dprof.size() * sizeof(double),
                           hipMemcpyHostToDevice, S->stream));
    launch_shift_profiles(S->stream, S->d, S->om[0], S->ps[0], S->prof + 2 * ny);
    HIP_TRY(hipMemcpyAsync(S->prof, prof.data(), prof.size() * sizeof(double), hipMemcpyHostToDevice,
                           S->stream));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(S->stream));   // the host tables above are copied from
    set_wall_state(S, *walls, prof);
    return VS_OK;
}

vs_status vs_diagnostics(vs_state* S, double* sigma_t, double out[6]) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (!out) return fail(VS_E_ARG, "out is NULL");
    const Dims& d = S->d;
    // the source fields are free between calls: the velocity goes there first
    launch_diagnostics(S->stream, d, S->phi[S->cur], S->om, S->ps, S->prof, S->vz_lo, S->vz_hi,
                       S->p.eta, S->p.model, S->p.eps, S->p.sigma, sigma_t, S->part, S->scal,
                       S->src);
    HIP_TRY(hipGetLastError());
    double sc[SC_NSCAL];
    const vs_status rs = read_status(S, sc, nullptr);
    if (rs != VS_OK) return rs;
    const double h3 = d.h * d.h * d.h;
    const double cF = 3.0 * std::sqrt(2.0) * S->p.kappa / (8.0 * S->p.eps * S->p.eps * S->p.eps);
    out[0] = h3 * sc[SC_DG_OMEGA];
    out[1] = h3 * sc[SC_DG_PSI];
    out[2] = (S->p.model == VS_BENDING ? cF : 1.0) * h3 * sc[SC_DG_ENERGY];
    out[3] = sc[SC_DG_SMAX];
    out[4] = h3 * sc[SC_DG_GAUGE];
    out[5] = sc[SC_DG_VMAX];
    return VS_OK;
}

vs_status vs_field_offset(const vs_state* S, int32_t field, size_t* byte_offset) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (!byte_offset) return fail(VS_E_ARG, "byte_offset is NULL");
    const double* p = nullptr;
    switch (field) {
        case VS_PHI: p = S->phi[S->cur]; break;
        case VS_MU: p = S->mu; break;
        case VS_OMEGA_X: case VS_OMEGA_Y: case VS_OMEGA_Z: p = S->om[field - VS_OMEGA_X]; break;
        case VS_PSI_X: case VS_PSI_Y: case VS_PSI_Z: p = S->ps[field - VS_PSI_X]; break;
        default: return fail(VS_E_ARG, "unknown field id %d", field);
    }
    *byte_offset = (size_t)((const char*)p - S->ws);
    return VS_OK;
}

vs_status vs_log_read(vs_state* S, double* out, int32_t cap, int32_t* n) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (!out || !n) return fail(VS_E_ARG, "out and n are required");
    if (cap < 1) return fail(VS_E_ARG, "cap must be >= 1");
    std::vector<double> recs;
    long long total = 0;
    const vs_status rs = read_log(S, recs, total);
    if (rs != VS_OK) return rs;
    const long long kept = (long long)(recs.size() / kLogFields);
    const long long m = kept < cap ? kept : cap;
    if (m > 0)
        std::memcpy(out, &recs[(size_t)(kept - m) * kLogFields], (size_t)m * kLogFields * sizeof(double));
    *n = (int32_t)m;
    return VS_OK;
}

vs_status vs_get_scalars(vs_state* S, double out[VS_NSCALARS]) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (!out) return fail(VS_E_ARG, "out is NULL");
    double sc[SC_NSCAL];
    const vs_status rs = read_status(S, sc, nullptr);
    if (rs != VS_OK) return rs;
    out[VS_S_V] = sc[SC_V];
    out[VS_S_A] = sc[SC_A];
    out[VS_S_V0] = sc[SC_V0];
    out[VS_S_A0] = sc[SC_A0];
    out[VS_S_LAMBDA_V] = sc[SC_LAMV];
    out[VS_S_GAMMA_A] = sc[SC_GAMMA];
    out[VS_S_RELRES] = S->last_relres;
    out[VS_S_STEP] = (double)S->step;
    out[VS_S_CYCLES] = (double)S->last_cycles;
    return VS_OK;
}

namespace {
struct BlobHeader {
    char magic[8];
    int32_t nx, ny, nz, kind;
    int64_t step;
    double u0, u1;            // wall speeds
    double scal[SC_NSCAL];
};

// Whether p points into device memory (a checkpoint may live on the device: then every copy
// stays on the device). Host memory the runtime does not know reports an error: cleared.
bool device_blob(const void* p) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}
}  // namespace

vs_status vs_save_state(vs_state* S, void* blob, size_t* bytes) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (!bytes) return fail(VS_E_ARG, "bytes is NULL");
    const size_t N = (size_t)S->g.nx * S->g.ny * S->g.nz;
    const size_t need = sizeof(BlobHeader) + 8 * N * sizeof(double);
    if (!blob) {
        *bytes = need;
        return VS_OK;
    }
    if (*bytes < need) return fail(VS_E_ARG, "blob has %zu bytes, needs %zu", *bytes, need);
    HIP_TRY(hipStreamSynchronize(S->stream));
    const bool dev = device_blob(blob);
    BlobHeader hd{};
    std::memcpy(hd.magic, "VSSTATE2", 8);
    hd.nx = S->g.nx;
    hd.ny = S->g.ny;
    hd.nz = S->g.nz;
    hd.kind = S->w.kind;
    hd.step = S->step;
    hd.u0 = S->w.u0;
    hd.u1 = S->w.u1;
    HIP_TRY(hipMemcpy(hd.scal, S->scal, sizeof hd.scal, hipMemcpyDeviceToHost));
    if (dev)
        HIP_TRY(hipMemcpy(blob, &hd, sizeof hd, hipMemcpyHostToDevice));
    else
        std::memcpy(blob, &hd, sizeof hd);
    double* dst = (double*)((char*)blob + sizeof hd);
    const double* src[8] = {S->phi[S->cur], S->mu, S->om[0], S->om[1], S->om[2], S->ps[0], S->ps[1], S->ps[2]};
    for (int q = 0; q < 8; ++q)
        HIP_TRY(hipMemcpyAsync(dst + q * N, src[q], N * sizeof(double),
                               dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    *bytes = need;
    return VS_OK;
}

vs_status vs_load_state(vs_state* S, const void* blob, size_t bytes) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (!blob) return fail(VS_E_ARG, "blob is NULL");
    const size_t N = (size_t)S->g.nx * S->g.ny * S->g.nz;
    const size_t need = sizeof(BlobHeader) + 8 * N * sizeof(double);
    if (bytes < need) return fail(VS_E_ARG, "blob has %zu bytes, needs %zu", bytes, need);
    const bool dev = device_blob(blob);
    BlobHeader hd;
    if (dev)
        HIP_TRY(hipMemcpy(&hd, blob, sizeof hd, hipMemcpyDeviceToHost));
    else
        std::memcpy(&hd, blob, sizeof hd);
    if (std::memcmp(hd.magic, "VSSTATE2", 8) != 0) return fail(VS_E_ARG, "not a vs_save_state blob");
    if (hd.nx != S->g.nx || hd.ny != S->g.ny || hd.nz != S->g.nz) return fail(VS_E_ARG, "grid mismatch");
    if (hd.kind != S->w.kind) return fail(VS_E_ARG, "wall kind mismatch");
    HIP_TRY(hipStreamSynchronize(S->stream));
    const double* src = (const double*)((const char*)blob + sizeof hd);
    double* dst[8] = {S->phi[S->cur], S->mu, S->om[0], S->om[1], S->om[2], S->ps[0], S->ps[1], S->ps[2]};
    for (int q = 0; q < 8; ++q)
        HIP_TRY(hipMemcpyAsync(dst[q], src + q * N, N * sizeof(double),
                               dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    HIP_TRY(hipMemcpy(S->scal, hd.scal, sizeof hd.scal, hipMemcpyHostToDevice));
    // the checkpoint holds no time increments: the refined mode's predictor starts over
    const int no_hist[2] = {0, 0};
    HIP_TRY(hipMemcpy(S->istat + IS_HIST, no_hist, sizeof no_hist, hipMemcpyHostToDevice));
    S->step = hd.step;
    S->gamma_host = hd.scal[SC_GAMMA];
    if (hd.u0 != S->w.u0 || hd.u1 != S->w.u1) {
        // the fields carry the saved walls: restore the wall tables with them
        vs_walls w = S->w;
        w.u0 = hd.u0;
        w.u1 = hd.u1;
        const std::vector<double> prof = wall_tables(S->g, w);
        HIP_TRY(hipMemcpy(S->prof, prof.data(), prof.size() * sizeof(double), hipMemcpyHostToDevice));
        set_wall_state(S, w, prof);
    }
    return VS_OK;
}

vs_status vs_profile(vs_state* S, int32_t enable) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    HIP_TRY(hipStreamSynchronize(S->stream));
    if (enable) release_events(S);
    S->prof_on = enable != 0;
    return VS_OK;
}

int32_t vs_profile_count(void) { return K_NCLASS; }

const char* vs_profile_name(int32_t k) { return (k >= 0 && k < K_NCLASS) ? kClassNames[k] : ""; }

vs_status vs_profile_read(vs_state* S, int32_t kernel, double* total_ms, int64_t* launches) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (kernel < 0 || kernel >= K_NCLASS) return fail(VS_E_ARG, "kernel class out of range");
    HIP_TRY(hipStreamSynchronize(S->stream));
    double t = 0.0;
    int64_t n = 0;
    for (auto& u : S->ev_used) {
        if (u.first != kernel) continue;
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, u.second.first, u.second.second));
        t += ms;
        ++n;
    }
    if (total_ms) *total_ms = t;
    if (launches) *launches = n;
    return VS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------ autotuner
namespace {

// Picks the tuned launch shapes of S's grid by timing each candidate on S's own data: the
// phi update's x-slab length (written into the free phi buffer), the volume/area partials'
// block cap and the chemical potential's form (they recompute mu and the scalars from the same
// phi; the partial sums' order differs with the cap, so mu and the scalars are saved first, mu
// in the source buffer, which every step rewrites before use, and restored at the end), the
// flow residual's block cap (partials only) and the pair tridiagonal solves' segment layout
// (spectral scratch only). One coordinate at a time, each candidate launched kReps times after
// one warm-up launch, the fastest mean kept. The state's fields and scalars come out as they
// went in.
vs_status autotune_state(vs_state* S, Tuning* picked) {
    constexpr int kReps = 5;
    HIP_TRY(hipStreamSynchronize(S->stream));
    const size_t fbytes = (size_t)S->g.nx * S->g.ny * S->g.nz * sizeof(double);
    double sc_save[SC_NSCAL];
    HIP_TRY(hipMemcpy(sc_save, S->scal, sizeof sc_save, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpyAsync(S->src[2], S->mu, fbytes, hipMemcpyDeviceToDevice, S->stream));
    const StepCfg c = step_cfg(S);
    const double dt = 1e-12;   // the advance's output buffer is scratch; any dt does
    const StepArgs A = step_args(S, S->cur, dt, false);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(VS_E_HIP, "hipEventCreate failed");
    }
    hipError_t err = hipSuccess;
    auto time = [&](auto launch) -> float {
        launch();
        (void)hipEventRecord(e0, S->stream);
        for (int r = 0; r < kReps; ++r) launch();
        (void)hipEventRecord(e1, S->stream);
        hipError_t e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess && err == hipSuccess) err = e;
        return ms / kReps;
    };
    const Prec pr = S->f32 ? P32 : P64;
    Tuning t = tuning_for(S->d);
    auto pick = [&](int* field, std::initializer_list<int> cands, auto launch) {
        int best = *field;
        float tb = 1e30f;
        for (int v : cands) {
            *field = v;
            set_tuning(S->d, t);
            const float ms = time(launch);
            if (ms < tb) {
                tb = ms;
                best = v;
            }
        }
        *field = best;
        set_tuning(S->d, t);
    };
    pick(&t.adv_slab, {2, 4, 8}, [&] { launch_advance(c.st, c.d, pr, A.adv); });
    pick(&t.va_maxb, {256, 512, 1024, 2048}, [&] {
        launch_va_partials(c.st, c.d, A.va);
        launch_mu(c.st, c.d, c.model, pr, A.mu);
    });
    // the chemical potential's form: LDS tiles, or register marching (n_z in {64, 128, 256})
    // with 1 or 2 rows per wave and 2 .. 16 planes per slab, as one coordinate
    {
        const int zpl = S->d.nz / 64;
        const bool reg_ok = S->d.nz % 64 == 0 && (zpl == 1 || zpl == 2 || zpl == 4);
        const int cand[][2] = {{0, 8}, {1, 2}, {1, 4}, {1, 8}, {1, 16}, {2, 2}, {2, 4}, {2, 8}, {2, 16}};
        int bk = t.mu_kind, bn = t.mu_ni;
        float tb = 1e30f;
        for (const auto& cd : cand) {
            if (cd[0] > 0 && !reg_ok) continue;
            t.mu_kind = cd[0];
            t.mu_ni = cd[1];
            set_tuning(S->d, t);
            const float ms = time([&] {
                launch_va_partials(c.st, c.d, A.va);
                launch_mu(c.st, c.d, c.model, pr, A.mu);
            });
            if (ms < tb) {
                tb = ms;
                bk = cd[0];
                bn = cd[1];
            }
        }
        t.mu_kind = bk;
        t.mu_ni = bn;
        set_tuning(S->d, t);
    }
    pick(&t.res_maxb, {512, 1024, 2048, 4096},
         [&] { launch_resid_flow_over(c.st, c.d, false, S->f32 ? A.resc[0] : A.res); });
    if (fused_flow_ok(S->d) && seg_has_alt(S->d.M))
        pick(&t.seg_alt, {0, 1}, [&] {
            launch_tri_pair(c.st, c.d, S->f32, S->f32, S->f32 ? A.trc[0] : A.tri);
        });
    // the transforms of the FP64 flow pass: two 1D passes per direction, or one plane pass;
    // timed with the inverse writing back into the spectral buffers it reads (each block, or
    // the plane pass's each row, reads all it transforms before it writes), so no field changes
    if (!S->f32 && fused_flow_ok(S->d) && plane_fits(S->d)) {
        Over<ZArgs> zin = A.zout6;
        for (int q = 0; q < 6; ++q) zin.one.u[q] = (double*)A.hx6.one.spec[q];
        pick(&t.plane, {0, 1}, [&] {
            if (t.plane) {
                launch_plane(c.st, c.d, true, 3, A.zfwd, A.hx3);
                launch_plane(c.st, c.d, false, 6, zin, A.hx6);
            } else {
                launch_hz(c.st, c.d, c.pz, false, 3, A.zfwd);
                launch_hx(c.st, c.d, c.px, false, 3, A.hx3);
                launch_hx(c.st, c.d, c.px, false, 6, A.hx6);
                launch_hz(c.st, c.d, c.pz, false, 6, zin);
            }
        });
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(VS_E_HIP, "autotune timing failed: %s", hipGetErrorString(err));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(S->mu, S->src[2], fbytes, hipMemcpyDeviceToDevice, S->stream));
    HIP_TRY(hipMemcpyAsync(S->scal, sc_save, sizeof sc_save, hipMemcpyHostToDevice, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    set_tuning(S->d, t, !S->f32);
    if (picked) *picked = t;
    return VS_OK;
}

}  // namespace

extern "C" vs_status vs_set_launch_shapes(const vs_grid* grid, const int32_t shapes[7]) {
    vs_status st = check_grid(grid);
    if (st != VS_OK) return st;
    if (!shapes) return fail(VS_E_ARG, "shapes is NULL");
    const Tuning t{shapes[0], shapes[1], shapes[2], shapes[3], shapes[4], shapes[5], shapes[6]};
    if (t.adv_slab < 1 || t.adv_slab > 64) return fail(VS_E_ARG, "adv_slab must be in [1, 64]");
    if (t.va_maxb < 64 || t.va_maxb > kMaxPartialBlocks)
        return fail(VS_E_ARG, "va_maxb must be in [64, %d]", kMaxPartialBlocks);
    if (t.res_maxb < 64 || t.res_maxb > kMaxPartialBlocks)
        return fail(VS_E_ARG, "res_maxb must be in [64, %d]", kMaxPartialBlocks);
    if (t.seg_alt != 0 && t.seg_alt != 1) return fail(VS_E_ARG, "seg_alt must be 0 or 1");
    if (t.mu_kind < 0 || t.mu_kind > 2) return fail(VS_E_ARG, "mu_kind must be 0, 1 or 2");
    if (t.mu_ni < 1 || t.mu_ni > 64) return fail(VS_E_ARG, "mu_ni must be in [1, 64]");
    if (t.plane != 0 && t.plane != 1) return fail(VS_E_ARG, "plane must be 0 or 1");
    Dims d{grid->nx, grid->ny, grid->nz, grid->ny - 2, grid->h, 0.0, 0.0};
    set_tuning(d, t, true);
    return VS_OK;
}

extern "C" vs_status vs_autotune(vs_state* S, int32_t picked[7]) {
    if (!S) return fail(VS_E_STATE, "state is NULL");
    if (S->prof_on) return fail(VS_E_ARG, "vs_autotune: switch the event timer off first");
    Tuning t{};
    const vs_status st = autotune_state(S, &t);
    if (st != VS_OK) return st;
    if (picked) {
        picked[0] = t.adv_slab;
        picked[1] = t.va_maxb;
        picked[2] = t.res_maxb;
        picked[3] = t.seg_alt;
        picked[4] = t.mu_kind;
        picked[5] = t.mu_ni;
        picked[6] = t.plane;
    }
    return VS_OK;
}

// ------------------------------------------------------------------------------ batches
// Instances of one grid class (same grid, precision, model and cycle count) step together:
// each kernel of a step is launched once for all instances of the class, its per-instance
// arguments read from device tables (Over in vs_internal.h). One launch per class fills the
// GPU at every grid size and evens out the persistent plane passes, whose work comes in whole
// (plane, component) units, one per CU at a time: a single 128^3 instance has 3 x 126 units
// for 256 CUs in the forward pass (two rounds, the second half empty), thirteen have 4,914
// (twenty rounds, 96% full). Measured on batch64: 1.10e10 cell-updates/s with one group per
// class against 1.05e10 with groups of about 2^21 nodes (which kept more of each hand-off in
// the 256 MB Infinity Cache). Two steps of every class are captured into one HIP graph (two
// steps bring every instance's phi buffer back to where it started), the classes spread over
// the batch streams, and replayed. Instances outside the fused forms (FP64 with more than one
// cycle per solve) are stepped one by one inside the same graph.
struct BatchClass {
    Dims d{};
    FftPlan px{}, pz{};
    bool f32 = false;
    int model = 0, mc = 1;
    std::vector<vs_state*> st;
    StepArgs A[2];                      // the two captured steps, tables in vs_batch::dtab
};

struct vs_batch {
    std::vector<vs_state*> st;
    std::vector<BatchClass> cls;
    std::vector<vs_state*> loose;       // stepped one by one (on the last stream)
    std::vector<hipStream_t> streams;   // class c runs on streams[c % size]
    std::vector<hipEvent_t> ev;         // fork event + one join event per stream
    hipStream_t origin = nullptr;       // the caller's stream: graph launches go here
    hipStream_t cap = nullptr;          // private stream the graph is captured from
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    char* dtab = nullptr;               // device argument tables of the class launches
    size_t dtab_bytes = 0;
    std::vector<double> dt;             // time steps baked into the captured graph
    std::vector<long long> gen;         // each instance's walls_gen at capture
};

namespace {

void batch_release_graph(vs_batch* B) {
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
}

bool same_class(const vs_state* a, const vs_state* b) {
    return a->g.nx == b->g.nx && a->g.ny == b->g.ny && a->g.nz == b->g.nz && a->g.h == b->g.h &&
           a->f32 == b->f32 && a->p.model == b->p.model &&
           a->p.poisson_max_cycles == b->p.poisson_max_cycles;
}

bool class_eligible(const vs_state* S) {
    return fused_flow_ok(S->d) && (S->f32 || S->p.poisson_max_cycles == 1);
}


double batch_dt(const vs_batch* B, const vs_state* S, const double* dt) {
    for (size_t i = 0; i < B->st.size(); ++i)
        if (B->st[i] == S) return dt[i];
    return 0.0;
}

// Builds every class's two-step argument tables on the host (each instance with its own phi
// buffers, dt, walls and parameters), uploads them in one copy, and points the classes'
// launches at them.
vs_status build_tables(vs_batch* B, const double* dt) {
    std::vector<char> host;
    std::vector<size_t> offs;   // table offsets, in the order of the classes, steps and fields
    auto put = [&](const void* src, size_t bytes) {
        const size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + bytes);
        std::memcpy(host.data() + off, src, bytes);
        return off;
    };
    for (BatchClass& C : B->cls) {
        const int n = (int)C.st.size();
        for (int k = 0; k < 2; ++k) {
            std::vector<StepArgs> per;
            for (vs_state* S : C.st) {
                const int par = (S->cur + k) & 1;
                per.push_back(step_args(S, par, batch_dt(B, S, dt), k == 1 && C.mc == 1));
            }
            StepArgs& A = C.A[k];
#define VS_GATHER(F)                                                                        \
            {                                                                               \
                using AT = decltype(A.F.one);                                               \
                std::vector<AT> v;                                                          \
                for (const StepArgs& x : per) v.push_back(x.F.one);                         \
                A.F.one = v[0];                                                             \
                A.F.n = n;                                                                  \
                A.F.tab = nullptr;                                                          \
                offs.push_back(put(v.data(), v.size() * sizeof(AT)));                       \
            }
            VS_STEP_FIELDS(VS_GATHER)
#undef VS_GATHER
        }
    }
    if (host.size() > B->dtab_bytes) {
        if (B->dtab) (void)hipFree(B->dtab);
        B->dtab = nullptr;
        B->dtab_bytes = 0;
        HIP_TRY(hipMalloc((void**)&B->dtab, host.size()));
        B->dtab_bytes = host.size();
    }
    if (!host.empty())
        HIP_TRY(hipMemcpy(B->dtab, host.data(), host.size(), hipMemcpyHostToDevice));
    size_t q = 0;
    for (BatchClass& C : B->cls)
        for (int k = 0; k < 2; ++k) {
            StepArgs& A = C.A[k];
#define VS_SETTAB(F)                                                                        \
            A.F.tab = reinterpret_cast<decltype(A.F.tab)>(B->dtab + offs[q++]);
            VS_STEP_FIELDS(VS_SETTAB)
#undef VS_SETTAB
        }
    return VS_OK;
}

// One step of a class: every kernel launched once over the class's tables.
void enqueue_class_step(const BatchClass& C, int k, hipStream_t st) {
    const StepCfg c{st, C.d, C.px, C.pz, C.f32, C.model, C.mc, 0.0, false, nullptr};
    const StepArgs& A = C.A[k];
    launch_advance(st, C.d, C.f32 ? P32 : P64, A.adv);
    enqueue_va_mu_args(c, A);
    enqueue_flow_args(c, A, k == 0 && C.mc == 1, C.mc);
}

// Capture two time steps of every class and loose instance: fork from the capture stream to
// the batch streams, enqueue, join back.
vs_status batch_capture(vs_batch* B, const double* dt) {
    batch_release_graph(B);
    vs_status st = build_tables(B, dt);
    if (st != VS_OK) return st;
    const int ns = (int)B->streams.size();
    HIP_TRY(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    auto body = [&]() -> hipError_t {
        hipError_t e = hipEventRecord(B->ev[0], B->cap);
        if (e != hipSuccess) return e;
        for (int k = 0; k < ns; ++k)
            if ((e = hipStreamWaitEvent(B->streams[k], B->ev[0], 0)) != hipSuccess) return e;
        for (int k = 0; k < 2; ++k)
            for (size_t c = 0; c < B->cls.size(); ++c)
                enqueue_class_step(B->cls[c], k, B->streams[c % ns]);
        for (vs_state* S : B->loose) {
            const double d = batch_dt(B, S, dt);
            enqueue_step(S, d, true);
            enqueue_step(S, d, false);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (int k = 0; k < ns; ++k) {
            if ((e = hipEventRecord(B->ev[1 + k], B->streams[k])) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(B->cap, B->ev[1 + k], 0)) != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const hipError_t eb = body();
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(B->cap, &g);
    if (eb != hipSuccess) st = fail(VS_E_HIP, "batch capture failed: %s", hipGetErrorString(eb));
    else if (ee != hipSuccess) st = fail(VS_E_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ee));
    if (st != VS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    B->graph = g;
    HIP_TRY(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->dt.assign(dt, dt + B->st.size());
    B->gen.clear();
    for (vs_state* S : B->st) B->gen.push_back(S->walls_gen);
    return VS_OK;
}

}  // namespace

extern "C" {

vs_status vs_batch_create(vs_state* const* states, int32_t n, void* stream, int32_t nstreams,
                          vs_batch** out) {
    if (!out) return fail(VS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!states || n < 1) return fail(VS_E_ARG, "need n >= 1 states");
    if (nstreams < 1) return fail(VS_E_ARG, "nstreams must be >= 1");
    for (int i = 0; i < n; ++i) {
        if (!states[i]) return fail(VS_E_STATE, "state %d is NULL", i);
        for (int k = 0; k < i; ++k)
            if (states[k] == states[i]) return fail(VS_E_ARG, "state %d appears twice", i);
    }
    vs_batch* B = new vs_batch();
    B->st.assign(states, states + n);
    B->origin = (hipStream_t)stream;
    // the instances of each class, in input order
    std::vector<std::vector<vs_state*>> by_class;
    for (vs_state* S : B->st) {
        if (!class_eligible(S)) {
            B->loose.push_back(S);
            continue;
        }
        bool placed = false;
        for (auto& v : by_class)
            if (same_class(v[0], S)) {
                v.push_back(S);
                placed = true;
                break;
            }
        if (!placed) by_class.push_back({S});
    }
    for (const auto& v : by_class) {
        const vs_state* S0 = v[0];
        BatchClass C;
        C.d = S0->d;
        C.px = S0->px;
        C.pz = S0->pz;
        C.f32 = S0->f32;
        C.model = S0->p.model;
        C.mc = S0->p.poisson_max_cycles;
        C.st = v;
        B->cls.push_back(C);
    }
    const int groups = (int)B->cls.size() + (B->loose.empty() ? 0 : 1);
    const int ns = nstreams < groups ? nstreams : groups;
    auto bail = [&](vs_status e) {
        if (B->cap) (void)hipStreamDestroy(B->cap);
        for (hipStream_t q : B->streams) (void)hipStreamDestroy(q);
        for (hipEvent_t x : B->ev) (void)hipEventDestroy(x);
        delete B;
        return e;
    };
    if (hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(VS_E_HIP, "hipStreamCreate failed"));
    for (int k = 0; k < ns; ++k) {
        hipStream_t q = nullptr;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(VS_E_HIP, "hipStreamCreate failed"));
        B->streams.push_back(q);
    }
    for (int k = 0; k <= ns; ++k) {
        hipEvent_t x = nullptr;
        if (hipEventCreateWithFlags(&x, hipEventDisableTiming) != hipSuccess)
            return bail(fail(VS_E_HIP, "hipEventCreate failed"));
        B->ev.push_back(x);
    }
    // finish each state's pending work, then move it onto a batch stream (loose instances
    // run on the last one)
    for (int i = 0; i < n; ++i) {
        vs_state* S = B->st[i];
        if (hipStreamSynchronize(S->stream) != hipSuccess) return bail(fail(VS_E_HIP, "sync failed"));
        S->prof_on = false;
        S->stream = B->streams[ns - 1];
    }
    for (size_t c = 0; c < B->cls.size(); ++c)
        for (vs_state* S : B->cls[c].st) S->stream = B->streams[c % ns];
    // launch shapes of every grid class not tuned yet, on its first instance
    for (BatchClass& C : B->cls) {
        if (tuned(C.d, C.st[0]->f32)) continue;
        const vs_status st = autotune_state(C.st[0], nullptr);
        if (st != VS_OK) {
            vs_batch_destroy(B);
            return st;
        }
    }
    *out = B;
    return VS_OK;
}

vs_status vs_batch_step(vs_batch* B, const double* dt, int32_t nsteps) {
    if (!B) return fail(VS_E_STATE, "batch is NULL");
    if (!dt) return fail(VS_E_ARG, "dt is NULL");
    if (nsteps < 2 || (nsteps & 1)) return fail(VS_E_ARG, "nsteps must be even and >= 2");
    const size_t n = B->st.size();
    for (size_t i = 0; i < n; ++i) {
        vs_state* S = B->st[i];
        if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return fail(VS_E_ARG, "dt[%zu] must be > 0", i);
        if (!(S->p.flags & VS_ALLOW_UNSTABLE) && dt[i] * stability_rate(S) > 2.0)
            return fail(VS_E_UNSTABLE, "instance %zu: dt = %.4g exceeds the forward-Euler bound %.4g",
                        i, dt[i], 2.0 / stability_rate(S));
    }
    for (size_t i = 0; i < n; ++i) {
        const vs_status st = ensure_inertial_table(B->st[i], dt[i]);
        if (st != VS_OK) return st;
    }
    bool same = B->exec && B->dt.size() == n && B->gen.size() == n;
    for (size_t i = 0; same && i < n; ++i) same = B->dt[i] == dt[i] && B->gen[i] == B->st[i]->walls_gen;
    if (!same) {
        const vs_status st = batch_capture(B, dt);
        if (st != VS_OK) return st;
    }
    for (size_t i = 0; i < n; ++i) launch_reset_stats(B->origin, B->st[i]->scal, B->st[i]->istat);
    HIP_TRY(hipGetLastError());
    for (int r = 0; r < nsteps / 2; ++r) HIP_TRY(hipGraphLaunch(B->exec, B->origin));
    HIP_TRY(hipStreamSynchronize(B->origin));
    vs_status worst = VS_OK;
    for (size_t i = 0; i < n; ++i) {
        B->st[i]->step += nsteps;
        const vs_status st = collect(B->st[i], "vs_batch_step");
        if (st != VS_OK && worst == VS_OK) worst = st;
    }
    return worst;
}

void vs_batch_destroy(vs_batch* B) {
    if (!B) return;
    (void)hipStreamSynchronize(B->origin);
    for (hipStream_t q : B->streams) (void)hipStreamSynchronize(q);
    batch_release_graph(B);
    if (B->dtab) (void)hipFree(B->dtab);
    for (hipEvent_t x : B->ev) (void)hipEventDestroy(x);
    // states keep working after the batch: give them back a valid stream (the origin)
    for (vs_state* S : B->st) S->stream = B->origin;
    for (hipStream_t q : B->streams) (void)hipStreamDestroy(q);
    (void)hipStreamDestroy(B->cap);
    delete B;
}

void vs_destroy(vs_state* S) {
    if (!S) return;
    (void)hipStreamSynchronize(S->stream);
    release_events(S);
    for (hipEvent_t e : S->ev_pool) (void)hipEventDestroy(e);
    delete S;
}

}  // extern "C"
