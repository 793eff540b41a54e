/*
 * vs.h — C ABI of the MI355X (gfx950) library for the vorticity–stream-vector phase-field
 * method (Gallen, Muñoz Biosca, Castro, Hernández-Machado, arXiv 2601.05031).
 *
 * One call of vs_step advances the coupled system of the main text, eq. (5a)–(5c)
 * (supplementary eq. (29a)–(29c)) by forward Euler, in the segregated order of the
 * "Numerical implementation" section: (1) advance phi, (2) solve the vorticity Poisson
 * problem, (3) solve the stream-vector Poisson problem.
 *
 * Grid ("Numerical implementation"): nodes (i h, j h, k h), 0 <= i < nx, 0 <= j < ny,
 * 0 <= k < nz, equal spacing h. x and z are periodic; the channel walls are the node planes
 * j = 0 and j = ny-1 (height H = (ny-1) h); the imposed flow runs along +z.
 *
 * Layout of every scalar field in device memory: nx*ny*nz doubles, index (i*ny + j)*nz + k
 * (z fastest). Vector fields are three such arrays (x, y, z components).
 *
 * Conventions shared by all calls:
 *  - Every call returns a vs_status; 0 is success, negative values are errors. No call
 *    aborts the process. vs_last_error() returns a message for the calling thread's last
 *    failed call (valid until the next call on that thread).
 *  - Ownership: the caller owns all device memory (the workspace, phi0, f, u, adjoint
 *    buffers) and the HIP stream; the library owns the opaque vs_state (host memory only).
 *    The workspace must outlive the state. Inputs are copied; outputs are read in place at
 *    vs_field_offset() inside the workspace.
 *  - Streams: all device work is enqueued on the stream given to vs_init, in order.
 *    vs_step, vs_poisson_solve, vs_get_scalars and vs_save_state synchronise that stream
 *    before they return.
 *  - Threads: one vs_state per thread at a time; calls on one state are not re-entrant.
 *  - Argument errors are detected on the host before anything is enqueued.
 */
#ifndef VS_H
#define VS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VS_OK = 0,
    VS_E_ARG = -1,          /* invalid argument (sizes, non-positive h, eta, M, eps, dt ...) */
    VS_E_WORKSPACE = -2,    /* workspace missing, too small or misaligned (256 B)           */
    VS_E_HIP = -3,          /* a HIP runtime call failed                                   */
    VS_E_NOCONV = -4,       /* a Poisson solve missed rtol after max_cycles cycles         */
    VS_E_NONFINITE = -5,    /* NaN or Inf seen in a residual norm or in V, A               */
    VS_E_UNSTABLE = -6,     /* dt above the linear forward-Euler bound; nothing enqueued   */
    VS_E_STATE = -7,        /* null or unusable state                                     */
    VS_E_UNSUPPORTED = -8   /* call or mode not available for these parameters, or size   */
} vs_status;

/* vs_walls.kind */
enum { VS_POISEUILLE = 1, VS_COUETTE = 2 };
/* vs_params.model */
enum { VS_BENDING = 1, VS_CAHN_HILLIARD = 2 };
/* vs_params.precision: VS_FP64 runs every step in FP64 and solves each Poisson problem by one
 * exact spectral pass. VS_FP32_REFINED (the reduced-precision mode) keeps phi, omega, psi and
 * the vorticity source S in FP64 and stores mu and every spectral intermediate as FP32: the
 * phi update is computed in FP32 arithmetic (the increment added to the FP64 phi); the
 * chemical potential is computed in FP64 and stored as FP32 (FP32 arithmetic there costs ~1e-5
 * in mu); the volume/area integrals are FP64; each step's two flow problems run
 * defect-correction cycles: an FP64 residual, its correction solved in FP32 (transforms and
 * tridiagonal solves), an FP64 update, an FP64 check, until the relative residuals meet
 * poisson_rtol (up to poisson_max_cycles; the initial solve takes at least 4). The first cycle
 * of a step starts from omega and psi extrapolated in time from the last two steps'
 * increments (held in FP32 in the workspace: 48 bytes per node more than VS_FP64): quadratic
 * extrapolation leaves a residual small enough that one FP32 cycle usually meets rtol = 1e-10,
 * where the previous step's fields alone need two. The first two steps after vs_init or
 * vs_load_state (checkpoints hold no increments) extrapolate from fewer steps. S stays FP64
 * because FP32 rounding of S alone moves the small components of psi by ~3e-6. It needs nx, nz
 * in {32, 48, 64, 96, 128, 192, 256} and 4 <= ny - 2 <= 256. In this mode
 * vs_field_offset(VS_MU) points at nx*ny*nz floats. */
enum { VS_FP64 = 1, VS_FP32_REFINED = 2 };
/* vs_params.flags */
enum { VS_ALLOW_UNSTABLE = 1 };
/* vs_field_offset field ids */
enum {
    VS_PHI = 0, VS_MU = 1,
    VS_OMEGA_X = 2, VS_OMEGA_Y = 3, VS_OMEGA_Z = 4,
    VS_PSI_X = 5, VS_PSI_Y = 6, VS_PSI_Z = 7,
    VS_NFIELDS = 8
};
/* vs_get_scalars slots */
enum {
    VS_S_V = 0, VS_S_A = 1, VS_S_V0 = 2, VS_S_A0 = 3, VS_S_LAMBDA_V = 4, VS_S_GAMMA_A = 5,
    VS_S_RELRES = 6,   /* largest final relative residual of the Poisson solves of the last call */
    VS_S_STEP = 7,     /* number of completed time steps since vs_init                            */
    VS_S_CYCLES = 8,   /* Poisson refinement cycles run by the last vs_step call (all solves)      */
    VS_NSCALARS = 9
};
/* Per-step log records (vs_log_read): fields of one record */
enum {
    VS_L_INDEX = 0,    /* record number since vs_init (0: the initial solve, n: time step n)       */
    VS_L_CYCLES = 1,   /* Poisson cycles counted so far in the vs_step call that ran the step      */
    VS_L_RELRES = 2,   /* the larger final relative residual of the step's two flow solves        */
    VS_L_V = 3, VS_L_A = 4, VS_L_LAMBDA_V = 5, VS_L_GAMMA_A = 6,   /* of the step's new phi      */
    VS_L_CONV = 7,     /* 1 if both solves met poisson_rtol                                        */
    VS_LOG_FIELDS = 8,
    VS_LOG_CAP = 4096  /* records kept (a ring in the workspace: the oldest are overwritten)        */
};

/* Grid ("Numerical implementation"). ny counts both wall rows; ny >= 3.
 * nx, nz >= 4, even, of the form 2^a 3^b, at most 512 (the periodic directions are
 * diagonalised by fast transforms of these lengths); ny * nz <= 2^20 (one x-plane) and
 * nx * ny * nz <= 2^30. Larger grids fail with VS_E_ARG / VS_E_UNSUPPORTED. */
typedef struct {
    int32_t nx, ny, nz;
    double h;
} vs_grid;

/* Imposed channel flow along +z ("Boundary conditions"). The walls carry the flow without a
 * body: Dirichlet values of psi and omega on j = 0 and j = ny-1 derived from v by
 * v = curl psi (eq. (3)) and omega = curl v (eq. (4)):
 *   VS_POISEUILLE, centreline speed u0:  v_z = 4 u0 y (H-y)/H^2,
 *       psi_x = -(4 u0/H^2)(H y^2/2 - y^3/3), omega_x = (4 u0/H^2)(H - 2y);
 *   VS_COUETTE, wall speeds u0 (y = 0) and u1 (y = H):  v_z = u0 + (u1-u0) y/H,
 *       psi_x = -(u0 y + (u1-u0) y^2/(2H)), omega_x = (u1-u0)/H.
 * All other components are zero on the walls. Wall nodes move with the wall. */
typedef struct {
    int32_t kind;
    double u0, u1;
} vs_walls;

/* Physical and solver parameters.
 *  eta       viscosity (eq. (5b), > 0)
 *  mobility  M of eq. (5a) (> 0)
 *  eps       interface width of the bending energy (SM eq. (30), > 0)
 *  kappa     bending modulus (SM eq. (30), >= 0)
 *  sigma     Cahn–Hilliard coefficient (eq. F_CH, SM (31), > 0 for that model)
 *  gamma0    constant part of the surface-tension coefficient gamma_A of SM eq. (35)
 *  rate_V    volume penalty: lambda_V = 2 rate_V (V0 - V)/(M |Omega|)   (0 = off)
 *  k_A       area penalty:   gamma_A = gamma0 + k_A (A - A0)/A0          (0 = off)
 *  bend_scale  multiplies C_b = 3 sqrt(2) kappa/(8 eps^3) of SM eq. (35) (1.0 = as printed)
 *  poisson_rtol, poisson_max_cycles: each Poisson solve of vs_step runs up to max_cycles
 *            refinement cycles until ||b - L_h u||_2 <= rtol ||b||_2 over the three
 *            components (b includes the wall terms); max_cycles in [1, 16].
 *  flags     VS_ALLOW_UNSTABLE skips the forward-Euler stability check of vs_step.
 *  rho       fluid density of the inertial variant (SM "Time-dependency and inertial flow",
 *            eq. (36)): (rho/eta) d(omega)/dt - lap omega = -(1/eta) grad phi x grad mu,
 *            taken implicitly in each step, (L_h - a) omega^{n+1} = S - a omega^n with
 *            a = rho/(eta dt); omega^0 is the quasi-steady field of eq. (5b). 0 = eq. (5b).
 *            rho > 0 needs precision VS_FP64 and poisson_max_cycles = 1 (VS_E_UNSUPPORTED
 *            otherwise); vs_grad_step and vs_set_walls return VS_E_UNSUPPORTED for it. */
typedef struct {
    int32_t model;
    int32_t precision;
    double eta, mobility, eps, kappa, sigma;
    double gamma0;
    double rate_V, k_A;
    double bend_scale;
    double poisson_rtol;
    int32_t poisson_max_cycles;
    int32_t flags;
    double rho;
} vs_params;

typedef struct vs_state vs_state;

/* Size in bytes of the device workspace vs_init needs for this grid and parameters. */
vs_status vs_workspace_bytes(const vs_grid* grid, const vs_params* params, size_t* bytes);

/* Create a state. phi0: device pointer to nx*ny*nz doubles (initial phase field, copied).
 * workspace: device memory of at least vs_workspace_bytes bytes, 256-byte aligned, owned by
 * the caller. stream: a hipStream_t (NULL = default stream).
 * Initialisation: V0 = V[phi0], A0 = A[phi0] (SM eq. (37), (32)), lambda_V = 0,
 * gamma_A = gamma0, mu from phi0, then omega and psi solved from phi0 with the no-body
 * fields as the initial guess. Synchronises the stream. */
vs_status vs_init(const vs_grid* grid, const vs_walls* walls, const vs_params* params,
                  const double* phi0, void* workspace, size_t bytes, void* stream,
                  vs_state** out);

/* Solve the discrete Poisson problem L_h u = f ("Numerical implementation"; the operator of
 * eq. (5b), (5c)) on the interior rows 1 <= j <= ny-2 with the Dirichlet values stored in u
 * on j = 0 and j = ny-1, periodic in x and z, for one scalar field.
 * f: device, nx*ny*nz doubles, wall rows ignored. u: device, in: initial guess and wall
 * values, out: solution (wall rows unchanged). Runs refinement cycles until
 * ||f - L_h u||_2 <= rtol ||f~||_2 (f~ = f minus the wall terms) or max_cycles (1..16).
 * cycles_out, relres_out may be NULL. Returns VS_E_NOCONV (u still written) if rtol was not
 * reached. Uses the state's scratch space; does not touch the state's fields. Synchronises. */
vs_status vs_poisson_solve(vs_state* state, const double* f, double* u, double rtol,
                           int32_t max_cycles, int32_t* cycles_out, double* relres_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): vs_poisson_solve without a state or workspace.
 * Same problem, arguments, convergence rule and results as vs_poisson_solve on a state of
 * this grid (f, u: device, nx*ny*nz doubles; u in: initial guess and wall values, out:
 * solution), enqueued on `stream` (a hipStream_t, NULL = default) and synchronised before the
 * call returns. Its scratch (one FP64 spectral field, the twiddle and pivot tables, residual
 * partials, status words) is a static device array of vs_noalloc_scratch_bytes() bytes
 * (48 MiB), one per device, held until the process ends; grids whose scratch does not fit
 * (8 nx ny nz bytes plus the tables: up to 128 x 128 x 256 at nx = nz = 128) return
 * VS_E_WORKSPACE before anything is enqueued. The call allocates nothing: no hipMalloc,
 * hipFree or allocating library routine. The tables are uploaded (from host memory) only
 * when the grid differs from the previous call's on that device. Every call on a device
 * shares that device's scratch: calls that overlap on one device (other threads, other
 * streams) race and must not be issued. */
vs_status vs_poisson_solve_noalloc(const vs_grid* grid, const double* f, double* u, double rtol,
                                   int32_t max_cycles, void* stream, int32_t* cycles_out,
                                   double* relres_out);
/* Size in bytes of the static scratch of vs_poisson_solve_noalloc on each device. */
size_t vs_noalloc_scratch_bytes(void);

/* Advance nsteps >= 1 time steps of size dt > 0 (main text eq. (5a)–(5c), forward Euler).
 * Per step: phi^{n+1} = phi^n + dt [M (L_h mu^n + lambda_V^n) - (curl psi^n) . D phi^n];
 * V, A, lambda_V, gamma_A and mu from phi^{n+1}; omega^{n+1} from
 * L_h omega = (1/eta) D phi x D mu; psi^{n+1} from L_h psi = -omega.
 * Returns VS_E_UNSTABLE before enqueuing anything if dt exceeds the linear bound
 * 2 / (M (12/h^2) [C_b (2 + 12 eps^2/h^2)^2 + 12 |gamma_A|/h^2]) (bending) or
 * 2 / (M (12/h^2)(2 + 12 sigma/h^2)) (Cahn–Hilliard), unless VS_ALLOW_UNSTABLE is set.
 * Device-side failures (VS_E_NOCONV, VS_E_NONFINITE) are reported at the end of the call,
 * after all nsteps have run. Synchronises the stream once, at the end. With rho > 0 the
 * first call with a new dt also synchronises before it enqueues anything, to upload that
 * dt's vorticity pivots (so it cannot run under stream capture). */
vs_status vs_step(vs_state* state, double dt, int32_t nsteps);

/* Reverse step of one time step (the discrete adjoint of vs_step's update, FP64 mode only;
 * VS_E_UNSUPPORTED in VS_FP32_REFINED and for the inertial variant, rho > 0). The state must hold level n as vs_step leaves it
 * (phi^n with its mu^n, omega^n, psi^n and multipliers), e.g. reloaded from a vs_save_state
 * checkpoint and advanced to n. With a = dL/dphi^{n+1}:
 *   adj_prev = (d phi^{n+1} / d phi^n)^T a, where mu^n, psi^n (through the vorticity and
 *              stream-vector problems, main text eq. (5b), (5c)), lambda_V^n and gamma_A^n
 *              are differentiated as functions of phi^n (SM eq. (32), (35), (37), (38)) and
 *              V0, A0 are held fixed;
 *   dparams[0] += a^T d phi^{n+1} / d kappa;
 *   dparams[1] += a^T d phi^{n+1} / d s, where s scales both wall speeds (u0, u1) -> (s u0,
 *              s u1) at s = 1 (every wall table is linear in the wall speeds).
 * adj_next, adj_prev: device, nx*ny*nz doubles each, z fastest, must not alias; dparams: host,
 * 2 doubles, accumulated. The two adjoint Poisson solves are verified to poisson_rtol like the
 * forward ones (VS_E_NOCONV otherwise). The state's fields are left unchanged (the reverse
 * step uses the spectral scratch and the spare phi buffer). Synchronises the stream once. */
vs_status vs_grad_step(vs_state* state, double dt, const double* adj_next, double* adj_prev,
                       double dparams[2]);

/* Time-dependent walls (SM "Time-dependency and inertial flow": only the boundary data
 * change). New wall speeds of the same kind (Poiseuille: u0 = centreline speed; Couette:
 * u0, u1 = wall speeds) take effect now: the Poisson problems are linear in the wall data and
 * the no-body channel fields solve them exactly, so omega_x and psi_x shift by the difference
 * of the no-body fields (equal to re-solving the flow with the new walls), and the next steps
 * use the new wall speeds. An oscillatory flow calls this before each vs_step. A batch that
 * holds the state re-captures its graph on its next vs_batch_step. Checkpoints carry the
 * walls. VS_E_ARG if the kind differs; VS_E_UNSUPPORTED for the inertial variant (rho > 0).
 * Synchronises the stream. */
vs_status vs_set_walls(vs_state* state, const vs_walls* walls);

/* Diagnostics of the current state, on the device (synchronises the stream):
 *   out[0] = int |omega - omega_0|^2, out[1] = int |psi - psi_0|^2: the flow observables of
 *            the results section, about the no-body channel fields omega_0, psi_0 of the
 *            current walls (trapezoid rule in y);
 *   out[2] = free energy: bending, SM eq. (30) without the area term,
 *            3 sqrt(2) kappa/(8 eps^3) int g^2; Cahn-Hilliard, eq. F_CH,
 *            int 1/4 (phi^2 - 1)^2 + (sigma/2) |grad phi|^2;
 *   out[3] = max sigma_t;
 *   out[4] = gauge defect int (div psi)^2 over the interior rows, central differences (the
 *            Coulomb gauge div psi = 0 is assumed, not imposed: main text after eq. (7));
 *   out[5] = max |v| over the nodes (curl psi inside, the wall speed on the walls).
 * sigma_t: device, nx*ny*nz doubles, or NULL: the in-plane shear-stress intensity of the
 * section "In plane shear", sqrt(s_xy^2 + s_yz^2 + s_xz^2) with s_ij = eta (d_j v_i + d_i v_j)
 * by central differences of v (curl psi inside, the wall speed on the walls), on the interior
 * rows; 0 on the wall rows. */
vs_status vs_diagnostics(vs_state* state, double* sigma_t, double out[6]);

/* Byte offset, inside the workspace, of field `field` (VS_PHI ... VS_PSI_Z) as it stands
 * now (phi moves between two buffers from step to step: query after each vs_step). */
vs_status vs_field_offset(const vs_state* state, int32_t field, size_t* byte_offset);

/* Copy the VS_NSCALARS global scalars (slots VS_S_*) to host memory `out`. Synchronises. */
vs_status vs_get_scalars(vs_state* state, double out[VS_NSCALARS]);

/* The per-step log: the device appends one record (VS_L_* fields) per time step, written by
 * the step's final flow check (and one for the initial solve of vs_init), in every mode, single
 * states and batches alike. The last VS_LOG_CAP records are kept. vs_log_read copies the
 * most recent min(cap, kept) records, oldest first, to host memory out (cap * VS_LOG_FIELDS
 * doubles) and sets *n to their count. Synchronises. With the environment variable VS_LOG set
 * (to anything), vs_step prints the records of its steps to stderr, one line per step. */
vs_status vs_log_read(vs_state* state, double* out, int32_t cap, int32_t* n);

/* Checkpoint: write phi, mu, omega, psi, the scalars, the wall speeds and the step count into
 * blob, which may be host memory or device memory (device allocations are detected; then the
 * fields are copied device to device, so a rollout can keep its checkpoints in HBM). With
 * blob == NULL only *bytes is set to the size needed. Synchronises. */
vs_status vs_save_state(vs_state* state, void* blob, size_t* bytes);
/* Restore a checkpoint written by vs_save_state for the same grid and wall kind, from host or
 * device memory. In VS_FP32_REFINED the time extrapolation of the flow fields starts over (the
 * next steps may take more cycles; the fields agree with an uninterrupted run to within the
 * solve tolerance, not bit for bit). Synchronises. */
vs_status vs_load_state(vs_state* state, const void* blob, size_t bytes);

/* Per-kernel timing with HIP events on the state's stream, for measurement tools:
 * vs_profile(state, 1) starts recording an event pair around every kernel launch,
 * vs_profile(state, 0) stops, vs_profile_read returns, for kernel class `kernel`
 * (0 <= kernel < vs_profile_count()), the summed duration in ms and the launch count since
 * the last vs_profile(state, 1). vs_profile_name gives the class name. */
vs_status vs_profile(vs_state* state, int32_t enable);
int32_t vs_profile_count(void);
const char* vs_profile_name(int32_t kernel);
vs_status vs_profile_read(vs_state* state, int32_t kernel, double* total_ms, int64_t* launches);

/* Launch-shape autotuner. Times, on the state's own data, the candidate launch shapes of its
 * grid: the x-slab length of the phi update (2, 4, 8 planes per lane), the block caps of the
 * volume/area partials (256 .. 2048) and of the flow residual (512 .. 4096), the form of the
 * chemical potential (LDS tiles, or for nz in {64, 128, 256} register marching with 1 or 2
 * rows per wave and 2 .. 16 planes per slab; all forms give the same bits) and, for
 * ny - 2 in {30, 46, 62, 94, 126, 254}, the segment layout of the tridiagonal solves (the
 * default or one with twice/half the lanes per mode) and, in FP64 with nx = nz in
 * {32, 48, 64, 96, 128}, whether the x and z transforms of a direction run as one pass over
 * each (x, z) plane held in LDS (plane = 1) or as two line passes (0), one coordinate at a
 * time, and keeps the fastest for every state of that grid in this process. The state's fields
 * are not changed. picked (may be NULL): adv_slab, va_maxb, res_maxb, seg_alt, mu_kind, mu_ni,
 * plane. Synchronises. */
vs_status vs_autotune(vs_state* state, int32_t picked[7]);
/* Set the launch shapes of a grid by hand (the seven values vs_autotune reports, e.g. from an
 * earlier tuning run), for every state of that grid in this process from the next launch on.
 * Shapes that the grid cannot use fall back to the default form (the register-marching
 * chemical potential needs nz in {64, 128, 256}; seg_alt needs ny - 2 in the list above).
 * Checks ranges only; results are unchanged except in the order of the partial sums and, with
 * plane = 1, in the rounding of the z transforms (their rows are paired differently). */
vs_status vs_set_launch_shapes(const vs_grid* grid, const int32_t shapes[7]);

/* Batches (many independent instances, e.g. vesicles of different grids and parameters,
 * stepped together: one launch per kernel and grid class instead of one persistent launch).
 * vs_batch_create groups n states made by vs_init (each keeps its own workspace) into grid
 * classes (same grid, precision, model and poisson_max_cycles): every kernel of a time step
 * is launched once per class, each instance's pointers and parameters read from a device
 * table of argument structs (allocated by the batch: a few KB per instance). Grids of a class
 * not tuned yet are tuned first (vs_autotune on the class's first instance; for an FP64
 * class, a grid tuned only by FP32-refined states is tuned again, since its transform form
 * was left at the default). Instances outside the fused forms (FP64 with
 * poisson_max_cycles > 1) are stepped one by one. It creates min(nstreams, groups) HIP
 * streams (groups: the classes, plus one for those instances; group g runs on stream
 * g % nstreams) and moves every state onto its stream; `stream` (a hipStream_t, NULL =
 * default) is the origin the batch forks from and joins to. vs_batch_step captures two time
 * steps of every class into one HIP graph (redone when a dt or a wall speed changes) and
 * replays it nsteps/2 times on the origin stream. nsteps must be even. dt: host array of n
 * time steps. Each instance is checked against its stability bound first; statuses are
 * collected after one synchronisation (the first failing instance's status is returned).
 * Results are bitwise those of stepping each instance alone. vs_batch_destroy frees the batch
 * and moves the states back to the origin stream; the states stay valid and are destroyed by
 * vs_destroy. A state belongs to at most one batch; do not call vs_step on it while the batch
 * exists. */
typedef struct vs_batch vs_batch;
vs_status vs_batch_create(vs_state* const* states, int32_t n, void* stream, int32_t nstreams,
                          vs_batch** out);
vs_status vs_batch_step(vs_batch* batch, const double* dt, int32_t nsteps);
void vs_batch_destroy(vs_batch* batch);

/* Free the host-side state (the workspace stays the caller's). NULL is ignored. */
void vs_destroy(vs_state* state);

/* Message of the calling thread's last failed call ("" if none). */
const char* vs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VS_H */
