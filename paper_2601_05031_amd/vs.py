"""ctypes binding of libvs (include/vs.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libvs. PyTorch provides the device
workspace (one uint8 tensor) and the HIP stream; fields are exposed as torch views into the
workspace. If libvs.so has not been built, loading fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvs.so")

# status codes
VS_OK = 0
VS_E_ARG = -1
VS_E_WORKSPACE = -2
VS_E_HIP = -3
VS_E_NOCONV = -4
VS_E_NONFINITE = -5
VS_E_UNSTABLE = -6
VS_E_STATE = -7
VS_E_UNSUPPORTED = -8
STATUS_NAMES = {0: "VS_OK", -1: "VS_E_ARG", -2: "VS_E_WORKSPACE", -3: "VS_E_HIP", -4: "VS_E_NOCONV",
                -5: "VS_E_NONFINITE", -6: "VS_E_UNSTABLE", -7: "VS_E_STATE", -8: "VS_E_UNSUPPORTED"}

VS_POISEUILLE, VS_COUETTE = 1, 2
VS_BENDING, VS_CAHN_HILLIARD = 1, 2
VS_FP64, VS_FP32_REFINED = 1, 2
VS_ALLOW_UNSTABLE = 1

FIELDS = {"phi": 0, "mu": 1, "omega_x": 2, "omega_y": 3, "omega_z": 4, "psi_x": 5, "psi_y": 6, "psi_z": 7}
SCALARS = ["V", "A", "V0", "A0", "lambda_V", "gamma_A", "relres", "step", "cycles"]
LOG_FIELDS = ["index", "cycles", "relres", "V", "A", "lambda_V", "gamma_A", "conv"]
VS_LOG_CAP = 4096

_WALL_KINDS = {"poiseuille": VS_POISEUILLE, "couette": VS_COUETTE}
_MODELS = {"bending": VS_BENDING, "cahn_hilliard": VS_CAHN_HILLIARD}
_PRECISIONS = {"fp64": VS_FP64, "fp32_refined": VS_FP32_REFINED}


class VsGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double)]


class VsWalls(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("u0", ctypes.c_double), ("u1", ctypes.c_double)]


class VsParams(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("eta", ctypes.c_double), ("mobility", ctypes.c_double), ("eps", ctypes.c_double),
                ("kappa", ctypes.c_double), ("sigma", ctypes.c_double), ("gamma0", ctypes.c_double),
                ("rate_V", ctypes.c_double), ("k_A", ctypes.c_double),
                ("bend_scale", ctypes.c_double), ("poisson_rtol", ctypes.c_double),
                ("poisson_max_cycles", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("rho", ctypes.c_double)]


class VsError(RuntimeError):
    def __init__(self, code: int, call: str, message: str):
        self.code = code
        self.call = call
        super().__init__(f"{call}: {STATUS_NAMES.get(code, code)}: {message}")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libvs.so from the package directory (built by paper_2601_05031_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_05031_amd.build`")
    # PyTorch provides the device memory and streams, and ships its own HIP runtime (soname
    # libamdhip64.so.7, loaded by its libraries under another name). Loaded first, that runtime
    # also serves libvs; loaded after libvs, it would be a second runtime beside the system one
    # and the first of them to be used does not see the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, sz, i32, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    sigs = {
        "vs_workspace_bytes": (i32, [P(VsGrid), P(VsParams), P(sz)]),
        "vs_init": (i32, [P(VsGrid), P(VsWalls), P(VsParams), vp, vp, sz, vp, P(vp)]),
        "vs_poisson_solve": (i32, [vp, vp, vp, dbl, i32, P(i32), P(dbl)]),
        "vs_poisson_solve_noalloc": (i32, [P(VsGrid), vp, vp, dbl, i32, vp, P(i32), P(dbl)]),
        "vs_noalloc_scratch_bytes": (sz, []),
        "vs_step": (i32, [vp, dbl, i32]),
        "vs_grad_step": (i32, [vp, dbl, vp, vp, P(dbl)]),
        "vs_field_offset": (i32, [vp, i32, P(sz)]),
        "vs_get_scalars": (i32, [vp, P(dbl)]),
        "vs_log_read": (i32, [vp, P(dbl), i32, P(i32)]),
        "vs_save_state": (i32, [vp, vp, P(sz)]),
        "vs_load_state": (i32, [vp, vp, sz]),
        "vs_profile": (i32, [vp, i32]),
        "vs_profile_count": (i32, []),
        "vs_profile_name": (ctypes.c_char_p, [i32]),
        "vs_profile_read": (i32, [vp, i32, P(dbl), P(ctypes.c_int64)]),
        "vs_destroy": (None, [vp]),
        "vs_set_walls": (i32, [vp, P(VsWalls)]),
        "vs_diagnostics": (i32, [vp, vp, P(dbl)]),
        "vs_autotune": (i32, [vp, P(i32)]),
        "vs_set_launch_shapes": (i32, [P(VsGrid), P(i32)]),
        "vs_batch_create": (i32, [P(vp), i32, vp, i32, P(vp)]),
        "vs_batch_step": (i32, [vp, P(dbl), i32]),
        "vs_batch_destroy": (None, [vp]),
        "vs_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code: int, call: str):
    if code != VS_OK:
        raise VsError(code, call, lib().vs_last_error().decode())


def make_params(model="bending", precision="fp64", eta=1.0, mobility=1.0, eps=1.0, kappa=1.0,
                sigma=1.0, gamma0=0.0, rate_V=0.0, k_A=0.0, bend_scale=1.0, rtol=1e-10,
                max_cycles=3, allow_unstable=False, rho=0.0) -> VsParams:
    return VsParams(_MODELS[model], _PRECISIONS[precision], eta, mobility, eps, kappa, sigma,
                    gamma0, rate_V, k_A, bend_scale, rtol, max_cycles,
                    VS_ALLOW_UNSTABLE if allow_unstable else 0, rho)


def workspace_bytes(grid, params: VsParams) -> int:
    g = VsGrid(*grid) if not isinstance(grid, VsGrid) else grid
    n = ctypes.c_size_t(0)
    _check(lib().vs_workspace_bytes(ctypes.byref(g), ctypes.byref(params), ctypes.byref(n)),
           "vs_workspace_bytes")
    return n.value


SHAPE_KEYS = ("adv_slab", "va_maxb", "res_maxb", "seg_alt", "mu_kind", "mu_ni", "plane")


def set_launch_shapes(grid, shapes: dict):
    """vs_set_launch_shapes: launch shapes for every state of this grid (nx, ny, nz[, h])."""
    g = VsGrid(grid[0], grid[1], grid[2], float(grid[3]) if len(grid) > 3 else 1.0)
    arr = (ctypes.c_int32 * 7)(*[int(shapes[k]) for k in SHAPE_KEYS])
    _check(lib().vs_set_launch_shapes(ctypes.byref(g), arr), "vs_set_launch_shapes")


def noalloc_scratch_bytes() -> int:
    return int(lib().vs_noalloc_scratch_bytes())


def poisson_solve_noalloc(f, u, h=1.0, rtol=1e-10, max_cycles=3, stream=None):
    """vs_poisson_solve_noalloc: solve L_h u = f in place in the float64 CUDA tensor u (walls
    held fixed) with the library's static scratch; no workspace, no state. Returns (code,
    cycles, relres); codes other than VS_OK and VS_E_NOCONV raise."""
    import torch

    for t in (f, u):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.dim() != 3:
            raise ValueError("f and u must be contiguous 3-d float64 tensors")
    if tuple(f.shape) != tuple(u.shape):
        raise ValueError("f and u must have the same shape")
    g = VsGrid(int(u.shape[0]), int(u.shape[1]), int(u.shape[2]), float(h))
    if stream is None:
        stream = torch.cuda.current_stream(u.device)
    cyc = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    code = lib().vs_poisson_solve_noalloc(ctypes.byref(g), ctypes.c_void_p(f.data_ptr()),
                                          ctypes.c_void_p(u.data_ptr()), float(rtol),
                                          int(max_cycles), ctypes.c_void_p(stream.cuda_stream),
                                          ctypes.byref(cyc), ctypes.byref(rel))
    if code not in (VS_OK, VS_E_NOCONV):
        _check(code, "vs_poisson_solve_noalloc")
    return code, cyc.value, rel.value


class Solver:
    """One simulation on one GPU: owns a torch workspace tensor and a vs_state."""

    def __init__(self, grid, walls: dict, params: dict, phi0, device="cuda:0", stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.grid = VsGrid(grid[0], grid[1], grid[2], float(grid[3]) if len(grid) > 3 else 1.0)
        self.walls = VsWalls(_WALL_KINDS[walls["kind"]], float(walls["u0"]), float(walls.get("u1", 0.0)))
        p = dict(params)
        self.params = make_params(**p)
        nbytes = workspace_bytes(self.grid, self.params)
        # 256 bytes of slack so the base can be aligned whatever the allocator returns
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._pad = (-base) % 256
        self.ws_ptr = base + self._pad
        self.ws_bytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        phi0_t = torch.as_tensor(phi0, dtype=torch.float64).to(self.device).contiguous()
        shape = (self.grid.nx, self.grid.ny, self.grid.nz)
        if tuple(phi0_t.shape) != shape:
            raise ValueError(f"phi0 has shape {tuple(phi0_t.shape)}, grid is {shape}")
        torch.cuda.current_stream(self.device).synchronize()
        st = ctypes.c_void_p(0)
        _check(lib().vs_init(ctypes.byref(self.grid), ctypes.byref(self.walls), ctypes.byref(self.params),
                             ctypes.c_void_p(phi0_t.data_ptr()), ctypes.c_void_p(self.ws_ptr),
                             ctypes.c_size_t(nbytes), ctypes.c_void_p(self.stream.cuda_stream),
                             ctypes.byref(st)), "vs_init")
        self._st = st
        self.shape = shape

    # ------------------------------------------------------------------ core calls
    def step(self, dt: float, nsteps: int = 1):
        _check(lib().vs_step(self._st, float(dt), int(nsteps)), "vs_step")

    def poisson_solve(self, f, u, rtol=1e-10, max_cycles=3):
        """Solve L_h u = f in place in the torch float64 tensor u (walls held fixed)."""
        cyc = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        for t in (f, u):
            if t.dtype != self.torch.float64 or not t.is_contiguous() or tuple(t.shape) != self.shape:
                raise ValueError("f and u must be contiguous float64 tensors of the grid shape")
        code = lib().vs_poisson_solve(self._st, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                      float(rtol), int(max_cycles), ctypes.byref(cyc), ctypes.byref(rel))
        if code not in (VS_OK, VS_E_NOCONV):
            _check(code, "vs_poisson_solve")
        return code, cyc.value, rel.value

    def grad_step(self, dt, adj_next, adj_prev):
        """Reverse step at the state's level n: adj_prev = (d phi^{n+1}/d phi^n)^T adj_next;
        returns this step's (dL/dkappa, dL/ds) terms (s scales the wall speeds)."""
        for t in (adj_next, adj_prev):
            if t.dtype != self.torch.float64 or not t.is_contiguous() or tuple(t.shape) != self.shape:
                raise ValueError("adjoints must be contiguous float64 tensors of the grid shape")
        dp = (ctypes.c_double * 2)()
        _check(lib().vs_grad_step(self._st, float(dt), ctypes.c_void_p(adj_next.data_ptr()),
                                  ctypes.c_void_p(adj_prev.data_ptr()), dp), "vs_grad_step")
        return dp[0], dp[1]

    def field(self, name: str):
        """Torch float64 view of a field inside the workspace (valid until the next step)."""
        off = ctypes.c_size_t(0)
        _check(lib().vs_field_offset(self._st, FIELDS[name], ctypes.byref(off)), "vs_field_offset")
        n = self.shape[0] * self.shape[1] * self.shape[2]
        start = self._pad + off.value
        if name == "mu" and self.params.precision == VS_FP32_REFINED:
            # the refined mode keeps mu as FP32 (include/vs.h)
            return self._ws[start:start + 4 * n].view(self.torch.float32).view(*self.shape)
        return self._ws[start:start + 8 * n].view(self.torch.float64).view(*self.shape)

    def fields(self):
        """Every field as a float64 numpy array."""
        return {k: self.field(k).double().cpu().numpy() for k in FIELDS}

    def scalars(self) -> dict:
        out = (ctypes.c_double * len(SCALARS))()
        _check(lib().vs_get_scalars(self._st, out), "vs_get_scalars")
        return dict(zip(SCALARS, list(out)))

    def log(self, cap: int = VS_LOG_CAP):
        """The per-step log (vs_log_read): up to cap most recent records, oldest first, as an
        array of shape (n, len(LOG_FIELDS))."""
        import numpy as np
        out = (ctypes.c_double * (cap * len(LOG_FIELDS)))()
        n = ctypes.c_int32(0)
        _check(lib().vs_log_read(self._st, out, cap, ctypes.byref(n)), "vs_log_read")
        return np.frombuffer(out, dtype=np.float64, count=n.value * len(LOG_FIELDS)).reshape(
            n.value, len(LOG_FIELDS)).copy()

    def set_walls(self, u0: float, u1: float = 0.0):
        """New wall speeds (same kind) from now on: the time-dependent-walls hook."""
        w = VsWalls(self.walls.kind, float(u0), float(u1))
        _check(lib().vs_set_walls(self._st, ctypes.byref(w)), "vs_set_walls")
        self.walls = w

    def diagnostics(self, sigma_t=None) -> dict:
        """Observables, free energy and max shear-stress intensity; fills sigma_t (a float64
        tensor of the grid shape) with the shear-stress intensity if given."""
        if sigma_t is not None and (sigma_t.dtype != self.torch.float64 or not sigma_t.is_contiguous()
                                    or tuple(sigma_t.shape) != self.shape):
            raise ValueError("sigma_t must be a contiguous float64 tensor of the grid shape")
        out = (ctypes.c_double * 6)()
        ptr = ctypes.c_void_p(sigma_t.data_ptr()) if sigma_t is not None else None
        _check(lib().vs_diagnostics(self._st, ptr, out), "vs_diagnostics")
        return {"obs_omega": out[0], "obs_psi": out[1], "energy": out[2], "sigma_t_max": out[3],
                "gauge_defect": out[4], "speed_max": out[5]}

    def save(self, device: bool = False):
        """Checkpoint as bytes (host), or as a uint8 tensor on the solver's device."""
        n = ctypes.c_size_t(0)
        _check(lib().vs_save_state(self._st, None, ctypes.byref(n)), "vs_save_state")
        if device:
            blob = self.torch.empty(n.value, dtype=self.torch.uint8, device=self._ws.device)
            _check(lib().vs_save_state(self._st, ctypes.c_void_p(blob.data_ptr()), ctypes.byref(n)),
                   "vs_save_state")
            return blob
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().vs_save_state(self._st, buf, ctypes.byref(n)), "vs_save_state")
        return buf.raw

    def load(self, blob):
        """Restore a checkpoint from save(): bytes, or a device uint8 tensor."""
        if isinstance(blob, (bytes, bytearray)):
            _check(lib().vs_load_state(self._st, bytes(blob), len(blob)), "vs_load_state")
            return
        if blob.dtype != self.torch.uint8 or not blob.is_contiguous():
            raise ValueError("a device checkpoint is a contiguous uint8 tensor from save(device=True)")
        _check(lib().vs_load_state(self._st, ctypes.c_void_p(blob.data_ptr()), blob.numel()),
               "vs_load_state")

    # ---------------------------------------------------------------- measurement
    def autotune(self) -> dict:
        """vs_autotune: pick this grid's launch shapes by timing them on this state's data."""
        out = (ctypes.c_int32 * 7)()
        _check(lib().vs_autotune(self._st, out), "vs_autotune")
        return dict(zip(SHAPE_KEYS, list(out)))

    def profile(self, on: bool):
        _check(lib().vs_profile(self._st, 1 if on else 0), "vs_profile")

    def profile_read(self) -> dict:
        res = {}
        for k in range(lib().vs_profile_count()):
            ms = ctypes.c_double(0.0)
            n = ctypes.c_int64(0)
            _check(lib().vs_profile_read(self._st, k, ctypes.byref(ms), ctypes.byref(n)), "vs_profile_read")
            res[lib().vs_profile_name(k).decode()] = (ms.value, n.value)
        return res

    def close(self):
        if getattr(self, "_st", None):
            lib().vs_destroy(self._st)
            self._st = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many Solvers stepped together: their steps are captured into one HIP graph (each
    instance on its own stream, forked from and joined to the origin stream) and replayed."""

    def __init__(self, solvers, nstreams=8, stream=None):
        import torch

        self.solvers = list(solvers)
        n = len(self.solvers)
        origin = stream if stream is not None else torch.cuda.current_stream()
        arr = (ctypes.c_void_p * n)(*[s._st for s in self.solvers])
        b = ctypes.c_void_p(0)
        _check(lib().vs_batch_create(arr, n, ctypes.c_void_p(origin.cuda_stream), int(nstreams),
                                     ctypes.byref(b)), "vs_batch_create")
        self._b = b

    def step(self, dts, nsteps: int):
        n = len(self.solvers)
        if not hasattr(dts, "__len__"):
            dts = [dts] * n
        arr = (ctypes.c_double * n)(*[float(x) for x in dts])
        _check(lib().vs_batch_step(self._b, arr, int(nsteps)), "vs_batch_step")

    def close(self):
        if getattr(self, "_b", None):
            lib().vs_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rollout_gradient(solver: "Solver", dt: float, nsteps: int, target, checkpoint_every: int = 10):
    """L = ||phi^N - target||^2 (sum over nodes) of an nsteps rollout from the solver's current
    state, and (L, dL/dkappa, dL/ds, dL/dphi^0 with V0, A0 fixed). The forward pass keeps a
    vs_save_state checkpoint every checkpoint_every steps; the reverse sweep reloads the nearest
    checkpoint and recomputes forward to each level (bit-identical to the first pass) before
    its vs_grad_step. The solver is left at the initial state."""
    torch = solver.torch
    ce = max(1, int(checkpoint_every))
    ckpt = {0: solver.save(device=True)}   # checkpoints stay in HBM
    for n in range(nsteps):
        solver.step(dt, 1)
        if (n + 1) % ce == 0:
            ckpt[n + 1] = solver.save(device=True)
    r = solver.field("phi") - target
    loss = float((r * r).sum())
    a = (2.0 * r).contiguous()
    b = torch.empty_like(a)
    kb = sb = 0.0
    for n in range(nsteps - 1, -1, -1):
        base = max(k for k in ckpt if k <= n)
        solver.load(ckpt[base])
        if n > base:
            solver.step(dt, n - base)
        dk, ds = solver.grad_step(dt, a, b)
        kb += dk
        sb += ds
        a, b = b, a
    solver.load(ckpt[0])
    return loss, kb, sb, a


def rollout_loss(workload, kappa, scale, target, nsteps=None, checkpoint_every=10, device="cuda:0"):
    """torch.autograd.Function form of rollout_gradient: kappa and scale are 0-d float64 CPU
    tensors (the bending modulus and the wall-speed scale); returns the loss as a 0-d tensor
    whose backward gives dL/dkappa and dL/dscale."""
    import torch

    class _Rollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, k, sc):
            w = workload.with_(kappa=float(k), u0=float(sc) * workload.u0, u1=float(sc) * workload.u1)
            sol = solver_for(w, device=device)
            try:
                L, kb, sb, _ = rollout_gradient(sol, w.dt, nsteps or w.nsteps, target, checkpoint_every)
            finally:
                sol.close()
            # dL/dscale: s scales the walls of w, whose speeds are scale * u; d/dscale = (1/scale) d/ds
            ctx.save_for_backward(torch.tensor([kb, sb / float(sc)], dtype=torch.float64))
            return torch.tensor(L, dtype=torch.float64)

        @staticmethod
        def backward(ctx, g):
            (gr,) = ctx.saved_tensors
            return g * gr[0], g * gr[1]

    return _Rollout.apply(kappa, scale)


def solver_for(workload, device="cuda:0", precision="fp64", phi0=None, **overrides) -> "Solver":
    """Build a Solver from a workloads.Workload (its seeded phi0 unless one is given)."""
    w = workload.with_(**overrides) if overrides else workload
    p = w.params()
    rtol = p.pop("rtol")
    mc = p.pop("max_cycles")
    return Solver((w.grid.nx, w.grid.ny, w.grid.nz, w.grid.h), w.walls(),
                  dict(p, rtol=rtol, max_cycles=mc, precision=precision),
                  w.phi0() if phi0 is None else phi0, device=device)
