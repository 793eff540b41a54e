"""Benchmark of the FP64 time step on one MI355X.

Workload (vesicle128): 128^3 grid, plane Poiseuille channel (centreline 0.05, walls at y = 0
and y = 127), prolate vesicle of area-equivalent radius 24 and reduced volume 0.8, bending
with volume/area penalties, dt = 5e-4. One benchmark step advances three instances, kappa =
0.5, 1 and 2, by one time step each (three full passes of the hot path: phi update, mu,
vorticity solve, stream-vector solve). Inputs are resident in HBM before the timed region.

Prints one JSON line. `value` is cell-updates/s over the timed steps; `roofline` is the
dominant kernel's algorithmic bytes per launch over its mean event-timed duration, against
the 8 TB/s HBM peak; `cpu_baseline` is the CPU oracle on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s & steps/s at 128³: FP64 vs FP32-refined vs batched; % HBM peak"
HBM_PEAK_GBS = 8000.0
KAPPAS = (0.5, 1.0, 2.0)


def kernel_bytes(name: str, nx: int, ny: int, nz: int) -> float | None:
    """Algorithmic HBM bytes of one launch: each input read once, each output written once
    (FP64). Ni counts the interior rows the Poisson kernels touch. The two Poisson right-hand
    sides differ (vorticity: phi, mu; stream vector: omega); their kernels are timed apart."""
    N = nx * ny * nz
    Ni = nx * (ny - 2) * nz
    table = {
        "advance": 48 * N,            # phi, mu, psi_x, psi_y, psi_z in; phi' out
        "va_partials": 8 * N,         # phi in
        "mu": 16 * N,                 # phi in; mu out
        "source": 16 * N + 24 * Ni,   # phi, mu in; S(3) out on the interior rows
        "rhs_dht_z_omega": 48 * Ni,   # S(3) in; 3 spectral fields out
        "rhs_dht_z_psi": 48 * Ni,     # omega(3) in; 3 spectral fields out
        "dht_x": 48 * Ni,             # 3 spectral fields in and out
        "tridiag_y": 48 * Ni,         # 3 spectral fields in and out
        "tridiag_pair": 72 * Ni,      # source modes in; vorticity and stream-vector modes out
        "dht_z_out": 48 * Ni,         # 3 spectral fields in; 3 solution fields out
        "dht_x_pair": 96 * Ni,        # omega and psi modes (6 fields) in and out
        "dht_z_out_pair": 96 * Ni,    # 6 spectral fields in; omega(3), psi(3) out
        "resid_norm_omega": 48 * Ni,  # S(3), omega(3) in
        "resid_norm_psi": 48 * Ni,    # omega(3), psi(3) in
        "resid_norm_flow": 72 * Ni,   # omega(3), S(3), psi(3) in: both flow residuals
        "dht_zx": 48 * Ni,            # plane form: S(3) in; 3 spectral fields out
        "dht_xz_pair": 96 * Ni,       # plane form: 6 spectral fields in; omega(3), psi(3) out
    }
    return table.get(name)


def code_tokens(src: str) -> str:
    """C++ source without comments, whitespace runs collapsed: what the compiler sees."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def source_hash(kernel: str) -> str:
    """Hash of the code (comments aside) of the source files that hold a kernel, to tie
    stored counters to the code they were taken on."""
    names = (["k_explicit.hip", "stencil.h"] if kernel in ("advance", "va_partials", "mu", "source")
             else ["k_spectral.hip", "k_solve.hip", "spectral.h", "fft_reg.h", "flow_check.h"])
    h = hashlib.sha256()
    for fname in names:
        with open(os.path.join(ROOT, "paper_2601_05031_amd", "csrc", fname)) as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was taken on the
    current source of that kernel; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"source_sha256_16:\s*(\w+)", txt)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_b or m_hash.group(1) != source_hash(kernel):
        return None
    return float(m_b.group(1))


def _oracle_steps(budget_s: float):
    """The CPU oracle on the vesicle128 workload (kappa = 1): init, then as many steps as fit in
    about budget_s seconds (at least 2), on one thread. Returns (steps, seconds)."""
    import oracle as O
    from workloads import workload

    w = workload("vesicle128")
    g = O.Grid(*w.grid.shape, h=w.grid.h)
    walls = O.Walls(w.wall_kind, w.u0, w.u1)
    p = O.Params(model=w.model, eta=w.eta, mobility=w.mobility, eps=w.eps, kappa=1.0,
                 sigma=w.sigma, gamma0=w.gamma0, rate_V=w.rate_V, k_A=w.k_A, bend_scale=w.bend_scale)
    s = O.init_state(g, walls, p, w.phi0())
    # one thread: scipy.fft runs with one worker by default; BLAS/OpenMP pools are held to one
    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(1)
    except ImportError:
        limit = None
    t0 = time.perf_counter()
    n = 0
    while n < 2 or (time.perf_counter() - t0) < budget_s:
        s = O.step(s, w.dt, g, walls, p)
        n += 1
    t = time.perf_counter() - t0
    if limit is not None:
        limit.restore_original_limits()
    return n, t


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(workload, budget_s: float, all_cores: bool = True):
    """The CPU oracle (numpy/scipy FP64, one thread per process) on the same 128^3 workload:
    first one process alone, then one process per host core, each stepping its own copy of
    the workload (started as CPU-only copies of this script, `--cpu-worker`), aggregate
    throughput. `value` is the all-core figure; the single-thread one is kept beside it."""
    import subprocess

    N = workload.grid.N
    n1, t1 = _oracle_steps(budget_s)
    single = {"value": N * n1 / t1, "steps_per_s": n1 / t1, "cores": 1,
              "sample": f"{n1} time steps in {t1:.1f} s"}
    out = {"value": single["value"], "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
           "sample": f"{workload.name} kappa=1, 128x128x128 after init, numpy/scipy FP64 "
                     f"(one thread per process): {single['sample']}",
           "single_thread": single}
    ncore = host_cores()
    if not all_cores or ncore < 2:
        return out
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", str(budget_s)]
    procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=env,
                              text=True) for _ in range(ncore)]
    steps, secs = 0, 0.0
    for pr in procs:
        o, _ = pr.communicate(timeout=30 * budget_s + 300)
        r = json.loads(o.strip().splitlines()[-1])
        steps += r["steps"]
        secs = max(secs, r["seconds"])
    out.update({"value": N * steps / secs, "cores": ncore, "steps_per_s": steps / secs,
                "sample": f"{workload.name} kappa=1, 128x128x128 after init, numpy/scipy FP64, "
                          f"{ncore} processes of one thread each ({steps} time steps, slowest "
                          f"process {secs:.1f} s); one process alone: {single['sample']}"})
    return out


def compare_precisions(P, torch, steps: int) -> dict:
    """droplet256 (128 x 128 x 256 Cahn-Hilliard droplet in Couette flow): the same steps in
    FP64 and in the FP32-refined mode (FP32-stored spectral solves, FP64 defect correction to
    the same rtol), timed alike; the refined fields are compared with the FP64 ones."""
    from workloads import workload

    w = workload("droplet256", max_cycles=1)
    N = w.grid.N
    out = {"workload": w.name, "grid": list(w.grid.shape), "steps": steps, "poisson_rtol": w.rtol}
    fields = {}
    for prec, mc in (("fp64", 1), ("fp32_refined", 2)):
        s = P.solver_for(w, precision=prec, max_cycles=mc)
        s.step(w.dt, 3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(w.dt, steps)
        t = time.perf_counter() - t0
        sc = s.scalars()
        fields[prec] = s.fields()
        out[prec] = {"cell_updates_per_s": N * steps / t, "ms_per_step": 1e3 * t / steps,
                     "max_relres": sc["relres"], "cycles_per_solve": sc["cycles"] / (2.0 * steps)}
        s.close()
        del s
        torch.cuda.empty_cache()
    import numpy as np

    errs = {}
    for k, ref in fields["fp64"].items():
        nb = float(np.linalg.norm(ref))
        errs[k] = float(np.linalg.norm(fields["fp32_refined"][k] - ref)) / (nb if nb > 0 else 1.0)
    out["fp32_refined_rel_l2_vs_fp64"] = errs
    out["speedup_fp32_refined_over_fp64"] = (out["fp32_refined"]["cell_updates_per_s"]
                                             / out["fp64"]["cell_updates_per_s"])
    print(f"bench: droplet256 fp64 {out['fp64']['ms_per_step']:.3f} ms/step, fp32-refined "
          f"{out['fp32_refined']['ms_per_step']:.3f} ms/step "
          f"({out['fp32_refined']['cycles_per_solve']:.2f} cycles/solve), max field error "
          f"{max(errs.values()):.2e}", file=sys.stderr, flush=True)
    return out


def batched_run(P, torch, steps: int, nstreams: int) -> dict:
    """The 64-instance batch (grids drawn from 48^3..128^3, instance i seeded with 1000 + i):
    every instance advanced `steps` time steps through one captured HIP graph per two steps,
    against the same instances stepped one after another with vs_step."""
    from collections import Counter

    from workloads import batch_instances

    ws = batch_instances(64)
    t0 = time.perf_counter()
    phis = [w.phi0() for w in ws]
    print(f"bench: batch seed shapes built in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    cells = sum(w.grid.N for w in ws)
    dts = [w.dt for w in ws]
    out = {"workload": "batch64", "instances": len(ws), "steps": steps, "streams": nstreams,
           "grids": {f"{n}^3": c for n, c in sorted(Counter(w.grid.nx for w in ws).items())},
           "cells_per_batch_step": cells, "poisson_rtol": ws[0].rtol}
    for prec, mc in (("fp32_refined", 2), ("fp64", 1)):
        solvers = [P.solver_for(w, precision=prec, max_cycles=mc, phi0=phi) for w, phi in zip(ws, phis)]
        b = P.Batch(solvers, nstreams=nstreams)
        b.step(dts, 2)                        # capture + first replay, untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(dts, steps)
        tb = time.perf_counter() - t0
        b.close()
        sc = [s.scalars() for s in solvers]
        for s, dt in zip(solvers, dts):       # the same work, one instance after another
            s.step(dt, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, dt in zip(solvers, dts):
            s.step(dt, steps)
        ts = time.perf_counter() - t0
        out[prec] = {"cell_updates_per_s": cells * steps / tb, "ms_per_batch_step": 1e3 * tb / steps,
                     "instance_steps_per_s": len(ws) * steps / tb,
                     "sequential_cell_updates_per_s": cells * steps / ts,
                     "speedup_over_sequential": ts / tb,
                     "max_relres": max(x["relres"] for x in sc),
                     "cycles_per_solve": sum(x["cycles"] for x in sc) / (2.0 * steps * len(ws)),
                     "poisson_max_cycles": mc}
        print(f"bench: batch64 {prec}: {1e3 * tb / steps:.2f} ms/batch step "
              f"({cells * steps / tb:.3e} cell-updates/s), sequential {1e3 * ts / steps:.2f} ms",
              file=sys.stderr, flush=True)
        # each grid class alone as a batch: the per-cell rate of the class's kernels
        per = {}
        for n in sorted({w.grid.nx for w in ws}):
            sel = [s for s, w in zip(solvers, ws) if w.grid.nx == n]
            dsel = [dt for dt, w in zip(dts, ws) if w.grid.nx == n]
            bc = P.Batch(sel, nstreams=nstreams)
            bc.step(dsel, 2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bc.step(dsel, steps)
            tc = time.perf_counter() - t0
            bc.close()
            per[f"{n}^3"] = {"instances": len(sel),
                             "cell_updates_per_s": sum(x.grid.N for x in ws if x.grid.nx == n) * steps / tc}
        out[prec]["per_class"] = per
        print(f"bench: batch64 {prec} per class: " +
              ", ".join(f"{k} {v['cell_updates_per_s']:.3e}" for k, v in per.items()),
              file=sys.stderr, flush=True)
        for s in solvers:
            s.close()
        del solvers, b
        torch.cuda.empty_cache()
    return out


def adjoint_run(P, torch, nsteps: int, checkpoint_every: int = 10) -> dict:
    """The 96^3 differentiation workload: a rollout gradient (forward with vs_save_state
    checkpoints, then in reverse: reload, recompute to the level, vs_grad_step) of
    L = ||phi^n - target||^2, target from kappa = 1.5 and 1.2 times the wall speed; and
    the reverse step alone, timed on a fixed state. One verified cycle per Poisson solve, the
    launch configuration of the headline."""
    from workloads import workload

    w = workload("adjoint96", max_cycles=1)   # one verified cycle per solve, as the headline
    N = w.grid.N
    st = P.solver_for(w.with_(kappa=1.5, u0=1.2 * w.u0))
    tuning = st.autotune()   # launch shapes of the 96^3 grid, for the forward and reverse steps
    st.step(w.dt, nsteps)
    target = st.field("phi").clone()
    st.close()
    s = P.solver_for(w)
    P.rollout_gradient(s, w.dt, 2, target, checkpoint_every)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(w.dt, nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    s2 = P.solver_for(w)
    t0 = time.perf_counter()
    L, kb, sb, _ = P.rollout_gradient(s2, w.dt, nsteps, target, checkpoint_every)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    a = torch.randn(w.grid.shape, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    s2.grad_step(w.dt, a, b)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        s2.grad_step(w.dt, a, b)
    torch.cuda.synchronize()
    t_rev = (time.perf_counter() - t0) / reps
    # per-kernel event timing of the reverse step (a separate pass)
    s2.profile(True)
    for _ in range(5):
        s2.grad_step(w.dt, a, b)
    prof = s2.profile_read()
    s2.profile(False)
    rev_kernels = {k: {"mean_us": round(1e3 * ms / n, 2), "launches_per_step": n / 5}
                   for k, (ms, n) in prof.items() if n}
    s.close()
    s2.close()
    ce = max(1, checkpoint_every)
    recompute = sum(n - (n // ce) * ce for n in range(nsteps))
    out = {"workload": "adjoint96", "grid": list(w.grid.shape), "steps": nsteps,
           "poisson_max_cycles": w.max_cycles,
           "checkpoint_every": ce, "forward_ms_per_step": 1e3 * t_fwd / nsteps,
           "reverse_ms_per_step": 1e3 * t_rev,
           "reverse_cell_updates_per_s": N / t_rev,
           "rollout_gradient_s": t_grad,
           "rollout_forward_steps": nsteps + recompute, "rollout_reverse_steps": nsteps,
           "loss": L, "dL_dkappa": kb, "dL_dscale": sb, "reverse_kernels": rev_kernels,
           "autotuned": tuning}
    print(f"bench: adjoint96 forward {1e3 * t_fwd / nsteps:.3f} ms/step, reverse "
          f"{1e3 * t_rev:.3f} ms/step, rollout gradient of {nsteps} steps {t_grad:.2f} s",
          file=sys.stderr, flush=True)
    return out


def diagnostics_run(P, torch, base) -> dict:
    """vs_diagnostics on the 128^3 vesicle after 20 steps: the shear-stress field and the
    reductions, timed over 10 calls."""
    s = P.solver_for(base)
    s.step(base.dt, 20)
    sig = torch.empty(base.grid.shape, dtype=torch.float64, device="cuda")
    d = s.diagnostics(sig)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        s.diagnostics(sig)
    t = (time.perf_counter() - t0) / reps
    s.close()
    return {"workload": base.name, "ms_per_call": 1e3 * t, "values_after_20_steps": d}


def inertial_run(P, torch, base, nsteps: int, rho: float = 1e-3) -> dict:
    """The 128^3 vesicle with the inertial vorticity equation (SM eq. (36), implicit in time,
    a = rho/(eta dt)): nsteps steps of the kappa = 1 instance, one verified solve per step."""
    w = base.with_(rho=rho, max_cycles=1)
    s = P.solver_for(w)
    s.step(w.dt, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(w.dt, nsteps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    relres = s.scalars()["relres"]
    s.close()
    a = rho / (w.eta * w.dt)
    print(f"bench: inertial {w.name} rho={rho} (a h^2 = {a * w.grid.h ** 2:.3g}): "
          f"{1e3 * t / nsteps:.3f} ms/step", file=sys.stderr, flush=True)
    return {"workload": w.name, "rho": rho, "a_h2": a * w.grid.h ** 2, "steps": nsteps,
            "poisson_max_cycles": 1, "ms_per_step": 1e3 * t / nsteps,
            "cell_updates_per_s": w.grid.N * nsteps / t, "max_relres": relres}


def copy_ceiling(torch) -> float:
    """Device-to-device copy of a 1 GiB FP64 buffer (read + write bytes per second, GB/s): the
    practical streaming ceiling next to the nominal 8 TB/s."""
    a = torch.empty((1 << 30) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / 10
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / t / 1e9


def system_info(torch) -> dict:
    """The device, the software versions and the current clocks (each None if unreadable)."""
    info = {"device": None, "arch": None, "compute_units": None, "hip": torch.version.hip,
            "torch": torch.__version__, "rocm": None, "clocks": None}
    try:
        pr = torch.cuda.get_device_properties(0)
        info.update(device=pr.name, arch=pr.gcnArchName, compute_units=pr.multi_processor_count)
    except Exception:
        pass
    try:
        with open("/opt/rocm/.info/version") as f:
            info["rocm"] = f.read().strip()
    except OSError:
        pass
    try:
        import subprocess
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True,
                           timeout=30)
        card = next(iter(json.loads(r.stdout).values()))
        info["clocks"] = {k.rstrip(": "): v for k, v in card.items() if "clk" in k.lower()}
    except Exception:
        pass
    return info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--max-cycles", type=int, default=1,
                    help="Poisson refinement cycles per solve (each solve is verified on the device)")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision-steps", type=int, default=500,
                    help="steps of the FP64 vs FP32-refined comparison on droplet256 (0 = skip)")
    ap.add_argument("--graph-steps", type=int, default=-1,
                    help="steps of the headline instances replayed as one graph (-1: --steps, 0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=100,
                    help="steps of the 64-instance batch (0 = skip)")
    ap.add_argument("--batch-streams", type=int, default=2)
    ap.add_argument("--adjoint-steps", type=int, default=50,
                    help="steps of the 96^3 rollout gradient (0 = skip)")
    ap.add_argument("--inertial-steps", type=int, default=200,
                    help="steps of the 128^3 vesicle with the inertial vorticity equation (0 = skip)")
    ap.add_argument("--no-diagnostics", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (calibrates HBM counters)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (no vs_autotune before the timed steps)")
    ap.add_argument("--launch-shapes", type=str, default="",
                    help="fixed launch shapes of the 128^3 grid instead of vs_autotune, as "
                         "adv_slab=8,va_maxb=512,... (profiler runs: no candidate launches)")
    ap.add_argument("--cpu-single-only", action="store_true",
                    help="time the CPU oracle on one thread only")
    ap.add_argument("--repeats", type=int, default=4,
                    help="further timed regions like the first, reported beside `value` (0 = none)")
    ap.add_argument("--cpu-worker", type=float, default=0.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    args.profile_steps = max(1, args.profile_steps)   # the roofline needs one profiled step

    if args.cpu_worker > 0:
        # a CPU-only worker of the all-core oracle baseline: no GPU, one JSON line
        n, t = _oracle_steps(args.cpu_worker)
        print(json.dumps({"steps": n, "seconds": t}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py: the library runs one simulation per GPU on one GPU; --gpus {args.gpus} "
              "is not supported (the multi-GPU decomposition is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2601_05031_amd as P
    from workloads import workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    base = workload("vesicle128", max_cycles=args.max_cycles)
    nx, ny, nz = base.grid.shape
    N = base.grid.N
    print(f"bench: building {len(KAPPAS)} solvers for {base.name} {base.grid.shape}", file=sys.stderr,
          flush=True)
    solvers = [P.solver_for(base, kappa=k) for k in KAPPAS]
    tuning = None
    if args.launch_shapes:
        tuning = {k: int(v) for k, v in (kv.split("=") for kv in args.launch_shapes.split(","))}
        P.set_launch_shapes(base.grid.shape + (base.grid.h,), tuning)
        print(f"bench: fixed launch shapes {tuning}", file=sys.stderr, flush=True)
    elif not args.no_autotune:
        tuning = solvers[1].autotune()   # launch shapes of the 128^3 grid, shared by all three
        print(f"bench: autotuned launch shapes {tuning}", file=sys.stderr, flush=True)
    for s in solvers:
        s.step(base.dt, args.warmup)
    torch.cuda.synchronize()

    # ---- timed region: K benchmark steps = K time steps of each kappa instance
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    per_kappa = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k, s in zip(KAPPAS, solvers):
        a = time.perf_counter()
        s.step(base.dt, args.steps)
        per_kappa[str(k)] = time.perf_counter() - a
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    total_cells = len(KAPPAS) * N * args.steps
    value = total_cells / wall
    relres = max(s.scalars()["relres"] for s in solvers)
    print(f"bench: timed {args.steps} steps x {len(KAPPAS)} instances in {wall:.3f} s "
          f"(events {gpu_ms:.1f} ms), max relres {relres:.2e}", file=sys.stderr, flush=True)
    # the same timed region again (the run-to-run spread; `value` is the first)
    repeats = [value]
    for _ in range(max(0, args.repeats)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in solvers:
            s.step(base.dt, args.steps)
        torch.cuda.synchronize()
        repeats.append(total_cells / (time.perf_counter() - t0))
    relres = max(relres, max(s.scalars()["relres"] for s in solvers))
    if len(repeats) > 1:
        print(f"bench: {len(repeats)} timed regions: " + " ".join(f"{v:.4e}" for v in repeats),
              file=sys.stderr, flush=True)

    # ---- per-kernel event timing on the kappa = 1 instance (a separate pass)
    s1 = solvers[1]
    s1.profile(True)
    s1.step(base.dt, args.profile_steps)
    prof = s1.profile_read()
    s1.profile(False)
    # the clocks just after the timed and profiled steps (rocm-smi runs for a while with the
    # GPU idle, so not between the two)
    sysinfo = system_info(torch)
    kern = {}
    for name, (ms, n) in prof.items():
        if n == 0:
            continue
        kern[name] = {"total_ms": ms, "launches": n, "mean_us": 1e3 * ms / n}
    ranked = sorted(((v["total_ms"], k) for k, v in kern.items() if kernel_bytes(k, nx, ny, nz)),
                    reverse=True)
    dom = ranked[0][1]
    dom_bytes = kernel_bytes(dom, nx, ny, nz)
    dom_mean_s = kern[dom]["mean_us"] * 1e-6
    achieved = dom_bytes / dom_mean_s / 1e9
    traffic = stored_traffic(dom, base.name)
    ceiling = copy_ceiling(torch)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "timer": "per-launch start/stop events written by the dispatch packets "
                         "(hipExtLaunchKernelGGL), mean over the profiled steps",
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": dom_bytes, "mean_launch_us": round(kern[dom]["mean_us"], 2),
                "copy_ceiling": round(ceiling, 1), "frac_of_copy_ceiling": round(achieved / ceiling, 4)}
    step_bytes = sum(kernel_bytes(k, nx, ny, nz) * v["launches"] for k, v in kern.items()
                     if kernel_bytes(k, nx, ny, nz)) / args.profile_steps
    step_kernel_ms = sum(v["total_ms"] for v in kern.values()) / args.profile_steps

    # ---- the same three instances as one batch: one grid class, so every kernel of a step is
    # launched once for all three (the plane passes' last rounds fill better) and two steps are
    # replayed as one captured graph; an extra figure, `value` stays the plain sequential
    # vs_step path above
    headline_graph = None
    gsteps = args.steps if args.graph_steps < 0 else args.graph_steps
    if gsteps >= 2:
        b = P.Batch(solvers, nstreams=len(solvers))
        b.step(base.dt, 2)                      # capture + first replay, untimed
        torch.cuda.synchronize()
        kb = gsteps - (gsteps & 1)
        t0 = time.perf_counter()
        b.step(base.dt, kb)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        b.close()
        headline_graph = {"cell_updates_per_s": len(KAPPAS) * N * kb / tg, "steps": kb,
                          "ms_per_step": 1e3 * tg / kb,
                          "max_relres": max(s.scalars()["relres"] for s in solvers)}
        print(f"bench: the {len(KAPPAS)} instances as one graph: {1e3 * tg / kb:.3f} ms/step "
              f"({len(KAPPAS) * N * kb / tg:.3e} cell-updates/s)", file=sys.stderr, flush=True)

    for s in solvers:
        s.close()
    del solvers
    torch.cuda.empty_cache()

    precision = None
    if args.precision_steps > 0:
        precision = compare_precisions(P, torch, args.precision_steps)

    batched = None
    if args.batch_steps > 0:
        batched = batched_run(P, torch, args.batch_steps + (args.batch_steps & 1), args.batch_streams)

    adjoint = None
    if args.adjoint_steps > 0:
        adjoint = adjoint_run(P, torch, args.adjoint_steps)

    inertial = None
    if args.inertial_steps > 0:
        inertial = inertial_run(P, torch, base, args.inertial_steps)

    diagnostics = None
    if not args.no_diagnostics:
        diagnostics = diagnostics_run(P, torch, base)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(base, args.cpu_budget, not args.cpu_single_only)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": base.name, "grid": [nx, ny, nz], "kappa": list(KAPPAS),
                   "instances_per_step": len(KAPPAS), "dt": base.dt, "precision": "fp64",
                   "poisson_rtol": base.rtol, "poisson_max_cycles": args.max_cycles,
                   "flow": "poiseuille u0=0.05", "penalties": {"rate_V": base.rate_V, "k_A": base.k_A}},
        "steps_per_s_per_instance": len(KAPPAS) * args.steps / wall,
        "max_relres": relres,
        "timed_regions": {"values": repeats, "median": sorted(repeats)[len(repeats) // 2],
                          "note": "value is the first; each region is the same K steps of every instance"},
        "system": sysinfo,
        "per_kappa_cell_updates_per_s": {k: N * args.steps / t for k, t in per_kappa.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": {k: {"mean_us": round(v["mean_us"], 2), "launches_per_step": v["launches"] / args.profile_steps}
                    for k, v in kern.items()},
        "step_algorithmic_bytes": step_bytes,
        "step_kernel_ms": step_kernel_ms,
        "step_algorithmic_frac_hbm": (step_bytes / (step_kernel_ms * 1e-3) / 1e9) / HBM_PEAK_GBS,
        "instances_as_one_graph": headline_graph,
        "fp64_vs_fp32_refined": precision,
        "batched": batched,
        "adjoint": adjoint,
        "diagnostics": diagnostics,
        "inertial": inertial,
        "autotuned": tuning,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
