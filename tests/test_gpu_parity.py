"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle, element by element.

Bar (FP64): relative L2 error <= 1e-9 per field (phi, mu, omega, psi); Poisson solves alone
<= 1e-12. Every case prints its name, shape and seed before it touches the GPU.
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import workload
from workloads.shapes import GridSpec, phi_sphere

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2601_05031_amd as P  # noqa: E402
from paper_2601_05031_amd import vs as V  # noqa: E402

TOL = 1e-9
FIELD_NAMES = ["phi", "mu", "omega_x", "omega_y", "omega_z", "psi_x", "psi_y", "psi_z"]


def say(msg):
    print(msg, flush=True)


def rel_l2(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def oracle_objs(w):
    g = O.Grid(*w.grid.shape, h=w.grid.h)
    walls = O.Walls(w.wall_kind, w.u0, w.u1)
    p = O.Params(model=w.model, eta=w.eta, mobility=w.mobility, eps=w.eps, kappa=w.kappa,
                 sigma=w.sigma, gamma0=w.gamma0, rate_V=w.rate_V, k_A=w.k_A, bend_scale=w.bend_scale)
    return g, walls, p


def ref_fields(s):
    d = {"phi": s.phi, "mu": s.mu}
    for c, ax in enumerate("xyz"):
        d["omega_" + ax] = s.omega[c]
        d["psi_" + ax] = s.psi[c]
    return d


def compare(got, ref, tol=TOL, label=""):
    errs = {k: rel_l2(got[k], ref[k]) for k in FIELD_NAMES}
    say(f"  {label} " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not (v <= tol)}
    assert not bad, bad
    return errs


def run_both(w, nsteps):
    say(f"case {w.name} grid={w.grid.shape} seed={w.seed} model={w.model} walls={w.wall_kind} "
        f"nsteps={nsteps}")
    s = P.solver_for(w)
    if nsteps:
        s.step(w.dt, nsteps)
    got = s.fields()
    sc = s.scalars()
    s.close()
    g, walls, p = oracle_objs(w)
    ref = O.run(g, walls, p, w.phi0(), w.dt, nsteps)
    return got, sc, ref


# ------------------------------------------------------------------------- Poisson alone
# row counts M = ny - 2 that select each tridiagonal layout: the two-lane twisted solve
# (M = 1, 258), and 4 or 8 register segments per mode with every segment length bound
# (M = 4: one row each; 5, 17, 31: ragged; 68; 148)
@pytest.mark.parametrize("shape,h", [((24, 7, 12), 1.0), ((32, 33, 48), 0.5), ((96, 19, 96), 1.3),
                                     ((8, 3, 6), 1.0), ((16, 6, 12), 1.0), ((16, 70, 18), 0.7),
                                     ((12, 150, 8), 1.0), ((8, 260, 6), 1.0)])
def test_poisson_solve_matches_oracle(shape, h):
    say(f"case poisson shape={shape} h={h}")
    w = workload("vesicle32").with_(grid=GridSpec(*shape, h=h), shape="sphere", R0=2.0)
    s = P.solver_for(w)
    rng = np.random.default_rng(11)
    f = rng.standard_normal(shape)
    u0 = rng.standard_normal(shape)
    ft = torch.tensor(f, device="cuda")
    ut = torch.tensor(u0, device="cuda")
    code, cycles, rel = s.poisson_solve(ft, ut, rtol=1e-12, max_cycles=3)
    u = ut.cpu().numpy()
    s.close()
    g = O.Grid(*shape, h=h)
    ref = O.poisson_solve(f[:, 1:-1, :], u0[:, 0, :], u0[:, -1, :], g)
    err = rel_l2(u[:, 1:-1, :], ref)
    say(f"  code={code} cycles={cycles} relres={rel:.2e} relL2={err:.2e}")
    assert code == V.VS_OK and rel <= 1e-12 and cycles >= 1
    assert err <= 1e-12
    assert np.array_equal(u[:, 0, :], u0[:, 0, :]) and np.array_equal(u[:, -1, :], u0[:, -1, :])


# every transform length the library accepts (even 2^a 3^b in [4, 512]); each appears once along
# x and once along z, paired so that short and long lengths meet
def _smooth23(n):
    while n % 2 == 0:
        n //= 2
    while n % 3 == 0:
        n //= 3
    return n == 1


LENGTHS = [n for n in range(4, 513, 2) if _smooth23(n)]


@pytest.mark.parametrize("i", range(len(LENGTHS)))
def test_poisson_every_transform_length(i):
    nx, nz = LENGTHS[i], LENGTHS[(i + 13) % len(LENGTHS)]
    shape = (nx, 6, nz)
    say(f"case poisson-length shape={shape}")
    w = workload("vesicle32").with_(grid=GridSpec(*shape), shape="sphere", R0=1.5)
    s = P.solver_for(w)
    rng = np.random.default_rng(100 + i)
    f = rng.standard_normal(shape)
    u0 = rng.standard_normal(shape)
    ft = torch.tensor(f, device="cuda")
    ut = torch.tensor(u0, device="cuda")
    code, cycles, rel = s.poisson_solve(ft, ut, rtol=1e-12, max_cycles=3)
    u = ut.cpu().numpy()
    s.close()
    ref = O.poisson_solve(f[:, 1:-1, :], u0[:, 0, :], u0[:, -1, :], O.Grid(*shape))
    err = rel_l2(u[:, 1:-1, :], ref)
    say(f"  code={code} cycles={cycles} relres={rel:.2e} relL2={err:.2e}")
    assert code == V.VS_OK and rel <= 1e-12
    assert err <= 1e-12


def test_poisson_zero_rhs_zero_walls_gives_zero():
    say("case poisson zero rhs")
    w = workload("vesicle32")
    s = P.solver_for(w)
    ft = torch.zeros(w.grid.shape, dtype=torch.float64, device="cuda")
    ut = torch.ones(w.grid.shape, dtype=torch.float64, device="cuda")
    ut[:, 0, :] = 0
    ut[:, -1, :] = 0
    code, cycles, rel = s.poisson_solve(ft, ut, rtol=1e-10, max_cycles=2)
    s.close()
    assert code == V.VS_OK and rel == 0.0
    assert float(ut.abs().max()) == 0.0


# ---------------------------------------------------------------------- init and steps
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_init_parity_vesicle32(seed):
    w = workload("vesicle32", seed=seed)
    got, sc, ref = run_both(w, 0)
    compare(got, ref_fields(ref), label="init")
    assert sc["V0"] == pytest.approx(ref.V0, rel=1e-12)
    assert sc["A0"] == pytest.approx(ref.A0, rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_step_parity_vesicle32(seed):
    w = workload("vesicle32", seed=seed)
    got, sc, ref = run_both(w, w.nsteps)
    compare(got, ref_fields(ref), label="5 steps")
    assert sc["V"] == pytest.approx(ref.V, rel=1e-12)
    assert sc["A"] == pytest.approx(ref.A, rel=1e-11)
    assert sc["relres"] <= w.rtol
    assert sc["step"] == w.nsteps


def test_step_parity_penalties_and_tension():
    """Volume/area penalties and a surface tension on, ragged small grid, Couette walls."""
    w = workload("vesicle32", grid=GridSpec(24, 21, 36), wall_kind="couette", u0=-0.03, u1=0.05,
                 R0=6.0, gamma0=0.2, rate_V=10.0, k_A=1.0, kappa=0.5, seed=4, dt=5e-4)
    got, sc, ref = run_both(w, 6)
    compare(got, ref_fields(ref), label="6 steps")
    # lambda_V = 2 rate_V (V0 - V)/(M |Omega|) is a small difference of two large volumes, so
    # its bound is the one V and V0 carry (relative 1e-12 each), not a relative one on lambda_V
    assert sc["V"] == pytest.approx(ref.V, rel=1e-12)
    assert sc["V0"] == pytest.approx(ref.V0, rel=1e-12)
    g, _, p = oracle_objs(w)
    lam_bound = 2.0 * p.rate_V * 1e-12 * (abs(ref.V) + abs(ref.V0)) / (p.mobility * g.domain_volume)
    assert abs(sc["lambda_V"] - ref.lam_V) <= lam_bound, (sc["lambda_V"], ref.lam_V, lam_bound)
    assert sc["gamma_A"] == pytest.approx(ref.gamma_A, rel=1e-9, abs=1e-14)


@pytest.mark.parametrize("seed", [0, 2])
def test_step_parity_one_cycle(seed):
    """One verified cycle per solve (the benchmark's setting): same fields as the oracle."""
    w = workload("vesicle32", seed=seed, max_cycles=1)
    got, sc, ref = run_both(w, w.nsteps)
    compare(got, ref_fields(ref), label="5 steps, 1 cycle")
    assert sc["relres"] <= w.rtol


@pytest.mark.parametrize("shape", [None, (16, 24, 48), (16, 24, 24), (16, 24, 64),
                                   (16, 24, 128), (12, 20, 256)])
def test_combined_flow_residual_matches_separate_passes(shape):
    """With one cycle per solve the two flow residuals run as one combined pass; with two
    cycles each solve is verified by its own residual pass. The direct solve converges in
    cycle 0 either way, so the fields agree bit for bit and the largest relative residual
    of the two verifications agrees to rounding. The combined pass has two forms, by n_z:
    one z per lane (n_z = 24, 48: not a multiple of 32), and two z per lane in row segments
    of 16, 32 or 64 lanes (n_z = 32 for the vesicle32 case, 64, 128, 256)."""
    if shape is None:
        w = workload("vesicle32", seed=3)
    else:
        w = workload("droplet256", grid=GridSpec(*shape), R0=5.0)
    say(f"case combined vs separate flow residuals {w.name} {w.grid.shape}")
    one = P.solver_for(w, max_cycles=1)
    two = P.solver_for(w, max_cycles=2)
    one.step(w.dt, 3)
    two.step(w.dt, 3)
    f1, f2 = one.fields(), two.fields()
    r1, r2 = one.scalars()["relres"], two.scalars()["relres"]
    one.close()
    two.close()
    for k in FIELD_NAMES:
        assert np.array_equal(f1[k], f2[k]), k
    say(f"  relres combined={r1:.6e} separate={r2:.6e}")
    assert 0.0 < r1 <= w.rtol
    assert r1 == pytest.approx(r2, rel=1e-12)


def test_step_parity_cahn_hilliard_couette():
    """Cahn-Hilliard droplet in plane Couette flow (walls at -/+0.05)."""
    w = workload("droplet256", grid=GridSpec(48, 32, 96), R0=9.0, nsteps=5)
    got, sc, ref = run_both(w, 5)
    compare(got, ref_fields(ref), label="CH 5 steps")


@pytest.mark.parametrize("ny", [6, 40, 96, 128, 140, 256, 260])
def test_step_parity_tall_channels(ny):
    """Cahn-Hilliard droplet in Couette flow across the tridiagonal layouts (M = ny - 2)."""
    R = min(4.0, 0.3 * (ny - 1))
    w = workload("droplet256", grid=GridSpec(16, ny, 24), R0=R, nsteps=3)
    got, sc, ref = run_both(w, 3)
    compare(got, ref_fields(ref), label=f"ny={ny}")


# n_z a multiple of 64: the two-z-per-lane explicit and residual kernels with 32-lane row
# segments (64, 192) or whole 64-lane segments (128), bending and Cahn-Hilliard, one solve
@pytest.mark.parametrize("shape,name", [((32, 20, 64), "vesicle32"), ((24, 18, 192), "droplet256"),
                                        ((16, 26, 128), "droplet256")])
def test_step_parity_two_z_kernels(shape, name):
    w = workload(name, grid=GridSpec(*shape), R0=5.0, nsteps=3, max_cycles=1)
    if name == "vesicle32":
        w = w.with_(rate_V=10.0, k_A=1.0)
    got, sc, ref = run_both(w, 3)
    compare(got, ref_fields(ref), label=f"{name} {shape}")
    assert sc["cycles"] == 6 and sc["relres"] <= w.rtol


@pytest.mark.parametrize("shape", [(486, 6, 512), (512, 7, 432)])
def test_step_parity_longest_transforms(shape):
    """Whole steps at the longest transform lengths (the general Stockham plans, and z lines
    of 512 and 432 nodes in the two-z and one-z residual paths)."""
    w = workload("droplet256", grid=GridSpec(*shape), R0=2.0, nsteps=2)
    got, sc, ref = run_both(w, 2)
    compare(got, ref_fields(ref), label=f"{shape}")


@pytest.mark.parametrize("kappa,nsteps", [(1.0, 10), (0.5, 10), (2.0, 10)])
def test_step_parity_vesicle128_full_size(kappa, nsteps):
    """The 128^3 prolate vesicle at full size, first steps of each kappa of the benchmark,
    in the launch configuration the benchmark times (one verified cycle per Poisson solve,
    the combined residual pass, the checks of all but the last step inside the next advance,
    all steps in one call). The oracle takes about two seconds per step."""
    w = workload("vesicle128", nsteps=nsteps, max_cycles=1, kappa=kappa)
    got, sc, ref = run_both(w, nsteps)
    compare(got, ref_fields(ref), label=f"128^3 kappa={kappa} {nsteps} steps")
    assert sc["cycles"] == 2 * nsteps and sc["relres"] <= w.rtol


def test_no_body_channel_is_exact():
    """phi = -1: omega_x and psi_x are the linear and cubic wall profiles to roundoff."""
    say("case no-body poiseuille 16x31x16")
    w = workload("vesicle32", grid=GridSpec(16, 31, 16))
    s = P.Solver((16, 31, 16, 1.0), w.walls(), dict(kappa=1.0), -np.ones((16, 31, 16)))
    s.step(1e-3, 2)
    got = s.fields()
    s.close()
    g, walls, _ = oracle_objs(w)
    _, psx, omx = O.wall_profiles(g, walls)
    assert np.max(np.abs(got["omega_x"] - omx[None, :, None])) < 1e-15
    assert np.max(np.abs(got["psi_x"] - psx[None, :, None])) < 1e-13
    for k in ("omega_y", "omega_z", "psi_y", "psi_z", "mu"):
        assert np.max(np.abs(got[k])) < 1e-15
    assert np.max(np.abs(got["phi"] + 1.0)) == 0.0


def test_phi_budget_on_gpu():
    """Delta(sum_w phi) over one GPU step = dt (M lambda_V W - sum_w v . D phi), with v and
    D phi evaluated on the GPU's own psi and phi."""
    w = workload("vesicle32", rate_V=10.0, k_A=1.0, seed=3)
    say(f"case budget {w.grid.shape}")
    s = P.solver_for(w)
    g, walls, p = oracle_objs(w)
    W = float(np.sum(g.weights() * np.ones(g.shape)))
    for _ in range(3):
        f0 = s.fields()
        lam = s.scalars()["lambda_V"]
        v = O.velocity(np.stack([f0["psi_x"], f0["psi_y"], f0["psi_z"]]), g, walls)
        dx, dy, dz = O.grad_mirror(f0["phi"], g.h)
        adv = float(np.sum(g.weights() * (v[0] * dx + v[1] * dy + v[2] * dz)))
        before = float(np.sum(g.weights() * f0["phi"]))
        s.step(w.dt, 1)
        after = float(np.sum(g.weights() * s.field("phi").cpu().numpy()))
        assert abs((after - before) - w.dt * (lam * W - adv)) < 1e-10 * abs(before)
    s.close()


def test_largest_segmented_grid_against_oracle_parts():
    """The largest grid of the segmented tridiagonal layout at the longest transforms:
    512 x 258 x 512 (M = 256, 67.6 M nodes), where the whole oracle step takes too long. The
    explicit part of a step is checked against the oracle's own functions applied to the GPU's
    state before the step (the phi update of SM (29a) with v = curl psi, then mu of the new
    phi); the two Poisson solves are verified on the device to rtol in one cycle (also with the
    checks taken inside the next advance); every field stays finite."""
    w = workload("droplet256", grid=GridSpec(512, 258, 512), R0=60.0, max_cycles=1)
    say(f"case largest segmented grid {w.grid.shape}")
    s = P.solver_for(w)
    s.step(w.dt, 1)
    g, walls, p = oracle_objs(w)
    lam = s.scalars()["lambda_V"]
    phi = s.field("phi").cpu().numpy()
    mu = s.field("mu").cpu().numpy()
    psi = np.stack([s.field(k).cpu().numpy() for k in ("psi_x", "psi_y", "psi_z")])
    v = O.velocity(psi, g, walls)
    del psi
    want = O.advance_phi(phi, mu, v, lam, w.dt, g, p)
    del mu, v
    s.step(w.dt, 1)
    # the increments compared, not phi itself (an increment is ~1e-4 of phi)
    e_phi = rel_l2(s.field("phi").cpu().numpy() - phi, want - phi)
    del phi
    want = O.chemical_potential(want, g, p, s.scalars()["gamma_A"])
    e_mu = rel_l2(s.field("mu").cpu().numpy(), want)
    del want
    say(f"  phi increment {e_phi:.2e}, mu {e_mu:.2e} against the oracle's functions")
    assert e_phi <= 1e-12 and e_mu <= 1e-12
    s.step(w.dt, 2)
    sc = s.scalars()
    say(f"  relres {sc['relres']:.2e} cycles {sc['cycles']}")
    assert sc["cycles"] == 4 and sc["relres"] <= w.rtol, sc
    for k in FIELD_NAMES:
        assert bool(torch.isfinite(s.field(k)).all()), k
    s.close()


# ------------------------------------------------------------- determinism and checkpoints
def test_repeat_runs_bitwise_equal_and_checkpoint_resume():
    w = workload("vesicle32", seed=1)
    say("case determinism/checkpoint vesicle32")
    a = P.solver_for(w)
    a.step(w.dt, 4)
    fa = a.fields()
    b = P.solver_for(w)
    b.step(w.dt, 2)
    blob = b.save()
    b.step(w.dt, 2)
    fb = b.fields()
    c = P.solver_for(w.with_(seed=2))
    c.load(blob)
    c.step(w.dt, 2)
    fc = c.fields()
    for k in FIELD_NAMES:
        assert np.array_equal(fa[k], fb[k]), k
        assert np.array_equal(fa[k], fc[k]), k
    assert c.scalars()["step"] == 4
    for s in (a, b, c):
        s.close()


def test_device_checkpoint_equals_host_checkpoint():
    """A checkpoint kept in device memory restores the same state as one in host memory,
    into the same or another solver, and the two blobs hold the same bytes."""
    w = workload("vesicle32", seed=4)
    say("case device checkpoint vesicle32")
    a = P.solver_for(w, max_cycles=1)
    a.step(w.dt, 2)
    hb = a.save()
    db = a.save(device=True)
    assert db.is_cuda and db.numel() == len(hb)
    assert bytes(db.cpu().numpy().tobytes()) == hb
    a.step(w.dt, 2)
    ref = a.fields()
    b = P.solver_for(w.with_(seed=6), max_cycles=1)
    b.load(db)
    b.step(w.dt, 2)
    a.load(hb)
    a.step(w.dt, 2)
    fa, fb = a.fields(), b.fields()
    for k in FIELD_NAMES:
        assert np.array_equal(fa[k], ref[k]), k
        assert np.array_equal(fb[k], ref[k]), k
    assert b.scalars()["step"] == 4
    a.close()
    b.close()


# ------------------------------------------------------------------------- error paths
def test_unstable_dt_rejected_before_enqueue():
    w = workload("vesicle32")
    say("case unstable dt")
    s = P.solver_for(w)
    before = s.fields()["phi"]
    C_b = 3 * math.sqrt(2) / 8
    bound = 2.0 / (12 * C_b * 14**2)
    with pytest.raises(V.VsError) as e:
        s.step(1.01 * bound, 1)
    assert e.value.code == V.VS_E_UNSTABLE
    assert np.array_equal(s.fields()["phi"], before)
    s.step(0.99 * bound, 1)   # just below the bound is accepted
    s.close()


def test_step_argument_errors_leave_the_state():
    """No step (nsteps < 1) and a time step that is not a positive finite number are argument
    errors, found on the host: nothing runs, the fields and the step count stay."""
    w = workload("vesicle32", grid=GridSpec(16, 12, 16), R0=3.0)
    say("case step argument errors")
    s = P.solver_for(w)
    before = s.fields()
    for dt, n in [(w.dt, 0), (w.dt, -3), (0.0, 1), (-w.dt, 1), (float("nan"), 1), (float("inf"), 1)]:
        with pytest.raises(V.VsError) as e:
            s.step(dt, n)
        assert e.value.code == V.VS_E_ARG, (dt, n)
    after = s.fields()
    assert s.scalars()["step"] == 0
    for k in before:
        assert np.array_equal(after[k], before[k]), k
    s.step(w.dt, 1)
    assert s.scalars()["step"] == 1
    s.close()


def test_unreachable_tolerance_reports_noconv():
    w = workload("vesicle32")
    say("case noconv")
    s = P.solver_for(w)
    f = torch.randn(w.grid.shape, dtype=torch.float64, device="cuda")
    u = torch.zeros(w.grid.shape, dtype=torch.float64, device="cuda")
    code, cycles, rel = s.poisson_solve(f, u, rtol=1e-30, max_cycles=2)
    assert code == V.VS_E_NOCONV and cycles == 2 and 0 < rel < 1e-12
    s.close()


def test_nan_injection_reports_nonfinite():
    w = workload("vesicle32")
    say("case nan injection")
    s = P.solver_for(w)
    blob = bytearray(s.save())
    hdr = len(blob) - 8 * 8 * w.grid.N
    arr = np.frombuffer(blob, dtype=np.float64, count=w.grid.N, offset=hdr).copy()
    arr[1000] = np.nan
    blob[hdr:hdr + 8 * w.grid.N] = arr.tobytes()
    s.load(bytes(blob))
    with pytest.raises(V.VsError) as e:
        s.step(w.dt, 1)
    assert e.value.code == V.VS_E_NONFINITE
    s.close()


def test_nan_injection_reports_nonfinite_over_several_steps():
    """Several steps in one call: the flow checks of all but the last step run inside the
    next step's advance kernel; a NaN still surfaces as NONFINITE at the end of the call."""
    w = workload("vesicle32")
    say("case nan injection, 3 steps in one call")
    s = P.solver_for(w, max_cycles=1)
    blob = bytearray(s.save())
    hdr = len(blob) - 8 * 8 * w.grid.N
    arr = np.frombuffer(blob, dtype=np.float64, count=w.grid.N, offset=hdr).copy()
    arr[777] = np.nan
    blob[hdr:hdr + 8 * w.grid.N] = arr.tobytes()
    s.load(bytes(blob))
    with pytest.raises(V.VsError) as e:
        s.step(w.dt, 3)
    assert e.value.code == V.VS_E_NONFINITE
    s.close()


@pytest.mark.parametrize("nsteps", [1, 2, 5])
def test_every_flow_check_runs_once_per_step(nsteps):
    """With one cycle per solve each step runs two checks (vorticity, stream vector), whether
    in the standalone check kernel or in the next step's advance kernel."""
    w = workload("vesicle32", seed=5)
    say(f"case check count nsteps={nsteps}")
    s = P.solver_for(w, max_cycles=1)
    s.step(w.dt, nsteps)
    sc = s.scalars()
    s.close()
    assert sc["cycles"] == 2 * nsteps
    assert 0.0 < sc["relres"] <= w.rtol


def test_phi_sphere_helper_shapes():
    g = GridSpec(8, 8, 8)
    assert phi_sphere(g, 2.0, 1.0).shape == (8, 8, 8)


# ------------------------------------------------------------------ FP32-refined mode
TOL_REFINED = 1e-6


def test_refined_poisson_needs_and_gets_refinement():
    """FP32-stored spectral solves inside FP64 defect correction reach rtol = 1e-12 after a
    few cycles; one cycle alone stops near FP32 accuracy."""
    shape = (32, 33, 48)
    say(f"case refined poisson {shape}")
    w = workload("vesicle32").with_(grid=GridSpec(*shape, h=0.5), shape="sphere", R0=4.0)
    s = P.solver_for(w, precision="fp32_refined")
    rng = np.random.default_rng(5)
    f = rng.standard_normal(shape)
    u0 = rng.standard_normal(shape)
    g = O.Grid(*shape, h=0.5)
    ref = O.poisson_solve(f[:, 1:-1, :], u0[:, 0, :], u0[:, -1, :], g)
    ft = torch.tensor(f, device="cuda")
    ut = torch.tensor(u0, device="cuda")
    code1, cyc1, rel1 = s.poisson_solve(ft, ut, rtol=1e-12, max_cycles=1)
    ut = torch.tensor(u0, device="cuda")
    code, cycles, rel = s.poisson_solve(ft, ut, rtol=1e-12, max_cycles=6)
    err = rel_l2(ut.cpu().numpy()[:, 1:-1, :], ref)
    s.close()
    say(f"  one cycle: relres={rel1:.2e}; refined: cycles={cycles} relres={rel:.2e} relL2={err:.2e}")
    assert code1 == V.VS_E_NOCONV and 1e-9 < rel1 < 1e-5
    assert code == V.VS_OK and 2 <= cycles <= 6 and rel <= 1e-12 and err <= 1e-10


@pytest.mark.parametrize("seed", [0, 1])
def test_refined_step_parity_vesicle32(seed):
    w = workload("vesicle32", seed=seed, max_cycles=4)
    say(f"case refined vesicle32 seed={seed}")
    s = P.solver_for(w, precision="fp32_refined")
    s.step(w.dt, w.nsteps)
    got = s.fields()
    sc = s.scalars()
    s.close()
    g, walls, p = oracle_objs(w)
    ref = O.run(g, walls, p, w.phi0(), w.dt, w.nsteps)
    compare(got, ref_fields(ref), tol=TOL_REFINED, label="refined 5 steps")
    assert sc["relres"] <= w.rtol


def test_refined_predictor_one_cycle_per_solve():
    """The refined mode's first correction cycle of a step starts from the fields extrapolated
    in time from the last two increments (held in FP32), so after the first steps one FP32
    cycle per solve meets rtol, where the previous step's fields alone need two. A checkpoint
    holds no increments: a reloaded state starts the predictor over and reaches the same fields
    to within the solve tolerance."""
    w = workload("droplet256", grid=GridSpec(64, 34, 64), R0=10.0, nsteps=12, max_cycles=4)
    say(f"case refined predictor droplet {w.grid.shape}")
    s = P.solver_for(w, precision="fp32_refined")
    s.step(w.dt, 2)
    first = s.scalars()["cycles"] / 4.0
    blob = s.save()
    s.step(w.dt, 10)
    later = s.scalars()["cycles"] / 20.0
    got = s.fields()
    assert s.scalars()["relres"] <= w.rtol
    s.close()
    r = P.solver_for(w, precision="fp32_refined")
    r.load(blob)
    r.step(w.dt, 10)
    again = r.scalars()["cycles"] / 20.0
    rel = r.fields()
    r.close()
    say(f"  cycles/solve: steps 1-2 {first:.2f}, steps 3-12 {later:.2f}, after reload {again:.2f}")
    assert first >= 1.5 and later <= 1.1 and again <= 1.3
    g, walls, p = oracle_objs(w)
    ref = ref_fields(O.run(g, walls, p, w.phi0(), w.dt, 12))
    compare(got, ref, tol=TOL_REFINED, label="refined predictor 12 steps")
    compare(rel, ref, tol=TOL_REFINED, label="refined predictor, reloaded at step 2")


# every lane layout of the predicted-residual pass (two z per lane in row segments of 8, 16, 32
# and 64 lanes) and of the z passes around it
@pytest.mark.parametrize("shape", [(32, 20, 48), (32, 22, 96), (32, 18, 128), (32, 14, 256)])
def test_refined_predictor_shapes_match_oracle(shape):
    w = workload("droplet256", grid=GridSpec(*shape), R0=5.0, nsteps=8, max_cycles=4)
    say(f"case refined predictor {w.grid.shape}")
    s = P.solver_for(w, precision="fp32_refined")
    s.step(w.dt, 8)
    got = s.fields()
    sc = s.scalars()
    s.close()
    g, walls, p = oracle_objs(w)
    ref = ref_fields(O.run(g, walls, p, w.phi0(), w.dt, 8))
    compare(got, ref, tol=TOL_REFINED, label=f"refined predictor {shape} 8 steps")
    assert sc["relres"] <= w.rtol


_DROPLET_REF = {}


def _droplet256_oracle(nsteps):
    """The oracle's droplet256 run (about 6 s a step), shared by both precision cases."""
    if nsteps not in _DROPLET_REF:
        w = workload("droplet256", nsteps=nsteps)
        g, walls, p = oracle_objs(w)
        _DROPLET_REF[nsteps] = ref_fields(O.run(g, walls, p, w.phi0(), w.dt, nsteps))
    return _DROPLET_REF[nsteps]


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_droplet256_full_size(precision):
    """The Cahn-Hilliard droplet in Couette flow at its full 128 x 128 x 256 size, first 10
    steps, against the FP64 oracle: FP64 in the benchmark's launch configuration (one verified
    solve; 256-long z lines, two z per lane) at the FP64 bar, and the refined mode (FP32
    sweeps and corrections, FP64 defect correction to rtol = 1e-10) at 1e-6 per field."""
    nsteps = 10
    mc = 1 if precision == "fp64" else 4
    w = workload("droplet256", nsteps=nsteps, max_cycles=mc)
    say(f"case droplet256 {w.grid.shape} precision={precision} max_cycles={mc} nsteps={nsteps}")
    s = P.solver_for(w, precision=precision)
    s.step(w.dt, nsteps)
    got = s.fields()
    sc = s.scalars()
    s.close()
    ref = _droplet256_oracle(nsteps)
    compare(got, ref, tol=TOL if precision == "fp64" else TOL_REFINED,
            label=f"droplet256 {precision} {nsteps} steps")
    assert sc["relres"] <= w.rtol
