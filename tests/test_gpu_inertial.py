"""GPU parity of the inertial variant (SM "Time-dependency and inertial flow", eq. (36)):
the vorticity taken implicitly in time, (L_h - a) omega^{n+1} = S - a omega^n with
a = rho/(eta dt), against the CPU FP64 oracle, element by element.

Bar: relative L2 error <= 1e-9 per field, as for eq. (5b). Covers a weak and a strong shift
(a h^2 = 1 and 500), a ragged non-cubic Couette channel with the Cahn-Hilliard potential, a
change of dt between calls (the shifted pivots are rebuilt), a batch (bit-identical to the
instances stepped alone) and the calls the variant does not support.
"""
import numpy as np
import pytest

import oracle as O
from workloads import batch_instances, workload
from workloads.shapes import GridSpec

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
                 sigma=w.sigma, gamma0=w.gamma0, rate_V=w.rate_V, k_A=w.k_A,
                 bend_scale=w.bend_scale, rho=w.rho)
    return g, walls, p


def as_fields(s):
    d = {"phi": s.phi, "mu": s.mu}
    for c, ax in enumerate("xyz"):
        d["omega_" + ax] = s.omega[c]
        d["psi_" + ax] = s.psi[c]
    return d


def compare(got, ref, label):
    errs = {k: rel_l2(got[k], ref[k]) for k in FIELD_NAMES}
    say(f"  {label} " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not (v <= TOL)}
    assert not bad, bad


def oracle_steps(w, schedule):
    """The oracle stepped through [(dt, nsteps), ...] from the workload's phi0."""
    g, walls, p = oracle_objs(w)
    s = O.init_state(g, walls, p, w.phi0())
    for dt, n in schedule:
        for _ in range(n):
            s = O.step(s, dt, g, walls, p)
    return s


CASES = [
    # bending membrane, Poiseuille, a h^2 = rho/(eta dt) h^2 = 1 and 500
    ("vesicle32-weak", workload("vesicle32", rho=1e-3, max_cycles=1, rate_V=10.0, k_A=1.0), 4),
    ("vesicle32-strong", workload("vesicle32", rho=0.5, max_cycles=1), 3),
    # n_z = 128: the two-z-per-lane forms of the source, advance and residual kernels
    ("vesicle-nz128", workload("vesicle32", grid=GridSpec(32, 34, 128), rho=0.05, max_cycles=1,
                               rate_V=10.0, k_A=1.0), 3),
    # Cahn-Hilliard droplet in a ragged Couette channel (M = 31 rows, nz = 48)
    ("droplet-couette", workload("droplet256", grid=GridSpec(32, 33, 48), shape="sphere", R0=7.0,
                                 rho=0.02, max_cycles=1, eta=0.7), 4),
]


@pytest.mark.parametrize("label,w,nsteps", CASES, ids=[c[0] for c in CASES])
def test_inertial_matches_oracle(label, w, nsteps):
    say(f"case inertial {label} grid={w.grid.shape} model={w.model} walls={w.wall_kind} "
        f"rho={w.rho} eta={w.eta} dt={w.dt} nsteps={nsteps}")
    s = P.solver_for(w)
    g, walls, p = oracle_objs(w)
    compare(s.fields(), as_fields(O.init_state(g, walls, p, w.phi0())), "init")
    s.step(w.dt, nsteps)
    got = s.fields()
    sc = s.scalars()
    s.close()
    assert sc["step"] == nsteps
    compare(got, as_fields(oracle_steps(w, [(w.dt, nsteps)])), f"after {nsteps}")


def test_inertial_dt_change_rebuilds_the_shifted_pivots():
    w = workload("vesicle32", rho=0.01, max_cycles=1)
    sched = [(1e-3, 2), (5e-4, 2), (1e-3, 1)]
    say(f"case inertial-dt-change grid={w.grid.shape} rho={w.rho} schedule={sched}")
    s = P.solver_for(w)
    for dt, n in sched:
        s.step(dt, n)
    got = s.fields()
    s.close()
    compare(got, as_fields(oracle_steps(w, sched)), "dt schedule")


def test_inertial_batch_equals_single_instances():
    ws = [w.with_(rho=0.05 * (i + 1), max_cycles=1)
          for i, w in enumerate(x for x in batch_instances(64) if x.grid.nx <= 64)][:3]
    nsteps = 4
    say(f"case inertial-batch n={len(ws)} grids={[w.grid.nx for w in ws]} "
        f"rho={[w.rho for w in ws]} nsteps={nsteps}")
    singles = []
    for w in ws:
        s = P.solver_for(w)
        s.step(w.dt, 2)
        s.step(2 * w.dt, nsteps - 2)
        singles.append(s.fields())
        s.close()
    solvers = [P.solver_for(w) for w in ws]
    b = V.Batch(solvers, nstreams=4)
    b.step([w.dt for w in ws], 2)
    b.step([2 * w.dt for w in ws], nsteps - 2)     # new dt: new pivots, new capture
    b.close()
    for w, s, ref in zip(ws, solvers, singles):
        got = s.fields()
        s.close()
        for k in FIELD_NAMES:
            assert np.array_equal(got[k], ref[k]), (w.name, k)


def test_inertial_unsupported_calls():
    w = workload("vesicle32", rho=0.1, max_cycles=1)
    say(f"case inertial-unsupported grid={w.grid.shape}")
    s = P.solver_for(w)
    a = torch.zeros(s.shape, dtype=torch.float64, device="cuda:0")
    b = torch.zeros_like(a)
    with pytest.raises(V.VsError) as e:
        s.grad_step(w.dt, a, b)
    assert e.value.code == V.VS_E_UNSUPPORTED
    with pytest.raises(V.VsError) as e:
        s.set_walls(0.02)
    assert e.value.code == V.VS_E_UNSUPPORTED
    s.step(w.dt, 1)                  # the state is untouched by the rejected calls
    assert s.scalars()["step"] == 1
    s.close()
