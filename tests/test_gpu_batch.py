"""GPU batches: many independent instances stepped through one captured HIP graph.

A batch runs exactly the kernels vs_step runs, on other streams, so every instance must come
out bit-identical to the same instance stepped alone, and within the FP64 bar of the oracle.
"""
import numpy as np
import pytest

import oracle as O
from workloads import batch_instances

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2601_05031_amd as P  # noqa: E402
from paper_2601_05031_amd import vs as V  # noqa: E402

FIELD_NAMES = ["phi", "mu", "omega_x", "omega_y", "omega_z", "psi_x", "psi_y", "psi_z"]


def say(msg):
    print(msg, flush=True)


def rel_l2(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def small_instances(k):
    """The first k batch instances with a 48^3 or 64^3 grid (the oracle runs them in seconds)."""
    out = [w for w in batch_instances(64) if w.grid.nx <= 64]
    return out[:k]


def test_batch_instances_recipe():
    ws = batch_instances(64)
    assert len(ws) == 64
    assert {w.grid.nx for w in ws} == {48, 64, 96, 128}
    assert {w.wall_kind for w in ws} == {"poiseuille", "couette"}
    for w in ws:
        assert 0.15 * w.grid.H <= w.R0 <= 0.25 * w.grid.H
        assert 0.5 <= w.kappa <= 2.0 and 0.7 <= w.prolate_Vr <= 0.95


# (fp64, 1) and (fp32_refined, 3): every kernel launched once per grid class over the device
# argument tables; (fp64, 3): FP64 with correction cycles, stepped instance by instance inside
# the graph; plane = 1: the FP64 transforms as plane passes over the tables
@pytest.mark.parametrize("precision,mc,plane", [("fp64", 1, 0), ("fp64", 1, 1), ("fp64", 3, 1),
                                                ("fp32_refined", 3, 0)])
def test_batch_bitwise_equals_single_instances(precision, mc, plane):
    ws = [w.with_(max_cycles=mc) for w in small_instances(5)]
    nsteps = 4
    say(f"case batch-vs-single precision={precision} max_cycles={mc} plane={plane} n={len(ws)} "
        f"grids={[w.grid.nx for w in ws]} seeds={[w.seed for w in ws]} nsteps={nsteps}")
    # the batch tunes the launch shapes of every grid it has not seen (vs_autotune); bitwise
    # equality needs the same shapes (block partial layouts) on both sides: fix them first
    for w in ws:
        V.set_launch_shapes(w.grid.shape + (w.grid.h,), dict(adv_slab=2, va_maxb=512, res_maxb=2048,
                                                             seg_alt=1, mu_kind=0, mu_ni=8, plane=plane))
    singles = []
    for w in ws:
        s = P.solver_for(w, precision=precision)
        s.step(w.dt, nsteps)
        singles.append((s.fields(), s.scalars(), s.log()))
        s.close()
    solvers = [P.solver_for(w, precision=precision) for w in ws]
    b = V.Batch(solvers, nstreams=4)
    b.step([w.dt for w in ws], 2)
    b.step([w.dt for w in ws], nsteps - 2)      # replays the captured graph
    b.close()
    # log fields compared bit for bit: all but the cycles (counted per call) and the relative
    # residual (its partial sums are added in a block of the size of the kernel that runs the
    # check: the next step's advance, or the check kernel after a call's or a graph's last step)
    keep = [i for i, k in enumerate(V.LOG_FIELDS) if k not in ("cycles", "relres")]
    ir = V.LOG_FIELDS.index("relres")
    for w, s, (ref, rsc, rlog) in zip(ws, solvers, singles):
        got = s.fields()
        sc = s.scalars()
        for k in FIELD_NAMES:
            assert np.array_equal(got[k], ref[k]), (w.name, k)
        assert sc["step"] == nsteps and sc["V"] == rsc["V"] and sc["A"] == rsc["A"]
        # the per-step log: the same records, written by the batch's checks
        glog = s.log()
        assert glog.shape == rlog.shape == (nsteps + 1, len(V.LOG_FIELDS)), (glog.shape, rlog.shape)
        assert np.array_equal(glog[:, keep], rlog[:, keep]), w.name
        assert np.allclose(glog[:, ir], rlog[:, ir], rtol=1e-12, atol=0.0), w.name
        # the states keep working after the batch is gone
        s.step(w.dt, 1)
        s.close()


@pytest.mark.parametrize("precision,mc,tol", [("fp64", 1, 1e-9), ("fp32_refined", 4, 1e-6)])
def test_batch_matches_oracle(precision, mc, tol):
    ws = [w.with_(max_cycles=mc) for w in small_instances(3)]
    nsteps = 2
    say(f"case batch-vs-oracle precision={precision} n={len(ws)} grids={[w.grid.nx for w in ws]} "
        f"nsteps={nsteps}")
    solvers = [P.solver_for(w, precision=precision) for w in ws]
    b = V.Batch(solvers, nstreams=8)
    b.step([w.dt for w in ws], nsteps)
    b.close()
    for w, s in zip(ws, solvers):
        got = s.fields()
        s.close()
        g = O.Grid(*w.grid.shape, h=w.grid.h)
        walls = O.Walls(w.wall_kind, w.u0, w.u1)
        p = O.Params(model=w.model, eta=w.eta, mobility=w.mobility, eps=w.eps, kappa=w.kappa,
                     sigma=w.sigma, gamma0=w.gamma0, rate_V=w.rate_V, k_A=w.k_A,
                     bend_scale=w.bend_scale)
        ref = O.run(g, walls, p, w.phi0(), w.dt, nsteps)
        refd = {"phi": ref.phi, "mu": ref.mu}
        for c, ax in enumerate("xyz"):
            refd["omega_" + ax] = ref.omega[c]
            refd["psi_" + ax] = ref.psi[c]
        errs = {k: rel_l2(got[k], refd[k]) for k in FIELD_NAMES}
        say(f"  {w.name} n={w.grid.nx} " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()))
        assert max(errs.values()) <= tol, errs


def test_batch_rejects_odd_steps_and_unstable_dt():
    ws = small_instances(2)
    say(f"case batch-errors n={len(ws)}")
    solvers = [P.solver_for(w) for w in ws]
    b = V.Batch(solvers)
    with pytest.raises(V.VsError) as e:
        b.step([w.dt for w in ws], 3)
    assert e.value.code == V.VS_E_ARG
    with pytest.raises(V.VsError) as e:
        b.step([ws[0].dt, 10.0], 2)
    assert e.value.code == V.VS_E_UNSTABLE
    for dts, n in [([w.dt for w in ws], 0), ([float("nan"), ws[1].dt], 2), ([ws[0].dt, 0.0], 2)]:
        with pytest.raises(V.VsError) as e:
            b.step(dts, n)
        assert e.value.code == V.VS_E_ARG, (dts, n)
    b.close()
    for s in solvers:
        assert s.scalars()["step"] == 0
        s.close()
