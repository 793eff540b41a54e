"""Launch shapes: every form the autotuner chooses between computes the same step.

The chemical potential's register-marching form (z rows whole in a wave) and the LDS-tile form
sum the same terms in the same order, so the fields agree bit for bit; the other shapes (slab
lengths, block caps, segment layouts) change only the order of partial sums and the segment
elimination, so they agree with the oracle at the FP64 bar. The plane form of the transforms
(both 1D transforms of a direction in one pass over an (x, z) plane in LDS) pairs the z lines
differently (x-rows i, i+1 instead of consecutive interior rows), so it differs from the line
form by rounding only. vs_autotune leaves the state's fields unchanged."""
import numpy as np
import pytest

import oracle as O
from workloads import workload
from workloads.shapes import GridSpec

torch = pytest.importorskip("torch")

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2601_05031_amd as P  # noqa: E402
from paper_2601_05031_amd import vs as V  # noqa: E402

FIELD_NAMES = ["phi", "mu", "omega_x", "omega_y", "omega_z", "psi_x", "psi_y", "psi_z"]
DEFAULT = dict(adv_slab=4, va_maxb=1024, res_maxb=1024, seg_alt=0, mu_kind=0, mu_ni=8, plane=0)


def rel_l2(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def run(w, shapes, nsteps, precision="fp64"):
    P.vs.set_launch_shapes(w.grid.shape + (w.grid.h,), shapes)
    s = P.solver_for(w, precision=precision)
    s.step(w.dt, nsteps)
    f = s.fields()
    s.close()
    return f


# n_z = 64, 128, 256: one, two and four z per lane in the register-marching form; bending and
# Cahn-Hilliard; ragged row groups (ny not a multiple of 2 or 8)
@pytest.mark.parametrize("name,shape", [("vesicle32", (24, 34, 64)), ("vesicle32", (16, 21, 128)),
                                        ("droplet256", (12, 19, 256)), ("droplet256", (24, 26, 128))])
@pytest.mark.parametrize("mu_kind,mu_ni", [(1, 2), (1, 16), (2, 8), (2, 5), (2, 2)])
def test_register_mu_is_bitwise_the_tile_mu(name, shape, mu_kind, mu_ni):
    w = workload(name, grid=GridSpec(*shape), R0=4.0, nsteps=3, max_cycles=1)
    if name == "vesicle32":
        w = w.with_(rate_V=10.0, k_A=1.0)
    print(f"case mu forms {name} {shape} kind={mu_kind} ni={mu_ni}", flush=True)
    ref = run(w, DEFAULT, 3)
    got = run(w, dict(DEFAULT, mu_kind=mu_kind, mu_ni=mu_ni), 3)
    P.vs.set_launch_shapes(w.grid.shape + (w.grid.h,), DEFAULT)
    for k in FIELD_NAMES:
        assert np.array_equal(got[k], ref[k]), k


@pytest.mark.parametrize("shapes", [dict(adv_slab=2, va_maxb=256, res_maxb=4096, seg_alt=1, mu_kind=2, mu_ni=4, plane=0),
                                    dict(adv_slab=8, va_maxb=2048, res_maxb=512, seg_alt=1, mu_kind=1, mu_ni=16, plane=0)])
def test_other_shapes_match_the_oracle(shapes):
    w = workload("vesicle32", grid=GridSpec(32, 32, 64), nsteps=3, max_cycles=1, rate_V=10.0, k_A=1.0)
    print(f"case shapes {shapes}", flush=True)
    got = run(w, shapes, 3)
    P.vs.set_launch_shapes(w.grid.shape + (w.grid.h,), DEFAULT)
    g = O.Grid(*w.grid.shape)
    walls = O.Walls(w.wall_kind, w.u0, w.u1)
    p = O.Params(model=w.model, kappa=w.kappa, eps=w.eps, gamma0=w.gamma0, rate_V=w.rate_V, k_A=w.k_A)
    ref = O.run(g, walls, p, w.phi0(), w.dt, 3)
    refd = {"phi": ref.phi, "mu": ref.mu}
    for c, ax in enumerate("xyz"):
        refd["omega_" + ax] = ref.omega[c]
        refd["psi_" + ax] = ref.psi[c]
    errs = {k: rel_l2(got[k], refd[k]) for k in FIELD_NAMES}
    print("  " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()), flush=True)
    assert max(errs.values()) <= 1e-9, errs


def test_autotune_leaves_the_state_unchanged():
    w = workload("vesicle32", grid=GridSpec(32, 32, 128), nsteps=2, max_cycles=1, rate_V=10.0, k_A=1.0)
    print("case autotune state", flush=True)
    s = P.solver_for(w)
    s.step(w.dt, 2)
    before = s.fields()
    sc0 = s.scalars()
    picks = s.autotune()
    after = s.fields()
    sc1 = s.scalars()
    s.close()
    P.vs.set_launch_shapes(w.grid.shape + (w.grid.h,), DEFAULT)
    print(f"  picks {picks}", flush=True)
    assert picks["adv_slab"] in (2, 4, 8) and picks["mu_kind"] in (0, 1, 2) and picks["plane"] in (0, 1)
    for k in FIELD_NAMES:
        assert np.array_equal(before[k], after[k]), k
    for k in ("V", "A", "V0", "A0", "lambda_V", "gamma_A"):
        assert sc0[k] == sc1[k], k


def oracle_fields(w, nsteps):
    g = O.Grid(*w.grid.shape, h=w.grid.h)
    walls = O.Walls(w.wall_kind, w.u0, w.u1)
    p = O.Params(model=w.model, eta=w.eta, mobility=w.mobility, eps=w.eps, kappa=w.kappa,
                 sigma=w.sigma, gamma0=w.gamma0, rate_V=w.rate_V, k_A=w.k_A, bend_scale=w.bend_scale)
    ref = O.run(g, walls, p, w.phi0(), w.dt, nsteps)
    refd = {"phi": ref.phi, "mu": ref.mu}
    for c, ax in enumerate("xyz"):
        refd["omega_" + ax] = ref.omega[c]
        refd["psi_" + ax] = ref.psi[c]
    return refd


# every plane size (n_x = n_z = 32 .. 128, one to sixteen loads per lane), ragged and tall
# channels, both models and wall kinds; the oracle at the two smallest
@pytest.mark.parametrize("name,shape,oracle", [("vesicle32", (32, 21, 32), True),
                                               ("droplet256", (48, 19, 48), True),
                                               ("vesicle32", (64, 34, 64), False),
                                               ("droplet256", (96, 12, 96), False),
                                               ("vesicle32", (128, 10, 128), False)])
@pytest.mark.parametrize("mc", [1, 3])
def test_plane_transforms_match_line_transforms(name, shape, oracle, mc):
    w = workload(name, grid=GridSpec(*shape), R0=min(shape) / 4.0, nsteps=3, max_cycles=mc)
    if name == "vesicle32":
        w = w.with_(rate_V=10.0, k_A=1.0, wall_kind="couette", u0=-0.03, u1=0.05)
    print(f"case plane {name} {shape} mc={mc}", flush=True)
    ref = run(w, DEFAULT, 3)
    got = run(w, dict(DEFAULT, plane=1), 3)
    P.vs.set_launch_shapes(w.grid.shape + (w.grid.h,), DEFAULT)
    errs = {k: rel_l2(got[k], ref[k]) for k in FIELD_NAMES}
    print("  vs line form " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()), flush=True)
    assert max(errs.values()) <= 1e-12, errs
    if oracle:
        refd = oracle_fields(w, 3)
        errs = {k: rel_l2(got[k], refd[k]) for k in FIELD_NAMES}
        print("  vs oracle " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()), flush=True)
        assert max(errs.values()) <= 1e-9, errs


def test_plane_transforms_in_the_reverse_step():
    w = workload("vesicle32", grid=GridSpec(32, 21, 32), R0=6.0, nsteps=2, max_cycles=1,
                 rate_V=3.0, k_A=0.7, gamma0=0.2)
    print("case plane reverse step", flush=True)
    rng = np.random.default_rng(5)
    a = rng.standard_normal(w.grid.shape)
    outs = []
    for plane in (0, 1):
        P.vs.set_launch_shapes(w.grid.shape + (w.grid.h,), dict(DEFAULT, plane=plane))
        s = P.solver_for(w)
        s.step(w.dt, 2)
        at = torch.tensor(a, device="cuda")
        bt = torch.zeros_like(at)
        kb, sb = s.grad_step(w.dt, at, bt)
        outs.append((bt.cpu().numpy(), kb, sb))
        s.close()
    P.vs.set_launch_shapes(w.grid.shape + (w.grid.h,), DEFAULT)
    (b0, k0, s0), (b1, k1, s1) = outs
    e = rel_l2(b1 - a, b0 - a)
    print(f"  increment {e:.1e} kappa {k0:.15e} {k1:.15e} s {s0:.15e} {s1:.15e}", flush=True)
    assert e <= 1e-12
    assert k1 == pytest.approx(k0, rel=1e-12) and s1 == pytest.approx(s0, rel=1e-12, abs=1e-18)
