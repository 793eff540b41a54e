"""Pins of the oracle's reverse step (oracle/adjoint.py) to the forward oracle.

Each transposed operator is checked against its forward operator through the identity
<A^T a, b> = <a, A b> on random arrays; the whole reverse step and a checkpointed rollout are
checked against central finite differences of the forward oracle (in phi, kappa and the wall
speed scale s). None of these checks re-types the adjoint's formulas.
"""
import numpy as np
import pytest

import oracle as O
from oracle import adjoint as AD
from workloads.shapes import GridSpec, alm_coefficients, phi_sh_vesicle, phi_sphere

RNG = np.random.default_rng(17)


def dot(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("shape,h", [((6, 7, 8), 1.0), ((5, 4, 6), 0.7)])
def test_transposes_against_forward_operators(shape, h):
    g = O.Grid(*shape, h=h)
    a = RNG.standard_normal(shape)
    b = RNG.standard_normal(shape)
    assert dot(AD.lap_mirror_T(a, g), b) == pytest.approx(dot(a, O.lap_mirror(b, h)), rel=1e-12)
    gb = O.grad_mirror(b, h)
    for c in range(3):
        assert dot(AD.grad_mirror_T(a, c, h), b) == pytest.approx(dot(a, gb[c]), rel=1e-12, abs=1e-12)
    psi = RNG.standard_normal((3,) + shape)
    bi = RNG.standard_normal((3, shape[0], shape[1] - 2, shape[2]))
    lhs = dot(AD.curl_interior_T(bi, h, shape[1]), psi)
    assert lhs == pytest.approx(dot(bi, O.curl_interior(psi, h)), rel=1e-12)


def test_poisson_adjoint_against_forward_solve():
    g = O.Grid(8, 9, 6, h=0.8)
    b = RNG.standard_normal((8, 7, 6))
    lo = RNG.standard_normal((8, 6))
    hi = RNG.standard_normal((8, 6))
    ub = RNG.standard_normal((8, 7, 6))
    u = O.poisson_solve(b, lo, hi, g)
    bb, lob, hib = AD.poisson_adjoint(ub, g)
    assert dot(ub, u) == pytest.approx(dot(bb, b) + dot(lob, lo) + dot(hib, hi), rel=1e-11)


def _case(model, kind):
    g = O.Grid(12, 11, 14, 1.0)
    gs = GridSpec(12, 11, 14)
    if kind == O.POISEUILLE:
        walls = O.Walls(kind, 0.05, 0.0)
    else:
        walls = O.Walls(kind, -0.04, 0.06)
    if model == O.BENDING:
        p = O.Params(model=model, kappa=1.3, gamma0=0.2, rate_V=3.0, k_A=0.7, eta=1.2,
                     mobility=0.9)
        phi0 = phi_sh_vesicle(gs, 3.5, alm_coefficients(3, 0.05), np.sqrt(2.0))
    else:
        p = O.Params(model=model, sigma=1.1, rate_V=2.0, eta=0.8)
        phi0 = phi_sphere(gs, 3.2, np.sqrt(2.2))
    return g, walls, p, phi0


def _level_state(phi, g, walls, p, V0, A0):
    """The level-n state as the forward step leaves it, rebuilt from phi alone (R9)."""
    V = O.volume(phi, g)
    A = O.area(phi, g, p.eps)
    lam, gam = O.multipliers(V, A, V0, A0, g, p)
    mu = O.chemical_potential(phi, g, p, gam)
    om, ps = O.solve_flow(phi, mu, g, walls, p)
    return O.State(phi, mu, om, ps, V0, A0, V, A, lam, gam, 0)


@pytest.mark.parametrize("model", [O.BENDING, O.CAHN_HILLIARD])
@pytest.mark.parametrize("kind", [O.POISEUILLE, O.COUETTE])
def test_reverse_step_matches_finite_differences(model, kind):
    g, walls, p, phi0 = _case(model, kind)
    dt = 1e-3
    s0 = O.init_state(g, walls, p, phi0)
    s = O.step(s0, dt, g, walls, p)                 # lambda_V, gamma_A away from their start
    a = RNG.standard_normal(g.shape)
    dphi = RNG.standard_normal(g.shape)
    pb, kb, sb = AD.grad_step(s, a, dt, g, walls, p)

    def J(phi, pp, sc):
        ww = AD.scaled_walls(walls, sc)
        st = _level_state(phi, g, ww, pp, s0.V0, s0.A0)
        return dot(a, O.step(st, dt, g, ww, pp).phi - phi)

    e = 1e-6
    fd = (J(s.phi + e * dphi, p, 1.0) - J(s.phi - e * dphi, p, 1.0)) / (2 * e) + dot(a, dphi)
    assert dot(pb, dphi) == pytest.approx(fd, rel=1e-7)
    e = 1e-4
    fds = (J(s.phi, p, 1.0 + e) - J(s.phi, p, 1.0 - e)) / (2 * e)
    assert sb == pytest.approx(fds, rel=1e-6)
    if model == O.BENDING:
        pk = lambda k: O.Params(**{**p.__dict__, "kappa": k})  # noqa: E731
        fdk = (J(s.phi, pk(p.kappa + e), 1.0) - J(s.phi, pk(p.kappa - e), 1.0)) / (2 * e)
        assert kb == pytest.approx(fdk, rel=1e-6)
    else:
        assert kb == 0.0


def test_rollout_gradient_and_checkpoints():
    g, walls, p, phi0 = _case(O.BENDING, O.POISEUILLE)
    dt, n = 1e-3, 6
    target = O.run(g, walls, O.Params(**{**p.__dict__, "kappa": 1.5}), phi0, dt, n).phi
    L, kb, sb, _ = AD.rollout_gradient(g, walls, p, phi0, dt, n, target)
    L2, kb2, sb2, _ = AD.rollout_gradient(g, walls, p, phi0, dt, n, target, checkpoint_every=4)
    assert (L2, kb2, sb2) == (L, kb, sb)

    def loss(kappa, sc):
        pp = O.Params(**{**p.__dict__, "kappa": kappa})
        r = O.run(g, AD.scaled_walls(walls, sc), pp, phi0, dt, n).phi - target
        return float(np.sum(r * r))

    e = 1e-4
    assert kb == pytest.approx((loss(p.kappa + e, 1.0) - loss(p.kappa - e, 1.0)) / (2 * e), rel=1e-5)
    assert sb == pytest.approx((loss(p.kappa, 1.0 + e) - loss(p.kappa, 1.0 - e)) / (2 * e), rel=1e-5)
