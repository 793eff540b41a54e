"""Write the oracle regression fixture oracle_small.json from the CPU oracle alone.

The paper prints no worked numerical example, so the oracle's pins are closed forms, library
routines and brute force (tests/test_oracle_*.py). This fixture records what the pinned
oracle computes for one small seeded case, so that a later change to the oracle's arithmetic
shows up as a difference. Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from workloads import workload  # noqa: E402
from workloads.shapes import GridSpec  # noqa: E402

# a bending vesicle with both penalties in plane Poiseuille flow, and a Cahn-Hilliard droplet
# in plane Couette flow, on small non-cubic grids; two steps each
CASES = {
    "bending_poiseuille": dict(name="vesicle32", grid=(12, 14, 16), R0=4.0, rate_V=10.0, k_A=1.0,
                               gamma0=0.1),
    "ch_couette": dict(name="droplet256", grid=(16, 12, 10), R0=3.5),
}
NSTEPS = 2
# sampled nodes (i, j, k) of every field
NODES = [(0, 0, 0), (3, 1, 5), (6, 5, 7), (11, 10, 9), (5, 7, 2)]


def case_workload(spec):
    kw = {k: v for k, v in spec.items() if k not in ("name", "grid")}
    return workload(spec["name"], grid=GridSpec(*spec["grid"]), **kw)


def oracle_run(w):
    g = O.Grid(*w.grid.shape, h=w.grid.h)
    walls = O.Walls(w.wall_kind, w.u0, w.u1)
    p = O.Params(model=w.model, eta=w.eta, mobility=w.mobility, eps=w.eps, kappa=w.kappa,
                 sigma=w.sigma, gamma0=w.gamma0, rate_V=w.rate_V, k_A=w.k_A,
                 bend_scale=w.bend_scale)
    return O.run(g, walls, p, w.phi0(), w.dt, NSTEPS)


def summary(s):
    fields = {"phi": s.phi, "mu": s.mu}
    for c, ax in enumerate("xyz"):
        fields["omega_" + ax] = s.omega[c]
        fields["psi_" + ax] = s.psi[c]
    out = {"scalars": {"V": s.V, "A": s.A, "V0": s.V0, "A0": s.A0, "lambda_V": s.lam_V,
                       "gamma_A": s.gamma_A}}
    for k, f in fields.items():
        out[k] = {"l2": float(np.linalg.norm(f)), "sum": float(f.sum()),
                  "samples": [float(f[n]) for n in NODES if all(a < b for a, b in zip(n, f.shape))]}
    return out


def main():
    data = {"source": "tests/golden/make_golden.py (CPU oracle only)", "nsteps": NSTEPS,
            "nodes": NODES, "cases": {}}
    for name, spec in CASES.items():
        data["cases"][name] = {"spec": spec, "result": summary(oracle_run(case_workload(spec)))}
    with open(os.path.join(HERE, "oracle_small.json"), "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
