"""CPU FP64 oracle of the vorticity-stream-vector phase-field time step.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package. The HIP library never calls it and
shares no code with it; the two meet only in the seeded inputs of ``workloads``.
The reverse (adjoint) step lives in ``oracle.adjoint``.
"""
from .vsref import (  # noqa: F401
    BENDING,
    CAHN_HILLIARD,
    POISEUILLE,
    COUETTE,
    no_body_fields,
    solve_flow,
    Grid,
    Params,
    Walls,
    State,
    lap_mirror,
    grad_mirror,
    lap_interior,
    curl_interior,
    wall_profiles,
    chemical_potential,
    velocity,
    advance_phi,
    vorticity_source,
    poisson_solve,
    volume,
    area,
    multipliers,
    init_state,
    step,
    run,
    bending_energy,
)
