"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module builds initial phase fields (vesicle and droplet seed shapes), random
shape coefficients and the parameter sets of the named workloads. It holds none of
the method's arithmetic: no operator, chemical potential, boundary table, Poisson
solve or time step lives here. Both the CPU oracle and the HIP library receive the
arrays produced here as plain inputs.
"""
from .shapes import (  # noqa: F401
    GridSpec,
    alm_coefficients,
    real_sph_harm,
    phi_sh_vesicle,
    phi_prolate,
    phi_prolate_sh,
    phi_sphere,
    prolate_axes,
    prolate_area,
)
from .configs import Workload, WORKLOADS, batch_instances, workload  # noqa: F401
