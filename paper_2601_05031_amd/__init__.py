"""MI355X (gfx950) implementation of the vorticity-stream-vector phase-field time step
(arXiv 2601.05031): HIP kernels behind the C ABI of include/vs.h, with a ctypes binding."""
from .vs import (  # noqa: F401
    FIELDS,
    Batch,
    SCALARS,
    Solver,
    VsError,
    lib,
    make_params,
    rollout_gradient,
    rollout_loss,
    set_launch_shapes,
    solver_for,
    workspace_bytes,
)
