"""MI355X implementation of the coupled implicit radiation step of Norman,
Reynolds & So (arXiv:0908.2654): Newton on the grey flux-limited-diffusion
radiation energy, gas energy and neutral hydrogen over one operator-split
step, with the Schur-complement diffusion system solved by geometric
multigrid in hand-written HIP kernels (librh.so, C ABI in include/rh.h).

Importing the package loads librh.so and fails if it is not built.
"""
from ._lib import RhError, RhParams, RhStepStats, default_params  # noqa: F401
from .solver import Solver, cosmic_time, cosmology_at, params_from_workload, workspace_bytes  # noqa: F401
from .solver import MultigroupSolver, multigroup_constants, multigroup_params  # noqa: F401
