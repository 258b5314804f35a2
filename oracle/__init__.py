"""FP64 CPU oracle for the coupled implicit radiation step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only the tests, the smoke check of the entry module and the
CPU-baseline leg of the benchmark do.  It shares no code with the HIP path;
the only module both use is ``workloads`` (seeded input generators).

What it computes: one step of the implicit subsystem of the paper's
operator split (Algorithm section, step (v)): the root U^{n+1} =
(E, e, n_HI) of the nonlinear residual made of the gas-energy residual,
the chemistry residual and the two-level theta-method residual of the grey
flux-limited-diffusion equation (equations labelled gas_residual,
chemistry_residual and radiation_residual), with the flux limiter of the
limiter equation and convergence measured in the RMS norm (rmsnorm).

Modules:
  constants   physical constants (CGS)
  grey        grey-spectrum constants of the T_B = 1e5 K blackbody (grey_definition)
  cosmology   expansion factor a(t) and H(t) from the Friedmann equation
  rates       case-B recombination, cooling and photo rates
  model       parameters, face limiter, residual f(U), local solutions, norm
  newton      globalised Newton step with sparse direct linear solves
  adjoint     adjoint of the step (implicit-function theorem, sparse transposes)
  analytic    Stromgren radius and the Shapiro-Giroux I-front law
  diagnostics I-front radius, budgets
  controller  adaptive time steps with the temporal accuracy tau_tol
  advection   donor-cell advection of the step's fields (operator split, step (iv))

Parity status of each function is stated in its module header.
"""
from .constants import *  # noqa: F401,F403
from . import grey, cosmology, rates, model, newton, adjoint, analytic, diagnostics, controller, advection  # noqa: F401
from .model import Params, StepContext, params_from_workload, initial_state, source_field  # noqa: F401
from .newton import step, run  # noqa: F401
