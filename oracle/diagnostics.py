"""Diagnostics (oracle): I-front radius and conservation budgets.

I-front radius: volume-equivalent radius of the ionised region,
  V_ion = sum_P (x_P - x0)/(1 - x0) h^3 (proper cell volume),
  r_I = (3 V_ion / (4 pi))^(1/3)   (a corner source covers an octant: V x 8).
Photon-energy budget of one theta step with zero-flux or periodic walls:
the diffusion fluxes telescope at both time levels, so the change of the
total radiation energy is dt times the theta-weighted sum of the Hubble,
absorption and source terms (photon_budget_defect).
"""
import math

import numpy as np

from .constants import C_LIGHT


def ionised_fraction(n, nH):
    return 1.0 - np.asarray(n) / np.asarray(nH)


def front_radius(n, nH, x0, h_proper, corner=False):
    x = ionised_fraction(n, nH)
    V = float(np.sum((x - x0) / (1.0 - x0))) * h_proper ** 3
    if corner:
        V *= 8.0
    return (3.0 * V / (4.0 * math.pi)) ** (1.0 / 3.0)


def photon_budget_defect(p, ctx, E1, n1):
    """Relative defect of the discrete photon-energy budget of one theta
    step with zero-flux or periodic walls, where the diffusion fluxes of
    both time levels telescope:
      sum (E^{n+1} - E^n) = dt sum [ theta (-H_{n+1} E^{n+1} - c kappa_{n+1} E^{n+1} + src)
                                   + (1 - theta) (-H_n E^n - c kappa_n E^n + src) ],
    kappa_m = sigma_E n^m / a_m^3 (radiation_residual summed over the cells)."""
    th = p.theta
    sE = p.grey["sigma_E"]
    kap1 = sE * n1 / ctx.a_1 ** 3
    kapn = sE * ctx.nn / ctx.a_n ** 3
    impl = -ctx.H_1 * E1 - C_LIGHT * kap1 * E1 + ctx.src
    expl = -ctx.H_n * ctx.En - C_LIGHT * kapn * ctx.En + ctx.src
    lhs = float(np.sum(E1 - ctx.En))
    rhs = ctx.dt * (th * float(np.sum(impl)) + (1.0 - th) * float(np.sum(expl)))
    scale = ctx.dt * float(np.sum(th * (np.abs(C_LIGHT * kap1 * E1) + np.abs(ctx.H_1 * E1))
                                  + (1.0 - th) * (np.abs(C_LIGHT * kapn * ctx.En)
                                                  + np.abs(ctx.H_n * ctx.En))
                                  + np.abs(ctx.src))) + 1e-300
    return abs(lhs - rhs) / scale
