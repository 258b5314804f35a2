"""Diagnostics (oracle): I-front radius and conservation budgets.

I-front radius: volume-equivalent radius of the ionised region,
  V_ion = sum_P (x_P - x0)/(1 - x0) h^3 (proper cell volume),
  r_I = (3 V_ion / (4 pi))^(1/3)   (a corner source covers an octant: V x 8).
Photon-energy budget of one backward-Euler step with zero-flux or periodic
walls: the diffusion fluxes telescope, so
  sum (E^{n+1} - E^n) = dt sum (-H_{n+1} E - c kappa E + src)  (theta = 1).
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
    """Relative defect of the discrete photon-energy budget (theta = 1)."""
    kap = p.grey["sigma_E"] * n1 / ctx.a_1 ** 3
    lhs = float(np.sum(E1 - ctx.En))
    rhs = ctx.dt * float(np.sum(-ctx.H_1 * E1 - C_LIGHT * kap * E1 + ctx.src))
    scale = ctx.dt * float(np.sum(np.abs(C_LIGHT * kap * E1) + np.abs(ctx.src)
                                  + np.abs(ctx.H_1 * E1))) + 1e-300
    return abs(lhs - rhs) / scale
