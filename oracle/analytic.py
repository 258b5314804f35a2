"""Closed-form and quadrature references (oracle).

Stromgren radius (verification section, equation SG-stromgren_radius):
  r_S = (3 Ndot / (4 pi alpha_B n_H^2))^(1/3)
Static growth of the I-front in a uniform medium (textbook):
  r_I(t) = r_S (1 - exp(-t/t_rec))^(1/3),  t_rec = 1/(alpha_B n_H)
Cosmological I-front (equations SG-solution, SG-tau, SG-F), with
lambda = alpha_B n_H0 / H_0 / (1+z_0) and the integration variable the
scale factor normalised to 1 at z_0:
  r_I/r_S0 = ( lambda e^{-tau(a)} int_1^a e^{tau(b)} [1-2q0+2q0(1+z0)/b]^(-1/2) db )^(1/3)
  tau(a)   = lambda [6 q0^2 (1+z0)^2]^-1 [F(a) - F(1)]
  F(a)     = [2 - 4 q0 - 2 q0 (1+z0)/a] [1 - 2 q0 + 2 q0 (1+z0)/a]^(1/2)
Pins: the photon-counting limit lambda -> 0 and tau(a) = int alpha n_H dt
for q0 = 1/2 (tests).
Fourier decay of one backward-Euler step of a constant-coefficient
periodic diffusion: amplification 1/(1 + dt D (4/h^2) sum_d sin^2(pi k_d/N_d)).
"""
import math

import numpy as np
from scipy import integrate


def stromgren_radius(Ndot, alpha_B, nH):
    return (3.0 * Ndot / (4.0 * math.pi * alpha_B * nH * nH)) ** (1.0 / 3.0)


def static_front(t, Ndot, alpha_B, nH):
    rs = stromgren_radius(Ndot, alpha_B, nH)
    trec = 1.0 / (alpha_B * nH)
    return rs * (1.0 - np.exp(-np.asarray(t) / trec)) ** (1.0 / 3.0)


def sg_F(a, q0, z0):
    u = 2.0 * q0 * (1.0 + z0) / a
    return (2.0 - 4.0 * q0 - u) * math.sqrt(1.0 - 2.0 * q0 + u)


def sg_tau(a, lam, q0, z0):
    return lam / (6.0 * q0 * q0 * (1.0 + z0) ** 2) * (sg_F(a, q0, z0) - sg_F(1.0, q0, z0))


def sg_front(a, lam, q0, z0):
    """r_I / r_S0 at normalised scale factor a >= 1."""
    def integrand(b):
        return math.exp(sg_tau(b, lam, q0, z0)) / math.sqrt(1.0 - 2.0 * q0 + 2.0 * q0 * (1.0 + z0) / b)
    val, _ = integrate.quad(integrand, 1.0, a, epsabs=0.0, epsrel=1e-13, limit=200)
    return (lam * math.exp(-sg_tau(a, lam, q0, z0)) * val) ** (1.0 / 3.0)


def fourier_amplification(dt, D, h, k, dims):
    s = sum(math.sin(math.pi * k[d] / dims[d]) ** 2 for d in range(3))
    return 1.0 / (1.0 + dt * D * 4.0 / (h * h) * s)
