"""Rate coefficients (oracle).

The paper sends the heating, cooling and recombination formulas to the
literature without printing them; it states alpha_B ~ 2.59e-13 cm^3/s for
case-B recombination (verification section).  This project fixes these
definitions (fits as published in the cited literature, hydrogen only):

  case-B recombination (Hui & Gnedin 1997):
      lam = 2 * 157807 K / T
      alpha_B(T) = 2.753e-14 lam^1.5 / (1 + (lam/2.740)^0.407)^2.242  cm^3/s
  case-B recombination cooling (Hui & Gnedin 1997):
      L_rec(T) = 3.435e-30 T lam^1.970 / (1 + (lam/2.250)^0.376)^3.720  erg cm^3/s
      multiplies n_e n_HII
  collisional-excitation cooling (Cen 1992):
      L_ce(T) = 7.5e-19 exp(-118348/T) / (1 + sqrt(T/1e5))  erg cm^3/s
      multiplies n_e n_HI
  Compton cooling off the CMB (derived from Thomson scattering):
      4 sigma_T a_rad k_B T_cmb^4 (T - T_cmb) n_e / (m_e c),  T_cmb = 2.725 (1+z)
All densities proper.  Every function accepts complex arrays so that the
oracle can differentiate by the complex step.
Pins: alpha_B(1e4 K) against the paper's 2.59e-13; the Compton coefficient
against its closed form value 5.6e-36 (tests).  The fit coefficients
themselves are this project's definitions (parity unpinned by the paper).
"""
import numpy as np

from .constants import SIGMA_T, A_RAD, K_BOLTZ, M_E, C_LIGHT, T_CMB0

T_TR_H = 157807.0


def alpha_B_fit(T):
    lam = 2.0 * T_TR_H / T
    return 2.753e-14 * lam ** 1.5 / (1.0 + (lam / 2.740) ** 0.407) ** 2.242


def cool_recB(T):
    lam = 2.0 * T_TR_H / T
    return 3.435e-30 * T * lam ** 1.970 / (1.0 + (lam / 2.250) ** 0.376) ** 3.720


def cool_collexc(T):
    return 7.5e-19 * np.exp(-118348.0 / T) / (1.0 + np.sqrt(T / 1.0e5))


COMPTON_COEFF = 4.0 * SIGMA_T * A_RAD * K_BOLTZ * T_CMB0 ** 4 / (M_E * C_LIGHT)


def cool_compton(T, ne, zp1):
    """Compton cooling rate per unit proper volume [erg cm^-3 s^-1]."""
    return COMPTON_COEFF * zp1 ** 4 * (T - T_CMB0 * zp1) * ne
