"""Grey-spectrum constants (oracle).

The grey radiation energy is the integral of the frequency-dependent energy
from the hydrogen threshold h nu_0 = 13.6 eV upward with a fixed spectral
shape chi_E(nu), a T_B = 1e5 K blackbody (Physical Model section,
equation grey_definition).  The paper fixes the shape but not sigma(nu) nor
the weighting; this oracle reads them as: sigma(nu) = sigma_0 (nu_0/nu)^3,
opacity energy-weighted, photoionisation photon-weighted, heating = absorbed
energy minus threshold energy per ionisation (exact energy bookkeeping).

With x = h nu/(k T_B), x0 = h nu_0/(k T_B):
  I_E   = int_x0^inf x^3/(e^x-1) dx        I_N  = int_x0^inf x^2/(e^x-1) dx
  I_sE  = x0^3 int_x0^inf 1/(e^x-1) dx     I_sN = x0^3 int_x0^inf 1/(x(e^x-1)) dx
  sigma_E = sigma_0 I_sE / I_E             (energy-weighted cross-section)
  K_Gamma = sigma_0 I_sN / (k T_B I_E)     (Gamma = c K_Gamma E_proper)
  K_G     = sigma_E - h nu_0 K_Gamma       (G = c K_G n_HI E, proper)
  eps_bar = k T_B I_E / I_N                (mean photon energy of the spectrum)
The integrals are evaluated by adaptive quadrature (the definitions).
Pins: closed forms and series for all four integrals (tests).
A monochromatic source at nu_0 gives sigma_E = sigma_0, K_Gamma =
sigma_0/(h nu_0), K_G = 0, eps_bar = h nu_0.
"""
import numpy as np
from scipy import integrate

from .constants import K_BOLTZ, EV_ERG


def _tail_integral(fun, x0):
    val, _ = integrate.quad(fun, x0, np.inf, epsabs=0.0, epsrel=2e-14, limit=400)
    return val


def blackbody_integrals(x0: float):
    """(I_E, I_N, I_sE, I_sN) by quadrature of their defining integrals."""
    def bose(x):  # 1/(e^x - 1) without overflow for large x
        return np.exp(-x) / -np.expm1(-x)
    I_E = _tail_integral(lambda x: x ** 3 * bose(x), x0)
    I_N = _tail_integral(lambda x: x ** 2 * bose(x), x0)
    I_sE = x0 ** 3 * _tail_integral(bose, x0)
    I_sN = x0 ** 3 * _tail_integral(lambda x: bose(x) / x, x0)
    return I_E, I_N, I_sE, I_sN


def grey_constants(spectrum: int, T_bb: float, hnu0_eV: float, sigma0: float):
    """Return dict(sigma_E, K_Gamma, K_G, eps_bar, hnu0) in CGS.

    spectrum 0 = monochromatic at h nu_0, 1 = blackbody at T_bb.
    """
    hnu0 = hnu0_eV * EV_ERG
    if spectrum == 0:
        return dict(sigma_E=sigma0, K_Gamma=sigma0 / hnu0, K_G=0.0,
                    eps_bar=hnu0, hnu0=hnu0)
    kT = K_BOLTZ * T_bb
    x0 = hnu0 / kT
    I_E, I_N, I_sE, I_sN = blackbody_integrals(x0)
    sigma_E = sigma0 * I_sE / I_E
    K_Gamma = sigma0 * I_sN / (kT * I_E)
    K_G = sigma_E - hnu0 * K_Gamma
    eps_bar = kT * I_E / I_N
    return dict(sigma_E=sigma_E, K_Gamma=K_Gamma, K_G=K_G, eps_bar=eps_bar, hnu0=hnu0)
