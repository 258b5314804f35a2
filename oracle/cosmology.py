"""Expansion factor a(t) and Hubble rate H(t) (oracle).

a(t) = 1/(1+z) is obtained from the Friedmann equation for the assumed
parameters (Physical Model section).  Closed forms:
  static:     a = 1, H = 0
  EdS (Omega_m = 1):    a = (1.5 H0 t)^(2/3),  H = 2/(3t)
  flat LCDM:  a = (Om/OL)^(1/3) sinh^(2/3)(1.5 sqrt(OL) H0 t),
              H = H0 sqrt(Om a^-3 + OL)
t is cosmic time since a = 0, in seconds.
Pin: both closed forms against numerical integration of the Friedmann
equation (tests).
"""
import math

from .constants import H100_S

STATIC, EDS, FLAT_LCDM = 0, 1, 2


class Cosmology:
    def __init__(self, kind: int, hubble_h: float = 0.7, Omega_m: float = 1.0,
                 Omega_L: float = 0.0):
        self.kind = int(kind)
        self.H0 = hubble_h * H100_S
        self.Om = Omega_m
        self.OL = Omega_L
        if self.kind == EDS and abs(Omega_m - 1.0) > 1e-12:
            raise ValueError("EdS requires Omega_m = 1")
        if self.kind == FLAT_LCDM and abs(Omega_m + Omega_L - 1.0) > 1e-12:
            raise ValueError("flat LCDM requires Omega_m + Omega_L = 1")

    def a(self, t: float) -> float:
        if self.kind == STATIC:
            return 1.0
        if self.kind == EDS:
            return (1.5 * self.H0 * t) ** (2.0 / 3.0)
        s = math.sinh(1.5 * math.sqrt(self.OL) * self.H0 * t)
        return (self.Om / self.OL) ** (1.0 / 3.0) * s ** (2.0 / 3.0)

    def hubble(self, t: float) -> float:
        """H = (da/dt)/a."""
        if self.kind == STATIC:
            return 0.0
        if self.kind == EDS:
            return 2.0 / (3.0 * t)
        a = self.a(t)
        return self.H0 * math.sqrt(self.Om / a ** 3 + self.OL)

    def time_of_a(self, a: float) -> float:
        if self.kind == STATIC:
            raise ValueError("static cosmology has no time-redshift relation")
        if self.kind == EDS:
            return a ** 1.5 / (1.5 * self.H0)
        return 2.0 / (3.0 * math.sqrt(self.OL) * self.H0) * \
            math.asinh(math.sqrt(self.OL / self.Om) * a ** 1.5)

    def time_of_z(self, z: float) -> float:
        return self.time_of_a(1.0 / (1.0 + z))
