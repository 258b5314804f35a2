"""Expansion factor a(t) and Hubble rate H(t) (oracle).

a(t) = 1/(1+z) is obtained from the Friedmann equation for the assumed
parameters (Physical Model section).  Closed forms:
  static:     a = 1, H = 0
  EdS (Omega_m = 1):    a = (1.5 H0 t)^(2/3),  H = 2/(3t)
  flat LCDM:  a = (Om/OL)^(1/3) sinh^(2/3)(1.5 sqrt(OL) H0 t),
              H = H0 sqrt(Om a^-3 + OL)
  open (OL = 0, 0 < Om < 1; the q0 = Om/2 = 0.05 runs of the verification
  section): with Ok = 1 - Om the Friedmann equation H^2 = H0^2 (Om a^-3 +
  Ok a^-2) has the parametric solution
              a = A (cosh eta - 1),  t = B (sinh eta - eta),
              A = Om / (2 Ok),  B = Om / (2 H0 Ok^1.5),
  and a(t) takes the root eta of sinh eta - eta = t / B.
t is cosmic time since a = 0, in seconds.
Pin: every closed form against numerical integration of the Friedmann
equation (tests).
"""
import math

from scipy import optimize

from .constants import H100_S

STATIC, EDS, FLAT_LCDM, OPEN = 0, 1, 2, 3


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
        if self.kind == OPEN:
            if not (0.0 < Omega_m < 1.0) or Omega_L != 0.0:
                raise ValueError("open cosmology requires 0 < Omega_m < 1 and Omega_L = 0")
            Ok = 1.0 - Omega_m
            self._A = Omega_m / (2.0 * Ok)
            self._B = Omega_m / (2.0 * self.H0 * Ok ** 1.5)

    @staticmethod
    def _sinh_minus(eta):
        """sinh(eta) - eta without cancellation at small eta."""
        if eta < 0.1:
            e2 = eta * eta
            return eta * e2 / 6.0 * (1.0 + e2 / 20.0 * (1.0 + e2 / 42.0 * (1.0 + e2 / 72.0)))
        return math.sinh(eta) - eta

    def _eta_of_t(self, t):
        tau = t / self._B
        hi = max(1.0, (6.0 * tau) ** (1.0 / 3.0))
        while self._sinh_minus(hi) < tau:
            hi *= 2.0
        return optimize.brentq(lambda x: self._sinh_minus(x) - tau, 0.0, hi, xtol=1e-300,
                               rtol=4.0 * 2.0 ** -52, maxiter=500)

    def a(self, t: float) -> float:
        if self.kind == STATIC:
            return 1.0
        if self.kind == EDS:
            return (1.5 * self.H0 * t) ** (2.0 / 3.0)
        if self.kind == OPEN:
            eta = self._eta_of_t(t)
            ch = 2.0 * math.sinh(0.5 * eta) ** 2  # cosh(eta) - 1
            return self._A * ch
        s = math.sinh(1.5 * math.sqrt(self.OL) * self.H0 * t)
        return (self.Om / self.OL) ** (1.0 / 3.0) * s ** (2.0 / 3.0)

    def hubble(self, t: float) -> float:
        """H = (da/dt)/a."""
        if self.kind == STATIC:
            return 0.0
        if self.kind == EDS:
            return 2.0 / (3.0 * t)
        a = self.a(t)
        if self.kind == OPEN:
            return self.H0 * math.sqrt(self.Om / a ** 3 + (1.0 - self.Om) / a ** 2)
        return self.H0 * math.sqrt(self.Om / a ** 3 + self.OL)

    def time_of_a(self, a: float) -> float:
        if self.kind == STATIC:
            raise ValueError("static cosmology has no time-redshift relation")
        if self.kind == EDS:
            return a ** 1.5 / (1.5 * self.H0)
        if self.kind == OPEN:
            eta = math.acosh(1.0 + a / self._A)
            return self._B * self._sinh_minus(eta)
        return 2.0 / (3.0 * math.sqrt(self.OL) * self.H0) * \
            math.asinh(math.sqrt(self.OL / self.Om) * a ** 1.5)

    def time_of_z(self, z: float) -> float:
        return self.time_of_a(1.0 / (1.0 + z))
