"""Discretisation of the implicit subsystem (oracle): parameters, face
limiter, diffusion operator, local analytic solutions, residual and norm.

The implicit subsystem (Algorithm section, step (v); equations
RT-cons_energy, RT-chemical_ionization, RT-cons_radiation) is written in
comoving CGS for pure hydrogen (N_s = 1, species HI):

  state   U = (E, e, n), E comoving radiation energy [erg cm^-3],
          e specific gas energy [erg g^-1] (no hydro, so e = e_c),
          n = n_HI comoving [cm^-3]
  inputs  n_H comoving [cm^-3], src = 4 pi eta comoving [erg cm^-3 s^-1]

Residual (equations gas_residual, chemistry_residual, radiation_residual):
  f_e = e - S_e(U),   f_n = n - S_n(U)
  f_E = E - E^n - dt theta     ( L_{n+1} E   - H_{n+1} E   + src - c kappa_{n+1} E   )
              - dt (1-theta)   ( L_n     E^n - H_n     E^n + src - c kappa_n     E^n )
  kappa_m = sigma_E n / a_m^3 (proper opacity; the residual's "c k E" is c kappa E),
  (L_m E)_P = sum over the 6 faces f=(P,Q) of D_f / (a_m^2 h^2) (E_Q - E_P).

Flux limiter on a face f = (P,Q) (equation limiter, kappa_S = 0), lagged to
the start of the step so both time levels use the same D:
  Ebar = max((E^n_P + E^n_Q)/2, E_floor)
  R    = max(|E^n_Q - E^n_P| / (a_n h Ebar), R_min),  R_min = 1/(a_n L_box)
  kap  = (kappa^n_P + kappa^n_Q)/2
  D    = c (2 kap + R) / (6 kap^2 + 3 kap R + R^2)   [proper cm^2/s]
Boundaries per face: zero-flux (D = 0), periodic (wrap), outflow (ghost
E = E_floor, ghost opacity = the boundary cell's).

Local solutions S_n, S_e (the paper cites analytic solutions of an
O(dt^2)-accurate approximation of the local ODEs for given E without
printing them).  Reading: the local ODEs
  dn/dt = A - B n,   A = alpha_B(T) n_e n_H,  B = alpha_B(T) n_e + Gamma,
      n_e = (n_H - n)/a^3 (proper), Gamma = c K_Gamma max(E,0)/a^3
  de/dt = -2 H e + q, q = (G - Lambda)/rho, rho = m_H n_H/a^3,
      G = c K_G (n/a^3)(max(E,0)/a^3), Lambda = L_rec n_e n_HII + L_ce n_e n_HI + Compton
are discretised by the same two-level theta method as the radiation
equation, with the implicit-level coefficients taken at U (a_{n+1},
H_{n+1}) and the explicit level at U^n (a_n, H_n), and the resulting
relation is solved analytically for the new value with those
coefficients held fixed:
  S_n = (n^n + dt [theta A(U) + (1-theta)(A^n - B^n n^n)]) / (1 + theta dt B(U))
  S_e = (e^n + dt [theta q(U) + (1-theta)(q^n - 2 H_n e^n)]) / (1 + 2 theta dt H_{n+1})
This is second order for theta = 1/2 and first order (backward Euler) for
the default theta = 1.  It keeps the discrete system monotone: c kappa E
with kappa at the implicit level grows with E, so the root is unique and
every absorbed photon is one ionisation (exact photon bookkeeping).  The
exponential solution of the frozen-coefficient ODE does not have this
property: E n(E) ~ E e^{-beta E} falls for beta E > 1, which gives several
roots once a cell's optical depth per step exceeds e.
Temperature T = (gamma-1) mu m_H e / k_B with mu = 1/(1+x), x = 1 - n/n_H
(the printed equations compose to an extra factor gamma-1; the standard
ideal-gas relation is used).  Isothermal runs fix T = T_iso and drop e.

Norm (equation rmsnorm) with per-component weights:
  ||f|| = sqrt( sum_P [(f_E/E_s)^2 + (f_e/e^n)^2 + (f_n/n_H)^2] / (N (N_s+2)) )
  E_s = max(max E^n, dt max src, E_floor); isothermal runs have 2 unknowns/cell.

Time levels: a_n, H_n for the explicit parts and the limiter; a_{n+1},
H_{n+1} for the implicit parts (radiation and local ODEs).

Parity status: the residual, limiter and operator are pinned by closed
forms (limiter limits, Fourier eigenvalues, manufactured solution, budget
identities); S_n/S_e are pinned, through many small steps, against
numerical integration of the local ODE system (first-order convergence at
theta = 1, second order at theta = 1/2) and by exact photon bookkeeping.
The explicit level (theta < 1) is pinned by that second-order rate, by
the two-level photon-energy budget at theta = 0.51 and 0.6, and by the
closed-form amplification of a Fourier mode at theta = 1/2 in an
expanding background.  The theta-method form of S_n/S_e is a reading (the
paper does not print them); the rate-fit coefficients are this project's
definitions (parity unpinned beyond alpha_B at 1e4 K and the Compton
coefficient).  This module is test infrastructure: only the tests, the
smoke check and the benchmark's CPU baseline use it.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

from .constants import C_LIGHT, K_BOLTZ, M_H, GAMMA_ADIABATIC
from . import grey as _grey
from . import rates as _rates
from .cosmology import Cosmology, STATIC

ZEROFLUX, PERIODIC, OUTFLOW = 0, 1, 2
COOL_RECB, COOL_COLLEXC, COOL_COMPTON = 1, 2, 4


@dataclass
class Params:
    dims: tuple
    box: float                    # comoving x edge [cm]; cells are cubes of h = box/nx
    bc: tuple                     # (x-, x+, y-, y+, z-, z+)
    isothermal: bool
    T_iso: float
    grey: dict
    rates: int                    # 0 constant alpha_B, 1 fit
    alphaB_const: float
    cooling: int
    cosmo: Cosmology
    theta: float = 1.0
    E_floor: float = 1.0e-40
    R_min: Optional[float] = None  # None -> 1/(a_n box)
    gamma: float = GAMMA_ADIABATIC
    newton_tol: float = 1.0e-8
    newton_max_it: int = 30
    ls_max_cuts: int = 10
    armijo: float = 1.0e-4

    @property
    def h(self) -> float:
        return self.box / self.dims[0]

    @property
    def ncells(self) -> int:
        return int(np.prod(self.dims))

    @property
    def nvars(self) -> int:
        return 2 if self.isothermal else 3

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


def validate(p: Params):
    if len(p.dims) != 3 or min(p.dims) < 1:
        raise ValueError("dims")
    for d in range(3):
        lo, hi = p.bc[2 * d], p.bc[2 * d + 1]
        if (lo == PERIODIC) != (hi == PERIODIC):
            raise ValueError("periodic boundaries must be paired")
        if lo == PERIODIC and p.dims[d] < 3:
            raise ValueError("periodic dimension needs at least 3 cells")
    if not (0.0 < p.theta <= 1.0):
        raise ValueError("theta must lie in (0, 1]")
    if p.box <= 0:
        raise ValueError("box")


def params_from_workload(w, **overrides) -> Params:
    g = _grey.grey_constants(w.spectrum, w.T_bb, w.hnu0_eV, w.sigma0)
    cos = Cosmology(w.cosmology, w.hubble_h, w.Omega_m, w.Omega_L)
    p = Params(dims=tuple(w.dims), box=w.box_comoving_cm, bc=tuple(w.bc),
               isothermal=bool(w.isothermal), T_iso=w.T_iso, grey=g,
               rates=w.rates, alphaB_const=w.alphaB_const, cooling=w.cooling,
               cosmo=cos, theta=w.theta, newton_tol=w.newton_tol)
    p = replace(p, **overrides)
    validate(p)
    return p


def schedule(p: Params, w):
    """(t0, dt, nsteps) of a workload, in seconds."""
    if w.dt_Myr is not None:
        from .constants import MYR_S
        t0 = 0.0 if p.cosmo.kind == STATIC else p.cosmo.time_of_z(w.z_start)
        return t0, w.dt_Myr * MYR_S, w.nsteps
    t0 = p.cosmo.time_of_z(w.z_start)
    t1 = p.cosmo.time_of_z(w.z_end)
    return t0, (t1 - t0) / w.nsteps, w.nsteps


# ---------------------------------------------------------------------------
# state helpers
# ---------------------------------------------------------------------------
def gas_energy(p: Params, T, x):
    """Specific gas energy for temperature T and ionised fraction x."""
    mu = 1.0 / (1.0 + x)
    return K_BOLTZ * T / ((p.gamma - 1.0) * mu * M_H)


def temperature(p: Params, e, n, nH):
    x = 1.0 - n / nH
    mu = 1.0 / (1.0 + x)
    return (p.gamma - 1.0) * mu * M_H * e / K_BOLTZ


def initial_state(p: Params, nH, x0: float, T0: float, E0: float):
    """Uniform E, ionised fraction x0, temperature T0 (T_iso if isothermal)."""
    T = p.T_iso if p.isothermal else T0
    E = np.full(p.dims, E0, dtype=np.float64)
    n = (1.0 - x0) * np.asarray(nH, dtype=np.float64)
    e = np.full(p.dims, gas_energy(p, T, x0), dtype=np.float64)
    return E, e, n


def source_field(p: Params, photon_rate):
    """src = 4 pi eta [erg cm^-3 s^-1 comoving] from photons/s per cell."""
    return np.asarray(photon_rate, dtype=np.float64) * p.grey["eps_bar"] / p.h ** 3


# ---------------------------------------------------------------------------
# complex-step-safe elementary functions
# ---------------------------------------------------------------------------
def cabs(x):
    """|x| continued analytically from the real axis (sign of the real part)."""
    if np.iscomplexobj(x):
        return x * np.where(x.real < 0, -1.0, 1.0)
    return np.abs(x)


def cmax(x, y):
    """max by real part (branch kept under complex perturbations)."""
    if np.iscomplexobj(x) or np.iscomplexobj(y):
        xr = np.real(x)
        yr = np.real(y)
        return np.where(xr >= yr, x, y)
    return np.maximum(x, y)


# ---------------------------------------------------------------------------
# ghosts, faces and the diffusion operator
# ---------------------------------------------------------------------------
def pad(X, d: int, lo: int, hi: int, ghost_lo, ghost_hi):
    """X with one ghost layer on each side of axis d.

    PERIODIC wraps; OUTFLOW and ZEROFLUX take the given ghost values
    (ZEROFLUX ghosts never enter a result because their faces carry D = 0).
    """
    n = X.shape[d]
    first = np.take(X, [0], axis=d)
    last = np.take(X, [n - 1], axis=d)
    if lo == PERIODIC:
        glo, ghi = last, first
    else:
        glo = np.broadcast_to(ghost_lo, first.shape).astype(X.dtype) if np.ndim(ghost_lo) == 0 \
            else np.asarray(ghost_lo, dtype=X.dtype).reshape(first.shape)
        ghi = np.broadcast_to(ghost_hi, last.shape).astype(X.dtype) if np.ndim(ghost_hi) == 0 \
            else np.asarray(ghost_hi, dtype=X.dtype).reshape(last.shape)
    return np.concatenate([glo, X, ghi], axis=d)


def limiter_D(c, kap, R):
    """Flux-limited diffusion coefficient (equation limiter, kappa_S = 0)."""
    return c * (2.0 * kap + R) / (6.0 * kap * kap + 3.0 * kap * R + R * R)


def face_D(p: Params, En, kap_n, a_n: float, R_min: float):
    """D on every face: list over d of arrays with n_d + 1 faces along axis d.

    Face f along d lies between cell f-1 and cell f (faces 0 and n_d are the
    boundary faces).
    """
    h = p.h
    out = []
    for d in range(3):
        lo, hi = p.bc[2 * d], p.bc[2 * d + 1]
        Ep = pad(En, d, lo, hi, p.E_floor, p.E_floor)
        kfirst = np.take(kap_n, [0], axis=d)
        klast = np.take(kap_n, [kap_n.shape[d] - 1], axis=d)
        kp = pad(kap_n, d, lo, hi, kfirst, klast)
        n = En.shape[d]
        EL = np.take(Ep, np.arange(0, n + 1), axis=d)
        ER = np.take(Ep, np.arange(1, n + 2), axis=d)
        kL = np.take(kp, np.arange(0, n + 1), axis=d)
        kR = np.take(kp, np.arange(1, n + 2), axis=d)
        Ebar = cmax(0.5 * (EL + ER), p.E_floor)
        R = cmax(cabs(ER - EL) / (a_n * h * Ebar), R_min)
        kap = 0.5 * (kL + kR)
        D = limiter_D(C_LIGHT, kap, R)
        sl = [slice(None)] * 3
        if lo == ZEROFLUX:
            sl[d] = 0
            D[tuple(sl)] = 0.0
        if hi == ZEROFLUX:
            sl[d] = n
            D[tuple(sl)] = 0.0
        out.append(D)
    return out


def apply_L(p: Params, cf, E):
    """(L E)_P = sum_f cf_f (E_Q - E_P) with face coefficients cf (list over d)."""
    out = np.zeros_like(E)
    for d in range(3):
        lo, hi = p.bc[2 * d], p.bc[2 * d + 1]
        Ep = pad(E, d, lo, hi, p.E_floor, p.E_floor)
        n = E.shape[d]
        Eup = np.take(Ep, np.arange(2, n + 2), axis=d)
        Edn = np.take(Ep, np.arange(0, n), axis=d)
        cup = np.take(cf[d], np.arange(1, n + 1), axis=d)
        cdn = np.take(cf[d], np.arange(0, n), axis=d)
        out = out + cup * (Eup - E) + cdn * (Edn - E)
    return out


# ---------------------------------------------------------------------------
# per-step context
# ---------------------------------------------------------------------------
@dataclass
class StepContext:
    t_n: float
    dt: float
    a_n: float
    a_1: float
    H_n: float
    H_1: float
    nH: np.ndarray
    src: np.ndarray
    En: np.ndarray
    en: np.ndarray
    nn: np.ndarray
    R_min: float
    D: list = field(default_factory=list)
    cf_n: list = field(default_factory=list)
    cf_1: list = field(default_factory=list)
    E_s: float = 1.0


def make_context(p: Params, t_n, dt, nH, src, En, en, nn, Dfaces=None) -> StepContext:
    cos = p.cosmo
    a_n, a_1 = cos.a(t_n), cos.a(t_n + dt)
    H_n, H_1 = cos.hubble(t_n), cos.hubble(t_n + dt)
    R_min = p.R_min if p.R_min is not None else 1.0 / (a_n * p.box)
    ctx = StepContext(t_n=t_n, dt=dt, a_n=a_n, a_1=a_1, H_n=H_n, H_1=H_1,
                      nH=nH, src=src, En=En, en=en, nn=nn, R_min=R_min)
    kap_n = p.grey["sigma_E"] * nn / a_n ** 3
    ctx.D = face_D(p, En, kap_n, a_n, R_min) if Dfaces is None else Dfaces
    h2 = p.h * p.h
    ctx.cf_n = [D / (a_n * a_n * h2) for D in ctx.D]
    ctx.cf_1 = [D / (a_1 * a_1 * h2) for D in ctx.D]
    ctx.E_s = max(float(np.max(np.real(En))), dt * float(np.max(src)), p.E_floor)
    return ctx


# ---------------------------------------------------------------------------
# local solutions and rates
# ---------------------------------------------------------------------------
def alpha_B(p: Params, T):
    if p.rates == 0:
        return p.alphaB_const + 0.0 * T
    return _rates.alpha_B_fit(T)


def cooling(p: Params, T, ne, nHII, nHI, zp1):
    lam = 0.0 * T
    if p.cooling & COOL_RECB:
        lam = lam + _rates.cool_recB(T) * ne * nHII
    if p.cooling & COOL_COLLEXC:
        lam = lam + _rates.cool_collexc(T) * ne * nHI
    if p.cooling & COOL_COMPTON:
        lam = lam + _rates.cool_compton(T, ne, zp1)
    return lam


def _rates_at(p: Params, E, e, n, nH, a: float, T=None):
    """(A, B, q) of the local ODEs at state (E, e, n) and scale factor a."""
    a3 = a ** 3
    Epos = cmax(E, 0.0)
    if T is None:
        T = (p.T_iso + 0.0 * n) if p.isothermal else temperature(p, e, n, nH)
    ne = (nH - n) / a3
    alpha = alpha_B(p, T)
    A = alpha * ne * nH
    B = alpha * ne + C_LIGHT * p.grey["K_Gamma"] * Epos / a3
    if p.isothermal:
        return A, B, None
    nHI = n / a3
    nHII = (nH - n) / a3
    G = C_LIGHT * p.grey["K_G"] * nHI * Epos / a3
    Lam = cooling(p, T, ne, nHII, nHI, 1.0 / a)
    q = (G - Lam) / (M_H * nH / a3)
    return A, B, q


def local_S(p: Params, ctx: StepContext, E, e, n):
    """(S_n, S_e) at state (E, e, n); S_e is None for isothermal runs."""
    th = p.theta
    dt = ctx.dt
    A, B, q = _rates_at(p, E, e, n, ctx.nH, ctx.a_1)
    num_n = ctx.nn + dt * th * A
    if th < 1.0:
        An, Bn, qn = _rates_at(p, ctx.En, ctx.en, ctx.nn, ctx.nH, ctx.a_n)
        num_n = num_n + dt * (1.0 - th) * (An - Bn * ctx.nn)
    Sn = num_n / (1.0 + th * dt * B)
    if p.isothermal:
        return Sn, None
    num_e = ctx.en + dt * th * q
    if th < 1.0:
        num_e = num_e + dt * (1.0 - th) * (qn - 2.0 * ctx.H_n * ctx.en)
    Se = num_e / (1.0 + 2.0 * th * dt * ctx.H_1)
    return Sn, Se


def f_E(p: Params, ctx: StepContext, E, n):
    """Radiation residual (equation radiation_residual, theta method)."""
    th = p.theta
    dt = ctx.dt
    sE = p.grey["sigma_E"]
    kap_1 = sE * n / ctx.a_1 ** 3
    impl = apply_L(p, ctx.cf_1, E) - ctx.H_1 * E + ctx.src - C_LIGHT * kap_1 * E
    out = E - ctx.En - dt * th * impl
    if th < 1.0:
        kap_n = sE * ctx.nn / ctx.a_n ** 3
        expl = apply_L(p, ctx.cf_n, ctx.En) - ctx.H_n * ctx.En + ctx.src \
            - C_LIGHT * kap_n * ctx.En
        out = out - dt * (1.0 - th) * expl
    return out


def residual(p: Params, ctx: StepContext, E, e, n):
    """(f_E, f_e, f_n); f_e is None for isothermal runs."""
    Sn, Se = local_S(p, ctx, E, e, n)
    fn = n - Sn
    fe = None if Se is None else e - Se
    return f_E(p, ctx, E, n), fe, fn


def norm(p: Params, ctx: StepContext, fE, fe, fn) -> float:
    """Weighted RMS norm (equation rmsnorm)."""
    s = np.sum((np.real(fE) / ctx.E_s) ** 2) + np.sum((np.real(fn) / ctx.nH) ** 2)
    if fe is not None:
        s += np.sum((np.real(fe) / ctx.en) ** 2)
    return float(np.sqrt(s / (p.ncells * p.nvars)))


def admissible(p: Params, ctx: StepContext, E, e, n) -> bool:
    ok = bool(np.all(n >= 0.0) and np.all(n <= ctx.nH))
    if not p.isothermal:
        ok = ok and bool(np.all(e > 0.0))
    return ok
