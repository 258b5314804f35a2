"""Hydrogen + helium chemistry with multigroup flux-limited diffusion (oracle).

TEST INFRASTRUCTURE ONLY (like the rest of this package).

The paper evolves a grey radiation energy obtained by integrating the
multi-frequency FLD equation (equation cons_radiation_multifreq) over
frequencies above the hydrogen threshold with a prescribed spectral shape
(equation grey_definition), for pure hydrogen; it gives the electron
density with helium (equation electron_density, second branch) and names
multigroup FLD with helium ionisation as the first extension under
development (Conclusions and outlook).  This module is that extension,
built from the same equations with the readings below (none is printed in
the paper; all are this project's definitions):

Groups.  G groups between lower edges nu_0 = edges[0] < edges[1] < ... (the
last extends to infinity).  Within each group the spectrum keeps the
T_B blackbody shape (the grey reading, applied per group); E_g is the
group's comoving energy density.  With x = h nu / (k T_B) and
b(x) = 1 / (e^x - 1):
  I_g      = int_g x^3 b dx                      (group energy)
  f_g      = I_g / sum_h I_h                     (source energy fraction)
  sigma_E,s,g = int_g sigma_s x^3 b dx / I_g      (energy-weighted)
  K_Gam,s,g   = int_g sigma_s x^2 b dx / (k T_B I_g)   (Gamma_s = c sum_g K_Gam,s,g E_g)
  K_G,s,g     = sigma_E,s,g - h nu_s K_Gam,s,g     (heating: absorbed minus threshold)
with sigma_s(nu) = sigma_s0 (nu_s / nu)^p above the species threshold nu_s
(p = 3 by default), for HI (the run's h nu_0 and sigma_0), HeI (24.587 eV,
7.42e-18 cm^2) and HeII (hydrogenic: 4 h nu_0, sigma_0 / 4).  The source
splits as src_g = f_g src (src from photon rates with the whole spectrum's
mean photon energy, as in the grey case).  One group and no helium give
exactly the grey constants.

Species.  n_H, n_He = y_He n_H (comoving, fixed); unknowns n_HI, n_HeI,
n_HeII; n_HII = n_H - n_HI, n_HeIII = n_He - n_HeI - n_HeII.  Electron
density (equation electron_density, helium branch, whose 1/4 and 1/2
convert helium mass densities in units of m_H to number densities):
n_e = n_HII + n_HeII + 2 n_HeIII.  Mass density rho = m_H (n_H + 4 n_He);
mean molecular weight mu = (n_H + 4 n_He) / (n_H + n_He + n_e);
T = (gamma - 1) mu m_H e / k_B (the hydrogen-only reading generalised).

Chemistry (equation chemical_ionization per species; proper densities in
the rates, comoving unknowns):
  dn_HI/dt   = alpha_H n_e n_HII - Gamma_HI n_HI
  dn_HeI/dt  = alpha_HeII n_e n_HeII - Gamma_HeI n_HeI
  dn_HeII/dt = Gamma_HeI n_HeI - (Gamma_HeII + alpha_HeII n_e) n_HeII
               + alpha_HeIII n_e n_HeIII
i.e. dy/dt = a - M y for y = (n_HI, n_HeI, n_HeII) with
  a = (alpha_H n_e n_H, 0, alpha_HeIII n_e n_He),
  M = [[alpha_H n_e + Gamma_HI, 0, 0],
       [0, Gamma_HeI, -alpha_HeII n_e],
       [0, alpha_HeIII n_e - Gamma_HeI, Gamma_HeII + (alpha_HeII + alpha_HeIII) n_e]].
Recombination: alpha_H the case-B fit of the hydrogen-only model;
alpha_HeII = 1.26e-14 lam^0.75 cm^3/s, lam = 2 * 285335 K / T (case B,
HeII -> HeI); alpha_HeIII(T) = 2 alpha_H(T/4) (hydrogenic ion, Z = 2).
Gas energy: de/dt = -2 H e + (G - Lambda) / rho with heating
G = c sum_s sum_g K_G,s,g n_s E_g (proper) and cooling: the hydrogen-only
set (with the full n_e) plus helium recombination cooling
k_B T alpha_HeII n_e n_HeII and 8 L_recB(T/4) n_e n_HeIII (hydrogenic
scaling of the hydrogen case-B cooling); no helium collisional cooling.

Discretisation: the hydrogen-only step's, per group and per species: the
theta-method radiation residual per group with the group's opacity
kappa_g = sum_s sigma_E,s,g n_s / a^3, the flux limiter per group lagged to
(E_g^n, kappa_g^n); no energy exchange between groups (the grey reading of
the Hubble term, -H E_g, per group); the local solutions by the theta
method with coefficients frozen at U (implicit level) and U^n (explicit):
  (I + theta dt M(U)) S = y^n + dt [theta a(U) + (1 - theta)(a^n - M^n y^n)]
  S_e as in the hydrogen-only model with the multigroup q.
Norm: the RMS norm over all unknowns, weights E_s,g (per group, as E_s),
e^n, n_H for HI and n_He for the helium species.

Solver (oracle only): Newton on the group energies with the local unknowns
re-solved per cell at each trial (the hydrogen-only globalisation); the
Newton direction from the full sparse Jacobian (complex step, colouring of
the 7-point stencil), solved directly.  After the local re-solve this is
the Schur direction of the paper's elimination.
Parity pins (tests): group constants against series; one group without
helium equals the grey step; groups with a flat cross-section sum to the
grey step; exact energy conservation (radiation + gas + ionisation energy)
without recombination or cooling; per-group photon budgets; convergence to
the local ODE system at first (theta = 1) and second (theta = 1/2) order.
Parity unpinned by the paper: every helium rate, cross-section and the
group structure.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy import integrate

from . import model as M
from . import rates as R
from .constants import C_LIGHT, EV_ERG, K_BOLTZ, M_H
from .newton import NewtonFailure, stencil_colours, stencil_neighbours

HEI_EV, HEI_SIGMA0 = 24.587, 7.42e-18
T_TR_HEI = 285335.0


@dataclass
class MGParams:
    base: M.Params                  # grid, walls, cosmology, theta, floors, Newton settings
    edges_eV: tuple = (13.6,)       # lower group edges (first = the hydrogen threshold)
    y_he: float = 0.0               # n_He / n_H
    T_bb: float = 1.0e5
    sigma_power: float = 3.0
    recombination: bool = True      # False: every alpha = 0 (pins)
    groups: dict = field(default_factory=dict)

    @property
    def G(self) -> int:
        return len(self.edges_eV)

    @property
    def he(self) -> bool:
        return self.y_he > 0.0

    @property
    def nloc(self) -> int:
        """local unknowns per cell: (e,) n_HI (, n_HeI, n_HeII)"""
        return (0 if self.base.isothermal else 1) + 1 + (2 if self.he else 0)

    @property
    def nvars(self) -> int:
        return self.G + self.nloc


def _bose(x):
    return np.exp(-x) / -np.expm1(-x)


def _quad(f, a, b):
    val, _ = integrate.quad(f, a, b, epsabs=0.0, epsrel=2e-14, limit=400)
    return val


def group_constants(edges_eV, T_bb, sigma0, hnu0_eV, power=3.0):
    """Per-group constants: dict with frac[g], sigE[s][g], KGam[s][g], KG[s][g]
    (s = 0 HI, 1 HeI, 2 HeII) and eps_bar, by quadrature of the defining
    integrals."""
    kT = K_BOLTZ * T_bb
    xe = [e * EV_ERG / kT for e in edges_eV] + [np.inf]
    G = len(edges_eV)
    thr = [hnu0_eV * EV_ERG / kT, HEI_EV * EV_ERG / kT, 4.0 * hnu0_eV * EV_ERG / kT]
    sig0 = [sigma0, HEI_SIGMA0, sigma0 / 4.0]
    I = np.array([_quad(lambda x: x ** 3 * _bose(x), xe[g], xe[g + 1]) for g in range(G)])
    sigE = np.zeros((3, G))
    KGam = np.zeros((3, G))
    for s in range(3):
        xs = thr[s]
        for g in range(G):
            lo, hi = max(xe[g], xs), xe[g + 1]
            if lo >= hi:
                continue
            sE = _quad(lambda x: (xs / x) ** power * x ** 3 * _bose(x), lo, hi)
            sN = _quad(lambda x: (xs / x) ** power * x ** 2 * _bose(x), lo, hi)
            sigE[s, g] = sig0[s] * sE / I[g]
            KGam[s, g] = sig0[s] * sN / (kT * I[g])
    hnu = np.array(thr) * kT
    KG = sigE - hnu[:, None] * KGam
    I_all = _quad(lambda x: x ** 3 * _bose(x), xe[0], np.inf)
    N_all = _quad(lambda x: x ** 2 * _bose(x), xe[0], np.inf)
    return dict(frac=I / I.sum(), sigE=sigE, KGam=KGam, KG=KG, hnu=hnu,
                eps_bar=kT * I_all / N_all, I=I)


def make_params(base: M.Params, edges_eV=(13.6,), y_he=0.0, T_bb=1.0e5, sigma_power=3.0,
                recombination=True) -> MGParams:
    if abs(edges_eV[0] * EV_ERG - base.grey["hnu0"]) > 1e-9 * base.grey["hnu0"]:
        raise ValueError("the first group edge must be the hydrogen threshold")
    if any(b <= a for a, b in zip(edges_eV, edges_eV[1:])):
        raise ValueError("group edges must increase")
    sigma0 = base.grey["sigma0"]
    mp = MGParams(base=base, edges_eV=tuple(edges_eV), y_he=float(y_he), T_bb=T_bb,
                  sigma_power=sigma_power, recombination=recombination)
    mp.groups = group_constants(edges_eV, T_bb, sigma0, edges_eV[0], sigma_power)
    return mp


def params_from_workload(w, edges_eV=(13.6,), y_he=0.0, **over) -> MGParams:
    base = M.params_from_workload(w, **over)
    base.grey["sigma0"] = w.sigma0
    return make_params(base, edges_eV, y_he, w.T_bb)


# ---------------------------------------------------------------------------
# state, context
# ---------------------------------------------------------------------------
def initial_state(mp: MGParams, nH, x0, T0, E0):
    """E_g = f_g E0, n_HI = (1 - x0) n_H, helium neutral to the same
    fraction (n_HeI = (1 - x0) n_He, n_HeII = x0 n_He), e from T0."""
    p = mp.base
    nH = np.asarray(nH, dtype=np.float64)
    nHe = mp.y_he * nH
    E = np.stack([np.full(p.dims, f * E0) for f in mp.groups["frac"]])
    y = np.stack([(1.0 - x0) * nH, (1.0 - x0) * nHe, x0 * nHe])
    T = p.T_iso if p.isothermal else T0
    ne = x0 * nH + x0 * nHe
    mu = (nH + 4.0 * nHe) / (nH + nHe + ne)
    e = K_BOLTZ * T / ((p.gamma - 1.0) * mu * M_H) * np.ones(p.dims)
    return E, e, y


@dataclass
class Ctx:
    t_n: float
    dt: float
    a_n: float
    a_1: float
    H_n: float
    H_1: float
    nH: np.ndarray
    nHe: np.ndarray
    src: np.ndarray
    En: np.ndarray
    en: np.ndarray
    yn: np.ndarray
    cf_n: list
    cf_1: list
    E_s: np.ndarray


def opacity(mp: MGParams, y, a):
    """kappa_g (proper) for each group from the species densities y."""
    sE = mp.groups["sigE"]
    return np.stack([sum(sE[s, g] * y[s] for s in range(3)) / a ** 3 for g in range(mp.G)])


def make_context(mp: MGParams, t_n, dt, nH, src, En, en, yn) -> Ctx:
    p = mp.base
    cos = p.cosmo
    a_n, a_1 = cos.a(t_n), cos.a(t_n + dt)
    H_n, H_1 = cos.hubble(t_n), cos.hubble(t_n + dt)
    R_min = p.R_min if p.R_min is not None else 1.0 / (a_n * p.box)
    kap_n = opacity(mp, yn, a_n)
    h2 = p.h * p.h
    cf_n, cf_1 = [], []
    for g in range(mp.G):
        D = M.face_D(p, En[g], kap_n[g], a_n, R_min)
        cf_n.append([Dd / (a_n * a_n * h2) for Dd in D])
        cf_1.append([Dd / (a_1 * a_1 * h2) for Dd in D])
    srcg = np.stack([f * src for f in mp.groups["frac"]])
    E_s = np.array([max(float(np.max(np.real(En[g]))), dt * float(np.max(srcg[g])), p.E_floor)
                    for g in range(mp.G)])
    return Ctx(t_n=t_n, dt=dt, a_n=a_n, a_1=a_1, H_n=H_n, H_1=H_1, nH=nH, nHe=mp.y_he * nH,
               src=srcg, En=En, en=en, yn=yn, cf_n=cf_n, cf_1=cf_1, E_s=E_s)


# ---------------------------------------------------------------------------
# rates and local solutions
# ---------------------------------------------------------------------------
def alpha_HeII(T):
    lam = 2.0 * T_TR_HEI / T
    return 1.26e-14 * lam ** 0.75


def alpha_HeIII(mp, T):
    return 2.0 * M.alpha_B(mp.base, T / 4.0)


def _rates(mp: MGParams, ctx: Ctx, E, e, y, a):
    """(avec, Mmat, q) of the local ODEs at state (E, e, y) and scale factor a."""
    p = mp.base
    nH, nHe = ctx.nH, ctx.nHe
    a3 = a ** 3
    nHI, nHeI, nHeII = y[0], y[1], y[2]
    nHII = nH - nHI
    nHeIII = nHe - nHeI - nHeII
    ne_c = nHII + nHeII + 2.0 * nHeIII
    ne = ne_c / a3
    if p.isothermal:
        T = p.T_iso + 0.0 * nHI
    else:
        mu = (nH + 4.0 * nHe) / (nH + nHe + ne_c)
        T = (p.gamma - 1.0) * mu * M_H * e / K_BOLTZ
    rec = 1.0 if mp.recombination else 0.0
    aH = rec * M.alpha_B(p, T)
    aHeII = rec * alpha_HeII(T) if mp.he else 0.0 * T
    aHeIII = rec * alpha_HeIII(mp, T) if mp.he else 0.0 * T
    KGam = mp.groups["KGam"]
    Ep = [M.cmax(E[g], 0.0) / a3 for g in range(mp.G)]
    Gam = [C_LIGHT * sum(KGam[s, g] * Ep[g] for g in range(mp.G)) for s in range(3)]
    avec = [aH * ne * nH, 0.0 * nHI, aHeIII * ne * nHe]
    Mm = [[aH * ne + Gam[0], 0.0 * nHI, 0.0 * nHI],
          [0.0 * nHI, Gam[1], -aHeII * ne],
          [0.0 * nHI, aHeIII * ne - Gam[1], Gam[2] + (aHeII + aHeIII) * ne]]
    q = None
    if not p.isothermal:
        KG = mp.groups["KG"]
        heat = C_LIGHT * sum(KG[s, g] * (y[s] / a3) * Ep[g] for s in range(3) for g in range(mp.G))
        lam = M.cooling(p, T, ne, nHII / a3, nHI / a3, 1.0 / a)
        if mp.he and (p.cooling & M.COOL_RECB):
            lam = lam + K_BOLTZ * T * aHeII * ne * nHeII / a3 \
                + rec * 8.0 * R.cool_recB(T / 4.0) * ne * nHeIII / a3
        q = (heat - lam) / (M_H * (nH + 4.0 * nHe) / a3)
    return avec, Mm, q


def local_S(mp: MGParams, ctx: Ctx, E, e, y):
    """(S_y (3 x dims), S_e) at state (E, e, y): the theta-method local
    solutions with coefficients frozen at U (and at U^n for the explicit part)."""
    p = mp.base
    th, dt = p.theta, ctx.dt
    a1, M1, q1 = _rates(mp, ctx, E, e, y, ctx.a_1)
    rhs = [ctx.yn[s] + dt * th * a1[s] for s in range(3)]
    if th < 1.0:
        a0, M0, q0 = _rates(mp, ctx, ctx.En, ctx.en, ctx.yn, ctx.a_n)
        for s in range(3):
            r = a0[s] - sum(M0[s][k] * ctx.yn[k] for k in range(3))
            rhs[s] = rhs[s] + dt * (1.0 - th) * r
    c = th * dt
    S0 = rhs[0] / (1.0 + c * M1[0][0])
    a11, a12 = 1.0 + c * M1[1][1], c * M1[1][2]
    a21, a22 = c * M1[2][1], 1.0 + c * M1[2][2]
    det = a11 * a22 - a12 * a21
    S1 = (a22 * rhs[1] - a12 * rhs[2]) / det
    S2 = (-a21 * rhs[1] + a11 * rhs[2]) / det
    Se = None
    if not p.isothermal:
        num = ctx.en + dt * th * q1
        if th < 1.0:
            num = num + dt * (1.0 - th) * (q0 - 2.0 * ctx.H_n * ctx.en)
        Se = num / (1.0 + 2.0 * th * dt * ctx.H_1)
    return np.stack([S0, S1, S2]), Se


def f_E(mp: MGParams, ctx: Ctx, E, y):
    """Radiation residual of every group (theta method)."""
    p = mp.base
    th, dt = p.theta, ctx.dt
    k1 = opacity(mp, y, ctx.a_1)
    out = []
    for g in range(mp.G):
        impl = M.apply_L(p, ctx.cf_1[g], E[g]) - ctx.H_1 * E[g] + ctx.src[g] - C_LIGHT * k1[g] * E[g]
        r = E[g] - ctx.En[g] - dt * th * impl
        if th < 1.0:
            kn = opacity(mp, ctx.yn, ctx.a_n)
            expl = M.apply_L(p, ctx.cf_n[g], ctx.En[g]) - ctx.H_n * ctx.En[g] + ctx.src[g] \
                - C_LIGHT * kn[g] * ctx.En[g]
            r = r - dt * (1.0 - th) * expl
        out.append(r)
    return np.stack(out)


def residual(mp: MGParams, ctx: Ctx, E, e, y):
    """(f_E (G x dims), f_e or None, f_y (3 x dims))."""
    Sy, Se = local_S(mp, ctx, E, e, y)
    fy = y - Sy
    fe = None if Se is None else e - Se
    return f_E(mp, ctx, E, y), fe, fy


def norm(mp: MGParams, ctx: Ctx, fE, fe, fy) -> float:
    p = mp.base
    s = sum(np.sum((np.real(fE[g]) / ctx.E_s[g]) ** 2) for g in range(mp.G))
    s += np.sum((np.real(fy[0]) / ctx.nH) ** 2)
    if mp.he:
        s += np.sum((np.real(fy[1]) / ctx.nHe) ** 2) + np.sum((np.real(fy[2]) / ctx.nHe) ** 2)
    if fe is not None:
        s += np.sum((np.real(fe) / ctx.en) ** 2)
    return float(np.sqrt(s / (p.ncells * mp.nvars)))


# ---------------------------------------------------------------------------
# local solve
# ---------------------------------------------------------------------------
def _pack_loc(mp, e, y):
    parts = [] if mp.base.isothermal else [e]
    parts.append(y[0])
    if mp.he:
        parts += [y[1], y[2]]
    return np.stack(parts)


def _unpack_loc(mp, z, e_fixed, ctx):
    i = 0
    if mp.base.isothermal:
        e = e_fixed
    else:
        e = z[0]
        i = 1
    zero = 0.0 * z[i]
    if mp.he:
        y = np.stack([z[i], z[i + 1], z[i + 2]])
    else:
        y = np.stack([z[i], zero, zero])
    return e, y


def _floc(mp, ctx, E, z, e_fixed):
    e, y = _unpack_loc(mp, z, e_fixed, ctx)
    Sy, Se = local_S(mp, ctx, E, e, y)
    parts = [] if mp.base.isothermal else [e - Se]
    parts.append(y[0] - Sy[0])
    if mp.he:
        parts += [y[1] - Sy[1], y[2] - Sy[2]]
    return np.stack(parts)


def _loc_scales(mp, ctx):
    sc = [] if mp.base.isothermal else [ctx.en]
    sc.append(ctx.nH)
    if mp.he:
        sc += [ctx.nHe, ctx.nHe]
    return np.stack(sc)


def local_solve(mp: MGParams, ctx: Ctx, E, e_init, y_init, tol=1e-15, max_it=100):
    """Per-cell root of the local equations at fixed E (damped Newton with
    complex-step Jacobians; steps shortened per cell so that the state stays
    admissible: 0 <= n_HI <= n_H, n_HeI, n_HeII >= 0, n_HeI + n_HeII <= n_He,
    e > 0)."""
    p = mp.base
    L = mp.nloc
    nH, nHe = ctx.nH, ctx.nHe
    y = np.array(y_init, dtype=np.float64)
    y[0] = np.clip(y[0], 0.0, nH)
    if mp.he:
        y[1] = np.clip(y[1], 0.0, nHe)
        y[2] = np.clip(y[2], 0.0, nHe - y[1])
    e0 = ctx.en if p.isothermal else np.maximum(np.array(e_init, dtype=np.float64), 1e-300)
    z = _pack_loc(mp, e0, y)
    sc = _loc_scales(mp, ctx)
    for it in range(max_it):
        f = _floc(mp, ctx, E, z, ctx.en)
        Jm = np.empty((L, L) + p.dims)
        for j in range(L):
            h = 1e-20 * np.maximum(np.abs(z[j]), 1e-30 * sc[j])
            zc = z.astype(np.complex128)
            zc[j] = zc[j] + 1j * h
            Jm[:, j] = np.imag(_floc(mp, ctx, E, zc, ctx.en)) / h
        A = np.moveaxis(Jm.reshape(L, L, -1), 2, 0)
        b = np.moveaxis(f.reshape(L, -1), 1, 0)
        dz = -np.linalg.solve(A, b[..., None])[..., 0]
        dz = np.moveaxis(dz, 0, 1).reshape((L,) + p.dims)
        lam = np.ones(p.dims)
        e_c, y_c = _unpack_loc(mp, z, ctx.en, ctx)
        e_d, y_d = _unpack_loc(mp, dz, 0.0 * ctx.en, ctx)

        def cap(lam, val, step, bound_lo=None, bound_hi=None):
            if bound_lo is not None:
                m = val + step < bound_lo
                lam = np.where(m, np.minimum(lam, 0.9 * (val - bound_lo) / np.where(m, -step, 1.0)), lam)
            if bound_hi is not None:
                m = val + step > bound_hi
                lam = np.where(m, np.minimum(lam, 0.9 * (bound_hi - val) / np.where(m, step, 1.0)), lam)
            return lam
        lam = cap(lam, y_c[0], y_d[0], 0.0, nH)
        if mp.he:
            lam = cap(lam, y_c[1], y_d[1], 0.0, None)
            lam = cap(lam, y_c[2], y_d[2], 0.0, None)
            # n_HeIII = n_He - n_HeI - n_HeII >= 0; it starts at exactly 0, so
            # a step that exceeds the bound only by rounding is not cut
            tot, dtot = y_c[1] + y_c[2], y_d[1] + y_d[2]
            over = tot + dtot > nHe * (1.0 + 1e-12)
            lam = np.where(over, cap(lam, tot, dtot, None, nHe), lam)
        if not p.isothermal:
            lam = cap(lam, e_c, e_d, 0.0, None)
        z = z + lam * dz
        # step size: relative to e for the gas energy, to n_H / n_He for species
        ref = sc.copy()
        if not p.isothermal:
            ref[0] = z[0]
        small = float(np.max(np.abs(lam * dz) / ref))
        if small <= tol and np.all(lam == 1.0):
            e, y = _unpack_loc(mp, z, ctx.en, ctx)
            return e, y
    raise NewtonFailure("multigroup local solve did not converge")


# ---------------------------------------------------------------------------
# Newton on the full system
# ---------------------------------------------------------------------------
def _residual_vec(mp, ctx, E, z):
    """All residual components per cell, stacked [f_E,g ..., f_loc ...]."""
    e, y = _unpack_loc(mp, z, ctx.en, ctx)
    return np.concatenate([f_E(mp, ctx, E, y), _floc(mp, ctx, E, z, ctx.en)])


def full_jacobian(mp: MGParams, ctx: Ctx, E, z):
    """Sparse Jacobian of all residual components with respect to all
    unknowns (unknown k of cell P has index k * N + P), by the complex step:
    group energies one stencil colour at a time, local unknowns all cells at
    once (they enter only their own cell's equations)."""
    p = mp.base
    N = p.ncells
    G, L = mp.G, mp.nloc
    V = G + L
    colours, ncol = stencil_colours(p.dims)
    col = colours.ravel()
    nbs = stencil_neighbours(p)
    sc = _loc_scales(mp, ctx)
    rows, cols, vals = [], [], []
    for g in range(G):
        hE = 1e-20 * np.maximum(np.abs(E[g]), 1e-30 * ctx.E_s[g]).ravel()
        for c in range(ncol):
            Ec = E.astype(np.complex128)
            pert = np.where(col == c, hE, 0.0).reshape(p.dims)
            Ec[g] = Ec[g] + 1j * pert
            R_ = np.imag(_residual_vec(mp, ctx, Ec, z.astype(np.complex128))).reshape(V, N)
            for _, nb in nbs:
                P = np.nonzero(nb >= 0)[0]
                Q = nb[P]
                m = col[Q] == c
                P, Q = P[m], Q[m]
                for r in range(V):
                    rows.append(r * N + P)
                    cols.append(g * N + Q)
                    vals.append(R_[r, P] / hE[Q])
    for j in range(L):
        h = (1e-20 * np.maximum(np.abs(z[j]), 1e-30 * sc[j])).ravel()
        zc = z.astype(np.complex128)
        zc[j] = zc[j] + 1j * h.reshape(p.dims)
        R_ = np.imag(_residual_vec(mp, ctx, E.astype(np.complex128), zc)).reshape(V, N)
        P = np.arange(N)
        for r in range(V):
            rows.append(r * N + P)
            cols.append((G + j) * N + P)
            vals.append(R_[r] / h)
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(V * N, V * N))
    J.sum_duplicates()
    J.eliminate_zeros()
    return J


def step(mp: MGParams, t_n, dt, nH, src, E, e, y, *, tol=None, stats=None):
    """One implicit step: returns (E (G x dims), e, y (3 x dims))."""
    p = mp.base
    tol = p.newton_tol if tol is None else tol
    nH = np.asarray(nH, dtype=np.float64)
    src = np.asarray(src, dtype=np.float64)
    En, en, yn = (np.array(X, dtype=np.float64) for X in (E, e, y))
    ctx = make_context(mp, t_n, dt, nH, src, En, en, yn)
    E = En.copy()
    e, y = local_solve(mp, ctx, E, en, yn)
    fE, fe, fy = residual(mp, ctx, E, None if p.isothermal else e, y)
    nrm = norm(mp, ctx, fE, fe, fy)
    hist, cuts = [], 0
    N = p.ncells
    for k in range(p.newton_max_it + 1):
        if not np.isfinite(nrm):
            raise FloatingPointError("non-finite residual norm")
        hist.append(nrm)
        if nrm <= tol:
            break
        if k == p.newton_max_it:
            raise NewtonFailure(f"no convergence after {k} iterations (||f|| = {nrm:.3e})")
        z = _pack_loc(mp, e, y)
        J = full_jacobian(mp, ctx, E, z)
        rhs = -_residual_vec(mp, ctx, E, z).reshape(-1)
        d = spla.spsolve(J.tocsc(), rhs)
        dE = d[: mp.G * N].reshape((mp.G,) + p.dims)
        dz = d[mp.G * N:].reshape((mp.nloc,) + p.dims)
        de_, dy_ = _unpack_loc(mp, dz, 0.0 * en, ctx)
        lam = 1.0
        for cut in range(p.ls_max_cuts + 1):
            Et = E + lam * dE
            try:
                et, yt = local_solve(mp, ctx, Et, None if p.isothermal else e + lam * de_,
                                     y + lam * dy_)
            except NewtonFailure:
                lam *= 0.5
                cuts += 1
                continue
            ft = residual(mp, ctx, Et, None if p.isothermal else et, yt)
            nt = norm(mp, ctx, *ft)
            if nt <= (1.0 - p.armijo * lam) * nrm:
                break
            lam *= 0.5
            cuts += 1
        else:
            raise NewtonFailure(f"line search failed at iteration {k} (||f|| = {nrm:.3e})")
        E, e, y = Et, et, yt
        fE, fe, fy = ft
        nrm = nt
    if stats is not None:
        stats.update(newton_its=len(hist) - 1, history=hist, ls_cuts=cuts, res_final=hist[-1])
    return E, (en.copy() if p.isothermal else e), y


def photon_budget_defects(mp: MGParams, ctx: Ctx, E1, y1):
    """Per-group relative defect of the discrete photon-energy budget with
    zero-flux or periodic walls (the diffusion telescopes at both levels)."""
    th = mp.base.theta
    k1 = opacity(mp, y1, ctx.a_1)
    kn = opacity(mp, ctx.yn, ctx.a_n)
    out = []
    for g in range(mp.G):
        impl = -ctx.H_1 * E1[g] - C_LIGHT * k1[g] * E1[g] + ctx.src[g]
        expl = -ctx.H_n * ctx.En[g] - C_LIGHT * kn[g] * ctx.En[g] + ctx.src[g]
        lhs = float(np.sum(E1[g] - ctx.En[g]))
        rhs = ctx.dt * (th * float(np.sum(impl)) + (1.0 - th) * float(np.sum(expl)))
        scale = ctx.dt * float(np.sum(np.abs(C_LIGHT * k1[g] * E1[g]) + np.abs(ctx.src[g])
                                      + np.abs(C_LIGHT * kn[g] * ctx.En[g]))) + 1e-300
        out.append(abs(lhs - rhs) / scale)
    return out
