"""Advection half of the operator split (oracle; test infrastructure only).

Step (iv) of the method's time step (Algorithm section) moves the chemical
number densities and the radiation energy with the gas velocity before the
implicit step (v) starts from the advected values (equations
enzo-chemical_ionization and enzo-cons_radiation: d_t q + (1/a) div(q v) = 0
for q = n_i and q = E, with comoving divergence and proper peculiar velocity
v).  The hydrodynamics that produce v (PPM, pressure, gravity) are not part
of this implementation; v is a prescribed input.  Readings used (identical on
the GPU side):

  * conserved quantities per cell: E, n_H, n_HI (so n_HII = n_H - n_HI moves
    with the same fluxes) and n_H e, the gas energy density up to the
    constant m_H (e is energy per unit mass); e is recovered as
    (n_H e)_new / n_H_new.  Isothermal runs do not touch e.  Only the
    advective part of the gas-energy equation belongs here; its pressure,
    gravity and expansion terms belong to the hydrodynamics.
  * v is cell-centred (one value per cell and axis).  The velocity of the
    face between cells P and Q is (v_P + v_Q)/2.  At a zero-flux wall the
    face velocity is 0 (closed box); at an outflow wall it is the boundary
    cell's velocity and the ghost cell holds the boundary cell's values
    (zero-gradient inflow).  Periodic axes wrap.
  * first-order donor-cell (upwind) fluxes, unsplit: with the face Courant
    number u = dt_s v_face / (a h), the flux through a face is u q_L when
    u > 0 and u q_R otherwise, and q_P changes by the sum of its inflows
    minus its outflows.  The cell's outgoing Courant number is the sum over
    its six faces of the parts of u pointing out of the cell; when it is at
    most 1 everywhere the update is a convex combination (positive, and the
    ratios e and n_HI / n_H stay within their neighbours' range).
  * dt is split into m equal substeps, m = max(1, ceil(C / cfl)) with C the
    largest outgoing Courant number over the whole dt at a(t_0) (a grows
    with t in every cosmology here, so every substep stays below cfl); each
    substep uses a at its own midpoint.

Parity: pinned in the tests by exact translation at Courant number 1, the
binomial closed form of repeated donor-cell steps at Courant number c < 1,
exact conservation with periodic and closed walls, preservation of uniform
ratios under any velocity field, the neighbour-range bound, a uniform state
under uniform flow through outflow walls, and the centroid displacement
int v / a dt in an expanding universe.
"""
from __future__ import annotations

import math

import numpy as np

from . import model as M
from . import newton as ON


def _faces(p: M.Params, v, d: int):
    """Face velocities along axis d: array with n_d + 1 faces (face f lies
    between cells f-1 and f; faces 0 and n_d are the walls)."""
    lo, hi = p.bc[2 * d], p.bc[2 * d + 1]
    n = v.shape[d]
    first = np.take(v, [0], axis=d)
    last = np.take(v, [n - 1], axis=d)
    if lo == M.PERIODIC:
        vp = np.concatenate([last, v, first], axis=d)
        vL = np.take(vp, np.arange(0, n + 1), axis=d)
        vR = np.take(vp, np.arange(1, n + 2), axis=d)
        return 0.5 * (vL + vR)
    inner = 0.5 * (np.take(v, np.arange(0, n - 1), axis=d) + np.take(v, np.arange(1, n), axis=d))
    wlo = first if lo == M.OUTFLOW else np.zeros_like(first)
    whi = last if hi == M.OUTFLOW else np.zeros_like(last)
    return np.concatenate([wlo, inner, whi], axis=d)


def courant(p: M.Params, v, scale: float) -> float:
    """Largest outgoing Courant number of one cell for the face velocities
    times scale (scale = dt / (a h))."""
    out = np.zeros(p.dims)
    for d in range(3):
        f = _faces(p, v[d], d) * scale
        n = p.dims[d]
        up = np.take(f, np.arange(1, n + 1), axis=d)
        dn = np.take(f, np.arange(0, n), axis=d)
        out += np.maximum(up, 0.0) + np.maximum(-dn, 0.0)
    return float(out.max())


def donor_step(p: M.Params, v, q, scale: float):
    """One donor-cell substep of the conserved fields q (list of arrays) with
    face Courant numbers scale * face velocity."""
    new = [np.array(x, dtype=np.float64) for x in q]
    for d in range(3):
        lo, hi = p.bc[2 * d], p.bc[2 * d + 1]
        u = _faces(p, v[d], d) * scale
        n = p.dims[d]
        for i, x in enumerate(q):
            # ghost values: periodic wrap, else the boundary cell's own value
            xp = M.pad(x, d, lo, hi, np.take(x, [0], axis=d), np.take(x, [n - 1], axis=d))
            left = np.take(xp, np.arange(0, n + 1), axis=d)
            right = np.take(xp, np.arange(1, n + 2), axis=d)
            F = np.where(u > 0.0, u * left, u * right)
            new[i] -= np.take(F, np.arange(1, n + 1), axis=d) - np.take(F, np.arange(0, n), axis=d)
    return new


def substeps(p: M.Params, t0: float, dt: float, v, cfl: float) -> tuple[int, float]:
    """(m, C): substep count and the largest outgoing Courant number over dt."""
    a0 = p.cosmo.a(t0)
    C = courant(p, v, dt / (a0 * p.h))
    return max(1, math.ceil(C / cfl)), C


def advect(p: M.Params, t0: float, dt: float, v, nH, E, e, n, cfl: float = 0.9):
    """Advect (n_H, E, e, n_HI) over [t0, t0 + dt] with velocity v = (vx, vy, vz)
    [proper cm/s]; returns ((nH, E, e, n), m)."""
    if not (dt > 0 and 0 < cfl <= 1):
        raise ValueError("need dt > 0 and 0 < cfl <= 1")
    v = [np.asarray(c, dtype=np.float64) for c in v]
    m, _ = substeps(p, t0, dt, v, cfl)
    return advect_substeps(p, t0, dt, m, v, nH, E, e, n), m


def advect_substeps(p: M.Params, t0: float, dt: float, m: int, v, nH, E, e, n):
    """The m substeps of advect over [t0, t0 + dt]; returns (nH, E, e, n)."""
    v = [np.asarray(c, dtype=np.float64) for c in v]
    ds = dt / m
    nH = np.array(nH, dtype=np.float64)
    E = np.array(E, dtype=np.float64)
    n = np.array(n, dtype=np.float64)
    e = None if p.isothermal else np.array(e, dtype=np.float64)
    for s in range(m):
        a_mid = p.cosmo.a(t0 + (s + 0.5) * ds)
        scale = ds / (a_mid * p.h)
        if p.isothermal:
            nH, E, n = donor_step(p, v, [nH, E, n], scale)
        else:
            nH1, E, n, rho_e = donor_step(p, v, [nH, E, n, nH * e], scale)
            e = rho_e / nH1
            nH = nH1
    return nH, E, e, n


def split_step(p: M.Params, t0: float, dt: float, v, nH, src, E, e, n, cfl: float = 0.9,
               tol=None, stats=None):
    """One operator-split step: advection over dt, then the implicit step from
    the advected values (steps (iv) and (v) of the time step); returns
    (nH, E, e, n) at t0 + dt."""
    (nH1, Ea, ea, na), m = advect(p, t0, dt, v, nH, E, e, n, cfl)
    if stats is not None:
        stats["substeps"] = m
    if p.isothermal:
        ea = np.zeros_like(Ea) if e is None else np.asarray(e, dtype=np.float64)
    E1, e1, n1 = ON.step(p, t0, dt, nH1, src, Ea, ea, na, tol=tol, stats=stats)
    return nH1, E1, e1, n1
