"""Adjoint of the implicit step (oracle).

The step map U^{n+1} = Phi(U^n; src, n_H) is defined implicitly by
f(U^{n+1}; U^n, src, n_H) = 0 (Algorithm section: the root of the nonlinear
residual).  By the implicit-function theorem, for lambda = dJ/dU^{n+1}:

  J_U^T mu = lambda,                 J_U = df/dU^{n+1} at the converged state
  dJ/dU^n  = -(df/dU^n)^T mu
  dJ/dsrc  = -(df/dsrc)^T mu,  dJ/dn_H = -(df/dn_H)^T mu

Every block is built by the complex step from the oracle's own residual:
the local blocks per cell, J_EE and df_E/d(E^n, n^n) (the lagged face
limiter D(E^n, kappa^n) and, for theta < 1, the explicit part) by coloured
stencil Jacobians.  J_U^T mu = lambda is solved directly on the full sparse
system (no Schur reduction), so the oracle shares no algebra with the
reduced adjoint of the GPU path.

Objective used by the tests (volume-averaged ionised fraction at the final
step): J = (1/N) sum_P (1 - n_P / n_H,P); parameters src = 4 pi eta per cell
and n_H per cell, where n_H also sets the initial neutral density
n^0 = (1 - x0) n_H (the initial temperature is fixed, so e^0 does not
depend on n_H).

Parity: pinned by central finite differences of J through forward oracle
steps, and by the dot-product identity with the tangent-linear step (tests).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import model as M
from . import newton as ON


def _jacobians(p, t_n, dt, nH, src, Un, U1):
    """All blocks at (U^n, U^{n+1}) as sparse matrices in the unknown order
    (n, e, E) per field block (isothermal: (n, E))."""
    En, en, nn = (np.asarray(a, dtype=np.float64) for a in Un)
    E1, e1, n1 = (np.asarray(a, dtype=np.float64) for a in U1)
    ctx = M.make_context(p, t_n, dt, nH, src, En, en, nn)
    ee1 = None if p.isothermal else e1
    D = sp.diags
    N = p.ncells
    # --- d f / d U^{n+1}
    loc = ON.local_jacobian(p, ctx, E1, ee1, n1)
    JEE, JEn = ON.radiation_jacobian(p, ctx, E1, n1)
    # --- d f / d U^n: local residuals through S_n, S_e (diagonal)
    def local_wrt(name):
        h = ON._cstep_h({"En": En, "en": en, "nn": nn}[name],
                        {"En": ctx.E_s, "en": np.abs(en), "nn": nH}[name])
        args = {"En": En.astype(complex), "en": en.astype(complex), "nn": nn.astype(complex)}
        args[name] = args[name] + 1j * h
        c2 = M.make_context(p, t_n, dt, nH, src, args["En"], args["en"], args["nn"],
                            Dfaces=ctx.D)
        Sn, Se = M.local_S(p, c2, E1, ee1, n1)
        dn = (-np.imag(Sn) / h).ravel()
        de = None if Se is None else (-np.imag(Se) / h).ravel()
        return dn, de
    # --- d f_E / d(E^n, n^n) through the limiter and the explicit part (stencil)
    def fE_of(Enz, nnz):
        c2 = M.make_context(p, t_n, dt, nH, src, Enz, en, nnz)
        return M.f_E(p, c2, E1, n1)
    hE = ON._cstep_h(En, ctx.E_s)
    hn = ON._cstep_h(nn, nH)
    JEEn = ON.stencil_jacobian(p, lambda z: fE_of(z, nn.astype(complex)), En.astype(complex), hE)
    JEnn = ON.stencil_jacobian(p, lambda z: fE_of(En.astype(complex), z), nn.astype(complex), hn)
    # --- d f / d n_H (local residuals only; f_E does not contain n_H)
    hH = ON._cstep_h(nH, nH)
    c3 = M.StepContext(**{**ctx.__dict__, "nH": nH + 1j * hH})
    Sn, Se = M.local_S(p, c3, E1, ee1, n1)
    dfn_dnH = (-np.imag(Sn) / hH).ravel()
    dfe_dnH = None if Se is None else (-np.imag(Se) / hH).ravel()

    dn_nn, de_nn = local_wrt("nn")
    dn_En, de_En = local_wrt("En")
    if p.isothermal:
        JU = sp.bmat([[D(loc["fn_n"]), D(loc["fn_E"])],
                      [D(JEn), JEE]], format="csc")
        JUn = sp.bmat([[D(dn_nn), D(dn_En)],
                       [JEnn, JEEn]], format="csc")
        Jsrc = sp.vstack([sp.csr_matrix((N, N)), -dt * sp.identity(N)]).tocsc()
        JnH = sp.vstack([D(dfn_dnH), sp.csr_matrix((N, N))]).tocsc()
    else:
        dn_en, de_en = local_wrt("en")
        JU = sp.bmat([[D(loc["fn_n"]), D(loc["fn_e"]), D(loc["fn_E"])],
                      [D(loc["fe_n"]), D(loc["fe_e"]), D(loc["fe_E"])],
                      [D(JEn), None, JEE]], format="csc")
        JUn = sp.bmat([[D(dn_nn), D(dn_en), D(dn_En)],
                       [D(de_nn), D(de_en), D(de_En)],
                       [JEnn, None, JEEn]], format="csc")
        Jsrc = sp.vstack([sp.csr_matrix((2 * N, N)), -dt * sp.identity(N)]).tocsc()
        JnH = sp.vstack([D(dfn_dnH), D(dfe_dnH), sp.csr_matrix((N, N))]).tocsc()
    return JU, JUn, Jsrc, JnH


def _stack(p, E, e, n):
    parts = [np.ravel(n)] + ([] if p.isothermal else [np.ravel(e)]) + [np.ravel(E)]
    return np.concatenate(parts)


def _unstack(p, v):
    N = p.ncells
    n = v[:N].reshape(p.dims)
    if p.isothermal:
        return v[N:].reshape(p.dims), None, n
    return v[2 * N:].reshape(p.dims), v[N:2 * N].reshape(p.dims), n


def adjoint_step(p, t_n, dt, nH, src, Un, U1, lam):
    """lam = (lE, le, ln) = dJ/dU^{n+1}; returns (dJ/dU^n as (lE, le, ln),
    dJ/dsrc, dJ/dn_H) through this step (le is None for isothermal runs)."""
    JU, JUn, Jsrc, JnH = _jacobians(p, t_n, dt, nH, src, Un, U1)
    rhs = _stack(p, *lam)
    mu = spla.spsolve(JU.T.tocsc(), rhs)
    lam_n = _unstack(p, -(JUn.T @ mu))
    g_src = -(Jsrc.T @ mu).reshape(p.dims)
    g_nH = -(JnH.T @ mu).reshape(p.dims)
    return lam_n, g_src, g_nH


def tangent_step(p, t_n, dt, nH, src, Un, U1, dUn, dsrc, dnH):
    """Tangent-linear step: dU^{n+1} for perturbations (dU^n, dsrc, dn_H)."""
    JU, JUn, Jsrc, JnH = _jacobians(p, t_n, dt, nH, src, Un, U1)
    rhs = -(JUn @ _stack(p, *dUn)) - Jsrc @ np.ravel(dsrc) - JnH @ np.ravel(dnH)
    return _unstack(p, spla.spsolve(JU.tocsc(), rhs))


def objective(nH, n):
    """Volume-averaged ionised fraction."""
    return float(np.mean(1.0 - n / nH))


def gradient(p, t0, dt, nsteps, nH, src, x0, T0, E0, tol=1e-13):
    """dJ/dsrc and dJ/dn_H of J = mean x_HII after nsteps, through forward
    steps with checkpoints and adjoint steps in reverse."""
    E, e, n = M.initial_state(p, nH, x0, T0, E0)
    traj = [(E, e, n)]
    for s in range(nsteps):
        E, e, n = ON.step(p, t0 + s * dt, dt, nH, src, E, e, n, tol=tol)
        traj.append((E, e, n))
    N = p.ncells
    lE = np.zeros(p.dims)
    le = None if p.isothermal else np.zeros(p.dims)
    ln = -1.0 / (N * nH)
    g_src = np.zeros(p.dims)
    g_nH = traj[-1][2] / (N * nH * nH)       # direct dependence of J on n_H
    for s in reversed(range(nsteps)):
        (lE, le, ln), gs, gh = adjoint_step(p, t0 + s * dt, dt, nH, src, traj[s], traj[s + 1],
                                            (lE, le, ln))
        g_src += gs
        g_nH += gh
    g_nH += (1.0 - x0) * ln                   # initial condition n^0 = (1 - x0) n_H
    return objective(nH, traj[-1][2]), g_src, g_nH
