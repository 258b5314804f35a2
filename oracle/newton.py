"""Globalised Newton solve of one implicit step (oracle).

The paper solves f(U) = 0 for U^{n+1} with a globalised inexact Newton
method whose linear systems J(U_k) s_k = -f(U_k) are reduced by a Schur
complement to a modified radiation equation (Algorithm section).  The
root does not depend on how the linear systems are solved, so this oracle
solves them exactly (sparse direct).

Globalisation (a reading; the paper leaves the details to its companion
paper): Newton acts on E, and the local equations f_n = f_e = 0 are
solved per cell for each E (nonlinear elimination of the local
unknowns).  The Newton matrix of the reduced residual f_E(E, n(E), e(E))
is exactly the Schur complement of the paper's linear system, so each
iteration still solves the modified radiation equation; the linear
back-substitution for (n, e) is replaced by the per-cell re-solve, which
keeps every iterate admissible (0 <= n <= n_H, e > 0).

  E_0 = E^n, (n_0, e_0) = local solve at E_0
  repeat: evaluate ||f(U_k)||; stop when <= tol
          local 2x2 (1x1 isothermal) blocks B = d(f_n,f_e)/d(n,e) and
          C = d(f_n,f_e)/dE by the complex step; J_En = d f_E/d n (diagonal)
          and the 7-point J_EE by the complex step on f_E (linear in E)
          S = J_EE - diag(J_En (B^-1 C)_n),  r = -f_E + J_En (B^-1 f_loc)_n
          S dE = r (sparse direct)
          backtracking: lambda = 1, 1/2, ... on E_k + lambda dE with the
          local re-solve, until ||f|| <= (1 - 1e-4 lambda) ||f(U_k)||; a
          trial whose local re-solve does not converge has no residual and
          counts as no decrease (lambda is halved)

Parity: pinned by the full-system solve against the Schur route (same
Newton direction), by quadratic convergence of the iterates and by the
physics pins (tests).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import model as M


class NewtonFailure(RuntimeError):
    pass


# ---------------------------------------------------------------------------
# colouring for complex-step Jacobians of 7-point-stencil functions
# ---------------------------------------------------------------------------
def _axis_colours(n: int) -> np.ndarray:
    q = n // 3
    c = np.empty(n, dtype=np.int64)
    c[: 3 * q] = np.arange(3 * q) % 3
    c[3 * q:] = 3 + np.arange(n - 3 * q)
    return c


def stencil_colours(dims):
    """Colours such that no 7-point stencil holds two cells of one colour
    (periodic wrap included)."""
    cx, cy, cz = (_axis_colours(n) for n in dims)
    col = (cx[:, None, None] + 5 * cy[None, :, None] + 25 * cz[None, None, :])
    uniq, inv = np.unique(col.ravel(), return_inverse=True)
    return inv.reshape(dims), len(uniq)


def stencil_neighbours(p: M.Params):
    """List of (offset name, flat index array) for the 7 stencil points;
    index -1 marks a neighbour outside a non-periodic boundary."""
    nx, ny, nz = p.dims
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    out = [("c", ((I * ny + J) * nz + K).ravel())]
    for d, n in enumerate(p.dims):
        for s in (-1, 1):
            idx = [I.copy(), J.copy(), K.copy()]
            idx[d] = idx[d] + s
            valid = np.ones(p.dims, dtype=bool)
            if p.bc[2 * d] == M.PERIODIC:
                idx[d] = idx[d] % n
            else:
                valid = (idx[d] >= 0) & (idx[d] < n)
                idx[d] = np.clip(idx[d], 0, n - 1)
            flat = (idx[0] * ny + idx[1]) * nz + idx[2]
            out.append((f"{d}{s:+d}", np.where(valid, flat, -1).ravel()))
    return out


def stencil_jacobian(p: M.Params, func, x, hstep):
    """Sparse Jacobian of a 7-point-stencil map func: R^N -> R^N by the
    complex step with one evaluation per colour.

    hstep: per-cell step (array) -- entry (P, j) = Im func(x + i h v_c)[P] / h_j.
    """
    colours, ncol = stencil_colours(p.dims)
    N = p.ncells
    col = colours.ravel()
    hflat = np.broadcast_to(hstep, p.dims).ravel()
    JV = np.empty((ncol, N))
    for c in range(ncol):
        pert = np.where(col == c, hflat, 0.0).reshape(p.dims)
        JV[c] = np.imag(func(x + 1j * pert)).ravel()
    rows, cols, vals = [], [], []
    for _, nb in stencil_neighbours(p):
        P = np.nonzero(nb >= 0)[0]
        j = nb[P]
        rows.append(P)
        cols.append(j)
        vals.append(JV[col[j], P] / hflat[j])
    J = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    J.sum_duplicates()
    return J


def _cstep_h(x, scale):
    """Complex-step size: tiny relative to the value itself (the functions are
    nonlinear on the scale of the value, e.g. the limiter in E where E is
    1e-35), with a floor far below the field's scale for zero values."""
    return 1e-20 * np.maximum(np.abs(x), 1e-30 * np.abs(scale))


def local_jacobian(p: M.Params, ctx: M.StepContext, E, e, n, wrt_E=True):
    """Derivatives of the local residuals by the complex step.

    Returns dict with 'fn_n','fn_e','fn_E','fe_n','fe_e','fe_E' (flat arrays;
    the e-entries are absent for isothermal runs).
    """
    out = {}
    hn = _cstep_h(n, ctx.nH)
    Sn, Se = M.local_S(p, ctx, E, e, n + 1j * hn)
    out["fn_n"] = (1.0 - np.imag(Sn) / hn).ravel()
    if Se is not None:
        out["fe_n"] = (-np.imag(Se) / hn).ravel()
    if wrt_E:
        hE = _cstep_h(E, ctx.E_s)
        Sn, Se = M.local_S(p, ctx, E + 1j * hE, e, n)
        out["fn_E"] = (-np.imag(Sn) / hE).ravel()
        if Se is not None:
            out["fe_E"] = (-np.imag(Se) / hE).ravel()
    if not p.isothermal:
        he = _cstep_h(e, np.abs(ctx.en))
        Sn, Se = M.local_S(p, ctx, E, e + 1j * he, n)
        out["fn_e"] = (-np.imag(Sn) / he).ravel()
        out["fe_e"] = (1.0 - np.imag(Se) / he).ravel()
    return out


def radiation_jacobian(p: M.Params, ctx: M.StepContext, E, n):
    """(J_EE sparse, J_En diagonal as a flat array) by the complex step."""
    JEE = stencil_jacobian(p, lambda Ez: M.f_E(p, ctx, Ez, n), E.astype(complex),
                           np.ones(p.dims))
    hn = _cstep_h(n, ctx.nH)
    JEn = (np.imag(M.f_E(p, ctx, E, n + 1j * hn)) / hn).ravel()
    return JEE, JEn


# ---------------------------------------------------------------------------
# linear solves
# ---------------------------------------------------------------------------
def solve_full(p, loc, JEE, JEn, fE, fe, fn, dense=False):
    """Solve the whole Newton system (unknown order n, [e,] E)."""
    N = p.ncells
    D = sp.diags
    if p.isothermal:
        J = sp.bmat([[D(loc["fn_n"]), D(loc["fn_E"])],
                     [D(JEn), JEE]], format="csc")
        rhs = -np.concatenate([fn.ravel(), fE.ravel()])
    else:
        J = sp.bmat([[D(loc["fn_n"]), D(loc["fn_e"]), D(loc["fn_E"])],
                     [D(loc["fe_n"]), D(loc["fe_e"]), D(loc["fe_E"])],
                     [D(JEn), None, JEE]], format="csc")
        rhs = -np.concatenate([fn.ravel(), fe.ravel(), fE.ravel()])
    s = np.linalg.solve(J.toarray(), rhs) if dense else spla.spsolve(J, rhs)
    dn = s[:N]
    if p.isothermal:
        return s[N:], None, dn
    return s[2 * N:], s[N:2 * N], dn


def local_inverse_terms(p, loc, fe, fn):
    """(B^-1 f_loc, B^-1 C) per cell, as dicts of flat arrays."""
    if p.isothermal:
        b = loc["fn_n"]
        return {"n": fn.ravel() / b}, {"n": loc["fn_E"] / b}
    a11, a12, a21, a22 = loc["fn_n"], loc["fn_e"], loc["fe_n"], loc["fe_e"]
    det = a11 * a22 - a12 * a21
    f1, f2 = fn.ravel(), fe.ravel()
    c1, c2 = loc["fn_E"], loc["fe_E"]
    Bf = {"n": (a22 * f1 - a12 * f2) / det, "e": (-a21 * f1 + a11 * f2) / det}
    BC = {"n": (a22 * c1 - a12 * c2) / det, "e": (-a21 * c1 + a11 * c2) / det}
    return Bf, BC


def schur_operator(p, loc, JEE, JEn, fe, fn, fE):
    """(S, r_S, B^-1 f_loc, B^-1 C) of the Schur reduction."""
    Bf, BC = local_inverse_terms(p, loc, fe, fn)
    S = (JEE - sp.diags(JEn * BC["n"])).tocsr()
    r = -fE.ravel() + JEn * Bf["n"]
    return S, r, Bf, BC


def check_schur_dominance(S):
    """Assert the Schur operator keeps a positive shift: diag > sum |offdiag|."""
    d = S.diagonal()
    off = np.asarray(abs(S).sum(axis=1)).ravel() - np.abs(d)
    if not np.all(d - off > 0):
        raise NewtonFailure("Schur operator lost diagonal dominance")


DIRECT_MAX = 8192


def solve_spd(S, r):
    """Solve the symmetric positive definite Schur system.

    Sparse LU for small systems; above DIRECT_MAX unknowns conjugate
    gradients with a diagonal preconditioner to a relative residual of
    1e-14, restarted on the true residual (iterative refinement) while the
    attained residual is above 1e-12 of ||r||, at most three times: on
    ill-conditioned operators the recursively updated CG residual drifts
    from the true one.  The attained residual is accepted down to the
    rounding floor of its own evaluation, 16 eps || |S| |x| + |r| ||.
    """
    if S.shape[0] <= DIRECT_MAX:
        return spla.spsolve(S.tocsc(), r)
    rn = np.linalg.norm(r)
    if rn == 0.0:
        return np.zeros_like(r)
    Minv = sp.diags(1.0 / S.diagonal())
    absS = abs(S)
    x = np.zeros_like(r)
    info = 0

    def accepted(res, x):
        floor = 16.0 * np.finfo(np.float64).eps * np.linalg.norm(absS @ np.abs(x) + np.abs(r))
        return res <= max(1e-12 * rn, floor)

    for _ in range(4):
        res_vec = r - S @ x
        res = np.linalg.norm(res_vec)
        if accepted(res, x):
            return x
        dx, info = spla.cg(S, res_vec, rtol=1e-14, atol=0.0, maxiter=50000, M=Minv)
        x = x + dx
    res = np.linalg.norm(S @ x - r)
    if not accepted(res, x):
        raise NewtonFailure(f"CG residual {res / rn:.2e} (info {info})")
    return x


def solve_schur(p, loc, JEE, JEn, fE, fe, fn):
    S, r, Bf, BC = schur_operator(p, loc, JEE, JEn, fe, fn, fE)
    check_schur_dominance(S)
    dE = solve_spd(S, r)
    dn = -Bf["n"] - BC["n"] * dE
    de = None if p.isothermal else -Bf["e"] - BC["e"] * dE
    return dE, de, dn


# ---------------------------------------------------------------------------
# local solve
# ---------------------------------------------------------------------------
def local_solve(p: M.Params, ctx: M.StepContext, E, n_init, e_init, tol=1e-15, max_it=80):
    """Per-cell root (n, e) of f_n = f_e = 0 at fixed E (damped Newton).

    Steps are shortened per cell so that n stays in [0, n_H] and e > 0.
    """
    nH = ctx.nH
    n = np.clip(np.array(n_init, dtype=np.float64), 0.0, nH)
    e = None if p.isothermal else np.maximum(np.array(e_init, dtype=np.float64), 1e-300)
    for it in range(max_it):
        Sn, Se = M.local_S(p, ctx, E, e, n)
        fn = n - Sn
        loc = local_jacobian(p, ctx, E, e, n, wrt_E=False)
        if p.isothermal:
            dn = -fn.ravel() / loc["fn_n"]
            de = None
        else:
            fe = e - Se
            a11, a12, a21, a22 = loc["fn_n"], loc["fn_e"], loc["fe_n"], loc["fe_e"]
            det = a11 * a22 - a12 * a21
            f1, f2 = fn.ravel(), fe.ravel()
            dn = -(a22 * f1 - a12 * f2) / det
            de = -(-a21 * f1 + a11 * f2) / det
        dn = dn.reshape(p.dims)
        lam = np.ones(p.dims)
        lo = n + dn < 0.0
        lam = np.where(lo, np.minimum(lam, 0.9 * n / np.where(lo, -dn, 1.0)), lam)
        hi = n + dn > nH
        lam = np.where(hi, np.minimum(lam, 0.9 * (nH - n) / np.where(hi, dn, 1.0)), lam)
        if de is not None:
            de = de.reshape(p.dims)
            neg = e + de <= 0.0
            lam = np.where(neg, np.minimum(lam, 0.9 * e / np.where(neg, -de, 1.0)), lam)
            e = e + lam * de
        n = n + lam * dn
        small = np.max(np.abs(lam * dn) / nH)
        if de is not None:
            small = max(small, float(np.max(np.abs(lam * de) / e)))
        if small <= tol and np.all(lam == 1.0):
            return n, e
    raise NewtonFailure("local solve did not converge")


# ---------------------------------------------------------------------------
# Newton step
# ---------------------------------------------------------------------------
def newton_direction(p, ctx, E, e, n, fE, fe, fn, solver="schur"):
    """Newton direction (dE, de, dn) of the full system at U = (E, e, n)."""
    loc = local_jacobian(p, ctx, E, e, n)
    JEE, JEn = radiation_jacobian(p, ctx, E, n)
    if solver == "schur":
        dE, de, dn = solve_schur(p, loc, JEE, JEn, fE, fe, fn)
    else:
        dE, de, dn = solve_full(p, loc, JEE, JEn, fE, fe, fn, dense=(solver == "dense"))
    dE = dE.reshape(p.dims)
    dn = dn.reshape(p.dims)
    de = None if de is None else de.reshape(p.dims)
    return dE, de, dn


def step(p: M.Params, t_n: float, dt: float, nH, src, E, e, n, *, solver="schur",
         tol=None, stats=None):
    """Advance (E, e, n) = U^n over dt; returns (E, e, n) at t_n + dt.

    Raises NewtonFailure when Newton or the line search fails, and
    FloatingPointError on a non-finite residual.
    """
    tol = p.newton_tol if tol is None else tol
    nH = np.asarray(nH, dtype=np.float64)
    src = np.asarray(src, dtype=np.float64)
    if not (np.all(np.isfinite(src)) and np.all(np.isfinite(nH))):
        raise FloatingPointError("non-finite input")
    En, en, nn = (np.array(X, dtype=np.float64) for X in (E, e, n))
    ctx = M.make_context(p, t_n, dt, nH, src, En, en, nn)
    E = En.copy()
    n, e = local_solve(p, ctx, E, nn, en)
    if p.isothermal:
        e = en.copy()
    hist = []
    fE, fe, fn = M.residual(p, ctx, E, None if p.isothermal else e, n)
    nrm = M.norm(p, ctx, fE, fe, fn)
    cuts_total = 0
    for k in range(p.newton_max_it + 1):
        if not np.isfinite(nrm):
            raise FloatingPointError("non-finite residual norm")
        hist.append(nrm)
        if nrm <= tol:
            break
        if k == p.newton_max_it:
            raise NewtonFailure(f"no convergence after {k} iterations (||f|| = {nrm:.3e})")
        ee = None if p.isothermal else e
        dE, de, dn = newton_direction(p, ctx, E, ee, n, fE, fe, fn, solver)
        lam = 1.0
        for cut in range(p.ls_max_cuts + 1):
            Et = E + lam * dE
            try:
                nt, et = local_solve(p, ctx, Et, n + lam * dn,
                                     None if de is None else e + lam * de)
            except NewtonFailure:
                # no local solution at this trial: no residual, so no decrease
                lam *= 0.5
                cuts_total += 1
                continue
            ft = M.residual(p, ctx, Et, et, nt)
            nt_norm = M.norm(p, ctx, *ft)
            if nt_norm <= (1.0 - p.armijo * lam) * nrm:
                break
            lam *= 0.5
            cuts_total += 1
        else:
            raise NewtonFailure(f"line search failed at iteration {k} (||f|| = {nrm:.3e})")
        E, n = Et, nt
        if not p.isothermal:
            e = et
        fE, fe, fn = ft
        nrm = nt_norm
    if stats is not None:
        stats.update(newton_its=len(hist) - 1, history=hist, ls_cuts=cuts_total,
                     res_final=hist[-1], E_s=ctx.E_s)
    return E, e, n


def run(p: M.Params, t0: float, dt: float, nsteps: int, nH, src, E, e, n, *,
        solver="schur", tol=None, callback=None):
    """nsteps implicit steps; returns final (E, e, n) and per-step stats."""
    all_stats = []
    t = t0
    for s in range(nsteps):
        st = {}
        E, e, n = step(p, t, dt, nH, src, E, e, n, solver=solver, tol=tol, stats=st)
        t += dt
        all_stats.append(st)
        if callback is not None:
            callback(s, t, E, e, n)
    return E, e, n, all_stats
