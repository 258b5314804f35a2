"""Adaptive implicit time stepping (oracle).

The verification runs pair theta = 0.51 with a "desired temporal solution
accuracy" tau_tol = 0.001 and the norm exponent p = 2 (Verification section,
solver settings of the Shapiro-Giroux runs); the step-size rule itself is in
the method's companion paper, which is not available here.  Reading used
(identical on the GPU side):

  * after an accepted step from U^n to U^{n+1}, the weighted change
        w = sqrt( sum_P [(dE/E_s)^2 + (de/e^n)^2 + (dn/n_H)^2] / (N (N_s+2)) )
    uses the weights of the Newton norm (equation rmsnorm) with the step's
    E_s = max(max E^n, dt max src, E_floor) (isothermal: no e term, 2
    unknowns per cell);
  * the next step is dt * clamp(tau_tol / w, 0.1, 2), capped by dt_max and
    shortened so the last step lands on t_end;
  * an attempt is rejected, the state kept at U^n and the step halved when
    the Newton step fails or some E^{n+1} < -1e-10 E_s (for theta < 1 the
    explicit part can flip the sign of E in optically thick cells); twelve
    rejections in a row end the run.

There is no rejection for accuracy: the radiation field equilibrates within
one step of any size once a source switches on, so a change-based rejection
could shrink the step forever.

Parity: pinned in the tests by the first-order convergence of the final
state in tau_tol against an ODE reference (uniform medium, uniform source),
by the controller's equilibrium w -> tau_tol, by exact landing on t_end and
by rejection and recovery on the theta = 0.51 Stromgren sphere (there the
explicit half of large steps drives the local solutions out of [0, n_H]).
"""
from __future__ import annotations

import numpy as np

from . import model as M
from . import newton as ON

MAX_REJECTS = 12
GROWTH_MAX = 2.0
SHRINK_MIN = 0.1
NEG_TOL = 1e-10


def change_norm(p: M.Params, E_s: float, U1, Un, nH) -> tuple[float, float]:
    """(w, max(-E^{n+1}/E_s)) of a step from Un to U1."""
    E1, e1, n1 = U1
    En, en, nn = Un
    s = np.sum(((E1 - En) / E_s) ** 2) + np.sum(((n1 - nn) / nH) ** 2)
    if not p.isothermal:
        s += np.sum(((e1 - en) / en) ** 2)
    nvars = 2 if p.isothermal else 3
    return float(np.sqrt(s / (p.ncells * nvars))), float(np.max(-E1 / E_s))


def step_scale(p: M.Params, dt: float, E, src) -> float:
    """E_s of a step (the weight of E in the norms)."""
    return max(float(np.max(E)), dt * float(np.max(src)), p.E_floor)


def advance(p: M.Params, t0: float, t_end: float, dt0: float, tau_tol: float, dt_max: float,
            nH, src, E, e, n, tol=None):
    """Adaptive steps from t0 to t_end; returns ((E, e, n), stats)."""
    if not (t_end > t0 and dt0 > 0 and tau_tol > 0 and dt_max > 0):
        raise ValueError("need t_end > t0 and dt0, tau_tol, dt_max > 0")
    eps_t = 1e-12 * max(abs(t_end), t_end - t0)
    t, dt = t0, min(dt0, dt_max)
    U = tuple(np.array(X, dtype=np.float64) for X in (E, e, n))
    stats = {"steps": 0, "rejected": 0, "rejected_negative": 0, "newton_its": 0, "dt": [],
             "w": []}
    rejects = 0
    while t_end - t > eps_t:
        last = dt >= t_end - t - eps_t
        dt_try = t_end - t if last else dt
        st = {}
        try:
            U1 = ON.step(p, t, dt_try, nH, src, *U, tol=tol, stats=st)
            w, neg = change_norm(p, step_scale(p, dt_try, U[0], src), U1, U, nH)
            ok = neg <= NEG_TOL and np.isfinite(w)
            stats["rejected_negative"] += int(neg > NEG_TOL)
        except (ON.NewtonFailure, FloatingPointError):
            ok = False
        if not ok:
            stats["rejected"] += 1
            rejects += 1
            if rejects >= MAX_REJECTS:
                raise ON.NewtonFailure(f"step rejected {MAX_REJECTS} times in a row at t = {t}")
            dt = 0.5 * dt_try
            continue
        rejects = 0
        U = U1
        t = t_end if last else t + dt_try
        stats["steps"] += 1
        stats["newton_its"] += st.get("newton_its", 0)
        stats["dt"].append(dt_try)
        stats["w"].append(w)
        factor = min(GROWTH_MAX, max(SHRINK_MIN, tau_tol / w)) if w > 0 else GROWTH_MAX
        dt = min(dt_try * factor, dt_max)
    stats["dt_next"] = dt
    stats["t_reached"] = t
    return U, stats
