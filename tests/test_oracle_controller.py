"""Pins of the oracle's adaptive step controller (oracle/controller.py)
against things the controller does not compute itself: an ODE reference
solution, the controller's own equilibrium, exact landing on t_end, and the
positivity safeguard of the theta = 0.51 path."""
import numpy as np
import pytest
from scipy import integrate

import workloads as W
from gpu_cases import CASES, make_workload, oracle_inputs
from oracle import controller as C
from oracle import model as M
from oracle.constants import MYR_S

import test_oracle_pins as TP


def _uniform_case():
    w = TP._uniform_cell_workload(W.SPEC_MONO, True, W.COSMO_STATIC)
    p = M.params_from_workload(w)
    nHv, srcv, T_span = 1e-3, 2e-27, 2.0 * MYR_S
    nH = np.full(w.dims, nHv)
    src = np.full(w.dims, srcv)
    U0 = M.initial_state(p, nH, 1.2e-3, 100.0, 1e-35)
    f = TP._ode_rhs(p, nHv, srcv, None)
    scale = np.array([srcv * T_span, nHv, U0[1].flat[0]])

    def g(tau, y):
        return np.array(f(tau * T_span, y * scale)) * T_span / scale
    y0 = np.array([U0[0].flat[0], U0[2].flat[0], U0[1].flat[0]]) / scale
    sol = integrate.solve_ivp(g, (0.0, 1.0), y0, method="Radau", rtol=1e-12, atol=1e-14)
    assert sol.status == 0, sol.message
    return p, nH, src, U0, T_span, sol.y[:, -1] * scale


def test_controller_first_order_in_tau_and_lands_on_t_end():
    """Uniform medium with a uniform source: the final state converges to
    the ODE solution linearly in tau_tol (backward Euler), the weighted
    change per step settles at tau_tol, and the steps sum to the interval."""
    p, nH, src, U0, T_span, ref = _uniform_case()
    errs = []
    for tau in (1e-2, 2.5e-3):
        (E, e, n), st = C.advance(p, 0.0, T_span, T_span / 1000, tau, T_span, nH, src, *U0,
                                  tol=1e-13)
        errs.append(max(abs(E.flat[0] - ref[0]) / abs(ref[0]), abs(n.flat[0] - ref[1]) / nH.flat[0]))
        assert st["rejected"] == 0
        assert st["t_reached"] == T_span
        assert sum(st["dt"]) == pytest.approx(T_span, rel=1e-12)
        assert np.median(np.array(st["w"]) / tau) == pytest.approx(1.0, rel=0.3)
    assert 2.5 < errs[0] / errs[1] < 8.0, errs


def test_controller_theta051_rejects_and_stays_admissible():
    """theta = 0.51 with 0.5 Myr steps on the optically thick Stromgren
    sphere: the explicit half of the step over-ionises (the local solution
    leaves [0, n_H], so the local solve fails) or flips the sign of E;
    such attempts are rejected and halved, and the run ends admissible."""
    CASES["sg8"] = (0, (8, 8, 8), {"theta": 0.51})
    w = make_workload("sg8")
    op, inp = oracle_inputs(w)
    t0, t1 = inp["t0"], inp["t0"] + 1.0 * MYR_S
    (E, e, n), st = C.advance(op, t0, t1, 0.5 * MYR_S, 1e-2, 0.5 * MYR_S, inp["nH"], inp["src"],
                              inp["E"], inp["e"], inp["n"])
    assert st["rejected"] >= 1 and st["steps"] >= 2
    assert st["t_reached"] == t1
    assert E.min() >= -1e-10 * max(E.max(), float(np.max(inp["src"])) * min(st["dt"]))
    x = 1.0 - n / inp["nH"]
    assert np.all(x >= 0.0) and np.all(x <= 1.0) and x.mean() > 0.01


def test_controller_rejects_invalid_arguments():
    p, nH, src, U0, T_span, _ = _uniform_case()
    with pytest.raises(ValueError):
        C.advance(p, 1.0, 1.0, 0.1, 1e-3, 1.0, nH, src, *U0)
    with pytest.raises(ValueError):
        C.advance(p, 0.0, 1.0, 0.1, 0.0, 1.0, nH, src, *U0)
