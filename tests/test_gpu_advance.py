"""rh_advance (adaptive implicit steps) through the C ABI against the
oracle's controller (oracle/controller.py), and a long theta = 0.51 run."""
import numpy as np
import pytest

import workloads as W
from gpu_cases import CASES, make_workload, oracle_inputs, to_dev
from oracle import controller as OC
from oracle import model as OM
from oracle.constants import MYR_S

pytestmark = pytest.mark.gpu


def _gpu_advance(w, inp, t0, t1, dt0, tau, dt_max, dev, **prm):
    import paper_0908_2654_amd as P
    s = P.Solver(P.params_from_workload(w, **prm), device=dev)
    d = lambda a: to_dev(a, dev)  # noqa: E731
    E, e, n = d(inp["E"]), d(inp["e"]), d(inp["n"])
    st = s.advance(t0, t1, dt0, tau, dt_max, d(inp["nH"]), d(inp["src"]), E, e, n)
    s.close()
    return (E.cpu().numpy(), e.cpu().numpy(), n.cpu().numpy()), st


def _compare(g, o, nH, gst, ost):
    print("gpu", {k: gst[k] for k in ("steps", "rejected", "dt_min", "dt_max", "dt_next")},
          "oracle", ost["steps"], ost["rejected"], min(ost["dt"]), max(ost["dt"]), ost["dt_next"])
    assert gst["steps"] == ost["steps"] and gst["rejected"] == ost["rejected"]
    assert gst["dt_min"] == pytest.approx(min(ost["dt"]), rel=1e-6)
    assert gst["dt_max"] == pytest.approx(max(ost["dt"]), rel=1e-6)
    assert gst["dt_next"] == pytest.approx(ost["dt_next"], rel=1e-6)
    assert gst["change_last"] == pytest.approx(ost["w"][-1], rel=1e-6)
    Eg, eg, ng = g
    Eo, eo, no = o
    assert np.max(np.abs(Eg - Eo)) <= 1e-8 * np.max(np.abs(Eo))
    assert np.max(np.abs(ng - no) / nH) <= 1e-8


def test_advance_theta051_matches_oracle(hip_device):
    """theta = 0.51, 0.5 Myr first step on an 8^3 Stromgren sphere: the same
    rejections, accepted steps and step sizes as the oracle's controller,
    and the same final state (both sides converge Newton to 1e-12)."""
    CASES["sg8"] = (0, (8, 8, 8), {"theta": 0.51})
    w = make_workload("sg8")
    op, inp = oracle_inputs(w, newton_tol=1e-12)
    t0, t1 = inp["t0"], inp["t0"] + 1.0 * MYR_S
    o, ost = OC.advance(op, t0, t1, 0.5 * MYR_S, 1e-2, 0.5 * MYR_S, inp["nH"], inp["src"],
                        inp["E"], inp["e"], inp["n"], tol=1e-12)
    g, gst = _gpu_advance(w, inp, t0, t1, 0.5 * MYR_S, 1e-2, 0.5 * MYR_S, hip_device,
                          newton_tol=1e-12, precision=0)
    assert ost["rejected"] >= 1
    assert gst["t_reached"] == t1
    _compare(g, o, inp["nH"], gst, ost)


def test_advance_uniform_medium_matches_oracle(hip_device):
    """Uniform medium with a uniform source (2^3 cells): the controller's
    step sequence ends where the oracle's does."""
    import test_oracle_pins as TP
    w = TP._uniform_cell_workload(W.SPEC_MONO, True, W.COSMO_STATIC)
    op = OM.params_from_workload(w, newton_tol=1e-12)
    nH = np.full(w.dims, 1e-3)
    src = np.full(w.dims, 2e-27)
    E, e, n = OM.initial_state(op, nH, 1.2e-3, 100.0, 1e-35)
    inp = {"nH": nH, "src": src, "E": E, "e": e, "n": n}
    T = 2.0 * MYR_S
    o, ost = OC.advance(op, 0.0, T, T / 1000, 1e-2, T, nH, src, E, e, n, tol=1e-12)
    g, gst = _gpu_advance(w, inp, 0.0, T, T / 1000, 1e-2, T, hip_device, newton_tol=1e-12,
                          precision=0)
    _compare(g, o, nH, gst, ost)


def test_advance_theta051_soak_mixed(hip_device):
    """Long adaptive run of the paper's theta = 0.51 setting on a 32^3
    lognormal field with 32 sources (mixed precision, tau_tol = 1e-3):
    it reaches the end, every state stays admissible."""
    CASES["ln32"] = (2, (32, 32, 32), {"theta": 0.51})
    w = make_workload("ln32")
    op, inp = oracle_inputs(w)
    t0 = inp["t0"]
    t1 = t0 + 5.0 * MYR_S
    (E, e, n), st = _gpu_advance(w, inp, t0, t1, 0.5 * MYR_S, 1e-3, 0.5 * MYR_S, hip_device,
                                 precision=1)
    print(st)
    assert st["t_reached"] == t1 and st["steps"] >= 10
    assert np.all(np.isfinite(E)) and np.all(np.isfinite(e)) and np.all(np.isfinite(n))
    x = 1.0 - n / inp["nH"]
    assert np.all(x >= -1e-12) and np.all(x <= 1.0 + 1e-12)
    assert np.all(e > 0)
    assert E.min() >= -1e-10 * E.max()
