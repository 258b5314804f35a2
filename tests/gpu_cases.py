"""Shared helpers of the GPU parity tests: workload cases, oracle-built
inputs (both sides get the same arrays, all made by the oracle and the
seeded generators), GPU and oracle trajectories, error metrics."""
import numpy as np

import workloads as W
from oracle import model as OM, newton as ON

# name -> (workload id, dims, Workload field overrides)
CASES = {
    "stromgren16": (0, (16, 16, 16), {}),
    "lognormal_ragged": (2, (24, 20, 36), {}),
    "eds_cooling16": (1, (16, 16, 16), {}),
    "outflow_corner": (0, (16, 16, 16), {
        "bc": (W.BC_ZEROFLUX, W.BC_OUTFLOW) * 3, "sources": "corner"}),
    "theta06_smalldt": (2, (16, 16, 16), {"theta": 0.6, "dt_Myr": 0.02}),
    # tall grids: with smoother=2 the finest level runs the fused marching
    # sweep (its tiles need nz >= 64 and ny >= 16 in FP32, nz >= 32 and ny >= 8 in
    # FP64, nx >= 4)
    "lognormal_tall": (2, (8, 16, 64), {"n_sources": 6}),
    "stromgren_tall": (0, (8, 16, 64), {}),
    # several x chunks and ragged (y, z) tiles: the marching kernels take
    # 32-plane chunks (the second one 8 planes), FP32 tiles 16 x 64 (y: 16,
    # 16, 8; z: 64, 16) and FP64 tiles 8 x 32 (z: 32, 32, 16); the FP64
    # level below the finest (20 x 20 x 40) is ragged too
    "lognormal_mid": (2, (40, 40, 80), {"n_sources": 10}),
}

# solver parameters per case (on top of the workload's)
CASE_PARAMS = {"lognormal_tall": {"smoother": 2}, "stromgren_tall": {"smoother": 2},
               "lognormal_mid": {"smoother": 2}}


def case_params(name):
    return dict(CASE_PARAMS.get(name, {}))


def make_workload(name):
    cfg, dims, over = CASES[name]
    w = W.scaled(cfg, dims)
    for k, v in over.items():
        setattr(w, k, v)
    return w


def oracle_inputs(w, **poverrides):
    op = OM.params_from_workload(w, **poverrides)
    nH = W.density_field(w)
    src = OM.source_field(op, W.photon_rate_field(w))
    E, e, n = OM.initial_state(op, nH, w.x0, w.T0, w.E0)
    t0, dt, ns = OM.schedule(op, w)
    return op, dict(nH=nH, src=src, E=E, e=e, n=n, t0=t0, dt=dt)


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


def gpu_trajectory(w, inp, nsteps, dev="cuda:0", **prm_over):
    import paper_0908_2654_amd as P
    prm = P.params_from_workload(w, **prm_over)
    s = P.Solver(prm, device=dev)
    nH, src = to_dev(inp["nH"], dev), to_dev(inp["src"], dev)
    E, e, n = (to_dev(inp[k], dev) for k in ("E", "e", "n"))
    stats = []
    for k in range(nsteps):
        stats.append(s.step(inp["t0"] + k * inp["dt"], inp["dt"], nH, src, E, e, n))
    out = tuple(x.cpu().numpy() for x in (E, e, n))
    s.close()
    return out, stats


def oracle_trajectory(op, inp, nsteps, tol):
    E, e, n = inp["E"], inp["e"], inp["n"]
    stats = []
    for k in range(nsteps):
        st = {}
        E, e, n = ON.step(op, inp["t0"] + k * inp["dt"], inp["dt"], inp["nH"], inp["src"],
                          E, e, n, tol=tol, stats=st)
        stats.append(st)
    return (E, e, n), stats


def errors(g, o, nH, iso, phi_E_rel=1e-20):
    """Max relative errors with floors: E (phi_E = phi_E_rel max|E|), e (none),
    x_HII (1e-6); plus the normwise E error."""
    Eg, eg, ng = g
    Eo, eo, no = o
    phi = phi_E_rel * np.max(np.abs(Eo))
    err = {
        "E": float(np.max(np.abs(Eg - Eo) / np.maximum(np.abs(Eo), phi))),
        "E_l2": float(np.linalg.norm(Eg - Eo) / np.linalg.norm(Eo)),
        "x": float(np.max(np.abs(ng - no) / nH / np.maximum(1.0 - no / nH, 1e-6))),
    }
    if not iso:
        err["e"] = float(np.max(np.abs(eg - eo) / np.abs(eo)))
    return err


_ORACLE_CACHE = {}


def cached(key, fn):
    """Memoise an oracle result for the session (large cases are reused by
    several tests)."""
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = fn()
    return _ORACLE_CACHE[key]


def elementwise(g, o, floor_rel):
    """max_P |g - o| / max(|o|, floor_rel * max|o|)."""
    g = np.asarray(g).ravel()
    o = np.asarray(o).ravel()
    fl = floor_rel * np.max(np.abs(o))
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), fl)))
