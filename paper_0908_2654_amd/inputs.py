"""Device inputs of a workload for the GPU path (initial state, emissivity,
time schedule).  Marshalling only: the seeded generators make the density
and the photon rates on the host; the library turns them into the step's
fields (rh_initial_state, rh_source_field) and supplies the cosmic-time
relation (rh_cosmic_time), so nothing here depends on the CPU oracle.
"""
import numpy as np
import torch

import workloads as W

from .solver import Solver, cosmic_time


def schedule(w, params):
    """(t0, dt, nsteps) in seconds for a workload."""
    if w.dt_Myr is not None:
        t0 = 0.0 if w.cosmology == W.COSMO_STATIC else cosmic_time(params, 1.0 / (1.0 + w.z_start))
        return t0, w.dt_Myr * W.MYR_S, w.nsteps
    t0 = cosmic_time(params, 1.0 / (1.0 + w.z_start))
    t1 = cosmic_time(params, 1.0 / (1.0 + w.z_end))
    return t0, (t1 - t0) / w.nsteps, w.nsteps


def device_inputs(w, solver: Solver, nH_host=None):
    """dict of device tensors nH, src, E, e, nHI (float64) for workload w."""
    dev = solver.device
    nH = W.density_field(w) if nH_host is None else nH_host
    Q = W.photon_rate_field(w)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)  # noqa: E731
    nH_t = to(nH)
    out = {"nH": nH_t, "src": torch.empty_like(nH_t), "E": torch.empty_like(nH_t),
           "e": torch.empty_like(nH_t), "nHI": torch.empty_like(nH_t)}
    solver.source_field(to(Q), out["src"])
    T = w.T_iso if w.isothermal else w.T0
    solver.initial_state(nH_t, w.x0, T, w.E0, out["E"], out["e"], out["nHI"])
    return out
