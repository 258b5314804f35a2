"""Device inputs of a workload for the GPU path (initial state, emissivity,
time schedule).  Input preparation only; the step itself runs in librh.

The emissivity uses the library's own mean photon energy of the spectrum
(rh_get_constants) and the schedule its own cosmic-time relation
(rh_cosmic_time), so nothing here depends on the CPU oracle.
"""
import numpy as np
import torch

import workloads as W

from .solver import Solver, cosmic_time

K_BOLTZ = 1.380649e-16
M_H = 1.6735575e-24


def schedule(w, params):
    """(t0, dt, nsteps) in seconds for a workload."""
    if w.dt_Myr is not None:
        t0 = 0.0 if w.cosmology == W.COSMO_STATIC else cosmic_time(params, 1.0 / (1.0 + w.z_start))
        return t0, w.dt_Myr * W.MYR_S, w.nsteps
    t0 = cosmic_time(params, 1.0 / (1.0 + w.z_start))
    t1 = cosmic_time(params, 1.0 / (1.0 + w.z_end))
    return t0, (t1 - t0) / w.nsteps, w.nsteps


def gas_energy(T, x, gamma=5.0 / 3.0):
    mu = 1.0 / (1.0 + x)
    return K_BOLTZ * T / ((gamma - 1.0) * mu * M_H)


def device_inputs(w, solver: Solver, nH_host=None):
    """dict of device tensors nH, src, E, e, nHI (float64) for workload w."""
    dev = solver.device
    nH = W.density_field(w) if nH_host is None else nH_host
    Q = W.photon_rate_field(w)
    c = solver.constants()
    src = Q * (c["eps_bar"] / c["h"] ** 3)
    T = w.T_iso if w.isothermal else w.T0
    nH_t = torch.from_numpy(np.ascontiguousarray(nH)).to(dev)
    out = {
        "nH": nH_t,
        "src": torch.from_numpy(src).to(dev),
        "E": torch.full(w.dims, w.E0, dtype=torch.float64, device=dev),
        "e": torch.full(w.dims, gas_energy(T, w.x0, solver.params.gamma), dtype=torch.float64,
                        device=dev),
        "nHI": (1.0 - w.x0) * nH_t,
    }
    return out
