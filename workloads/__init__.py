"""Seeded synthetic inputs for the coupled implicit radiation step.

This module is shared by the FP64 CPU oracle and the GPU path.  It holds
workload definitions (sizes, physical inputs, seeds) and the seeded
generators of the input fields: hydrogen density n_H, the list of point
sources (cell, photon rate) and the initial temperature / ionised fraction.
It contains none of the method's arithmetic: no grey constants, no rates,
no cosmology, no conversion of temperature into gas energy and no
conversion of photon rates into emissivity.  Each side does those itself.

Units: CGS.  Lengths are given both in kpc (as the workloads state them)
and converted to cm with the IAU parsec; times in Myr use the Julian year.

Field layout everywhere: C order [x][y][z], z fastest, float64.

The paper runs its reionisation test on a density field from a
cosmological N-body/hydro simulation, and its verification on a uniform
medium.  Neither dataset exists here; the lognormal Gaussian-random-field
densities below stand in for the simulated density (same grid sizes, a
power-law spectrum P(k) ~ k^-3 and a stated log-density spread), and the
uniform Stromgren-sphere media follow the verification section directly.
"""
from __future__ import annotations

import copy
import math
import dataclasses
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

KPC_CM = 3.0856775814913673e21      # 1 kpc in cm (IAU parsec)
MPC_CM = 1.0e3 * KPC_CM
MYR_S = 1.0e6 * 365.25 * 86400.0    # 1 Myr in s (Julian year)

# boundary-condition codes (per face x-,x+,y-,y+,z-,z+)
BC_ZEROFLUX = 0
BC_PERIODIC = 1
BC_OUTFLOW = 2

# cosmology codes
COSMO_STATIC = 0
COSMO_EDS = 1
COSMO_FLAT_LCDM = 2
COSMO_OPEN = 3

# spectrum codes
SPEC_MONO = 0
SPEC_BLACKBODY = 1

# recombination-rate codes
RATES_CONST = 0
RATES_FIT = 1

# cooling mask bits
COOL_RECB = 1
COOL_COLLEXC = 2
COOL_COMPTON = 4

PREC_FP64 = 0
PREC_MIXED = 1


@dataclass
class Workload:
    """One synthetic workload: grid, medium, sources, physics switches, schedule."""
    name: str
    dims: tuple                       # (nx, ny, nz)
    box_comoving_cm: float            # x edge of the box, comoving cm
    bc: tuple                         # 6 boundary codes
    # medium
    nH_mean: float                    # comoving cm^-3
    density: str = "uniform"          # "uniform" | "lognormal"
    sigma_ln: float = 0.0
    pk_index: float = -3.0
    seed_field: int = 0
    x0: float = 1.2e-3                # initial ionised fraction
    T0: float = 1.0e4                 # initial temperature, K
    E0: float = 1.0e-35               # initial radiation energy, erg cm^-3 comoving
    # sources
    sources: str = "centre"           # "centre" | "corner" | "random"
    n_sources: int = 1
    Q_median: float = 5.0e48          # photons / s
    sigma_lnQ: float = 0.0
    seed_src: int = 0
    # physics
    isothermal: bool = False
    T_iso: float = 1.0e4
    spectrum: int = SPEC_BLACKBODY
    T_bb: float = 1.0e5
    hnu0_eV: float = 13.6
    sigma0: float = 6.3e-18
    rates: int = RATES_FIT
    alphaB_const: float = 2.59e-13
    cooling: int = COOL_RECB | COOL_COLLEXC | COOL_COMPTON
    cosmology: int = COSMO_STATIC
    hubble_h: float = 0.7
    Omega_m: float = 1.0
    Omega_L: float = 0.0
    # schedule: static runs give dt directly; expanding runs give z range
    dt_Myr: Optional[float] = None
    z_start: Optional[float] = None
    z_end: Optional[float] = None
    nsteps: int = 1
    # solver
    theta: float = 1.0
    newton_tol: float = 1.0e-8
    precision: int = PREC_FP64
    mg_pre: int = 2
    mg_post: int = 2
    extra: dict = field(default_factory=dict)

    @property
    def ncells(self) -> int:
        return int(np.prod(self.dims))

    def replace(self, **kw) -> "Workload":
        w = copy.deepcopy(self)
        for k, v in kw.items():
            if not hasattr(w, k):
                raise AttributeError(k)
            setattr(w, k, v)
        return w


# ---------------------------------------------------------------------------
# The five benchmark workloads.  Stated values come from the workload
# descriptions; the values they leave open are fixed here: box and dt of the
# static lognormal runs, EdS h = 0.5, a blackbody spectrum whenever
# photoheating is on, periodic boundaries for the lognormal fields, zero-flux
# walls for the single-source spheres.
# ---------------------------------------------------------------------------
CONFIGS = {
    0: Workload(
        name="stromgren16_iso_fp64", dims=(16, 16, 16),
        box_comoving_cm=6.6 * KPC_CM, bc=(BC_ZEROFLUX,) * 6,
        nH_mean=1.0e-3, x0=1.2e-3, T0=1.0e4,
        sources="centre", n_sources=1, Q_median=5.0e48,
        isothermal=True, T_iso=1.0e4, spectrum=SPEC_MONO, sigma0=6.3e-18,
        rates=RATES_CONST, alphaB_const=2.59e-13, cooling=0,
        cosmology=COSMO_STATIC, dt_Myr=0.5, nsteps=20,
        newton_tol=1.0e-8, precision=PREC_FP64),
    1: Workload(
        name="stromgren64_eds_fp64", dims=(64, 64, 64),
        box_comoving_cm=80.0 * KPC_CM, bc=(BC_ZEROFLUX,) * 6,
        nH_mean=1.7e-7, x0=1.2e-3, T0=100.0,
        sources="centre", n_sources=1, Q_median=5.0e48,
        spectrum=SPEC_BLACKBODY, rates=RATES_FIT,
        cosmology=COSMO_EDS, hubble_h=0.5, Omega_m=1.0, Omega_L=0.0,
        z_start=10.0, z_end=4.0, nsteps=200,
        newton_tol=1.0e-8, precision=PREC_FP64),
    2: Workload(
        name="lognormal128_mixed", dims=(128, 128, 128),
        box_comoving_cm=6.6 * KPC_CM, bc=(BC_PERIODIC,) * 6,
        nH_mean=1.0e-3, density="lognormal", sigma_ln=1.0, seed_field=2,
        x0=1.2e-3, T0=100.0,
        sources="random", n_sources=32, Q_median=1.0e48, sigma_lnQ=1.0, seed_src=1002,
        spectrum=SPEC_BLACKBODY, rates=RATES_FIT,
        cosmology=COSMO_STATIC, dt_Myr=0.5, nsteps=20,
        newton_tol=1.0e-8, precision=PREC_MIXED),
    3: Workload(
        name="lognormal256_adjoint", dims=(256, 256, 256),
        box_comoving_cm=6.6 * KPC_CM, bc=(BC_PERIODIC,) * 6,
        nH_mean=1.0e-3, density="lognormal", sigma_ln=1.0, seed_field=3,
        x0=1.2e-3, T0=100.0,
        sources="random", n_sources=128, Q_median=1.0e48, sigma_lnQ=1.0, seed_src=1003,
        spectrum=SPEC_BLACKBODY, rates=RATES_FIT,
        cosmology=COSMO_STATIC, dt_Myr=0.5, nsteps=10,
        newton_tol=1.0e-8, precision=PREC_MIXED,
        extra={"seed_fd_cells": 2003, "n_fd_cells": 64, "fd_rel_step": 1.0e-6}),
    4: Workload(
        name="reion512_lcdm_mixed", dims=(512, 512, 512),
        box_comoving_cm=8.0 * MPC_CM, bc=(BC_PERIODIC,) * 6,
        nH_mean=1.7e-7, density="lognormal", sigma_ln=1.5, seed_field=4,
        x0=1.2e-3, T0=100.0,
        sources="random", n_sources=4096, Q_median=1.0e48, sigma_lnQ=1.0, seed_src=1004,
        spectrum=SPEC_BLACKBODY, rates=RATES_FIT,
        cosmology=COSMO_FLAT_LCDM, hubble_h=0.7, Omega_m=0.3, Omega_L=0.7,
        z_start=9.0, z_end=7.0, nsteps=50,
        newton_tol=1.0e-8, precision=PREC_MIXED,
        extra={"adjoint_last_steps": 8}),
}


# ---------------------------------------------------------------------------
# The four cosmological Stromgren-sphere runs of the verification section
# (its cosmology table): q0, z0, initial proper box L0, h, Omega_m, Omega_L,
# Omega_b.  One monochromatic 13.6 eV source of 5e48 photons/s in the lower
# corner (reflecting lower walls, outflow upper walls: the octant of a
# sphere, so the corner cell gets Q/8), constant case-B recombination
# (2.59e-13 cm^3/s at 1e4 K, the analytic solution's assumption), initially
# neutral gas, E = 1e-35, from z0 to z = 0.  The comoving hydrogen density is
# Omega_b times the critical density over m_H (at z0 = 4 this is the stated
# initial mass density: 1.175e-28 g cm^-3 for q0 = 0.5, 2.35e-28 for 0.05).
# ---------------------------------------------------------------------------
SG_ROWS = [
    (0.5, 4.0, 80.0, 0.5, 1.0, 0.0, 0.2),
    (0.05, 4.0, 60.0, 1.0, 0.1, 0.0, 0.1),
    (0.5, 10.0, 36.0, 0.5, 1.0, 0.0, 0.2),
    (0.05, 10.0, 27.0, 1.0, 0.1, 0.0, 0.1),
]
_G_CGS = 6.674e-8
_M_H = 1.6735575e-24
_H100 = 3.2407789e-18  # 100 km/s/Mpc in 1/s


def shapiro_giroux(row: int, dims=(32, 32, 32)) -> Workload:
    """Workload of row `row` (0-3) of the verification table."""
    q0, z0, L0_kpc, h, Om, OL, Ob = SG_ROWS[row]
    rho_crit = 3.0 * (h * _H100) ** 2 / (8.0 * math.pi * _G_CGS)
    return Workload(
        name=f"shapiro_giroux_q{q0:g}_z{z0:g}", dims=tuple(dims),
        box_comoving_cm=L0_kpc * (1.0 + z0) * KPC_CM, bc=(BC_ZEROFLUX, BC_OUTFLOW) * 3,
        nH_mean=Ob * rho_crit / _M_H, x0=0.0, T0=1.0e4, E0=1.0e-35,
        sources="corner", n_sources=1, Q_median=5.0e48,
        isothermal=True, T_iso=1.0e4, spectrum=SPEC_MONO, sigma0=6.3e-18,
        rates=RATES_CONST, alphaB_const=2.59e-13, cooling=0,
        cosmology=COSMO_EDS if q0 == 0.5 else COSMO_OPEN, hubble_h=h, Omega_m=Om,
        Omega_L=OL, z_start=z0, z_end=0.0, nsteps=1, theta=0.51,
        newton_tol=1.0e-8, precision=PREC_FP64,
        extra={"q0": q0, "z0": z0, "tau_tol": 1.0e-3})


def get(cfg) -> Workload:
    """Return a copy of a numbered workload (or pass a Workload through)."""
    if isinstance(cfg, Workload):
        return copy.deepcopy(cfg)
    return copy.deepcopy(CONFIGS[int(cfg)])


def scaled(cfg, dims) -> Workload:
    """Same medium, physics and seeds on another grid (same box)."""
    w = get(cfg)
    w.dims = tuple(int(d) for d in dims)
    return w


# ---------------------------------------------------------------------------
# generators
# ---------------------------------------------------------------------------
def gaussian_random_field(dims, pk_index: float, seed: int) -> np.ndarray:
    """Seeded periodic Gaussian random field with P(k) ~ |k|^pk_index.

    White noise is drawn in real space, filtered by sqrt(P(k)) in Fourier
    space (P(0) = 0), and the result normalised to sample mean 0, variance 1.
    """
    import scipy.fft as sfft
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nx, ny, nz))
    wk = sfft.rfftn(w, workers=-1)
    del w
    mx = np.fft.fftfreq(nx) * nx
    my = np.fft.fftfreq(ny) * ny
    mz = np.fft.rfftfreq(nz) * nz
    k2 = (mx[:, None, None] ** 2 + my[None, :, None] ** 2 + mz[None, None, :] ** 2)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (0.25 * pk_index), 0.0)
    wk *= amp
    del amp, k2
    d = sfft.irfftn(wk, s=(nx, ny, nz), workers=-1)
    del wk
    d -= d.mean()
    d /= d.std()
    return d


def velocity_field(dims, v_rms: float, pk_index: float = -3.0, seed: int = 100):
    """Seeded cell-centred peculiar velocity (vx, vy, vz) [cm/s]: three
    independent periodic Gaussian random fields with P(k) ~ |k|^pk_index,
    each scaled to standard deviation v_rms (compressive and rotational
    parts alike; smooth on the grid scale for pk_index <= -3)."""
    return tuple(v_rms * gaussian_random_field(dims, pk_index, seed + d) for d in range(3))


def density_field(w: Workload) -> np.ndarray:
    """Comoving hydrogen number density n_H [cm^-3], shape dims, float64."""
    if w.density == "uniform":
        return np.full(w.dims, w.nH_mean, dtype=np.float64)
    if w.density == "lognormal":
        d = gaussian_random_field(w.dims, w.pk_index, w.seed_field)
        s = w.sigma_ln
        n = np.exp(s * d - 0.5 * s * s)
        n *= w.nH_mean / n.mean()
        return n
    raise ValueError(w.density)


def source_list(w: Workload):
    """Point sources as (flat cell indices int64, photon rates float64 [1/s]).

    centre: the source is split equally over the 8 cells that share the
            grid-centre vertex (exact octant symmetry on even grids).
    corner: one eighth of the source in cell (0,0,0) (an octant of a full
            sphere around the lower corner).
    random: n_sources distinct cells drawn uniformly without replacement,
            rates lognormal with the given median and log-spread.
    """
    nx, ny, nz = w.dims
    if w.sources == "centre":
        cx, cy, cz = nx // 2, ny // 2, nz // 2
        cells = []
        for i in (cx - 1, cx):
            for j in (cy - 1, cy):
                for k in (cz - 1, cz):
                    cells.append((i * ny + j) * nz + k)
        return np.array(cells, dtype=np.int64), np.full(8, w.Q_median / 8.0)
    if w.sources == "corner":
        return np.array([0], dtype=np.int64), np.array([w.Q_median / 8.0])
    if w.sources == "random":
        rng = np.random.default_rng(w.seed_src)
        cells = rng.choice(nx * ny * nz, size=w.n_sources, replace=False).astype(np.int64)
        Q = w.Q_median * np.exp(w.sigma_lnQ * rng.standard_normal(w.n_sources))
        return cells, Q
    if w.sources == "none":
        return np.zeros(0, dtype=np.int64), np.zeros(0)
    raise ValueError(w.sources)


def photon_rate_field(w: Workload) -> np.ndarray:
    """Photon emission rate per cell [photons/s], shape dims (duplicates add)."""
    cells, Q = source_list(w)
    out = np.zeros(w.ncells, dtype=np.float64)
    np.add.at(out, cells, Q)
    return out.reshape(w.dims)


def fd_cells(w: Workload, n: Optional[int] = None, seed: Optional[int] = None) -> np.ndarray:
    """Seeded cells (flat indices) for finite-difference gradient checks."""
    seed = w.extra.get("seed_fd_cells", 2000) if seed is None else seed
    n = w.extra.get("n_fd_cells", 64) if n is None else n
    rng = np.random.default_rng(seed)
    return rng.choice(w.ncells, size=n, replace=False).astype(np.int64)


def schedule(w: Workload):
    """Describes the time schedule without computing any cosmology.

    Returns ("dt", dt_seconds) for runs with a fixed step, or
    ("z", z_start, z_end) for expanding runs, whose step is uniform in
    cosmic time between those redshifts (each side converts z to t itself).
    """
    if w.dt_Myr is not None:
        return ("dt", w.dt_Myr * MYR_S)
    return ("z", w.z_start, w.z_end)
