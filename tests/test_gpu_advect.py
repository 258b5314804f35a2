"""rh_advect (donor-cell advection of the step's fields, operator split step
(iv)) through the C ABI against the oracle (oracle/advection.py): whole
fields on small grids for both kernels (one thread per cell, and the x-marching
tiles on grids with nz >= 64, ny >= 8, ragged tiles included) and every wall
type; sampled cells of the 512^3 periodic reionisation volume; a split step
(advection, then the implicit step) against the oracle's; error paths."""
import numpy as np
import pytest

import workloads as W
from gpu_cases import errors, to_dev
from oracle import advection as OA
from oracle import model as OM
from oracle.constants import MYR_S

pytestmark = pytest.mark.gpu

P_, Z_, O_ = W.BC_PERIODIC, W.BC_ZEROFLUX, W.BC_OUTFLOW

# name -> (config, dims, overrides, target Courant number over dt)
ADV_CASES = {
    "simple_periodic": (2, (12, 10, 14), {}, 2.5),
    "simple_iso_walls": (0, (7, 9, 5), {"bc": (O_, Z_, Z_, O_, P_, P_), "isothermal": True}, 1.7),
    "march_periodic": (2, (16, 16, 64), {}, 2.5),
    "march_ragged_walls": (2, (20, 12, 72), {"bc": (O_, O_, Z_, Z_, P_, P_)}, 3.2),
    "march_ragged_mixed": (2, (6, 10, 66), {"bc": (P_, P_, Z_, O_, O_, Z_)}, 1.3),
    "march_iso_eds": (1, (16, 8, 64), {"isothermal": True}, 2.2),
    "march_lcdm": (4, (8, 16, 128), {}, 4.6),
}


def _case(name):
    cfg, dims, over, C = ADV_CASES[name]
    w = W.scaled(cfg, dims)
    for k, v in over.items():
        setattr(w, k, v)
    return w, C


def _fields(w, seed=7, smooth=True):
    """n_H from the workload; E, n_HI, e as independent seeded random fields
    (smooth Gaussian random fields, or white noise when smooth is False)."""
    nH = W.density_field(w)
    if smooth:
        g = [W.gaussian_random_field(w.dims, -2.0, seed + i) for i in range(3)]
    else:
        rng = np.random.default_rng(seed)
        g = [rng.standard_normal(w.dims) for _ in range(3)]
    E = 1e-14 * np.exp(g[0])
    n = nH / (1.0 + np.exp(g[1]))
    e = 1e12 * np.exp(0.5 * g[2])
    return nH, E, e, n


def _velocity_and_dt(op, w, t0, C):
    v = W.velocity_field(w.dims, 3.0e7, seed=101)
    C1 = OA.courant(op, v, 1.0 / (op.cosmo.a(t0) * op.h))
    return v, C / C1


def _gpu_advect(w, dev, t0, dt, v, nH, E, e, n, cfl):
    import paper_0908_2654_amd as P
    s = P.Solver(P.params_from_workload(w), device=dev)
    d = lambda a: to_dev(a, dev)  # noqa: E731
    g = [d(nH), d(E), d(e), d(n)]
    st = s.advect(t0, dt, [d(c) for c in v], *g, cfl=cfl)
    s.close()
    return [x.cpu().numpy() for x in g], st


@pytest.mark.parametrize("name", list(ADV_CASES))
def test_advect_parity(hip_device, name):
    w, C = _case(name)
    op = OM.params_from_workload(w)
    t0 = OM.schedule(op, w)[0]
    nH, E, e, n = _fields(w)
    v, dt = _velocity_and_dt(op, w, t0, C)
    cfl = 0.9
    (onH, oE, oe, on), m = OA.advect(op, t0, dt, v, nH, E, e, n, cfl)
    (gnH, gE, ge, gn), st = _gpu_advect(w, hip_device, t0, dt, v, nH, E, e, n, cfl)
    print(name, "substeps", m, st)
    assert st["substeps"] == m and m > 1
    assert st["courant"] == pytest.approx(C, rel=1e-12)
    for g, o in ((gnH, onH), (gE, oE), (gn, on)):
        assert np.max(np.abs(g - o)) <= 1e-13 * np.max(np.abs(o))
    if w.isothermal:
        np.testing.assert_array_equal(ge, e)
    else:
        assert np.max(np.abs(ge - oe) / oe) <= 1e-13


def test_advect_one_substep_to_rounding(hip_device):
    """One substep: both sides take the same operations in the same order
    (up to fused multiply-adds), so the march kernel agrees with the oracle
    to a few roundings of the fluxes."""
    w, _ = _case("march_ragged_walls")
    op = OM.params_from_workload(w)
    t0 = OM.schedule(op, w)[0]
    nH, E, e, n = _fields(w, seed=17)
    v, dt = _velocity_and_dt(op, w, t0, 0.8)
    (onH, oE, oe, on), m = OA.advect(op, t0, dt, v, nH, E, e, n, 0.9)
    (gnH, gE, ge, gn), st = _gpu_advect(w, hip_device, t0, dt, v, nH, E, e, n, 0.9)
    assert m == 1 and st["substeps"] == 1
    for g, o in ((gnH, onH), (gE, oE), (gn, on), (ge, oe)):
        assert np.max(np.abs(g - o) / np.abs(o)) <= 1e-14


def test_advect_full_size_sampled(hip_device):
    """512^3 periodic reionisation volume with a 300 km/s random velocity
    field over three substeps: the substep count matches the oracle's on the
    whole grid, sums are conserved, fields stay positive, and sampled cells
    (corners included) match the oracle run on a periodic block around each
    (the block is wider than the three substeps' dependence cone)."""
    w = W.get(4)
    op = OM.params_from_workload(w)
    t0 = OM.schedule(op, w)[0]
    nH, E, e, n = _fields(w, smooth=False)
    v, dt = _velocity_and_dt(op, w, t0, 2.5)
    m, C = OA.substeps(op, t0, dt, v, 0.9)
    assert m == 3
    import paper_0908_2654_amd as P
    dev = hip_device
    s = P.Solver(P.params_from_workload(w), device=dev)
    g = [to_dev(x, dev) for x in (nH, E, e, n)]
    gv = [to_dev(c, dev) for c in v]
    sums0 = [g[0].sum().item(), g[1].sum().item(), g[3].sum().item(), (g[0] * g[2]).sum().item()]
    st = s.advect(t0, dt, gv, *g, cfl=0.9)
    s.close()
    assert st["substeps"] == m
    assert st["courant"] == pytest.approx(C, rel=1e-12)
    sums1 = [g[0].sum().item(), g[1].sum().item(), g[3].sum().item(), (g[0] * g[2]).sum().item()]
    for a, b in zip(sums0, sums1):
        assert b == pytest.approx(a, rel=1e-12)
    assert min(x.min().item() for x in g) > 0.0
    rng = np.random.default_rng(5)
    N0 = w.dims[0]
    cells = [(0, 0, 0), (N0 - 1, N0 - 1, N0 - 1), (0, N0 - 1, 7), (N0 - 1, 3, 0)]
    cells += [tuple(int(c) for c in rng.integers(0, N0, 3)) for _ in range(28)]
    r = m + 2
    bw = 2 * r + 1
    bp = op.with_(dims=(bw, bw, bw), box=op.h * bw)
    for c in cells:
        idx = [np.arange(c[d] - r, c[d] + r + 1) % N0 for d in range(3)]
        cut = lambda X: X[np.ix_(*idx)]  # noqa: E731
        bnH, bE, be, bn = OA.advect_substeps(bp, t0, dt, m, [cut(x) for x in v], cut(nH), cut(E),
                                             cut(e), cut(n))
        got = [g[k][c].item() for k in range(4)]
        want = [bnH[r, r, r], bE[r, r, r], be[r, r, r], bn[r, r, r]]
        for a, b in zip(got, want):
            assert a == pytest.approx(b, rel=1e-13), c


def test_split_step_matches_oracle(hip_device):
    """Two operator-split steps (advection, then the implicit step from the
    advected fields) on a 24x20x36 lognormal volume with sources: the same
    trajectory as the oracle's split steps (FP64 path, Newton to 1e-12)."""
    import paper_0908_2654_amd as P
    w = W.scaled(2, (24, 20, 36))
    op = OM.params_from_workload(w, newton_tol=1e-12)
    nH = W.density_field(w)
    src = OM.source_field(op, W.photon_rate_field(w))
    E, e, n = OM.initial_state(op, nH, w.x0, w.T0, w.E0)
    t0, dt, _ = OM.schedule(op, w)
    v = W.velocity_field(w.dims, 3.0e7, seed=101)
    on = (nH, E, e, n)
    for k in range(2):
        on = OA.split_step(op, t0 + k * dt, dt, v, on[0], src, *on[1:], cfl=0.9, tol=1e-12)
    s = P.Solver(P.params_from_workload(w, newton_tol=1e-12, precision=0), device=hip_device)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    g = [d(nH), d(E), d(e), d(n)]
    gv = [d(c) for c in v]
    gs = d(src)
    for k in range(2):
        st = s.split_step(t0 + k * dt, dt, gv, g[0], gs, g[1], g[2], g[3], cfl=0.9)
        print("split step", k, st["advect"], st["newton_its"])
        assert st["advect"]["substeps"] >= 1
    s.close()
    gn = [x.cpu().numpy() for x in g]
    assert np.max(np.abs(gn[0] - on[0]) / on[0]) <= 1e-13
    err = errors((gn[1], gn[2], gn[3]), (on[1], on[2], on[3]), on[0], False, phi_E_rel=1e-12)
    print("errors", err)
    assert err["E"] < 1e-10 and err["x"] < 1e-10 and err["e"] < 1e-10


def test_advect_error_paths(hip_device):
    """A non-finite velocity is reported (fields untouched); cfl outside
    (0, 1] and dt <= 0 are invalid arguments."""
    import torch
    import paper_0908_2654_amd as P
    w = W.scaled(2, (8, 8, 8))
    s = P.Solver(P.params_from_workload(w), device=hip_device)
    f = [torch.rand(w.dims, dtype=torch.float64, device=hip_device) + 0.5 for _ in range(4)]
    v = [torch.zeros(w.dims, dtype=torch.float64, device=hip_device) for _ in range(3)]
    keep = [x.clone() for x in f]
    v[1][3, 4, 5] = float("nan")
    with pytest.raises(P.RhError) as ei:
        s.advect(0.0, 1.0, v, *f)
    assert "RH_ENONFINITE" in str(ei.value)
    for a, b in zip(f, keep):
        assert torch.equal(a, b)
    v[1][3, 4, 5] = 0.0
    for vv, ff in (([v[0], f[1], v[2]], f), (v, [f[0], f[0], f[2], f[3]])):
        with pytest.raises(P.RhError) as ei:              # aliasing arrays
            s.advect(0.0, 1.0, vv, *ff)
        assert "RH_EINVAL" in str(ei.value)
    for cfl, dt in ((0.0, 1.0), (1.5, 1.0), (0.5, 0.0), (0.5, -1.0)):
        with pytest.raises(P.RhError) as ei:
            s.advect(0.0, dt, v, *f, cfl=cfl)
        assert "RH_EINVAL" in str(ei.value)
    st = s.advect(0.0, 1.0, v, *f)           # zero velocity: one substep, nothing moves
    assert st["substeps"] == 1 and st["courant"] == 0.0
    for k in (0, 1, 3):
        assert torch.equal(f[k], keep[k])
    # e passes through (n_H e) / n_H: equal to a rounding
    assert ((f[2] - keep[2]).abs() / keep[2]).max().item() <= 2.3e-16
    s.close()
