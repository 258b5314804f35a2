"""Pins of the hydrogen + helium multigroup oracle (oracle/multigroup.py)
against what the mathematics fixes: closed forms of the group integrals,
the single-group hydrogen-only limit (the grey step), linear superposition
of groups with a flat cross-section, exact energy conservation, per-group
photon budgets, convergence of the time discretisation to the local ODE
system, and quadratic Newton convergence."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import workloads as W
from oracle import grey, model as M, multigroup as MG, newton as N
from oracle.constants import C_LIGHT, EV_ERG, K_BOLTZ, M_H

EDGES = (13.6, 24.587, 54.4)


def _bose_series_x3(x, kmax=400):
    """int_x^inf t^3 / (e^t - 1) dt by the Bose series."""
    k = np.arange(1, kmax + 1, dtype=np.float64)
    return float(np.sum(np.exp(-k * x) * (x ** 3 / k + 3 * x ** 2 / k ** 2 + 6 * x / k ** 3
                                          + 6 / k ** 4)))


def test_group_integrals_against_closed_forms():
    """Group energy integrals (Bose series), the sigma ~ nu^-3 species
    integrals x_s^3 int b dx = x_s^3 [ln(1 - e^-x)] and
    x_s^3 int b / x dx = x_s^3 sum_k [E1(k a) - E1(k b)]."""
    T = 1e5
    kT = K_BOLTZ * T
    g = MG.group_constants(EDGES, T, 6.3e-18, 13.6)
    xe = [e * EV_ERG / kT for e in EDGES] + [np.inf]
    I = [_bose_series_x3(xe[i]) - (_bose_series_x3(xe[i + 1]) if np.isfinite(xe[i + 1]) else 0.0)
         for i in range(3)]
    np.testing.assert_allclose(g["I"], I, rtol=1e-12)
    np.testing.assert_allclose(g["frac"].sum(), 1.0, rtol=1e-14)
    thr = [13.6, 24.587, 54.4]
    s0 = [6.3e-18, 7.42e-18, 6.3e-18 / 4]
    k = np.arange(1, 400, dtype=np.float64)
    for s in range(3):
        xs = thr[s] * EV_ERG / kT
        for i in range(3):
            a, b = max(xe[i], xs), xe[i + 1]
            if a >= b:
                assert g["sigE"][s, i] == 0.0 and g["KGam"][s, i] == 0.0
                continue
            lnb = 0.0 if not np.isfinite(b) else math.log(-math.expm1(-b))
            intb = lnb - math.log(-math.expm1(-a))
            E1b = 0.0 if not np.isfinite(b) else np.sum(special.exp1(k * b))
            intbx = float(np.sum(special.exp1(k * a)) - E1b)
            sigE = s0[s] * xs ** 3 * intb / I[i]
            KGam = s0[s] * xs ** 3 * intbx / (kT * I[i])
            assert g["sigE"][s, i] == pytest.approx(sigE, rel=1e-11)
            assert g["KGam"][s, i] == pytest.approx(KGam, rel=1e-11)
            assert g["KG"][s, i] == pytest.approx(sigE - thr[s] * EV_ERG * KGam, rel=1e-9, abs=1e-30)


def _grey_inputs(cfg, dims, **over):
    w = W.scaled(cfg, dims)
    p = M.params_from_workload(w, newton_tol=1e-12, **over)
    nH = W.density_field(w)
    src = M.source_field(p, W.photon_rate_field(w))
    t0, dt, _ = M.schedule(p, w)
    return w, p, nH, src, t0, dt


@pytest.mark.parametrize("cfg,dims", [(1, (6, 6, 6)), (2, (8, 6, 6))])
def test_one_group_without_helium_is_the_grey_step(cfg, dims):
    w, p, nH, src, t0, dt = _grey_inputs(cfg, dims)
    mp = MG.params_from_workload(w, newton_tol=1e-12)
    E, e, n = M.initial_state(p, nH, w.x0, w.T0, w.E0)
    Eg, eg, yg = MG.initial_state(mp, nH, w.x0, w.T0, w.E0)
    np.testing.assert_allclose(eg, e, rtol=1e-15)
    for k in range(2):
        E, e, n = N.step(p, t0 + k * dt, dt, nH, src, E, e, n, tol=1e-12)
        Eg, eg, yg = MG.step(mp, t0 + k * dt, dt, nH, src, Eg, eg, yg, tol=1e-12)
        assert np.max(np.abs(Eg[0] - E)) / np.max(np.abs(E)) < 1e-12
        assert np.max(np.abs(yg[0] - n) / nH) < 1e-12
        assert np.max(np.abs(eg - e) / e) < 1e-12
        assert np.all(yg[1] == 0.0) and np.all(yg[2] == 0.0)


def test_flat_cross_section_groups_sum_to_the_grey_step():
    """sigma(nu) = sigma_0 in every group: each group sees the same opacity
    and (the limiter depends on E only through |grad E| / E) the same
    diffusion, so the groups are the grey solution split by the source's
    energy fractions; the grey constants of a flat cross-section follow from
    the whole-spectrum integrals (sigma_E = sigma_0, K_Gamma =
    sigma_0 I_N / (k T I_E))."""
    w, p, nH, src, t0, dt = _grey_inputs(2, (8, 6, 6))
    x0 = p.grey["hnu0"] / (K_BOLTZ * w.T_bb)
    I_E, I_N, _, _ = grey.blackbody_integrals(x0)
    s0 = w.sigma0
    KGam = s0 * I_N / (K_BOLTZ * w.T_bb * I_E)
    flat = dict(p.grey, sigma_E=s0, K_Gamma=KGam, K_G=s0 - p.grey["hnu0"] * KGam)
    pf = p.with_(grey=flat)
    base = M.params_from_workload(w, newton_tol=1e-12)
    base.grey["sigma0"] = s0
    mp = MG.make_params(base, EDGES, 0.0, w.T_bb, sigma_power=0.0)
    f = mp.groups["frac"]
    E, e, n = M.initial_state(pf, nH, w.x0, w.T0, w.E0)
    Eg, eg, yg = MG.initial_state(mp, nH, w.x0, w.T0, w.E0)
    # both solvers to 1e-13: what is left is their Newton truncation (a wrong
    # split of the groups would differ at the percent level)
    for k in range(2):
        E, e, n = N.step(pf, t0 + k * dt, dt, nH, src, E, e, n, tol=1e-13)
        Eg, eg, yg = MG.step(mp, t0 + k * dt, dt, nH, src, Eg, eg, yg, tol=1e-13)
        for g in range(3):
            assert np.max(np.abs(Eg[g] - f[g] * E)) / np.max(np.abs(f[g] * E)) < 1e-8
        assert np.max(np.abs(yg[0] - n) / nH) < 1e-10
        assert np.max(np.abs(eg - e) / e) < 1e-8


def _he_run(cfg, dims, theta=1.0, y_he=0.08, recombination=True, dt_scale=1.0, **over):
    w = W.scaled(cfg, dims)
    w.theta = theta
    base = M.params_from_workload(w, newton_tol=1e-13, **over)
    base.grey["sigma0"] = w.sigma0
    mp = MG.make_params(base, EDGES, y_he, w.T_bb, recombination=recombination)
    nH = W.density_field(w)
    src = M.source_field(base, W.photon_rate_field(w))
    t0, dt, _ = M.schedule(base, w)
    return w, mp, nH, src, t0, dt * dt_scale


def test_energy_is_conserved_exactly_with_helium():
    """Static box with zero-flux walls, theta = 1, no recombination and no
    cooling: the radiation energy gained, the gas energy gained and the
    ionisation energy stored (13.6 eV per H ionisation, 24.6 eV per HeI ->
    HeII, 54.4 eV per HeII -> HeIII) add up to the emitted energy: every
    absorbed photon's energy is split between ionisation and heating."""
    w, mp, nH, src, t0, dt = _he_run(2, (8, 6, 6), recombination=False, cooling=0,
                                     bc=(W.BC_ZEROFLUX,) * 6)
    assert mp.base.cosmo.kind == 0
    E, e, y = MG.initial_state(mp, nH, w.x0, w.T0, w.E0)
    nHe = mp.y_he * nH
    # helium singly ionised to begin with, so that HeII -> HeIII takes place
    y[1], y[2] = 0.0 * nHe, nHe.copy()
    hnu = np.array([13.6, 24.587, 54.4]) * EV_ERG     # ionisation thresholds of HI, HeI, HeII
    rho = M_H * (nH + 4.0 * nHe)
    for k in range(2):
        E1, e1, y1 = MG.step(mp, k * dt, dt, nH, src, E, e, y, tol=1e-13)
        gained = np.sum(E1 - E) + np.sum(rho * (e1 - e))
        ion = np.sum(hnu[0] * (y[0] - y1[0]) + hnu[1] * (y[1] - y1[1])
                     + hnu[2] * ((nHe - y1[1] - y1[2]) - (nHe - y[1] - y[2])))
        emitted = dt * np.sum(src)
        assert gained + ion == pytest.approx(emitted, rel=1e-10)
        assert np.max((y[2] - y1[2]) / nHe) > 1e-3                         # HeII was ionised
        E, e, y = E1, e1, y1


@pytest.mark.parametrize("theta,cfg,dims", [(1.0, 2, (8, 6, 6)), (0.6, 2, (8, 6, 6)),
                                            (1.0, 1, (6, 6, 6))])
def test_photon_budget_per_group(theta, cfg, dims):
    w, mp, nH, src, t0, dt = _he_run(cfg, dims, theta=theta, dt_scale=0.05 if theta < 1 else 1.0)
    E, e, y = MG.initial_state(mp, nH, w.x0, w.T0, w.E0)
    for k in range(2):
        ctx = MG.make_context(mp, t0 + k * dt, dt, nH, src, E, e, y)
        E, e, y = MG.step(mp, t0 + k * dt, dt, nH, src, E, e, y, tol=1e-13)
        assert max(MG.photon_budget_defects(mp, ctx, E, y)) < 1e-10
        nHe = mp.y_he * nH
        assert np.all(y[0] >= 0) and np.all(y[0] <= nH)
        assert np.all(y[1] >= 0) and np.all(y[2] >= 0) and np.all(y[1] + y[2] <= nHe * (1 + 1e-14))


def _uniform_he(theta):
    w = W.get(1)
    w.dims = (2, 2, 2)
    w.bc = (W.BC_ZEROFLUX,) * 6
    w.theta = theta
    base = M.params_from_workload(w)
    base.grey["sigma0"] = w.sigma0
    return w, MG.make_params(base, EDGES, 0.08, w.T_bb)


def _ode_rhs(mp, nHv, srcv):
    """The local ODE system of a uniform cell (no gradients), written out
    from the model equations: group energies, species, gas energy."""
    p = mp.base
    gc = mp.groups
    nHe = mp.y_he * nHv

    def f(t, u):
        G = mp.G
        E = u[:G]
        nHI, nHeI, nHeII, e = u[G:]
        a = p.cosmo.a(t)
        H = p.cosmo.hubble(t)
        a3 = a ** 3
        nHII, nHeIII = nHv - nHI, nHe - nHeI - nHeII
        ne_c = nHII + nHeII + 2 * nHeIII
        ne = ne_c / a3
        mu = (nHv + 4 * nHe) / (nHv + nHe + ne_c)
        T = (p.gamma - 1) * mu * M_H * e / K_BOLTZ
        lam = 2 * 157807.0 / T
        aH = 2.753e-14 * lam ** 1.5 / (1 + (lam / 2.740) ** 0.407) ** 2.242
        aHeII = 1.26e-14 * (2 * 285335.0 / T) ** 0.75
        lam4 = 2 * 157807.0 / (T / 4)
        aHeIII = 2 * 2.753e-14 * lam4 ** 1.5 / (1 + (lam4 / 2.740) ** 0.407) ** 2.242
        y = [nHI, nHeI, nHeII]
        Ep = [max(x, 0.0) / a3 for x in E]
        Gam = [C_LIGHT * sum(gc["KGam"][s, g] * Ep[g] for g in range(G)) for s in range(3)]
        dE = [-H * E[g] + gc["frac"][g] * srcv
              - C_LIGHT * sum(gc["sigE"][s, g] * y[s] for s in range(3)) / a3 * E[g]
              for g in range(G)]
        dHI = aH * ne * nHII - Gam[0] * nHI
        dHeI = aHeII * ne * nHeII - Gam[1] * nHeI
        dHeII = Gam[1] * nHeI - (Gam[2] + aHeII * ne) * nHeII + aHeIII * ne * nHeIII
        heat = C_LIGHT * sum(gc["KG"][s, g] * y[s] / a3 * Ep[g] for s in range(3) for g in range(G))
        Lrec = 3.435e-30 * T * lam ** 1.970 / (1 + (lam / 2.250) ** 0.376) ** 3.720 * ne * nHII / a3
        Lce = 7.5e-19 * math.exp(-118348.0 / T) / (1 + math.sqrt(T / 1e5)) * ne * nHI / a3
        Lc = 5.61e-36 / a ** 4 * (T - 2.725 / a) * ne
        LHe = K_BOLTZ * T * aHeII * ne * nHeII / a3 + 8 * (
            3.435e-30 * (T / 4) * lam4 ** 1.970 / (1 + (lam4 / 2.250) ** 0.376) ** 3.720) * ne * nHeIII / a3
        de = -2 * H * e + (heat - Lrec - Lce - Lc - LHe) / (M_H * (nHv + 4 * nHe) / a3)
        return dE + [dHI, dHeI, dHeII, de]
    return f


@pytest.mark.parametrize("theta,order,counts,rtol", [(1.0, 1, (32, 64, 128), 0.08),
                                                     (0.5, 2, (8, 16, 32), 0.02)])
def test_helium_chemistry_converges_to_the_ode_system(theta, order, counts, rtol):
    """A uniform expanding, cooling cell with helium and three groups,
    non-stiff (every rate times the span below a few): the step converges to
    the ODE system at first order for theta = 1 and second order for
    theta = 1/2 in every component."""
    w, mp = _uniform_he(theta)
    nHv, srcv, T_span = 1.7e-13, 1e-39, 1e16
    dims = w.dims
    nH = np.full(dims, nHv)
    src = np.full(dims, srcv)
    t0 = mp.base.cosmo.time_of_z(10.0)
    E0, e0, y0 = MG.initial_state(mp, nH, 1.2e-3, 100.0, 1e-35)
    f = _ode_rhs(mp, nHv, srcv)
    u0 = np.concatenate([E0[:, 0, 0, 0], y0[:, 0, 0, 0], [e0.flat[0]]])
    scale = np.concatenate([np.full(mp.G, srcv * T_span), [nHv, mp.y_he * nHv, mp.y_he * nHv],
                            [e0.flat[0]]])

    def g(tau, v):
        return np.array(f(t0 + tau * T_span, v * scale)) * T_span / scale
    sol = integrate.solve_ivp(g, (0.0, 1.0), u0 / scale, method="Radau", rtol=1e-13, atol=1e-15)
    assert sol.status == 0
    ref = sol.y[:, -1] * scale
    errs = []
    for nsteps in counts:
        dt = T_span / nsteps
        E, e, y = E0, e0, y0
        t = t0
        for _ in range(nsteps):
            E, e, y = MG.step(mp, t, dt, nH, src, E, e, y, tol=1e-14)
            t += dt
        got = np.concatenate([E[:, 0, 0, 0], y[:, 0, 0, 0], [e.flat[0]]])
        errs.append(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3 * scale))
    errs = np.array(errs)
    ratio = errs[0] / errs[1], errs[1] / errs[2]
    np.testing.assert_allclose(ratio, 2.0 ** order, rtol=rtol)


@pytest.mark.parametrize("y_he", [0.08, 1.0])
def test_helium_recombination_regime_converges_first_order(y_he):
    """A dense static cell (n_H = 1e-3, strong hard source) where hydrogen and
    helium sit near photoionisation-recombination balance with helium mostly
    HeIII: recombination of every ion, the electrons of HeII and HeIII, the
    helium cooling and the temperature dependence all set the state.  Backward
    Euler steps from the smooth solution (after the ionisation transient,
    which is shorter than any step) converge at first order to the ODE
    system in every component.  y_He = 1 (as much helium as hydrogen, by
    number) makes the helium terms, its recombination cooling included,
    carry the energy balance."""
    w = W.get(2)
    w.dims = (2, 2, 2)
    w.bc = (W.BC_ZEROFLUX,) * 6
    w.theta = 1.0
    base = M.params_from_workload(w)
    base.grey["sigma0"] = w.sigma0
    mp = MG.make_params(base, EDGES, y_he, w.T_bb)
    nHv, srcv, T_pre, T_span = 1e-3, 1e-24, 2.5e14, 7.5e14
    nHe = mp.y_he * nHv
    f = _ode_rhs(mp, nHv, srcv)
    nH = np.full(w.dims, nHv)
    src = np.full(w.dims, srcv)
    E0, e0, y0 = MG.initial_state(mp, nH, 1.2e-3, 100.0, 1e-35)
    u0 = np.concatenate([E0[:, 0, 0, 0], y0[:, 0, 0, 0], [e0.flat[0]]])
    T_tot = T_pre + T_span
    scale = np.concatenate([np.full(mp.G, srcv * T_tot), [nHv, nHe, nHe], [e0.flat[0]]])

    def g(tau, v):
        return np.array(f(tau * T_tot, v * scale)) * T_tot / scale
    sol = integrate.solve_ivp(g, (0.0, 1.0), u0 / scale, method="Radau", rtol=1e-13, atol=1e-16,
                              dense_output=True)
    assert sol.status == 0
    ua = sol.sol(T_pre / T_tot) * scale
    ref = sol.y[:, -1] * scale
    assert ua[5] / nHe < 1e-6 and ua[4] / nHe < 1e-12 and ua[3] / nHv < 1e-8   # HeIII, H II
    full = lambda v: np.full(w.dims, v)  # noqa: E731
    Ea, ya, ea = np.stack([full(v) for v in ua[:3]]), np.stack([full(v) for v in ua[3:6]]), full(ua[6])
    errs = []
    for nsteps in (16, 32, 64):
        dt = T_span / nsteps
        E, e, y = Ea, ea, ya
        t = T_pre
        for _ in range(nsteps):
            E, e, y = MG.step(mp, t, dt, nH, src, E, e, y, tol=1e-14)
            t += dt
        got = np.concatenate([E[:, 0, 0, 0], y[:, 0, 0, 0], [e.flat[0]]])
        errs.append(np.abs(got - ref) / np.abs(ref))
    errs = np.array(errs)
    np.testing.assert_allclose((errs[0] / errs[1], errs[1] / errs[2]), 2.0, rtol=0.03)


def test_newton_converges_quadratically_with_helium():
    w, mp, nH, src, t0, dt = _he_run(2, (8, 6, 6))
    E, e, y = MG.initial_state(mp, nH, w.x0, w.T0, w.E0)
    st = {}
    MG.step(mp, t0, dt, nH, src, E, e, y, tol=1e-13, stats=st)
    h = st["history"]
    assert h[-1] <= 1e-13 and len(h) >= 4
    # quadratic: once ||f|| < 1e-2, each norm above the rounding floor (1e-12)
    # is bounded by a constant times the square of the previous one
    ratios = [h[i + 1] / h[i] ** 2 for i in range(len(h) - 1) if h[i] < 1e-2 and h[i + 1] > 1e-12]
    assert len(ratios) >= 2 and max(ratios) < 1e3
