"""Pins of the FP64 oracle against values the paper and the mathematics fix.

Each test names what it pins.  None of them re-types an oracle formula:
they use closed forms, series, textbook special cases, numerical ODE
integration, symmetry and conservation identities.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import workloads as W
from oracle import analytic, cosmology, diagnostics, grey, model as M, newton as N, rates
from oracle.constants import C_LIGHT, EV_ERG, K_BOLTZ, KPC_CM, M_H, MYR_S


# ---------------------------------------------------------------------------
# grey constants: quadrature against series / closed forms
# ---------------------------------------------------------------------------
def test_grey_integrals_closed_forms():
    x0 = 13.6 * EV_ERG / (K_BOLTZ * 1.0e5)
    I_E, I_N, I_sE, I_sN = grey.blackbody_integrals(x0)
    k = np.arange(1, 200)
    ek = np.exp(-k * x0)
    bose3 = np.sum(ek * (x0 ** 3 / k + 3 * x0 ** 2 / k ** 2 + 6 * x0 / k ** 3 + 6 / k ** 4))
    bose2 = np.sum(ek * (x0 ** 2 / k + 2 * x0 / k ** 2 + 2 / k ** 3))
    assert I_E == pytest.approx(bose3, rel=1e-13)
    assert I_N == pytest.approx(bose2, rel=1e-13)
    assert I_sE == pytest.approx(-x0 ** 3 * math.log(1.0 - math.exp(-x0)), rel=1e-13)
    assert I_sN == pytest.approx(x0 ** 3 * np.sum(special.exp1(k * x0)), rel=1e-13)


def test_grey_constants_monochromatic_and_bookkeeping():
    g = grey.grey_constants(0, 1e5, 13.6, 6.3e-18)
    assert g["sigma_E"] == 6.3e-18 and g["K_G"] == 0.0
    assert g["K_Gamma"] * g["hnu0"] == pytest.approx(6.3e-18, rel=1e-15)
    b = grey.grey_constants(1, 1e5, 13.6, 6.3e-18)
    # mean photon energy of the spectrum above 13.6 eV: within 3% of the
    # Wien-tail value k T_B (x0^3 + 3x0^2 + 6x0 + 6) / (x0^2 + 2x0 + 2)
    x0 = 13.6 * EV_ERG / (K_BOLTZ * 1e5)
    wien = K_BOLTZ * 1e5 * (x0 ** 3 + 3 * x0 ** 2 + 6 * x0 + 6) / (x0 ** 2 + 2 * x0 + 2)
    assert b["eps_bar"] == pytest.approx(wien, rel=0.03)
    assert b["sigma_E"] < 6.3e-18 and b["K_G"] > 0


# ---------------------------------------------------------------------------
# rates
# ---------------------------------------------------------------------------
def test_alphaB_matches_paper_value():
    # verification section: alpha_B ~ 2.59e-13 cm^3/s (at 1e4 K)
    assert rates.alpha_B_fit(1.0e4) == pytest.approx(2.59e-13, rel=2e-3)
    # monotone decreasing in T
    T = np.logspace(2, 6, 50)
    assert np.all(np.diff(rates.alpha_B_fit(T)) < 0)


def test_compton_coefficient():
    # textbook value of the Compton cooling coefficient: 5.65e-36 erg cm^-3 s^-1 K^-5 scale
    assert rates.COMPTON_COEFF == pytest.approx(5.6e-36, rel=1e-2)


# ---------------------------------------------------------------------------
# cosmology: closed forms against the Friedmann equation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,h,Om,OL", [(1, 0.5, 1.0, 0.0), (2, 0.7, 0.3, 0.7),
                                         (3, 1.0, 0.1, 0.0)])
def test_cosmology_against_friedmann(kind, h, Om, OL):
    c = cosmology.Cosmology(kind, h, Om, OL)
    H0 = c.H0
    a_start = 1e-3
    t_start = c.time_of_a(a_start)

    Ok = 1.0 - Om - OL  # curvature (open universe)

    def rhs(t, y):
        a = y[0]
        return [a * H0 * math.sqrt(Om / a ** 3 + Ok / a ** 2 + OL)]
    t_end = c.time_of_z(0.0)
    ts = np.linspace(t_start, t_end, 7)
    sol = integrate.solve_ivp(rhs, (t_start, t_end), [a_start], t_eval=ts,
                              rtol=1e-12, atol=1e-15, method="DOP853")
    for t, a_num in zip(sol.t, sol.y[0]):
        assert c.a(t) == pytest.approx(a_num, rel=1e-9)
        dt = 1e-6 * t
        dadt = (c.a(t + dt) - c.a(t - dt)) / (2 * dt)
        assert c.hubble(t) == pytest.approx(dadt / c.a(t), rel=1e-8)
    assert c.a(c.time_of_z(4.0)) == pytest.approx(0.2, rel=1e-13)


# ---------------------------------------------------------------------------
# limiter and diffusion operator
# ---------------------------------------------------------------------------
def test_limiter_limits():
    kap = 3.7e-21
    assert M.limiter_D(C_LIGHT, kap, 1e-40) == pytest.approx(C_LIGHT / (3 * kap), rel=1e-15)
    R = 2.1e-22
    assert M.limiter_D(C_LIGHT, 1e-60, R) == pytest.approx(C_LIGHT / R, rel=1e-15)
    assert M.limiter_D(C_LIGHT, kap, kap) == pytest.approx(0.3 * C_LIGHT / kap, rel=1e-15)


def _params(dims, bc, **kw):
    w = W.get(0)
    w.dims = dims
    w.bc = bc
    return M.params_from_workload(w, **kw)


@pytest.mark.parametrize("k", [(1, 0, 0), (2, 3, 1), (0, 4, 5)])
def test_operator_fourier_eigenvalue_periodic(k):
    dims = (12, 10, 14)
    p = _params(dims, (W.BC_PERIODIC,) * 6)
    c = 0.37
    cf = [np.full(tuple(n + (1 if d == dd else 0) for dd, n in enumerate(dims)), c)
          for d in range(3)]
    I, J, K = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    ph = 2 * np.pi * (k[0] * I / dims[0] + k[1] * J / dims[1] + k[2] * K / dims[2])
    E = np.cos(ph) + 0.3 * np.sin(ph)
    lam = -4 * c * sum(math.sin(math.pi * k[d] / dims[d]) ** 2 for d in range(3))
    np.testing.assert_allclose(M.apply_L(p, cf, E), lam * E, atol=1e-13)


def test_operator_neumann_eigenvalue_zeroflux():
    dims = (9, 7, 8)
    p = _params(dims, (W.BC_ZEROFLUX,) * 6)
    c = 1.3
    cf = []
    for d in range(3):
        shp = tuple(n + (1 if d == dd else 0) for dd, n in enumerate(dims))
        f = np.full(shp, c)
        sl = [slice(None)] * 3
        sl[d] = 0
        f[tuple(sl)] = 0.0
        sl[d] = dims[d]
        f[tuple(sl)] = 0.0
        cf.append(f)
    k = (2, 3, 1)
    I, J, K = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    E = (np.cos(np.pi * k[0] * (I + 0.5) / dims[0]) * np.cos(np.pi * k[1] * (J + 0.5) / dims[1])
         * np.cos(np.pi * k[2] * (K + 0.5) / dims[2]))
    lam = -4 * c * sum(math.sin(math.pi * k[d] / (2 * dims[d])) ** 2 for d in range(3))
    np.testing.assert_allclose(M.apply_L(p, cf, E), lam * E, atol=1e-13)


def test_operator_manufactured_second_order():
    """(L E) approximates (1/a^2) div(D grad E) to second order in h."""
    errs = []
    a = 0.25
    for N_ in (16, 32, 64):
        dims = (N_, N_, N_)
        p = _params(dims, (W.BC_PERIODIC,) * 6)
        L = 2.0
        h = L / N_
        x = (np.arange(N_) + 0.5) * h
        xf = np.arange(N_ + 1) * h
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        D = lambda x, y, z: 1.0 + 0.5 * np.sin(np.pi * x) * np.cos(np.pi * y)  # noqa: E731
        Ef = lambda x, y, z: np.sin(np.pi * x) + np.cos(np.pi * y) * np.sin(np.pi * z)  # noqa: E731
        cf = []
        for d in range(3):
            coords = [x, x, x]
            coords[d] = xf
            G = np.meshgrid(*coords, indexing="ij")
            cf.append(D(*G) / (a * a * h * h))
        LE = M.apply_L(p, cf, Ef(X, Y, Z))
        # exact (1/a^2) div(D grad E)
        pi = np.pi
        Dv = D(X, Y, Z)
        Dx = 0.5 * pi * np.cos(pi * X) * np.cos(pi * Y)
        Dy = -0.5 * pi * np.sin(pi * X) * np.sin(pi * Y)
        Ex = pi * np.cos(pi * X)
        Ey = -pi * np.sin(pi * Y) * np.sin(pi * Z)
        Ez = pi * np.cos(pi * Y) * np.cos(pi * Z)
        lap = -pi * pi * np.sin(pi * X) - 2 * pi * pi * np.cos(pi * Y) * np.sin(pi * Z)
        exact = (Dv * lap + Dx * Ex + Dy * Ey) / (a * a)
        errs.append(np.max(np.abs(LE - exact)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.8


# ---------------------------------------------------------------------------
# whole steps: special cases with closed forms
# ---------------------------------------------------------------------------
def test_fourier_mode_decay_one_step():
    """Transparent medium (sigma = 0): D = c/R_min uniform, so one step is a
    backward-Euler step of a constant-coefficient heat equation."""
    dims = (12, 12, 12)
    w = W.get(0)
    w.dims = dims
    w.bc = (W.BC_PERIODIC,) * 6
    w.sigma0 = 0.0
    w.alphaB_const = 0.0
    p = M.params_from_workload(w)
    nH = np.full(dims, 1e-3)
    I = np.arange(dims[0])[:, None, None] * np.ones(dims)
    k = (1, 0, 0)
    E0 = 1e-20 * (1.0 + 0.01 * np.cos(2 * np.pi * k[0] * I / dims[0]))
    e0 = np.full(dims, 1e12)
    n0 = 0.5 * nH
    dt = 1e-3 * MYR_S
    E1, e1, n1 = N.step(p, 0.0, dt, nH, np.zeros(dims), E0, e0, n0, tol=1e-14)
    D = C_LIGHT * p.box  # c / R_min, a = 1
    amp = analytic.fourier_amplification(dt, D, p.h, k, dims)
    got = (E1 - E1.mean()) / (E0 - E0.mean())
    assert 0.05 < amp < 0.95
    np.testing.assert_allclose(got[:, 0, 0][[0, 2, 4, 6]], amp, rtol=1e-9)
    assert E1.mean() == pytest.approx(E0.mean(), rel=1e-12)
    np.testing.assert_allclose(n1, n0, rtol=1e-15)


def test_fourier_mode_decay_theta_half_expanding():
    """Transparent medium in an Einstein-de Sitter background, theta = 1/2:
    D = c/R_min is uniform, and the two time levels of the
    comoving diffusion and Hubble terms give a Fourier mode the closed-form
    amplification
      g_k = (1 - dt/2 (lam_n + H_n)) / (1 + dt/2 (lam_1 + H_1)),
      lam_m = D / (a_m^2 h^2) 4 sum_d sin^2(pi k_d / N_d),
    and the mean g_0 (lam = 0): each level takes its own a_m and H_m.  R_min
    is set large enough that D = c/R_min and lam dt ~ 1 over a step of 5% of
    the cosmic time (a_1/a_n - 1 = 3%)."""
    dims = (12, 12, 12)
    w = W.get(0)
    w.dims = dims
    w.bc = (W.BC_PERIODIC,) * 6
    w.sigma0 = 0.0
    w.alphaB_const = 0.0
    w.theta = 0.5
    w.cosmology = W.COSMO_EDS
    w.hubble_h, w.Omega_m, w.Omega_L = 0.5, 1.0, 0.0
    t0 = M.params_from_workload(w).cosmo.time_of_z(10.0)
    dt = 0.05 * t0
    a_n = M.params_from_workload(w).cosmo.a(t0)
    h = w.box_comoving_cm / dims[0]
    s = 4.0 * math.sin(math.pi / dims[0]) ** 2
    R_min = C_LIGHT * s * dt / (a_n * h) ** 2  # lam_n dt = 1
    p = M.params_from_workload(w, R_min=R_min)
    nH = np.full(dims, 1e-3)
    I = np.arange(dims[0])[:, None, None] * np.ones(dims)
    k = (1, 0, 0)
    E0 = 1e-20 * (1.0 + 0.01 * np.cos(2 * np.pi * k[0] * I / dims[0]))
    e0 = np.full(dims, 1e12)
    n0 = 0.5 * nH
    E1, e1, n1 = N.step(p, t0, dt, nH, np.zeros(dims), E0, e0, n0, tol=1e-14)
    a_n, a_1 = p.cosmo.a(t0), p.cosmo.a(t0 + dt)
    H_n, H_1 = p.cosmo.hubble(t0), p.cosmo.hubble(t0 + dt)
    D = C_LIGHT / R_min
    lam_n, lam_1 = D * s / (a_n * p.h) ** 2, D * s / (a_1 * p.h) ** 2
    g0 = (1.0 - 0.5 * dt * H_n) / (1.0 + 0.5 * dt * H_1)
    gk = (1.0 - 0.5 * dt * (lam_n + H_n)) / (1.0 + 0.5 * dt * (lam_1 + H_1))
    assert abs(gk) < 0.95 and abs(lam_1 / lam_n - 1.0) > 0.05
    got = (E1 - E1.mean()) / (E0 - E0.mean())
    np.testing.assert_allclose(got[:, 0, 0][[0, 2, 4, 6]], gk, rtol=1e-9)
    assert E1.mean() == pytest.approx(g0 * E0.mean(), rel=1e-12)


def _uniform_cell_workload(spectrum, isothermal, cosmo):
    w = W.get(1)
    w.dims = (2, 2, 2)
    w.bc = (W.BC_ZEROFLUX,) * 6
    w.spectrum = spectrum
    w.isothermal = isothermal
    if isothermal:
        w.rates = W.RATES_CONST
    w.cosmology = cosmo
    if cosmo == W.COSMO_STATIC:
        w.dt_Myr, w.z_start, w.z_end = 1.0, None, None
    return w


def _ode_rhs(p, nH, src, tt):
    """Right-hand side of the local ODE system of the implicit subsystem
    (uniform medium, no gradients), written from the model equations."""
    sE, KG, KGam = p.grey["sigma_E"], p.grey["K_G"], p.grey["K_Gamma"]
    c = C_LIGHT

    def f(t, y):
        E, n, e = y
        a = p.cosmo.a(t)
        H = p.cosmo.hubble(t)
        a3 = a ** 3
        if p.isothermal:
            T = p.T_iso
            alpha = p.alphaB_const
        else:
            x = 1 - n / nH
            T = (p.gamma - 1) * M_H * e / ((1 + x) * K_BOLTZ)
            lam = 315614.0 / T
            alpha = 2.753e-14 * lam ** 1.5 / (1 + (lam / 2.740) ** 0.407) ** 2.242
        ne = (nH - n) / a3
        Gam = c * KGam * max(E, 0.0) / a3
        dE = -H * E + src - c * sE * n / a3 * E
        dn = alpha * ne * (nH - n) - Gam * n
        if p.isothermal:
            return [dE, dn, 0.0]
        nHI, nHII = n / a3, (nH - n) / a3
        G = c * KG * nHI * max(E, 0.0) / a3
        lam = 315614.0 / T
        Lrec = 3.435e-30 * T * lam ** 1.970 / (1 + (lam / 2.250) ** 0.376) ** 3.720 * ne * nHII
        Lce = 7.5e-19 * math.exp(-118348.0 / T) / (1 + math.sqrt(T / 1e5)) * ne * nHI
        Lc = 5.61e-36 / a ** 4 * (T - 2.725 / a) * ne
        de = -2 * H * e + (G - Lrec - Lce - Lc) / (M_H * nH / a3)
        return [dE, dn, de]
    return f


@pytest.mark.parametrize("case", ["iso_static_mono", "bb_eds_cooling"])
def test_local_terms_converge_to_ode_system(case):
    """Many small implicit steps of a uniform medium converge (first order)
    to the ODE system the implicit subsystem reduces to without gradients."""
    if case == "iso_static_mono":
        w = _uniform_cell_workload(W.SPEC_MONO, True, W.COSMO_STATIC)
        nHv, srcv, T_span = 1e-3, 2e-27, 2.0 * MYR_S
    else:
        w = _uniform_cell_workload(W.SPEC_BLACKBODY, False, W.COSMO_EDS)
        nHv, srcv, T_span = 1.7e-7, 1e-33, 40.0 * MYR_S
    p = M.params_from_workload(w)
    dims = w.dims
    nH = np.full(dims, nHv)
    src = np.full(dims, srcv)
    t0 = 0.0 if p.cosmo.kind == 0 else p.cosmo.time_of_z(10.0)
    E0, e0, n0 = M.initial_state(p, nH, 1.2e-3, 100.0, 1e-35)
    f = _ode_rhs(p, nHv, srcv, None)
    # integrate in scaled variables (E / E_ref, n / n_H, e / e_0, t / T_span)
    scale = np.array([srcv * T_span, nHv, e0.flat[0]])

    def g(tau, y):
        return np.array(f(t0 + tau * T_span, y * scale)) * T_span / scale
    y0 = np.array([E0.flat[0], n0.flat[0], e0.flat[0]]) / scale
    sol = integrate.solve_ivp(g, (0.0, 1.0), y0, method="Radau", rtol=1e-12, atol=1e-14)
    assert sol.status == 0, sol.message
    ref = sol.y[:, -1] * scale
    errs = []
    for nsteps in (16, 32, 64):
        dt = T_span / nsteps
        E, e, n = E0, e0, n0
        t = t0
        for _ in range(nsteps):
            E, e, n = N.step(p, t, dt, nH, src, E, e, n, tol=1e-13)
            t += dt
        err = [abs(E.flat[0] - ref[0]) / abs(ref[0]), abs(n.flat[0] - ref[1]) / nHv]
        if not p.isothermal:
            err.append(abs(e.flat[0] - ref[2]) / abs(ref[2]))
        errs.append(max(err))
    # first-order convergence of the backward-Euler discretisation
    assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.25)
    assert errs[1] / errs[2] == pytest.approx(2.0, rel=0.2)
    assert errs[2] < 0.05


@pytest.mark.parametrize("case", ["iso_static_mono", "bb_eds_cooling"])
def test_theta_half_is_second_order(case):
    """theta = 1/2 (trapezoidal in both the radiation residual and the local
    solutions): the explicit level enters with weight 1/2, and the step
    converges to the ODE system at second order (error ratio 4 per halving
    in every component).  A wrong time level in any explicit term (rates or
    opacity taken at U instead of U^n, a_{n+1} or H_{n+1} instead of a_n,
    H_n) drops some component to first order.  Regimes are chosen non-stiff
    (rate x step < 1) so the trapezoidal rule is in its asymptotic range;
    the expanding case spans a Hubble time of about 0.6."""
    if case == "iso_static_mono":
        w = _uniform_cell_workload(W.SPEC_MONO, True, W.COSMO_STATIC)
        nHv, srcv, T_span = 1e-6, 4e-30, 5e12
    else:
        w = _uniform_cell_workload(W.SPEC_BLACKBODY, False, W.COSMO_EDS)
        nHv, srcv, T_span = 1.7e-13, 1e-39, 1e16
    w.theta = 0.5
    p = M.params_from_workload(w)
    dims = w.dims
    nH = np.full(dims, nHv)
    src = np.full(dims, srcv)
    t0 = 0.0 if p.cosmo.kind == 0 else p.cosmo.time_of_z(10.0)
    E0, e0, n0 = M.initial_state(p, nH, 1.2e-3, 100.0, 1e-35)
    f = _ode_rhs(p, nHv, srcv, None)
    scale = np.array([srcv * T_span, nHv, e0.flat[0]])

    def g(tau, y):
        return np.array(f(t0 + tau * T_span, y * scale)) * T_span / scale
    y0 = np.array([E0.flat[0], n0.flat[0], e0.flat[0]]) / scale
    sol = integrate.solve_ivp(g, (0.0, 1.0), y0, method="Radau", rtol=1e-13, atol=1e-15)
    assert sol.status == 0, sol.message
    ref = sol.y[:, -1] * scale
    errs = []
    for nsteps in (8, 16, 32):
        dt = T_span / nsteps
        E, e, n = E0, e0, n0
        t = t0
        for _ in range(nsteps):
            E, e, n = N.step(p, t, dt, nH, src, E, e, n, tol=1e-14)
            t += dt
        err = [abs(E.flat[0] - ref[0]) / abs(ref[0]), abs(n.flat[0] - ref[1]) / nHv]
        if not p.isothermal:
            err.append(abs(e.flat[0] - ref[2]) / abs(ref[2]))
        errs.append(err)
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    np.testing.assert_allclose(ratios, 4.0, rtol=0.02)
    assert np.all(errs[-1] < 1e-3)


def test_photon_number_conservation_mono():
    """Monochromatic isothermal run without recombination or expansion:
    every absorbed photon ionises one atom, so the radiation energy gained
    equals the emitted energy minus h nu_0 per ionisation (exact)."""
    w = W.get(0)
    w.dims = (8, 8, 8)
    w.alphaB_const = 0.0
    p = M.params_from_workload(w)
    nH = W.density_field(w)
    src = M.source_field(p, W.photon_rate_field(w))
    E, e, n = M.initial_state(p, nH, w.x0, w.T0, w.E0)
    dt = 0.5 * MYR_S
    E1, e1, n1 = N.step(p, 0.0, dt, nH, src, E, e, n, tol=1e-13)
    gained = np.sum(E1 - E)
    emitted = dt * np.sum(src)
    ionisation = p.grey["hnu0"] * np.sum(n - n1)
    assert gained + ionisation == pytest.approx(emitted, rel=1e-10)


@pytest.mark.parametrize("cfg,dims", [(0, (8, 8, 8)), (2, (10, 12, 8)), (1, (8, 8, 8))])
def test_photon_energy_budget_telescopes(cfg, dims):
    w = W.scaled(cfg, dims)
    p = M.params_from_workload(w)
    nH = W.density_field(w)
    src = M.source_field(p, W.photon_rate_field(w))
    E, e, n = M.initial_state(p, nH, w.x0, w.T0, w.E0)
    t0, dt, _ = M.schedule(p, w)
    for s in range(2):
        ctx = M.make_context(p, t0 + s * dt, dt, nH, src, E, e, n)
        E, e, n = N.step(p, t0 + s * dt, dt, nH, src, E, e, n, tol=1e-13)
        assert diagnostics.photon_budget_defect(p, ctx, E, n) < 1e-10
        assert np.all(n >= 0) and np.all(n <= nH)


@pytest.mark.parametrize("cfg,dims,theta", [(0, (8, 8, 8), 0.51), (2, (10, 12, 8), 0.6),
                                            (1, (8, 8, 8), 0.51)])
def test_photon_energy_budget_theta_lt1(cfg, dims, theta):
    """The budget with both time levels (explicit weight 1 - theta): zero-flux
    walls (Stromgren, EdS sphere) and periodic walls (lognormal); short steps
    keep the explicit half admissible."""
    w = W.scaled(cfg, dims)
    w.theta = theta
    p = M.params_from_workload(w)
    nH = W.density_field(w)
    src = M.source_field(p, W.photon_rate_field(w))
    E, e, n = M.initial_state(p, nH, w.x0, w.T0, w.E0)
    t0, dt, _ = M.schedule(p, w)
    dt = dt * 0.02
    for s in range(3):
        ctx = M.make_context(p, t0 + s * dt, dt, nH, src, E, e, n)
        E, e, n = N.step(p, t0 + s * dt, dt, nH, src, E, e, n, tol=1e-13)
        assert diagnostics.photon_budget_defect(p, ctx, E, n) < 1e-10
        # the theta = 1 budget does not hold for this step (the explicit level matters)
        assert diagnostics.photon_budget_defect(p.with_(theta=1.0), ctx, E, n) > 1e-6
        assert np.all(n >= 0) and np.all(n <= nH)


def test_static_stromgren_growth_law():
    """Config-0 I-front against r_S (1 - exp(-t/t_rec))^(1/3) (verification
    section, Stromgren radius with alpha_B = 2.59e-13)."""
    w = W.get(0)
    p = M.params_from_workload(w)
    nH = W.density_field(w)
    src = M.source_field(p, W.photon_rate_field(w))
    E, e, n = M.initial_state(p, nH, w.x0, w.T0, w.E0)
    t0, dt, ns = M.schedule(p, w)
    r_num = {}
    t = t0
    for s in range(ns):
        E, e, n = N.step(p, t, dt, nH, src, E, e, n)
        t += dt
        if s + 1 in (2, 10, 20):
            r_num[s + 1] = diagnostics.front_radius(n, nH, w.x0, p.h)
    for s, r in r_num.items():
        r_an = analytic.static_front(s * dt, 5e48, 2.59e-13, 1e-3)
        assert r == pytest.approx(r_an, rel=0.03), s
    assert analytic.stromgren_radius(5e48, 2.59e-13, 1e-3) / KPC_CM == pytest.approx(5.393, rel=1e-3)


def test_octant_symmetry_centre_source():
    w = W.get(0)
    w.dims = (8, 8, 8)
    p = M.params_from_workload(w)
    nH = W.density_field(w)
    src = M.source_field(p, W.photon_rate_field(w))
    E, e, n = M.initial_state(p, nH, w.x0, w.T0, w.E0)
    E1, e1, n1 = N.step(p, 0.0, 0.5 * MYR_S, nH, src, E, e, n, tol=1e-13)
    for X in (E1, n1):
        for ax in range(3):
            np.testing.assert_allclose(X, np.flip(X, axis=ax), rtol=1e-9)
        np.testing.assert_allclose(X, np.transpose(X, (1, 0, 2)), rtol=1e-9)
        np.testing.assert_allclose(X, np.transpose(X, (2, 1, 0)), rtol=1e-9)


# ---------------------------------------------------------------------------
# Newton machinery
# ---------------------------------------------------------------------------
def _state_mid_run(cfg, dims, steps=1):
    w = W.scaled(cfg, dims)
    p = M.params_from_workload(w)
    nH = W.density_field(w)
    src = M.source_field(p, W.photon_rate_field(w))
    E, e, n = M.initial_state(p, nH, w.x0, w.T0, w.E0)
    t0, dt, _ = M.schedule(p, w)
    for s in range(steps):
        E, e, n = N.step(p, t0 + s * dt, dt, nH, src, E, e, n)
    return w, p, nH, src, E, e, n, t0 + steps * dt, dt


@pytest.mark.parametrize("cfg", [0, 2])
def test_schur_direction_equals_dense_full_system(cfg):
    w, p, nH, src, E, e, n, t, dt = _state_mid_run(cfg, (4, 4, 4))
    ctx = M.make_context(p, t, dt, nH, src, E, e, n)
    # a perturbed, locally inconsistent state exercises every block
    Ep = E * (1 + 0.3 * np.cos(np.arange(E.size)).reshape(E.shape))
    npert = n * (1 - 0.1 * np.sin(np.arange(E.size)).reshape(E.shape))
    ee = None if p.isothermal else e * 1.1
    f = M.residual(p, ctx, Ep, ee, npert)
    d_s = N.newton_direction(p, ctx, Ep, ee, npert, *f, solver="schur")
    d_d = N.newton_direction(p, ctx, Ep, ee, npert, *f, solver="dense")
    for a, b in zip(d_s, d_d):
        if a is not None:
            np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-13 * np.max(np.abs(b)))


def test_local_jacobian_complex_step_vs_central_differences():
    w, p, nH, src, E, e, n, t, dt = _state_mid_run(2, (4, 4, 4))
    ctx = M.make_context(p, t, dt, nH, src, E, e, n)
    loc = N.local_jacobian(p, ctx, E, e, n)
    for var, key_n, key_e, X in (("n", "fn_n", "fe_n", n), ("e", "fn_e", "fe_e", e),
                                 ("E", "fn_E", "fe_E", E)):
        h = 1e-6 * np.abs(X) + 1e-30

        def ev(Xp):
            args = {"E": E, "e": e, "n": n}
            args[var] = Xp
            Sn, Se = M.local_S(p, ctx, args["E"], args["e"], args["n"])
            return args["n"] - Sn, args["e"] - Se
        fp, fm = ev(X + h), ev(X - h)
        dn = ((fp[0] - fm[0]) / (2 * h)).ravel()
        de = ((fp[1] - fm[1]) / (2 * h)).ravel()
        np.testing.assert_allclose(loc[key_n], dn, rtol=1e-3, atol=1e-9 * np.max(np.abs(dn)))
        np.testing.assert_allclose(loc[key_e], de, rtol=1e-3, atol=1e-9 * np.max(np.abs(de)))


def test_newton_converges_quadratically():
    w = W.scaled(2, (8, 8, 8))
    p = M.params_from_workload(w)
    nH = W.density_field(w)
    src = M.source_field(p, W.photon_rate_field(w))
    E, e, n = M.initial_state(p, nH, w.x0, w.T0, w.E0)
    st = {}
    N.step(p, 0.0, 0.5 * MYR_S, nH, src, E, e, n, tol=1e-12, stats=st)
    h = st["history"]
    assert st["ls_cuts"] == 0
    # the last reductions are quadratic: r_{k+1} <= C r_k^2 with C of order 1/r_0
    # (pairs whose second member sits at the FP64 rounding floor, ~1e-14, say nothing)
    late = [(h[k], h[k + 1]) for k in range(len(h) - 1) if h[k] < 1e-3 and h[k + 1] > 1e-12]
    assert len(late) >= 2, h
    for r0, r1 in late:
        assert r1 <= 50.0 * r0 * r0 / h[0], h


def test_norm_unit_weights():
    """With unit weights the norm is ||w||_2 / sqrt(N (N_s + 2)) (rmsnorm)."""
    w = W.get(2)
    w.dims = (3, 4, 5)
    p = M.params_from_workload(w)
    ones = np.ones(w.dims)
    ctx = M.StepContext(t_n=0, dt=1.0, a_n=1, a_1=1, H_n=0, H_1=0, nH=ones, src=0 * ones,
                        En=ones, en=ones, nn=ones, R_min=1.0, E_s=1.0)
    rng = np.random.default_rng(0)
    a, b, c = (rng.standard_normal(w.dims) for _ in range(3))
    full = np.concatenate([a.ravel(), b.ravel(), c.ravel()])
    assert M.norm(p, ctx, a, b, c) == pytest.approx(
        np.linalg.norm(full) / math.sqrt(full.size), rel=1e-14)


def test_failures_are_reported():
    w = W.get(0)
    w.dims = (4, 4, 4)
    p = M.params_from_workload(w)
    nH = W.density_field(w)
    src = M.source_field(p, W.photon_rate_field(w))
    E, e, n = M.initial_state(p, nH, w.x0, w.T0, w.E0)
    bad = src.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(FloatingPointError):
        N.step(p, 0.0, 0.5 * MYR_S, nH, bad, E, e, n)
    with pytest.raises(N.NewtonFailure):
        N.step(p.with_(newton_max_it=1), 0.0, 0.5 * MYR_S, nH, src, E, e, n, tol=1e-15)
    with pytest.raises(ValueError):
        M.params_from_workload(w, theta=0.0)


# ---------------------------------------------------------------------------
# Shapiro-Giroux I-front law
# ---------------------------------------------------------------------------
def test_sg_front_photon_counting_limit():
    """lambda -> 0: no recombinations, r^3 = 3 Q (t - t0) / (4 pi n_H0)."""
    q0, z0 = 0.5, 4.0
    lam = 1e-9
    for a in (1.2, 2.0, 5.0):
        rel = analytic.sg_front(a, lam, q0, z0) ** 3
        # photon counting in units of r_S0^3 lambda: int_1^a [..]^(-1/2) db (q0 = 1/2)
        exact = lam * (2.0 / 3.0) * (a ** 1.5 - 1.0) / math.sqrt(1.0 + z0)
        assert rel == pytest.approx(exact, rel=1e-6)


def test_sg_tau_is_recombination_integral():
    """tau(a) = int alpha n_H dt for q0 = 1/2 (n_H ~ b^-3, dt ~ sqrt(b) db)."""
    q0, z0, lam = 0.5, 4.0, 2.2445
    for a in (1.5, 3.0):
        val, _ = integrate.quad(lambda b: b ** -2.5, 1.0, a)
        assert analytic.sg_tau(a, lam, q0, z0) == pytest.approx(lam * val / math.sqrt(1 + z0),
                                                                rel=1e-12)


def test_sg_tau_open_is_recombination_integral():
    """q0 = 0.05 (open universe, Omega_m = 0.1, h = 1): tau(a) equals the
    recombination integral alpha n_H0 int (a0/a(t))^3 dt along the open
    expansion law a(t) of the cosmology module, with
    lambda = alpha n_H0 / (H0 (1 + z0))."""
    q0, z0 = 0.05, 4.0
    cos = cosmology.Cosmology(cosmology.OPEN, 1.0, 2.0 * q0, 0.0)
    a0 = 1.0 / (1.0 + z0)
    t0 = cos.time_of_a(a0)
    alpha_nH0 = 1e-17  # s^-1; only the product enters
    lam = alpha_nH0 / (cos.H0 * (1.0 + z0))
    for abar in (1.5, 3.0, 5.0):
        t1 = cos.time_of_a(abar * a0)
        val, _ = integrate.quad(lambda t: (a0 / cos.a(t)) ** 3, t0, t1, epsabs=0.0,
                                epsrel=1e-12, limit=200)
        assert analytic.sg_tau(abar, lam, q0, z0) == pytest.approx(alpha_nH0 * val, rel=1e-9)


def test_sg_front_photon_counting_limit_open():
    """q0 = 0.05, lambda -> 0: r_I^3 / r_S0^3 = alpha n_H0 (t - t0) (every photon
    ionises one atom; r_S0^3 = 3 Q / (4 pi alpha n_H0^2)), with t(a) from the
    open expansion law."""
    q0, z0 = 0.05, 4.0
    cos = cosmology.Cosmology(cosmology.OPEN, 1.0, 2.0 * q0, 0.0)
    a0 = 1.0 / (1.0 + z0)
    t0 = cos.time_of_a(a0)
    lam = 1e-9
    for abar in (1.2, 2.0, 5.0):
        dt = cos.time_of_a(abar * a0) - t0
        exact = lam * cos.H0 * (1.0 + z0) * dt
        assert analytic.sg_front(abar, lam, q0, z0) ** 3 == pytest.approx(exact, rel=1e-6)
