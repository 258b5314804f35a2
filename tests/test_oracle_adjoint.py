"""Pins of the oracle adjoint: dot-product identity with the tangent-linear
step, and finite differences of J = mean x_HII through forward oracle steps
(step h = 1e-6 max(|p|, mean of the nonzero |p|); central differences, one
sided for parameters that are zero)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as OA, model as OM, newton as ON


def _case(cfg, dims, **over):
    w = W.scaled(cfg, dims)
    for k, v in over.items():
        setattr(w, k, v)
    p = OM.params_from_workload(w)
    nH = W.density_field(w)
    src = OM.source_field(p, W.photon_rate_field(w))
    t0, dt, _ = OM.schedule(p, w)
    return w, p, nH, src, t0, dt


CASES = {
    "iso_mono": (0, (6, 6, 6), {}),
    "lognormal_periodic": (2, (6, 4, 8), {"n_sources": 5}),
    "eds_cooling": (1, (4, 4, 4), {}),
    "theta06_outflow": (2, (4, 6, 4), {"n_sources": 3, "theta": 0.6, "dt_Myr": 0.05,
                                       "bc": (W.BC_ZEROFLUX, W.BC_OUTFLOW) * 3}),
}


@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_dot_product(case):
    cfg, dims, over = CASES[case]
    w, p, nH, src, t0, dt = _case(cfg, dims, **over)
    Un = OM.initial_state(p, nH, w.x0, w.T0, w.E0)
    Un = ON.step(p, t0, dt, nH, src, *Un, tol=1e-13)
    U1 = ON.step(p, t0 + dt, dt, nH, src, *Un, tol=1e-13)
    rng = np.random.default_rng(5)
    rv = lambda: rng.standard_normal(p.dims)  # noqa: E731
    scale = (np.max(Un[0]), np.max(Un[1]), np.max(nH))
    dUn = (rv() * scale[0], None if p.isothermal else rv() * scale[1], rv() * scale[2])
    dsrc, dnH = rv() * np.max(src), rv() * np.max(nH)
    wv = (rv(), None if p.isothermal else rv(), rv())
    tl = OA.tangent_step(p, t0 + dt, dt, nH, src, Un, U1, dUn, dsrc, dnH)
    (aE, ae, an), gs, gh = OA.adjoint_step(p, t0 + dt, dt, nH, src, Un, U1, wv)
    lhs = sum(np.sum(a * b) for a, b in zip(wv, tl) if a is not None)
    rhs = (np.sum(aE * dUn[0]) + np.sum(an * dUn[2]) + np.sum(gs * dsrc) + np.sum(gh * dnH)
           + (0.0 if p.isothermal else np.sum(ae * dUn[1])))
    assert lhs == pytest.approx(rhs, rel=1e-9)


def _fd_check(case, nsteps, nrand=3, ntop=3):
    cfg, dims, over = CASES[case]
    w, p, nH, src, t0, dt = _case(cfg, dims, **over)
    J0, g_src, g_nH = OA.gradient(p, t0, dt, nsteps, nH, src, w.x0, w.T0, w.E0)

    def x_final(nHx, srcx):
        E, e, n = OM.initial_state(p, nHx, w.x0, w.T0, w.E0)
        for s in range(nsteps):
            E, e, n = ON.step(p, t0 + s * dt, dt, nHx, srcx, E, e, n, tol=1e-13)
        return 1.0 - n / nHx
    rng = np.random.default_rng(11)
    for name, arr, g in (("nH", nH, g_nH), ("src", src, g_src)):
        top = np.argsort(-np.abs(g).ravel())[:ntop]
        cells = np.unique(np.concatenate([top, rng.choice(p.ncells, size=nrand, replace=False)]))
        nz = np.abs(arr[arr != 0])
        pbar = nz.mean() if nz.size else 1.0
        gmax = np.max(np.abs(g))
        for c in cells:
            h = 1e-6 * max(abs(arr.flat[c]), pbar)
            ap, am = arr.copy(), arr.copy()
            ap.flat[c] += h
            # a zero emissivity sits on the kink of max(E, 0) in the rates when
            # stepped negative: one-sided difference there, central elsewhere
            one_sided = arr.flat[c] == 0.0
            if not one_sided:
                am.flat[c] -= h
            xp = x_final(ap, src) if name == "nH" else x_final(nH, ap)
            xm = x_final(am, src) if name == "nH" else x_final(nH, am)
            # J(p+h) - J(p-h) from per-cell differences (no cancellation in J itself)
            fd = float(np.mean(xp - xm)) / (h if one_sided else 2 * h)
            denom = max(abs(fd), 1e-6 * gmax)
            if abs(g.flat[c]) < 1e-3 * gmax:
                # below the finite-difference resolution of this step: absolute check
                assert abs(g.flat[c] - fd) < 1e-6 * gmax, (name, c, g.flat[c], fd)
            else:
                assert abs(g.flat[c] - fd) / denom < 1e-4, (name, c, g.flat[c], fd)


@pytest.mark.parametrize("case,nsteps", [("iso_mono", 2), ("lognormal_periodic", 2),
                                         ("eds_cooling", 2), ("theta06_outflow", 1)])
def test_adjoint_gradient_against_central_differences(case, nsteps):
    _fd_check(case, nsteps)


CASES["stromgren_dark"] = (0, (12, 12, 12), {})


@pytest.mark.parametrize("case", ["stromgren_dark", "theta06_outflow"])
def test_limiter_jacobian_blocks_against_central_differences(case):
    """Columns of df_E/dE^n and df_E/dn^n (the lagged limiter, and the
    explicit part when theta < 1) against central differences with steps
    relative to each value, in the darkest cells (E^n many decades below its
    maximum, where the limiter is nonlinear on the scale of E^n itself) and
    in random cells."""
    cfg, dims, over = CASES[case]
    w, p, nH, src, t0, dt = _case(cfg, dims, **over)
    Un = OM.initial_state(p, nH, w.x0, w.T0, w.E0)
    Un = ON.step(p, t0, dt, nH, src, *Un, tol=1e-13)
    U1 = ON.step(p, t0 + dt, dt, nH, src, *Un, tol=1e-13)
    JU, JUn, _, _ = OA._jacobians(p, t0 + dt, dt, nH, src, Un, U1)
    N = p.ncells
    off = N if p.isothermal else 2 * N      # E block of the unknown order (n, [e,] E)
    JEEn = JUn[off:, off:].tocsc()
    JEnn = JUn[off:, :N].tocsc()

    def fE(En, nn):
        c = OM.make_context(p, t0 + dt, dt, nH, src, En, Un[1], nn)
        return OM.f_E(p, c, U1[0], U1[2]).ravel()
    if case == "stromgren_dark":
        assert np.min(Un[0]) < 1e-20 * np.max(Un[0])
    rng = np.random.default_rng(4)
    dark = np.argsort(Un[0].ravel())[:12]
    cols = np.unique(np.concatenate([dark, rng.choice(N, 12, replace=False)]))
    for j in cols:
        for k, J in ((0, JEEn), (1, JEnn)):
            base = [Un[0].copy(), Un[2].copy()]
            h = 1e-6 * abs(base[k].flat[j])
            bp = [b.copy() for b in base]
            bm = [b.copy() for b in base]
            bp[k].flat[j] += h
            bm[k].flat[j] -= h
            col = (fE(*bp) - fE(*bm)) / (2 * h)
            jc = J[:, j].toarray().ravel()
            scale = np.max(np.abs(col)) + 1e-300
            assert np.max(np.abs(jc - col)) <= 1e-3 * scale, (k, j, np.max(np.abs(jc - col)), scale)
