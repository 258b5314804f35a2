"""GPU parity of the hydrogen + helium multigroup step (rh_multigroup_*)
against the multigroup oracle (oracle/multigroup.py) on the same seeded
inputs: initial fields, residuals at perturbed states (elementwise), whole
steps in FP64 and mixed precision (elementwise), the one-group,
hydrogen-only limit against the grey GPU step, and one step of the 128^3
volume checked at sampled cells."""
import numpy as np
import pytest

import workloads as W
from gpu_cases import cached, elementwise, to_dev
from oracle import model as OM, multigroup as MG

pytestmark = pytest.mark.gpu

EDGES3 = (13.6, 24.587, 54.4)
EDGES4 = (13.6, 20.0, 30.0, 60.0)

# name -> (workload id, dims, Workload overrides, edges, y_he, steps)
MG_CASES = {
    "he3_lognormal": (2, (8, 8, 16), {"n_sources": 3}, EDGES3, 0.08, 2),
    "he4_eds": (1, (8, 8, 8), {}, EDGES4, 0.08, 2),
    "he3_theta06": (2, (8, 8, 8), {"theta": 0.6, "dt_Myr": 0.02, "n_sources": 2}, EDGES3, 0.08, 2),
    "he2_iso": (1, (8, 8, 8), {"isothermal": True}, EDGES3[:2], 0.08, 2),
    "he3_lcdm": (4, (8, 8, 8), {"n_sources": 4}, EDGES3, 0.08, 1),
    "h3_nohe": (2, (8, 8, 8), {"n_sources": 2}, EDGES3, 0.0, 2),
    # several workgroups and ragged sizes (residual only: the oracle's
    # direct solve would be slow here)
    "he3_ragged": (2, (24, 20, 36), {}, EDGES3, 0.08, 0),
}


def _setup(name, **pover):
    cfg, dims, over, edges, y_he, nsteps = MG_CASES[name]
    w = W.scaled(cfg, dims)
    for k, v in over.items():
        setattr(w, k, v)
    mp = MG.params_from_workload(w, edges, y_he, **pover)
    nH = W.density_field(w)
    src = OM.source_field(mp.base, W.photon_rate_field(w))
    t0, dt, _ = OM.schedule(mp.base, w)
    E, e, y = MG.initial_state(mp, nH, w.x0, w.T0, w.E0)
    return w, mp, dict(nH=nH, src=src, E=E, e=e, y=y, t0=t0, dt=dt, nsteps=nsteps)


def _solver(w, mp, dev, **prm):
    import paper_0908_2654_amd as P
    p = P.params_from_workload(w, **prm)
    m = P.multigroup_params(mp.edges_eV, mp.y_he, mp.sigma_power)
    return P.MultigroupSolver(p, m, device=dev)


def _gpu_state(inp, dev, iso):
    return (to_dev(inp["E"], dev), None if iso else to_dev(inp["e"], dev), to_dev(inp["y"], dev))


def test_initial_fields_match_oracle(hip_device):
    for name in ("he3_lognormal", "he2_iso", "h3_nohe"):
        w, mp, inp = _setup(name)
        s = _solver(w, mp, hip_device)
        E, e, y = s.empty_state()
        s.initial_state(to_dev(inp["nH"], hip_device), w.x0, w.T0, w.E0, E, e, y)
        assert elementwise(E.cpu().numpy(), inp["E"], 1e-30) < 1e-15, name
        nrows = 3 if mp.he else 1
        assert elementwise(y.cpu().numpy()[:nrows], inp["y"][:nrows], 1e-30) < 1e-15, name
        if e is not None:
            assert elementwise(e.cpu().numpy(), inp["e"], 1e-30) < 1e-14, name
        s.close()


def _perturbed(name, mp, inp):
    """U^n one oracle step on; U = U^n perturbed within the admissible set."""
    En, en, yn = cached(("mg_first", name), lambda: MG.step(
        mp, inp["t0"], inp["dt"], inp["nH"], inp["src"], inp["E"], inp["e"], inp["y"], tol=1e-10))
    rng = np.random.default_rng(7)
    E = En * (1 + 0.2 * rng.standard_normal(En.shape)) + 1e-3 * En.max() * rng.random(En.shape)
    nHe = mp.y_he * inp["nH"]
    y = yn.copy()
    y[0] = np.clip(yn[0] * (1 + 0.1 * rng.standard_normal(yn[0].shape)), 0, inp["nH"])
    if mp.he:
        y[1] = np.clip(yn[1] * (1 + 0.1 * rng.standard_normal(yn[1].shape)), 0, nHe)
        y[2] = np.clip(yn[2] * (1 + 0.1 * rng.standard_normal(yn[2].shape)), 0, nHe - y[1])
    e = en * (1 + 0.1 * rng.random(en.shape))
    return (En, en, yn), (E, e, y)


@pytest.mark.parametrize("name", list(MG_CASES))
def test_residual_parity(hip_device, name):
    w, mp, inp = _setup(name)
    if MG_CASES[name][5] == 0:
        # large case: U^n from the initial state perturbed instead of a step
        rng = np.random.default_rng(3)
        Un = (inp["E"] * (1 + 0.3 * rng.random(inp["E"].shape)), inp["e"], inp["y"])
        _, U = _perturbed_from(mp, inp, Un, rng)
    else:
        Un, U = _perturbed(name, mp, inp)
    t, dt = inp["t0"] + inp["dt"], inp["dt"]
    ctx = MG.make_context(mp, t, dt, inp["nH"], inp["src"], *Un)
    fE, fe, fy = MG.residual(mp, ctx, U[0], None if mp.base.isothermal else U[1], U[2])
    nrm = MG.norm(mp, ctx, fE, fe, fy)
    s = _solver(w, mp, hip_device)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    iso = mp.base.isothermal
    Ung = (d(Un[0]), None if iso else d(Un[1]), d(Un[2]))
    Ug = (d(U[0]), None if iso else d(U[1]), d(U[2]))
    gE, ge, gy, gnorm = s.residual(t, dt, d(inp["nH"]), d(inp["src"]), Ung, Ug)
    s.close()
    gE, gy = gE.cpu().numpy(), gy.cpu().numpy()
    errs = {f"fE{g}": elementwise(gE[g], fE[g], 1e-12) for g in range(mp.G)}
    errs["fHI"] = elementwise(gy[0], fy[0], 1e-12)
    if mp.he:
        errs["fHeI"] = elementwise(gy[1], fy[1], 1e-12)
        errs["fHeII"] = elementwise(gy[2], fy[2], 1e-12)
    if not iso:
        errs["fe"] = elementwise(ge.cpu().numpy(), fe, 1e-12)
    print(name, {k: f"{v:.1e}" for k, v in errs.items()}, gnorm, nrm)
    assert max(errs.values()) < 1e-11
    assert gnorm == pytest.approx(nrm, rel=1e-12)


def _perturbed_from(mp, inp, Un, rng):
    En, en, yn = Un
    E = En * (1 + 0.2 * rng.standard_normal(En.shape)) + 1e-3 * En.max() * rng.random(En.shape)
    nHe = mp.y_he * inp["nH"]
    y = yn.copy()
    y[0] = np.clip(inp["nH"] * rng.random(yn[0].shape), 0, inp["nH"])
    if mp.he:
        y[1] = nHe * 0.6 * rng.random(yn[1].shape)
        y[2] = (nHe - y[1]) * rng.random(yn[2].shape)
    e = en * (1 + 0.5 * rng.random(en.shape))
    return Un, (E, e, y)


def _oracle_traj(name, mp, inp, tol):
    def run():
        E, e, y = inp["E"], inp["e"], inp["y"]
        for k in range(inp["nsteps"]):
            E, e, y = MG.step(mp, inp["t0"] + k * inp["dt"], inp["dt"], inp["nH"], inp["src"],
                              E, e, y, tol=tol)
        return E, e, y
    return cached(("mg_traj", name, tol), run)


def _gpu_traj(name, w, mp, inp, dev, **prm):
    s = _solver(w, mp, dev, **prm)
    nH, src = to_dev(inp["nH"], dev), to_dev(inp["src"], dev)
    E, e, y = _gpu_state(inp, dev, mp.base.isothermal)
    stats = []
    for k in range(inp["nsteps"]):
        stats.append(s.step(inp["t0"] + k * inp["dt"], inp["dt"], nH, src, E, e, y))
    s.close()
    return (E.cpu().numpy(), None if e is None else e.cpu().numpy(), y.cpu().numpy()), stats


def _traj_errors(g, o, mp, nH):
    Eg, eg, yg = g
    Eo, eo, yo = o
    err = {f"E{k}": elementwise(Eg[k], Eo[k], 1e-12) for k in range(mp.G)}
    # species relative to their element's density (x floor 1e-6 as the grey tests)
    err["x_HI"] = float(np.max(np.abs(yg[0] - yo[0]) / nH / np.maximum(1 - yo[0] / nH, 1e-6)))
    if mp.he:
        nHe = mp.y_he * nH
        err["HeI"] = float(np.max(np.abs(yg[1] - yo[1]) / nHe))
        err["HeII"] = float(np.max(np.abs(yg[2] - yo[2]) / nHe))
    if eg is not None:
        err["e"] = float(np.max(np.abs(eg - eo) / np.abs(eo)))
    return err


TRAJ_CASES = [n for n, c in MG_CASES.items() if c[5] > 0]


@pytest.mark.parametrize("name", TRAJ_CASES)
def test_step_parity_fp64(hip_device, name):
    w, mp, inp = _setup(name, newton_tol=1e-12)
    o = _oracle_traj(name, mp, inp, 1e-12)
    g, st = _gpu_traj(name, w, mp, inp, hip_device, newton_tol=1e-12, precision=0)
    err = _traj_errors(g, o, mp, inp["nH"])
    print(name, "fp64", {k: f"{v:.1e}" for k, v in err.items()},
          [(s["newton_its"], s["lin_its_total"], s["lin_its_max"]) for s in st])
    assert max(err.values()) < 1e-10
    assert all(s["lin_cap_hits"] == 0 for s in st)


@pytest.mark.parametrize("name", ["he3_lognormal", "he2_iso"])
def test_step_parity_defect_correction(hip_device, name):
    """Each group's inner solve by plain FP64 defect correction around the
    V-cycle (krylov = 0) instead of conjugate gradients."""
    w, mp, inp = _setup(name, newton_tol=1e-12)
    o = _oracle_traj(name, mp, inp, 1e-12)
    g, st = _gpu_traj(name, w, mp, inp, hip_device, newton_tol=1e-12, precision=0, krylov=0)
    err = _traj_errors(g, o, mp, inp["nH"])
    print(name, "defect correction", {k: f"{v:.1e}" for k, v in err.items()},
          [(s["newton_its"], s["lin_its_total"], s["lin_its_max"]) for s in st])
    assert max(err.values()) < 1e-10
    assert all(s["lin_cap_hits"] == 0 for s in st)


@pytest.mark.parametrize("name", ["he3_lognormal", "he4_eds", "he3_lcdm"])
def test_step_parity_mixed(hip_device, name):
    w, mp, inp = _setup(name, newton_tol=1e-12)
    o = _oracle_traj(name, mp, inp, 1e-12)
    g, st = _gpu_traj(name, w, mp, inp, hip_device, newton_tol=1e-12, precision=1)
    err = _traj_errors(g, o, mp, inp["nH"])
    print(name, "mixed", {k: f"{v:.1e}" for k, v in err.items()},
          [(s["newton_its"], s["lin_its_total"], s["lin_its_max"]) for s in st])
    assert max(err.values()) < 1e-6


@pytest.mark.parametrize("cfg,dims", [(2, (24, 20, 36)), (1, (16, 16, 16))])
def test_one_group_without_helium_is_the_grey_gpu_step(hip_device, cfg, dims):
    """G = 1, y_He = 0: the multigroup step solves the grey step's equations
    (the local block reduces to (e, n_HI) and the group constants to the
    grey ones), so both GPU paths reach the same root."""
    import paper_0908_2654_amd as P
    w = W.scaled(cfg, dims)
    p = P.params_from_workload(w, newton_tol=1e-12, precision=0)
    op = OM.params_from_workload(w)
    nH = W.density_field(w)
    src = OM.source_field(op, W.photon_rate_field(w))
    t0, dt, _ = OM.schedule(op, w)
    E, e, n = OM.initial_state(op, nH, w.x0, w.T0, w.E0)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    grey = P.Solver(p, device=hip_device)
    mgs = P.MultigroupSolver(p, P.multigroup_params((p.hnu0_eV,), 0.0), device=hip_device)
    nHd, srcd = d(nH), d(src)
    Eg, eg, ng = d(E), d(e), d(n)
    Em, em = d(E[None]), d(e)
    ym = d(np.stack([n, 0 * n, 0 * n]))
    for k in range(3):
        grey.step(t0 + k * dt, dt, nHd, srcd, Eg, eg, ng)
        mgs.step(t0 + k * dt, dt, nHd, srcd, Em, em, ym)
        a = (Eg.cpu().numpy(), eg.cpu().numpy(), ng.cpu().numpy())
        b = (Em.cpu().numpy()[0], em.cpu().numpy(), ym.cpu().numpy()[0])
        eE = elementwise(b[0], a[0], 1e-12)
        ee = float(np.max(np.abs(b[1] - a[1]) / a[1]))
        ex = float(np.max(np.abs(b[2] - a[2]) / nH / np.maximum(1 - a[2] / nH, 1e-6)))
        print(k, eE, ee, ex)
        assert max(eE, ee, ex) < 1e-10
        assert np.all(ym.cpu().numpy()[1:] == 0.0)
    grey.close()
    mgs.close()


def test_step_restores_state_on_failure_and_rejects_bad_arguments(hip_device):
    from paper_0908_2654_amd import _lib
    w, mp, inp = _setup("he3_lognormal")
    s = _solver(w, mp, hip_device, newton_max_it=1, newton_tol=1e-14)
    nH, src = to_dev(inp["nH"], hip_device), to_dev(inp["src"], hip_device)
    E, e, y = _gpu_state(inp, hip_device, False)
    E0, e0, y0 = E.clone(), e.clone(), y.clone()
    with pytest.raises(_lib.RhError) as ex:
        s.step(inp["t0"], inp["dt"], nH, src, E, e, y)
    assert ex.value.status == _lib.RH_ENEWTON
    assert E.equal(E0) and e.equal(e0) and y.equal(y0)
    with pytest.raises(_lib.RhError) as ex:
        s.step(inp["t0"], -1.0, nH, src, E, e, y)
    assert ex.value.status == _lib.RH_EINVAL
    s.close()


def test_full_size_multigroup_step_sampled(hip_device):
    """The 128^3 lognormal volume (32 sources, periodic) with three groups and
    helium, in the configuration bench.py --multigroup times (mixed
    precision, FGMRES around the block sweep): one GPU step, then at sampled
    cells (source cells, the most ionised cells, random cells) the oracle
    evaluates on a periodic 3^3 block around the cell (a cell's residual
    needs only its face neighbours; the limiter floor is the whole box's)
    the residual of the GPU's solution, which rh_multigroup_residual also
    evaluated for the whole grid."""
    w = W.get(2)
    mp = MG.params_from_workload(w, EDGES3, 0.08)
    nH = W.density_field(w)
    src = OM.source_field(mp.base, W.photon_rate_field(w))
    t0, dt, _ = OM.schedule(mp.base, w)
    E0, e0, y0 = MG.initial_state(mp, nH, w.x0, w.T0, w.E0)
    s = _solver(w, mp, hip_device, precision=1)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    nHd, srcd = d(nH), d(src)
    Un = (d(E0), d(e0), d(y0))
    U = tuple(x.clone() for x in Un)
    st = s.step(t0, dt, nHd, srcd, *U)
    print("step", {k: st[k] for k in ("newton_its", "lin_its_total", "lin_its_max", "res_final")})
    assert st["lin_cap_hits"] == 0
    gE, ge, gy, gnorm = s.residual(t0, dt, nHd, srcd, Un, U)
    s.close()
    assert gnorm <= w.newton_tol and gnorm == pytest.approx(st["res_final"], rel=1e-6)
    U1 = tuple(x.cpu().numpy() for x in U)
    g = (gE.cpu().numpy(), ge.cpu().numpy(), gy.cpu().numpy())
    worst, sampled, cells = sampled_check(w, mp, nH, src, t0, dt, (E0, e0, y0), U1, g)
    print("cells", len(cells), "parity", worst, "oracle residual at sampled cells", sampled)
    assert worst["fE"] < 1e-12 and worst["fy"] < 1e-12 and worst["fe"] < 1e-12
    assert sampled["fE"] < 1e-5 and sampled["fy"] < 1e-5 and sampled["fe"] < 1e-5


def sampled_check(w, mp, nH, src, t0, dt, Un, U1, g):
    """Largest differences between the residual g = (fE, fe, fy) of state U1
    (step from Un) and the oracle's, at sampled cells each on a periodic
    3^3 block, relative to the size of the terms; and the oracle's residual
    there.  Returns (worst, sampled, cells)."""
    import dataclasses

    from oracle.constants import C_LIGHT
    E0, e0, y0 = Un
    E1, e1, y1 = U1
    gE, ge, gy = g
    dims = w.dims
    rng = np.random.default_rng(5)
    cells = [tuple(int(v) for v in c) for c in np.argwhere(src > 0)[:16]]
    x1 = 1.0 - y1[0] / nH
    top = np.argpartition(x1.ravel(), -64)[-64:]
    cells += [tuple(int(v) for v in np.unravel_index(i, dims)) for i in rng.choice(top, 16, replace=False)]
    cells += [tuple(int(rng.integers(0, n)) for n in dims) for _ in range(24)]
    a_n = mp.base.cosmo.a(t0)
    bp = mp.base.with_(dims=(3, 3, 3), box=3 * mp.base.h, R_min=1.0 / (a_n * mp.base.box),
                       bc=(1,) * 6)
    mpb = dataclasses.replace(mp, base=bp)
    srcg = np.stack([f * src for f in mp.groups["frac"]])
    E_s = [max(float(E0[g].max()), dt * float(srcg[g].max()), bp.E_floor) for g in range(mp.G)]
    nHe_all = mp.y_he * nH
    ctr = (1, 1, 1)
    worst = {"fE": 0.0, "fy": 0.0, "fe": 0.0}
    sampled = {"fE": 0.0, "fy": 0.0, "fe": 0.0}
    for c in cells:
        idx = [np.arange(c[k] - 1, c[k] + 2) % dims[k] for k in range(3)]
        cut = lambda X: X[np.ix_(*idx)]  # noqa: E731
        cutg = lambda X: np.stack([cut(X[g]) for g in range(X.shape[0])])  # noqa: E731
        ctx = MG.make_context(mpb, t0, dt, cut(nH), cut(src), cutg(E0), cut(e0), cutg(y0))
        Eb, eb, yb = cutg(E1), cut(e1), cutg(y1)
        fEo, feo, fyo = MG.residual(mpb, ctx, Eb, eb, yb)
        kap = MG.opacity(mpb, yb, ctx.a_1)
        for g in range(mp.G):
            cfs = sum(ctx.cf_1[g][a][ctr] + ctx.cf_1[g][a][tuple(2 if b == a else 1 for b in range(3))]
                      for a in range(3))
            scale = np.abs(Eb[g]).max() * (1.0 + dt * cfs) + abs(ctx.En[g][ctr]) \
                + dt * ctx.src[g][ctr] + dt * C_LIGHT * kap[g][ctr] * abs(Eb[g][ctr])
            worst["fE"] = max(worst["fE"], abs(gE[g][c] - fEo[g][ctr]) / scale)
            sampled["fE"] = max(sampled["fE"], abs(fEo[g][ctr]) / E_s[g])
        nHe = nHe_all[c]
        for sp_, ref in ((0, nH[c]), (1, nHe), (2, nHe)):
            worst["fy"] = max(worst["fy"], abs(gy[sp_][c] - fyo[sp_][ctr]) / ref)
            sampled["fy"] = max(sampled["fy"], abs(fyo[sp_][ctr]) / ref)
        worst["fe"] = max(worst["fe"], abs(ge[c] - feo[ctr]) / eb[ctr])
        sampled["fe"] = max(sampled["fe"], abs(feo[ctr]) / ctx.en[ctr])
    return worst, sampled, cells


def test_kernel_timing_covers_the_step(hip_device):
    """Per-kernel event timing of the multigroup step: the local solves, the
    coupled residuals, the FGMRES vector work and every group's multigrid
    are timed, and timing leaves the step's result bitwise unchanged."""
    w, mp, inp = _setup("he3_lognormal")
    s = _solver(w, mp, hip_device, precision=1)
    nH, src = to_dev(inp["nH"], hip_device), to_dev(inp["src"], hip_device)
    U0 = _gpu_state(inp, hip_device, mp.base.isothermal)
    U1 = tuple(x.clone() for x in U0)
    st0 = s.step(inp["t0"], inp["dt"], nH, src, *U0)
    s.set_kernel_timing(True)
    s.kernel_timing(reset=True)
    st1 = s.step(inp["t0"], inp["dt"], nH, src, *U1)
    kt = s.kernel_timing()
    s.set_kernel_timing(False)
    s.close()
    print({k: v for k, v in kt.items() if v[1]})
    for k in ("local_groups", "coupled_residual", "krylov", "residual_schur", "step_setup"):
        assert kt[k][1] > 0 and kt[k][0] > 0, k
    assert kt["rbgs_fine"][1] + kt["rbgs_fine_colour"][1] + kt["coarse_levels"][1] > 0
    assert st1["newton_its"] == st0["newton_its"] and st1["lin_its_total"] == st0["lin_its_total"]
    for a, b in zip(U0, U1):
        assert torch_equal(a, b)


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))
