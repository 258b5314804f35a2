"""Parity at the benchmark workloads' full sizes: the 64^3 EdS sphere, the
128^3 and 256^3 lognormal volumes and the 512^3 periodic reionisation
volume (flat LCDM, z = 9, 4096 sources), the last in the launch
configuration the benchmark times (mixed precision, conjugate gradients
with the V(2,2) preconditioner, fused marching kernels on the finest
level).  One implicit step runs on the GPU; the oracle then evaluates, cell
by cell at sampled cells (source cells, the most ionised cells, random
cells, corners; away from walls on walled axes), what the GPU evaluated
for the whole grid:

  * the residual f(U^{n+1}) of the GPU's solution (rh_residual), on a
    periodic 3^3 block around the cell (the residual of a cell needs only
    its face neighbours; the limiter floor R_min = 1/(a_n L_box) is the
    whole box's);
  * the Schur operator's row of the cell (rh_schur_operator): diagonal and
    the six couplings;
  * the step's own convergence: the GPU's RMS residual norm is below the
    Newton tolerance and the oracle's sampled residuals are small.
"""
import numpy as np
import pytest

import workloads as W
from gpu_cases import oracle_inputs, to_dev
from oracle.constants import C_LIGHT

pytestmark = pytest.mark.gpu


def _ranges(op):
    """Sampled index range per axis: all cells on periodic axes, the interior
    ones on walled axes (there a periodic 3^3 cut is a cell's true neighbourhood)."""
    return [(0, n) if op.bc[2 * d] == 1 else (1, n - 1) for d, n in enumerate(op.dims)]


def _cells(op, inp, n_src=16, n_front=16, n_rand=24, seed=3):
    rng = np.random.default_rng(seed)
    rg = _ranges(op)
    inside = lambda c: all(lo <= c[d] < hi for d, (lo, hi) in enumerate(rg))  # noqa: E731
    src_cells = [c for c in np.argwhere(inp["src"] > 0) if inside(c)]
    pick = rng.choice(len(src_cells), min(n_src, len(src_cells)), replace=False)
    cells = [tuple(int(v) for v in src_cells[i]) for i in pick]
    (a0, b0), (a1, b1), (a2, b2) = rg
    cells += [(a0, a1, a2), (b0 - 1, b1 - 1, b2 - 1), (a0, b1 - 1, a2 + 5), (b0 - 1, a1 + 2, a2)]
    cells += [tuple(int(rng.integers(lo, hi)) for lo, hi in rg) for _ in range(n_rand)]
    return cells, n_front


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_full_size_step_residual_and_operator_sampled(hip_device, cfg):
    """Each benchmark workload at its own size and precision (64^3 EdS FP64
    sphere, 128^3 and 256^3 lognormal volumes, and the 512^3 reionisation
    volume in exactly the benchmark's launch configuration)."""
    import paper_0908_2654_amd as P
    w = W.get(cfg)
    op, inp = oracle_inputs(w)
    t0, dt = inp["t0"], inp["dt"]
    prm = P.params_from_workload(w)
    if cfg == 4:
        assert prm.precision == 1 and prm.krylov == 1 and prm.mg_pre == 2 and prm.mg_post == 2
    s = P.Solver(prm, device=hip_device)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    nH, src = d(inp["nH"]), d(inp["src"])
    Un = tuple(d(inp[k]) for k in ("E", "e", "n"))
    U = tuple(x.clone() for x in Un)
    st = s.step(t0, dt, nH, src, *U)
    print("step", {k: st[k] for k in ("newton_its", "lin_its_total", "res_final")})
    fE, fe, fn, nrm = s.residual(t0, dt, nH, src, Un, U)
    assert nrm <= w.newton_tol and nrm == pytest.approx(st["res_final"], rel=1e-6)
    diag, cf = s.schur_operator(t0, dt, nH, src, Un, U)
    s.close()
    host = lambda X: X.cpu().numpy()  # noqa: E731
    Uh = tuple(host(x) for x in U)
    xh = 1.0 - Uh[2] / inp["nH"]
    worst, sampled, ncells = check_cells(op, inp, Uh, (host(fE), host(fe), host(fn)), host(diag),
                                         [host(c) for c in cf], xh)
    print(w.name, "cells", ncells, "parity", worst, "oracle residual at sampled cells", sampled)
    assert worst["fE"] < 1e-12 and worst["fn"] < 1e-12 and worst["fe"] < 1e-12
    assert worst["diag"] < 1e-12 and worst["off"] < 1e-12
    # the step's solution solves the oracle's equations at the sampled cells
    assert sampled["fE"] < 1e-5 and sampled["fn"] < 1e-5 and sampled["fe"] < 1e-5


@pytest.mark.parametrize("cfg,checked", [(3, (0, 5, 9)), (4, (5, 14, 24))])
def test_full_size_late_steps_sampled(hip_device, cfg, checked):
    """The states the benchmark times: the 512^3 volume advanced through
    steps 5..24 of its run (the timed window; checked at its first, middle
    and last step) and the 256^3 volume through its 10 steps, in their own
    launch configuration (mixed precision).  At each checked step the oracle
    evaluates, at sampled cells, the residual and the Schur row of the GPU's
    step from the GPU's checkpoint U^n, as in the first-step test, and every
    linear solve of the step reached the forcing delta_k = 1e-13 ||f(U_k)||
    (no solve stopped at the cycle cap)."""
    import paper_0908_2654_amd as P
    w = W.get(cfg)
    op, inp = oracle_inputs(w)
    t0, dt = inp["t0"], inp["dt"]
    prm = P.params_from_workload(w)
    s = P.Solver(prm, device=hip_device)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    nH, src = d(inp["nH"]), d(inp["src"])
    U = tuple(d(inp[k]) for k in ("E", "e", "n"))
    host = lambda X: X.cpu().numpy()  # noqa: E731
    for k in range(max(checked) + 1):
        t = t0 + k * dt
        Un = tuple(x.clone() for x in U) if k in checked else None
        st = s.step(t, dt, nH, src, *U)
        print(f"step {k}: newton={st['newton_its']} cycles={st['lin_its_total']} "
              f"max/solve={st['lin_its_max']} lin_res_max={st['lin_res_max']:.2e} "
              f"caps={st['lin_cap_hits']} res={st['res_final']:.2e}", flush=True)
        assert st["lin_cap_hits"] == 0 and st["lin_res_max"] <= prm.lin_forcing
        if Un is None:
            continue
        fE, fe, fn, nrm = s.residual(t, dt, nH, src, Un, U)
        assert nrm <= w.newton_tol and nrm == pytest.approx(st["res_final"], rel=1e-6)
        diag, cf = s.schur_operator(t, dt, nH, src, Un, U)
        Unh = tuple(host(x) for x in Un)
        Uh = tuple(host(x) for x in U)
        inp_k = dict(inp, E=Unh[0], e=Unh[1], n=Unh[2], t0=t)
        worst, sampled, ncells = check_cells(op, inp_k, Uh, (host(fE), host(fe), host(fn)),
                                             host(diag), [host(c) for c in cf],
                                             1.0 - Uh[2] / inp["nH"])
        print(w.name, "step", k, "cells", ncells, "parity", worst, "oracle residual", sampled,
              flush=True)
        assert worst["fE"] < 1e-12 and worst["fn"] < 1e-12 and worst["fe"] < 1e-12
        assert worst["diag"] < 1e-12 and worst["off"] < 1e-12
        assert sampled["fE"] < 1e-5 and sampled["fn"] < 1e-5 and sampled["fe"] < 1e-5
        del fE, fe, fn, diag, cf
    s.close()


def check_cells(op, inp, U, f, diag, cf, xh):
    """Largest differences between the given residual fields f = (fE, fe, fn)
    and Schur operator (diag, cf) of state U and the oracle's, at sampled
    cells (each on a periodic 3^3 block); and the oracle's residual there."""
    from oracle import model as OM, newton as ON
    fE, fe, fn = f
    t0, dt = inp["t0"], inp["dt"]
    dims = op.dims
    cells, n_front = _cells(op, inp)
    # the most ionised cells (after one step the H II regions are still
    # smaller than a cell): 16 of the 64 with the largest x_HII
    rg = _ranges(op)
    sl = tuple(slice(lo, hi) for lo, hi in rg)
    xin = xh[sl]
    top = np.argpartition(xin.ravel(), -64)[-64:]
    rng = np.random.default_rng(4)
    cells += [tuple(int(v) + lo for v, (lo, _) in zip(np.unravel_index(i, xin.shape), rg))
              for i in rng.choice(top, n_front, replace=False)]
    a_n = op.cosmo.a(t0)
    bp = op.with_(dims=(3, 3, 3), box=3 * op.h, R_min=1.0 / (a_n * op.box), bc=(1,) * 6)
    worst = {"fE": 0.0, "fn": 0.0, "fe": 0.0, "diag": 0.0, "off": 0.0}
    sampled = {"fE": 0.0, "fn": 0.0, "fe": 0.0}
    E_s = max(float(inp["E"].max()), dt * float(inp["src"].max()), op.E_floor)
    ctr = (1, 1, 1)
    for c in cells:
        idx = [np.arange(c[k] - 1, c[k] + 2) % dims[k] for k in range(3)]
        cut = lambda X: X[np.ix_(*idx)]  # noqa: E731
        nHb, srcb = cut(inp["nH"]), cut(inp["src"])
        Enb, enb, nnb = cut(inp["E"]), cut(inp["e"]), cut(inp["n"])
        Eb, eb, nb = (cut(x) for x in U)
        ctx = OM.make_context(bp, t0, dt, nHb, srcb, Enb, enb, nnb)
        fEo, feo, fno = OM.residual(bp, ctx, Eb, eb, nb)
        # residual parity, relative to the size of the terms whose
        # difference f_E is (E, E^n, dt src, dt c kappa E and the diffusion
        # couplings dt sum_f cf_f E)
        cfs = ctx.cf_1[0][ctr] + ctx.cf_1[0][2, 1, 1] + ctx.cf_1[1][ctr] + ctx.cf_1[1][1, 2, 1] \
            + ctx.cf_1[2][ctr] + ctx.cf_1[2][1, 1, 2]
        scaleE = np.abs(Eb).max() * (1.0 + dt * cfs) + abs(Enb[ctr]) + dt * srcb[ctr] \
            + dt * C_LIGHT * op.grey["sigma_E"] * nb[ctr] / ctx.a_1 ** 3 * abs(Eb[ctr])
        worst["fE"] = max(worst["fE"], abs(fE[c] - fEo[ctr]) / scaleE)
        worst["fn"] = max(worst["fn"], abs(fn[c] - fno[ctr]) / nHb[ctr])
        worst["fe"] = max(worst["fe"], abs(fe[c] - feo[ctr]) / eb[ctr])
        sampled["fE"] = max(sampled["fE"], abs(fEo[ctr]) / E_s)
        sampled["fn"] = max(sampled["fn"], abs(fno[ctr]) / nHb[ctr])
        sampled["fe"] = max(sampled["fe"], abs(feo[ctr]) / enb[ctr])
        # Schur operator row of the cell: diagonal and the six couplings
        loc = ON.local_jacobian(bp, ctx, Eb, eb, nb)
        JEE, JEn = ON.radiation_jacobian(bp, ctx, Eb, nb)
        S = ON.schur_operator(bp, loc, JEE, JEn, feo, fno, fEo)[0].tocsr()
        ci = np.ravel_multi_index(ctr, (3, 3, 3))
        worst["diag"] = max(worst["diag"], abs(diag[c] - S[ci, ci]) / abs(S[ci, ci]))
        for ax in range(3):
            dn = list(c)
            dn[ax] = (c[ax] - 1) % dims[ax]
            bu, bd = [1, 1, 1], [1, 1, 1]
            bu[ax], bd[ax] = 2, 0
            ju = np.ravel_multi_index(bu, (3, 3, 3))
            jd = np.ravel_multi_index(bd, (3, 3, 3))
            ref = max(abs(S[ci, ju]), abs(S[ci, jd]), 1e-300)
            worst["off"] = max(worst["off"], abs(-cf[ax][c] - S[ci, ju]) / ref,
                               abs(-cf[ax][tuple(dn)] - S[ci, jd]) / ref)
    return worst, sampled, len(cells)


def test_full_size_adjoint_matches_finite_differences(hip_device):
    """The adjoint of one step at 512^3 (mixed path) against central finite
    differences of the forward step, for J = mean x_HII: the directional
    derivatives along random one-signed perturbations of the source
    strengths (steps of 1%) and of n_H (steps of 0.05%) (a property that holds at any size; the oracle's transpose solve
    does not fit this grid).  Newton converges to 1e-11 on every forward
    step so that the differences resolve the change of J."""
    import torch

    import paper_0908_2654_amd as P
    w = W.get(4)
    op, inp = oracle_inputs(w)
    t0, dt = inp["t0"], inp["dt"]
    s = P.Solver(P.params_from_workload(w, precision=1, newton_tol=1e-11), device=hip_device)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    nH, src = d(inp["nH"]), d(inp["src"])
    U0 = tuple(d(inp[k]) for k in ("E", "e", "n"))
    N = float(op.ncells)

    def J(src_, nH_):
        U = tuple(x.clone() for x in U0)
        s.step(t0, dt, nH_, src_, *U)
        return float((1.0 - U[2] / nH_).sum().item() / N), U

    J0, U1 = J(src, nH)
    lE = torch.zeros_like(nH)
    le = torch.zeros_like(nH)
    ln = -1.0 / (N * nH)
    g_src = torch.zeros_like(nH)
    g_nH = torch.zeros_like(nH)
    s.adjoint_step(t0, dt, nH, src, U0, U1, (lE, le, ln), g_src, g_nH)
    g_nH_total = g_nH + U1[2] / (N * nH * nH)      # J's own dependence on n_H
    gen = torch.Generator(device="cpu").manual_seed(11)
    # one-signed directions (0.5..1.5 of each value): the change of J does not cancel
    u_src = (0.5 + torch.rand(op.dims, generator=gen, dtype=torch.float64)).to(hip_device)
    u_nH = (0.5 + torch.rand(op.dims, generator=gen, dtype=torch.float64)).to(hip_device)
    # step sizes: 1% of the sources; for n_H below the initial ionised
    # fraction (1.2e-3), so that n_HI^n <= n_H stays true
    results = {}
    for name, base, u, g, h in (("src", src, u_src, g_src, 1e-2),
                                ("nH", nH, u_nH, g_nH_total, 5e-4)):
        delta = base * u
        Jp = J(src + h * delta, nH)[0] if name == "src" else J(src, nH + h * delta)[0]
        Jm = J(src - h * delta, nH)[0] if name == "src" else J(src, nH - h * delta)[0]
        fd = (Jp - Jm) / (2.0 * h)
        adj = float((g * delta).sum().item())
        results[name] = (adj, fd, abs(adj - fd) / abs(fd))
    s.close()
    print("J", J0, "directional derivatives (adjoint, finite difference, rel)", results)
    for name, (adj, fd, rel) in results.items():
        assert rel < 1e-5, (name, adj, fd, rel)


def test_adjoint_per_cell_finite_differences_256(hip_device):
    """The 256^3 lognormal volume's adjoint check as the workload states it,
    on a subset: per-cell finite differences (relative steps 1e-6 for src,
    1e-3 for n_H; see tests/fd_cells.py) of J = mean x_HII with respect to
    src and n_H of 4 of the 64 seeded cells, after 3 mixed forward steps (the
    full check runs all 64 cells over 10 steps), to 1e-4."""
    from fd_cells import run
    res = run(n_cells=4, nsteps=3, dev=hip_device, log=lambda *a: print(*a, flush=True))
    assert len(res) == 8
    for c, name, kind, adj, fd, rel in res:
        assert rel < 1e-4, (c, name, kind, adj, fd, rel)
