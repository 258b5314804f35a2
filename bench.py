#!/usr/bin/env python3
"""Benchmark of the coupled implicit radiation step on one MI355X.

Metric: Mcell-updates/s per converged implicit step (||f|| <= 1e-8 in the
RMS norm), FP32-multigrid + FP64-refinement path, with the plain FP64 path
timed on the same states beside it.  A step is one rh_implicit_step over the
whole grid (face limiter, Newton iterations with local solves, residuals,
Schur operator, preconditioned multigrid solves, line search).

Default workload: the 512^3 reionisation-style volume (flat LCDM, z = 9 -> 7
in 50 steps, lognormal density sigma_ln = 1.5, 4096 lognormal sources).
Inputs are seeded synthetic fields and are resident in HBM before timing.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per fine cell of one launch of each kernel class
# (every input field read once, every output written once; halo re-reads
# and cache effects count zero).  T = 4 (mixed) or 8 (FP64) bytes per
# multigrid value.  A level's operator per cell: FP32 levels one 8-byte
# record (three faces and the shift in bfloat16), FP64 levels the diagonal
# and three face arrays (4 T).
def operator_bytes(T):
    return 8 if T == 4 else 4 * T


def algorithmic_bytes_per_cell(kind, T, iso=False):
    O = operator_bytes(T)
    return {
        # one full red-black sweep in one launch: x, b and the operator
        # read, the new x written
        "rbgs_fine": 3 * T + O,
        # one colour of a sweep: other-colour x, own b, the operator (FP32:
        # every record, for the own shift and + faces and the neighbours' -
        # faces; FP64: own diagonal, all three face arrays), own x written
        "rbgs_fine_colour": 1.5 * T + (O if T == 4 else 0.5 * T + 3 * T),
        # the V-cycle's last sweep, which also reads r and q for z.r, z.q
        "rbgs_fine_dots": 3 * T + O + 2 * 8,
        # residual fused with the restriction (x, b, operator in; coarse
        # right-hand side out), as the benchmark sizes run it
        "mg_residual_fine": 2 * T + O + T / 8,
        "restrict_fine": T + T / 8,
        "prolong_fine": T / 8 + 2 * T,
        # zT, p, x, diag, 3 cf in; p, q, x out (x += alpha p of the previous
        # iteration is folded into the direction kernel)
        "pcg_direction": T + 6 * 8 + 3 * 8,
        "pcg_update": 3 * 8 + T,            # r, q in; r, b out
        "pcg_precond": T + 2 * 8,           # zT, r, q in (dot products only)
        # ... and, mixed, the FP32 finest level's shift (bfloat16)
        "residual_schur": 8 * 8 + 2 * 8 + (2 if T == 4 else 0),
        "local_solve": (12 if not iso else 8) * 8 + (7 if not iso else 4) * 8,
        # ... and, mixed, the FP32 finest level's three faces (bfloat16)
        "step_setup": 3 * 8 + 3 * 8 + (3 * 2 if T == 4 else 0) + 8,
    }.get(kind)


def linear_iteration_bytes(T):
    """Algorithmic bytes per fine cell of one preconditioned CG iteration:
    the V(2,2) cycle on the finest level (three plain fused sweeps, the last
    sweep with the CG dot products, the fused residual + restriction and
    the prolongation), the levels below it (the same work on N/8 + N/64 +
    ... = N/7 cells, no dot products), the direction kernel (S p and the
    folded x update) and the update kernel."""
    b = algorithmic_bytes_per_cell
    fine = 3 * b("rbgs_fine", T) + b("rbgs_fine_dots", T) + b("mg_residual_fine", T) \
        + b("prolong_fine", T)
    coarse = (4 * b("rbgs_fine", T) + b("mg_residual_fine", T) + b("prolong_fine", T)) / 7.0
    return fine + coarse + b("pcg_direction", T) + b("pcg_update", T)


def step_bytes_per_cell(st, T, iso=False):
    """Algorithmic bytes per cell of one implicit step from its statistics:
    U^n copied in and the result copied out (3 fields each way), the face
    limiter, one local solve + residual per evaluation (the start, one trial
    per Newton iteration and one per line-search cut), the coarse-level
    operators per Newton iteration (on N/7 cells: fine shifts or diagonals
    in, coarse ones out; a bfloat16 shift on FP32 levels) and every linear
    iteration."""
    b = algorithmic_bytes_per_cell
    evals = 1 + st["newton_its"] + st["ls_cuts"]
    copies = 2 * 3 * 2 * 8
    S = 2 if T == 4 else T
    return (copies + b("step_setup", T) + evals * (b("local_solve", T, iso) + b("residual_schur", T))
            + st["newton_its"] * (3 * S / 7.0) + st["lin_its_total"] * linear_iteration_bytes(T))


def host_description():
    """CPU of the host: logical CPUs, model name and the BLAS thread pools."""
    import platform
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": i.get("internal_api"), "threads": i.get("num_threads")}
                for i in threadpool_info()]
    except Exception:  # threadpoolctl missing
        blas = None
    return {"os_cpu_count": os.cpu_count(), "model": model, "blas_pools": blas}


def measured_traffic(kind, workload):
    """HBM bytes per launch of `kind` from the committed counter record, or
    None when there is none or the kernels have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kind}_{workload.split('_')[0]}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    from paper_0908_2654_amd.profile_summary import kernels_sha256
    if rec.get("class") != kind or rec.get("kernels_source_sha256") != kernels_sha256():
        return None
    return float(rec["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


MG = {}


def run_path(P, w, prec, inp, state, t_start, dt, steps, timing, adjoint=False):
    """Time `steps` implicit steps; with adjoint=True also keep per-step
    checkpoints (outside the timed region) and time the adjoint steps of
    J = mean x_HII over the same steps, in reverse."""
    import torch
    prm = P.params_from_workload(w, precision=prec, **MG)
    s = P.Solver(prm, device=inp["nH"].device)
    E, e, n = (x.clone() for x in state)
    if timing:
        s.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    ckpt = [(E.clone(), e.clone(), n.clone())] if adjoint else None
    t_ck = 0.0
    for k in range(steps):
        stats.append(s.step(t_start + k * dt, dt, inp["nH"], inp["src"], E, e, n))
        if adjoint:
            torch.cuda.synchronize()
            tc = time.perf_counter()
            ckpt.append((E.clone(), e.clone(), n.clone()))
            torch.cuda.synchronize()
            t_ck += time.perf_counter() - tc
        log(f"  prec={prec} step {k}: newton={stats[-1]['newton_its']} "
            f"vcycles={stats[-1]['lin_its_total']} (max {stats[-1]['lin_its_max']}/solve, "
            f"caps {stats[-1]['lin_cap_hits']}, lin_res {stats[-1]['lin_res_max']:.1e}) "
            f"res={stats[-1]['res_final']:.2e} gpu_ms={stats[-1]['t_ms'][0]:.1f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0 - t_ck
    kt = s.kernel_timing() if timing else None
    if timing:
        s.set_kernel_timing(False)
    adj = None
    if adjoint:
        N = w.ncells
        lE = torch.zeros_like(E)
        le = torch.zeros_like(E)
        ln = -1.0 / (N * inp["nH"])
        g_src = torch.zeros_like(E)
        g_nH = torch.zeros_like(E)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ast = []
        for k in reversed(range(steps)):
            ast.append(s.adjoint_step(t_start + k * dt, dt, inp["nH"], inp["src"], ckpt[k],
                                      ckpt[k + 1], (lE, le, ln), g_src, g_nH))
        torch.cuda.synchronize()
        wa = time.perf_counter() - ta
        adj = {"ms_per_step": round(1e3 * wa / steps, 2),
               "ratio_to_forward": round(wa / wall, 3),
               "vcycles": [a["lin_its_total"] for a in ast],
               "lin_res_max": max(a["lin_res_max"] for a in ast),
               "lin_target": 1e-13,
               "objective": "mean x_HII after the timed steps; gradients wrt src and n_H",
               "finite": bool(torch.isfinite(g_src).all().item() and torch.isfinite(g_nH).all().item())}
        log(f"  adjoint: {adj['ms_per_step']} ms/step, ratio {adj['ratio_to_forward']}")
        del ckpt
    s.close()
    del s
    torch.cuda.empty_cache()
    return wall, stats, kt, (E, e, n), adj


ADV_V_RMS = 1.0e7   # cm/s per component: 100 km/s peculiar velocities
ADV_SEED = 101


def run_advection(P, w, inp, state, t, dt, reps=3):
    """The operator split's advection step (rh_advect) on the same fields
    with a seeded 100 km/s random velocity over the same dt: wall time of
    whole calls, and the substep kernel's average launch time from the
    library's events for its roofline (algorithmic bytes: n_H, E, n_HI, e and
    three velocities read, four fields written)."""
    import torch

    import workloads as W
    dev = inp["nH"].device
    v = [torch.from_numpy(c).to(dev) for c in W.velocity_field(w.dims, ADV_V_RMS, seed=ADV_SEED)]
    s = P.Solver(P.params_from_workload(w, precision=1), device=dev)
    f = [inp["nH"].clone()] + [x.clone() for x in state]
    nH, E, e, n = f
    st = s.advect(t, dt, v, nH, E, e, n)        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st = s.advect(t, dt, v, nH, E, e, n)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    s.set_kernel_timing(True)
    s.advect(t, dt, v, nH, E, e, n)
    kt = s.kernel_timing()
    s.set_kernel_timing(False)
    s.close()
    del v, f
    N = w.ncells
    ms_sub, cnt = kt["advect"][0] / kt["advect"][1], kt["advect"][1]
    bpc = 72 if w.isothermal else 88
    achieved = bpc * N / (ms_sub * 1e-3) / 1e9
    traffic = measured_traffic("advect", w.name)
    return {"ms_per_call": round(1e3 * wall, 3), "substeps": st["substeps"],
            "courant": round(st["courant"], 4),
            "Mcell_substeps_per_s": round(N * st["substeps"] / wall / 1e6, 1),
            "v_rms_km_s": ADV_V_RMS / 1e5,
            "courant_ms": round(kt["advect_courant"][0], 4),
            "roofline": {"bound": "hbm", "kernel": "advect", "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": None if traffic is None else round(traffic / 1e9, 3),
                         "traffic_bytes_per_cell": None if traffic is None else round(traffic / N, 2),
                         "bytes_per_cell": bpc, "avg_launch_ms": round(ms_sub, 4),
                         "launches": cnt}}


def cpu_baseline(w, nH_full, state, t, dt, sub=64):
    """The oracle, as it stands, on a bounded sample: one implicit step of a
    sub^3 block cut from a checkpoint of the timed window (the GPU state at
    the start of the first timed step: same cells, density, sources, fields,
    time and step), closed as a periodic box; BLAS limited to one thread,
    which is what NumPy's elementwise work and SciPy's sparse solvers use.
    A sample that is the whole grid keeps the workload's walls."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import model as OM, newton as ON
    ws = W.get(w)
    ws.dims = (sub, sub, sub)
    ws.box_comoving_cm = w.box_comoving_cm * sub / w.dims[0]
    if tuple(w.dims) != (sub, sub, sub):
        ws.bc = (W.BC_PERIODIC,) * 6
    cut = (slice(0, sub),) * 3
    nH = np.ascontiguousarray(nH_full[cut])
    Q = np.ascontiguousarray(W.photon_rate_field(w)[cut])
    E, e, n = (np.ascontiguousarray(x[cut].cpu().numpy()) for x in state)
    # the limiter floor of the whole box, R_min = 1 / (a_n L_box)
    a_n = OM.params_from_workload(w).cosmo.a(t)
    op = OM.params_from_workload(ws, newton_tol=1e-8, R_min=1.0 / (a_n * w.box_comoving_cm))
    src = OM.source_field(op, Q)
    st = {}
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        ON.step(op, t, dt, nH, src, E, e, n, stats=st)
        el = time.perf_counter() - t1
    return {
        "value": sub ** 3 / el / 1e6,
        "unit": "Mcell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one implicit step (Newton to ||f|| <= 1e-8, {st['newton_its']} iterations) of a "
                  f"{sub}^3 block of the GPU state at the start of the first timed step (same "
                  f"density, sources, fields, t and dt; "
                  + ("the whole grid" if tuple(w.dims) == (sub, sub, sub)
                     else "the block closed periodically")
                  + f"), {el:.1f} s on one thread (BLAS limited to 1)",
        "host": host_description(),
    }


MG_EDGES_EV = (13.6, 24.587, 54.4)   # groups split at the HeI and HeII thresholds
MG_Y_HE = 0.08                        # n_He / n_H (primordial helium by number)


def cpu_baseline_multigroup(w, nH_full, Q_full, state, t, dt, sub=8):
    """The multigroup oracle on a bounded sample: one step of a sub^3 block
    cut from the GPU state at the start of the first timed step (closed
    periodically, R_min of the whole box), one BLAS thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import model as OM, multigroup as OMG
    ws = W.get(w)
    ws.dims = (sub, sub, sub)
    ws.box_comoving_cm = w.box_comoving_cm * sub / w.dims[0]
    ws.bc = (W.BC_PERIODIC,) * 6
    cut = (slice(0, sub),) * 3
    a_n = OM.params_from_workload(w).cosmo.a(t)
    mp = OMG.params_from_workload(ws, MG_EDGES_EV, MG_Y_HE, newton_tol=1e-8,
                                  R_min=1.0 / (a_n * w.box_comoving_cm))
    nH = np.ascontiguousarray(nH_full[cut])
    src = OM.source_field(mp.base, np.ascontiguousarray(Q_full[cut]))
    E, e, y = state
    E = np.ascontiguousarray(E.cpu().numpy()[(slice(None),) + cut])
    e = np.ascontiguousarray(e.cpu().numpy()[cut])
    y = np.ascontiguousarray(y.cpu().numpy()[(slice(None),) + cut])
    st = {}
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        OMG.step(mp, t, dt, nH, src, E, e, y, stats=st)
        el = time.perf_counter() - t1
    return {"value": sub ** 3 / el / 1e6, "unit": "Mcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one multigroup step (Newton to ||f|| <= 1e-8, {st['newton_its']} "
                      f"iterations, sparse direct solves) of a {sub}^3 block of the GPU state at "
                      f"the start of the first timed step, {el:.1f} s on one thread",
            "host": host_description()}


def run_multigroup(args, dev):
    """Time the hydrogen + helium multigroup step (rh_multigroup_step) on the
    configured workload: three groups split at the helium thresholds,
    n_He / n_H = 0.08, mixed precision, Newton to 1e-8 with forcing 1e-13."""
    import numpy as np
    import torch

    import paper_0908_2654_amd as P
    import workloads as W
    from paper_0908_2654_amd.inputs import schedule
    w = W.get(args.config)
    prm = P.params_from_workload(w, precision=1, **MG)
    mgp = P.multigroup_params(MG_EDGES_EV, MG_Y_HE)
    log(f"multigroup workload {w.name} dims={w.dims}: generating inputs")
    nH_host = W.density_field(w)
    Q_host = W.photon_rate_field(w)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)  # noqa: E731
    nH = to(nH_host)
    src = torch.empty_like(nH)
    g = P.Solver(prm, device=dev)          # the source field uses the grey mean photon energy
    g.source_field(to(Q_host), src)
    g.close()
    del g
    s = P.MultigroupSolver(prm, mgp, device=dev)
    E, e, y = s.empty_state()
    s.initial_state(nH, w.x0, w.T0, w.E0, E, e, y)
    t0, dt, nsteps = schedule(w, prm)
    for k in range(args.warmup):
        st = s.step(t0 + k * dt, dt, nH, src, E, e, y)
        log(f"  warmup step {k}: newton={st['newton_its']} its={st['lin_its_total']} "
            f"sweeps<={st['lin_its_max']}")
    t_start = t0 + args.warmup * dt
    state0 = (E.clone(), e.clone(), y.clone())
    torch.cuda.synchronize()
    tw = time.perf_counter()
    stats = []
    for k in range(args.steps):
        stats.append(s.step(t_start + k * dt, dt, nH, src, E, e, y))
        x = stats[-1]
        log(f"  step {k}: newton={x['newton_its']} multigrid its={x['lin_its_total']} "
            f"sweeps<={x['lin_its_max']} caps={x['lin_cap_hits']} res={x['res_final']:.2e} "
            f"gpu_ms={x['t_ms'][0]:.1f}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw
    # per-kernel times: the first timed step again, with an event pair per launch
    E1, e1, y1 = (x.clone() for x in state0)
    s.set_kernel_timing(True)
    s.kernel_timing(reset=True)
    s.step(t_start, dt, nH, src, E1, e1, y1)
    kt = s.kernel_timing()
    s.set_kernel_timing(False)
    s.close()
    N = w.ncells
    value = N * args.steps / wall / 1e6
    # roofline of the dominant multigrid / CG kernel class: each launch covers
    # one group's N cells with the grey step's bytes (the multigroup-only
    # classes and the residual, which reads the helium fields too, have no
    # byte model here and are listed in kernels_ms only)
    best = None
    for kind in ("rbgs_fine", "rbgs_fine_colour", "rbgs_fine_dots", "mg_residual_fine",
                 "restrict_fine", "prolong_fine", "pcg_direction", "pcg_update", "pcg_precond"):
        ms, cnt = kt[kind]
        if cnt and (best is None or ms > best[1]):
            best = (kind, ms, cnt, algorithmic_bytes_per_cell(kind, 4))
    roof = None
    if best is not None:
        kind, ms, cnt, bpc = best
        avg_ms = ms / cnt
        achieved = bpc * N / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": kind, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "bytes_per_cell": bpc, "avg_launch_ms": round(avg_ms, 4),
                "launches": cnt}
    kernels = {k: {"ms_total": round(v[0], 2), "launches": v[1]} for k, v in kt.items() if v[1]}
    kernels["note"] = "first timed step, rerun with an event pair around every launch"
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (multigroup oracle on a bounded sample)")
        cpu = cpu_baseline_multigroup(w, nH_host, Q_host, state0, t_start, dt)
        log(f"cpu baseline: {cpu['value']:.5f} Mcell-updates/s")
    return {
        "metric": "Mcell-updates/s per multigroup implicit step (3 groups, H + He) at 1e-8 residual",
        "value": round(value, 2), "unit": "Mcell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 multigrid / f64 refinement", "data": "synthetic",
        "config": {"workload": w.name + "_3groups_he", "grid": list(w.dims),
                   "sources": w.n_sources, "group_edges_eV": list(MG_EDGES_EV), "y_he": MG_Y_HE,
                   "newton_tol": 1e-8, "lin_forcing": 1e-13,
                   "linear": "FGMRES(8) preconditioned by one block Gauss-Seidel sweep over the "
                             "groups, each group by PCG + V(2,2)"},
        "per_step": {"newton_its": [x["newton_its"] for x in stats],
                     "multigrid_its": [x["lin_its_total"] for x in stats],
                     "sweeps_max": [x["lin_its_max"] for x in stats],
                     "lin_res_max": [float(f"{x['lin_res_max']:.3g}") for x in stats],
                     "lin_cap_hits": [x["lin_cap_hits"] for x in stats],
                     "gpu_ms": [round(x["t_ms"][0], 1) for x in stats]},
        "roofline": roof,
        "kernels_ms": kernels,
        "cpu_baseline": cpu,
    }


def copy_bandwidth(dev, reps=5):
    """GB/s of a plain 1 GiB device-to-device copy (bytes read + written per
    second): the practical HBM ceiling of the box, for context."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-advection", action="store_true",
                    help="skip the operator split's advection step (rh_advect)")
    ap.add_argument("--mg-pre", type=int, default=2)
    ap.add_argument("--mg-post", type=int, default=2)
    ap.add_argument("--smoother", type=int, default=0,
                    help="0 auto, 1 one launch per colour, 2 fused sweep wherever it fits")
    ap.add_argument("--block-radius", type=int, default=2,
                    help="box radius of the block smoother around sources (0 off)")
    ap.add_argument("--block-levels", type=int, default=2,
                    help="multigrid levels with source boxes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for HBM counter scaling)")
    ap.add_argument("--multigroup", action="store_true",
                    help="time the hydrogen + helium multigroup step instead (its own line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the step has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_0908_2654_amd as P
    import workloads as W
    from paper_0908_2654_amd.inputs import device_inputs, schedule

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        # a plain copy of 2^28 float32 (1 GiB read, 1 GiB written), 3 times
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 << 28, "launches": 3}))
        return
    MG.update(mg_pre=args.mg_pre, mg_post=args.mg_post, smoother=args.smoother,
              mg_block_radius=args.block_radius, mg_block_levels=args.block_levels)
    if args.multigroup:
        print(json.dumps(run_multigroup(args, dev)), flush=True)
        return
    w = W.get(args.config)
    log(f"workload {w.name} dims={w.dims}: generating inputs")
    tg = time.perf_counter()
    nH_host = W.density_field(w)
    prm = P.params_from_workload(w, precision=1, **MG)
    s0 = P.Solver(prm, device=dev)
    inp = device_inputs(w, s0, nH_host=nH_host)
    t0, dt, nsteps = schedule(w, prm)
    log(f"inputs ready in {time.perf_counter() - tg:.1f} s; dt = {dt:.4e} s")
    copy_gbs = copy_bandwidth(dev)
    log(f"plain device copy: {copy_gbs:.0f} GB/s")
    state = [inp["E"], inp["e"], inp["nHI"]]
    for k in range(args.warmup):
        st = s0.step(t0 + k * dt, dt, inp["nH"], inp["src"], *state)
        log(f"  warmup step {k}: newton={st['newton_its']} vcycles={st['lin_its_total']}")
    torch.cuda.synchronize()
    s0.close()
    del s0
    torch.cuda.empty_cache()
    t_start = t0 + args.warmup * dt
    N = w.ncells

    # headline: the timed steps without per-kernel events
    wall_m, st_m, _, out_m, adj = run_path(P, w, 1, inp, state, t_start, dt, args.steps, False,
                                           adjoint=not args.no_adjoint)
    ms_m = 1e3 * wall_m / args.steps
    value = N * args.steps / wall_m / 1e6
    log(f"mixed: {ms_m:.1f} ms/step, {value:.1f} Mcell-updates/s")
    # per-kernel times: the first timed step again, with an event pair per launch
    _, _, kt_m, _, _ = run_path(P, w, 1, inp, state, t_start, dt, 1, True)

    fp64 = None
    if not args.no_fp64:
        wall_d, st_d, _, out_d, _ = run_path(P, w, 0, inp, state, t_start, dt, args.steps, False)
        bytes_d = [step_bytes_per_cell(x, 8, w.isothermal) for x in st_d]
        fp64 = {"value": N * args.steps / wall_d / 1e6, "ms_per_step": 1e3 * wall_d / args.steps,
                "newton_its": [x["newton_its"] for x in st_d],
                "vcycles": [x["lin_its_total"] for x in st_d],
                "lin_res_max": max(x["lin_res_max"] for x in st_d),
                "lin_cap_hits": sum(x["lin_cap_hits"] for x in st_d),
                "step_hbm_frac": round(sum(bytes_d) * N / wall_d / 1e9 / HBM_PEAK_GBS, 4)}
        dE = (out_m[0] - out_d[0]).abs().max().item() / out_d[0].abs().max().item()
        dx = ((out_m[2] - out_d[2]).abs() / inp["nH"]).max().item()
        fp64["max_diff_vs_mixed"] = {"E_rel_to_max": dE, "x_HII_abs": dx}
        log(f"fp64: {fp64['ms_per_step']:.1f} ms/step, {fp64['value']:.1f} Mcell-updates/s")

    # roofline of the dominant kernel (largest total time over the timed steps)
    T = 4
    best = None
    for kind, (ms, cnt) in kt_m.items():
        b = algorithmic_bytes_per_cell(kind, T, w.isothermal)
        if b is None or cnt == 0:
            continue
        if best is None or ms > best[1]:
            best = (kind, ms, cnt, b)
    kind, ms, cnt, bpc = best
    avg_ms = ms / cnt
    achieved = bpc * N / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(kind, w.name)
    roof = {"bound": "hbm", "kernel": kind, "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
            "traffic": None if traffic is None else round(traffic / 1e9, 3),
            "traffic_unit": "GB per launch (HBM, FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_bytes_per_cell": None if traffic is None else round(traffic / N, 2),
            "bytes_per_cell": bpc, "avg_launch_ms": round(avg_ms, 4), "launches": cnt}
    kernels = {k: {"ms_total": round(v[0], 2), "launches": v[1]} for k, v in kt_m.items() if v[1]}
    kernels["note"] = "first timed step, rerun with an event pair around every launch"

    adv = None
    if not args.no_advection:
        adv = run_advection(P, w, inp, state, t_start, dt)
        adv["roofline"]["copy_GBs"] = round(copy_gbs, 1)
        adv["roofline"]["frac_of_copy"] = round(adv["roofline"]["achieved"] / copy_gbs, 4)
        log(f"advection: {adv['ms_per_call']:.2f} ms per call, {adv['substeps']} substeps, "
            f"{adv['roofline']['avg_launch_ms']:.3f} ms per substep "
            f"({adv['roofline']['achieved']:.0f} GB/s algorithmic)")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        cpu = cpu_baseline(w, nH_host, state, t_start, dt, sub=min(64, w.dims[0]))
        log(f"cpu baseline: {cpu['value']:.4f} Mcell-updates/s")

    # whole-step algorithmic bytes (from each step's own statistics) and the
    # step-level HBM fraction over the timed steps
    bytes_m = [step_bytes_per_cell(x, 4, w.isothermal) for x in st_m]
    step_hbm = sum(bytes_m) * N / wall_m / 1e9
    gpu_ms = sorted(x["t_ms"][0] for x in st_m)
    phases = [round(sum(x["t_ms"][q] for x in st_m) / len(st_m), 2) for q in range(1, 6)]

    line = {
        "metric": "Mcell-updates/s per implicit step at 1e-8 residual: FP32-MG+refine vs FP64",
        "value": round(value, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_m, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 multigrid / f64 refinement",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.dims), "sources": w.n_sources,
                   "steps_of_run": f"{args.warmup}..{args.warmup + args.steps - 1} of {nsteps}",
                   "newton_tol": 1e-8, "lin_forcing": 1e-13,
                   "outer": f"PCG, V({args.mg_pre},{args.mg_post}) preconditioner"
                            + (f", source boxes of radius {args.block_radius} on "
                               f"{args.block_levels} levels" if args.block_radius else ""),
                   "lin_max_it": 500},
        "per_step": {"newton_its": [x["newton_its"] for x in st_m],
                     "vcycles": [x["lin_its_total"] for x in st_m],
                     "vcycles_max_per_solve": [x["lin_its_max"] for x in st_m],
                     "lin_res_max": [float(f"{x['lin_res_max']:.3g}") for x in st_m],
                     "lin_cap_hits": [x["lin_cap_hits"] for x in st_m],
                     "res_final": [float(f"{x['res_final']:.3g}") for x in st_m],
                     "forcing_reached": all(x["lin_cap_hits"] == 0 and x["lin_res_max"] <= 1e-13
                                            for x in st_m),
                     "gpu_ms_median": round(gpu_ms[len(gpu_ms) // 2], 2),
                     "phase_ms_mean": dict(zip(["setup", "local_residual", "coarse_setup",
                                                "vcycles", "outer_linear"], phases)),
                     "step_bytes_per_cell": [round(b, 1) for b in bytes_m],
                     "step_hbm_GBs": round(step_hbm, 1),
                     "step_hbm_frac": round(step_hbm / HBM_PEAK_GBS, 4)},
        "fp64_path": fp64,
        "roofline": roof,
        "adjoint": adj,
        "kernels_ms": kernels,
        "advection": adv,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
