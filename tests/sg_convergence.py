"""Shapiro-Giroux verification study (needs an MI355X; prints a table).

For each of the four rows of the verification section's cosmology table,
advance the GPU solver (rh_advance: theta = 0.51, tau_tol = 1e-3) from z0 to
z = 0 and compare the I-front radius with the analytic solution of the
section's equations SG-solution / SG-tau / SG-F.  The analytic r_I is the
comoving front radius in units of the proper Stromgren radius at z0, i.e.
r_I,comoving * a0 / r_S0.  Usage: python tests/sg_convergence.py 16 32 64 128
"""
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import analytic as OA  # noqa: E402
from oracle import diagnostics as OD  # noqa: E402

ALPHA_B = 2.59e-13
NDOT = 5e48
H100 = 3.2407789e-18
OUTPUTS = (1.1, 1.5, 2.0, 3.0, 5.0, 11.0)


def run_row(row, n, dev="cuda:0", tau=1e-3, outputs=OUTPUTS, log=None):
    """[(a/a0, r_I/r_S0 measured, analytic, relative error, steps)]."""
    import paper_0908_2654_amd as P
    from paper_0908_2654_amd.inputs import device_inputs
    w = W.shapiro_giroux(row, (n, n, n))
    q0, z0 = w.extra["q0"], w.extra["z0"]
    prm = P.params_from_workload(w)
    s = P.Solver(prm, device=dev)
    inp = device_inputs(w, s)
    E, e, nn = inp["E"], inp["e"], inp["nHI"]
    a0 = 1.0 / (1.0 + z0)
    nH0 = w.nH_mean / a0 ** 3                       # proper density at z0
    lam = ALPHA_B * nH0 / (w.hubble_h * H100) / (1.0 + z0)
    rS0 = (3.0 * NDOT / (4.0 * math.pi * ALPHA_B * nH0 ** 2)) ** (1.0 / 3.0)
    t = P.cosmic_time(prm, a0)
    dt, steps, out = 1e-3 * t, 0, []
    nH = inp["nH"].cpu().numpy()
    for A in outputs:
        if A > 1.0 + z0 + 1e-9:
            continue
        t1 = P.cosmic_time(prm, a0 * A)
        st = s.advance(t, t1, dt, tau, 1e30, inp["nH"], inp["src"], E, e, nn)
        steps, dt, t = steps + st["steps"], st["dt_next"], t1
        r_c = OD.front_radius(nn.cpu().numpy(), nH, 0.0, a0 * w.box_comoving_cm / n, corner=True)
        ra = OA.sg_front(A, lam, q0, z0)
        out.append((A, r_c / rS0, ra, r_c / rS0 / ra - 1.0, steps))
        if log:
            log(f"row {row} q0={q0:g} z0={z0:g} n={n}: a/a0={A:5.2f} r_I/r_S0={r_c / rS0:.4f} "
                f"analytic={ra:.4f} rel.err={r_c / rS0 / ra - 1.0:+.4f} steps={steps}")
    s.close()
    return out


if __name__ == "__main__":
    args = sys.argv[1:]
    taus = [1e-3]
    if "--tau" in args:
        i = args.index("--tau")
        taus = [float(v) for v in args[i + 1].split(",")]
        del args[i:i + 2]
    rows = range(4)
    if "--rows" in args:
        i = args.index("--rows")
        rows = [int(v) for v in args[i + 1].split(",")]
        del args[i:i + 2]
    for tau in taus:
        for n in [int(a) for a in args] or [32]:
            for row in rows:
                print(f"# tau_tol = {tau:g}", flush=True)
                run_row(row, n, tau=tau, log=lambda m: print(m, flush=True))
