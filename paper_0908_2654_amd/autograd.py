"""torch.autograd.Function over K implicit steps (checkpoint and adjoint).

RHRun.apply(src, nH, E0, e0, n0, solver, t0, dt, nsteps) -> (E, e, n) at
t0 + nsteps dt.  Forward runs rh_implicit_step K times and keeps the state
at every step (device checkpoints; 3 fields per step).  Backward runs
rh_adjoint_step from the last step to the first: each adjoint step solves
the transposed Newton system at the stored converged state (the same
symmetric Schur operator as the forward step, solved by the same
preconditioned multigrid) and returns dJ/dU^n plus the parameter
gradients dJ/dsrc and dJ/dn_H, accumulated over the steps.

Objectives, initial conditions and changes of variables (for example
n_H = rho / m_H, or n^0 = (1 - x0) n_H) are ordinary torch operations
around the function, so autograd composes them with the step adjoint.
"""
import torch


class RHRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, src, nH, E0, e0, n0, solver, t0, dt, nsteps):
        E, e, n = (x.detach().clone().contiguous() for x in (E0, e0, n0))
        src_d, nH_d = src.detach().contiguous(), nH.detach().contiguous()
        ckpt = [(E.clone(), e.clone(), n.clone())]
        stats = []
        for s in range(int(nsteps)):
            stats.append(solver.step(t0 + s * dt, dt, nH_d, src_d, E, e, n))
            ckpt.append((E.clone(), e.clone(), n.clone()))
        ctx.solver, ctx.t0, ctx.dt, ctx.nsteps = solver, t0, dt, int(nsteps)
        ctx.ckpt = ckpt
        ctx.src, ctx.nH = src_d, nH_d
        ctx.forward_stats = stats
        return E, e, n

    @staticmethod
    def backward(ctx, gE, ge, gn):
        ref = ctx.ckpt[-1][0]
        lE = torch.zeros_like(ref) if gE is None else gE.detach().clone().contiguous()
        le = torch.zeros_like(ref) if ge is None else ge.detach().clone().contiguous()
        ln = torch.zeros_like(ref) if gn is None else gn.detach().clone().contiguous()
        g_src = torch.zeros_like(ref)
        g_nH = torch.zeros_like(ref)
        ctx.adjoint_stats = []
        for s in reversed(range(ctx.nsteps)):
            st = ctx.solver.adjoint_step(ctx.t0 + s * ctx.dt, ctx.dt, ctx.nH, ctx.src,
                                         ctx.ckpt[s], ctx.ckpt[s + 1], (lE, le, ln),
                                         g_src, g_nH)
            ctx.adjoint_stats.append(st)
        iso = bool(ctx.solver.params.isothermal)
        return (g_src, g_nH, lE, None if iso else le, ln, None, None, None, None)
