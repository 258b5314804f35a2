"""The C ABI's bookkeeping around the step: initial fields and emissivity
made by the library (against the oracle's definitions), the per-phase GPU
times of rh_step_stats, and how a linear solve that stops at lin_max_it is
reported (forward step: counted; adjoint step: RH_ELINEAR, outputs kept)."""
import numpy as np
import pytest

from gpu_cases import make_workload, oracle_inputs, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["stromgren16", "eds_cooling16", "lognormal_ragged"])
def test_initial_state_and_source_field_match_oracle(hip_device, case):
    import torch

    import paper_0908_2654_amd as P
    import workloads as W
    from oracle import model as OM
    w = make_workload(case)
    op, inp = oracle_inputs(w)
    s = P.Solver(P.params_from_workload(w), device=hip_device)
    nH = to_dev(inp["nH"], hip_device)
    E, e, n, src = (torch.empty_like(nH) for _ in range(4))
    s.initial_state(nH, w.x0, w.T0, w.E0, E, e, n)
    s.source_field(to_dev(W.photon_rate_field(w), hip_device), src)
    s.close()
    np.testing.assert_allclose(E.cpu().numpy(), inp["E"], rtol=0, atol=0)
    np.testing.assert_allclose(n.cpu().numpy(), inp["n"], rtol=1e-15)
    np.testing.assert_allclose(e.cpu().numpy(), inp["e"], rtol=1e-14)
    np.testing.assert_allclose(src.cpu().numpy(), inp["src"], rtol=1e-14)
    assert np.count_nonzero(inp["src"]) > 0


def test_initial_state_rejects_bad_inputs(hip_device):
    import torch

    import paper_0908_2654_amd as P
    from paper_0908_2654_amd._lib import RH_EINVAL, RH_ENONFINITE, RhError
    w = make_workload("lognormal_ragged")
    s = P.Solver(P.params_from_workload(w), device=hip_device)
    nH = torch.full(w.dims, 1e-3, dtype=torch.float64, device=hip_device)
    E, e, n = (torch.empty_like(nH) for _ in range(3))
    with pytest.raises(RhError) as ex:
        s.initial_state(nH, 1.0, 100.0, 1e-35, E, e, n)
    assert ex.value.status == RH_EINVAL
    with pytest.raises(RhError) as ex:
        s.initial_state(nH, 0.0, 100.0, 1e-35, E, None, n)   # e needed: not isothermal
    assert ex.value.status == RH_EINVAL
    nH[3, 4, 5] = 0.0
    with pytest.raises(RhError) as ex:
        s.initial_state(nH, 1.2e-3, 100.0, 1e-35, E, e, n)
    assert ex.value.status == RH_ENONFINITE
    rates = torch.zeros_like(nH)
    rates[1, 1, 1] = float("nan")
    with pytest.raises(RhError) as ex:
        s.source_field(rates, E)
    assert ex.value.status == RH_ENONFINITE
    s.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_phase_times_partition_the_step(hip_device, precision):
    """t_ms[1..5] (setup, local+residual, coarse setup, V-cycles, outer
    iteration) are contiguous event intervals: they sum to the whole step's
    t_ms[0] within 5%, and each phase that ran took time.  With the default
    linear cap every solve reaches its forcing."""
    import paper_0908_2654_amd as P
    w = make_workload("lognormal_ragged")
    op, inp = oracle_inputs(w)
    s = P.Solver(P.params_from_workload(w, precision=precision), device=hip_device)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    nH, src = d(inp["nH"]), d(inp["src"])
    E, e, n = d(inp["E"]), d(inp["e"]), d(inp["n"])
    for k in range(2):
        st = s.step(inp["t0"] + k * inp["dt"], inp["dt"], nH, src, E, e, n)
        t = st["t_ms"]
        print(precision, k, ["%.3f" % v for v in t[:6]], st["lin_its_total"], st["lin_its_max"],
              st["lin_res_max"], st["lin_cap_hits"])
        assert t[0] > 0
        assert sum(t[1:6]) == pytest.approx(t[0], rel=0.05)
        assert all(v > 0 for v in t[1:6])
        assert t[6] == 0 and t[7] == 0
        assert st["lin_cap_hits"] == 0
        assert st["lin_res_max"] <= s.params.lin_forcing
        assert 0 < st["lin_its_max"] <= st["lin_its_total"]
    s.close()


def test_linear_cap_is_counted_in_the_forward_step(hip_device):
    """A cap of 2 cycles stops every linear solve short of the 1e-13 forcing:
    Newton still converges on its own test (inexact directions), and the
    statistics count every capped solve."""
    import paper_0908_2654_amd as P
    w = make_workload("lognormal_ragged")
    op, inp = oracle_inputs(w)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    s = P.Solver(P.params_from_workload(w, precision=1, lin_max_it=2, newton_max_it=200),
                 device=hip_device)
    E, e, n = d(inp["E"]), d(inp["e"]), d(inp["n"])
    st = s.step(inp["t0"], inp["dt"], d(inp["nH"]), d(inp["src"]), E, e, n)
    s.close()
    print(st)
    assert st["res_final"] <= s.params.newton_tol
    assert st["lin_cap_hits"] == st["newton_its"] > 0
    assert st["lin_its_max"] == 2
    assert st["lin_res_max"] > s.params.lin_forcing


def test_adjoint_fails_loudly_at_the_linear_cap(hip_device):
    """The adjoint's transpose solve has no outer correction: stopped short of
    its target it returns RH_ELINEAR and leaves lambda and the gradients as
    they were."""
    import torch

    import paper_0908_2654_amd as P
    from paper_0908_2654_amd._lib import RH_ELINEAR, RhError
    w = make_workload("lognormal_ragged")
    op, inp = oracle_inputs(w)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    s = P.Solver(P.params_from_workload(w), device=hip_device)
    nH, src = d(inp["nH"]), d(inp["src"])
    U0 = tuple(d(inp[k]) for k in ("E", "e", "n"))
    U1 = tuple(x.clone() for x in U0)
    s.step(inp["t0"], inp["dt"], nH, src, *U1)
    s.close()
    s = P.Solver(P.params_from_workload(w, lin_max_it=2), device=hip_device)
    rng = np.random.default_rng(1)
    lam = tuple(d(rng.standard_normal(w.dims)) for _ in range(3))
    lam0 = tuple(x.clone() for x in lam)
    g_src = torch.full_like(nH, 3.0)
    g_nH = torch.full_like(nH, -2.0)
    with pytest.raises(RhError) as ex:
        s.adjoint_step(inp["t0"], inp["dt"], nH, src, U0, U1, lam, g_src, g_nH)
    s.close()
    assert ex.value.status == RH_ELINEAR
    assert "lin_max_it" in str(ex.value)
    for a, b in zip(lam, lam0):
        assert torch.equal(a, b)
    assert torch.all(g_src == 3.0) and torch.all(g_nH == -2.0)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", ["lognormal_mid", "stromgren16"])
def test_source_boxes_keep_the_solution_and_cut_cycles(hip_device, case, precision):
    """The block smoother around sources (mg_block_radius = 2 on two levels)
    changes only the preconditioner: the Schur solve reaches the same
    solution as without it (both to a 1e-13 relative residual) in no more
    cycles, and a step reports its boxes; repeated solves are bitwise
    identical (deterministic source list, box order and colouring)."""
    import paper_0908_2654_amd as P
    from gpu_cases import case_params
    from test_gpu_parity import _schur_problem
    w, op, inp, Un, U, t, dt, b, x_ref = _schur_problem(case)
    d = lambda a: to_dev(a, hip_device)  # noqa: E731
    args = (t, dt, d(inp["nH"]), d(inp["src"]), tuple(map(d, Un)), tuple(map(d, U)),
            d(b.reshape(op.dims)))
    res = {}
    for R in (0, 2):
        s = P.Solver(P.params_from_workload(w, precision=precision, mg_block_radius=R,
                                            **case_params(case)), device=hip_device)
        x, its, rr = s.schur_solve(*args, rel_tol=1e-13, max_it=500)
        x2, its2, _ = s.schur_solve(*args, rel_tol=1e-13, max_it=500)
        s.set_kernel_timing(True)
        E, e, n = (d(inp[k]) for k in ("E", "e", "n"))
        st = s.step(inp["t0"], inp["dt"], d(inp["nH"]), d(inp["src"]), E, e, n)
        kt = s.kernel_timing()
        s.close()
        assert rr < 1e-12 and its2 == its and bool((x == x2).all())
        res[R] = (x.cpu().numpy().ravel(), its, st["source_boxes"], kt)
        print(case, precision, "radius", R, "cycles", its, "boxes", st["source_boxes"],
              "block launches", kt["block_relax"][1], kt["block_inverse"][1])
    assert res[0][2] == 0 and res[2][2] > 0
    assert res[0][3]["block_relax"][1] == 0 and res[2][3]["block_relax"][1] > 0
    assert res[2][3]["block_inverse"][1] > 0
    assert res[2][1] <= res[0][1]
    err = np.linalg.norm(res[2][0] - res[0][0]) / np.linalg.norm(res[0][0])
    assert err < 1e-10
    assert np.linalg.norm(res[2][0] - x_ref) / np.linalg.norm(x_ref) < 1e-10
