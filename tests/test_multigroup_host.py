"""Host side of the multigroup entry points (no GPU): the library's group
constants against the oracle's quadrature of the same integrals, the
one-group limit against the grey constants, and parameter validation."""
import numpy as np
import pytest

import workloads as W
from oracle import model as OM, multigroup as MG

EDGES = (13.6, 24.587, 54.4)


def _params(cfg=2, **over):
    import paper_0908_2654_amd as P
    w = W.scaled(cfg, (16, 16, 16))
    for k, v in over.items():
        setattr(w, k, v)
    return w, P.params_from_workload(w)


@pytest.mark.parametrize("edges,power,T_bb", [
    (EDGES, 3.0, None), ((13.6, 20.0, 30.0, 60.0), 3.0, None), ((13.6, 54.4), 2.5, None),
    (EDGES, 0.0, None), ((13.6, 16.0), 3.0, 3.0e4)])
def test_group_constants_match_oracle_quadrature(edges, power, T_bb):
    import paper_0908_2654_amd as P
    over = {} if T_bb is None else {"T_bb": T_bb}
    w, p = _params(**over)
    c = P.multigroup_constants(p, P.multigroup_params(edges, 0.08, power))
    o = MG.group_constants(edges, w.T_bb, w.sigma0, edges[0], power)
    np.testing.assert_allclose(c["frac"], o["frac"], rtol=1e-13)
    # species without absorption in a group (threshold above it) are exactly 0 on both sides
    for key, okey, tol in (("sigma_E", "sigE", 1e-13), ("K_Gamma", "KGam", 1e-13),
                           ("K_G", "KG", 1e-11)):
        a, b = np.array(c[key]), np.array(o[okey])
        assert np.all((a == 0) == (b == 0)), key
        nz = b != 0
        np.testing.assert_allclose(a[nz], b[nz], rtol=tol, err_msg=key)
    assert c["eps_bar"] == pytest.approx(o["eps_bar"], rel=1e-13)


def test_one_group_constants_are_the_grey_constants():
    import paper_0908_2654_amd as P
    w, p = _params()
    op = OM.params_from_workload(w)
    c = P.multigroup_constants(p, P.multigroup_params((p.hnu0_eV,), 0.0))
    assert c["frac"] == [1.0]
    assert c["sigma_E"][0][0] == pytest.approx(op.grey["sigma_E"], rel=1e-13)
    assert c["K_Gamma"][0][0] == pytest.approx(op.grey["K_Gamma"], rel=1e-13)
    assert c["K_G"][0][0] == pytest.approx(op.grey["K_G"], rel=1e-11)
    assert c["eps_bar"] == pytest.approx(op.grey["eps_bar"], rel=1e-13)


@pytest.mark.parametrize("bad", ["mono", "edge0", "order", "groups0", "groups5", "yhe", "power",
                                 "reserved"])
def test_invalid_multigroup_parameters_are_rejected(bad):
    import ctypes

    import paper_0908_2654_amd as P
    from paper_0908_2654_amd import _lib
    w, p = _params()
    mg = P.multigroup_params(EDGES, 0.08)
    if bad == "mono":
        p.spectrum = 0
    elif bad == "edge0":
        mg.edge_eV[0] = 13.0
    elif bad == "order":
        mg.edge_eV[2] = 20.0
    elif bad == "groups0":
        mg.groups = 0
    elif bad == "groups5":
        mg.groups = 5
    elif bad == "yhe":
        mg.y_he = -0.1
    elif bad == "power":
        mg.sigma_power = float("nan")
    elif bad == "reserved":
        mg.reserved = 1
    assert _lib.lib.rh_multigroup_workspace_bytes(ctypes.byref(p), ctypes.byref(mg)) == 0
    with pytest.raises(_lib.RhError) as ex:
        P.multigroup_constants(p, mg)
    assert ex.value.status == _lib.RH_EINVAL
    assert _lib.lib.rh_multigroup_last_error(None)


def test_workspace_grows_with_the_groups():
    import ctypes

    import paper_0908_2654_amd as P
    from paper_0908_2654_amd import _lib
    w, p = _params()
    grey = P.workspace_bytes(p)
    sizes = []
    for G in (1, 2, 3, 4):
        mg = P.multigroup_params((13.6, 20.0, 30.0, 60.0)[:G], 0.08)
        sizes.append(_lib.lib.rh_multigroup_workspace_bytes(ctypes.byref(p), ctypes.byref(mg)))
    N = 16 ** 3
    for G, b in zip((1, 2, 3, 4), sizes):
        # one grey workspace per group plus G^2 + 29 G + 17 coupled fields (17 G
        # of them the Krylov bases) and 12 x 1024 Krylov partial sums
        fields = (G * G + 29 * G + 17) * 8 * N + 12 * 1024 * 8
        assert b >= G * grey + fields
        assert b <= G * (grey + 256) + fields + 18 * 256
