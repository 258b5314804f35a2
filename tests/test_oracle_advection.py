"""Pins of the oracle's advection step (oracle/advection.py) against results
it does not compute itself: exact translation at Courant number 1, the
binomial closed form of repeated donor-cell steps, conservation, preserved
uniform ratios, the neighbour-range bound, uniform flow through outflow
walls, and the comoving displacement int v / a dt in an expanding universe."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import advection as A
from oracle import model as M
from oracle.cosmology import Cosmology, STATIC, EDS

P_, Z_, O_ = M.PERIODIC, M.ZEROFLUX, M.OUTFLOW


def _params(dims, bc, box=None, cosmo=None, iso=False):
    return M.Params(dims=tuple(dims), box=float(dims[0]) if box is None else box, bc=tuple(bc),
                    isothermal=iso, T_iso=1e4, grey={}, rates=0, alphaB_const=2.59e-13,
                    cooling=0, cosmo=cosmo or Cosmology(STATIC))


def _fields(rng, dims):
    nH = 1e-3 * (0.5 + rng.random(dims))
    E = 1e-14 * rng.random(dims)
    n = nH * rng.random(dims)
    e = 1e12 * (0.5 + rng.random(dims))
    return nH, E, e, n


def _uniform_v(dims, d, V):
    v = [np.zeros(dims) for _ in range(3)]
    v[d][...] = V
    return v


@pytest.mark.parametrize("d,sign", [(0, 1), (1, -1), (2, 1)])
def test_translation_at_courant_one(d, sign):
    """u = 1 on every face moves every field by exactly one cell per substep
    (h = 1, v = 2, dt = 1.5: three substeps of u = 1 at cfl = 1)."""
    dims = (8, 6, 5)
    p = _params(dims, (P_,) * 6)
    rng = np.random.default_rng(1)
    nH, E, e, n = _fields(rng, dims)
    (nH1, E1, e1, n1), m = A.advect(p, 0.0, 1.5, _uniform_v(dims, d, 2.0 * sign), nH, E, e, n,
                                    cfl=1.0)
    assert m == 3
    for X0, X1 in ((nH, nH1), (E, E1), (e, e1), (n, n1)):
        np.testing.assert_allclose(X1, np.roll(X0, 3 * sign, axis=d), rtol=5e-14, atol=0)


def test_binomial_closed_form():
    """k donor-cell substeps at Courant number c in uniform flow: the field is
    sum_j C(k,j) c^j (1-c)^(k-j) times the field shifted by j cells."""
    dims = (5, 4, 12)
    p = _params(dims, (P_,) * 6)
    rng = np.random.default_rng(2)
    nH, E, e, n = _fields(rng, dims)
    c, k = 0.37, 7
    v = _uniform_v(dims, 2, -1.0)
    state = (nH, E, e, n)
    for _ in range(k):
        state, m = A.advect(p, 0.0, c, v, *state, cfl=1.0)
        assert m == 1
    for X0, X1 in ((E, state[1]), (nH, state[0]), (nH * e, state[0] * state[2])):
        ref = sum(math.comb(k, j) * c ** j * (1 - c) ** (k - j) * np.roll(X0, -j, axis=2)
                  for j in range(k + 1))
        np.testing.assert_allclose(X1, ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("bc", [(P_,) * 6, (Z_,) * 6, (Z_, Z_, P_, P_, Z_, Z_)])
def test_conservation(bc):
    """Periodic and closed walls: the sums of n_H, E, n_HI and n_H e do not
    change under a random compressive velocity field."""
    dims = (7, 9, 6)
    p = _params(dims, bc)
    rng = np.random.default_rng(3)
    nH, E, e, n = _fields(rng, dims)
    v = [rng.standard_normal(dims) for _ in range(3)]
    (nH1, E1, e1, n1), m = A.advect(p, 0.0, 2.0, v, nH, E, e, n, cfl=0.8)
    assert m > 1
    for X0, X1 in ((nH, nH1), (E, E1), (n, n1), (nH * e, nH1 * e1)):
        assert X1.sum() == pytest.approx(X0.sum(), rel=1e-13)
        assert X1.min() >= 0.0


@pytest.mark.parametrize("bc", [(P_,) * 6, (O_, O_, Z_, Z_, P_, P_)])
def test_uniform_ratios_preserved(bc):
    """e and the neutral fraction n_HI / n_H uniform stay uniform whatever the
    velocity and density fields: they move with the mass."""
    dims = (6, 7, 8)
    p = _params(dims, bc)
    rng = np.random.default_rng(4)
    nH = 1e-3 * (0.2 + rng.random(dims))
    v = [rng.standard_normal(dims) for _ in range(3)]
    e = np.full(dims, 3.3e12)
    n = 0.3 * nH
    (nH1, _, e1, n1), m = A.advect(p, 0.0, 1.0, v, nH, np.zeros(dims), e, n, cfl=0.9)
    assert np.abs(nH1 - nH).max() > 1e-5
    np.testing.assert_allclose(e1, 3.3e12, rtol=1e-14)
    np.testing.assert_allclose(n1 / nH1, 0.3, rtol=1e-14)


def test_neighbour_range_bound():
    """One substep at outgoing Courant number <= 1 makes each new e a convex
    combination of the old e of the cell and its six neighbours."""
    dims = (6, 6, 6)
    p = _params(dims, (P_,) * 6)
    rng = np.random.default_rng(5)
    nH, E, e, n = _fields(rng, dims)
    v = [rng.standard_normal(dims) for _ in range(3)]
    C = A.courant(p, v, 1.0)
    (_, _, e1, _), m = A.advect(p, 0.0, 1.0 / C, v, nH, E, e, n, cfl=1.0)
    assert m == 1
    lo, hi = e.copy(), e.copy()
    for d in range(3):
        for s in (1, -1):
            lo = np.minimum(lo, np.roll(e, s, axis=d))
            hi = np.maximum(hi, np.roll(e, s, axis=d))
    assert np.all(e1 >= lo * (1 - 1e-14)) and np.all(e1 <= hi * (1 + 1e-14))
    # and the range is really used: far from the cell's own value somewhere
    assert np.abs(e1 - e).max() > 0.05 * e.max()


def test_outflow_walls_keep_uniform_flow_uniform():
    """Uniform state in uniform flow through outflow walls: the inflow face
    brings in the boundary cell's own values, so nothing changes; closed
    walls instead pile the gas up against the downstream wall."""
    dims = (8, 4, 4)
    v = _uniform_v(dims, 0, 0.7)
    ones = np.ones(dims)
    p = _params(dims, (O_, O_, P_, P_, P_, P_))
    (nH1, E1, e1, n1), m = A.advect(p, 0.0, 3.0, v, 1e-3 * ones, 1e-14 * ones, 1e12 * ones,
                                    4e-4 * ones, cfl=0.9)
    assert m == 3
    for X1, val in ((nH1, 1e-3), (E1, 1e-14), (e1, 1e12), (n1, 4e-4)):
        np.testing.assert_allclose(X1, val, rtol=1e-14)
    pz = _params(dims, (Z_, Z_, P_, P_, P_, P_))
    (nHz, _, _, _), _ = A.advect(pz, 0.0, 3.0, v, 1e-3 * ones, ones, ones, ones, cfl=0.9)
    assert nHz[-1].min() > 1.5e-3 and nHz[0].max() < 0.5e-3
    assert nHz.sum() == pytest.approx(1e-3 * ones.sum(), rel=1e-14)


def test_centroid_moves_by_int_v_over_a_dt():
    """Uniform flow in an Einstein-de Sitter universe: a profile's centroid
    moves by exactly the sum of the substeps' Courant numbers, and that sum
    approximates int v / (a h) dt (from a = 0.1 to about 0.2) to the
    midpoint rule's second-order error."""
    dims = (256, 3, 3)
    cos = Cosmology(EDS, hubble_h=0.7, Omega_m=1.0)
    t0, t1 = cos.time_of_a(0.1), cos.time_of_a(0.2)
    box = 3.0e24
    p = _params(dims, (P_,) * 6, box=box, cosmo=cos)
    h = p.h
    x = np.arange(dims[0])[:, None, None] * np.ones(dims)
    E = np.exp(-0.5 * ((x - 40.0) / 4.0) ** 2)
    exact_cells = integrate.quad(lambda t: 1.0 / cos.a(t), t0, t1, epsabs=0, epsrel=1e-13)[0] / h
    V = 60.0 / exact_cells   # move ~60 cells
    v = _uniform_v(dims, 0, V)
    (_, E1, _, _), m = A.advect(p, t0, t1 - t0, v, np.ones(dims), E, np.ones(dims),
                                np.zeros(dims), cfl=0.9)
    ds = (t1 - t0) / m
    scheme = sum(ds * V / (cos.a(t0 + (s + 0.5) * ds) * h) for s in range(m))
    cen0 = (x * E).sum() / E.sum()
    cen1 = (x * E1).sum() / E1.sum()
    assert E1[-20:].max() < 1e-12 * E1.max()          # nothing wrapped round
    assert cen1 - cen0 == pytest.approx(scheme, rel=1e-11)
    assert scheme == pytest.approx(V * exact_cells, rel=2.0 / m ** 2)
    assert abs(scheme - V * exact_cells) > 0           # a really varies over the step


def test_isothermal_leaves_e_alone():
    dims = (5, 5, 5)
    p = _params(dims, (P_,) * 6, iso=True)
    rng = np.random.default_rng(6)
    nH, E, e, n = _fields(rng, dims)
    v = [rng.standard_normal(dims) for _ in range(3)]
    (nH1, E1, e1, n1), _ = A.advect(p, 0.0, 1.0, v, nH, E, e, n)
    assert e1 is None
    assert n1.sum() == pytest.approx(n.sum(), rel=1e-13)
