"""Pins for the oracle's time stepping (Algorithm "Nonstationary Linear Problem",
backward Euler with the lumped mass of eq. mass_lumping) and for the Sec. 5.1 data."""
import numpy as np
import pytest

import workloads as W
from oracle import fem, hierarchy as Hh, mesh as M, multigrid as MG, timestep as TS


def test_td_source_matches_finite_differences():
    """f = d_t theta - 0.01 lap theta + b . grad theta of the exact solution, formed by
    central differences (independent of the closed-form derivatives)."""
    rng = np.random.default_rng(1)
    th = W.td_exact
    for t, x, y in rng.uniform(0.0, 1.0, (20, 3)) * np.array([2.0, 1.0, 1.0]):
        d, d2 = 1e-5, 1e-4
        dt = (th(t + d, x, y) - th(t - d, x, y)) / (2 * d)
        dy = (th(t, x, y + d) - th(t, x, y - d)) / (2 * d)
        lap = (th(t, x + d2, y) + th(t, x - d2, y) + th(t, x, y + d2) + th(t, x, y - d2) - 4 * th(t, x, y)) / d2 ** 2
        assert W.td_source(t, x, y) == pytest.approx(dt - 0.01 * lap - dy, abs=1e-6)


def _run(wl, steps, exact, source, rtol=None):
    h = Hh.build(wl.with_(rtol=rtol) if rtol else wl)
    mgo = MG.Multigrid(h)
    ops = TS.operators(h)
    X = ops.coords
    theta0 = exact(0.0, X[:, 0], X[:, 1])
    F, G = [], []
    for k in range(1, steps + 1):
        f, g = TS.nodal_data(ops, wl, exact, source, k * wl.dt)
        F.append(f)
        G.append(g)
    return h, ops, TS.run(h, mgo, ops, theta0, F, G, wl.dt)


@pytest.mark.parametrize("adaptive", [False, True])
def test_linear_data_reproduced_exactly(adaptive):
    """theta = 0.3 + 0.5 x - 0.7 y is steady, linear (so in every Q1 space, hanging nodes
    included) and solves the problem with f = b . grad theta = 0.7: lumped mass, lifting of
    the Dirichlet data, H^T and the masks must all be right for the scheme to return it
    to solver accuracy."""
    wl = W.td_time(4)
    if adaptive:
        wl = wl.with_(coarse=(8, 8), h0=0.125, rounds=(("uniform",), ("band", 0.5, 0.5, 0.3, 0.05),
                                                       ("band", 0.5, 0.5, 0.3, 0.05)))
    lin = lambda t, x, y: 0.3 + 0.5 * x - 0.7 * y
    src = lambda t, x, y: 0.7 + 0.0 * x
    h, ops, res = _run(wl, 3, lin, src, rtol=1e-13)
    if adaptive:
        assert h.finest.mesh.is_hanging.any()
    X = ops.coords
    for r in res:
        assert np.abs(r.theta - lin(0, X[:, 0], X[:, 1])).max() < 1e-11


def test_first_order_in_time_against_the_exact_solution():
    """Sec. 5.1: the L2 error at T = 2 against theta_ex is below 1e-3 with dt = 0.02 and
    halves with dt (backward Euler is first order; the O(h^2) part is far smaller)."""
    errs = []
    for dt in (0.02, 0.01):
        wl = W.td_time(6, dt=dt)
        h, ops, res = _run(wl, int(round(2.0 / dt)), W.td_exact, W.td_source)
        errs.append(MG.l2_error(h, res[-1].theta, lambda p: W.td_exact(2.0, p[:, 0], p[:, 1])))
    assert errs[0] < 1e-3
    assert 0.45 < errs[1] / errs[0] < 0.55, errs


def test_rhs_operator_structure():
    """R = [Z H^T M_l | -Z H^T A E_g]: constrained rows of R are empty; the Q block of a
    uniform mesh is the lumped mass (h^2 inside, h^2 / 2 on edges) on free rows."""
    wl = W.td_time(3)
    h = Hh.build(wl)
    ops = TS.operators(h)
    N = h.finest.ndof
    rows = np.diff(ops.R.indptr)
    assert np.all(rows[ops.mask] == 0)
    Q = ops.R[:, :N].toarray()
    m = fem.lumped_mass(h.finest.mesh)
    assert np.allclose(np.diag(Q)[~ops.mask], m[~ops.mask], rtol=0, atol=1e-17)
    assert np.allclose(m[~ops.mask], (1 / 8) ** 2)
    assert ops.R.shape == (N, N + len(ops.g_idx))
