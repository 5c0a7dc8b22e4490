"""Pins for the oracle's smoother, V-cycle and outer iterations.

* brute force: the dense error-propagation matrix of the V-cycle, built recursively from
  dense matrices, predicts the iterated oracle V-cycle;
* brute force: (F)GMRES iterates equal the minimal-residual point of the Krylov space;
* closed form: manufactured solution u = sin(pi x) sin(pi y) gives O(h^2) L2 error;
* library routine: MG / FGMRES solutions agree with a sparse direct solve;
* textbook analysis: h-independent V(2,2) rate below 0.1 for 2D Q1 Poisson (the paper
  states that the iteration counts hardly vary with the mesh level, Sec. 5.1).
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import hierarchy as Hh, multigrid as MG


def _dense_propagator(hier, mg):
    L = hier.L
    E = [None] * (L + 1)
    A0 = hier.levels[0].A.toarray()
    n0 = A0.shape[0]
    if mg.coarse_mode == W.COARSE_EXACT:
        E[0] = np.zeros((n0, n0))
    else:
        S0 = _dense_S(mg, 0, n0)
        E[0] = np.linalg.matrix_power(np.eye(n0) - mg.omega * S0 @ A0, mg.coarse_sweeps)
    for l in range(1, L + 1):
        lv = hier.levels[l]
        A = lv.A.toarray()
        n = A.shape[0]
        Sm = np.eye(n) - mg.omega * _dense_S(mg, l, n) @ A
        Ac = hier.levels[l - 1].A.toarray()
        Binv = (np.eye(Ac.shape[0]) - E[l - 1]) @ np.linalg.inv(Ac)
        C = np.eye(n) - lv.P.toarray() @ Binv @ lv.R.toarray() @ A
        E[l] = np.linalg.matrix_power(Sm, mg.nu2) @ C @ np.linalg.matrix_power(Sm, mg.nu1)
    return E[L]


def _dense_S(mg, l, n):
    S = mg.S[l]
    b = S.shape[1]
    out = np.zeros((n, n))
    for i in range(S.shape[0]):
        out[i * b:(i + 1) * b, i * b:(i + 1) * b] = S[i]
    return out


@pytest.mark.parametrize("wl,kw", [
    (W.c1_poisson(2), {}),
    (W.c2_td(band_rounds=2, uniform_rounds=0, delta=0.05), {}),
    (W.c3_elasticity(1), {"nu1": 1, "nu2": 3}),
    (W.c4_oseen(1), {"coarse_mode": W.COARSE_SMOOTH, "coarse_sweeps": 5}),
])
def test_vcycle_matches_dense_propagator(wl, kw):
    h = Hh.build(wl)
    mg = MG.Multigrid(h, **kw)
    E = _dense_propagator(h, mg)
    rng = np.random.default_rng(5)
    n = h.finest.ndof
    xs = rng.standard_normal(n)
    xs[h.finest.mask.ravel()] = 0.0
    b = h.finest.A @ xs
    x0 = rng.standard_normal(n)
    x, _ = mg.mg_iteration(b, x0=x0, fixed_iters=3)
    e_pred = np.linalg.matrix_power(E, 3) @ (x0 - xs)
    assert np.linalg.norm((x - xs) - e_pred) <= 1e-12 * max(1.0, np.linalg.norm(x0 - xs))
    # the V-cycle from 0 is the linear map (I - E) A^{-1}
    v = mg.vcycle(b)
    Ad = h.finest.A.toarray()
    assert np.allclose(v, (np.eye(n) - E) @ np.linalg.solve(Ad, b), rtol=0,
                       atol=1e-12 * np.abs(xs).max())


def _krylov_minres_point(A, b, x0, k, M=None):
    r0 = b - A @ x0
    cols = []
    v = r0.copy()
    for _ in range(k):
        z = v if M is None else M(v)
        cols.append(z)
        v = A @ z
    # search space span{M r0, M A M r0, ...}: Z_j = M (AM)^j r0
    Z = np.stack(cols, axis=1)
    Q, _ = np.linalg.qr(Z)
    y, *_ = np.linalg.lstsq(A @ Q, r0, rcond=None)
    return x0 + Q @ y


@pytest.mark.parametrize("use_mg", [False, True])
def test_fgmres_is_minimal_residual(use_mg):
    h = Hh.build(W.c2_td(band_rounds=1, uniform_rounds=1, delta=0.05))
    mg = MG.Multigrid(h)
    A = h.finest.A
    Ad = A.toarray()
    b = h.b
    M = mg.vcycle if use_mg else (lambda v: v)
    for k in (1, 3, 6):
        x, st = mg.fgmres(b, fixed_iters=k, m=10, precond=M)
        ref = _krylov_minres_point(Ad, b, np.zeros_like(b), k, M)
        assert st.iters == k
        assert np.linalg.norm(b - Ad @ x) == pytest.approx(np.linalg.norm(b - Ad @ ref), rel=1e-8)
        assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)


def test_fgmres_exact_preconditioner_one_step():
    h = Hh.build(W.c2_td(band_rounds=1, uniform_rounds=1, delta=0.05))
    mg = MG.Multigrid(h)
    lu = spla.splu(h.finest.A.tocsc())
    x, st = mg.fgmres(h.b, precond=lu.solve, rtol=1e-12)
    assert st.iters == 1 and st.converged


def test_manufactured_quadratic_convergence():
    exact = lambda p: np.sin(math.pi * p[:, 0]) * np.sin(math.pi * p[:, 1])
    errs = []
    for r in (3, 4, 5, 6):
        h = Hh.build(W.c1_poisson(r))
        x, st = MG.Multigrid(h).solve(h.b)
        assert st.converged
        errs.append(MG.l2_error(h, x, exact))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.05), ratios


def test_poisson_rate_h_independent():
    rates = []
    for r in (3, 5, 7):
        h = Hh.build(W.c1_poisson(r))
        x, st = MG.Multigrid(h).mg_iteration(h.b, fixed_iters=8)
        hist = np.array(st.history)
        rates.append((hist[-1] / hist[-4]) ** (1 / 3))
    assert max(rates) < 0.1
    assert rates[-1] - rates[-2] < 0.02      # saturates: 17^2 ... 257^2 within 0.1


@pytest.mark.parametrize("wl", [W.c1_poisson(5), W.c2_td(band_rounds=3, uniform_rounds=1),
                                W.c3_elasticity(2), W.c4_oseen(2), W.c3_adaptive("edge", 3)])
def test_solution_matches_direct_solve(wl):
    h = Hh.build(wl)
    x, st = MG.Multigrid(h).solve(h.b)
    assert st.converged
    A = h.finest.A.tocsc()
    xd = spla.spsolve(A, h.b)
    assert np.linalg.norm(h.b - A @ x) <= wl.rtol * np.linalg.norm(h.b) * (1 + 1e-12)
    # error bounded by the condition number times the residual tolerance
    cond_est = 1.0 / (spla.eigs(A, k=1, sigma=0, return_eigenvectors=False, which="LM").__abs__()[0]
                      / abs(spla.eigs(A, k=1, return_eigenvectors=False, which="LM")[0]))
    assert np.linalg.norm(x - xd) <= 10 * cond_est * wl.rtol * np.linalg.norm(xd)


def test_constrained_dofs_stay_zero():
    h = Hh.build(W.c3_adaptive("edge", 3))
    x, st = MG.Multigrid(h).solve(h.b)
    assert np.all(x[h.finest.mask.ravel()] == 0.0)
