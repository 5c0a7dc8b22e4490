"""Pins for the oracle's Chebyshev smoother (the Chebyshev iteration for S A, Saad,
Iterative Methods for Sparse Linear Systems, Sec. 12.3; a stronger smoother of the
fixed-matrix family, Sec. 6) and for its power-iteration eigenvalue estimate.

The recurrence is checked against the closed form it must produce: after k steps the
error is p_k(S A) e_0 with p_k(t) = T_k((theta - t) / delta) / T_k(theta / delta), T_k the
Chebyshev polynomial of the first kind, evaluated here through an eigendecomposition of
the dense S A (independent of the recurrence)."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import workloads as W
from oracle import hierarchy as Hh, multigrid as MG


def _dense_S(mg, l, n):
    S = mg.S[l]
    b = S.shape[1]
    out = np.zeros((n, n))
    for i in range(S.shape[0]):
        out[i * b:(i + 1) * b, i * b:(i + 1) * b] = S[i]
    return out


def _poly_of(SA, lam, lo, hi, k):
    """p_k(S A) through the eigenvalues of S A (real: S A is similar to a symmetric
    matrix for symmetric A and SPD S)."""
    a, c = lo * lam, hi * lam
    theta, delta = (c + a) / 2, (c - a) / 2
    w, V = np.linalg.eig(SA)
    assert np.abs(w.imag).max() < 1e-10
    w, V = w.real, V.real
    coef = [0.0] * k + [1.0]
    p = npcheb.chebval((theta - w) / delta, coef) / npcheb.chebval(theta / delta, coef)
    return V @ np.diag(p) @ np.linalg.inv(V)


def _cheb(wl, **kw):
    return wl.with_(smoother=W.SMOOTH_CHEBYSHEV, **kw)


@pytest.mark.parametrize("wl", [_cheb(W.c1_poisson(2)), _cheb(W.c3_elasticity(1), cheb_lo=0.15)],
                         ids=["poisson9", "elast5"])
def test_chebyshev_steps_apply_the_chebyshev_polynomial(wl):
    h = Hh.build(wl)
    mg = MG.Multigrid(h)
    L = h.L
    A = h.finest.A.toarray()
    n = A.shape[0]
    SA = _dense_S(mg, L, n) @ A
    rng = np.random.default_rng(3)
    xs = rng.standard_normal(n)
    b = A @ xs
    x0 = rng.standard_normal(n)
    for k in (1, 2, 3, 5):
        x = mg.chebyshev(L, x0, b, k)
        pred = _poly_of(SA, mg.lam[L], mg.cheb_lo, mg.cheb_hi, k) @ (xs - x0)
        assert np.linalg.norm((xs - x) - pred) <= 1e-11 * np.linalg.norm(xs - x0), k


def test_one_chebyshev_step_is_jacobi_with_the_interval_midpoint():
    """Degree 1: x + S (b - A x) / theta, theta the midpoint of the interval."""
    wl = _cheb(W.c1_poisson(3))
    h = Hh.build(wl)
    mg = MG.Multigrid(h)
    rng = np.random.default_rng(4)
    n = h.finest.ndof
    x, b = rng.standard_normal(n), rng.standard_normal(n)
    theta = 0.5 * (mg.cheb_lo + mg.cheb_hi) * mg.lam[h.L]
    jac = MG.Multigrid(h, omega=1.0 / theta)
    assert np.allclose(mg.chebyshev(h.L, x, b, 1), jac.smooth(h.L, x, b), rtol=0, atol=1e-14)


def test_power_estimate_converges_to_the_largest_eigenvalue():
    """With many steps the estimate reaches max |eig(S A)| (dense eigenvalues); with the
    default 12 steps it is already within 10 % on the 17^2 Poisson mesh."""
    wl = _cheb(W.c1_poisson(3))
    h = Hh.build(wl)
    mg = MG.Multigrid(h)
    n = h.finest.ndof
    lmax = np.abs(np.linalg.eigvals(_dense_S(mg, h.L, n) @ h.finest.A.toarray())).max()
    assert abs(mg.power_estimate(h.L, 2000) - lmax) <= 1e-6 * lmax
    assert abs(mg.lam[h.L] - lmax) <= 0.1 * lmax


def test_vcycle_with_chebyshev_matches_dense_propagator():
    """E_l = p_nu2(S A) (I - P (I - E_{l-1}) A_{l-1}^{-1} R A) p_nu1(S A), E_0 = 0 (exact
    coarse solve): three MG iterations apply E_L^3 to the initial error."""
    wl = _cheb(W.c3_elasticity(1), nu1=2, nu2=3)
    h = Hh.build(wl)
    mg = MG.Multigrid(h)
    E = [np.zeros((h.levels[0].A.shape[0],) * 2)]
    for l in range(1, h.L + 1):
        lv = h.levels[l]
        A = lv.A.toarray()
        n = A.shape[0]
        SA = _dense_S(mg, l, n) @ A
        Ac = h.levels[l - 1].A.toarray()
        Binv = (np.eye(Ac.shape[0]) - E[l - 1]) @ np.linalg.inv(Ac)
        C = np.eye(n) - lv.P.toarray() @ Binv @ lv.R.toarray() @ A
        E.append(_poly_of(SA, mg.lam[l], mg.cheb_lo, mg.cheb_hi, mg.nu2) @ C
                 @ _poly_of(SA, mg.lam[l], mg.cheb_lo, mg.cheb_hi, mg.nu1))
    rng = np.random.default_rng(5)
    n = h.finest.ndof
    xs = rng.standard_normal(n)
    xs[h.finest.mask.ravel()] = 0.0
    b = h.finest.A @ xs
    x0 = rng.standard_normal(n)
    x, _ = mg.mg_iteration(b, x0=x0, fixed_iters=3)
    pred = np.linalg.matrix_power(E[-1], 3) @ (x0 - xs)
    assert np.linalg.norm((x - xs) - pred) <= 1e-11 * np.linalg.norm(x0 - xs)


def test_chebyshev_contracts_faster_than_damped_block_jacobi_on_elasticity():
    """The reason for the stronger smoother: on the 9^3-node elasticity problem the
    V(2,2) error propagator's spectral radius is smaller with the Chebyshev smoother on
    [0.15, 1.1] lambda than with damped block Jacobi (omega = 0.6)."""
    rates = []
    for wl in (W.c3_elasticity(2), _cheb(W.c3_elasticity(2))):
        h = Hh.build(wl)
        mg = MG.Multigrid(h)
        n = h.finest.ndof
        E = np.eye(n) - np.column_stack([mg.vcycle(h.finest.A @ e) for e in np.eye(n)])
        rates.append(np.abs(np.linalg.eigvals(E)).max())
    assert rates[1] < 0.8 * rates[0], rates
