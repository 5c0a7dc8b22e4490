"""Smoother, coarse solve, V-cycle and outer iterations in FP64 (oracle, test-only).

  * Smoother (Sec. 4.1 "Geometric Multigrid CUDA"): x <- x + omega S (b - A x) with a
    fixed matrix S; here S = inverse of the nodal diagonal blocks of A (damped Jacobi for
    one component, nodal block-Jacobi / point-Vanka for systems).  Sweeps are
    simultaneous (Jacobi), every sweep a full update.
  * Stronger smoother (Sec. 6 names stronger smoothers as the next step): the nu steps of
    a smoothing phase as the Chebyshev iteration for S A on [lo, hi] * lambda (Saad,
    Iterative Methods for Sparse Linear Systems, Sec. 12.3, Algorithm "Chebyshev
    acceleration"), lambda the largest eigenvalue of S A estimated by power iteration.
  * Coarse problem (Algorithm "Geometric multigrid solver", step 0): A_0^{-1} b_0 by a
    dense LU solve; the paper's GPU variant of a few smoothing sweeps is mode SMOOTH.
  * V-cycle: Algorithm "Geometric multigrid solver": pre-smooth nu1 times, restrict the
    residual, recurse with initial value 0, prolongate and add, post-smooth nu2 times.
  * MG iteration x_n = GMG(L, x_{n-1}, b) (same algorithm), and GMRES preconditioned by
    one V-cycle (Sec. 4.2: modified Gram-Schmidt, Givens rotations, at most m steps per
    restart), in its flexible right-preconditioned form (Saad, Sec. 9.4.1), so that the
    preconditioner may change between steps.
  * Stopping rule (reading): ||b - A x||_2 <= rtol ||b||_2 in FP64 over all rows.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

import workloads as W


def diag_blocks(rowptr, col, val) -> np.ndarray:
    """The nodal diagonal blocks A_ii (n, b, b) of a BSR matrix."""
    n = len(rowptr) - 1
    out = np.zeros((n, val.shape[1], val.shape[2]))
    r = np.repeat(np.arange(n), np.diff(rowptr))
    d = r == col
    assert np.bincount(r[d], minlength=n).min() == 1
    out[r[d]] = val[d]
    return out


def smoother_blocks(level) -> np.ndarray:
    """S = blockdiag(A)^{-1}, one b x b inverse per node."""
    return np.linalg.inv(diag_blocks(level.rowptr, level.col, level.val))


@dataclasses.dataclass
class SolveStats:
    iters: int = 0              # V-cycles applied
    restarts: int = 0
    res0: float = 0.0
    res_final: float = 0.0
    converged: bool = False
    history: list = dataclasses.field(default_factory=list)


class Multigrid:
    def __init__(self, hier, omega=None, nu1=None, nu2=None, coarse_mode=None, coarse_sweeps=None):
        wl = hier.wl
        self.h = hier
        self.omega = wl.omega if omega is None else omega
        self.nu1 = wl.nu1 if nu1 is None else nu1
        self.nu2 = wl.nu2 if nu2 is None else nu2
        self.coarse_mode = wl.coarse_mode if coarse_mode is None else coarse_mode
        self.coarse_sweeps = wl.coarse_sweeps if coarse_sweeps is None else coarse_sweeps
        self.S = [smoother_blocks(lv) for lv in hier.levels]
        self.smoother = wl.smoother
        self.cheb_lo, self.cheb_hi = wl.cheb_lo, wl.cheb_hi
        self.lam = [None] * len(hier.levels)
        if self.smoother == W.SMOOTH_CHEBYSHEV:
            for l in range(1, len(hier.levels)):
                self.lam[l] = self.power_estimate(l, wl.power_its)
        A0 = hier.levels[0].A.toarray()
        self.A0 = A0
        self.lu0 = sla.lu_factor(A0)

    # -- building blocks ---------------------------------------------------------
    def apply_S(self, l: int, r: np.ndarray) -> np.ndarray:
        S = self.S[l]
        b = S.shape[1]
        return np.einsum("nij,nj->ni", S, r.reshape(-1, b)).ravel()

    def smooth(self, l: int, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        """One damped (block-)Jacobi sweep x + omega S (b - A x)."""
        A = self.h.levels[l].A
        return x + self.omega * self.apply_S(l, b - A @ x)

    def power_estimate(self, l: int, its: int) -> float:
        """Largest eigenvalue of S A by power iteration: v = Weyl vector / its norm, then
        `its` times w = S A v, lambda = ||w||, v = w / lambda; the last lambda."""
        A = self.h.levels[l].A
        v = W.weyl_vec(A.shape[0])
        v = v / np.linalg.norm(v)
        lam = 0.0
        for _ in range(its):
            w = self.apply_S(l, A @ v)
            lam = float(np.linalg.norm(w))
            v = w / lam
        return lam

    def chebyshev(self, l: int, x: np.ndarray, b: np.ndarray, k: int) -> np.ndarray:
        """k steps of the Chebyshev iteration for A x = b preconditioned by S, for a
        spectrum of S A in [a, c] = [lo, hi] * lambda: theta = (c + a)/2, delta = (c - a)/2,
        sigma = theta/delta; d_0 = S r_0 / theta; x_{j+1} = x_j + d_j;
        rho_0 = 1/sigma, rho_{j+1} = 1/(2 sigma - rho_j),
        d_{j+1} = rho_{j+1} rho_j d_j + (2 rho_{j+1}/delta) S r_{j+1}."""
        A = self.h.levels[l].A
        a, c = self.cheb_lo * self.lam[l], self.cheb_hi * self.lam[l]
        theta, delta = (c + a) / 2, (c - a) / 2
        sigma = theta / delta
        rho = 1.0 / sigma
        d = self.apply_S(l, b - A @ x) / theta
        for j in range(k):
            x = x + d
            if j + 1 < k:
                rho_next = 1.0 / (2.0 * sigma - rho)
                d = rho_next * rho * d + (2.0 * rho_next / delta) * self.apply_S(l, b - A @ x)
                rho = rho_next
        return x

    def smooth_phase(self, l: int, x: np.ndarray, b: np.ndarray, k: int) -> np.ndarray:
        """A pre- or post-smoothing phase of k steps on level l >= 1."""
        if k == 0:
            return x
        if self.smoother == W.SMOOTH_CHEBYSHEV:
            return self.chebyshev(l, x, b, k)
        for _ in range(k):
            x = self.smooth(l, x, b)
        return x

    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        if self.coarse_mode == W.COARSE_EXACT:
            return sla.lu_solve(self.lu0, b)
        x = np.zeros_like(b)
        for _ in range(self.coarse_sweeps):
            x = self.smooth(0, x, b)
        return x

    def gmg(self, l: int, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        """GMG(l, x, b) of the Algorithm "Geometric multigrid solver"."""
        if l == 0:
            return self.coarse_solve(b)                         # step 0
        lv = self.h.levels[l]
        x = self.smooth_phase(l, x, b, self.nu1)                # step 1
        d = lv.R @ (b - lv.A @ x)                               # step 2
        y = self.gmg(l - 1, np.zeros(lv.R.shape[0]), d)         # step 3
        x = x + lv.P @ y                                        # step 4
        x = self.smooth_phase(l, x, b, self.nu2)                # step 5
        return x

    def vcycle(self, b: np.ndarray) -> np.ndarray:
        """One V-cycle on the finest level from the initial value 0."""
        return self.gmg(self.h.L, np.zeros_like(b), b)

    # -- outer iterations --------------------------------------------------------
    def residual_norm(self, x, b):
        return float(np.linalg.norm(b - self.h.finest.A @ x))

    def mg_iteration(self, b, x0=None, rtol=None, maxit=None, fixed_iters=None):
        """x_n = GMG(L, x_{n-1}, b) until ||b - A x_n|| <= rtol ||b|| (or fixed_iters)."""
        wl = self.h.wl
        rtol = wl.rtol if rtol is None else rtol
        maxit = wl.maxit if maxit is None else maxit
        x = np.zeros_like(b) if x0 is None else x0.copy()
        st = SolveStats()
        bn = float(np.linalg.norm(b))
        res = self.residual_norm(x, b)
        st.res0 = res
        st.history.append(res)
        while True:
            if fixed_iters is None and res <= rtol * bn:
                st.converged = True
                break
            if st.iters >= (maxit if fixed_iters is None else fixed_iters):
                break
            x = self.gmg(self.h.L, x, b)
            st.iters += 1
            res = self.residual_norm(x, b)
            st.history.append(res)
        st.res_final = res
        return x, st

    def fgmres(self, b, x0=None, rtol=None, m=None, maxit=None, fixed_iters=None,
               precond: Optional[Callable] = None):
        """Restarted flexible GMRES(m), right preconditioner = one V-cycle (Sec. 4.2).

        Modified Gram-Schmidt, Givens rotations; the inner loop stops when the
        updated residual estimate |g_{j+1}| <= rtol ||b||; after every restart cycle
        the true residual decides.  `fixed_iters` runs exactly that many inner steps
        (restarting every m) and ignores the tolerance."""
        wl = self.h.wl
        rtol = wl.rtol if rtol is None else rtol
        m = wl.gmres_m if m is None else m
        maxit = wl.maxit if maxit is None else maxit
        M = self.vcycle if precond is None else precond
        A = self.h.finest.A
        x = np.zeros_like(b) if x0 is None else x0.copy()
        st = SolveStats()
        bn = float(np.linalg.norm(b))
        tol = rtol * bn
        limit = maxit if fixed_iters is None else fixed_iters
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        st.res0 = beta
        st.history.append(beta)
        while True:
            if fixed_iters is None and beta <= tol:
                st.converged = True
                break
            if st.iters >= limit or beta == 0.0:
                break
            V = [r / beta]
            Z = []
            Hh = np.zeros((m + 1, m))
            cs = np.zeros(m)
            sn = np.zeros(m)
            g = np.zeros(m + 1)
            g[0] = beta
            k = 0
            for j in range(m):
                Z.append(M(V[j]))
                st.iters += 1
                w = A @ Z[j]
                for i in range(j + 1):                              # modified Gram-Schmidt
                    Hh[i, j] = float(w @ V[i])
                    w = w - Hh[i, j] * V[i]
                Hh[j + 1, j] = float(np.linalg.norm(w))
                breakdown = Hh[j + 1, j] == 0.0
                if not breakdown:
                    V.append(w / Hh[j + 1, j])
                for i in range(j):                                  # previous rotations
                    t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                    Hh[i + 1, j] = -sn[i] * Hh[i, j] + cs[i] * Hh[i + 1, j]
                    Hh[i, j] = t
                den = float(np.hypot(Hh[j, j], Hh[j + 1, j]))      # new rotation
                cs[j] = Hh[j, j] / den
                sn[j] = Hh[j + 1, j] / den
                Hh[j, j] = den
                Hh[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                k = j + 1
                st.history.append(abs(g[j + 1]))
                if breakdown or st.iters >= limit:
                    break
                if fixed_iters is None and abs(g[j + 1]) <= tol:
                    break
            y = sla.solve_triangular(Hh[:k, :k], g[:k], lower=False)
            for i in range(k):
                x = x + y[i] * Z[i]
            st.restarts += 1
            r = b - A @ x
            beta = float(np.linalg.norm(r))
        st.res_final = beta
        st.converged = beta <= tol
        return x, st

    def solve(self, b, x0=None, **kw):
        if self.h.wl.outer == W.OUTER_FGMRES:
            return self.fgmres(b, x0, **kw)
        return self.mg_iteration(b, x0, **kw)


def l2_error(hier, x, exact: Callable, comp: int = 0) -> float:
    """L2 norm of u_h - u for component `comp` on the finest mesh, 3-point tensor Gauss
    per direction, u_h = H x (hanging values interpolated) evaluated per leaf from its
    corner values; exact(points) returns that component's values."""
    from . import fem
    top = hier.finest
    mesh = top.mesh
    xf = mesh.H @ x.reshape(mesh.n, -1)[:, comp]
    s, x0, nodes = fem.leaf_table(mesh)
    qp, qw = fem.tensor_rule(mesh.dim, 3)
    phi, _ = fem.ref_basis(mesh.dim, qp)
    uh = np.einsum("qa,ea->eq", phi, xf[nodes])
    xq = x0[:, None, :] + s[:, None, None] * qp[None, :, :]
    ue = exact(xq.reshape(-1, mesh.dim)).reshape(uh.shape)
    err2 = np.einsum("q,e,eq->", qw, s ** mesh.dim, (uh - ue) ** 2)
    return float(np.sqrt(err2))
