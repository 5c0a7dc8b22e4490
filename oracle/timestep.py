"""Time stepping of a linear problem with a fixed matrix (oracle, test-only).

Algorithm "Nonstationary Linear Problem" (Sec. 4): the matrices are assembled once,
then every time step assembles a right-hand side and solves one linear system, with the
matrix reused in every step.  The problem of Sec. 5.1 is discretised by backward Euler
with step dt and the lumped mass of eq. mass_lumping in both the time derivative and
the right-hand side (the paper proposes the lumped right-hand side to move its assembly
to the GPU; using the same lumped mass in the matrix keeps the scheme consistent):

    (M_l / dt + A) theta_n = M_l (theta_{n-1} / dt + f_n),   theta_n = g_n on the
                                                              Dirichlet boundary,

A the spatial Q1 operator, f_n the nodal values of the source at t_n, g_n those of the
Dirichlet data.  With the constraints eliminated as in the stationary problems
(A_t = Z (H^T A_t,full H) Z + I_C, x the free unknowns, theta = H x + g):

    b_n = Z H^T M_l (theta_{n-1} / dt + f_n) - Z H^T A_t,full E_g g_n,
    x_n = solve(A_t, b_n) by the workload's outer loop (GMRES preconditioned by the
          V-cycle, Sec. 4.2) from the previous x as initial guess,
    theta_n = H x_n, then theta_n = g_n on the Dirichlet degrees of freedom.

`operators` builds the fixed matrices of the right-hand side: R = [Q | -G] with
Q = Z H^T M_l and G = Z H^T A_t,full E_g (E_g the injection of the Dirichlet degrees of
freedom), so that b_n = R [theta_{n-1} / dt + f_n ; g_n].
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse as sp

from . import fem


@dataclasses.dataclass
class TimeOperators:
    R: sp.csr_matrix          # N x (N + n_g): [Q | -G]
    H: sp.csr_matrix          # N x N (DoF level; identity rows on regular nodes)
    g_idx: np.ndarray         # n_g Dirichlet DoF indices
    mask: np.ndarray          # N bool, constrained DoFs
    coords: np.ndarray        # (n_nodes, dim) node coordinates


def operators(hier) -> TimeOperators:
    wl = hier.wl
    top = hier.finest
    mesh = top.mesh
    b = wl.block
    n = mesh.n
    N = n * b
    mask = fem.dof_mask(mesh, wl)
    on = mesh.boundary_mask(wl.dir_faces)
    dmask = np.zeros((n, b), bool)
    for c in range(b):
        if wl.dir_comps >> c & 1:
            dmask[on, c] = True
    g_idx = np.nonzero(dmask.ravel())[0]
    Hd = sp.kron(mesh.H, sp.identity(b), format="csr")          # DoF-level H
    Z = sp.diags((~mask.ravel()).astype(np.float64))
    m = fem.lumped_mass(mesh)
    Ml = sp.diags(np.repeat(m, b))
    keys, vals = fem.assemble_full(mesh, wl)                     # includes the M_l / dt term
    rows = []
    for ci in range(b):
        for cj in range(b):
            rows.append(sp.csr_matrix((vals[:, ci, cj], ((keys // n) * b + ci, (keys % n) * b + cj)),
                                      shape=(N, N)))
    Afull = sum(rows[1:], rows[0]).tocsr()
    Eg = sp.csr_matrix((np.ones(len(g_idx)), (g_idx, np.arange(len(g_idx)))), shape=(N, len(g_idx)))
    Q = (Z @ Hd.T @ Ml).tocsr()
    G = (Z @ Hd.T @ Afull @ Eg).tocsr()
    R = sp.hstack([Q, -G], format="csr")
    R.sort_indices()
    return TimeOperators(R=R, H=Hd.tocsr(), g_idx=g_idx, mask=mask.ravel(), coords=mesh.coords)


def nodal_data(ops: TimeOperators, wl, exact, source, t: float):
    """Nodal source values f(t, x_i) (N) and Dirichlet values g(t, x_j) (n_g) of a scalar
    problem."""
    X = ops.coords
    f = source(t, X[:, 0], X[:, 1])
    g = exact(t, X[:, 0], X[:, 1])[ops.g_idx]
    return f, g


@dataclasses.dataclass
class StepResult:
    theta: np.ndarray
    iters: int
    res_final: float


def run(hier, mg, ops: TimeOperators, theta0: np.ndarray, F: np.ndarray, Gv: np.ndarray,
        dt: float) -> List[StepResult]:
    """Backward Euler steps n = 1 .. len(F): F[n-1] = f_n (N), Gv[n-1] = g_n (n_g)."""
    theta = theta0.copy()
    x = np.where(ops.mask, 0.0, theta0)
    out = []
    for f, g in zip(F, Gv):
        b = ops.R @ np.concatenate([theta / dt + f, g])
        x, st = mg.solve(b, x0=x)
        theta = ops.H @ x
        theta[ops.g_idx] = g
        out.append(StepResult(theta.copy(), st.iters, st.res_final))
    return out
