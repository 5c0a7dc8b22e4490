"""The multigrid level hierarchy of one workload (oracle, test-only).

Sec. 2.2: start from the finest adaptive mesh Omega_L and coarsen globally until the
coarse grid Omega_0 is reached; every level spans the whole domain (global multigrid).
Reading: every level is rediscretised with the same bilinear form (the paper's "V_l
the corresponding finite element spaces"), not built by Galerkin products.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

import workloads as W
from . import fem, mesh as M, transfer


@dataclasses.dataclass
class Level:
    mesh: M.Mesh
    rowptr: np.ndarray          # node-level BSR of the constrained operator
    col: np.ndarray
    val: np.ndarray             # (nnzb, b, b)
    A: sp.csr_matrix            # the same operator as scalar CSR (dof = node*b + comp)
    mask: np.ndarray            # (n, b) bool, True = constrained dof
    Pt: Optional[sp.csr_matrix]  # scalar P~ from the next coarser level (None on level 0)
    P: Optional[sp.csr_matrix]   # system prolongation M_f (P~ (x) I) M_c
    R: Optional[sp.csr_matrix]   # R = P^T

    @property
    def n(self):
        return self.mesh.n

    @property
    def ndof(self):
        return self.A.shape[0]


@dataclasses.dataclass
class Hierarchy:
    wl: W.Workload
    levels: List[Level]
    b: np.ndarray               # finest right-hand side, flat (ndof,) or (ndof, nrhs)
    f_full: np.ndarray          # unconstrained finest load (n, b[, nrhs])

    @property
    def L(self):
        return len(self.levels) - 1

    @property
    def finest(self):
        return self.levels[-1]


def build_level(wl, forest) -> Level:
    mesh = M.Mesh(forest)
    keys, vals = fem.assemble_full(mesh, wl)
    rowptr, col, val = fem.constrain(mesh, wl, keys, vals)
    A = fem.bsr_to_csr(rowptr, col, val)
    mask = fem.dof_mask(mesh, wl)
    return Level(mesh, rowptr, col, val, A, mask, None, None, None)


def build(wl: W.Workload, nrhs: int = 1) -> Hierarchy:
    finest = M.build_forest(wl)
    forests = M.hierarchy_forests(finest)
    # the coarse mesh may be any level of the hierarchy (Sec. 2.2); levels below it are unused
    forests = forests[min(wl.coarse_level, len(forests) - 1):]
    levels = [build_level(wl, f) for f in forests]
    for l in range(1, len(levels)):
        fine, coarse = levels[l], levels[l - 1]
        fine.Pt = transfer.prolongation(fine.mesh, coarse.mesh)
        fine.P = transfer.system_prolongation(fine.Pt, fine.mask, coarse.mask)
        fine.R = fine.P.T.tocsr()
    top = levels[-1]
    if wl.rhs == W.RHS_NOISE:
        xi = W.noise(wl.seed, top.n, nrhs)
        cols = []
        for r in range(nrhs):
            f_full = fem.assemble_load(top.mesh, wl, xi[:, r:r + 1])
            cols.append(fem.constrain_load(top.mesh, wl, f_full).ravel())
        b = np.stack(cols, axis=1) if nrhs > 1 else cols[0]
        f_full = None
    else:
        f_full = fem.assemble_load(top.mesh, wl)
        b = fem.constrain_load(top.mesh, wl, f_full).ravel()
    return Hierarchy(wl, levels, b, f_full)
