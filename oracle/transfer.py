"""Grid transfer matrices between consecutive levels (oracle, test-only).

Sec. 4.1 "Geometric Multigrid CUDA", eq. (prolongation): the fine coefficients are
u_i^{l+1} = sum_j chi_ij u_j^l with the same element-local coefficients on every cell,
written as one global sparse matrix P_l; restriction is R_l = P_l^T.

Reading: the element-local coefficients are the values of the coarse nodal basis at the
fine nodes.  Globally, (Q)_ij = phi_j^coarse(x_i^fine) is assigned once per fine node
(not summed over cells), the coarse hanging-node constraints are folded in,
P~ = Q H_coarse, and exact zeros are dropped so the pattern is canonical.  Every
weight is a sum of products of 1, 1/2 and 1/4, hence exact in binary floating point.
For systems P = M_f (P~ (x) I_b) M_c with M = I - diag(constrained-DoF mask), and
R = P^T.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def prolongation(fine_mesh, coarse_mesh) -> sp.csr_matrix:
    """Scalar P~ (n_fine x n_coarse), CSR with sorted column indices."""
    ff, fc = fine_mesh.forest, coarse_mesh.forest
    assert ff.D == fc.D and ff.vshape == fc.vshape
    dim, D = ff.dim, ff.D
    p = fine_mesh.coords_lat                                   # (nf, dim) (x, y[, z])
    ncell = [fc.cell_shape[dim - 1 - a] for a in range(dim)]   # finest cells per axis
    cell = np.minimum(p, np.array(ncell) - 1)                  # a finest cell touching p
    dep = fc.dep[tuple(cell[:, a] for a in reversed(range(dim)))].astype(np.int64)
    size = np.left_shift(1, D - dep)
    anchor = (cell // size[:, None]) * size[:, None]
    xi_num = p - anchor                                        # local coordinate * size
    assert np.all((xi_num >= 0) & (xi_num <= size[:, None]))
    rows, cols, vals = [], [], []
    for off in itertools.product((0, 1), repeat=dim):
        off = np.array(off)
        w = np.ones(len(p))
        for a in range(dim):
            t = xi_num[:, a] / size
            w *= t if off[a] else 1.0 - t
        corner = anchor + off[None, :] * size[:, None]
        lin = np.ravel_multi_index(tuple(corner[:, a] for a in reversed(range(dim))), fc.vshape)
        cn = coarse_mesh.node_of_lin[lin]
        assert np.all(cn >= 0)
        rows.append(np.arange(len(p)))
        cols.append(cn)
        vals.append(w)
    Q = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine_mesh.n, coarse_mesh.n))
    Pt = (Q @ coarse_mesh.H).tocsr()
    Pt.sum_duplicates()
    Pt.eliminate_zeros()
    Pt.sort_indices()
    return Pt


def system_prolongation(Pt: sp.csr_matrix, mask_f: np.ndarray, mask_c: np.ndarray) -> sp.csr_matrix:
    """P = M_f (P~ (x) I_b) M_c on the scalar dof numbering node * b + component."""
    b = mask_f.shape[1]
    P = sp.kron(Pt, sp.identity(b, format="csr"), format="csr")
    Mf = sp.diags((~mask_f.ravel()).astype(np.float64))
    Mc = sp.diags((~mask_c.ravel()).astype(np.float64))
    return (Mf @ P @ Mc).tocsr()
