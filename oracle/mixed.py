"""Reduced-precision V-cycle steps, emulated on the host (oracle, test-only).

The paper names single precision as its most promising next step (Sec. 5.4: the
bandwidth-bound SpMV gains arithmetic intensity).  In the mixed form the V-cycle runs in
FP32 on an operator stored in FP32, or as FP16 / BF16 codes with one power-of-two scale
per scalar row (oracle.codec), while the outer defect stays FP64.

This module gives, for each step of the cycle, the exact value of the step applied to
the FP32 data the cycle holds: the stored values as decoded in FP32 (decoding is exact:
2^e q with q of 11 or 8 significant bits), the smoother blocks as the FP64 inverses of
the diagonal blocks rounded once to FP32, the damping factor rounded to FP32, and the
FP32 input vectors.  The products are formed in FP64 (exact enough to serve as the
reference of an FP32 evaluation); `fp32_row_bound` gives the standard a-priori bound
of evaluating such a row sum in FP32 (Higham, Accuracy and Stability of Numerical
Algorithms, Sec. 3.1: |fl(sum) - sum| <= gamma_k sum |terms|, gamma_k = k u / (1 - k u),
u = 2^-24), which the tests use as the tolerance.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import codec
from .multigrid import smoother_blocks

U32 = 2.0 ** -24


def block_csr(level) -> sp.csr_matrix:
    """Scalar CSR of the level's BSR operator with every stored block entry kept (explicit
    zeros included), rows and columns dof = node * b + component, columns sorted."""
    rowptr, col, val = level.rowptr, level.col, level.val
    n, b = len(rowptr) - 1, val.shape[1]
    blk_of_row = np.repeat(np.arange(n), np.diff(rowptr))
    # scalar row (i, c) holds, for each block k of node row i, the b entries val[k, c, :]
    rows, cols, data = [], [], []
    for c in range(b):
        for cc in range(b):
            rows.append(blk_of_row * b + c)
            cols.append(col.astype(np.int64) * b + cc)
            data.append(val[:, c, cc])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    data = np.concatenate(data)
    order = np.lexsort((cols, rows))
    rows, cols, data = rows[order], cols[order], data[order]
    indptr = np.zeros(n * b + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n * b), out=indptr[1:])
    return sp.csr_matrix((data, cols, indptr), shape=(n * b, n * b))


def stored_operator(level, fmt: str) -> sp.csr_matrix:
    """The cycle operator as the mixed form stores it, decoded in FP32 (values held as
    FP64 numbers that are exact FP32 values).  fmt: 'fp32', 'fp16' or 'bf16'."""
    A = block_csr(level)
    if fmt == "fp32":
        vals = A.data.astype(np.float32)
    else:
        e, q = codec.encode(A, fmt)
        vals = codec.decode_f32(A, e, q, fmt)
    return sp.csr_matrix((vals.astype(np.float64), A.indices, A.indptr), shape=A.shape)


def stored_smoother(level) -> np.ndarray:
    """Smoother blocks of the FP32 cycle: the FP64 inverses rounded once to FP32."""
    return smoother_blocks(level).astype(np.float32).astype(np.float64)


def f32(x) -> np.ndarray:
    """Round to FP32 (held as FP64)."""
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def apply_blocks(S: np.ndarray, r: np.ndarray) -> np.ndarray:
    b = S.shape[1]
    return np.einsum("nij,nj->ni", S, r.reshape(-1, b)).ravel()


def sweep(A32, S32, omega, x32, b32) -> np.ndarray:
    """x + omega32 S32 (b - A32 x) on FP32 data, evaluated exactly in FP64."""
    return x32 + f32(omega) * apply_blocks(S32, b32 - A32 @ x32)


def sweep0(S32, omega, b32) -> np.ndarray:
    return f32(omega) * apply_blocks(S32, b32)


def fp32_row_bound(terms_per_row: np.ndarray, magnitude: np.ndarray) -> np.ndarray:
    """gamma_k * magnitude per row for sums of k terms evaluated in FP32."""
    k = terms_per_row.astype(np.float64)
    return k * U32 / (1.0 - k * U32) * magnitude
