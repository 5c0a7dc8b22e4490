"""Pins for the oracle's FP32 emulation of the reduced-precision cycle steps."""
import numpy as np
import pytest

import workloads as W
from oracle import hierarchy as Hh, mixed as MX, multigrid as MG


@pytest.fixture(scope="module")
def hier():
    return Hh.build(W.c4_oseen(2))


def test_block_csr_keeps_every_block_entry(hier):
    """The scalar view of the BSR operator equals the oracle's CSR operator entry by entry
    and stores all nnzb * b^2 block entries (explicit zeros of the blocks included)."""
    lv = hier.finest
    A = MX.block_csr(lv)
    b = lv.val.shape[1]
    assert A.nnz == len(lv.col) * b * b
    assert np.array_equal(A.toarray(), lv.A.toarray())
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    same = rows[1:] == rows[:-1]
    assert np.all(np.diff(A.indices.astype(np.int64))[same] > 0)       # sorted, unique per row


@pytest.mark.parametrize("fmt,bound", [("fp32", 2.0 ** -24), ("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_stored_operator_error_bounds(hier, fmt, bound):
    """Stored values are single roundings: |stored - a| <= u_fmt |a| for entries in the
    format's normal range relative to their row scale (FP16 below 2^-14 s_i: absolute
    2^-25 s_i), and exact zeros stay zero."""
    lv = hier.finest
    A = MX.block_csr(lv)
    S = MX.stored_operator(lv, fmt)
    assert np.array_equal(S.indices, A.indices) and np.array_equal(S.indptr, A.indptr)
    err = np.abs(S.data - A.data)
    assert np.all(S.data[A.data == 0.0] == 0.0)
    if fmt == "fp16":
        from oracle import codec
        e = codec.row_exponents(A)
        s = np.ldexp(1.0, e[np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))])
        small = np.abs(A.data) < 2.0 ** -14 * s
        assert np.all(err[~small] <= bound * np.abs(A.data[~small]))
        assert np.all(err[small] <= 2.0 ** -25 * s[small])
    else:
        assert np.all(err <= bound * np.abs(A.data))


def test_emulated_sweep_is_the_fp64_sweep_on_exact_data(hier):
    """With FP64 data and an FP32-exact damping factor the emulated sweep formulas are the
    FP64 oracle's smoother (same formula, same block application)."""
    mgo = MG.Multigrid(hier, omega=0.75)
    for l, lv in enumerate(hier.levels):
        x = W.rand_vec(10 + l, lv.ndof)
        b = W.rand_vec(20 + l, lv.ndof)
        S = MG.smoother_blocks(lv)
        got = MX.sweep(MX.block_csr(lv), S, 0.75, x, b)
        assert np.allclose(got, mgo.smooth(l, x, b), rtol=0, atol=1e-14 * np.abs(got).max())
        assert np.allclose(MX.sweep0(S, 0.75, b), mgo.smooth(l, np.zeros_like(b), b), rtol=0, atol=1e-15)


def test_fp32_row_bound_covers_fp32_sums():
    """Sequential FP32 sums of random terms stay within gamma_k sum |terms|."""
    rng = np.random.default_rng(0)
    for k in (3, 27, 108):
        t = rng.standard_normal((2000, k)).astype(np.float32)
        acc = np.zeros(2000, np.float32)
        for j in range(k):
            acc = (acc + t[:, j]).astype(np.float32)
        exact = t.astype(np.float64).sum(axis=1)
        bnd = MX.fp32_row_bound(np.full(2000, k), np.abs(t.astype(np.float64)).sum(axis=1))
        assert np.all(np.abs(acc - exact) <= bnd)
