"""Pins for the oracle's element matrices, assembly, constraints and grid transfers.

Closed forms (tensor-product Q1 matrices, Laplace stencils), kernels of the unconstrained
operators (constants, rigid-body modes), symmetry, the Galerkin identity of nested
conforming spaces on uniform and hanging meshes, and exact properties of P~.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import fem, hierarchy as Hh, mesh as M, transfer

K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])          # int phi_i' phi_j' on [0,1]
M1 = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0       # int phi_i phi_j
G1 = np.array([[-1.0, 1.0], [-1.0, 1.0]]) / 2.0     # int phi_i (test) phi_j' (trial)


def _kron_local(*mats):
    """Tensor product in the local corner order a = o_x + 2 o_y (+ 4 o_z)."""
    out = np.ones((1, 1))
    for m in mats:                      # x first -> fastest index
        out = np.kron(m, out)
    return out


def test_laplace_element_closed_form():
    for s in (1.0, 0.25):
        Ke = fem.element_matrices(W.c1_poisson(), np.array([s]), np.zeros((1, 2)))[0, :, :, 0, 0]
        ref = _kron_local(K1, M1) + _kron_local(M1, K1)       # (1/s)*s in 2D
        assert np.allclose(Ke, ref, rtol=0, atol=1e-15)
    wl3 = W.c3_elasticity().with_(pde=W.PDE_POISSON, block=1)
    s = 0.5
    Ke = fem.element_matrices(wl3, np.array([s]), np.zeros((1, 3)))[0, :, :, 0, 0]
    ref = s * (_kron_local(K1, M1, M1) + _kron_local(M1, K1, M1) + _kron_local(M1, M1, K1))
    assert np.allclose(Ke, ref, rtol=0, atol=1e-15)


def test_td_element_closed_form():
    wl = W.c2_td()
    s = 0.125
    Ke = fem.element_matrices(wl, np.array([s]), np.zeros((1, 2)))[0, :, :, 0, 0]
    bx, by = wl.bvec
    tau = float(fem.supg_tau(wl, np.array([s]))[0])
    diff = _kron_local(K1, M1) + _kron_local(M1, K1)
    conv = s * (bx * _kron_local(G1, M1) + by * _kron_local(M1, G1))
    # (b.grad phi_b)(b.grad phi_a): x-y cross terms use G1 in both factors
    stab = (bx * bx * _kron_local(K1, M1) + by * by * _kron_local(M1, K1)
            + bx * by * (_kron_local(G1.T, G1) + _kron_local(G1, G1.T)))
    ref = wl.eps * diff + conv + tau * stab
    assert np.allclose(Ke, ref, rtol=0, atol=1e-15)
    # tau formula: h_K = s |b| / max|b_k|, Pe = |b| h_K / (2 eps), tau = h_K/(2|b|) L(Pe)
    nb = np.hypot(bx, by)
    hk = s * nb / max(abs(bx), abs(by))
    pe = nb * hk / (2 * wl.eps)
    assert tau == pytest.approx(hk / (2 * nb) * (1 / np.tanh(pe) - 1 / pe), rel=1e-14)
    # series branch agrees with the direct formula where both are accurate
    x = np.array([0.009, 0.0099])
    assert np.allclose(fem.langevin(x), 1 / np.tanh(x) - 1 / x, rtol=1e-9)


def _stencil_row(wl, rounds, centre_offset):
    f = M.build_forest(wl.with_(rounds=(("uniform",),) * rounds))
    m = M.Mesh(f)
    keys, vals = fem.assemble_full(m, wl)
    n = m.n
    A = sp.csr_matrix((vals[:, 0, 0], (keys // n, keys % n)), shape=(n, n))
    mid = tuple(s // 2 for s in f.vshape)
    lin = np.ravel_multi_index(mid, f.vshape)
    i = m.node_of_lin[lin]
    out = {}
    for off in np.ndindex(*(3,) * f.dim):
        o = np.array(off) - 1
        q = tuple(np.array(mid) + o)
        j = m.node_of_lin[np.ravel_multi_index(q, f.vshape)]
        out[tuple(o)] = A[i, j]
    return out, f.hf


def test_assembled_laplace_stencils():
    st, h = _stencil_row(W.c1_poisson(), 3, 0)
    for o, v in st.items():
        k = sum(abs(np.array(o)))
        assert v == pytest.approx({0: 8 / 3, 1: -1 / 3, 2: -1 / 3}[k], abs=1e-14)
    wl3 = W.c3_elasticity().with_(pde=W.PDE_POISSON, block=1)
    st, h = _stencil_row(wl3, 2, 0)
    for o, v in st.items():
        k = sum(abs(np.array(o)))
        assert v == pytest.approx({0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}[k], abs=1e-15)


def _full_matrix(wl):
    f = M.build_forest(wl)
    m = M.Mesh(f)
    keys, vals = fem.assemble_full(m, wl)
    n, b = m.n, wl.block
    A = np.zeros((n * b, n * b))
    for k, v in zip(keys, vals):
        i, j = divmod(int(k), n)
        A[i * b:(i + 1) * b, j * b:(j + 1) * b] += v
    return m, A


def test_constants_in_kernel_poisson_td():
    for wl in (W.c1_poisson(3), W.c2_td(band_rounds=2, uniform_rounds=1)):
        m, A = _full_matrix(wl)
        assert np.abs(A @ np.ones(m.n)).max() < 1e-13


def test_rigid_modes_in_kernel_elasticity():
    m, A = _full_matrix(W.c3_adaptive("vertex", 2))
    X = m.coords
    modes = []
    for c in range(3):
        u = np.zeros((m.n, 3))
        u[:, c] = 1
        modes.append(u.ravel())
    for p, q in [(0, 1), (1, 2), (0, 2)]:
        u = np.zeros((m.n, 3))
        u[:, p] = X[:, q]
        u[:, q] = -X[:, p]
        modes.append(u.ravel())
    for u in modes:
        assert np.abs(A @ u).max() < 1e-14
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    assert np.sum(ev < 1e-10) == 6 and ev.min() > -1e-12


def test_oseen_pressure_block_kills_constants():
    wl = W.c4_oseen(1)
    m, A = _full_matrix(wl)
    App = A[0::4, 0::4]
    assert np.abs(App @ np.ones(m.n)).max() < 1e-14
    # velocity-velocity block is diagonal in the component index
    for ci in range(1, 4):
        for cj in range(1, 4):
            if ci != cj:
                assert np.abs(A[ci::4, cj::4]).max() == 0.0


@pytest.mark.parametrize("wl", [W.c1_poisson(3), W.c3_elasticity(2)])
def test_symmetry_uniform_bitwise(wl):
    h = Hh.build(wl)
    for lv in h.levels:
        assert (lv.A != lv.A.T).nnz == 0


@pytest.mark.parametrize("wl", [W.c2_td(band_rounds=2, uniform_rounds=1).with_(pde=W.PDE_POISSON),
                                W.c3_adaptive("edge", 3)])
def test_symmetry_hanging_and_spd(wl):
    h = Hh.build(wl)
    for lv in h.levels:
        d = abs(lv.A - lv.A.T)
        assert (d.max() if d.nnz else 0.0) <= 1e-15 * abs(lv.A).max()
    A = h.finest.A.toarray()
    np.linalg.cholesky(0.5 * (A + A.T))


def test_constrained_rows_are_identity():
    h = Hh.build(W.c3_adaptive("edge", 3))
    lv = h.finest
    A = lv.A.tocsr()
    for i in np.nonzero(lv.mask.ravel())[0][:500]:
        row = A.getrow(i)
        nz = row.indices[row.data != 0]
        assert list(nz) == [i] and row[0, i] == 1.0
        col = A.getcol(i).tocoo()
        assert list(col.row[col.data != 0]) == [i]


@pytest.mark.parametrize("wl", [W.c1_poisson(3),
                                W.c2_td(band_rounds=2, uniform_rounds=1).with_(pde=W.PDE_POISSON),
                                W.c3_elasticity(2),
                                W.c3_adaptive("edge", 3)])
def test_galerkin_identity(wl):
    """Nested conforming spaces + exact quadrature: P^T A_f P = A_c on free dofs."""
    h = Hh.build(wl)
    for l in range(1, len(h.levels)):
        f, c = h.levels[l], h.levels[l - 1]
        G = (f.P.T @ f.A @ f.P).toarray()
        Ac = c.A.toarray()
        free = ~c.mask.ravel()
        D = G[np.ix_(free, free)] - Ac[np.ix_(free, free)]
        assert np.abs(D).max() <= 1e-13 * np.abs(Ac).max()


def test_prolongation_exact_properties():
    for wl in (W.c1_poisson(3), W.c2_td(band_rounds=3, uniform_rounds=1, delta=0.05),
               W.c3_adaptive("edge", 4), W.c3_adaptive("vertex", 3)):
        h = Hh.build(wl)
        for l in range(1, len(h.levels)):
            f, c = h.levels[l], h.levels[l - 1]
            Pt = f.Pt
            # P~ applied to the constant / a linear function is exact (dyadic arithmetic)
            one = np.ones(c.n)
            assert np.array_equal(Pt @ one, np.ones(f.n))
            coef = np.array([0.75, -1.5, 0.625][: wl.dim])
            gc = c.mesh.coords @ coef + 0.125
            gf = f.mesh.coords @ coef + 0.125
            assert np.array_equal(Pt @ gc, gf)
            # weights are dyadic and never refer to a coarse hanging node
            assert np.all(Pt.data * 64 == np.round(Pt.data * 64))
            assert not np.any(c.mesh.is_hanging[Pt.indices])
            # R = P^T bitwise
            assert (f.R != f.P.T).nnz == 0


@pytest.mark.parametrize("r", [2, 3, 6])
def test_prolongation_tensor_nnz(r):
    """1D P~ between uniform meshes with e_c coarse cells has 3 e_c + 1 entries;
    tensor products multiply (129^3: 193^3 = 7,189,057)."""
    f1 = M.Mesh(M.build_forest(W.c1_poisson(r)))
    fc = M.Mesh(M.build_forest(W.c1_poisson(r)).coarsened())
    Pt = transfer.prolongation(f1, fc)
    ec = 2 ** r
    assert Pt.nnz == (3 * ec + 1) ** 2
    assert (3 * 64 + 1) ** 3 == 7189057


def test_load_closed_form():
    """Constant load: sum of all entries = |Omega| * f; 2D disk load integrates the
    indicator with 3-point Gauss on every cell."""
    wl = W.c3_elasticity(1)
    m = M.Mesh(M.build_forest(wl))
    f = fem.assemble_load(m, wl)
    assert f[:, 1].sum() == pytest.approx(-1.0, abs=1e-14)
    assert np.all(f[:, [0, 2]] == 0.0)
    wl = W.c1_poisson(4)
    m = M.Mesh(M.build_forest(wl))
    f = fem.assemble_load(m, wl)
    # int 2 pi^2 sin(pi x) sin(pi y) over the unit square = 8
    assert f.sum() == pytest.approx(8.0, rel=1e-6)
