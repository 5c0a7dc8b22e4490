"""Pins for the oracle's explicit pressure-correction step (Sec. 5.3, Algorithm "The fully
discrete solution procedure for the Navier-Stokes equations") and parity of the native
generator's matrices with the oracle's.

Pins (independent of how the oracle builds its matrices):
  * lumped masses sum to the volume of the domain (eq. mass_lumping: m_i = int phi_i);
  * the Laplacians annihilate linear functions on interior rows; they are symmetric;
  * C_a g = -(d_a g) m on interior rows for linear g (integration by parts of
    (g, d_a phi_i) with phi_i vanishing on the boundary);
  * D u = (div u, phi^p_q) equals 3 m_p for u = (x, y, z) on every pressure node (div u
    = 3 and int phi^p_q = m_p) -- this fixes C, P and their product;
  * P reproduces linear functions; the pressure hierarchy satisfies the Galerkin
    identity P^T K_f P = K_c on unpinned nodes (nested tensor grids, exact integrals);
  * the grading reproduces the printed formulas at their end points and midpoints.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import multigrid as MG, ns


@pytest.fixture(scope="module")
def small():
    return ns.build_operators((4, 4, 8))


def test_grading_formulas():
    x = ns.graded_coords(32, "x")
    assert x[0] == 0.0 and x[-1] == 1.0 and np.all(np.diff(x) > 0)
    assert x[16] == pytest.approx(0.5, abs=1e-15)
    assert x[8] == pytest.approx(0.5 * (1 + np.cos(24 * np.pi / 32)), abs=1e-15)
    z = ns.graded_coords(64, "z", 2.0)
    assert z[0] == 0.0 and z[-1] == 2.0
    assert z[32] == pytest.approx(2.0 * (1 + np.sin(-np.pi / 4)), abs=1e-15)
    assert z[1] - z[0] < z[-1] - z[-2]                # finest cells at the bottom
    v = ns.refine_coords(x)
    assert len(v) == 65 and np.allclose(v[1::2], 0.5 * (x[:-1] + x[1:]), rtol=0, atol=0)


def test_lumped_masses_sum_to_volume(small):
    assert small.m_v.sum() == pytest.approx(2.0, rel=1e-13)
    assert small.m_p.sum() == pytest.approx(2.0, rel=1e-13)
    assert np.all(small.m_v > 0) and np.all(small.m_p > 0)


def _interior(X, lengths=(1.0, 1.0, 2.0)):
    return ~((X == 0.0).any(axis=1) | (X[:, 0] == lengths[0]) | (X[:, 1] == lengths[1]) | (X[:, 2] == lengths[2]))


def test_laplacian_and_derivative_matrices(small):
    X = small.coords_v
    inner = _interior(X)
    lin = 0.3 + 0.5 * X[:, 0] - 0.7 * X[:, 1] + 0.2 * X[:, 2]
    assert np.abs((small.K_v @ lin)[inner]).max() < 1e-12
    assert abs(small.K_v - small.K_v.T).max() < 1e-15
    grads = (0.5, -0.7, 0.2)
    for a in range(3):
        got = (small.C[a] @ lin)[inner]
        assert np.allclose(got, -grads[a] * small.m_v[inner], rtol=1e-12, atol=1e-15), a


def test_divergence_of_a_linear_field(small):
    """D u = sum_a G_a^T u_a = (div u, phi^p) = 3 m_p for u = (x, y, z), on every node."""
    X = small.coords_v
    du = ns.divergence(small, X.copy())
    assert np.allclose(du, 3.0 * small.m_p, rtol=1e-12, atol=1e-16)


def test_pressure_hierarchy_galerkin_and_interpolation(small):
    H = ns.pressure_hierarchy(small.xp, 3, ns.pressure_workload())
    for l in range(1, len(H.levels)):
        f, c = H.levels[l], H.levels[l - 1]
        free = ~c.mask[:, 0]
        G = (f.P.T @ f.A @ f.P - c.A).toarray()[np.ix_(free, free)]
        assert np.abs(G).max() < 1e-13 * abs(c.A).max()
        assert np.allclose(np.asarray(f.Pt.sum(axis=1)).ravel(), 1.0, rtol=0, atol=1e-15)
    # the velocity-pressure interpolation reproduces linear functions of the pressure mesh
    Xp = np.stack(np.meshgrid(*small.xp, indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    g = lambda Y: 1.0 + 2.0 * Y[:, 0] - Y[:, 1] + 0.5 * Y[:, 2]
    assert np.allclose(small.P @ g(Xp), g(small.coords_v), rtol=0, atol=1e-13)


def test_momentum_step_keeps_rest_state():
    """With no moving wall, no forcing and u = p = q = 0, the explicit step stays at 0."""
    ops = ns.build_operators((4, 4, 8))
    ops.dir_val[:] = 0.0
    u = ns.momentum(ops, np.zeros((ops.n_v, 3)), np.zeros(ops.n_p), np.zeros((ops.n_v, 3)), 1e-3, 1e-4)
    assert np.abs(u).max() == 0.0


def test_projection_reduces_divergence():
    """Steps 1-2 of the scheme: after the pressure increment the next momentum step's
    discrete divergence is smaller than the unprojected one (a sanity property of the
    pressure correction, measured over a few steps from rest)."""
    ops = ns.build_operators((4, 4, 8))
    wl = ns.pressure_workload().with_(smoother=W.SMOOTH_CHEBYSHEV, gmres_m=30)
    H = ns.pressure_hierarchy(ops.xp, 2, wl)
    mg = MG.Multigrid(H)
    out = ns.run(ops, mg, 3, 1e-3, 1e-4)
    assert all(np.isfinite(o.u).all() for o in out)
    # the pressure increment solves K_p q = -(1/k) D u^m on unpinned nodes
    du = ns.divergence(ops, out[-1].u)
    r = H.finest.A @ out[-1].q - ns.pressure_rhs(du, 1e-4, H.finest.mask[:, 0])
    assert np.linalg.norm(r) <= 1e-7 * np.linalg.norm(du / 1e-4)


@pytest.mark.parametrize("cells,levels", [((4, 4, 8), 3), ((8, 8, 16), 3)])
def test_generator_matches_oracle(cells, levels):
    from paper_2405_05047_amd import gen
    o = ns.build_operators(cells)
    g = gen.build_ns(cells, n_levels=levels)
    assert (g.n_v, g.n_p) == (o.n_v, o.n_p)

    def csr(rp, ci, v, shape):
        return sp.csr_matrix((v, ci, rp), shape=shape)

    def close(A, B):
        d = (A - B).tocsr()
        d.eliminate_zeros()
        return abs(d).max() if d.nnz else 0.0

    nv, npr = o.n_v, o.n_p
    assert close(csr(g.V_rowptr, g.V_col, g.K_val, (nv, nv)), o.K_v) <= 1e-14 * abs(o.K_v).max()
    for a in range(3):
        assert close(csr(g.V_rowptr, g.V_col, g.C_val[a], (nv, nv)), o.C[a]) <= 1e-15
        Ga = csr(g.G_rowptr, g.G_col, g.G_val[a], (nv, npr))
        assert close(Ga, o.G[a]) <= 1e-15 * max(1.0, abs(o.G[a]).max())
        assert close(csr(g.D_rowptr, g.D_col, g.D_val[a], (npr, nv)), o.G[a].T.tocsr()) <= 1e-15
    assert np.allclose(g.m_v, o.m_v, rtol=1e-15, atol=0) and np.allclose(g.m_p, o.m_p, rtol=1e-15, atol=0)
    assert np.array_equal(g.dir_mask.astype(bool), o.dir_mask) and np.array_equal(g.dir_val, o.dir_val)
    assert np.allclose(g.coords_v, o.coords_v, rtol=0, atol=1e-15)
    H = ns.pressure_hierarchy(o.xp, levels, ns.pressure_workload())
    assert len(g.levels) == len(H.levels)
    for gl, ol in zip(g.levels, H.levels):
        A = csr(gl.rowptr, gl.col, gl.val.ravel(), (gl.n, gl.n))
        assert close(A, ol.A) <= 1e-14 * abs(ol.A).max()
        assert np.array_equal(gl.mask.astype(bool), ol.mask)
        if ol.Pt is not None:
            Pg = csr(gl.p_rowptr, gl.p_col, gl.p_val, ol.Pt.shape)
            assert close(Pg, ol.Pt) <= 1e-15
