"""Native generator against the oracle (CPU): structures bit-exact, values to rounding.

The generator (C++, closed-form tensor-product element matrices, row-parallel
constrained assembly) and the oracle (NumPy, Gauss quadrature, sparse products
H^T A H) share no code; they meet only in the seeded workload."""
import numpy as np
import pytest

import workloads as W
from oracle import hierarchy as Hh
from paper_2405_05047_amd import gen

CASES = [W.c1_poisson(4), W.c2_td(band_rounds=3, uniform_rounds=1), W.c2_td(band_rounds=4),
         W.c3_elasticity(3), W.c3_adaptive("edge", 4), W.c3_adaptive("vertex", 4),
         W.c3_adaptive("face", 3), W.c4_oseen(3), W.c4_oseen(2, tall=True), W.td_time(5)] + W.batch_problems(3, max_levels=6)

# time-dependent problems: a uniform mesh, and an adaptive one with hanging nodes (band
# refinement reaching close to the Dirichlet boundary)
TIME_CASES = [W.td_time(5), W.td_time(4).with_(coarse=(8, 8), h0=0.125, rounds=(
    ("uniform",), ("band", 0.5, 0.5, 0.3, 0.05), ("band", 0.5, 0.5, 0.45, 0.06)))]


@pytest.mark.parametrize("wl", CASES, ids=[w.name for w in CASES])
def test_generator_matches_oracle(wl):
    p = gen.build(wl)
    h = Hh.build(wl)
    assert len(p.levels) == len(h.levels)
    for l, (g, o) in enumerate(zip(p.levels, h.levels)):
        assert g.n == o.n
        assert np.array_equal(g.rowptr, o.rowptr)
        assert np.array_equal(g.col, o.col)
        assert np.array_equal(g.mask.astype(bool), o.mask)
        assert np.array_equal(g.lattice[:, :wl.dim], o.mesh.coords_lat)
        assert np.array_equal(g.hang_node, o.mesh.hang_nodes)
        mo = np.sort(np.where(o.mesh.hang_masters >= 0, o.mesh.hang_masters, -1), axis=1)
        assert np.array_equal(np.sort(g.hang_master, axis=1), mo)
        r = np.repeat(np.arange(g.n), np.diff(g.rowptr))
        rowmax = np.zeros(g.n)
        np.maximum.at(rowmax, r, np.abs(o.val).reshape(len(r), -1).max(axis=1))
        err = np.abs(g.val - o.val).reshape(len(r), -1).max(axis=1) / rowmax[r]
        assert err.max() <= 1e-14
        if l > 0:
            assert np.array_equal(g.p_rowptr, o.Pt.indptr)
            assert np.array_equal(g.p_col, o.Pt.indices)
            assert np.array_equal(g.p_val, o.Pt.data)            # dyadic: bit-exact
    assert np.abs(p.b - h.b).max() <= 1e-14 * max(np.abs(h.b).max(), 1e-300)


@pytest.mark.parametrize("wl", TIME_CASES, ids=["uniform", "adaptive"])
def test_time_operators_match_oracle(wl):
    """R = [Z H^T M_l | -Z H^T A_full E_g], H and the Dirichlet DoF list of a
    time-stepping run: patterns and the dyadic / lumped-mass entries bit-exact, the
    lifting entries to rounding; the operators with their lumped mass term likewise."""
    from oracle import timestep as TS
    p = gen.build(wl, time_ops=True)
    h = Hh.build(wl)
    ops = TS.operators(h)
    t = p.time
    assert np.array_equal(t.g_idx, ops.g_idx)
    assert np.array_equal(t.R_rowptr, ops.R.indptr) and np.array_equal(t.R_col, ops.R.indices)
    scale = np.abs(ops.R.data).max()
    assert np.abs(t.R_val - ops.R.data).max() <= 1e-14 * scale
    H = ops.H.tocsr()
    H.sort_indices()
    assert np.array_equal(t.H_rowptr, H.indptr) and np.array_equal(t.H_col, H.indices)
    assert np.array_equal(t.H_val, H.data)
    assert np.array_equal(t.coords, ops.coords)
    if wl.rounds[-1][0] == "band":
        assert h.finest.mesh.is_hanging.any()
    for g, o in zip(p.levels, h.levels):
        assert np.array_equal(g.col, o.col)
        assert np.abs(g.val - o.val).max() <= 1e-14 * np.abs(o.val).max()


def test_noise_rhs_multi():
    wl = W.batch_problems(1, max_levels=5)[0]
    p = gen.build(wl, nrhs=3)
    h = Hh.build(wl, nrhs=3)
    assert p.b.shape == h.b.shape
    assert np.abs(p.b - h.b).max() <= 1e-15 * np.abs(h.b).max()


@pytest.mark.slow
def test_generator_c2_full_structure():
    """Full-size transport-diffusion workload (about 1.0e6 nodes, 9 levels)."""
    wl = W.c2_td()
    p = gen.build(wl)
    h = Hh.build(wl)
    assert [lv.n for lv in p.levels] == [lv.n for lv in h.levels]
    assert 0.95e6 <= p.finest.n <= 1.05e6
    for g, o in zip(p.levels, h.levels):
        assert np.array_equal(g.col, o.col) and np.array_equal(g.rowptr, o.rowptr)
    assert np.array_equal(p.finest.p_val, h.finest.Pt.data)


@pytest.mark.parametrize("wl", [W.c2_td(band_rounds=3, uniform_rounds=1), W.c3_adaptive("edge", 3)],
                         ids=["td_band", "edge3"])
def test_generator_cells_are_the_leaves(wl):
    """The exported leaves (input of the GPU assembly): corner a sits at the first corner
    plus the edge length along every axis whose bit is set in a, and the leaf volumes sum
    to the domain's."""
    p = gen.build(wl)
    for lv in p.levels:
        d = wl.dim
        lat = lv.lattice[:, :d].astype(np.int64)
        c0 = lat[lv.cells[:, 0]]
        step = lat[lv.cells[:, 1]][:, 0] - c0[:, 0]
        assert np.all(step > 0)
        for a in range(1 << d):
            off = np.array([(a >> k) & 1 for k in range(d)])
            assert np.array_equal(lat[lv.cells[:, a]], c0 + step[:, None] * off[None, :])
        vol = np.prod(np.array(wl.coarse[:d], float) * wl.h0)
        assert np.sum(lv.cell_size ** d) == pytest.approx(vol, rel=1e-13)
        ratio = lv.cell_size / step
        assert np.allclose(ratio, ratio[0], rtol=1e-13, atol=0)
