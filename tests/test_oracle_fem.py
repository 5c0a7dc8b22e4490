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


# ---------------------------------------------------------------- elasticity form (Sec. 5.2)
def _linear_field(m, comp, axis):
    """Nodal vector (n * 3) of the displacement u = x_axis e_comp (exact in Q1)."""
    u = np.zeros((m.n, 3))
    u[:, comp] = m.coords[:, axis]
    return u.ravel()


def test_elasticity_energy_closed_forms():
    """a(u, v) = 2 mu (eps(u), eps(v)) + lambda (div u, div v) on linear fields, which Q1
    reproduces and 2-point Gauss integrates exactly, over the unit cube (|Omega| = 1):
    uniaxial stretch u = (x, 0, 0): 2 mu + lambda; pure shear u = (y, 0, 0): mu;
    a((x,0,0), (0,y,0)) = lambda (only the div-div term couples them).  lambda != mu, so
    exchanging the two coefficients anywhere in the form fails these."""
    wl = W.c3_elasticity(1).with_(lam=1.0, mu=0.5)
    m, A = _full_matrix(wl)
    ux = _linear_field(m, 0, 0)
    uy = _linear_field(m, 1, 1)
    sh = _linear_field(m, 0, 1)
    assert ux @ A @ ux == pytest.approx(2 * wl.mu + wl.lam, abs=1e-13)
    assert sh @ A @ sh == pytest.approx(wl.mu, abs=1e-13)
    assert ux @ A @ uy == pytest.approx(wl.lam, abs=1e-13)
    # a rotation-free symmetric shear u = (y, x, 0): eps_xy = 1, energy 2 mu * 2 = 4 mu
    ss = _linear_field(m, 0, 1) + _linear_field(m, 1, 0)
    assert ss @ A @ ss == pytest.approx(4 * wl.mu, abs=1e-13)
    # dilatation u = x: eps = I, div u = 3 -> 6 mu + 9 lambda
    dl = _linear_field(m, 0, 0) + _linear_field(m, 1, 1) + _linear_field(m, 2, 2)
    assert dl @ A @ dl == pytest.approx(6 * wl.mu + 9 * wl.lam, abs=1e-12)


def test_elasticity_manufactured_O_h2():
    """Manufactured displacement u = sin(pi x) sin(pi y) sin(pi z) c (clamped cube), load
    f = -mu lap u - (lambda + mu) grad div u: the L2 error of the discrete solution falls
    by ~4 per refinement in every component (a swapped lambda/mu, a sign error in the
    load or in the form would leave an O(1) error)."""
    from scipy.sparse.linalg import cg
    from oracle import multigrid as MG
    errs = []
    for r in (2, 3, 4):
        h = Hh.build(W.elasticity_mms(r).with_(coarse_level=99))     # finest level only
        x, info = cg(h.finest.A, h.b, rtol=1e-12, maxiter=5000)      # SPD; far below the O(h^2) error
        assert info == 0
        errs.append([MG.l2_error(h, x, lambda p, c=c: fem.elasticity_mms_displacement(p)[:, c], comp=c)
                     for c in range(3)])
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios[-1] > 3.7) and np.all(ratios[-1] < 4.3), ratios
    assert errs[-1].max() < 2e-2 * np.abs(W.ELAST_MMS_DIR).max()


def test_elasticity_mms_load_matches_finite_differences():
    """The closed-form load equals -div sigma(u) formed by central differences of the
    manufactured displacement (independent of the Hessian formula)."""
    wl = W.elasticity_mms(2)
    rng = np.random.default_rng(3)
    x = rng.uniform(0.1, 0.9, (20, 3))
    d = 1e-3
    u = fem.elasticity_mms_displacement

    def grad(p):                       # (n, 3 comps, 3 dirs)
        g = np.zeros((len(p), 3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = d
            g[:, :, k] = (u(p + e) - u(p - e)) / (2 * d)
        return g

    def sigma(p):
        g = grad(p)
        eps = 0.5 * (g + g.transpose(0, 2, 1))
        tr = np.trace(eps, axis1=1, axis2=2)
        return 2 * wl.mu * eps + wl.lam * tr[:, None, None] * np.eye(3)[None]

    div = np.zeros((len(x), 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = d
        div += (sigma(x + e)[:, :, k] - sigma(x - e)[:, :, k]) / (2 * d)
    assert np.allclose(fem.elasticity_mms_load(wl, x), -div, rtol=0, atol=1e-4)


# ---------------------------------------------------------------- flow step (Oseen) blocks
def test_oseen_coupling_and_mass_blocks():
    """Signs and placement of the velocity-pressure coupling and of the mass term:
      * (div u, q) row p, columns u_k (block B) and -(p, div v) row v_k, column p
        (block C) satisfy C = -B^T entry by entry;
      * B (x e_1) = lumped masses (int phi_i, since div(x e_1) = 1) at every node;
      * C (p = x) at interior velocity rows of component 1 = +int phi_i (integration by
        parts: -(x, d_x phi_i) = (1, phi_i)), 0 for the other components;
      * 1^T A_{u_k u_k} 1 = |Omega| / dt (grad and beta.grad of a constant vanish)."""
    wl = W.c4_oseen(1)
    m, A = _full_matrix(wl)
    n = m.n
    B = np.stack([A[0::4, 1 + k::4] for k in range(3)])          # (3, n, n): row p, col u_k
    C = np.stack([A[1 + k::4, 0::4] for k in range(3)])          # row u_k, col p
    for k in range(3):
        assert np.array_equal(C[k], -B[k].T)
    lumped = fem.assemble_load(m, wl.with_(rhs=W.RHS_NOISE, block=1), np.ones((n, 1)))[:, 0]
    X = m.coords
    assert np.allclose(B[0] @ X[:, 0], lumped, rtol=0, atol=1e-15)
    assert np.allclose(B[1] @ X[:, 1], lumped, rtol=0, atol=1e-15)
    interior = ~m.boundary_mask(0b111111)
    Cp = C[0] @ X[:, 0]
    assert np.allclose(Cp[interior], lumped[interior], rtol=0, atol=1e-15)
    assert np.abs(C[1] @ X[:, 0])[interior].max() < 1e-15
    for k in range(3):
        Auu = A[1 + k::4, 1 + k::4]
        assert np.ones(n) @ Auu @ np.ones(n) == pytest.approx(1.0 / wl.dt, rel=1e-13)


def test_beta_divergence_free_and_curl():
    """beta = curl(psi) for psi = sum_k a_k sin(2 pi kappa_k.x + phi_k) e_{j_k} (scaled):
    compared with the curl of psi by central differences, and its divergence by central
    differences vanishes; the analytic bound keeps max |beta| <= 1."""
    fields = W.oseen_fields(0)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 1.0, (50, 3))
    d = 1e-5

    def psi(p):
        out = np.zeros((len(p), 3))
        for k in range(8):
            out[:, fields["j"][k]] += fields["a"][k] * np.sin(2 * np.pi * p @ fields["kappa"][k] + fields["phi"][k])
        return out * fields["scale"]

    J = np.zeros((len(x), 3, 3))           # J[:, i, k] = d psi_i / d x_k
    for k in range(3):
        e = np.zeros(3)
        e[k] = d
        J[:, :, k] = (psi(x + e) - psi(x - e)) / (2 * d)
    curl = np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], axis=1)
    beta = fem.beta_field(fields, x)
    assert np.allclose(beta, curl, rtol=0, atol=1e-8)
    div = np.zeros(len(x))
    for k in range(3):
        e = np.zeros(3)
        e[k] = d
        div += (fem.beta_field(fields, x + e)[:, k] - fem.beta_field(fields, x - e)[:, k]) / (2 * d)
    assert np.abs(div).max() < 1e-8
    g = rng.uniform(0.0, 1.0, (20000, 3))
    assert np.sqrt((fem.beta_field(fields, g) ** 2).sum(axis=1)).max() <= 1.0


@pytest.mark.parametrize("wl", [W.c2_td(band_rounds=3, uniform_rounds=1), W.c3_adaptive("edge", 3)])
def test_lumped_mass(wl):
    """Lumped masses m_i = sum_j (phi_j, phi_i) = int phi_i (mass lumping by row sums):
    the load of nodal ones equals the Gauss-integrated load of f = 1 at every node
    (hanging ones included), and they sum to |Omega|."""
    m = M.Mesh(M.build_forest(wl))
    wl1 = wl.with_(block=1, pde=W.PDE_POISSON)
    lumped = fem.assemble_load(m, wl1.with_(rhs=W.RHS_NOISE), np.ones((m.n, 1)))[:, 0]
    ref = fem.assemble_load(m, wl1.with_(rhs=W.RHS_CONST, rhs_const=(1.0,)))[:, 0]
    assert np.allclose(lumped, ref, rtol=1e-14, atol=0)
    assert lumped.sum() == pytest.approx(float(np.prod(np.array(wl.coarse) * wl.h0)), rel=1e-14)
