"""Q1 finite elements on axis-aligned boxes: element matrices, assembly, constraints.

Oracle (test-only).  Follows Sec. 2.1 (equal-order Q^r elements with r = 1, nodal
blocks A_ij in R^{n_c x n_c}, vectors with n_c components per node) and Sec. 2.2 (the
hanging-node matrix H: the assembled residual is multiplied by H^T; the solution is
recovered as H x).  Element integrals use tensor Gauss rules: 2 points per direction for
bilinear forms (exact for the constant-coefficient forms on boxes), 3 points for loads.

Readings (the paper gives no formulas for these):
  * Constrained degrees of freedom (hanging nodes: all components; Dirichlet nodes: the
    listed components) are eliminated symmetrically:
        A = Z (H^T A_full H) Z + I_C,   b = Z H^T (f - A_full g),  g = 0 here,
    Z = identity with zeros on constrained rows.  The block pattern is symbolic:
    block (i, j), i != j, is stored when (H^T N H)_ij != 0 for the node pattern N of
    A_full and both nodes carry at least one free component; diagonal blocks always.
  * Streamline stabilisation (transport-diffusion): tau_K (b.grad u, b.grad v)_K on the
    left and tau_K (f, b.grad v)_K on the right, tau_K = h_K/(2|b|) (coth Pe - 1/Pe),
    Pe = |b| h_K / (2 eps), h_K = s |b| / max_k |b_k| (chord through the centre of a
    square of side s along b).
  * Lumped mass term (time-dependent problems, eq. mass_lumping): c * M_l with
    M_l = diag(m_i), m_i = sum_j (phi_j, phi_i) = int phi_i, added element by element as
    c |K| / 2^dim on the diagonal of each cell's corners (before the constraints).
  * Flow step (4 components p, u, v, w): (1/dt)(u,v) + nu (grad u, grad v)
    + (beta.grad u, v) - (p, div v) + (div u, q) + sum_K delta_K (grad p, grad q)_K,
    delta_K = alpha0 / (nu / s^2 + |beta(x_K)| / s + 1/dt), beta at the 2-point
    Gauss points for the convection term and at the cell centre for delta_K.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp

import workloads as W


# ------------------------------------------------------------------ quadrature / basis
def gauss01(npts: int):
    """Gauss-Legendre points and weights on [0, 1]."""
    if npts == 2:
        g = 0.5 / math.sqrt(3.0)
        return np.array([0.5 - g, 0.5 + g]), np.array([0.5, 0.5])
    if npts == 3:
        g = 0.5 * math.sqrt(0.6)
        return np.array([0.5 - g, 0.5, 0.5 + g]), np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])
    raise ValueError(npts)


def corner_offsets(dim: int) -> np.ndarray:
    """Local corner a -> offset (o_x, o_y[, o_z]) in {0,1}^dim, a = o_x + 2 o_y + 4 o_z."""
    return np.array([[(a >> k) & 1 for k in range(dim)] for a in range(1 << dim)], np.int64)


def tensor_rule(dim: int, npts: int):
    """Reference points (nq, dim) on [0,1]^dim and weights (nq,)."""
    p, w = gauss01(npts)
    pts, wts = [], []
    for idx in itertools.product(range(npts), repeat=dim):
        pts.append([p[i] for i in idx])
        wts.append(np.prod([w[i] for i in idx]))
    return np.array(pts), np.array(wts)


def ref_basis(dim: int, pts: np.ndarray):
    """Q1 basis values (nq, nb) and reference gradients (nq, nb, dim) at `pts`."""
    off = corner_offsets(dim)
    nq, nb = len(pts), len(off)
    phi = np.ones((nq, nb))
    dphi = np.ones((nq, nb, dim))
    for a in range(nb):
        for k in range(dim):
            hat = pts[:, k] if off[a, k] else 1.0 - pts[:, k]
            dhat = 1.0 if off[a, k] else -1.0
            phi[:, a] *= hat
            for m in range(dim):
                dphi[:, a, m] *= dhat if m == k else hat
    return phi, dphi


def langevin(pe):
    """coth(Pe) - 1/Pe, with its series for small Pe (the direct form cancels there)."""
    pe = np.asarray(pe, dtype=np.float64)
    small = pe < 1e-2
    with np.errstate(divide="ignore", invalid="ignore"):
        direct = 1.0 / np.tanh(pe) - 1.0 / pe
    series = pe / 3.0 - pe ** 3 / 45.0 + 2.0 * pe ** 5 / 945.0
    return np.where(small, series, direct)


def supg_tau(wl, s):
    """Stabilisation parameter tau_K for square cells of side s (see module docstring);
    zero when the workload switches the stabilisation off."""
    b = np.asarray(wl.bvec, dtype=np.float64)
    nb = math.sqrt(float(b @ b))
    if nb == 0.0 or not wl.supg:
        return np.zeros_like(np.asarray(s, dtype=np.float64))
    hk = np.asarray(s, dtype=np.float64) * nb / float(np.max(np.abs(b)))
    pe = nb * hk / (2.0 * wl.eps)
    return hk / (2.0 * nb) * langevin(pe)


# ------------------------------------------------------------------ coefficient fields
def beta_field(fields, x):
    """Seeded divergence-free convection field at points x (n, 3)."""
    out = np.zeros((len(x), 3))
    for k in range(8):
        e = np.zeros(3)
        e[fields["j"][k]] = 1.0
        cr = np.cross(fields["kappa"][k], e)
        ang = 2.0 * math.pi * (x @ fields["kappa"][k]) + fields["phi"][k]
        out += (fields["a"][k] * 2.0 * math.pi * np.cos(ang))[:, None] * cr[None, :]
    return out * fields["scale"]


def forcing_field(fields, x):
    """Seeded smooth velocity forcing at points x (n, 3)."""
    out = np.zeros((len(x), 3))
    for m in range(4):
        ang = 2.0 * math.pi * (x @ fields["fk"][m]) + fields["fphi"][m]
        out[:, fields["fi"][m]] += fields["fc"][m] * np.sin(ang)
    return out


def elasticity_mms_displacement(x):
    """Manufactured displacement u = sin(pi x) sin(pi y) sin(pi z) c, c = ELAST_MMS_DIR,
    at points x (n, 3); zero on the boundary of the unit cube."""
    s = np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2])
    return s[:, None] * np.asarray(W.ELAST_MMS_DIR)[None, :]


def elasticity_mms_load(wl, x):
    """Body load f = -div sigma(u) of the manufactured displacement, with
    sigma = 2 mu eps(u) + lambda div(u) I (Sec. 5.2), i.e. f = -mu lap u - (lambda + mu)
    grad div u.  For u = s c with s = sin(pi x) sin(pi y) sin(pi z): lap u = -3 pi^2 s c
    and grad div u = Hess(s) c, Hess(s)_ii = -pi^2 s, Hess(s)_ij = pi^2 cos cos sin."""
    c = np.asarray(W.ELAST_MMS_DIR)
    sn = np.sin(np.pi * x)
    cs = np.cos(np.pi * x)
    s = sn[:, 0] * sn[:, 1] * sn[:, 2]
    hess = np.empty((len(x), 3, 3))
    for i in range(3):
        for j in range(3):
            if i == j:
                hess[:, i, j] = -np.pi ** 2 * s
            else:
                k = 3 - i - j
                hess[:, i, j] = np.pi ** 2 * cs[:, i] * cs[:, j] * sn[:, k]
    lap = -3.0 * np.pi ** 2 * s[:, None] * c[None, :]
    return -wl.mu * lap - (wl.lam + wl.mu) * np.einsum("nij,j->ni", hess, c)


# ------------------------------------------------------------------ element matrices
def element_matrices(wl, s, x0):
    """Element matrices Ke (ne, nb, nb, b, b) for boxes of side s (ne,) with lower
    corners x0 (ne, dim).  Ke[e, a, c_b, ci, cj]: test corner a / component ci, trial
    corner c_b / component cj.  Integrals by the 2-point tensor Gauss rule."""
    dim, b = wl.dim, wl.block
    qp, qw = tensor_rule(dim, 2)
    phi, dphi_ref = ref_basis(dim, qp)
    nb = phi.shape[1]
    s = np.asarray(s, dtype=np.float64)
    ne = len(s)
    jac = s ** dim                                     # |det J|
    # physical gradients: (ne, nq, nb, dim)
    dphi = dphi_ref[None, :, :, :] / s[:, None, None, None]
    wq = qw[None, :] * jac[:, None]                    # (ne, nq)
    Ke = np.zeros((ne, nb, nb, b, b))
    grad_grad = np.einsum("eq,eqak,eqbk->eab", wq, dphi, dphi)       # (grad phi_b, grad phi_a)
    if wl.pde == W.PDE_POISSON:
        Ke[:, :, :, 0, 0] = grad_grad
    elif wl.pde == W.PDE_TD:
        bv = np.asarray(wl.bvec, dtype=np.float64)
        bgrad = np.einsum("k,eqak->eqa", bv, dphi)                    # b . grad phi
        conv = np.einsum("eq,eqb,qa->eab", wq, bgrad, phi)           # (b.grad phi_b, phi_a)
        tau = supg_tau(wl, s)
        stab = np.einsum("eq,eqb,eqa->eab", wq, bgrad, bgrad) * tau[:, None, None]
        Ke[:, :, :, 0, 0] = wl.eps * grad_grad + conv + stab
    elif wl.pde == W.PDE_ELASTICITY:
        # 2 mu (eps(u), eps(v)) + lambda (div u, div v), u = phi_b e_cj, v = phi_a e_ci
        for ci in range(dim):
            for cj in range(dim):
                t1 = np.einsum("eq,eqa,eqb->eab", wq, dphi[..., cj], dphi[..., ci])   # d_cj phi_a d_ci phi_b
                t2 = np.einsum("eq,eqa,eqb->eab", wq, dphi[..., ci], dphi[..., cj])   # d_ci phi_a d_cj phi_b
                Ke[:, :, :, ci, cj] = wl.mu * t1 + wl.lam * t2
                if ci == cj:
                    Ke[:, :, :, ci, cj] += wl.mu * grad_grad
    elif wl.pde == W.PDE_OSEEN:
        fields = W.oseen_fields(wl.seed)
        xq = x0[:, None, :] + s[:, None, None] * qp[None, :, :]     # (ne, nq, 3)
        beta = beta_field(fields, xq.reshape(-1, 3)).reshape(ne, len(qp), 3)
        mass = np.einsum("eq,qa,qb->eab", wq, phi, phi)
        bgrad = np.einsum("eqk,eqbk->eqb", beta, dphi)
        conv = np.einsum("eq,eqb,qa->eab", wq, bgrad, phi)
        xc = x0 + 0.5 * s[:, None]
        bc = beta_field(fields, xc)
        bnorm = np.sqrt(np.sum(bc * bc, axis=1))
        delta = wl.pspg_alpha / (wl.nu / (s * s) + bnorm / s + 1.0 / wl.dt)
        Ke[:, :, :, 0, 0] = delta[:, None, None] * grad_grad
        for k in range(3):
            # (div u, q): row p, column u_k:  d_k phi_b * phi_a
            Ke[:, :, :, 0, 1 + k] = np.einsum("eq,eqb,qa->eab", wq, dphi[..., k], phi)
            # -(p, div v): row v_k, column p: -phi_b d_k phi_a
            Ke[:, :, :, 1 + k, 0] = -np.einsum("eq,qb,eqa->eab", wq, phi, dphi[..., k])
            Ke[:, :, :, 1 + k, 1 + k] = mass / wl.dt + wl.nu * grad_grad + conv
    else:
        raise ValueError(wl.pde)
    if wl.mass_coef != 0.0:
        lumped = wl.mass_coef * jac / nb                # c |K| / 2^dim per corner
        for a in range(nb):
            for ci in range(b):
                Ke[:, a, a, ci, ci] += lumped
    return Ke


def element_loads(wl, s, x0, xi=None, node_ids=None):
    """Element load vectors Fe (ne, nb, b) by the 3-point tensor Gauss rule."""
    dim, b = wl.dim, wl.block
    qp, qw = tensor_rule(dim, 3)
    phi, dphi_ref = ref_basis(dim, qp)
    s = np.asarray(s, dtype=np.float64)
    ne = len(s)
    wq = qw[None, :] * (s ** dim)[:, None]
    xq = x0[:, None, :] + s[:, None, None] * qp[None, :, :]
    Fe = np.zeros((ne, phi.shape[1], b))
    if wl.rhs == W.RHS_SINSIN:
        f = 2.0 * math.pi ** 2 * np.sin(math.pi * xq[..., 0]) * np.sin(math.pi * xq[..., 1])
        Fe[..., 0] = np.einsum("eq,eq,qa->ea", wq, f, phi)
    elif wl.rhs == W.RHS_DISK:
        dx = xq[..., 0] - 0.5
        dy = xq[..., 1] - 0.5
        f = np.where(dx * dx + dy * dy < 0.3 * 0.3, 1.0, 0.0)
        Fe[..., 0] = np.einsum("eq,eq,qa->ea", wq, f, phi)
        if wl.pde == W.PDE_TD:
            bv = np.asarray(wl.bvec, dtype=np.float64)
            dphi = dphi_ref[None] / s[:, None, None, None]
            bgrad = np.einsum("k,eqak->eqa", bv, dphi)
            tau = supg_tau(wl, s)
            Fe[..., 0] += tau[:, None] * np.einsum("eq,eq,eqa->ea", wq, f, bgrad)
    elif wl.rhs == W.RHS_CONST:
        for c in range(b):
            Fe[..., c] = wl.rhs_const[c] * np.einsum("eq,qa->ea", wq, phi)
    elif wl.rhs == W.RHS_FIELD:
        fields = W.oseen_fields(wl.seed)
        fv = forcing_field(fields, xq.reshape(-1, 3)).reshape(ne, len(qp), 3)
        for k in range(3):
            Fe[..., 1 + k] = np.einsum("eq,eq,qa->ea", wq, fv[..., k], phi)
    elif wl.rhs == W.RHS_ELAST_MMS:
        fv = elasticity_mms_load(wl, xq.reshape(-1, 3)).reshape(ne, len(qp), 3)
        for k in range(3):
            Fe[..., k] = np.einsum("eq,eq,qa->ea", wq, fv[..., k], phi)
    elif wl.rhs in (W.RHS_NOISE, W.RHS_NONE):
        pass
    else:
        raise ValueError(wl.rhs)
    return Fe


# ------------------------------------------------------------------ assembly
def leaf_table(mesh):
    """Per-leaf side length, lower corner (physical) and corner node ids (ne, nb)."""
    f = mesh.forest
    dep, anc = f.leaves()
    size = (1 << (f.D - dep)).astype(np.int64)
    off = corner_offsets(f.dim)
    corners = anc[:, None, :] + off[None, :, :] * size[:, None, None]   # (ne, nb, dim) lattice
    lin = np.ravel_multi_index(tuple(corners[..., k] for k in reversed(range(f.dim))), f.vshape)
    nodes = mesh.node_of_lin[lin]
    assert np.all(nodes >= 0)
    return size * f.hf, anc * f.hf, nodes


def lumped_mass(mesh) -> np.ndarray:
    """m_i = sum_j (phi_j, phi_i) = int phi_i per node (all nodes, hanging included): each
    cell gives |K| / 2^dim to each of its corners (eq. mass_lumping)."""
    s, x0, nodes = leaf_table(mesh)
    dim = mesh.dim
    return np.bincount(nodes.ravel(), weights=np.repeat(s ** dim / (1 << dim), nodes.shape[1]),
                       minlength=mesh.n)


def dof_mask(mesh, wl) -> np.ndarray:
    """(n, b) bool: constrained = hanging node (all components) or Dirichlet component."""
    m = np.zeros((mesh.n, wl.block), bool)
    m[mesh.is_hanging, :] = True
    on = mesh.boundary_mask(wl.dir_faces)
    for c in range(wl.block):
        if wl.dir_comps >> c & 1:
            m[on, c] = True
    return m


def assemble_full(mesh, wl, chunk: int = 1 << 15):
    """Unconstrained global matrix over all nodes, including hanging ones.

    Returns (keys, vals): sorted unique node-pair keys i*n + j and the summed b x b
    blocks (nnzb, b, b)."""
    s, x0, nodes = leaf_table(mesh)
    n, nb, b = mesh.n, nodes.shape[1], wl.block
    rows = np.repeat(nodes, nb, axis=1)              # (ne, nb*nb): a-major
    cols = np.tile(nodes, (1, nb))
    keys = rows.astype(np.int64) * n + cols
    ukeys, inv = np.unique(keys.ravel(), return_inverse=True)
    inv = inv.reshape(keys.shape)
    vals = np.zeros((len(ukeys), b, b))
    for lo in range(0, len(s), chunk):
        hi = min(lo + chunk, len(s))
        Ke = element_matrices(wl, s[lo:hi], x0[lo:hi]).reshape(hi - lo, nb * nb, b, b)
        idx = inv[lo:hi].ravel()
        for ci in range(b):
            for cj in range(b):
                vals[:, ci, cj] += np.bincount(idx, weights=Ke[:, :, ci, cj].ravel(),
                                               minlength=len(ukeys))
    return ukeys, vals


def assemble_load(mesh, wl, xi=None) -> np.ndarray:
    """Unconstrained load vector over all nodes (n, b)."""
    n, b = mesh.n, wl.block
    f = np.zeros((n, b))
    if wl.rhs == W.RHS_NOISE:
        # lumped mass times nodal noise: m_i = sum over cells touching i of |K| / 2^dim
        s, x0, nodes = leaf_table(mesh)
        m = np.bincount(nodes.ravel(), weights=np.repeat(s ** wl.dim / (1 << wl.dim), nodes.shape[1]),
                        minlength=n)
        return (m[:, None] * xi[:, :b])
    s, x0, nodes = leaf_table(mesh)
    Fe = element_loads(wl, s, x0)
    for c in range(b):
        f[:, c] = np.bincount(nodes.ravel(), weights=Fe[..., c].ravel(), minlength=n)
    return f


def _keys_to_csr(keys, n, data=None):
    r = keys // n
    c = keys % n
    if data is None:
        data = np.ones(len(keys))
    return sp.csr_matrix((data, (r, c)), shape=(n, n))


def constrain(mesh, wl, keys, vals):
    """A = Z (H^T A_full H) Z + I_C as node-level BSR arrays (Sec. 2.2 and the readings
    in the module docstring).  Returns (rowptr, col, val (nnzb, b, b))."""
    n, b = mesh.n, wl.block
    H = mesh.H.tocsr()
    mask = dof_mask(mesh, wl)
    free_node = ~mask.all(axis=1)
    # symbolic pattern from the node pattern of A_full
    N = _keys_to_csr(keys, n)
    Np = (H.T @ N @ H).tocsr()
    Np.sum_duplicates()
    Np.sort_indices()
    r = np.repeat(np.arange(n), np.diff(Np.indptr))
    c = Np.indices.astype(np.int64)
    keep = (r == c) | (free_node[r] & free_node[c])
    pk = r[keep] * n + c[keep]
    pk = np.union1d(pk, np.arange(n, dtype=np.int64) * (n + 1))   # every diagonal block
    pr, pc = pk // n, pk % n
    out = np.zeros((len(pk), b, b))
    for ci in range(b):
        for cj in range(b):
            Acc = _keys_to_csr(keys, n, vals[:, ci, cj])
            Ac = (H.T @ Acc @ H).tocoo()
            ak = Ac.row.astype(np.int64) * n + Ac.col
            pos = np.searchsorted(pk, ak)
            ok = (pos < len(pk))
            ok[ok] &= pk[pos[ok]] == ak[ok]
            # every structurally nonzero entry whose row and column are free must be stored
            fr = ~mask[Ac.row, ci] & ~mask[Ac.col, cj]
            if np.any(fr & ~ok & (Ac.data != 0.0)):
                raise AssertionError("free entry outside the symbolic pattern")
            sel = ok & fr
            out[pos[sel], ci, cj] = Ac.data[sel]
            diag = (pr == pc) & mask[pr, ci] if ci == cj else None
            if diag is not None:
                out[diag, ci, cj] = 1.0
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(pr, minlength=n), out=rowptr[1:])
    return rowptr, pc, out


def constrain_load(mesh, wl, f_full):
    """b = Z H^T f (g = 0)."""
    bvec = mesh.H.T @ f_full
    bvec[dof_mask(mesh, wl)] = 0.0
    return bvec


def bsr_to_csr(rowptr, col, val) -> sp.csr_matrix:
    """Scalar CSR of a node-level BSR matrix (dof index = node * b + component)."""
    n = len(rowptr) - 1
    b = val.shape[1]
    return sp.bsr_matrix((val, col, rowptr), shape=(n * b, n * b)).tocsr()
