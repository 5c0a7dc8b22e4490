"""Explicit pressure-correction step for the incompressible Navier-Stokes equations
(oracle, test-only).

Sec. 5.3, Algorithm "The fully discrete solution procedure for the Navier-Stokes
equations": Q1-iso-Q2 / Q1 elements (velocity Q1 on the once uniformly refined mesh
Omega_{h/2}, pressure Q1 on Omega_h), the lumped mass of eq. mass_lumping, and the
convective term by interpolation of u (x) u (eq. conv_mass_lumping), evaluated with the
nodal products of eq. tp and the matrices C_{h,a} = (phi_j, d_a phi_i) of eq. multC.
Per time step m, with s = p^{m-1} + q^{m-1}:

  Step 1 (explicit momentum), free velocity DoFs (i, c):
      m_i u^m_ic = m_i (f_ic + u_ic / k) - nu (K u_c)_i + sum_a (C_a (u_a * u_c))_i
                   + (G_c s)_i,     G_c = (phi^p_q, d_c phi^v_i);
      Dirichlet DoFs take their boundary values.
  Step 2 (pressure Poisson): (grad q, grad phi) = -(1/k) (div u^m, phi):
      K_p q = -(1/k) D u^m,  D u = sum_a G_a^T u_a,
      solved by FGMRES preconditioned by the V-cycle (Sec. 4.2) on the pressure mesh
      hierarchy, one pressure node pinned to zero on every level (the Neumann problem
      fixes q up to a constant; the right-hand side is compatible, so the pinned
      equation holds by itself).
  Step 3 (pressure update): m^p p^m = m^p (p^{m-1} + q^m) - nu D u^m.

Every matrix is a sum of Kronecker products of one-dimensional P1 matrices on the
graded coordinates (Q1 on a tensor grid of boxes), which is exact: the mass, stiffness
and first-derivative matrices of the hat functions, and the coarse hat functions
written in the fine ones by their nodal interpolation P (nested grids), so that the
mixed pressure / velocity integrals are G_a = C_a P.

Node numbering is lexicographic with x fastest: node (i, j, k) = (k ny + j) nx + i
(nx, ny, nz node counts); velocity vectors are node-major / component-minor.

Readings (the paper is silent or garbled):
  * the viscous term enters with the physical sign: nu (grad u, grad chi) on the left,
    so -nu K u on the right-hand side of Step 1;
  * the grading of z is scaled by the domain height 2 so that the mesh covers
    (0,1) x (0,1) x (0,2); x and y use the printed cosine grading (ascending order);
  * the velocity mesh is the equidistant refinement: one midpoint inserted per cell and
    direction.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse as sp

import workloads as W
from . import multigrid as MG


# ------------------------------------------------------------------ coordinates
def graded_coords(n_cells: int, axis: str, length: float = 1.0) -> np.ndarray:
    """Sec. 5.3 grading: x, y: (1 - cos(i pi / N)) / 2 (the printed points, ascending);
    z: 1 + sin((k - N) pi / (2 N)) scaled by the domain length."""
    i = np.arange(n_cells + 1, dtype=np.float64)
    if axis in ("x", "y"):
        c = 0.5 * (1.0 - np.cos(i * np.pi / n_cells))
    else:
        c = 1.0 + np.sin((i - n_cells) * np.pi / (2.0 * n_cells))
    c[0], c[-1] = 0.0, 1.0
    return length * c


def refine_coords(c: np.ndarray) -> np.ndarray:
    """Equidistant refinement: the midpoint of every cell inserted."""
    out = np.empty(2 * len(c) - 1)
    out[0::2] = c
    out[1::2] = 0.5 * (c[:-1] + c[1:])
    return out


# ------------------------------------------------------------------ 1D P1 matrices
def p1_matrices(x: np.ndarray):
    """Mass M, stiffness K, derivative C (C_ij = (phi_j, phi_i')) and lumped mass m of the
    hat functions on the grid x, cell by cell from the exact element matrices."""
    n = len(x)
    h = np.diff(x)
    rows, cols = [], []
    vm, vk, vc = [], [], []
    for e in range(n - 1):
        he = h[e]
        loc = [e, e + 1]
        Me = he / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
        Ke = 1.0 / he * np.array([[1.0, -1.0], [-1.0, 1.0]])
        # (phi_j, phi_i'): phi_i' = -1/h (left), +1/h (right); int phi_j = h / 2
        Ce = 0.5 * np.array([[-1.0, -1.0], [1.0, 1.0]])
        for a in range(2):
            for b in range(2):
                rows.append(loc[a])
                cols.append(loc[b])
                vm.append(Me[a, b])
                vk.append(Ke[a, b])
                vc.append(Ce[a, b])
    M = sp.csr_matrix((vm, (rows, cols)), shape=(n, n))
    K = sp.csr_matrix((vk, (rows, cols)), shape=(n, n))
    C = sp.csr_matrix((vc, (rows, cols)), shape=(n, n))
    m = np.zeros(n)
    m[:-1] += h / 2
    m[1:] += h / 2
    return M, K, C, m


def interp_1d(xc: np.ndarray, xf: np.ndarray) -> sp.csr_matrix:
    """Nodal interpolation of the coarse hats at the fine nodes (fine x coarse)."""
    rows, cols, vals = [], [], []
    for i, x in enumerate(xf):
        e = min(np.searchsorted(xc, x, side="right") - 1, len(xc) - 2)
        t = (x - xc[e]) / (xc[e + 1] - xc[e])
        for j, w in ((e, 1.0 - t), (e + 1, t)):
            if w != 0.0:
                rows.append(i)
                cols.append(j)
                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(xf), len(xc)))


def kron3(az, ay, ax) -> sp.csr_matrix:
    """Operator on the lexicographic (z, y, x) node numbering with x fastest."""
    return sp.kron(az, sp.kron(ay, ax, format="csr"), format="csr").tocsr()


# ------------------------------------------------------------------ operators
@dataclasses.dataclass
class NSOperators:
    xp: List[np.ndarray]           # pressure-mesh coordinates per axis
    xv: List[np.ndarray]           # velocity-mesh coordinates per axis
    n_v: int
    n_p: int
    m_v: np.ndarray                # lumped velocity mass (n_v)
    m_p: np.ndarray                # lumped pressure mass (n_p)
    K_v: sp.csr_matrix             # velocity Laplacian (grad phi_j, grad phi_i)
    C: List[sp.csr_matrix]         # C_a = (phi_j, d_a phi_i), a = x, y, z
    P: sp.csr_matrix               # pressure hats in velocity hats (n_v x n_p)
    G: List[sp.csr_matrix]         # G_a = C_a P = (phi^p_q, d_a phi^v_i)  (n_v x n_p)
    K_p: sp.csr_matrix             # pressure Laplacian
    dir_mask: np.ndarray           # (n_v, 3) bool: Dirichlet velocity DoFs
    dir_val: np.ndarray            # (n_v, 3) boundary values
    coords_v: np.ndarray           # (n_v, 3)


def build_operators(cells=(32, 32, 64), lengths=(1.0, 1.0, 2.0)) -> NSOperators:
    xp = [graded_coords(cells[0], "x", lengths[0]), graded_coords(cells[1], "y", lengths[1]),
          graded_coords(cells[2], "z", lengths[2])]
    xv = [refine_coords(c) for c in xp]
    mats_v = [p1_matrices(c) for c in xv]
    mats_p = [p1_matrices(c) for c in xp]
    (Mx, Kx, Cx, mx), (My, Ky, Cy, my), (Mz, Kz, Cz, mz) = mats_v
    K_v = kron3(Mz, My, Kx) + kron3(Mz, Ky, Mx) + kron3(Kz, My, Mx)
    C = [kron3(Mz, My, Cx), kron3(Mz, Cy, Mx), kron3(Cz, My, Mx)]
    m_v = np.kron(mz, np.kron(my, mx))
    (Mpx, Kpx, _, mpx), (Mpy, Kpy, _, mpy), (Mpz, Kpz, _, mpz) = mats_p
    K_p = kron3(Mpz, Mpy, Kpx) + kron3(Mpz, Kpy, Mpx) + kron3(Kpz, Mpy, Mpx)
    m_p = np.kron(mpz, np.kron(mpy, mpx))
    Px, Py, Pz = (interp_1d(c, f) for c, f in zip(xp, xv))
    P = kron3(Pz, Py, Px)
    G = [(Ca @ P).tocsr() for Ca in C]
    nx, ny, nz = (len(c) for c in xv)
    X = np.stack(np.meshgrid(xv[0], xv[1], xv[2], indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    on = ((X[:, 0] == 0.0) | (X[:, 0] == lengths[0]) | (X[:, 1] == 0.0) | (X[:, 1] == lengths[1])
          | (X[:, 2] == 0.0) | (X[:, 2] == lengths[2]))
    dir_mask = np.repeat(on[:, None], 3, axis=1)
    dir_val = np.zeros((len(X), 3))
    dir_val[X[:, 0] == lengths[0], 1] = 1.0                # the moving wall x = 1: u = (0, 1, 0)
    return NSOperators(xp=xp, xv=xv, n_v=nx * ny * nz, n_p=K_p.shape[0], m_v=m_v, m_p=m_p, K_v=K_v.tocsr(),
                       C=[c.tocsr() for c in C], P=P, G=G, K_p=K_p.tocsr(), dir_mask=dir_mask,
                       dir_val=dir_val, coords_v=X)


# ------------------------------------------------------------------ pressure hierarchy
@dataclasses.dataclass
class PLevel:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray                # (nnz, 1, 1)
    A: sp.csr_matrix
    mask: np.ndarray               # (n, 1) bool: the pinned node
    Pt: sp.csr_matrix = None
    P: sp.csr_matrix = None
    R: sp.csr_matrix = None

    @property
    def ndof(self):
        return self.A.shape[0]


@dataclasses.dataclass
class PHierarchy:
    wl: W.Workload
    levels: List[PLevel]

    @property
    def L(self):
        return len(self.levels) - 1

    @property
    def finest(self):
        return self.levels[-1]


def pressure_level(coords) -> PLevel:
    mats = [p1_matrices(c) for c in coords]
    (Mx, Kx, _, _), (My, Ky, _, _), (Mz, Kz, _, _) = mats
    A = (kron3(Mz, My, Kx) + kron3(Mz, Ky, Mx) + kron3(Kz, My, Mx)).tocsr()
    n = A.shape[0]
    mask = np.zeros((n, 1), bool)
    mask[0] = True                                        # pinned node (0, 0, 0)
    Z = sp.diags((~mask[:, 0]).astype(np.float64))
    A = (Z @ A @ Z + sp.diags(mask[:, 0].astype(np.float64))).tocsr()
    A.sort_indices()
    return PLevel(n=n, rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32),
                  val=A.data.reshape(-1, 1, 1).copy(), A=A, mask=mask)


def pressure_hierarchy(xp, n_levels: int, wl: W.Workload) -> PHierarchy:
    """Levels by uniform coarsening of the graded tensor grid (every other coordinate);
    the prolongation is the tensor product of 1D nodal interpolations."""
    coords = [list(xp)]
    for _ in range(n_levels - 1):
        coords.append([c[0::2] for c in coords[-1]])
    coords = coords[::-1]
    levels = [pressure_level(c) for c in coords]
    for l in range(1, len(levels)):
        f, c = levels[l], levels[l - 1]
        Pt = kron3(*(interp_1d(cc, ff) for cc, ff in zip(coords[l - 1][::-1], coords[l][::-1])))
        f.Pt = Pt
        Mf = sp.diags((~f.mask[:, 0]).astype(np.float64))
        Mc = sp.diags((~c.mask[:, 0]).astype(np.float64))
        f.P = (Mf @ Pt @ Mc).tocsr()
        f.R = f.P.T.tocsr()
    return PHierarchy(wl=wl, levels=levels)


def pressure_workload(rtol=1e-8) -> W.Workload:
    """Solver settings of the pressure Poisson problem (GMRES + V-cycle, Sec. 5.3)."""
    return W.Workload(name="ns_pressure", dim=3, coarse=(1, 1, 1), h0=1.0, rounds=(), pde=W.PDE_POISSON,
                      block=1, omega=0.8, nu1=2, nu2=2, outer=W.OUTER_FGMRES, gmres_m=10, rtol=rtol,
                      maxit=400)


# ------------------------------------------------------------------ Algorithm steps
def momentum(ops: NSOperators, u: np.ndarray, s: np.ndarray, f: np.ndarray, nu: float, k: float) -> np.ndarray:
    """Step 1: u (n_v, 3) at t_{m-1}, s = p + q (n_p), f (n_v, 3) -> u^m (n_v, 3)."""
    rhs = ops.m_v[:, None] * (f + u / k)
    for c in range(3):
        rhs[:, c] -= nu * (ops.K_v @ u[:, c])
        for a in range(3):
            rhs[:, c] += ops.C[a] @ (u[:, a] * u[:, c])      # eq. tp, then eq. multC
        rhs[:, c] += ops.G[c] @ s
    out = k * rhs / ops.m_v[:, None]
    return np.where(ops.dir_mask, ops.dir_val, out)


def divergence(ops: NSOperators, u: np.ndarray) -> np.ndarray:
    """D u = sum_a G_a^T u_a = (div u_h, phi^p_q) for every pressure node q."""
    return sum(ops.G[a].T @ u[:, a] for a in range(3))


def pressure_rhs(du: np.ndarray, k: float, pinned: np.ndarray) -> np.ndarray:
    return np.where(pinned, 0.0, -du / k)


def pressure_update(ops: NSOperators, p: np.ndarray, q: np.ndarray, du: np.ndarray, nu: float) -> np.ndarray:
    """Step 3 with the lumped pressure mass."""
    return p + q - nu * du / ops.m_p


@dataclasses.dataclass
class StepOut:
    u: np.ndarray
    p: np.ndarray
    q: np.ndarray
    iters: int


def run(ops: NSOperators, mg: MG.Multigrid, steps: int, nu: float, k: float, u0=None, f=None) -> List[StepOut]:
    """Algorithm steps 1-3 for `steps` time steps from u0 (default 0, p = q = 0); each
    pressure solve starts from the previous q."""
    u = np.zeros((ops.n_v, 3)) if u0 is None else u0.copy()
    u = np.where(ops.dir_mask, ops.dir_val, u)
    p = np.zeros(ops.n_p)
    q = np.zeros(ops.n_p)
    f = np.zeros((ops.n_v, 3)) if f is None else f
    pinned = mg.h.finest.mask[:, 0]
    out = []
    for _ in range(steps):
        u = momentum(ops, u, p + q, f, nu, k)
        du = divergence(ops, u)
        q, st = mg.solve(pressure_rhs(du, k, pinned), x0=q)
        p = pressure_update(ops, p, q, du, nu)
        out.append(StepOut(u.copy(), p.copy(), q.copy(), st.iters))
    return out
