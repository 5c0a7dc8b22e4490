"""ctypes binding of the native problem generator (libmggen.so, include/mggen.h).

Argument marshalling only: the meshing, coarsening, assembly and transfer construction
all run in the C++ library.  `build(wl)` returns a `Problem` whose levels hold numpy
copies of the library's arrays (level 0 = coarsest).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import List, Optional

import numpy as np

import workloads as W
from ._native import load

_lib = None


class Round(C.Structure):
    _fields_ = [("kind", C.c_int32), ("axes", C.c_int32), ("p", C.c_double * 4)]


class Config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("coarse", C.c_int32 * 3), ("h0", C.c_double),
                ("n_rounds", C.c_int32), ("rounds", C.POINTER(Round)),
                ("pde", C.c_int32), ("block", C.c_int32), ("eps", C.c_double),
                ("bvec", C.c_double * 3), ("lam", C.c_double), ("mu", C.c_double),
                ("nu", C.c_double), ("dt", C.c_double), ("pspg_alpha", C.c_double),
                ("dir_faces", C.c_int32), ("dir_comps", C.c_int32), ("rhs", C.c_int32),
                ("rhs_const", C.c_double * 4),
                ("kappa", (C.c_double * 3) * 8), ("a", C.c_double * 8), ("phi", C.c_double * 8),
                ("scale", C.c_double), ("j", C.c_int32 * 8),
                ("fk", (C.c_double * 3) * 4), ("fc", C.c_double * 4), ("fphi", C.c_double * 4),
                ("fi", C.c_int32 * 4), ("no_supg", C.c_int32), ("mass_coef", C.c_double),
                ("time_ops", C.c_int32)]


class TimeView(C.Structure):
    _fields_ = [("n_dofs", C.c_int32), ("n_g", C.c_int32), ("r_nnz", C.c_int64), ("h_nnz", C.c_int64),
                ("R_rowptr", C.POINTER(C.c_int32)), ("R_col", C.POINTER(C.c_int32)),
                ("R_val", C.POINTER(C.c_double)), ("H_rowptr", C.POINTER(C.c_int32)),
                ("H_col", C.POINTER(C.c_int32)), ("H_val", C.POINTER(C.c_double)),
                ("g_idx", C.POINTER(C.c_int32)), ("coords", C.POINTER(C.c_double))]


class LevelView(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("block", C.c_int32), ("nnzb", C.c_int64),
                ("rowptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double)), ("p_cols", C.c_int32), ("p_nnz", C.c_int64),
                ("p_rowptr", C.POINTER(C.c_int32)), ("p_col", C.POINTER(C.c_int32)),
                ("p_val", C.POINTER(C.c_double)), ("dof_mask", C.POINTER(C.c_uint8)),
                ("n_hanging", C.c_int32), ("hang_node", C.POINTER(C.c_int32)),
                ("hang_master", C.POINTER(C.c_int32)), ("hang_weight", C.POINTER(C.c_double)),
                ("node_lattice", C.POINTER(C.c_int32)), ("max_depth", C.c_int32)]


class CellsView(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("corners", C.c_int32), ("corner", C.POINTER(C.c_int32)),
                ("size", C.POINTER(C.c_double))]


class NSConfig(C.Structure):
    _fields_ = [("cells", C.c_int32 * 3), ("length", C.c_double * 3), ("n_levels", C.c_int32)]


class NSView(C.Structure):
    _fields_ = [("n_v", C.c_int32), ("n_p", C.c_int32), ("v_nnz", C.c_int64),
                ("V_rowptr", C.POINTER(C.c_int32)), ("V_col", C.POINTER(C.c_int32)),
                ("K_val", C.POINTER(C.c_double)), ("C_val", C.POINTER(C.c_double) * 3),
                ("g_nnz", C.c_int64), ("G_rowptr", C.POINTER(C.c_int32)), ("G_col", C.POINTER(C.c_int32)),
                ("G_val", C.POINTER(C.c_double) * 3), ("d_nnz", C.c_int64),
                ("D_rowptr", C.POINTER(C.c_int32)), ("D_col", C.POINTER(C.c_int32)),
                ("D_val", C.POINTER(C.c_double) * 3), ("m_v", C.POINTER(C.c_double)),
                ("m_p", C.POINTER(C.c_double)), ("dir_mask", C.POINTER(C.c_uint8)),
                ("dir_val", C.POINTER(C.c_double)), ("coords_v", C.POINTER(C.c_double))]


def lib():
    global _lib
    if _lib is None:
        L = load("libmggen.so")
        L.mggen_build.argtypes = [C.POINTER(Config), C.POINTER(C.c_void_p)]
        L.mggen_build.restype = C.c_int
        L.mggen_num_levels.argtypes = [C.c_void_p]
        L.mggen_num_levels.restype = C.c_int32
        L.mggen_level.argtypes = [C.c_void_p, C.c_int32, C.POINTER(LevelView)]
        L.mggen_level.restype = C.c_int
        L.mggen_rhs.argtypes = [C.c_void_p]
        L.mggen_rhs.restype = C.POINTER(C.c_double)
        L.mggen_rhs_noise.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double)]
        L.mggen_rhs_noise.restype = C.c_int
        L.mggen_time_ops.argtypes = [C.c_void_p, C.POINTER(TimeView)]
        L.mggen_time_ops.restype = C.c_int
        L.mggen_free.argtypes = [C.c_void_p]
        L.mggen_free.restype = None
        L.mggen_last_error.argtypes = []
        L.mggen_last_error.restype = C.c_char_p
        L.mggen_level_cells.argtypes = [C.c_void_p, C.c_int32, C.POINTER(CellsView)]
        L.mggen_level_cells.restype = C.c_int
        L.mgns_build.argtypes = [C.POINTER(NSConfig), C.POINTER(C.c_void_p)]
        L.mgns_build.restype = C.c_int
        L.mgns_operators.argtypes = [C.c_void_p, C.POINTER(NSView)]
        L.mgns_operators.restype = C.c_int
        L.mgns_num_levels.argtypes = [C.c_void_p]
        L.mgns_num_levels.restype = C.c_int32
        L.mgns_pressure_level.argtypes = [C.c_void_p, C.c_int32, C.POINTER(LevelView)]
        L.mgns_pressure_level.restype = C.c_int
        L.mgns_free.argtypes = [C.c_void_p]
        L.mgns_free.restype = None
        L.mgns_last_error.argtypes = []
        L.mgns_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _arr(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


@dataclasses.dataclass
class GenLevel:
    n: int
    block: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray              # (nnzb, b, b)
    p_cols: int
    p_rowptr: Optional[np.ndarray]
    p_col: Optional[np.ndarray]
    p_val: Optional[np.ndarray]
    mask: np.ndarray             # (n, b) uint8
    hang_node: np.ndarray
    hang_master: np.ndarray      # (k, 4)
    hang_weight: np.ndarray      # (k, 4)
    lattice: np.ndarray          # (n, 3)
    max_depth: int
    cells: Optional[np.ndarray] = None      # (n_cells, 2^dim) leaf corner nodes
    cell_size: Optional[np.ndarray] = None  # (n_cells,) leaf edge lengths

    @property
    def nnzb(self):
        return len(self.col)


@dataclasses.dataclass
class TimeOps:
    """Right-hand-side operators of a time-stepping run on the finest level (CSR)."""
    n_dofs: int
    R_rowptr: np.ndarray         # n_dofs + 1; R is n_dofs x (n_dofs + n_g)
    R_col: np.ndarray
    R_val: np.ndarray
    H_rowptr: np.ndarray         # n_dofs + 1; H is n_dofs x n_dofs
    H_col: np.ndarray
    H_val: np.ndarray
    g_idx: np.ndarray            # n_g Dirichlet DoFs
    coords: np.ndarray           # (n_nodes, dim)

    @property
    def n_g(self):
        return len(self.g_idx)


@dataclasses.dataclass
class Problem:
    wl: W.Workload
    levels: List[GenLevel]
    b: Optional[np.ndarray]      # finest rhs (n*b,), None for noise problems
    _handle: Optional[int] = None
    time: Optional[TimeOps] = None

    @property
    def finest(self):
        return self.levels[-1]


def config_of(wl: W.Workload):
    cfg = Config()
    cfg.dim = wl.dim
    for a in range(3):
        cfg.coarse[a] = wl.coarse[a] if a < wl.dim else 1
    cfg.h0 = wl.h0
    rounds = (Round * max(1, wl.n_rounds))()
    for k, r in enumerate(wl.rounds):
        if r[0] == "uniform":
            rounds[k].kind = 0
        elif r[0] == "band":
            rounds[k].kind = 1
            for q in range(4):
                rounds[k].p[q] = r[1 + q]
        elif r[0] == "corner":
            rounds[k].kind = 2
            rounds[k].axes = r[1]
            rounds[k].p[0] = r[2]
        else:
            raise ValueError(r)
    cfg.n_rounds = wl.n_rounds
    cfg.rounds = C.cast(rounds, C.POINTER(Round))
    cfg.pde = wl.pde
    cfg.block = wl.block
    cfg.eps = wl.eps
    for a in range(len(wl.bvec)):
        cfg.bvec[a] = wl.bvec[a]
    cfg.lam, cfg.mu, cfg.nu, cfg.dt, cfg.pspg_alpha = wl.lam, wl.mu, wl.nu, wl.dt, wl.pspg_alpha
    cfg.dir_faces, cfg.dir_comps, cfg.rhs = wl.dir_faces, wl.dir_comps, wl.rhs
    cfg.no_supg = 0 if wl.supg else 1
    cfg.mass_coef = wl.mass_coef
    for a in range(len(wl.rhs_const)):
        cfg.rhs_const[a] = wl.rhs_const[a]
    if wl.pde == W.PDE_OSEEN or wl.rhs == W.RHS_FIELD:
        f = W.oseen_fields(wl.seed)
        for k in range(8):
            for q in range(3):
                cfg.kappa[k][q] = f["kappa"][k, q]
            cfg.a[k], cfg.phi[k], cfg.j[k] = f["a"][k], f["phi"][k], int(f["j"][k])
        cfg.scale = f["scale"]
        for m in range(4):
            for q in range(3):
                cfg.fk[m][q] = f["fk"][m, q]
            cfg.fc[m], cfg.fphi[m], cfg.fi[m] = f["fc"][m], f["fphi"][m], int(f["fi"][m])
    return cfg, rounds


def build(wl: W.Workload, nrhs: int = 1, time_ops: bool = False) -> Problem:
    L = lib()
    cfg, keep = config_of(wl)
    cfg.time_ops = 1 if time_ops else 0
    h = C.c_void_p()
    rc = L.mggen_build(C.byref(cfg), C.byref(h))
    if rc != 0:
        raise RuntimeError(f"mggen_build failed ({rc}): {L.mggen_last_error().decode()}")
    try:
        levels = []
        for l in range(L.mggen_num_levels(h)):
            v = LevelView()
            rc = L.mggen_level(h, l, C.byref(v))
            if rc != 0:
                raise RuntimeError(L.mggen_last_error().decode())
            n, b, nnzb = v.n_nodes, v.block, v.nnzb
            has_p = bool(v.p_rowptr)
            levels.append(GenLevel(
                n=n, block=b,
                rowptr=_arr(v.rowptr, n + 1, np.int32), col=_arr(v.col, nnzb, np.int32),
                val=_arr(v.val, nnzb * b * b, np.float64).reshape(nnzb, b, b),
                p_cols=v.p_cols,
                p_rowptr=_arr(v.p_rowptr, n + 1, np.int32) if has_p else None,
                p_col=_arr(v.p_col, v.p_nnz, np.int32) if has_p else None,
                p_val=_arr(v.p_val, v.p_nnz, np.float64) if has_p else None,
                mask=_arr(v.dof_mask, n * b, np.uint8).reshape(n, b),
                hang_node=_arr(v.hang_node, v.n_hanging, np.int32),
                hang_master=_arr(v.hang_master, 4 * v.n_hanging, np.int32).reshape(-1, 4),
                hang_weight=_arr(v.hang_weight, 4 * v.n_hanging, np.float64).reshape(-1, 4),
                lattice=_arr(v.node_lattice, 3 * n, np.int32).reshape(n, 3),
                max_depth=v.max_depth))
            cv = CellsView()
            if L.mggen_level_cells(h, l, C.byref(cv)) != 0:
                raise RuntimeError(L.mggen_last_error().decode())
            levels[-1].cells = _arr(cv.corner, cv.n_cells * cv.corners, np.int32).reshape(cv.n_cells, cv.corners)
            levels[-1].cell_size = _arr(cv.size, cv.n_cells, np.float64)
        # the coarse mesh may be any level of the hierarchy; drop the levels below it
        levels = levels[min(wl.coarse_level, len(levels) - 1):]
        levels[0].p_rowptr = levels[0].p_col = levels[0].p_val = None
        levels[0].p_cols = 0
        top = levels[-1]
        if wl.rhs == W.RHS_NOISE:
            xi = np.ascontiguousarray(W.noise(wl.seed, top.n, nrhs))
            out = np.zeros((top.n, nrhs))
            rc = L.mggen_rhs_noise(h, xi.ctypes.data_as(C.POINTER(C.c_double)), nrhs,
                                   out.ctypes.data_as(C.POINTER(C.c_double)))
            if rc != 0:
                raise RuntimeError(L.mggen_last_error().decode())
            b = out[:, 0].copy() if nrhs == 1 else out
        else:
            b = _arr(L.mggen_rhs(h), top.n * top.block, np.float64)
        tops = None
        if time_ops:
            v = TimeView()
            if L.mggen_time_ops(h, C.byref(v)) != 0:
                raise RuntimeError(L.mggen_last_error().decode())
            N = v.n_dofs
            tops = TimeOps(n_dofs=N, R_rowptr=_arr(v.R_rowptr, N + 1, np.int32),
                           R_col=_arr(v.R_col, v.r_nnz, np.int32), R_val=_arr(v.R_val, v.r_nnz, np.float64),
                           H_rowptr=_arr(v.H_rowptr, N + 1, np.int32),
                           H_col=_arr(v.H_col, v.h_nnz, np.int32), H_val=_arr(v.H_val, v.h_nnz, np.float64),
                           g_idx=_arr(v.g_idx, v.n_g, np.int32),
                           coords=_arr(v.coords, top.n * wl.dim, np.float64).reshape(top.n, wl.dim))
        return Problem(wl, levels, b, time=tops)
    finally:
        L.mggen_free(h)


# ---------------------------------------------------------------- pressure-correction workload
@dataclasses.dataclass
class PressureLevel:
    """One pressure multigrid level in the layout mg.Hierarchy takes (block 1)."""
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray              # (nnz, 1, 1)
    p_cols: int
    p_rowptr: Optional[np.ndarray]
    p_col: Optional[np.ndarray]
    p_val: Optional[np.ndarray]
    mask: np.ndarray             # (n, 1) uint8, the pinned node
    block: int = 1

    @property
    def nnzb(self):
        return len(self.col)


@dataclasses.dataclass
class NSProblem:
    """Matrices of the explicit pressure-correction step (host CSR arrays)."""
    cells: tuple
    n_v: int
    n_p: int
    V_rowptr: np.ndarray
    V_col: np.ndarray
    K_val: np.ndarray
    C_val: List[np.ndarray]
    G_rowptr: np.ndarray
    G_col: np.ndarray
    G_val: List[np.ndarray]
    D_rowptr: np.ndarray
    D_col: np.ndarray
    D_val: List[np.ndarray]
    m_v: np.ndarray
    m_p: np.ndarray
    dir_mask: np.ndarray         # (n_v, 3) uint8
    dir_val: np.ndarray          # (n_v, 3)
    coords_v: np.ndarray         # (n_v, 3)
    levels: List[PressureLevel]  # pressure hierarchy, coarsest first


def build_ns(cells=(32, 32, 64), lengths=(1.0, 1.0, 2.0), n_levels=5) -> NSProblem:
    L = lib()
    cfg = NSConfig()
    for a in range(3):
        cfg.cells[a] = int(cells[a])
        cfg.length[a] = float(lengths[a])
    cfg.n_levels = int(n_levels)
    h = C.c_void_p()
    if L.mgns_build(C.byref(cfg), C.byref(h)) != 0:
        raise RuntimeError(L.mgns_last_error().decode())
    try:
        v = NSView()
        if L.mgns_operators(h, C.byref(v)) != 0:
            raise RuntimeError(L.mgns_last_error().decode())
        nv, npr = v.n_v, v.n_p
        f64, i32 = np.float64, np.int32
        levels = []
        for l in range(L.mgns_num_levels(h)):
            lv = LevelView()
            if L.mgns_pressure_level(h, l, C.byref(lv)) != 0:
                raise RuntimeError(L.mgns_last_error().decode())
            n = lv.n_nodes
            has_p = l > 0
            levels.append(PressureLevel(
                n=n, rowptr=_arr(lv.rowptr, n + 1, i32), col=_arr(lv.col, lv.nnzb, i32),
                val=_arr(lv.val, lv.nnzb, f64).reshape(-1, 1, 1), p_cols=lv.p_cols,
                p_rowptr=_arr(lv.p_rowptr, n + 1, i32) if has_p else None,
                p_col=_arr(lv.p_col, lv.p_nnz, i32) if has_p else None,
                p_val=_arr(lv.p_val, lv.p_nnz, f64) if has_p else None,
                mask=_arr(lv.dof_mask, n, np.uint8).reshape(n, 1)))
        return NSProblem(
            cells=tuple(cells), n_v=nv, n_p=npr,
            V_rowptr=_arr(v.V_rowptr, nv + 1, i32), V_col=_arr(v.V_col, v.v_nnz, i32),
            K_val=_arr(v.K_val, v.v_nnz, f64), C_val=[_arr(v.C_val[a], v.v_nnz, f64) for a in range(3)],
            G_rowptr=_arr(v.G_rowptr, nv + 1, i32), G_col=_arr(v.G_col, v.g_nnz, i32),
            G_val=[_arr(v.G_val[a], v.g_nnz, f64) for a in range(3)],
            D_rowptr=_arr(v.D_rowptr, npr + 1, i32), D_col=_arr(v.D_col, v.d_nnz, i32),
            D_val=[_arr(v.D_val[a], v.d_nnz, f64) for a in range(3)],
            m_v=_arr(v.m_v, nv, f64), m_p=_arr(v.m_p, npr, f64),
            dir_mask=_arr(v.dir_mask, nv * 3, np.uint8).reshape(nv, 3),
            dir_val=_arr(v.dir_val, nv * 3, f64).reshape(nv, 3),
            coords_v=_arr(v.coords_v, nv * 3, f64).reshape(nv, 3), levels=levels)
    finally:
        L.mgns_free(h)
