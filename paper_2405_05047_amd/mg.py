"""ctypes binding of the HIP solver library (libmgq1.so, include/mgq1.h).

Argument marshalling only: every step of the V-cycle and of the outer loops runs in the
library's HIP kernels.  Device vectors are torch tensors (FP64, contiguous, on the
current device); PyTorch provides only memory and the stream.  There is no fallback:
a missing library raises at load time.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np

import workloads as W
from ._native import load

_lib = None

PREC = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fp64dict": 4}


class LevelIn(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("block", C.c_int32), ("nnzb", C.c_int64),
                ("A_rowptr", C.c_void_p), ("A_col", C.c_void_p), ("A_val", C.c_void_p),
                ("p_cols", C.c_int32), ("p_nnz", C.c_int64),
                ("P_rowptr", C.c_void_p), ("P_col", C.c_void_p), ("P_val", C.c_void_p),
                ("dof_mask", C.c_void_p), ("smoother_blocks", C.c_void_p)]


class Config(C.Structure):
    _fields_ = [("omega", C.c_double), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("coarse_mode", C.c_int32), ("coarse_sweeps", C.c_int32),
                ("precision", C.c_int32), ("outer", C.c_int32), ("gmres_m", C.c_int32),
                ("maxit", C.c_int32), ("rtol", C.c_double), ("use_graph", C.c_int32),
                ("slot_batch", C.c_int32), ("smoother", C.c_int32), ("power_its", C.c_int32),
                ("cheb_lo", C.c_double), ("cheb_hi", C.c_double)]


class NSIn(C.Structure):
    _fields_ = [("n_v", C.c_int32), ("n_p", C.c_int32), ("V_rowptr", C.c_void_p), ("V_col", C.c_void_p),
                ("K_val", C.c_void_p), ("C_val", C.c_void_p * 3), ("G_rowptr", C.c_void_p), ("G_col", C.c_void_p),
                ("G_val", C.c_void_p * 3), ("D_rowptr", C.c_void_p), ("D_col", C.c_void_p),
                ("D_val", C.c_void_p * 3), ("m_v", C.c_void_p), ("m_p", C.c_void_p), ("dir_mask", C.c_void_p),
                ("dir_val", C.c_void_p), ("nu", C.c_double), ("dt", C.c_double)]


class AsmCoef(C.Structure):
    _fields_ = [("pde", C.c_int32), ("supg", C.c_int32), ("eps", C.c_double), ("bvec", C.c_double * 3),
                ("lam", C.c_double), ("mu", C.c_double), ("mass_coef", C.c_double)]


class AsmIn(C.Structure):
    _fields_ = [("dim", C.c_int32), ("block", C.c_int32), ("n_nodes", C.c_int32), ("n_cells", C.c_int32),
                ("cell_corner", C.c_void_p), ("cell_size", C.c_void_p), ("n_hanging", C.c_int32),
                ("hang_node", C.c_void_p), ("hang_master", C.c_void_p), ("hang_weight", C.c_void_p),
                ("dof_mask", C.c_void_p), ("nnzb", C.c_int64), ("A_rowptr", C.c_void_p), ("A_col", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
                ("converged", C.c_int32), ("res0", C.c_double), ("res_final", C.c_double),
                ("t_solve_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SYMBOLS = ["mg_setup_hierarchy", "mg_vcycle", "mg_solve", "mg_solve_fixed", "mg_level_defect",
           "mg_level_spmv", "mg_level_sweep", "mg_level_sweep0", "mg_level_restrict",
           "mg_level_prolong", "mg_coarse_solve", "mg_level_info", "mg_num_levels",
           "mg_validate_level", "mg_destroy", "mg_status_string", "mg_last_error",
           "mg_setup_batch", "mg_batch_offsets", "mg_solve_batch", "mg_destroy_batch",
           "mg_level_tuning", "mg_outer_defect", "mg_level_export", "mg_time_setup", "mg_time_rhs",
           "mg_time_theta", "mg_time_run", "mg_time_destroy", "mg_outer_defect_noalloc",
           "mg_level_smooth", "mg_level_eigen_estimate", "mg_ns_setup", "mg_ns_momentum", "mg_ns_divergence",
           "mg_ns_pressure_update", "mg_ns_run", "mg_ns_destroy", "mg_asm_setup", "mg_asm_values",
           "mg_asm_destroy", "mg_level_transfer_format", "mg_level_dictionary"]


def lib():
    global _lib
    if _lib is None:
        L = load("libmgq1.so")
        vp, i32 = C.c_void_p, C.c_int32
        L.mg_setup_hierarchy.argtypes = [C.POINTER(LevelIn), i32, C.POINTER(Config), i32, vp, C.POINTER(vp)]
        L.mg_vcycle.argtypes = [vp, vp, vp, i32, vp]
        L.mg_outer_defect.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mg_outer_defect_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mg_level_export.argtypes = [vp, i32, vp, vp]
        L.mg_solve.argtypes = [vp, vp, vp, C.POINTER(Stats), vp]
        L.mg_solve_fixed.argtypes = [vp, vp, vp, i32, C.POINTER(Stats), vp]
        L.mg_level_defect.argtypes = [vp, i32, vp, vp, vp, i32, vp]
        L.mg_level_spmv.argtypes = [vp, i32, vp, vp, vp]
        L.mg_level_sweep.argtypes = [vp, i32, vp, vp, vp, vp]
        L.mg_level_sweep0.argtypes = [vp, i32, vp, vp, vp]
        L.mg_level_smooth.argtypes = [vp, i32, vp, vp, vp, i32, i32, vp]
        L.mg_level_eigen_estimate.argtypes = [vp, i32, C.POINTER(C.c_double)]
        L.mg_level_restrict.argtypes = [vp, i32, vp, vp, vp]
        L.mg_level_prolong.argtypes = [vp, i32, vp, vp, vp]
        L.mg_coarse_solve.argtypes = [vp, vp, vp, vp]
        L.mg_level_info.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_int64)]
        L.mg_level_tuning.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        L.mg_level_transfer_format.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.mg_level_dictionary.argtypes = [vp, i32, C.POINTER(i32)]
        L.mg_num_levels.argtypes = [vp]
        L.mg_num_levels.restype = i32
        L.mg_validate_level.argtypes = [C.POINTER(LevelIn), C.POINTER(LevelIn)]
        L.mg_destroy.argtypes = [vp]
        L.mg_destroy.restype = None
        L.mg_status_string.argtypes = [C.c_int]
        L.mg_status_string.restype = C.c_char_p
        L.mg_last_error.argtypes = []
        L.mg_last_error.restype = C.c_char_p
        L.mg_setup_batch.argtypes = [C.POINTER(C.POINTER(LevelIn)), C.POINTER(i32), i32, i32,
                                     C.POINTER(Config), i32, vp, C.POINTER(vp)]
        L.mg_batch_offsets.argtypes = [vp, C.POINTER(C.c_int64)]
        L.mg_solve_batch.argtypes = [vp, vp, vp, C.POINTER(Stats), vp]
        L.mg_destroy_batch.argtypes = [vp]
        L.mg_destroy_batch.restype = None
        L.mg_time_setup.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, C.c_double, vp, C.POINTER(vp)]
        L.mg_time_rhs.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mg_time_theta.argtypes = [vp, vp, vp, vp, vp]
        L.mg_time_run.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.mg_time_destroy.argtypes = [vp]
        L.mg_time_destroy.restype = None
        L.mg_ns_setup.argtypes = [C.POINTER(NSIn), vp, vp, C.POINTER(vp)]
        L.mg_ns_momentum.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.mg_ns_divergence.argtypes = [vp, vp, vp, vp, vp]
        L.mg_ns_pressure_update.argtypes = [vp, vp, vp, vp, vp]
        L.mg_ns_run.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.mg_ns_destroy.argtypes = [vp]
        L.mg_ns_destroy.restype = None
        L.mg_asm_setup.argtypes = [C.POINTER(AsmIn), vp, C.POINTER(vp)]
        L.mg_asm_values.argtypes = [vp, C.POINTER(AsmCoef), vp, vp]
        L.mg_asm_destroy.argtypes = [vp]
        L.mg_asm_destroy.restype = None
        for name in SYMBOLS:
            if name not in ("mg_destroy", "mg_status_string", "mg_last_error", "mg_num_levels",
                            "mg_destroy_batch", "mg_time_destroy", "mg_ns_destroy", "mg_asm_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class MGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def _check(rc):
    if rc != 0:
        L = lib()
        raise MGError(rc, L.mg_last_error().decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    assert a.is_contiguous(), "device arrays must be contiguous"
    return a.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def level_structs(levels, smoother_blocks=None):
    """mg_level_in array from host levels (objects with rowptr, col, val, p_*, mask);
    smoother_blocks: None or one (n, b, b) array (or None) per level."""
    keep = []
    arr = (LevelIn * len(levels))()
    for l, lv in enumerate(levels):
        parts = [np.ascontiguousarray(lv.rowptr, np.int32), np.ascontiguousarray(lv.col, np.int32),
                 np.ascontiguousarray(lv.val, np.float64), np.ascontiguousarray(lv.mask, np.uint8)]
        keep += parts
        s = arr[l]
        s.n_nodes, s.block, s.nnzb = lv.n, lv.block, len(parts[1])
        s.A_rowptr, s.A_col, s.A_val, s.dof_mask = (p.ctypes.data for p in parts)
        if smoother_blocks is not None and smoother_blocks[l] is not None:
            sb = np.ascontiguousarray(smoother_blocks[l], np.float64)
            assert sb.size == lv.n * lv.block * lv.block
            keep.append(sb)
            s.smoother_blocks = sb.ctypes.data
        if l > 0 and lv.p_rowptr is not None:
            pp = [np.ascontiguousarray(lv.p_rowptr, np.int32), np.ascontiguousarray(lv.p_col, np.int32),
                  np.ascontiguousarray(lv.p_val, np.float64)]
            keep += pp
            s.p_cols, s.p_nnz = lv.p_cols, len(pp[1])
            s.P_rowptr, s.P_col, s.P_val = (p.ctypes.data for p in pp)
    return arr, keep


def config_from(wl: W.Workload, precision="fp64", **over) -> Config:
    c = Config()
    c.omega = over.get("omega", wl.omega)
    c.nu1 = over.get("nu1", wl.nu1)
    c.nu2 = over.get("nu2", wl.nu2)
    c.coarse_mode = over.get("coarse_mode", wl.coarse_mode)
    c.coarse_sweeps = over.get("coarse_sweeps", wl.coarse_sweeps)
    c.precision = PREC[precision]
    c.outer = over.get("outer", wl.outer)
    c.gmres_m = over.get("gmres_m", wl.gmres_m)
    c.maxit = over.get("maxit", wl.maxit)
    c.rtol = over.get("rtol", wl.rtol)
    c.use_graph = over.get("use_graph", 1)
    c.slot_batch = over.get("slot_batch", 0)
    c.smoother = over.get("smoother", wl.smoother)
    c.power_its = over.get("power_its", wl.power_its)
    c.cheb_lo = over.get("cheb_lo", wl.cheb_lo)
    c.cheb_hi = over.get("cheb_hi", wl.cheb_hi)
    return c


class Hierarchy:
    """A device-resident multigrid hierarchy (library handle)."""

    def __init__(self, levels, cfg: Config, stream=None, smoother_blocks=None):
        L = lib()
        arr, keep = level_structs(levels, smoother_blocks)
        h = C.c_void_p()
        self.cfg = cfg
        _check(L.mg_setup_hierarchy(arr, len(levels), C.byref(cfg), 0, _stream(stream), C.byref(h)))
        self.h = h
        self.n_levels = L.mg_num_levels(h)
        self.sizes = [self.level_info(l) for l in range(self.n_levels)]

    def close(self):
        if getattr(self, "h", None):
            lib().mg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, l):
        n, b, nnzb = C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().mg_level_info(self.h, l, C.byref(n), C.byref(b), C.byref(nnzb)))
        return n.value, b.value, nnzb.value

    def tuning(self, l):
        """(slot batch in use, measured us per sweep for the default / other size)."""
        kb, t0, t1 = C.c_int32(), C.c_double(), C.c_double()
        _check(lib().mg_level_tuning(self.h, l, C.byref(kb), None, C.byref(t0), C.byref(t1)))
        return kb.value, t0.value, t1.value

    def col_bytes(self, l):
        """Bytes per stored column index of level l's operators (2 or 4)."""
        cb = C.c_int32()
        _check(lib().mg_level_tuning(self.h, l, None, C.byref(cb), None, None))
        return cb.value

    def transfer_format(self, l):
        """(bytes per column index of P~, of R, bytes per weight) between levels l-1 and l."""
        pc, rc, wb = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().mg_level_transfer_format(self.h, l, C.byref(pc), C.byref(rc), C.byref(wb)))
        return pc.value, rc.value, wb.value

    def dictionary_blocks(self, l):
        """Distinct blocks of level l's operator in the dictionary form (0: plain values)."""
        n = C.c_int32()
        _check(lib().mg_level_dictionary(self.h, l, C.byref(n)))
        return n.value

    def ndof(self, l=-1):
        n, b, _ = self.sizes[l]
        return n * b

    @property
    def cycle_fp64(self):
        """True when the V-cycle (and the step-wise entry points) work on FP64 vectors."""
        return self.cfg.precision in (PREC["fp64"], PREC["fp64dict"])

    # -- whole-path entry points
    def vcycle(self, b, x, x_is_zero=True, stream=None):
        _check(lib().mg_vcycle(self.h, _ptr(b), _ptr(x), int(bool(x_is_zero)), _stream(stream)))

    def outer_defect(self, b, x, r, norm, stream=None):
        """r = b - A_L x and norm[0] = ||r|| in FP64 (device tensors)."""
        _check(lib().mg_outer_defect(self.h, _ptr(b), _ptr(x), _ptr(r), _ptr(norm), _stream(stream)))

    def outer_defect_noalloc(self, b, x, r, norm, stream=None):
        """outer_defect with the partial sums in the library's static device array (the
        call allocates nothing; calls overlapping on one GPU race)."""
        _check(lib().mg_outer_defect_noalloc(self.h, _ptr(b), _ptr(x), _ptr(r), _ptr(norm), _stream(stream)))

    def export(self, l):
        """Stored cycle operator of level l in BSR order: (values (nnzb, b, b) of the storage
        dtype: float64, float32 or uint16 codes; row exponents (n * b,) int8 or None).  A
        block-dictionary handle keeps no per-block values: the library refuses it (MGError)."""
        n, b, nnzb = self.sizes[l]
        prec = self.cfg.precision
        dt = {0: np.float64, 1: np.float32, 2: np.uint16, 3: np.uint16, 4: np.float64}[prec]
        vals = np.zeros((nnzb, b, b), dt)
        ex = np.zeros(n * b, np.int8) if prec in (2, 3) else None
        _check(lib().mg_level_export(self.h, l, vals.ctypes.data, None if ex is None else ex.ctypes.data))
        return vals, ex

    def solve(self, b, x, stream=None, fixed=None):
        st = Stats()
        if fixed is None:
            rc = lib().mg_solve(self.h, _ptr(b), _ptr(x), C.byref(st), _stream(stream))
        else:
            rc = lib().mg_solve_fixed(self.h, _ptr(b), _ptr(x), int(fixed), C.byref(st), _stream(stream))
        if rc not in (0, -5):
            _check(rc)
        return st.as_dict()

    # -- step-wise entry points
    def defect(self, l, b, x, r, masked=False, stream=None):
        _check(lib().mg_level_defect(self.h, l, _ptr(b), _ptr(x), _ptr(r), int(masked), _stream(stream)))

    def spmv(self, l, x, y, stream=None):
        _check(lib().mg_level_spmv(self.h, l, _ptr(x), _ptr(y), _stream(stream)))

    def sweep(self, l, b, x, xo, stream=None):
        _check(lib().mg_level_sweep(self.h, l, _ptr(b), _ptr(x), _ptr(xo), _stream(stream)))

    def sweep0(self, l, b, xo, stream=None):
        _check(lib().mg_level_sweep0(self.h, l, _ptr(b), _ptr(xo), _stream(stream)))

    def smooth(self, l, b, x, xo, sweeps, stream=None):
        """The level's smoothing phase of `sweeps` steps from x (None: from 0) into xo."""
        _check(lib().mg_level_smooth(self.h, l, _ptr(b), _ptr(x), _ptr(xo), int(x is None), int(sweeps),
                                     _stream(stream)))

    def eigen_estimate(self, l):
        """Power-iteration estimate of the largest eigenvalue of S_l A_l (Chebyshev handles)."""
        v = C.c_double()
        _check(lib().mg_level_eigen_estimate(self.h, l, C.byref(v)))
        return v.value

    def restrict(self, l, r, d, stream=None):
        _check(lib().mg_level_restrict(self.h, l, _ptr(r), _ptr(d), _stream(stream)))

    def prolong(self, l, y, x, stream=None):
        _check(lib().mg_level_prolong(self.h, l, _ptr(y), _ptr(x), _stream(stream)))

    def coarse_solve(self, b, x, stream=None):
        _check(lib().mg_coarse_solve(self.h, _ptr(b), _ptr(x), _stream(stream)))


class Batch:
    """Many independent hierarchies (same block size) solved together with `nrhs`
    right-hand sides each; batch vectors are the problems' (node, component, rhs)-ordered
    vectors concatenated, problem p at offsets[p]:offsets[p + 1]."""

    def __init__(self, problems, cfg: Config, nrhs=1, stream=None):
        L = lib()
        P = len(problems)
        keep, ptrs = [], (C.POINTER(LevelIn) * P)()
        nl = (C.c_int32 * P)()
        for p, levels in enumerate(problems):
            arr, k = level_structs(levels)
            keep += [arr, k]
            ptrs[p] = C.cast(arr, C.POINTER(LevelIn))
            nl[p] = len(levels)
        h = C.c_void_p()
        self.cfg, self.nrhs, self.n_problems = cfg, nrhs, P
        _check(L.mg_setup_batch(ptrs, nl, P, nrhs, C.byref(cfg), 0, _stream(stream), C.byref(h)))
        self.h = h
        off = (C.c_int64 * (P + 1))()
        _check(L.mg_batch_offsets(h, off))
        self.offsets = np.array(off[:], dtype=np.int64)

    @property
    def size(self):
        return int(self.offsets[-1])

    def close(self):
        if getattr(self, "h", None):
            lib().mg_destroy_batch(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, b, x, stream=None):
        """Returns (status, list of per-instance stats dicts, instance p * nrhs + q)."""
        n = self.n_problems * self.nrhs
        st = (Stats * n)()
        rc = lib().mg_solve_batch(self.h, _ptr(b), _ptr(x), st, _stream(stream))
        if rc not in (0, -5):
            _check(rc)
        return rc, [st[i].as_dict() for i in range(n)]


class TimeStepper:
    """Backward-Euler time stepping on a hierarchy whose operator holds the M_l / dt term
    (library object mg_time): every step forms b = R [theta / dt + f ; g] on the device,
    solves with the hierarchy from the previous solution and sets theta = H x (Dirichlet
    values on the Dirichlet DoFs).  `ops` carries R, H and g_idx as host CSR arrays."""

    def __init__(self, hier: Hierarchy, ops, dt: float, stream=None):
        L = lib()
        a = [np.ascontiguousarray(ops.R_rowptr, np.int32), np.ascontiguousarray(ops.R_col, np.int32),
             np.ascontiguousarray(ops.R_val, np.float64), np.ascontiguousarray(ops.H_rowptr, np.int32),
             np.ascontiguousarray(ops.H_col, np.int32), np.ascontiguousarray(ops.H_val, np.float64),
             np.ascontiguousarray(ops.g_idx, np.int32)]
        t = C.c_void_p()
        _check(L.mg_time_setup(hier.h, len(a[6]), *(_ptr(v) for v in a), float(dt), _stream(stream),
                               C.byref(t)))
        self.t, self.hier, self.n_g = t, hier, len(a[6])

    def close(self):
        if getattr(self, "t", None):
            lib().mg_time_destroy(self.t)
            self.t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rhs(self, theta, f, g, b, stream=None):
        _check(lib().mg_time_rhs(self.t, _ptr(theta), _ptr(f), _ptr(g), _ptr(b), _stream(stream)))

    def theta(self, x, g, theta, stream=None):
        _check(lib().mg_time_theta(self.t, _ptr(x), _ptr(g), _ptr(theta), _stream(stream)))

    def run(self, theta, F, G, x, history=None, stream=None):
        """len(F) steps (F: steps x n, G: steps x n_g device tensors); theta and x are
        updated in place; returns the per-step stats dicts."""
        steps = int(F.shape[0])
        st = (Stats * max(steps, 1))()
        _check(lib().mg_time_run(self.t, steps, _ptr(theta), _ptr(F), _ptr(G) if self.n_g else None, _ptr(x),
                                 _ptr(history), st, _stream(stream)))
        return [st[i].as_dict() for i in range(steps)]


class PressureCorrection:
    """The explicit pressure-correction step (library object mg_ns) on a pressure
    hierarchy: `prob` carries the host CSR matrices (gen.NSProblem)."""

    def __init__(self, prob, pressure: Hierarchy, nu: float, dt: float, stream=None):
        L = lib()
        keep = []

        def a(v, dt_):
            arr = np.ascontiguousarray(v, dt_)
            keep.append(arr)
            return arr.ctypes.data

        i32, f64 = np.int32, np.float64
        s = NSIn()
        s.n_v, s.n_p = prob.n_v, prob.n_p
        s.V_rowptr, s.V_col, s.K_val = a(prob.V_rowptr, i32), a(prob.V_col, i32), a(prob.K_val, f64)
        s.G_rowptr, s.G_col = a(prob.G_rowptr, i32), a(prob.G_col, i32)
        s.D_rowptr, s.D_col = a(prob.D_rowptr, i32), a(prob.D_col, i32)
        for c in range(3):
            s.C_val[c] = a(prob.C_val[c], f64)
            s.G_val[c] = a(prob.G_val[c], f64)
            s.D_val[c] = a(prob.D_val[c], f64)
        s.m_v, s.m_p = a(prob.m_v, f64), a(prob.m_p, f64)
        s.dir_mask, s.dir_val = a(prob.dir_mask, np.uint8), a(prob.dir_val, f64)
        s.nu, s.dt = float(nu), float(dt)
        t = C.c_void_p()
        _check(L.mg_ns_setup(C.byref(s), pressure.h, _stream(stream), C.byref(t)))
        self.t, self.pressure = t, pressure

    def close(self):
        if getattr(self, "t", None):
            lib().mg_ns_destroy(self.t)
            self.t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def momentum(self, u, p, q, u_out, f=None, stream=None):
        _check(lib().mg_ns_momentum(self.t, _ptr(u), _ptr(p), _ptr(q), _ptr(f), _ptr(u_out), _stream(stream)))

    def divergence(self, u, du, rhs, stream=None):
        _check(lib().mg_ns_divergence(self.t, _ptr(u), _ptr(du), _ptr(rhs), _stream(stream)))

    def pressure_update(self, p, q, du, stream=None):
        _check(lib().mg_ns_pressure_update(self.t, _ptr(p), _ptr(q), _ptr(du), _stream(stream)))

    def run(self, steps, u, p, q, f=None, stream=None):
        st = (Stats * max(int(steps), 1))()
        _check(lib().mg_ns_run(self.t, int(steps), _ptr(u), _ptr(p), _ptr(q), _ptr(f), st, _stream(stream)))
        return [st[i].as_dict() for i in range(int(steps))]


ASM_PDE = {W.PDE_POISSON: 0, W.PDE_TD: 1, W.PDE_ELASTICITY: 2}


def asm_coef(wl: W.Workload) -> AsmCoef:
    """Coefficients of the workload's operator for the GPU assembly."""
    c = AsmCoef()
    c.pde = ASM_PDE[wl.pde]
    c.supg = 1 if (wl.pde == W.PDE_TD and wl.supg) else 0
    c.eps = wl.eps
    for a in range(len(wl.bvec)):
        c.bvec[a] = wl.bvec[a]
    c.lam, c.mu, c.mass_coef = wl.lam, wl.mu, wl.mass_coef
    return c


class Assembly:
    """GPU assembly of one level's constrained operator (library object mg_asm) from the
    level's mesh (leaf corners and sizes, hanging nodes, DoF mask, block pattern)."""

    def __init__(self, level, dim, stream=None):
        L = lib()
        keep = []

        def a(v, dt_):
            arr = np.ascontiguousarray(v, dt_)
            keep.append(arr)
            return arr.ctypes.data

        s = AsmIn()
        s.dim, s.block, s.n_nodes = dim, level.block, level.n
        s.n_cells = len(level.cell_size)
        s.cell_corner, s.cell_size = a(level.cells, np.int32), a(level.cell_size, np.float64)
        s.n_hanging = len(level.hang_node)
        if s.n_hanging:
            s.hang_node = a(level.hang_node, np.int32)
            s.hang_master = a(level.hang_master, np.int32)
            s.hang_weight = a(level.hang_weight, np.float64)
        s.dof_mask = a(level.mask, np.uint8)
        s.nnzb = len(level.col)
        s.A_rowptr, s.A_col = a(level.rowptr, np.int32), a(level.col, np.int32)
        t = C.c_void_p()
        _check(L.mg_asm_setup(C.byref(s), _stream(stream), C.byref(t)))
        self.t, self.nnzb, self.block = t, s.nnzb, level.block

    def close(self):
        if getattr(self, "t", None):
            lib().mg_asm_destroy(self.t)
            self.t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def values(self, coef: AsmCoef, val, stream=None):
        """Fill val (device FP64, nnzb * b * b) with the operator's block values."""
        _check(lib().mg_asm_values(self.t, C.byref(coef), _ptr(val), _stream(stream)))


def validate_level(level, coarser=None) -> int:
    """Host-only structural validation; returns the status code (0 = valid)."""
    arr, keep = level_structs([coarser, level] if coarser is not None else [level])
    if coarser is not None:
        return lib().mg_validate_level(C.byref(arr[1]), C.byref(arr[0]))
    return lib().mg_validate_level(C.byref(arr[0]), None)


def last_error() -> str:
    return lib().mg_last_error().decode()
