"""Host-side checks of the C ABI (no GPU): every symbol declared in include/*.h is
exported, and the host validator rejects malformed inputs with MG_EINVAL."""
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W
from paper_2405_05047_amd import gen, mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)          # drop comments
    return sorted(set(re.findall(r"\b((?:mg|mggen|mgns)_[a-z0-9_]+)\s*\(", txt)))


@pytest.mark.parametrize("header,lib", [("mgq1.h", "libmgq1.so"), ("mggen.h", "libmggen.so"),
                                        ("mgns.h", "libmggen.so")])
def test_symbols_exported(header, lib):
    path = os.path.join(ROOT, "paper_2405_05047_amd", lib)
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [s for s in _declared(header) if s not in exported]
    assert not missing, missing


@pytest.fixture(scope="module")
def levels():
    return gen.build(W.c2_td(band_rounds=2, uniform_rounds=1)).levels


def _copy(lv):
    import copy
    return copy.deepcopy(lv)


def test_valid_levels_pass(levels):
    for l in range(len(levels)):
        assert mg.validate_level(levels[l], levels[l - 1] if l else None) == 0


@pytest.mark.parametrize("breakage", ["rowptr", "col_range", "col_order", "missing_diag", "mask_row",
                                      "mask_col", "nan", "p_col", "p_cols"])
def test_malformed_rejected(levels, breakage):
    lv = _copy(levels[-1])
    co = levels[-2]
    if breakage == "rowptr":
        lv.rowptr[5] = lv.rowptr[6] + 1
    elif breakage == "col_range":
        lv.col[3] = lv.n
    elif breakage == "col_order":
        k = lv.rowptr[100]
        lv.col[k], lv.col[k + 1] = lv.col[k + 1], lv.col[k]
    elif breakage == "missing_diag":
        i = int(np.nonzero(lv.mask[:, 0] == 0)[0][0])
        k = lv.rowptr[i] + int(np.nonzero(lv.col[lv.rowptr[i]:lv.rowptr[i + 1]] == i)[0][0])
        lv.col[k] = lv.col[k] + (1 if k + 1 < lv.rowptr[i + 1] else -1)
    elif breakage == "mask_row":
        i = int(np.nonzero(lv.mask[:, 0])[0][0])
        k = lv.rowptr[i]
        lv.val[k, 0, 0] = 2.0
    elif breakage == "mask_col":
        # a free row that references a constrained node with a nonzero entry: insert the
        # block (i, j) in sorted position (the generator's pattern drops such columns)
        j = int(np.nonzero(lv.mask[:, 0])[0][0])
        i = int(np.nonzero(lv.mask[:, 0] == 0)[0][0])
        row = lv.col[lv.rowptr[i]:lv.rowptr[i + 1]]
        assert j not in row
        k = int(lv.rowptr[i] + np.searchsorted(row, j))
        blk = np.zeros((1,) + lv.val.shape[1:])
        blk[0, 0, 0] = 0.5
        lv.col = np.insert(lv.col, k, j)
        lv.val = np.insert(lv.val, k, blk, axis=0)
        lv.rowptr = lv.rowptr.copy()
        lv.rowptr[i + 1:] += 1
    elif breakage == "nan":
        lv.val[7, 0, 0] = np.nan
    elif breakage == "p_col":
        lv.p_col[0] = co.n
    elif breakage == "p_cols":
        lv.p_cols = co.n + 1
    assert mg.validate_level(lv, co) == -1
    assert mg.last_error()


def test_smoother_blocks_validated(levels):
    """Caller smoother blocks must be finite (host validation, no device)."""
    lv = levels[-1]
    S = np.ones((lv.n, 1, 1))
    arr, keep = mg.level_structs([lv], [S])
    assert mg.lib().mg_validate_level(arr, None) == 0
    S[3] = np.inf
    arr, keep = mg.level_structs([lv], [S])
    assert mg.lib().mg_validate_level(arr, None) == -1
    assert "smoother" in mg.last_error()


@pytest.mark.parametrize("bad", ["nrhs3", "outer_ir", "coarse_smooth", "dictionary", "nrhs8_block3", "block_mismatch"])
def test_batch_setup_rejects_unsupported_requests(levels, bad):
    """mg_setup_batch refuses requests it does not implement before touching a device."""
    import ctypes as C
    wl = W.c2_td(band_rounds=2, uniform_rounds=1)
    cfg = mg.config_from(wl)
    problems, nrhs, want = [levels, levels], 1, -7
    if bad == "nrhs3":
        nrhs = 3
    elif bad == "outer_ir":
        cfg.outer = 0
    elif bad == "coarse_smooth":
        cfg.coarse_mode = 1
    elif bad == "dictionary":
        cfg.precision = mg.PREC["fp64dict"]
    elif bad == "nrhs8_block3":
        problems, nrhs = [gen.build(W.c3_elasticity(1)).levels], 8
    else:
        problems, want = [levels, gen.build(W.c3_elasticity(1)).levels], -1
    with pytest.raises(mg.MGError) as e:
        mg.Batch(problems, cfg, nrhs=nrhs, stream=C.c_void_p(0))
    assert e.value.code == want


def test_empty_inputs_rejected(levels):
    """A level without nodes and a hierarchy without levels are refused with MG_EINVAL
    before any device work."""
    import copy
    import ctypes as C
    e = copy.deepcopy(levels[0])
    e.n = 0
    e.rowptr = np.zeros(1, np.int32)
    e.col = np.zeros(0, np.int32)
    e.val = np.zeros((0, 1, 1))
    e.mask = np.zeros((0, 1), np.uint8)
    assert mg.validate_level(e, None) == -1
    L = mg.lib()
    h = C.c_void_p()
    arr = (mg.LevelIn * 1)()
    cfg = mg.config_from(W.c2_td())
    assert L.mg_setup_hierarchy(arr, 0, C.byref(cfg), 0, None, C.byref(h)) == -1
    assert not h.value


@pytest.mark.parametrize("field,value", [("omega", 0.0), ("nu1", -1), ("gmres_m", 0), ("gmres_m", 65),
                                         ("precision", 7), ("outer", 3), ("rtol", -1.0)])
def test_invalid_config_rejected(levels, field, value):
    """Invalid solver settings are refused by setup before any device work."""
    import ctypes as C
    cfg = mg.config_from(W.c2_td())
    setattr(cfg, field, value)
    arr, keep = mg.level_structs(levels)
    h = C.c_void_p()
    assert mg.lib().mg_setup_hierarchy(arr, len(levels), C.byref(cfg), 0, None, C.byref(h)) == -1
    assert mg.last_error()


def _asm_rc(level, dim):
    """Status of mg_asm_setup on a malformed level (refused before any device work)."""
    import ctypes as C
    L = mg.lib()
    keep = []

    def a(v, dt):
        arr = np.ascontiguousarray(v, dt)
        keep.append(arr)
        return arr.ctypes.data

    s = mg.AsmIn()
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
    return L.mg_asm_setup(C.byref(s), None, C.byref(t))


@pytest.mark.parametrize("breakage", ["corner", "weight", "unsorted", "sizes"])
def test_assembly_input_refused_on_host(breakage):
    """mg_asm_setup validates the mesh before touching the device: corners out of range
    and unsorted patterns are MG_EINVAL, non-dyadic hanging weights and more than 32 cell
    sizes are MG_EUNSUPPORTED."""
    import dataclasses
    wl = W.c2_td(band_rounds=2, uniform_rounds=1)
    lv = gen.build(wl).finest
    assert len(lv.hang_node) > 0
    if breakage == "corner":
        cells = lv.cells.copy()
        cells[3, 1] = lv.n
        bad, want = dataclasses.replace(lv, cells=cells), -1
    elif breakage == "weight":
        w = lv.hang_weight.copy()
        w[0, 0] = 0.3
        bad, want = dataclasses.replace(lv, hang_weight=w), -7
    elif breakage == "unsorted":
        col = lv.col.copy()
        i = int(np.nonzero(np.diff(lv.rowptr) >= 3)[0][0])
        k = lv.rowptr[i]
        col[k], col[k + 1] = col[k + 1], col[k]
        bad, want = dataclasses.replace(lv, col=col), -1
    else:
        sizes = lv.cell_size * (1.0 + 1e-3 * (np.arange(len(lv.cell_size)) % 40))
        bad, want = dataclasses.replace(lv, cell_size=sizes), -7
    assert _asm_rc(bad, wl.dim) == want
    assert mg.last_error()
