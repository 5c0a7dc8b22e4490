"""GPU parity: the HIP library (through its C ABI) against the oracle, element by element.

Both sides build their operators independently from the same seeded workload (the
library side through the native generator).  Tolerances (derived from the arithmetic):
  * one SpMV / defect / sweep / transfer step: |gpu - oracle| <= 1e-12 * scale, scale the
    infinity norm of |A||x| (plus |b|, |x| where they enter); a row sum of <= 27 blocks
    in FP64 with operands equal to 1e-15 relative is accurate to ~1e-14 of that scale;
  * one V-cycle: 1e-12 relative (normwise);
  * solutions: 1e-10 relative after the same number of cycles (fixed-count runs) and for
    converged solves (the iteration counts are asserted equal).
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import hierarchy as Hh, multigrid as MG

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


CASES = {
    "poisson33": W.c1_poisson(4),
    "td_band": W.c2_td(band_rounds=3, uniform_rounds=1),
    "elast17": W.c3_elasticity(3),
    "oseen17": W.c4_oseen(3),
    "edge4": W.c3_adaptive("edge", 4),
    "oseen_tall": W.c4_oseen(2, tall=True),
    "td_band_cl3": W.c2_td(band_rounds=3, uniform_rounds=1).with_(coarse_level=3),
    "elast17_cl2": W.c3_elasticity(3).with_(coarse_level=2),
}

_cache = {}


def _pair(name):
    if name not in _cache:
        from paper_2405_05047_amd import gen, mg
        wl = CASES[name]
        _log("building", name)
        o = Hh.build(wl)
        p = gen.build(wl)
        h = mg.Hierarchy(p.levels, mg.config_from(wl))
        _cache[name] = (wl, o, MG.Multigrid(o), p, h)
    return _cache[name]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rand(seed, n):
    return W.rand_vec(seed, n)


@pytest.mark.parametrize("name", list(CASES))
def test_level_structure(name):
    wl, o, mgo, p, h = _pair(name)
    assert h.n_levels == len(o.levels)
    for l, lv in enumerate(o.levels):
        n, b, nnzb = h.sizes[l]
        assert (n, b) == (lv.n, wl.block) and nnzb == len(lv.col)


@pytest.mark.parametrize("name", list(CASES))
def test_spmv_defect_parity(name):
    wl, o, mgo, p, h = _pair(name)
    for l, lv in enumerate(o.levels):
        _log(name, "spmv level", l)
        x = _rand(100 + l, lv.ndof)
        b = _rand(200 + l, lv.ndof)
        scale = max(np.abs(abs(lv.A) @ np.abs(x)).max(), np.abs(b).max())
        y = torch.zeros(lv.ndof, dtype=torch.float64, device="cuda")
        h.spmv(l, dev(x), y)
        assert np.abs(host(y) - lv.A @ x).max() <= 1e-12 * scale
        r = torch.zeros_like(y)
        h.defect(l, dev(b), dev(x), r)
        assert np.abs(host(r) - (b - lv.A @ x)).max() <= 1e-12 * scale
        h.defect(l, dev(b), dev(x), r, masked=True)
        ref = b - lv.A @ x
        ref[lv.mask.ravel()] = 0.0
        got = host(r)
        assert np.all(got[lv.mask.ravel()] == 0.0)
        assert np.abs(got - ref).max() <= 1e-12 * scale


@pytest.mark.parametrize("name", list(CASES))
def test_smoother_parity(name):
    wl, o, mgo, p, h = _pair(name)
    for l, lv in enumerate(o.levels):
        _log(name, "sweep level", l)
        x = _rand(300 + l, lv.ndof)
        b = _rand(400 + l, lv.ndof)
        ref = mgo.smooth(l, x, b)
        xo = torch.zeros(lv.ndof, dtype=torch.float64, device="cuda")
        h.sweep(l, dev(b), dev(x), xo)
        scale = np.abs(ref).max() + np.abs(abs(lv.A) @ np.abs(x)).max()
        assert np.abs(host(xo) - ref).max() <= 1e-12 * scale
        h.sweep0(l, dev(b), xo)
        ref0 = mgo.smooth(l, np.zeros_like(b), b)
        assert np.abs(host(xo) - ref0).max() <= 1e-12 * np.abs(ref0).max()


@pytest.mark.parametrize("name", list(CASES))
def test_transfer_parity(name):
    wl, o, mgo, p, h = _pair(name)
    for l in range(1, len(o.levels)):
        _log(name, "transfer level", l)
        f, c = o.levels[l], o.levels[l - 1]
        r = _rand(500 + l, f.ndof)
        d = torch.zeros(c.ndof, dtype=torch.float64, device="cuda")
        h.restrict(l, dev(r), d)
        ref = f.R @ r
        got = host(d)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(r).max() * 8
        assert np.all(got[c.mask.ravel()] == 0.0)
        y = _rand(600 + l, c.ndof)
        x = _rand(700 + l, f.ndof)
        xt = dev(x)
        h.prolong(l, dev(y), xt)
        ref = x + f.P @ y
        assert np.abs(host(xt) - ref).max() <= 1e-13 * (np.abs(x).max() + np.abs(y).max())


@pytest.mark.parametrize("name", list(CASES))
def test_coarse_solve_parity(name):
    wl, o, mgo, p, h = _pair(name)
    b = _rand(800, o.levels[0].ndof)
    b[o.levels[0].mask.ravel()] = 0.0
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    h.coarse_solve(dev(b), x)
    ref = mgo.coarse_solve(b)
    assert np.abs(host(x) - ref).max() <= 1e-12 * np.abs(ref).max() * max(1.0, np.linalg.cond(mgo.A0) / 1e3)


@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_parity_and_determinism(name):
    wl, o, mgo, p, h = _pair(name)
    _log(name, "vcycle")
    b = o.b.copy()
    ref = mgo.vcycle(b)
    x1 = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(x1)
    h.vcycle(dev(b), x1)
    h.vcycle(dev(b), x2)
    g1, g2 = host(x1), host(x2)
    assert np.array_equal(g1, g2)                       # bitwise deterministic
    assert np.abs(g1 - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", list(CASES))
def test_fixed_cycles_parity(name):
    wl, o, mgo, p, h = _pair(name)
    _log(name, "fixed cycles")
    k = 6
    ref, st_ref = mgo.solve(o.b, fixed_iters=k)
    x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    st = h.solve(dev(o.b), x, fixed=k)
    assert st["iters"] == st_ref.iters == k
    assert np.linalg.norm(host(x) - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", list(CASES))
def test_converged_solution_parity(name):
    wl, o, mgo, p, h = _pair(name)
    _log(name, "solve")
    ref, st_ref = mgo.solve(o.b)
    x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    st = h.solve(dev(o.b), x)
    _log(name, "gpu", st, "oracle iters", st_ref.iters)
    assert st["converged"] == 1 and st_ref.converged
    assert st["iters"] == st_ref.iters
    got = host(x)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
    res = np.linalg.norm(o.b - o.finest.A @ got)
    assert res <= wl.rtol * np.linalg.norm(o.b) * (1 + 1e-9)


def test_single_level_hierarchy():
    from paper_2405_05047_amd import gen, mg
    wl = W.c1_poisson(0)
    o = Hh.build(wl)
    p = gen.build(wl)
    h = mg.Hierarchy(p.levels, mg.config_from(wl))
    assert h.n_levels == 1
    b = _rand(900, o.finest.ndof)
    b[o.finest.mask.ravel()] = 0
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    h.vcycle(dev(b), x)
    assert np.abs(host(x) - MG.Multigrid(o).vcycle(b)).max() <= 1e-13


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("name", ["td_band", "elast17", "oseen17"])
def test_mixed_precision_reaches_fp64_tolerance(name, prec):
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    _log(name, "mixed", prec)
    h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
    x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    st = h.solve(dev(o.b), x)
    got = host(x)
    res = np.linalg.norm(o.b - o.finest.A @ got)
    ref, st_ref = mgo.solve(o.b)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _log(name, prec, "iters", st["iters"], "fp64 iters", st_ref.iters, "rel err vs fp64 oracle", err)
    assert st["converged"] == 1
    assert res <= wl.rtol * np.linalg.norm(o.b) * (1 + 1e-9)
    assert err <= 1e-6


@pytest.mark.parametrize("name", ["td_band", "elast17", "oseen17"])
def test_tail_kernel_parity(name, monkeypatch):
    """The optional single-workgroup tail (levels below MGQ1_TAIL_DOFS in one launch)
    computes the same V-cycle."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    monkeypatch.setenv("MGQ1_TAIL_DOFS", "100000")
    h = mg.Hierarchy(p.levels, mg.config_from(wl))
    ref = mgo.vcycle(o.b)
    x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    h.vcycle(dev(o.b), x)
    assert np.abs(host(x) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["td_band", "oseen17", "td_band_cl3"])
def test_graph_and_eager_agree(name):
    """FGMRES with the captured per-step graphs gives the same result bit for bit as the
    eager launches, also on repeated calls."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    he = mg.Hierarchy(p.levels, mg.config_from(wl, use_graph=0))
    hg = mg.Hierarchy(p.levels, mg.config_from(wl, use_graph=1))
    b = dev(o.b)
    xe = torch.zeros_like(b)
    st_e = he.solve(b, xe)
    ge = host(xe)
    for rep in range(3):
        xg = torch.zeros_like(b)
        st_g = hg.solve(b, xg)
        torch.cuda.synchronize()
        assert st_g["iters"] == st_e["iters"]
        assert np.array_equal(host(xg), ge), rep


@pytest.mark.parametrize("name", ["poisson33", "td_band", "elast17", "oseen17", "edge4"])
def test_slot_batch_variants_bitwise_equal(name):
    """Both slot-batch sizes (and the autotuned choice) run the FMAs in slot order, so the
    V-cycle and the solve are bitwise identical whichever size a level uses."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    kb_pairs = {1: (8, 16), 3: (4, 8), 4: (4, 8)}[wl.block]
    outs = []
    for kb in (0,) + kb_pairs:
        h = mg.Hierarchy(p.levels, mg.config_from(wl, slot_batch=kb))
        for l in range(h.n_levels):
            used, t0, t1 = h.tuning(l)
            assert used in kb_pairs and (kb == 0 or used == kb)
            assert (t0 > 0 and t1 > 0) if kb == 0 else (t0 == 0 and t1 == 0)
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        h.vcycle(dev(o.b), x)
        xs = torch.zeros_like(x)
        st = h.solve(dev(o.b), xs)
        outs.append((host(x), host(xs), st["iters"]))
    for v, s, it in outs[1:]:
        assert np.array_equal(v, outs[0][0]) and np.array_equal(s, outs[0][1]) and it == outs[0][2]


def test_slot_batch_rejects_unbuilt_size():
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair("td_band")
    with pytest.raises(mg.MGError):
        mg.Hierarchy(p.levels, mg.config_from(wl, slot_batch=5))


@pytest.mark.parametrize("name", ["poisson33", "td_band", "td_band_cl3"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_fused_presmoothing_bitwise_equal(name, prec, monkeypatch):
    """For one component per node the first two pre-sweeps run as one pass that forms
    x1 = omega S b on the fly; it gives bitwise the V-cycle of the two separate sweeps."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    outs = []
    for off in ("0", "1"):
        monkeypatch.setenv("MGQ1_NO_FUSE", off)
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        h.vcycle(dev(o.b), x)
        outs.append(host(x))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("name", ["td_band", "elast17"])
def test_zero_rhs_and_exact_initial_guess(name):
    """b = 0 is solved by x = 0 without a cycle; an initial guess that already satisfies the
    tolerance is returned unchanged."""
    import scipy.sparse.linalg as sla
    wl, o, mgo, p, h = _pair(name)
    z = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(z)
    st = h.solve(z, x)
    assert st["iters"] == 0 and st["converged"] == 1 and np.all(host(x) == 0.0)
    xe = sla.spsolve(o.finest.A.tocsc(), o.b)
    x = dev(xe)
    st = h.solve(dev(o.b), x)
    assert st["iters"] == 0 and st["converged"] == 1 and np.array_equal(host(x), xe)


@pytest.mark.parametrize("name", ["poisson33", "td_band", "elast17", "oseen17", "edge4"])
@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_column_formats_bitwise_equal(name, prec, monkeypatch):
    """Operators whose column differences fit 16 bits are read in that format; the result
    is bitwise the one of the 32-bit column indices."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    outs = []
    for off in ("0", "1"):
        monkeypatch.setenv("MGQ1_NO_COL16", off)
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        st = h.solve(dev(o.b), x)
        outs.append((host(x), st["iters"]))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


@pytest.mark.parametrize("name", ["poisson33", "td_band", "elast17", "oseen17", "edge4"])
@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_slice_widths_bitwise_equal(name, prec, monkeypatch):
    """Levels whose slices are padded to one uniform width (the kernels then compute each
    slice's slot range) give bitwise the result of variable slice widths: padding slots add
    exact zeros.  Also covers the transfer matrices, which follow the same rule."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    outs = []
    for off in ("0", "1"):
        monkeypatch.setenv("MGQ1_NO_ELL", off)
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        st = h.solve(dev(o.b), x)
        outs.append((host(x), st["iters"]))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


@pytest.mark.parametrize("name", ["elast17", "oseen17", "edge4"])
@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_sorted_rows_neutral(name, prec, monkeypatch):
    """Block rows sorted by length inside windows of slices (a row keeps its own slot
    order, only its lane moves): the V-cycle is bitwise that of node order; solves differ
    only by the summation order of the Krylov inner products."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    vc, sol = [], []
    for off in ("0", "1"):
        monkeypatch.setenv("MGQ1_NO_SORT", off)
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        h.vcycle(dev(o.b), x)
        vc.append(host(x))
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        st = h.solve(dev(o.b), x)
        sol.append((host(x), st["iters"]))
    assert np.array_equal(vc[0], vc[1])
    assert abs(sol[0][1] - sol[1][1]) <= 1
    assert np.linalg.norm(sol[0][0] - sol[1][0]) <= 1e-8 * np.linalg.norm(sol[1][0])


@pytest.mark.parametrize("name", ["poisson33", "td_band", "elast17", "edge4"])
@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_mixed_column_format_bitwise_equal(name, prec, monkeypatch):
    """Slices whose columns do not fit 16-bit offsets read the 32-bit indices while the
    others read the offsets (here every 17th slice is forced to the 32-bit form); the
    result is bitwise that of 32-bit indices everywhere."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    outs = []
    for env in ({"MGQ1_WIDE_EVERY": "17", "MGQ1_NO_COL16": "0"}, {"MGQ1_WIDE_EVERY": "0", "MGQ1_NO_COL16": "1"}):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
        if env["MGQ1_NO_COL16"] == "0":
            assert h.col_bytes(h.n_levels - 1) == 2
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        st = h.solve(dev(o.b), x)
        outs.append((host(x), st["iters"]))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


@pytest.mark.parametrize("name", ["poisson33", "td_band", "elast17", "oseen17", "edge4", "oseen_tall"])
@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_compact_transfers_bitwise_equal(name, prec, monkeypatch):
    """Transfers in the node form (one lane per node; 16-bit column offsets, 8-bit weight
    codes w = code / 128 for the dyadic weights of nested box meshes, and the column mask
    bits packed into one 32-bit word per slot) give bitwise the restriction,
    prolongation, V-cycle and solve of the per-DoF form with 32-bit columns and FP32/FP64
    weights: the codes decode exactly and every row keeps its slot order."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    outs = []
    for plain in ("0", "1"):
        monkeypatch.setenv("MGQ1_PLAIN_TRANSFERS", plain)
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
        fmt = [h.transfer_format(l) for l in range(1, h.n_levels)]
        if plain == "1":
            assert all(f[0] == 4 and f[1] == 4 and f[2] in (4, 8) for f in fmt), fmt
        else:
            assert fmt[-1] == (2, 2, 1), fmt
            compact = fmt
        steps = []
        if prec == "fp64":
            for l in range(1, h.n_levels):
                f, c = o.levels[l], o.levels[l - 1]
                d = torch.zeros(c.ndof, dtype=torch.float64, device="cuda")
                h.restrict(l, dev(_rand(900 + l, f.ndof)), d)
                xt = dev(_rand(950 + l, f.ndof))
                h.prolong(l, dev(_rand(990 + l, c.ndof)), xt)
                steps += [host(d), host(xt)]
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        h.vcycle(dev(o.b), x)
        vc = host(x)
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        st = h.solve(dev(o.b), x)
        outs.append((steps, vc, host(x), st["iters"]))
    (s0, v0, x0, i0), (s1, v1, x1, i1) = outs
    assert all(np.array_equal(a, b) for a, b in zip(s0, s1))
    assert np.array_equal(v0, v1) and np.array_equal(x0, x1) and i0 == i1
    _log(name, prec, "compact transfers bitwise equal; formats", compact)


@pytest.mark.parametrize("change", ["off_grid", "not_fp32", "negative", "large"])
@pytest.mark.parametrize("name", ["td_band", "elast17"])
def test_transfers_fall_back_per_level(name, change, monkeypatch):
    """One P~ weight of the finest level that the 8-bit code w * 128 in [0, 255] cannot
    hold (w (1 + 2^-20), w (1 + 2^-40), -w, or 2.5): that level's transfers fall back by
    themselves to the per-DoF form with 32-bit columns and FP32 weights (FP64 for
    w (1 + 2^-40), which FP32 does not hold), the coarser levels keep the form they had,
    and restriction, prolongation, V-cycle and a fixed-count solve are bitwise those of
    the per-DoF form on every level."""
    import dataclasses
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    levels = list(p.levels)
    fin = levels[-1]
    pv = fin.p_val.copy()
    j = int(np.flatnonzero((pv > 0) & (pv < 1))[0])
    pv[j] = {"off_grid": pv[j] * (1 + 2.0 ** -20), "not_fp32": pv[j] * (1 + 2.0 ** -40),
             "negative": -pv[j], "large": 2.5}[change]
    levels[-1] = dataclasses.replace(fin, p_val=pv)
    before = [h64.transfer_format(l) for l in range(1, h64.n_levels)]
    assert before[-1] == (2, 2, 1), before
    outs = []
    for plain in ("0", "1"):
        monkeypatch.setenv("MGQ1_PLAIN_TRANSFERS", plain)
        h = mg.Hierarchy(levels, mg.config_from(wl))
        fmt = [h.transfer_format(l) for l in range(1, h.n_levels)]
        if plain == "0":
            wbytes = 8 if change == "not_fp32" else 4
            assert fmt[:-1] == before[:-1] and fmt[-1] == (4, 4, wbytes), (fmt, before)
        steps = []
        for l in range(1, h.n_levels):
            f, c = o.levels[l], o.levels[l - 1]
            d = torch.zeros(c.ndof, dtype=torch.float64, device="cuda")
            h.restrict(l, dev(_rand(1500 + l, f.ndof)), d)
            xt = dev(_rand(1550 + l, f.ndof))
            h.prolong(l, dev(_rand(1590 + l, c.ndof)), xt)
            steps += [host(d), host(xt)]
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        h.vcycle(dev(o.b), x)
        vc = host(x)
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        h.solve(dev(o.b), x, fixed=4)
        outs.append((steps, vc, host(x)))
    (s0, v0, x0), (s1, v1, x1) = outs
    assert all(np.array_equal(a, b) for a, b in zip(s0, s1))
    assert np.array_equal(v0, v1) and np.array_equal(x0, x1)


@pytest.mark.parametrize("name", ["poisson33", "td_band", "elast17", "oseen17", "edge4", "oseen_tall"])
def test_dictionary_form_bitwise_equal(name):
    """MG_PREC_FP64_DICT stores each level's distinct FP64 blocks once and a 16-bit index
    per stored block: the kernels read the same doubles in the same order, so every step
    (SpMV, defect, sweep on every level), the V-cycle and the solve are bitwise those of
    the plain FP64 handle."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    hd = mg.Hierarchy(p.levels, mg.config_from(wl, precision="fp64dict"))
    nd = [hd.dictionary_blocks(l) for l in range(hd.n_levels)]
    assert nd[-1] > 0, nd
    for l, lv in enumerate(o.levels):
        x = dev(_rand(1300 + l, lv.ndof))
        b = dev(_rand(1350 + l, lv.ndof))
        outs = []
        for h in (h64, hd):
            y = torch.zeros_like(x)
            h.spmv(l, x, y)
            xo = torch.zeros_like(x)
            h.sweep(l, b, x, xo)
            outs.append((host(y), host(xo)))
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1]), l
    res = []
    for h in (h64, hd):
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        h.vcycle(dev(o.b), x)
        v = host(x)
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        st = h.solve(dev(o.b), x)
        res.append((v, host(x), st["iters"]))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1]) and res[0][2] == res[1][2]
    with pytest.raises(mg.MGError, match="dictionary"):
        hd.export(hd.n_levels - 1)
    _log(name, "dictionary form bitwise equal; distinct blocks per level", nd)


def test_dictionary_form_with_chebyshev():
    """The Chebyshev-accelerated smoother on the dictionary form: bitwise the plain FP64
    solve."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair("elast17")
    res = []
    for prec in ("fp64", "fp64dict"):
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec, smoother=W.SMOOTH_CHEBYSHEV))
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        st = h.solve(dev(o.b), x)
        res.append((host(x), st["iters"]))
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1] == res[1][1]


@pytest.mark.parametrize("perturbed", [40000, "all"])
def test_dictionary_form_large_and_refused_tables(perturbed):
    """The finest elasticity operator with `perturbed` of its blocks (those between two
    unconstrained nodes) scaled by distinct factors 1 + 1e-6 u: about 40,000 distinct
    blocks still form a dictionary (a 2.9 MB table read through the caches), more than
    65,535 leave that level's values plain while the coarser levels keep theirs.  Either
    way every step and the solve are bitwise those of the plain FP64 handle on the same
    operators."""
    import dataclasses
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair("elast17")
    levels = list(p.levels)
    fin = levels[-1]
    nnzb = len(fin.val)
    # blocks coupling two unconstrained nodes (constrained rows and columns stay identity)
    free = ~fin.mask.astype(bool).any(axis=1)
    sel = np.flatnonzero(free[np.repeat(np.arange(fin.n), np.diff(fin.rowptr))] & free[fin.col])
    sel = sel if perturbed == "all" else sel[:perturbed]
    val = fin.val.copy()
    val[sel] *= (1.0 + 1e-6 * _rand(1400, len(sel)))[:, None, None]
    levels[-1] = dataclasses.replace(fin, val=val)
    distinct = len(np.unique(val.reshape(nnzb, -1).view(np.uint64), axis=0))
    assert (distinct > 65535) == (perturbed == "all"), distinct
    hp = mg.Hierarchy(levels, mg.config_from(wl))
    hd = mg.Hierarchy(levels, mg.config_from(wl, precision="fp64dict"))
    nd = [hd.dictionary_blocks(l) for l in range(hd.n_levels)]
    if perturbed == "all":
        assert nd[-1] == 0, nd
    else:
        assert distinct <= nd[-1] <= distinct + 1, (nd, distinct)   # + the zero padding block
    assert all(n > 0 for n in nd[1:-1]), nd
    L = hd.n_levels - 1
    x = dev(_rand(1401, fin.n * fin.block))
    b = dev(_rand(1402, fin.n * fin.block))
    outs = []
    for h in (hp, hd):
        y = torch.zeros_like(x)
        h.spmv(L, x, y)
        xo = torch.zeros_like(x)
        h.sweep(L, b, x, xo)
        z = torch.zeros_like(x)
        st = h.solve(b, z)
        outs.append((host(y), host(xo), host(z), st["iters"]))
    for a, c in zip(outs[0], outs[1]):
        assert np.array_equal(a, c)
    _log("perturbed", perturbed, "distinct", distinct, "dictionary blocks per level", nd)


def _drop_masked_prolongation_rows(levels):
    """The levels with every P~ row of a fully masked fine node emptied.  Such a row never
    reaches a result: the prolongation leaves masked DoFs unchanged and the V-cycle's fine
    defect is zero there, so the restriction only loses terms w * 0."""
    import dataclasses
    out = [levels[0]]
    for lv in levels[1:]:
        keep = ~lv.mask.all(axis=1)
        ln = np.diff(lv.p_rowptr) * keep
        rp = np.concatenate([[0], np.cumsum(ln)]).astype(lv.p_rowptr.dtype)
        sel = np.repeat(keep, np.diff(lv.p_rowptr))
        out.append(dataclasses.replace(lv, p_rowptr=rp, p_col=lv.p_col[sel].copy(), p_val=lv.p_val[sel].copy()))
    return out


@pytest.mark.parametrize("name", ["td_band", "elast17", "edge4"])
def test_node_form_with_empty_rows_bitwise_equal(name, monkeypatch):
    """Transfers with empty rows (fully masked fine nodes without P~ entries): the node
    form's lanes of empty rows read the slot's base column and add 0 * x to +0, the per-DoF
    form reads column 0; prolongation, restriction and V-cycle agree bit for bit."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    levels = _drop_masked_prolongation_rows(p.levels)
    assert any(np.any(np.diff(lv.p_rowptr) == 0) for lv in levels[1:])
    outs = []
    for plain in ("0", "1"):
        monkeypatch.setenv("MGQ1_PLAIN_TRANSFERS", plain)
        h = mg.Hierarchy(levels, mg.config_from(wl))
        assert h.transfer_format(h.n_levels - 1)[0] == (4 if plain == "1" else 2)
        res = []
        for l in range(1, h.n_levels):
            f, c = o.levels[l], o.levels[l - 1]
            d = torch.zeros(c.ndof, dtype=torch.float64, device="cuda")
            h.restrict(l, dev(_rand(1100 + l, f.ndof)), d)
            xt = dev(_rand(1150 + l, f.ndof))
            h.prolong(l, dev(_rand(1190 + l, c.ndof)), xt)
            res += [host(d), host(xt)]
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        h.vcycle(dev(o.b), x)
        res.append(host(x))
        outs.append(res)
    assert all(np.array_equal(a, b) for a, b in zip(*outs))
    # and the V-cycle equals the one with the full transfers (masked rows never reach it)
    x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    h64.vcycle(dev(o.b), x)
    assert np.abs(host(x) - outs[0][-1]).max() <= 1e-14 * np.abs(host(x)).max()


@pytest.mark.parametrize("name", ["td_band", "elast17"])
@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_load_kinds_bitwise_equal(name, prec, monkeypatch):
    """Operator streams read with non-temporal or ordinary loads (chosen per level by its
    size) give bitwise the same solve."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h64 = _pair(name)
    outs = []
    for kind in ("nt", "t"):
        monkeypatch.setenv("MGQ1_LOADS", kind)
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
        x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
        st = h.solve(dev(o.b), x)
        outs.append((host(x), st["iters"]))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


@pytest.mark.parametrize("name", ["poisson33", "td_band", "elast17", "oseen17", "edge4"])
def test_vcycle_from_initial_iterate(name):
    """GMG(L, x, b) with a nonzero initial iterate (mg_vcycle, x_is_zero = 0) against the
    oracle's recursion from the same x, for V(2,2) and for an odd sweep count V(1,2)."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h = _pair(name)
    x0 = _rand(950, o.finest.ndof)
    x0[o.finest.mask.ravel()] = 0.0
    ref = mgo.gmg(o.L, x0.copy(), o.b)
    x = dev(x0)
    h.vcycle(dev(o.b), x, x_is_zero=False)
    assert np.abs(host(x) - ref).max() <= 1e-12 * np.abs(ref).max()
    h12 = mg.Hierarchy(p.levels, mg.config_from(wl, nu1=1, nu2=2))
    mg12 = MG.Multigrid(o, nu1=1, nu2=2)
    ref = mg12.gmg(o.L, x0.copy(), o.b)
    x = dev(x0)
    h12.vcycle(dev(o.b), x, x_is_zero=False)
    assert np.abs(host(x) - ref).max() <= 1e-12 * np.abs(ref).max()
    # from zero the two forms agree bitwise
    xa = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    xb = torch.zeros_like(xa)
    h.vcycle(dev(o.b), xa)
    h.vcycle(dev(o.b), xb, x_is_zero=False)
    ref0 = mgo.vcycle(o.b)
    assert np.abs(host(xb) - ref0).max() <= 1e-12 * np.abs(ref0).max()
    assert np.abs(host(xa) - host(xb)).max() <= 1e-12 * np.abs(ref0).max()


@pytest.mark.parametrize("name", ["td_band", "elast17", "oseen17"])
def test_mixed_vcycle_from_initial_iterate(name):
    """The mixed form's GMG(L, x, b) stays within FP32 accuracy of the FP64 recursion."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h = _pair(name)
    hm = mg.Hierarchy(p.levels, mg.config_from(wl, precision="fp32"))
    x0 = _rand(951, o.finest.ndof)
    x0[o.finest.mask.ravel()] = 0.0
    ref = mgo.gmg(o.L, x0.copy(), o.b)
    x = dev(x0)
    hm.vcycle(dev(o.b), x, x_is_zero=False)
    assert np.linalg.norm(host(x) - ref) <= 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["td_band", "elast17", "oseen17"])
def test_caller_smoother_blocks(name):
    """mg_level_in.smoother_blocks: the oracle's block inverses reproduce the derived
    smoother; a different fixed S (0.5 times them) is the one the sweeps then apply."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h = _pair(name)
    S = [MG.smoother_blocks(lv) for lv in o.levels]
    h1 = mg.Hierarchy(p.levels, mg.config_from(wl), smoother_blocks=S)
    h2 = mg.Hierarchy(p.levels, mg.config_from(wl), smoother_blocks=[0.5 * s for s in S])
    for l, lv in enumerate(o.levels):
        x = _rand(960 + l, lv.ndof)
        b = _rand(970 + l, lv.ndof)
        ref = mgo.smooth(l, x, b)
        scale = np.abs(ref).max() + np.abs(abs(lv.A) @ np.abs(x)).max()
        xo = torch.zeros(lv.ndof, dtype=torch.float64, device="cuda")
        h1.sweep(l, dev(b), dev(x), xo)
        assert np.abs(host(xo) - ref).max() <= 1e-12 * scale
        h2.sweep(l, dev(b), dev(x), xo)
        ref2 = x + wl.omega * 0.5 * mgo.apply_S(l, b - lv.A @ x)
        assert np.abs(host(xo) - ref2).max() <= 1e-12 * scale
    # the V-cycle with the oracle's blocks is the default V-cycle
    xa = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    h1.vcycle(dev(o.b), xa)
    ref = mgo.vcycle(o.b)
    assert np.abs(host(xa) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["td_band", "elast17", "oseen17"])
@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_outer_defect(name, prec):
    """mg_outer_defect: r = b - A_L x and ||r|| in FP64 on the finest FP64 operator,
    whatever the cycle precision."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h = _pair(name)
    hh = h if prec == "fp64" else mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
    x = _rand(980, o.finest.ndof)
    ref = o.b - o.finest.A @ x
    r = torch.zeros(len(x), dtype=torch.float64, device="cuda")
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    hh.outer_defect(dev(o.b), dev(x), r, nrm)
    scale = np.abs(o.b).max() + np.abs(abs(o.finest.A) @ np.abs(x)).max()
    assert np.abs(host(r) - ref).max() <= 1e-12 * scale
    assert abs(float(host(nrm)[0]) - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["poisson33", "td_band", "elast17"])
def test_coarse_smooth_mode(name):
    """MG_COARSE_SMOOTH (the paper's GPU coarse variant: a few smoothing sweeps from 0 on
    the coarse level): coarse step, V-cycle and a converged solve against the oracle."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, _ = _pair(name)
    wl = wl.with_(coarse_mode=W.COARSE_SMOOTH, coarse_sweeps=7)
    o = Hh.build(wl)
    mgo = MG.Multigrid(o)
    h = mg.Hierarchy(p.levels, mg.config_from(wl))
    b0 = _rand(990, o.levels[0].ndof)
    b0[o.levels[0].mask.ravel()] = 0.0
    x0 = torch.zeros(len(b0), dtype=torch.float64, device="cuda")
    h.coarse_solve(dev(b0), x0)
    ref = mgo.coarse_solve(b0)
    assert np.abs(host(x0) - ref).max() <= 1e-12 * np.abs(ref).max()
    x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    h.vcycle(dev(o.b), x)
    ref = mgo.vcycle(o.b)
    assert np.abs(host(x) - ref).max() <= 1e-12 * np.abs(ref).max()
    x.zero_()
    st = h.solve(dev(o.b), x)
    xr, st_ref = mgo.solve(o.b)
    assert st["converged"] == 1 and st_ref.converged and st["iters"] == st_ref.iters
    assert np.linalg.norm(host(x) - xr) <= 1e-10 * np.linalg.norm(xr)


def test_aliasing_rejected():
    """Outputs that alias inputs are refused with MG_EINVAL before any device work."""
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h = _pair("td_band")
    v = dev(o.b)
    w = torch.zeros_like(v)
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda")
    L = o.L
    calls = [lambda: h.vcycle(v, v), lambda: h.vcycle(v, v, x_is_zero=False),
             lambda: h.sweep(L, v, w, w), lambda: h.sweep(L, w, v, w), lambda: h.sweep0(L, v, v),
             lambda: h.spmv(L, v, v), lambda: h.defect(L, v, w, w), lambda: h.outer_defect(v, w, w, nrm)]
    for call in calls:
        with pytest.raises(mg.MGError) as e:
            call()
        assert e.value.code == -1
