"""GPU parity of the batched form: many independent problems with several right-hand
sides solved together (one launch per V-cycle step over all problems, lockstep FGMRES).

Batching does not change the mathematics, so every (problem, rhs) instance is compared
with the oracle's own single solve of that instance: FP64 batches to the single-solve
bars (iteration counts equal, 1e-10 relative solutions); FP32 batches reach the FP64
residual tolerance, with the error against the FP64 oracle bounded.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import hierarchy as Hh, multigrid as MG

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print("[gpu-batch]", *a, flush=True)
    sys.stdout.flush()


def _td_batch():
    # uneven problems: 3..5 levels, so the V-cycles of the batch have different depths
    return W.batch_problems(n_problems=4, base_seed=2000, max_levels=5, min_levels=3)


GROUPS = {
    "td_nrhs8": (_td_batch, 8),
    "td_nrhs1": (_td_batch, 1),
    "elast_nrhs1": (lambda: [W.c3_elasticity(2), W.c3_elasticity(3).with_(coarse_level=1),
                             W.c3_adaptive("edge", 3)], 1),
    "oseen_nrhs1": (lambda: [W.c4_oseen(2), W.c4_oseen(3), W.c4_oseen(2, seed=5)], 1),
}

_cache = {}


def _group(name):
    """(workloads, oracle hierarchies, generated problems, batch rhs (host, flat))."""
    if name not in _cache:
        from paper_2405_05047_amd import gen
        make, nrhs = GROUPS[name]
        wls = make()
        _log("building", name)
        ors = [Hh.build(wl, nrhs) for wl in wls]
        gps = [gen.build(wl, nrhs) for wl in wls]
        b = np.concatenate([np.asarray(o.b, np.float64).reshape(-1) for o in ors])
        _cache[name] = (wls, ors, gps, b, nrhs)
    return _cache[name]


def _oracle_solutions(name):
    key = ("ref", name)
    if key not in _cache:
        wls, ors, gps, b, nrhs = _group(name)
        refs = []
        for o in ors:
            mgo = MG.Multigrid(o)
            bb = np.asarray(o.b).reshape(o.finest.ndof, nrhs)
            for q in range(nrhs):
                refs.append(mgo.solve(np.ascontiguousarray(bb[:, q])))
        _cache[key] = refs
    return _cache[key]


def _batch(name, precision="fp64", use_graph=1):
    from paper_2405_05047_amd import mg
    wls, ors, gps, b, nrhs = _group(name)
    cfg = mg.config_from(wls[0], precision=precision, use_graph=use_graph)
    return mg.Batch([p.levels for p in gps], cfg, nrhs=nrhs)


def _instances(bt, x, ors, nrhs):
    """Split a batch vector into per-instance (problem, rhs) columns."""
    out = []
    for p, o in enumerate(ors):
        seg = x[bt.offsets[p]:bt.offsets[p + 1]].reshape(o.finest.ndof, nrhs)
        for q in range(nrhs):
            out.append(seg[:, q])
    return out


def test_batch_offsets_match_problem_sizes():
    wls, ors, gps, b, nrhs = _group("td_nrhs8")
    bt = _batch("td_nrhs8")
    sizes = np.diff(bt.offsets)
    assert list(sizes) == [o.finest.ndof * nrhs for o in ors]
    assert bt.size == len(b)


@pytest.mark.parametrize("name", list(GROUPS))
def test_batch_fp64_matches_single_solves(name):
    wls, ors, gps, b, nrhs = _group(name)
    refs = _oracle_solutions(name)
    bt = _batch(name)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    rc, st = bt.solve(bd, x)
    torch.cuda.synchronize()
    got = _instances(bt, x.cpu().numpy(), ors, nrhs)
    assert rc == 0
    for i, ((ref, sr), g, s) in enumerate(zip(refs, got, st)):
        _log(name, "instance", i, "gpu iters", s["iters"], "oracle iters", sr.iters)
        assert s["converged"] == 1 and sr.converged
        assert s["iters"] == sr.iters, i
        assert np.linalg.norm(g - ref) <= 1e-10 * np.linalg.norm(ref), i


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
@pytest.mark.parametrize("name", ["td_nrhs8", "elast_nrhs1", "oseen_nrhs1"])
def test_batch_mixed_reaches_fp64_tolerance(name, prec):
    wls, ors, gps, b, nrhs = _group(name)
    refs = _oracle_solutions(name)
    bt = _batch(name, precision=prec)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    rc, st = bt.solve(bd, x)
    torch.cuda.synchronize()
    got = _instances(bt, x.cpu().numpy(), ors, nrhs)
    bs = _instances(bt, b, ors, nrhs)
    assert rc == 0
    k = 0
    for p, o in enumerate(ors):
        for q in range(nrhs):
            g, (ref, sr) = got[k], refs[k]
            res = np.linalg.norm(bs[k] - o.finest.A @ g)
            err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
            _log(name, prec, "instance", k, "iters", st[k]["iters"], "fp64", sr.iters, "rel err", err)
            assert st[k]["converged"] == 1
            assert res <= wls[p].rtol * np.linalg.norm(bs[k]) * (1 + 1e-9)
            assert err <= 1e-6
            k += 1


def test_batch_graph_and_eager_agree():
    """Captured per-step graphs and plain launches give the same batch result bit for bit,
    also on repeated calls."""
    wls, ors, gps, b, nrhs = _group("td_nrhs8")
    be = _batch("td_nrhs8", use_graph=0)
    bg = _batch("td_nrhs8", use_graph=1)
    bd = torch.from_numpy(b).cuda()
    xe = torch.zeros_like(bd)
    rc, st_e = be.solve(bd, xe)
    ge = xe.cpu().numpy()
    for rep in range(3):
        xg = torch.zeros_like(bd)
        rc, st_g = bg.solve(bd, xg)
        torch.cuda.synchronize()
        assert [s["iters"] for s in st_g] == [s["iters"] for s in st_e]
        assert np.array_equal(xg.cpu().numpy(), ge), rep


def test_batch_nonzero_initial_guess_and_converged_instances():
    """An instance that starts at its solution is left untouched (0 iterations) while the
    others of the batch iterate exactly as in their single solves."""
    import scipy.sparse.linalg as sla
    wls, ors, gps, b, nrhs = _group("td_nrhs8")
    refs = _oracle_solutions("td_nrhs8")
    bt = _batch("td_nrhs8")
    x0 = np.zeros_like(b)
    # put instance (problem 1, rhs 3) at the direct solution of its system
    seg = x0[bt.offsets[1]:bt.offsets[2]].reshape(ors[1].finest.ndof, nrhs)
    bseg = b[bt.offsets[1]:bt.offsets[2]].reshape(ors[1].finest.ndof, nrhs)
    seg[:, 3] = sla.spsolve(ors[1].finest.A.tocsc(), bseg[:, 3])
    special = 1 * nrhs + 3
    bd = torch.from_numpy(b).cuda()
    x = torch.from_numpy(x0).cuda()
    rc, st = bt.solve(bd, x)
    torch.cuda.synchronize()
    assert rc == 0
    assert st[special]["iters"] == 0 and st[special]["converged"] == 1
    got = _instances(bt, x.cpu().numpy(), ors, nrhs)
    assert np.array_equal(got[special], seg[:, 3])
    for i, ((ref, sr), g) in enumerate(zip(refs, got)):
        if i != special:
            assert st[i]["iters"] == sr.iters, i
            assert np.linalg.norm(g - ref) <= 1e-10 * np.linalg.norm(ref), i


def test_batch_maxit_per_instance():
    """With a V-cycle budget below the iteration counts every instance stops at exactly
    that budget and reports no convergence."""
    from paper_2405_05047_amd import mg
    wls, ors, gps, b, nrhs = _group("td_nrhs1")
    cfg = mg.config_from(wls[0], maxit=3)
    bt = mg.Batch([p.levels for p in gps], cfg, nrhs=nrhs)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    rc, st = bt.solve(bd, x)
    assert rc == -5
    for s in st:
        assert s["iters"] == 3 and s["converged"] == 0


def test_batch_of_one_problem_and_single_level_member():
    """Degenerate batches: one problem alone, and a batch whose member has a single level
    (the V-cycle is the exact coarse solve, so FGMRES needs one cycle)."""
    import scipy.sparse.linalg as sla
    from paper_2405_05047_amd import gen, mg
    wls = [W.c2_td(band_rounds=1, uniform_rounds=1),
           W.c2_td(band_rounds=1, uniform_rounds=0).with_(coarse_level=5)]
    ors = [Hh.build(wl) for wl in wls]
    assert len(ors[1].levels) == 1
    gps = [gen.build(wl) for wl in wls]
    for members in ([0], [0, 1], [1]):
        cfg = mg.config_from(wls[members[0]])
        bt = mg.Batch([gps[k].levels for k in members], cfg, nrhs=1)
        b = np.concatenate([ors[k].b for k in members])
        bd = torch.from_numpy(b).cuda()
        x = torch.zeros_like(bd)
        rc, st = bt.solve(bd, x)
        assert rc == 0
        xs = x.cpu().numpy()
        for i, k in enumerate(members):
            seg = xs[bt.offsets[i]:bt.offsets[i + 1]]
            ref, sr = MG.Multigrid(ors[k]).solve(ors[k].b)
            assert st[i]["iters"] == sr.iters
            assert np.linalg.norm(seg - ref) <= 1e-10 * np.linalg.norm(ref)
            if k == 1:
                assert st[i]["iters"] == 1
                exact = sla.spsolve(ors[k].finest.A.tocsc(), ors[k].b)
                assert np.linalg.norm(seg - exact) <= 1e-10 * np.linalg.norm(exact)


def test_batch_zero_rhs_instances():
    """Instances with b = 0 are converged at x = 0 before any cycle; the others iterate."""
    wls, ors, gps, b, nrhs = _group("td_nrhs8")
    refs = _oracle_solutions("td_nrhs8")
    bt = _batch("td_nrhs8")
    b0 = b.copy()
    seg = b0[bt.offsets[2]:bt.offsets[3]].reshape(ors[2].finest.ndof, nrhs)
    seg[:, 5] = 0.0
    bd = torch.from_numpy(b0).cuda()
    x = torch.zeros_like(bd)
    rc, st = bt.solve(bd, x)
    assert rc == 0
    z = 2 * nrhs + 5
    assert st[z]["iters"] == 0 and st[z]["converged"] == 1
    got = _instances(bt, x.cpu().numpy(), ors, nrhs)
    assert np.all(got[z] == 0.0)
    for i, ((ref, sr), g) in enumerate(zip(refs, got)):
        if i != z:
            assert st[i]["iters"] == sr.iters, i


def test_batch_slot_batch_variants_bitwise_equal():
    """The batch autotuner's choices change no bit of the result."""
    from paper_2405_05047_amd import mg
    wls, ors, gps, b, nrhs = _group("td_nrhs8")
    bd = torch.from_numpy(b).cuda()
    outs = []
    for kb in (0, 8, 16):
        cfg = mg.config_from(wls[0], precision="fp32", slot_batch=kb)
        bt = mg.Batch([p.levels for p in gps], cfg, nrhs=nrhs)
        x = torch.zeros_like(bd)
        rc, st = bt.solve(bd, x)
        assert rc == 0
        outs.append((x.cpu().numpy(), [s["iters"] for s in st]))
    for x, it in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and it == outs[0][1]


def test_batch_column_formats_bitwise_equal(monkeypatch):
    wls, ors, gps, b, nrhs = _group("td_nrhs8")
    bd = torch.from_numpy(b).cuda()
    outs = []
    for off in ("0", "1"):
        monkeypatch.setenv("MGQ1_NO_COL16", off)
        bt = _batch("td_nrhs8", precision="fp16")
        x = torch.zeros_like(bd)
        rc, st = bt.solve(bd, x)
        assert rc == 0
        outs.append(x.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_batch_slice_widths_bitwise_equal(monkeypatch):
    wls, ors, gps, b, nrhs = _group("td_nrhs8")
    bd = torch.from_numpy(b).cuda()
    outs = []
    for off in ("0", "1"):
        monkeypatch.setenv("MGQ1_NO_ELL", off)
        bt = _batch("td_nrhs8", precision="fp32")
        x = torch.zeros_like(bd)
        rc, st = bt.solve(bd, x)
        assert rc == 0
        outs.append(x.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_batch_mixed_column_format_bitwise_equal(monkeypatch):
    wls, ors, gps, b, nrhs = _group("td_nrhs8")
    bd = torch.from_numpy(b).cuda()
    outs = []
    for every, off in (("17", "0"), ("0", "1")):
        monkeypatch.setenv("MGQ1_WIDE_EVERY", every)
        monkeypatch.setenv("MGQ1_NO_COL16", off)
        bt = _batch("td_nrhs8", precision="fp16")
        x = torch.zeros_like(bd)
        rc, st = bt.solve(bd, x)
        assert rc == 0
        outs.append(x.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
