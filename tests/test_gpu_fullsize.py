"""GPU parity at the benchmark sizes, in the configuration the benchmark times (autotuned
slot batches, graph-replayed FGMRES steps).

The oracle cannot run inside the test at these sizes, so `tests/golden/fullsize_*.json`
(written by tests/golden/make_fullsize.py, which calls only the oracle) holds its results
at a seeded sample of DoFs: one finest-level sweep of seeded vectors, one V-cycle of the
right-hand side, the converged solution and its iteration count.  Tolerances as in the
small-size parity tests: 1e-12 of the sweep scale, 1e-12 of max|V-cycle|, and the
solution within 1e-10 of its norm with equal iteration counts.  The uneven batch runs at
full size with properties (every instance converges to the FP64 tolerance) plus oracle
parity of its smallest members.
"""
import glob
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
FULL = {
    "c2": lambda: W.c2_td().with_(coarse_level=3),
    "c3": lambda: W.c3_elasticity().with_(coarse_level=2),
    "c4": lambda: W.c4_oseen().with_(coarse_level=2),
    "c3f": lambda: W.c3_adaptive("face", 6),
}
GOLDEN = sorted(os.path.basename(p)[9:-5] for p in glob.glob(os.path.join(HERE, "golden", "fullsize_*.json")))


def _log(*a):
    print("[gpu-full]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", GOLDEN)
def test_fullsize_sampled_parity(name):
    from paper_2405_05047_amd import gen, mg
    ref = json.load(open(os.path.join(HERE, "golden", f"fullsize_{name}.json")))
    wl = FULL[name]()
    assert wl.name == ref["workload"] and wl.coarse_level == ref["coarse_level"]
    _log(name, "generating", ref["ndof"], "DoFs")
    p = gen.build(wl)
    h = mg.Hierarchy(p.levels, mg.config_from(wl))
    N = h.ndof()
    assert N == ref["ndof"] and h.n_levels == ref["levels"]
    idx = np.array(ref["idx"], dtype=np.int64)
    L = h.n_levels - 1
    fmt = [h.transfer_format(l) for l in range(1, h.n_levels)]
    _log(name, "transfer formats (P col, R col, weight bytes)", fmt)
    if name in ("c3", "c4"):
        assert fmt[-1] == (2, 2, 1)      # uniform box meshes: the finest transfers in the node form
    _log(name, "sweep")
    x = torch.from_numpy(W.rand_vec(ref["sweep_x_seed"], N)).cuda()
    b = torch.from_numpy(W.rand_vec(ref["sweep_b_seed"], N)).cuda()
    xo = torch.zeros_like(x)
    h.sweep(L, b, x, xo)
    got = xo.cpu().numpy()[idx]
    assert np.abs(got - np.array(ref["sweep"])).max() <= 1e-12 * ref["sweep_scale"]
    _log(name, "vcycle")
    bd = torch.from_numpy(np.ascontiguousarray(p.b)).cuda()
    v = torch.zeros_like(bd)
    h.vcycle(bd, v)
    got = v.cpu().numpy()[idx]
    assert np.abs(got - np.array(ref["vcycle"])).max() <= 1e-12 * ref["vcycle_maxabs"]
    _log(name, "solve")
    xs = torch.zeros_like(bd)
    st = h.solve(bd, xs)
    _log(name, st, "oracle iters", ref["iters"])
    assert st["converged"] == 1 and st["iters"] == ref["iters"]
    got = xs.cpu().numpy()
    assert np.abs(got[idx] - np.array(ref["solution"])).max() <= 1e-10 * ref["solution_norm"]
    assert abs(np.linalg.norm(got) - ref["solution_norm"]) <= 1e-10 * ref["solution_norm"]
    if name in ("c2", "c3"):
        # the block-dictionary form at full size: bitwise the plain FP64 solve
        del h
        hd = mg.Hierarchy(p.levels, mg.config_from(wl, precision="fp64dict"))
        xd = torch.zeros_like(bd)
        std = hd.solve(bd, xd)
        _log(name, "dictionary form", [hd.dictionary_blocks(l) for l in range(hd.n_levels)], std["iters"])
        assert std["iters"] == st["iters"] and np.array_equal(xd.cpu().numpy(), got)


def test_fullsize_batch_converges_and_matches_oracle_members():
    """The 64-problem x 8-rhs batch in FP32-cycle mode: every instance reaches the FP64
    residual tolerance; the three smallest problems match the oracle's single solves."""
    import scipy.sparse as sp
    from oracle import hierarchy as Hh, multigrid as MG
    from paper_2405_05047_amd import gen, mg
    wls = W.batch_problems()
    nrhs = 8
    _log("batch: generating", len(wls), "problems")
    probs = [gen.build(wl, nrhs) for wl in wls]
    b = np.concatenate([np.asarray(q.b, np.float64).reshape(-1) for q in probs])
    bt = mg.Batch([q.levels for q in probs], mg.config_from(wls[0], precision="fp32"), nrhs=nrhs)
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    _log("batch: solving", bt.size, "unknowns")
    rc, st = bt.solve(bd, x)
    assert rc == 0 and all(s["converged"] == 1 for s in st)
    xs = x.cpu().numpy()
    for k, q in enumerate(probs):
        top = q.finest
        A = sp.bsr_matrix((top.val, top.col, top.rowptr), shape=(top.n, top.n)).tocsr()
        seg = slice(int(bt.offsets[k]), int(bt.offsets[k + 1]))
        X, B = xs[seg].reshape(top.n, nrhs), b[seg].reshape(top.n, nrhs)
        res = np.linalg.norm(B - A @ X, axis=0)
        assert np.all(res <= wls[k].rtol * np.linalg.norm(B, axis=0) * (1 + 1e-9)), k
    small = sorted(range(len(probs)), key=lambda k: probs[k].finest.n)[:3]
    for k in small:
        o = Hh.build(wls[k], nrhs)
        mgo = MG.Multigrid(o)
        seg = slice(int(bt.offsets[k]), int(bt.offsets[k + 1]))
        X = xs[seg].reshape(o.finest.ndof, nrhs)
        Bo = np.asarray(o.b).reshape(o.finest.ndof, nrhs)
        for q in range(nrhs):
            ref, sr = mgo.solve(np.ascontiguousarray(Bo[:, q]))
            err = np.linalg.norm(X[:, q] - ref) / np.linalg.norm(ref)
            _log("batch member", k, "rhs", q, "fp32-cycle rel err vs fp64 oracle", err)
            assert err <= 1e-6


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("name", GOLDEN)
def test_fullsize_mixed_precision_error(name, prec):
    """Mixed-precision solves at the benchmark sizes: the FP64 residual reaches the
    tolerance (library statistic, FP64 over all rows) and the solution agrees with the
    FP64 oracle's at the sampled DoFs to 1e-6 of the largest sampled entry (the error is
    logged)."""
    from paper_2405_05047_amd import gen, mg
    ref = json.load(open(os.path.join(HERE, "golden", f"fullsize_{name}.json")))
    wl = FULL[name]()
    p = gen.build(wl)
    h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=prec))
    idx = np.array(ref["idx"], dtype=np.int64)
    bd = torch.from_numpy(np.ascontiguousarray(p.b)).cuda()
    xs = torch.zeros_like(bd)
    st = h.solve(bd, xs)
    got = xs.cpu().numpy()
    sol = np.array(ref["solution"])
    err = np.abs(got[idx] - sol).max() / np.abs(sol).max()
    _log(name, prec, st, "sampled max error / max sampled |x_oracle|", err)
    assert st["converged"] == 1 and st["res_final"] <= wl.rtol * np.linalg.norm(p.b)
    assert err <= 1e-6
