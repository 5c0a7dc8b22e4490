"""Writes the full-size sampled references `fullsize_<name>.json` from the oracle alone.

For each benchmark workload at its full size this runs the oracle (FP64, test-only) and
stores, at a seeded sample of DoF indices: one finest-level smoothing sweep of seeded
vectors, one V-cycle of the workload's right-hand side from zero, and the converged
FGMRES solution, plus the norms the tolerances are scaled by and the iteration count.
Also `timestep_td10.json`: the first steps of the Sec. 5.1 time loop at 1,050,625 DoFs.
Run from the repository root:  python tests/golden/make_fullsize.py c2 c4 c3 c3f td10
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import hierarchy as Hh, multigrid as MG  # noqa: E402

FULL = {
    "c2": lambda: W.c2_td().with_(coarse_level=3),
    "c3": lambda: W.c3_elasticity().with_(coarse_level=2),
    "c4": lambda: W.c4_oseen().with_(coarse_level=2),
    "c3f": lambda: W.c3_adaptive("face", 6),
}
N_SAMPLES = 400


def make(name):
    wl = FULL[name]()
    t = time.time()
    o = Hh.build(wl)
    print(name, "oracle hierarchy", o.finest.ndof, "DoFs, %.0f s" % (time.time() - t), flush=True)
    mgo = MG.Multigrid(o)
    N = o.finest.ndof
    rng = np.random.default_rng(np.random.SeedSequence([4242, N]))
    idx = np.unique(np.concatenate([[0, N - 1], rng.choice(N, N_SAMPLES, replace=False)])).astype(np.int64)
    L = o.L
    x = W.rand_vec(11, N)
    b = W.rand_vec(12, N)
    sw = mgo.smooth(L, x, b)
    absAx = abs(o.finest.A) @ np.abs(x)
    t = time.time()
    v = mgo.vcycle(o.b)
    print(name, "V-cycle %.1f s" % (time.time() - t), flush=True)
    t = time.time()
    sol, st = mgo.solve(o.b)
    print(name, "solve %.1f s, %d cycles" % (time.time() - t, st.iters), flush=True)
    out = {"workload": wl.name, "coarse_level": wl.coarse_level, "ndof": int(N), "levels": len(o.levels),
           "idx": idx.tolist(),
           "sweep_x_seed": 11, "sweep_b_seed": 12,
           "sweep": sw[idx].tolist(), "sweep_scale": float(np.abs(sw).max() + absAx.max()),
           "vcycle": v[idx].tolist(), "vcycle_maxabs": float(np.abs(v).max()),
           "solution": sol[idx].tolist(), "solution_norm": float(np.linalg.norm(sol)),
           "iters": int(st.iters), "converged": bool(st.converged)}
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path, flush=True)


TIME_STEPS = 3


def make_time():
    """The Sec. 5.1 time loop at the paper's finest level (1,050,625 DoFs): the first
    TIME_STEPS backward-Euler steps, theta sampled after each, and the cycle counts."""
    from oracle import timestep as TS
    wl = W.td_time(10, coarse_level=4)       # the benchmark's configuration: exact solve on 33^2
    t = time.time()
    o = Hh.build(wl)
    print("td_time10 oracle hierarchy", o.finest.ndof, "DoFs, %.0f s" % (time.time() - t), flush=True)
    mgo = MG.Multigrid(o)
    ops = TS.operators(o)
    X = ops.coords
    N = o.finest.ndof
    theta0 = W.td_exact(0.0, X[:, 0], X[:, 1])
    F = [W.td_source(k * wl.dt, X[:, 0], X[:, 1]) for k in range(1, TIME_STEPS + 1)]
    G = [W.td_exact(k * wl.dt, X[:, 0], X[:, 1])[ops.g_idx] for k in range(1, TIME_STEPS + 1)]
    t = time.time()
    res = TS.run(o, mgo, ops, theta0, F, G, wl.dt)
    print("td_time10 %d steps %.1f s, cycles %s" % (TIME_STEPS, time.time() - t, [r.iters for r in res]), flush=True)
    rng = np.random.default_rng(np.random.SeedSequence([4243, N]))
    idx = np.unique(np.concatenate([[0, N - 1], rng.choice(N, N_SAMPLES, replace=False)])).astype(np.int64)
    out = {"workload": wl.name, "ndof": int(N), "dt": wl.dt, "coarse_level": wl.coarse_level, "idx": idx.tolist(),
           "theta": [r.theta[idx].tolist() for r in res], "theta_maxabs": [float(np.abs(r.theta).max()) for r in res],
           "iters": [int(r.iters) for r in res]}
    path = os.path.join(ROOT, "tests", "golden", "timestep_td10.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", path, flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c2", "c4"]:
        if n == "td10":
            make_time()
        else:
            make(n)
