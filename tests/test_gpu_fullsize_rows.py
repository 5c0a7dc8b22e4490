"""GPU parity at the benchmark sizes for the time-stepping driver, the pressure-correction
step and the GPU assembly, in the configuration the benchmark times.

  * time stepping, Sec. 5.1 at 1,050,625 DoFs: the first steps against the oracle's time
    loop sampled in `tests/golden/timestep_td10.json` (written by make_fullsize.py from the
    oracle alone; 1e-10 of max |theta|, equal cycle counts), then all 100 steps by
    property: every solve converges and the nodal error at T = 2 against the exact
    solution stays below 2e-3 (the paper's scheme is first order in dt = 0.02);
  * pressure correction on the graded 32x32x64 mesh: the oracle runs at this size in
    seconds, so the momentum step and D u from a seeded state are compared element by
    element (1e-12 of their scales); the first whole step from rest is checked exactly
    where no solve enters (u^1), by the residual in the oracle's matrix and the cycle
    count for the pressure increment (whose system has condition number ~1e9 here), and
    p^1 against the update formula; 20 further steps by property (every solve
    converges);
  * GPU assembly of every level of the 129^3 elasticity problem: a hierarchy built from
    the GPU-assembled values reproduces the oracle's sampled sweep and V-cycle of
    `fullsize_c3.json` (1e-12), and the values equal the generator's host assembly to 1e-13.
"""
import dataclasses
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


def _log(*a):
    print("[gpu-full2]", *a, flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_time_stepping_fullsize():
    from paper_2405_05047_amd import gen, mg
    ref = json.load(open(os.path.join(HERE, "golden", "timestep_td10.json")))
    wl = W.td_time(10, coarse_level=4)       # the benchmark's configuration
    assert wl.name == ref["workload"] and wl.dt == ref["dt"] and wl.coarse_level == ref["coarse_level"]
    p = gen.build(wl, time_ops=True)
    h = mg.Hierarchy(p.levels, mg.config_from(wl))
    ts = mg.TimeStepper(h, p.time, wl.dt)
    X = p.time.coords
    gi = p.time.g_idx
    assert p.time.n_dofs == ref["ndof"]
    steps = 100
    F = torch.from_numpy(np.stack([W.td_source(k * wl.dt, X[:, 0], X[:, 1]) for k in range(1, steps + 1)])).cuda()
    G = torch.from_numpy(np.stack([W.td_exact(k * wl.dt, X[:, 0], X[:, 1])[gi] for k in range(1, steps + 1)])).cuda()
    th0 = W.td_exact(0.0, X[:, 0], X[:, 1])
    th = torch.from_numpy(th0.copy()).cuda()
    x = torch.from_numpy(np.where(p.finest.mask.ravel() != 0, 0.0, th0)).cuda()
    idx = np.array(ref["idx"], np.int64)
    ns = len(ref["iters"])
    hist = torch.empty((ns, len(th0)), dtype=torch.float64, device="cuda")
    st = ts.run(th, F[:ns], G[:ns], x, history=hist)
    hh = host(hist)
    for k in range(ns):
        assert st[k]["iters"] == ref["iters"][k], (k, st[k]["iters"], ref["iters"][k])
        err = np.abs(hh[k][idx] - np.array(ref["theta"][k])).max() / ref["theta_maxabs"][k]
        assert err <= 1e-10, (k, err)
    st2 = ts.run(th, F[ns:], G[ns:], x)
    assert all(s["converged"] for s in st + st2)
    err = np.abs(host(th) - W.td_exact(steps * wl.dt, X[:, 0], X[:, 1])).max()
    _log("time stepping: 100 steps, nodal error at T=2", f"{err:.3e}")
    assert err < 2e-3


def test_pressure_correction_fullsize():
    from oracle import multigrid as MG, ns
    from paper_2405_05047_amd import gen, mg
    cells, levels, nu, dt = (32, 32, 64), 3, 1e-3, 1e-4      # the benchmark's configuration
    pw = ns.pressure_workload().with_(smoother=W.SMOOTH_CHEBYSHEV)     # FGMRES(10), as benchmarked
    ops = ns.build_operators(cells)
    H = ns.pressure_hierarchy(ops.xp, levels, pw)
    mgo = MG.Multigrid(H)
    prob = gen.build_ns(cells, n_levels=levels)
    hp = mg.Hierarchy(prob.levels, mg.config_from(pw))
    pc = mg.PressureCorrection(prob, hp, nu, dt)
    # kernels from a seeded state
    u = W.rand_vec(21, ops.n_v * 3).reshape(-1, 3)
    pp, q = W.rand_vec(22, ops.n_p), W.rand_vec(23, ops.n_p)
    ud = torch.from_numpy(u.copy()).cuda()
    out = torch.empty_like(ud.reshape(-1))
    pc.momentum(ud, torch.from_numpy(pp).cuda(), torch.from_numpy(q).cuda(), out)
    ref = ns.momentum(ops, u, pp + q, np.zeros_like(u), nu, dt)
    conv = sum(abs(ops.C[a]) @ np.abs(u[:, a:a + 1] * u) for a in range(3))
    scale = (np.abs(u) + dt / ops.m_v[:, None] * (nu * (abs(ops.K_v) @ np.abs(u)) + conv
                                                  + np.stack([abs(ops.G[c]) @ np.abs(pp + q) for c in range(3)], 1)))
    assert np.abs(host(out).reshape(-1, 3) - ref).max() <= 1e-12 * scale.max()
    du = torch.empty(ops.n_p, dtype=torch.float64, device="cuda")
    rhs = torch.empty_like(du)
    pc.divergence(ud, du, rhs)
    dref = ns.divergence(ops, u)
    dscale = sum(abs(ops.G[a]).T @ np.abs(u[:, a]) for a in range(3)).max()
    assert np.abs(host(du) - dref).max() <= 1e-12 * dscale
    # the first whole step from rest: u^1 involves no solve and is compared element by
    # element; q^1 solves the pinned pressure Poisson problem (condition number ~1e9 on
    # this mesh, so it is checked by its residual in the oracle's matrix and the cycle
    # count); p^1 = p^0 + q^1 - nu D u^1 / m_p from the library's own q^1 and D u^1
    r1 = ns.run(ops, mgo, 1, nu, dt)[0]
    ud = torch.from_numpy(np.where(ops.dir_mask, ops.dir_val, 0.0)).cuda()
    pd = torch.zeros(ops.n_p, dtype=torch.float64, device="cuda")
    qd = torch.zeros_like(pd)
    st = pc.run(1, ud, pd, qd)[0]
    assert st["converged"] == 1 and st["iters"] == r1.iters, (st["iters"], r1.iters)
    u1 = host(ud).reshape(-1, 3)
    assert np.abs(u1 - r1.u).max() <= 1e-12 * np.abs(r1.u).max()
    du1 = ns.divergence(ops, u1)
    rhs1 = ns.pressure_rhs(du1, dt, H.finest.mask[:, 0])
    q1 = host(qd)
    assert np.linalg.norm(rhs1 - H.finest.A @ q1) <= 1.01 * pw.rtol * np.linalg.norm(rhs1)
    p1 = ns.pressure_update(ops, np.zeros(ops.n_p), q1, du1, nu)
    assert np.abs(host(pd) - p1).max() <= 1e-12 * (np.abs(q1) + nu * np.abs(du1) / ops.m_p).max()
    # 20 more steps: every pressure solve converges
    st = pc.run(20, ud, pd, qd)
    assert all(s["converged"] for s in st) and np.isfinite(host(ud)).all()
    _log("pressure correction: cycles", r1.iters, [s["iters"] for s in st])


def test_gpu_assembled_elasticity_fullsize():
    from paper_2405_05047_amd import gen, mg
    ref = json.load(open(os.path.join(HERE, "golden", "fullsize_c3.json")))
    wl = W.c3_elasticity().with_(coarse_level=2)
    assert wl.name == ref["workload"]
    p = gen.build(wl)
    levels = []
    worst = 0.0
    for lv in p.levels:
        a = mg.Assembly(lv, wl.dim)
        val = torch.empty(lv.nnzb * 9, dtype=torch.float64, device="cuda")
        a.values(mg.asm_coef(wl), val)
        got = host(val).reshape(lv.val.shape)
        worst = max(worst, float(np.abs(got - lv.val).max() / np.abs(lv.val).max()))
        levels.append(dataclasses.replace(lv, val=got))
        del a, val
    assert worst <= 1e-13, worst
    h = mg.Hierarchy(levels, mg.config_from(wl))
    N = h.ndof()
    L = h.n_levels - 1
    idx = np.array(ref["idx"], np.int64)
    x = torch.from_numpy(W.rand_vec(ref["sweep_x_seed"], N)).cuda()
    b = torch.from_numpy(W.rand_vec(ref["sweep_b_seed"], N)).cuda()
    xo = torch.zeros_like(x)
    h.sweep(L, b, x, xo)
    assert np.abs(host(xo)[idx] - np.array(ref["sweep"])).max() <= 1e-12 * ref["sweep_scale"]
    bb = torch.from_numpy(np.ascontiguousarray(p.b)).cuda()
    v = torch.zeros_like(bb)
    h.vcycle(bb, v)
    assert np.abs(host(v)[idx] - np.array(ref["vcycle"])).max() <= 1e-12 * ref["vcycle_maxabs"]
    _log("gpu assembly c3: worst vs host generator", f"{worst:.2e}")
