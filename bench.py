"""Benchmark: V-cycle DoF/s to a fixed relative residual on one MI355X.

One step = one complete solve of the workload from x = 0 to ||b - A x|| <= rtol ||b||
(outer FP64 defect, FGMRES(10) preconditioned by one V(2,2)-cycle with damped Jacobi,
hanging-node-aware transfers, dense coarse solve), all in the library's HIP kernels;
inputs are resident in HBM before the timed region.  The default workload is the
largest configuration: 3D linear elasticity on 129^3 nodes (6,440,067 DoFs, 3x3 nodal
blocks, 7-level hierarchy), whose GB-sized operators stream from HBM.

Printed: one JSON line with the FP64 solve throughput as `value`, the mixed-precision
variants, the lossless block-dictionary form of the FP64 operators (bitwise the FP64
results), the roofline of the dominant kernel (finest-level smoothing sweep) against the
8 TB/s HBM peak, a measured device-copy rate, the same sweep on the 1M-unknown 2D
transport-diffusion problem (its 91 MB operator is served from the 256 MB memory-side
cache, reported separately), the oracle timed on the host and the batched form (64
uneven transport-diffusion problems x 8 right-hand sides solved together, against the
same 512 solves done one at a time).  Further sections: the same solve with the
Chebyshev smoother, the GPU assembly of every level's operator, 100 backward-Euler steps
of the Sec. 5.1 problem on 1,050,625 DoFs, and the Sec. 5.3 pressure-correction step on
the graded 32x32x64 mesh.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "V-cycle DoF/s to 1e-8 rel. residual (FP64 vs mixed/batched); SpMV HBM GB/s"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c2": (lambda: W.c2_td().with_(coarse_level=3),
           "2D transport-diffusion eps=1e-3 b=(1,0.5) SUPG Q1, annulus-refined adaptive mesh (hanging "
           "nodes), 1,010,113 DoFs, levels 3-8 of the 9-level hierarchy (6 in the cycle) with the exact "
           "coarse solve on level 3 (1,749 DoFs), "
           "FGMRES(10) + V(2,2) damped Jacobi w=0.8, rtol 1e-8"),
    "c1": (lambda: W.c1_poisson(), "2D Poisson Q1 33x33 nodes, 5 levels, MG iteration V(2,2) w=0.8, rtol 1e-10"),
    "c3": (lambda: W.c3_elasticity().with_(coarse_level=2),
           "3D elasticity Q1 129^3 nodes, 3x3 blocks, levels 2-6 of the 3^3..129^3 hierarchy (5 in the "
           "cycle) with the exact coarse solve on level 2 (9^3 nodes, 2,187 DoFs), FGMRES(10) + V(2,2) "
           "nodal block-Jacobi w=0.6, rtol 1e-8"),
    "c4": (lambda: W.c4_oseen().with_(coarse_level=2),
           "3D Oseen step Q1/Q1 65^3 nodes, 4x4 blocks, levels 2-5 of the 3^3..65^3 hierarchy (4 in the "
           "cycle) with the exact coarse solve on level 2 (9^3 nodes, 2,916 DoFs), FGMRES(10) + V(2,2) "
           "point-Vanka w=0.6, rtol 1e-8"),
    "c4b": (lambda: W.c4_oseen(rounds=6, tall=True).with_(coarse_level=2),
            "3D Oseen step Q1/Q1 129x129x65 nodes, 4x4 blocks, levels 2-6 of the 7-level hierarchy (5 in "
            "the cycle) with the exact coarse solve on level 2 (1,620 DoFs), FGMRES(10) + V(2,2) "
            "point-Vanka, rtol 1e-8"),
    "c3f": (lambda: W.c3_adaptive("face", 6),
            "3D elasticity Q1 on the face-refined cube mesh (8^3 coarse cubes, 5 rounds refining the cells "
            "next to the face x = 0), 683,741 nodes x 3 components with edge and face hanging nodes, 6-level "
            "hierarchy with the exact coarse solve on the 9^3-node level, FGMRES(10) + V(2,2) nodal "
            "block-Jacobi w=0.6, rtol 1e-8"),
}


# oracle samples for the CPU baseline of workloads too large to time whole on the host
SAMPLES = {
    "c3": lambda: W.c3_elasticity(5).with_(coarse_level=2),      # 65^3 nodes, 823,875 DoFs
    "c4b": lambda: W.c4_oseen().with_(coarse_level=2),           # 65^3 nodes
}

# operator streams up to this size are read with ordinary loads and stay in the 256 MB
# memory-side cache between kernels (the library's rule)
CACHED_STREAM_BYTES = 128 << 20


def sweep_bytes(n, b, nnzb, col_bytes=4):
    """Algorithmic bytes of one FP64 smoothing sweep: A values + column indices (4 B, or 2 B
    when the operator is stored with 16-bit offsets from a per-slot base) + int32 row pointers, x
    and b read, x_out written, nodal b x b inverse blocks read."""
    return nnzb * (b * b * 8 + col_bytes) + 4 * (n + 1) + 3 * n * b * 8 + n * b * b * 8


def dict_sweep_bytes(n, b, nnzb, col_bytes, ndict):
    """The same sweep with the operator in the dictionary form: a 16-bit block index and
    the column index per stored block, the distinct blocks once, vectors and smoother
    blocks as in sweep_bytes."""
    return nnzb * (2 + col_bytes) + ndict * b * b * 8 + 4 * (n + 1) + 3 * n * b * 8 + n * b * b * 8


def time_solves(torch, h, b, x, steps, warmup):
    for _ in range(warmup):
        x.zero_()
        h.solve(b, x)
    torch.cuda.synchronize()
    stats = []
    per = []
    t0 = time.perf_counter()
    for _ in range(steps):
        t = time.perf_counter()
        x.zero_()
        stats.append(h.solve(b, x))      # returns after the solve's final synchronisation
        per.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, stats, per


def counter_traffic(workload_name):
    """HBM bytes per launch of the finest-level FP64 sweep from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE runs scaled by a plain copy), or None when
    any HIP source of the library (kernels, or the runtime that decides the data layout) has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_sweep_fp64_counters.json")
    h = hashlib.sha256()
    try:
        with open(path) as f:
            table = json.load(f)
        csrc = os.path.join(ROOT, "paper_2405_05047_amd", "csrc")
        for name in sorted(os.listdir(csrc)):
            if name.endswith((".hip", ".h")):
                with open(os.path.join(csrc, name), "rb") as f:
                    h.update(f.read())
    except OSError:
        return None
    digest = h.hexdigest()
    entry = table.get(workload_name)
    if not entry or entry.get("sources_sha256") != digest:
        return None
    return entry["traffic_bytes_per_launch"]


def device_copy_gbs(torch, mib=256, reps=20):
    """Read + write rate of a plain device-to-device copy of `mib` MiB (HIP events)."""
    src = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2.0 * (mib << 20) / sec / 1e9


def sweep_roofline(torch, h, name, bound):
    """Algorithmic bytes of the finest-level FP64 sweep over its measured launch time."""
    L = h.n_levels - 1
    n, bs, nnzb = h.sizes[L]
    ksec = kernel_time(torch, h, L, n * bs)
    kbytes = sweep_bytes(n, bs, nnzb, h.col_bytes(L))
    achieved = kbytes / ksec / 1e9
    return {"bound": bound, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(name),
            "kernel": "k_sweep<B=%d,FP64> finest level" % bs, "bytes_per_launch": kbytes,
            "us_per_launch": round(ksec * 1e6, 2)}


def kernel_time(torch, h, level, n_dof, launches=50):
    """Average duration of the finest-level smoothing sweep with HIP events on the
    stream the library launches on (torch's current stream).  The launches are queued
    behind a bounded spin kernel, so the GPU runs them back to back even when one launch
    is shorter than the host's time to issue it (the 2D sweeps take ~19 us)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    xa = torch.rand(n_dof, dtype=torch.float64, device="cuda", generator=g)
    xb = torch.empty_like(xa)
    bb = torch.rand(n_dof, dtype=torch.float64, device="cuda", generator=g)
    for _ in range(5):
        h.sweep(level, bb, xa, xb)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(20_000_000)
    e0.record()
    for i in range(launches):
        if i % 2 == 0:
            h.sweep(level, bb, xa, xb)
        else:
            h.sweep(level, bb, xb, xa)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / launches * 1e-3


def _progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def batched(torch, gen, mg, n_problems, nrhs, steps, precisions=("fp64", "fp32", "fp16")):
    """The batched form: `n_problems` seeded transport-diffusion problems of uneven size
    (4-9 levels), `nrhs` seeded right-hand sides each, all solved in one lockstep FGMRES
    whose V-cycle steps are single launches over the whole batch; compared with the same
    solves done one problem and one right-hand side at a time (FP64 single-problem path)."""
    import scipy.sparse as sp
    wls = W.batch_problems(n_problems=n_problems)
    t = time.perf_counter()
    probs = []
    for k, wl in enumerate(wls):
        probs.append(gen.build(wl, nrhs))
        if k % 16 == 15:
            _progress(f"batch: generated {k + 1}/{len(wls)} problems")
    t_gen = time.perf_counter() - t
    sizes = [p.finest.n for p in probs]
    n_inst = n_problems * nrhs
    dofs = sum(sizes) * nrhs
    b = np.concatenate([np.asarray(p.b, np.float64).reshape(-1) for p in probs])
    bd = torch.from_numpy(b).cuda()
    x = torch.zeros_like(bd)
    res = {}
    for prec in precisions:
        t = time.perf_counter()
        bt = mg.Batch([p.levels for p in probs], mg.config_from(wls[0], precision=prec), nrhs=nrhs)
        t_setup = time.perf_counter() - t
        x.zero_()
        bt.solve(bd, x)                     # warm-up (captures the step graphs)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            rc, st = bt.solve(bd, x)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / steps
        xs = x.cpu().numpy()
        worst = 0.0
        for p, pr in enumerate(probs):
            top = pr.finest
            A = sp.bsr_matrix((top.val, top.col, top.rowptr), shape=(top.n, top.n)).tocsr()
            seg = slice(int(bt.offsets[p]), int(bt.offsets[p + 1]))
            X, B = xs[seg].reshape(top.n, nrhs), b[seg].reshape(top.n, nrhs)
            r = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
            worst = max(worst, float(r.max()))
        its = [s["iters"] for s in st]
        res[prec + "_batch"] = {"dof_per_s": dofs / sec, "ms_per_solve": sec * 1e3, "status": rc,
                                "converged": int(sum(s["converged"] for s in st)), "instances": n_inst,
                                "cycles_min": min(its), "cycles_max": max(its),
                                "max_rel_residual": worst, "setup_s": round(t_setup, 2)}
        _progress(f"batch {prec}: {sec * 1e3:.1f} ms for {n_inst} solves")
        del bt
    # the same solves one at a time with the single-problem FP64 path
    hs = [mg.Hierarchy(p.levels, mg.config_from(wl)) for p, wl in zip(probs, wls)]
    cols = []
    for p in probs:
        B = np.asarray(p.b, np.float64).reshape(p.finest.n, nrhs)
        cols.append([torch.from_numpy(np.ascontiguousarray(B[:, q])).cuda() for q in range(nrhs)])
    xq = torch.zeros(max(sizes), dtype=torch.float64, device="cuda")
    for h, c, n in zip(hs, cols, sizes):     # warm-up (graphs)
        xv = xq[:n]
        xv.zero_()
        h.solve(c[0], xv)
    torch.cuda.synchronize()
    t = time.perf_counter()
    iters = []
    for h, c, n in zip(hs, cols, sizes):
        xv = xq[:n]
        for q in range(nrhs):
            xv.zero_()
            iters.append(h.solve(c[q], xv)["iters"])
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    res["fp64_sequential"] = {"dof_per_s": dofs / sec, "ms_per_solve": sec * 1e3, "instances": n_inst,
                              "cycles_min": min(iters), "cycles_max": max(iters)}
    _progress(f"sequential fp64: {sec * 1e3:.1f} ms for {n_inst} solves")
    base = res["fp64_sequential"]["dof_per_s"]
    for k, v in res.items():
        v["speedup_vs_fp64_sequential"] = v["dof_per_s"] / base
    return {"workload": f"{n_problems} seeded 2D transport-diffusion problems (eps log-uniform in "
                        f"[1e-4,1e-1], random unit b, 4-9 levels, annulus-refined), {nrhs} seeded "
                        f"right-hand sides each, FGMRES(10) + V(2,2) w=0.6 to rtol 1e-8 per instance",
            "problems": n_problems, "nrhs": nrhs, "nodes_total": int(sum(sizes)), "dofs_total": int(dofs),
            "nodes_min": int(min(sizes)), "nodes_max": int(max(sizes)), "generator_s": round(t_gen, 1),
            "results": {k: {kk: (float(f"{vv:.6g}") if isinstance(vv, float) else vv) for kk, vv in v.items()}
                        for k, v in res.items()}}


def time_stepping(torch, gen, mg, n=10, steps=100):
    """Algorithm "Nonstationary Linear Problem" on the Sec. 5.1 problem at the paper's
    finest level (n = 10: 1,050,625 DoFs), dt = 0.02, 100 backward-Euler steps to T = 2:
    one hierarchy for all steps, each right-hand side formed on the GPU by the lumped mass,
    each solve from the previous solution.  Source and Dirichlet values of every step are
    made on the host and resident in HBM before the timed region."""
    wl = W.td_time(n, coarse_level=4)              # exact coarse solve on the 33^2 level
    p = gen.build(wl, time_ops=True)
    h = mg.Hierarchy(p.levels, mg.config_from(wl))
    ts = mg.TimeStepper(h, p.time, wl.dt)
    X = p.time.coords
    gi = p.time.g_idx
    F = np.stack([W.td_source(k * wl.dt, X[:, 0], X[:, 1]) for k in range(1, steps + 1)])
    G = np.stack([W.td_exact(k * wl.dt, X[:, 0], X[:, 1])[gi] for k in range(1, steps + 1)])
    th0 = W.td_exact(0.0, X[:, 0], X[:, 1])
    Fd, Gd = torch.from_numpy(F).cuda(), torch.from_numpy(G).cuda()
    th = torch.from_numpy(th0).cuda()
    x = torch.from_numpy(np.where(p.finest.mask.ravel() != 0, 0.0, th0)).cuda()
    ts.run(th, Fd[:2], Gd[:2], x)                   # warm-up (graphs)
    th.copy_(torch.from_numpy(th0))
    x.copy_(torch.from_numpy(np.where(p.finest.mask.ravel() != 0, 0.0, th0)))
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = ts.run(th, Fd, Gd, x)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    err = float(np.abs(th.cpu().numpy() - W.td_exact(steps * wl.dt, X[:, 0], X[:, 1])).max())
    its = [s["iters"] for s in st]
    N = p.time.n_dofs
    return {"workload": f"Sec. 5.1 transport-diffusion, uniform (2^{n}+1)^2 mesh, {N:,} DoFs, dt = {wl.dt}, "
                        f"{steps} backward-Euler steps, lumped mass, FGMRES(10) + V(2,2) Jacobi with the exact "
                        f"coarse solve on the 33^2 level (1,089 DoFs), rtol 1e-8",
            "dofs": N, "steps": steps, "total_s": round(sec, 4), "ms_per_step": round(sec / steps * 1e3, 3),
            "dof_per_s": N * steps / sec, "cycles_min": min(its), "cycles_max": max(its),
            "all_converged": all(s["converged"] for s in st), "max_nodal_error_at_T": err,
            "context_paper_h100_solve_s": 9.0}


def pressure_correction(torch, gen, mg, cells=(32, 32, 64), levels=3, steps=20, oracle_step=True):
    """Sec. 5.3 driven cavity: explicit momentum step, pressure Poisson solve (FGMRES(10) +
    V(2,2) with the Chebyshev smoother on the graded mesh) and pressure update per time
    step, from rest with the moving wall; dt = 1e-4, nu = 1e-3."""
    nu, dt = 1e-3, 1e-4
    prob = gen.build_ns(cells, n_levels=levels)
    pw = W.Workload(name="ns_pressure", dim=3, coarse=(1, 1, 1), h0=1.0, rounds=(), pde=W.PDE_POISSON, block=1,
                    omega=0.8, nu1=2, nu2=2, outer=W.OUTER_FGMRES, gmres_m=10, rtol=1e-8, maxit=400,
                    smoother=W.SMOOTH_CHEBYSHEV)
    hp = mg.Hierarchy(prob.levels, mg.config_from(pw))
    pc = mg.PressureCorrection(prob, hp, nu, dt)
    u0 = np.where(prob.dir_mask != 0, prob.dir_val, 0.0)
    u = torch.from_numpy(u0.copy()).cuda()
    pp = torch.zeros(prob.n_p, dtype=torch.float64, device="cuda")
    q = torch.zeros_like(pp)
    pc.run(2, u, pp, q)                             # warm-up (graphs)
    u.copy_(torch.from_numpy(u0))
    pp.zero_()
    q.zero_()
    torch.cuda.synchronize()
    t = time.perf_counter()
    st = pc.run(steps, u, pp, q)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    # the explicit parts alone (momentum + divergence + update) per step
    ub = torch.empty_like(u)
    du = torch.empty_like(pp)
    rhs = torch.empty_like(pp)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        pc.momentum(u, pp, q, ub)
        pc.divergence(ub, du, rhs)
        pc.pressure_update(pp, q, du)
    e1.record()
    torch.cuda.synchronize()
    explicit_ms = e0.elapsed_time(e1) / 20
    its = [s["iters"] for s in st]
    out = {"workload": f"Sec. 5.3 driven cavity, pressure Q1 on the graded {cells[0]}x{cells[1]}x{cells[2]} mesh "
                       f"({prob.n_p:,} nodes), velocity Q1 on its refinement ({prob.n_v:,} nodes x 3), "
                       f"{levels}-level pressure hierarchy (exact coarse solve on its coarsest level, "
                       f"{prob.levels[0].n:,} DoFs), "
                       f"dt = {dt}, nu = {nu}, {steps} steps from rest",
           "velocity_dofs": prob.n_v * 3, "pressure_dofs": prob.n_p, "steps": steps,
           "ms_per_step": round(sec / steps * 1e3, 3), "explicit_ms_per_step": round(explicit_ms, 4),
           "pressure_cycles_min": min(its), "pressure_cycles_max": max(its),
           "all_converged": all(s["converged"] for s in st)}
    if oracle_step:
        from threadpoolctl import threadpool_limits
        from oracle import multigrid as MG, ns
        with threadpool_limits(limits=1):
            ops = ns.build_operators(cells)
            H = ns.pressure_hierarchy(ops.xp, levels, pw)
            mgo = MG.Multigrid(H)
            t = time.perf_counter()
            ns.run(ops, mgo, 1, nu, dt)
            out["oracle_s_first_step"] = round(time.perf_counter() - t, 3)
            out["oracle_cores"] = 1
    return out


def gpu_assembly(torch, gen, mg, prob, wl, reps=5):
    """GPU-side assembly of every level's constrained operator of `prob` (the paper's CPU
    "init"): host symbolic phase once per mesh, then the numeric phase on the GPU (element
    matrices per cell size + one gather per stored block), timed with HIP events; checked
    against the generator's host assembly."""
    out = {"levels": []}
    total_ms = 0.0
    worst = 0.0
    for l, lv in enumerate(prob.levels):
        t = time.perf_counter()
        a = mg.Assembly(lv, wl.dim)
        t_sym = time.perf_counter() - t
        val = torch.empty(lv.nnzb * lv.block * lv.block, dtype=torch.float64, device="cuda")
        coef = mg.asm_coef(wl)
        a.values(coef, val)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            a.values(coef, val)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        total_ms += ms
        ref = np.asarray(lv.val).reshape(-1)
        worst = max(worst, float(np.abs(val.cpu().numpy() - ref).max() / np.abs(ref).max()))
        out["levels"].append({"level": l, "blocks": int(lv.nnzb), "numeric_ms": round(ms, 4),
                              "write_gbs": round(lv.nnzb * lv.block * lv.block * 8 / (ms * 1e-3) / 1e9, 1),
                              "host_symbolic_s": round(t_sym, 3)})
        del a, val
    out["numeric_ms_all_levels"] = round(total_ms, 4)
    out["max_rel_diff_vs_host_generator"] = worst
    return out


def cpu_baseline(wl, n_full, sample_wl=None, budget_s=30.0):
    """The oracle (NumPy/SciPy, FP64) timed on the host, single-threaded, on a bounded
    sample: the same workload, or (sample_wl) the same PDE, configuration and solver on a
    smaller mesh of the same family, whose per-DoF rate stands for the full size."""
    from threadpoolctl import threadpool_limits
    from oracle import hierarchy as Hh, multigrid as MG
    swl = sample_wl or wl
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        o = Hh.build(swl)
        t_build = time.perf_counter() - t
        mgo = MG.Multigrid(o)
        times = []
        while True:
            t = time.perf_counter()
            x, st = mgo.solve(o.b)
            times.append(time.perf_counter() - t)
            if sum(times) > budget_s / 2 or len(times) >= 3:
                break
    ts = float(np.median(times))
    rate = o.finest.ndof / ts
    if sample_wl is None:
        what = "full workload"
    else:
        what = (f"{swl.name}: the same PDE, solver and coarse level on {o.finest.ndof:,} DoFs; the oracle's "
                f"cost per cycle is linear in the DoFs and its cycle count mesh-independent, so this "
                f"per-DoF rate stands for the full {n_full:,} DoFs (extrapolated full solve "
                f"{n_full / rate:.1f} s)")
    return {"value": rate, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}; {len(times)} oracle solve(s) from x=0 to rtol ({st.iters} V-cycles, "
                      f"{ts:.2f} s median; setup {t_build:.1f} s excluded), single thread (SciPy sparse + "
                      f"NumPy, BLAS pinned to 1 thread)",
            "iters": st.iters, "host_nproc": os.cpu_count(),
            "host_cpus_usable": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--precisions", default="fp64,fp32,fp16,bf16,fp64dict",
                    help="variants; a '+cheb' suffix runs the variant with the Chebyshev smoother")
    ap.add_argument("--cheb-variants", default="fp64+cheb,fp16+cheb,fp64dict+cheb",
                    help="Chebyshev-smoothed variants added for the elasticity workloads ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cache-served", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the time-stepping and pressure-correction sections")
    ap.add_argument("--batch-problems", type=int, default=64,
                    help="problems of the batched section (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_2405_05047_amd import gen, mg

    torch.cuda.set_device(0)
    make, desc = WORKLOADS[args.workload]
    wl = make()
    t = time.perf_counter()
    prob = gen.build(wl)
    t_gen = time.perf_counter() - t
    top = prob.finest
    N = top.n * top.block
    b = torch.from_numpy(np.ascontiguousarray(prob.b)).cuda()
    x = torch.zeros_like(b)
    results = {}
    handles = {}
    variants = args.precisions.split(",")
    if wl.pde == W.PDE_ELASTICITY and args.cheb_variants:
        variants += [v for v in args.cheb_variants.split(",") if v not in variants]
    for prec in variants:
        t = time.perf_counter()
        base_prec, _, sm = prec.partition("+")
        over = {"smoother": W.SMOOTH_CHEBYSHEV} if sm == "cheb" else {}
        h = mg.Hierarchy(prob.levels, mg.config_from(wl, precision=base_prec, **over))
        t_setup = time.perf_counter() - t
        sec, stats, per = time_solves(torch, h, b, x, args.steps, args.warmup)
        xs = x.cpu().numpy()
        # FP64 residual of the last solution, recomputed on the host from the generator's operator
        import scipy.sparse as sp
        A = sp.bsr_matrix((top.val, top.col, top.rowptr), shape=(N, N)).tocsr()
        rel = float(np.linalg.norm(prob.b - A @ xs) / np.linalg.norm(prob.b))
        results[prec] = {"dof_per_s": N / sec, "ms_per_solve": sec * 1e3, "ms_min": min(per) * 1e3,
                         "ms_median": float(np.median(per)) * 1e3, "ms_max": max(per) * 1e3,
                         "cycles": stats[-1]["iters"],
                         "converged": all(s["converged"] for s in stats), "rel_residual": rel,
                         "setup_s": round(t_setup, 3),
                         "slot_batch_per_level": [h.tuning(l)[0] for l in range(h.n_levels)]}
        if base_prec == "fp64dict":
            # lossless: the distinct FP64 blocks once per level, a 16-bit index per stored block
            Ld = h.n_levels - 1
            nd, bsd, nnzbd = h.sizes[Ld]
            ndict = h.dictionary_blocks(Ld)
            results[prec]["dictionary_blocks_per_level"] = [h.dictionary_blocks(l) for l in range(h.n_levels)]
            if ndict:
                ksec = kernel_time(torch, h, Ld, nd * bsd)
                kbytes = dict_sweep_bytes(nd, bsd, nnzbd, h.col_bytes(Ld), ndict)
                results[prec]["finest_sweep"] = {"us_per_launch": round(ksec * 1e6, 2), "bytes_per_launch": kbytes,
                                                 "achieved_gbs": round(kbytes / ksec / 1e9, 1)}
        if sm == "cheb":
            results[prec]["smoother"] = (f"Chebyshev on [{wl.cheb_lo}, {wl.cheb_hi}] x lambda(S A), lambda by "
                                         f"{wl.power_its} power-iteration steps")
            h.close()
        else:
            handles[prec] = h
        _progress(f"{wl.name} {prec}: {sec * 1e3:.2f} ms per solve, {stats[-1]['iters']} cycles")
    base = results["fp64"]
    for prec, r in results.items():
        r["speedup_vs_fp64"] = r["dof_per_s"] / base["dof_per_s"]

    # a plain 256 MiB device copy: the measured copy peak (and the reference kernel for
    # scaling the HBM byte counters in the profiles)
    copy_gbs = device_copy_gbs(torch)

    # roofline of the dominant kernel: finest-level FP64 smoothing sweep.  Operator
    # streams above 128 MB bypass the memory-side cache (non-temporal loads) and come
    # from HBM; smaller ones are served from that cache and are labelled so.
    h64 = handles["fp64"]
    L = h64.n_levels - 1
    n, bs, nnzb = h64.sizes[L]
    op_bytes = nnzb * (bs * bs * 8 + h64.col_bytes(L))
    roof = sweep_roofline(torch, h64, wl.name, "hbm" if op_bytes > CACHED_STREAM_BYTES else "mall")
    roof["copy_gbs_measured"] = round(copy_gbs, 1)
    roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)

    out = {"metric": METRIC, "value": base["dof_per_s"], "unit": "DoF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": base["ms_per_solve"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": desc, "name": wl.name, "dofs": N, "levels": h64.n_levels,
                      "nnzb_finest": nnzb, "generator_s": round(t_gen, 2)},
           "roofline": roof,
           "host_nproc": os.cpu_count(),
           "variants": {k: {kk: (float(f"{vv:.6g}") if isinstance(vv, float) else vv) for kk, vv in v.items()}
                        for k, v in results.items()}}
    del handles, h64, h
    if args.workload != "c2" and not args.no_cache_served:
        # the same kernel on the 1M-unknown 2D problem, whose operator stays in the cache
        _progress("cache-served sweep (2D transport-diffusion)")
        mk2, _ = WORKLOADS["c2"]
        wl2 = mk2()
        p2 = gen.build(wl2)
        h2 = mg.Hierarchy(p2.levels, mg.config_from(wl2))
        r2 = sweep_roofline(torch, h2, wl2.name, "mall")
        r2["workload"] = f"{wl2.name}: {p2.finest.n:,} DoFs; its operator stream fits the 256 MB memory-side cache"
        out["roofline_cache_served"] = r2
        del h2, p2
    if not args.no_extra and wl.pde in mg.ASM_PDE:
        _progress("GPU assembly of every level")
        ga = gpu_assembly(torch, gen, mg, prob, wl)
        ga["workload"] = wl.name
        ga["host_generator_s"] = round(t_gen, 2)
        out["gpu_assembly"] = ga
    if not args.no_extra:
        _progress("time stepping (Sec. 5.1, 1,050,625 DoFs, 100 steps)")
        out["time_stepping"] = time_stepping(torch, gen, mg)
        _progress("pressure correction (Sec. 5.3)")
        out["pressure_correction"] = pressure_correction(torch, gen, mg, oracle_step=not args.no_cpu_baseline)
    if args.batch_problems > 0:
        _progress("batched section")
        out["batched"] = batched(torch, gen, mg, args.batch_problems, 8, args.batch_steps)
    if not args.no_cpu_baseline:
        _progress("cpu baseline (oracle)")
        sample = SAMPLES.get(args.workload)
        out["cpu_baseline"] = cpu_baseline(wl, N, sample() if sample else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
