"""Benchmark: V-cycle DoF/s to a fixed relative residual on one MI355X.

One step = one complete solve of the workload from x = 0 to ||b - A x|| <= rtol ||b||
(outer FP64 defect, FGMRES(10) preconditioned by one V(2,2)-cycle with damped Jacobi,
hanging-node-aware transfers, dense coarse solve), all in the library's HIP kernels;
inputs are resident in HBM before the timed region.  The default workload is the
adaptive 2D transport-diffusion problem (~1.0e6 DoFs, 9 levels).

Printed: one JSON line with the FP64 solve throughput as `value`, the mixed-precision
variants, the roofline of the dominant kernel (finest-level smoothing sweep) and the
oracle timed on the host.
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
           "nodes), 1,010,113 DoFs, 9-level hierarchy with the exact coarse solve on level 3 (1,749 DoFs), "
           "FGMRES(10) + V(2,2) damped Jacobi w=0.8, rtol 1e-8"),
    "c1": (lambda: W.c1_poisson(), "2D Poisson Q1 33x33 nodes, 5 levels, MG iteration V(2,2) w=0.8, rtol 1e-10"),
    "c3": (lambda: W.c3_elasticity().with_(coarse_level=2),
           "3D elasticity Q1 129^3 nodes, 3x3 blocks, 7-level hierarchy with the exact coarse solve on level 2 "
           "(2,187 DoFs), FGMRES(10) + V(2,2) nodal block-Jacobi w=0.6, rtol 1e-8"),
    "c4": (lambda: W.c4_oseen().with_(coarse_level=2),
           "3D Oseen step Q1/Q1 65^3 nodes, 4x4 blocks, 6-level hierarchy with the exact coarse solve on level 2 "
           "(2,916 DoFs), FGMRES(10) + V(2,2) point-Vanka w=0.6, rtol 1e-8"),
    "c4b": (lambda: W.c4_oseen(rounds=6, tall=True).with_(coarse_level=2),
            "3D Oseen step Q1/Q1 129x129x65 nodes, 4x4 blocks, 7-level hierarchy with the exact coarse solve "
            "on level 2 (1,620 DoFs), FGMRES(10) + V(2,2) point-Vanka, rtol 1e-8"),
}


def sweep_bytes(n, b, nnzb):
    """Algorithmic bytes of one FP64 smoothing sweep: A values + int32 column indices +
    int32 row pointers, x and b read, x_out written, nodal b x b inverse blocks read."""
    return nnzb * (b * b * 8 + 4) + 4 * (n + 1) + 3 * n * b * 8 + n * b * b * 8


def time_solves(torch, h, b, x, steps, warmup):
    for _ in range(warmup):
        x.zero_()
        h.solve(b, x)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        stats.append(h.solve(b, x))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, stats


def kernel_time(torch, h, level, n_dof, launches=50):
    """Average duration of the finest-level smoothing sweep with HIP events on the
    stream the library launches on (torch's current stream)."""
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
    e0.record()
    for i in range(launches):
        if i % 2 == 0:
            h.sweep(level, bb, xa, xb)
        else:
            h.sweep(level, bb, xb, xa)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / launches * 1e-3


def cpu_baseline(wl, budget_s=30.0):
    """The oracle (NumPy/SciPy, FP64) timed on the host on the same workload."""
    from threadpoolctl import threadpool_limits
    from oracle import hierarchy as Hh, multigrid as MG
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        o = Hh.build(wl)
        t_build = time.perf_counter() - t
        mgo = MG.Multigrid(o)
        times = []
        while True:
            t = time.perf_counter()
            x, st = mgo.solve(o.b)
            times.append(time.perf_counter() - t)
            if sum(times) > budget_s / 3 or len(times) >= 3:
                break
    ts = float(np.median(times))
    return {"value": o.finest.ndof / ts, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": f"full workload, {len(times)} oracle solve(s) from x=0 to rtol "
                      f"({st.iters} V-cycles, {ts:.2f} s median; setup {t_build:.1f} s excluded), "
                      f"single thread (SciPy sparse + NumPy, BLAS pinned to 1 thread)",
            "iters": st.iters}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precisions", default="fp64,fp32,fp16,bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    for prec in args.precisions.split(","):
        t = time.perf_counter()
        h = mg.Hierarchy(prob.levels, mg.config_from(wl, precision=prec))
        t_setup = time.perf_counter() - t
        sec, stats = time_solves(torch, h, b, x, args.steps, args.warmup)
        xs = x.cpu().numpy()
        # FP64 residual of the last solution, recomputed on the host from the generator's operator
        import scipy.sparse as sp
        A = sp.bsr_matrix((top.val, top.col, top.rowptr), shape=(N, N)).tocsr()
        rel = float(np.linalg.norm(prob.b - A @ xs) / np.linalg.norm(prob.b))
        results[prec] = {"dof_per_s": N / sec, "ms_per_solve": sec * 1e3, "cycles": stats[-1]["iters"],
                         "converged": all(s["converged"] for s in stats), "rel_residual": rel,
                         "setup_s": round(t_setup, 3)}
        handles[prec] = h
    base = results["fp64"]
    for prec, r in results.items():
        r["speedup_vs_fp64"] = r["dof_per_s"] / base["dof_per_s"]

    # a plain 256 MiB device copy: reference kernel for scaling the HBM byte counters
    src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst

    # roofline of the dominant kernel: finest-level FP64 smoothing sweep
    h64 = handles["fp64"]
    L = h64.n_levels - 1
    n, bs, nnzb = h64.sizes[L]
    ksec = kernel_time(torch, h64, L, n * bs)
    kbytes = sweep_bytes(n, bs, nnzb)
    achieved = kbytes / ksec / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_sweep<B=%d,FP64> finest level" % bs, "bytes_per_launch": kbytes,
            "us_per_launch": round(ksec * 1e6, 2)}

    out = {"metric": METRIC, "value": base["dof_per_s"], "unit": "DoF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": base["ms_per_solve"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": desc, "name": wl.name, "dofs": N, "levels": h64.n_levels,
                      "nnzb_finest": nnzb, "generator_s": round(t_gen, 2)},
           "roofline": roof,
           "variants": {k: {kk: (float(f"{vv:.6g}") if isinstance(vv, float) else vv) for kk, vv in v.items()}
                        for k, v in results.items()}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
