"""Benchmark: GIAMG-PCG solves/s on one MI355X, with the HBM roofline of the
dominant kernel and the CPU oracle timed beside it.

Workload (default): Helmholtz lambda = 10 on a 16 x 16 x 16 hexahedral mesh of
the unit cube, order p = 4 (274,625 nodes, 49,455,441 stored nonzeros),
interior vertices perturbed by U(-0.1 h, 0.1 h) (seed 2), right-hand side
i.i.d. N(0, 1) (seed 12), FP64 throughout, hierarchy p4 -> p2 -> p1 then
smoothed aggregation down to <= 2000 rows, Chebyshev degree 2, CG to
||r|| / ||b|| < 1e-10.  A step is one whole solve (the V-cycle-preconditioned
CG from x = 0 to the tolerance); the hierarchy is built once before timing
(its setup time, including the device Galerkin products, is reported apart).

Prints one JSON line.  Options: --gpus (1 only), --steps, --warmup,
--workload {cfg2,cfg3}, --no-cpu-baseline, --no-mixed.
"""
import argparse
import numpy as np
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
WORKLOADS = {
    # name: (n, p, lambda or None for log-uniform draw, mesh seed, rhs seed, lambda seed)
    "cfg2": dict(n=16, p=4, lam=10.0, mesh_seed=2, rhs_seed=12, lam_seed=None),
    "cfg3": dict(n=32, p=4, lam=None, mesh_seed=3, rhs_seed=23, lam_seed=13),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cheb_step.json")
KERNEL_SOURCES = ["paper_2512_15121_amd/csrc/kernels.hip", "paper_2512_15121_amd/csrc/kernels.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def problem(name):
    import synth
    w = WORKLOADS[name]
    lam = w["lam"] if w["lam"] is not None else synth.loguniform_lambda(w["lam_seed"])
    mesh = synth.hex_mesh(w["n"], w["p"], perturb=0.1, seed=w["mesh_seed"])
    b = synth.normal_rhs(mesh.n_nodes, w["rhs_seed"])
    return mesh, b, lam, w


def time_solves(torch, solver, bt, steps, warmup):
    x = torch.zeros_like(bt)
    for _ in range(warmup):
        x.zero_()
        solver.solve(bt, x, tol=1e-10)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        _, info = solver.solve(bt, x, tol=1e-10)
        infos.append(info)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, infos, x


def traffic_entry(workload):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    e = t.get(workload)
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(mesh, b, lam, w, gpu_iters):
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import hierarchy, krylov
    log("cpu baseline: building the oracle hierarchy")
    t0 = time.perf_counter()
    H = hierarchy.build(mesh.coords, mesh.l2g, w["p"], lam, hierarchy.Options())
    setup_s = time.perf_counter() - t0
    reps = 0
    t_total = 0.0
    iters = 0
    with threadpool_limits(1):
        while reps < 3 and t_total < 20.0:
            t0 = time.perf_counter()
            res = krylov.giamg_pcg(H, b, tol=1e-10)
            t_total += time.perf_counter() - t0
            iters = res.iters
            reps += 1
            log(f"cpu baseline: oracle solve {reps}: {iters} iterations")
    return {"value": reps / t_total, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} complete oracle solves (FP64 PCG to 1e-10, {iters} iterations each; "
                      f"GPU took {gpu_iters}) on the same hierarchy and right-hand side, "
                      f"BLAS limited to 1 thread; oracle setup {setup_s:.1f} s not timed"}


def batched_leg(torch, Solver, Options, k=64, reps=3):
    """Pressure-Poisson-like batch: lambda = 0, pure Neumann with node 0
    pinned, 20^3 perturbed mesh (seed 4), p = 3, 64 right-hand sides N(0,1)
    (seed 14) shifted to mean zero; FP32 V-cycle in FP64 flexible CG, block
    products, graph replay.  Compared with 64 single solves."""
    import synth
    mesh = synth.hex_mesh(20, 3, perturb=0.1, seed=4)
    B = synth.pinned_normal_batch(mesh.n_nodes, k, 14)
    s = Solver(mesh.coords, mesh.l2g, 3, 0.0, Options(bc="pin", precision="mixed"))
    Bt = torch.from_numpy(B).to("cuda:0")
    X = torch.zeros_like(Bt)
    s.solve_batch(Bt, X, tol=1e-10)          # tunes tiles, captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        X.zero_()
        _, infos = s.solve_batch(Bt, X, tol=1e-10)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    cols = [torch.from_numpy(np.ascontiguousarray(B[:, j])).to("cuda:0") for j in range(k)]
    x1 = torch.zeros_like(cols[0])
    s.solve(cols[0], x1, tol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters_single = []
    for j in range(k):
        x1.zero_()
        _, inf = s.solve(cols[j], x1, tol=1e-10)
        iters_single.append(inf.iters)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    out = {"workload": "20^3 p=3 pure Neumann + pin, lambda=0, 64 RHS, mixed",
           "nodes": mesh.n_nodes, "rhs": k,
           "rhs_solves_per_s": round(k / t_batch, 2),
           "single_solves_per_s": round(k / t_single, 2),
           "speedup_vs_single": round(t_single / t_batch, 2),
           "iters_max": max(i.iters for i in infos),
           "iters_single_max": max(iters_single),
           "worst_true_relres": max(i.true_relres for i in infos),
           "gbs": round(infos[0].bytes / t_batch / 1e9, 1)}
    s.close()
    log(f"batched: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the solve would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2512_15121_amd import Solver, Options

    dev = torch.device("cuda:0")
    mesh, b, lam, w = problem(args.workload)
    log(f"workload {args.workload}: n={w['n']} p={w['p']} nodes={mesh.n_nodes} lambda={lam:.6g}")
    t0 = time.perf_counter()
    solver = Solver(mesh.coords, mesh.l2g, w["p"], lam, Options())
    setup_s = time.perf_counter() - t0
    levels = [solver.level(l) for l in range(solver.num_levels())]
    log(f"setup {setup_s:.2f} s; levels {[(d['kind'], d['order'], d['rows'], d['nnz_A']) for d in levels]}")
    bt = torch.from_numpy(b).to(dev)
    elapsed, infos, x = time_solves(torch, solver, bt, args.steps, args.warmup)
    iters = infos[-1].iters
    assert all(i.status == 0 and i.iters == iters for i in infos)
    true_rel = infos[-1].true_relres
    bytes_per_solve = infos[-1].bytes
    value = args.steps / elapsed
    ms_per_step = 1000.0 * elapsed / args.steps
    log(f"fp64: {value:.2f} solves/s, {iters} iterations, true relres {true_rel:.2e}")

    # dominant kernel: fused Chebyshev step on the fine operator
    k_ms, k_bytes = solver.time_kernel("cheb_step", level=0, reps=50)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic_entry(args.workload),
                "kernel": "spmv_kernel<double, SPMV_CHEB_STEP> on the fine level",
                "bytes_per_launch": k_bytes, "ms_per_launch": round(k_ms, 5)}
    log(f"cheb_step fine: {k_ms*1e3:.1f} us, {achieved:.0f} GB/s")

    extra = {"iterations": iters, "true_relres": true_rel,
             "solve_gbs": round(bytes_per_solve / (ms_per_step * 1e-3) / 1e9, 1),
             "solve_bytes": bytes_per_solve,
             "setup_s": round(setup_s, 3), "setup_ms": solver.setup_times(),
             "levels": levels}
    for kname in ("spmv", "restrict", "prolong"):
        kms, kb = solver.time_kernel(kname, level=0, reps=20)
        extra[f"{kname}_fine_gbs"] = round(kb / (kms * 1e-3) / 1e9, 1)

    if not args.no_mixed:
        sm = Solver(mesh.coords, mesh.l2g, w["p"], lam, Options(precision="mixed"))
        el_m, inf_m, xm = time_solves(torch, sm, bt, args.steps, args.warmup)
        err = (torch.linalg.norm(xm - x) / torch.linalg.norm(x)).item()
        extra["mixed"] = {"solves_per_s": round(args.steps / el_m, 3),
                          "iterations": inf_m[-1].iters, "true_relres": inf_m[-1].true_relres,
                          "rel_diff_vs_fp64": err,
                          "solve_gbs": round(inf_m[-1].bytes / (el_m / args.steps) / 1e9, 1)}
        k32_ms, k32_b = sm.time_kernel("cheb_step", level=0, reps=50, fp32=True)
        extra["mixed"]["cheb_step_fp32_gbs"] = round(k32_b / (k32_ms * 1e-3) / 1e9, 1)
        log(f"mixed: {args.steps / el_m:.2f} solves/s, {inf_m[-1].iters} iterations")
        sm.close()

    if not args.no_batched:
        extra["batched"] = batched_leg(torch, Solver, Options)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mesh, b, lam, w, iters)
    solver.close()

    out = {
        "metric": "GIAMG-PCG solves/s at 1e-10 relative residual (FP64)",
        "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: Helmholtz lambda={lam:.6g}, {w['n']}^3 perturbed "
                               f"hex mesh, p={w['p']}, {mesh.n_nodes} nodes, Chebyshev-2, "
                               f"p{w['p']}->...->p1 + SA, tol 1e-10",
                   "nodes": mesh.n_nodes, "nnz": levels[0]["nnz_A"], "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
