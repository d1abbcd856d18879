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
--workload {helmholtz16_p4,helmholtz32_p4}, --no-cpu-baseline, --no-mixed, --no-modal, --no-batched,
--serving {small,medium,full,off}; diagnostic runs (their own JSON line):
--study, --batched-only, --pmc-probe.
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
    "helmholtz16_p4": dict(n=16, p=4, lam=10.0, mesh_seed=2, rhs_seed=12, lam_seed=None),
    "helmholtz32_p4": dict(n=32, p=4, lam=None, mesh_seed=3, rhs_seed=23, lam_seed=13),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cheb_step.json")
KERNEL_SOURCES = ["paper_2512_15121_amd/csrc/kernels.hip", "paper_2512_15121_amd/csrc/kernels.h"]


def kernel_source_hash():
    """Hash of the kernel sources' code: comments and blank lines do not
    count, so editing a comment does not retire the stored counters."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
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


def modal_leg(torch, Solver, Options, w, lam, reps=3):
    """The same workload in the appendix's modal basis (injection
    transfers): same mesh vertices, order, lambda and right-hand side
    distribution; FP64 GIAMG-PCG to 1e-10."""
    import synth
    mesh = synth.hex_mesh(w["n"], w["p"], perturb=0.1, seed=w["mesh_seed"], basis="modal")
    b = torch.from_numpy(synth.normal_rhs(mesh.n_nodes, w["rhs_seed"])).to("cuda:0")
    s = Solver(mesh.coords, mesh.l2g, w["p"], lam, Options(basis="modal"))
    levels = [s.level(l) for l in range(s.num_levels())]
    s.solve(b, tol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        x, info = s.solve(b, tol=1e-10)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    s.close()
    out = {"solves_per_s": round(1.0 / dt, 3), "iterations": info.iters,
           "true_relres": info.true_relres, "solve_gbs": round(info.bytes / dt / 1e9, 1),
           "levels": [(d["kind"], d["order"], d["rows"], d["nnz_A"], d["nnz_P"]) for d in levels]}
    log(f"modal: {out}")
    return out


def study(torch, Solver, Options, reps=3):
    """The paper's parameter studies at p = 5 (Section 3.2, detailed
    analysis: number of Chebyshev smoothing steps; p-coarsening by one or by
    two) on a synthetic workload of the benchmark's size: Helmholtz lambda =
    10 on a 13^3 perturbed hex mesh, p = 5 (287,496 dofs), N(0,1) right-hand
    side, FP64 GIAMG-PCG to 1e-10; both bases."""
    import synth
    rows = []
    for basis in ("nodal", "modal"):
        mesh = synth.hex_mesh(13, 5, perturb=0.1, seed=7, basis=basis)
        b = torch.from_numpy(synth.normal_rhs(mesh.n_nodes, 17)).to("cuda:0")
        for sched in ((), (3, 1), (4, 3, 2, 1)):
            for degree in (1, 2, 3, 4):
                t0 = time.perf_counter()
                s = Solver(mesh.coords, mesh.l2g, 5, 10.0,
                           Options(basis=basis, schedule=sched, degree=degree, maxit=2000))
                setup_s = time.perf_counter() - t0
                s.solve(b, tol=1e-10)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    x, info = s.solve(b, tol=1e-10)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps
                orders = [s.level(l)["order"] for l in range(s.num_levels())
                          if s.level(l)["kind"] == "p"]
                s.close()
                row = {"basis": basis, "schedule": "->".join(str(o) for o in orders),
                       "chebyshev_degree": degree, "iterations": info.iters,
                       "status": info.status, "solve_ms": round(dt * 1e3, 3),
                       "ms_per_iteration": round(dt * 1e3 / max(info.iters, 1), 4),
                       "solves_per_s": round(1.0 / dt, 3), "setup_s": round(setup_s, 3)}
                rows.append(row)
                log(f"study: {row}")
    return {"workload": "Helmholtz lambda=10, 13^3 perturbed hex mesh (seed 7), p=5, "
                        "287496 dofs, N(0,1) rhs (seed 17), FP64 GIAMG-PCG to 1e-10",
            "rows": rows}


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


def serving_leg(torch, Server, Options, n_req=200, n_range=(4, 8), p_range=(2, 4), slots=8,
                chunk=2, seed=5):
    """Serving trace: requests for Helmholtz problems on n^3 perturbed meshes,
    n and p uniform in the given ranges, one mesh seed and one lambda
    (log-uniform [0.1, 100]) per (n, p) key, right-hand sides N(0, 1); mixed
    GIAMG-PCG to 1e-10.  A warm-up pass builds every hierarchy; then a
    closed-loop pass (all requests submitted at once) gives the saturation
    throughput S, and open-loop passes with Poisson arrivals at 0.7 S and
    0.4 S give p50 / p99 latency (submission to solution in host memory)."""
    import threading
    import synth
    rng = np.random.Generator(np.random.PCG64(seed))
    srv = Server(hbm_budget=int(100e9), slots=slots, chunk=chunk, tol=1e-10)
    problems = {}
    trace = []
    for i in range(n_req):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        if (n, p) not in problems:
            mesh = synth.hex_mesh(n, p, perturb=0.1, seed=1000 + 10 * n + p)
            lam = synth.loguniform_lambda(2000 + 10 * n + p)
            pid = srv.add_problem(mesh.coords, mesh.l2g, p, lam, Options(precision="mixed"))
            problems[(n, p)] = (pid, mesh.n_nodes)
        pid, nn = problems[(n, p)]
        trace.append((pid, synth.normal_rhs(nn, 50000 + i)))

    def run(arrivals):
        lat = [0.0] * len(trace)
        status = [0] * len(trace)
        rids = [None] * len(trace)
        ready = [threading.Event() for _ in trace]

        def waiter():
            for i in range(len(trace)):
                ready[i].wait()
                if rids[i] is None:        # submission stopped early
                    status[i] = -1
                    continue
                try:
                    _, info, l = srv.wait(rids[i])
                    lat[i] = l
                    status[i] = info.status
                except Exception as e:      # recorded, reported as a failed request
                    status[i] = getattr(e, "code", -1)
                    log(f"serving: request {i} failed: {e}")
        th = threading.Thread(target=waiter, daemon=True)
        th.start()
        t0 = time.perf_counter()
        try:
            for i, (pid, b) in enumerate(trace):
                if arrivals is not None:
                    delay = arrivals[i] - (time.perf_counter() - t0)
                    if delay > 0:
                        time.sleep(delay)
                rids[i] = srv.submit(pid, b)
                ready[i].set()
        finally:
            for e in ready:                # release the waiter whatever happened
                e.set()
            th.join()
        return time.perf_counter() - t0, np.array(lat), status

    try:
        t_warm, _, _ = run(None)                # warm-up: every hierarchy set up once
        log(f"serving: warm-up pass {t_warm:.2f} s ({len(problems)} hierarchies)")
        t_closed, lat_closed, st_closed = run(None)
        sat = len(trace) / t_closed
        log(f"serving: closed loop {sat:.1f} solves/s")
        gaps = rng.exponential(1.0 / (0.7 * sat), size=len(trace))
        t_open, lat_open, st_open = run(np.cumsum(gaps))
        log(f"serving: open loop at 0.7 S: {len(trace) / t_open:.1f} solves/s")
        # a lighter load too: with arrivals spread over many hierarchies few
        # requests share a batch, so the open loop saturates below S
        gaps4 = rng.exponential(1.0 / (0.4 * sat), size=len(trace))
        t_open4, lat_open4, st_open4 = run(np.cumsum(gaps4))
        log(f"serving: open loop at 0.4 S: {len(trace) / t_open4:.1f} solves/s")
        stats = srv.stats()
    finally:
        srv.close()
    out = {"workload": f"{n_req} requests, n in {list(n_range)}, p in {list(p_range)}, "
                       f"{len(problems)} hierarchies, mixed, {slots} slots per hierarchy",
           "saturation_solves_per_s": round(sat, 2),
           "open_loop_rate": round(0.7 * sat, 2),
           "open_loop_solves_per_s": round(len(trace) / t_open, 2),
           "p50_ms": round(float(np.percentile(lat_open, 50)), 3),
           "p99_ms": round(float(np.percentile(lat_open, 99)), 3),
           "closed_p50_ms": round(float(np.percentile(lat_closed, 50)), 3),
           "closed_p99_ms": round(float(np.percentile(lat_closed, 99)), 3),
           "open_loop_04": {"rate": round(0.4 * sat, 2),
                            "solves_per_s": round(len(trace) / t_open4, 2),
                            "p50_ms": round(float(np.percentile(lat_open4, 50)), 3),
                            "p99_ms": round(float(np.percentile(lat_open4, 99)), 3)},
           "all_ok": all(s_ == 0 for s_ in st_closed + st_open + st_open4),
           "setups": stats["setups"], "cache_hits": stats["cache_hits"],
           "peak_bytes": stats["peak_bytes"]}
    log(f"serving: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="helmholtz16_p4", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-modal", action="store_true")
    ap.add_argument("--study", action="store_true",
                    help="only run the parameter studies at p = 5 (Chebyshev degree x "
                         "p-schedule x basis) and print them as one JSON line")
    ap.add_argument("--serving", default="small", choices=["small", "medium", "full", "off"])
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched leg (64 right-hand sides, 20^3 p = 3) and print "
                         "it as one JSON line (for kernel traces of the block products)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch a 1 GiB copy (3x) and the fine Chebyshev step (5x), "
                         "for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (the solve would "
              "shard by element slabs, one process per GPU, halos exchanged over RCCL)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2512_15121_amd import Solver, Options

    dev = torch.device("cuda:0")
    if args.study:
        print(json.dumps({"study": study(torch, Solver, Options)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_leg(torch, Solver, Options)}), flush=True)
        return
    mesh, b, lam, w = problem(args.workload)
    if args.pmc_probe:
        src = torch.zeros(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        solver = Solver(mesh.coords, mesh.l2g, w["p"], lam, Options())
        ms, by = solver.time_kernel("cheb_step", level=0, reps=5)
        solver.close()
        log(f"pmc probe: copy 3 x {src.numel() * 8} B; cheb_step 6 launches "
            f"({by:.0f} algorithmic bytes, {ms * 1e3:.1f} us each)")
        return
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
                "kernel": "spmv_stream_kernel<double, SPMV_CHEB_STEP, 16, 1> (staged gathers) on the fine level",
                "bytes_per_launch": k_bytes, "ms_per_launch": round(k_ms, 5)}
    log(f"cheb_step fine: {k_ms*1e3:.1f} us, {achieved:.0f} GB/s")
    # a plain 1 GiB device copy in the same run: the bandwidth a streaming
    # kernel reaches here (read + write bytes over its time)
    src = torch.zeros(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    extra_copy = {"copy_1gib_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}
    log(f"1 GiB copy: {copy_gbs:.0f} GB/s; Chebyshev step at {achieved / copy_gbs:.2f} of it")

    extra = {"iterations": iters, "true_relres": true_rel,
             "solve_gbs": round(bytes_per_solve / (ms_per_step * 1e-3) / 1e9, 1),
             "solve_bytes": bytes_per_solve,
             "setup_s": round(setup_s, 3), "setup_ms": solver.setup_times(),
             "levels": levels, **extra_copy}
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

    if not args.no_modal:
        extra["modal"] = modal_leg(torch, Solver, Options, w, lam)
    if not args.no_batched:
        extra["batched"] = batched_leg(torch, Solver, Options)
    if args.serving != "off":
        from paper_2512_15121_amd import Server
        try:
            if args.serving == "full":
                extra["serving"] = serving_leg(torch, Server, Options, n_req=2000, n_range=(4, 24),
                                               p_range=(2, 6))
            elif args.serving == "medium":
                extra["serving"] = serving_leg(torch, Server, Options, n_req=2000, n_range=(4, 16),
                                               p_range=(2, 6))
            else:
                extra["serving"] = serving_leg(torch, Server, Options)
        except Exception as e:
            extra["serving"] = {"error": str(e)}
            log(f"serving leg failed: {e}")

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
