"""Benchmark: GIAMG-PCG solves/s on one MI355X, with the HBM roofline of the
dominant kernel and the CPU oracle timed beside it.

Headline workload (default): Helmholtz -lap u + lambda u = f on a 32 x 32 x 32
hexahedral mesh of the unit cube, order p = 4 (2,146,689 nodes, 423,663,057
stored nonzeros), interior vertices perturbed by U(-0.1 h, 0.1 h) (seed 3),
lambda log-uniform on [0.1, 100] (seed 13), right-hand side i.i.d. N(0, 1)
(seed 23), hierarchy p4 -> p2 -> p1 then smoothed aggregation down to <= 2000
rows, Chebyshev degree 2, CG to ||r|| / ||b|| < 1e-10.  `value` is the FP64
solve rate; the mixed-precision form (FP32 V-cycle in FP64 flexible CG) on
the same problem is in extra.mixed.  A step is one whole solve from x = 0;
the hierarchy is built once before timing (setup time reported apart).

Roofline: the fused Chebyshev step on the fine operator, timed per launch by
HIP events its own dispatches record during the timed solves, against its
algorithmic bytes (values and 32-bit column ids per nonzero, row pointers,
the gathered vector and the output once, five row-local update streams);
the library's own format bytes and the rocprofv3 counter bytes are reported
beside them.

Prints one JSON line.  Options: --gpus (1 only), --steps, --warmup,
--workload {helmholtz32_p4,helmholtz16_p4}, --no-cpu-baseline, --no-mixed,
--no-modal, --no-batched, --no-small, --no-study, --serving
{small,medium,full,off}; diagnostic runs (their own JSON line): --study,
--batched-only, --serving-only, --pmc-probe.
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
# A manufactured-solution latency case: 4^3 uniform mesh, p = 2, lambda = 1,
# Jacobi smoothing (omega = 2/3, two sweeps), p2 -> p1.
MANUFACTURED = dict(n=4, p=2, lam=1.0)
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


def cheb_step_algorithmic_bytes(nnz, n, vb):
    """Bytes a fused Chebyshev step on an n-row operator with nnz stored
    nonzeros must move: each value (vb bytes) and a 32-bit column id, the
    int64 row pointers, the gathered vector and the new direction once, and
    the five row-local streams of the update (residual read and written,
    inverse diagonal read, iterate read and written)."""
    return (vb + 4.0) * nnz + 8.0 * (n + 1) + 2.0 * vb * n + 5.0 * vb * n


def time_solves(torch, solver, bt, steps, warmup):
    """W untimed solves, then K timed solves bracketed by device
    synchronisations.  During the timed solves every launch of the fine-level
    Chebyshev step is timed by events its dispatch records itself (no markers
    between kernels); returns the wall time, the infos, x and the mean
    duration (ms) and count of those launches."""
    x = torch.zeros_like(bt)
    for _ in range(warmup):
        x.zero_()
        solver.solve(bt, x, tol=1e-10)
    solver.profile_read(reset=True)
    solver.profile(True, fine_step_only=True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        _, info = solver.solve(bt, x, tol=1e-10)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    solver.profile(False)
    prof = solver.profile_read(reset=True)
    ms, cnt = prof["fine_step"]
    return elapsed, infos, x, (ms / cnt if cnt else float("nan")), cnt


def breakdown(torch, solver, bt, reps=2):
    """The paper's breakdown categories (Section 3.2) per solve, from HIP
    events around every phase of `reps` profiled solves (not timed runs)."""
    solver.profile_read(reset=True)
    solver.profile(True)
    x = torch.zeros_like(bt)
    for _ in range(reps):
        x.zero_()
        solver.solve(bt, x, tol=1e-10)
    torch.cuda.synchronize()
    solver.profile(False)
    p = solver.profile_read(reset=True)
    out = {"ms_per_solve": {k: round(v[0] / reps, 4) for k, v in p.items()
                            if isinstance(v, tuple) and v[1] > 0},
           "intervals_per_solve": {k: v[1] // reps for k, v in p.items()
                                   if isinstance(v, tuple) and v[1] > 0},
           "iterations_per_solve": p["iterations"] // max(p["solves"], 1)}
    return out


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


def cpu_baseline(mesh, b, lam, w, gpu_iters, name):
    """The oracle's whole FP64 solve on workload `name` (setup untimed), a
    few solves on one core; value in solves/s of that workload."""
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
            "sample": f"{reps} complete oracle solves of the {name} workload ({w['n']}^3 hexahedra, "
                      f"p = {w['p']}, {mesh.n_nodes} nodes; FP64 PCG to 1e-10, {iters} iterations each, "
                      f"the GPU took {gpu_iters} on it), BLAS limited to 1 thread; oracle setup "
                      f"{setup_s:.1f} s not timed; the headline workload's oracle setup does not fit "
                      f"a bench run"}


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


def study(torch, Solver, Options, reps=2, bases=("nodal", "modal")):
    """The paper's parameter studies at p = 5 (Section 3.2, detailed
    analysis: number of Chebyshev smoothing steps; p-coarsening by one or by
    two) on a synthetic workload of the benchmark's size: Helmholtz lambda =
    10 on a 13^3 perturbed hex mesh, p = 5 (287,496 dofs), N(0,1) right-hand
    side, FP64 GIAMG-PCG to 1e-10, with the phase breakdown of each
    configuration and the diagonally preconditioned CG on the same system."""
    import synth
    rows = []
    for basis in bases:
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
                bd = breakdown(torch, s, b, reps=1)["ms_per_solve"]
                s.close()
                row = {"basis": basis, "schedule": "->".join(str(o) for o in orders),
                       "chebyshev_degree": degree, "iterations": info.iters,
                       "status": info.status, "solve_ms": round(dt * 1e3, 3),
                       "ms_per_iteration": round(dt * 1e3 / max(info.iters, 1), 4),
                       "solves_per_s": round(1.0 / dt, 3), "setup_s": round(setup_s, 3),
                       "breakdown_ms": bd}
                rows.append(row)
                log(f"study: {basis} {row['schedule']} degree {degree}: {info.iters} it, "
                    f"{row['solves_per_s']}/s")
        if basis == "nodal":
            s = Solver(mesh.coords, mesh.l2g, 5, 10.0, Options(preconditioner="jacobi", maxit=20000))
            x, info = s.solve(b, tol=1e-10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = s.solve(b, tol=1e-10)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s.close()
            rows.append({"basis": basis, "schedule": "none (diagonal preconditioner)",
                         "iterations": info.iters, "status": info.status,
                         "solve_ms": round(dt * 1e3, 3),
                         "ms_per_iteration": round(dt * 1e3 / max(info.iters, 1), 4),
                         "solves_per_s": round(1.0 / dt, 3)})
            log(f"study: diagonal PCG {info.iters} it, {1.0 / dt:.3f}/s")
    return {"workload": "Helmholtz lambda=10, 13^3 perturbed hex mesh (seed 7), p=5, "
                        "287496 dofs, N(0,1) rhs (seed 17), FP64 GIAMG-PCG to 1e-10",
            "rows": rows}


def small_legs(torch, Solver, Options, steps=10):
    """The benchmark's two other single-solve workloads: Helmholtz lambda = 10
    on a 16^3 perturbed mesh at p = 4 (274,625 dofs; FP64 and mixed solves/s)
    and the manufactured-solution case (4^3 uniform, p = 2, Jacobi, load
    vector of f = (lambda + 3 pi^2) sin sin sin; latency per solve)."""
    import math
    import synth
    out = {}
    mesh, b, lam, w = problem("helmholtz16_p4")
    bt = torch.from_numpy(b).to("cuda:0")
    h16 = {}
    for prec in ("fp64", "mixed"):
        s = Solver(mesh.coords, mesh.l2g, w["p"], lam, Options(precision=prec))
        el, infos, _, step_ms, _ = time_solves(torch, s, bt, steps, 2)
        h16[prec] = {"solves_per_s": round(steps / el, 2), "iterations": infos[-1].iters,
                     "true_relres": infos[-1].true_relres,
                     "fine_step_us": round(step_ms * 1e3, 2)}
        s.close()
    out["helmholtz16_p4"] = h16
    log(f"helmholtz16_p4: {h16}")
    mm = synth.hex_mesh(MANUFACTURED["n"], MANUFACTURED["p"])
    s = Solver(mm.coords, mm.l2g, MANUFACTURED["p"], MANUFACTURED["lam"], Options(smoother="jacobi"))
    xq = s.quadrature_points()
    fq = (MANUFACTURED["lam"] + 3 * math.pi ** 2) * np.prod(np.sin(math.pi * xq), axis=2)
    bm = torch.from_numpy(s.load_vector(fq)).to("cuda:0")
    x = torch.zeros_like(bm)
    for _ in range(5):
        x.zero_()
        s.solve(bm, x, tol=1e-10)
    torch.cuda.synchronize()
    lat = []
    for _ in range(50):
        x.zero_()
        t0 = time.perf_counter()
        _, info = s.solve(bm, x, tol=1e-10)
        lat.append(time.perf_counter() - t0)
    s.close()
    out["manufactured_4cube_p2"] = {"latency_ms_p50": round(1e3 * float(np.median(lat)), 4),
                                    "latency_ms_p99": round(1e3 * float(np.percentile(lat, 99)), 4),
                                    "iterations": info.iters, "true_relres": info.true_relres,
                                    "gpu_solve_ms": round(info.solve_ms, 4)}
    log(f"manufactured_4cube_p2: {out['manufactured_4cube_p2']}")
    return out


def jacobi_leg(torch, Solver, Options, mesh, lam, w, bt):
    """The diagonally preconditioned CG baseline (the paper's DCG comparison)
    on the headline system: one FP64 solve to 1e-10 after one warm-up."""
    s = Solver(mesh.coords, mesh.l2g, w["p"], lam, Options(preconditioner="jacobi", maxit=50000))
    x = torch.zeros_like(bt)
    s.solve(bt, x, tol=1e-10)
    torch.cuda.synchronize()
    x.zero_()
    t0 = time.perf_counter()
    _, info = s.solve(bt, x, tol=1e-10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.close()
    out = {"solves_per_s": round(1.0 / dt, 4), "iterations": info.iters, "status": info.status,
           "true_relres": info.true_relres, "ms_per_iteration": round(dt * 1e3 / max(info.iters, 1), 4),
           "solve_gbs": round(info.bytes / dt / 1e9, 1)}
    log(f"jacobi pcg: {out}")
    return out


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
                chunk=2, seed=5, budget=100e9, min_window_s=3.0, precision="mixed", direct=False,
                hold_ms=0):
    """Serving trace: requests for Helmholtz problems on n^3 perturbed meshes,
    n and p uniform in the given ranges, one mesh seed and one lambda
    (log-uniform [0.1, 100]) per (n, p) key, right-hand sides N(0, 1);
    GIAMG-PCG to 1e-10 (mixed precision unless stated; direct=True keeps no
    staged-gather tables, which the block products of the server never read).  A warm-up pass builds every hierarchy; a closed-loop
    pass (every request submitted at once) gives the saturation throughput S;
    open-loop passes with Poisson arrivals at 0.7 S and 0.4 S replay the
    trace until the arrivals span at least min_window_s (so the latency tail
    of the last requests does not dominate the served rate) and give p50 /
    p99 latency (submission to solution in host memory), the offered and
    served rates, and the median latency of the first and the last quarter
    of the requests (growing latency means a growing queue)."""
    import threading
    import synth
    rng = np.random.Generator(np.random.PCG64(seed))
    srv = Server(hbm_budget=int(budget), slots=slots, chunk=chunk, tol=1e-10, hold_ms=hold_ms)
    problems = {}
    trace = []
    for i in range(n_req):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        if (n, p) not in problems:
            mesh = synth.hex_mesh(n, p, perturb=0.1, seed=1000 + 10 * n + p)
            lam = synth.loguniform_lambda(2000 + 10 * n + p)
            pid = srv.add_problem(mesh.coords, mesh.l2g, p, lam,
                                  Options(precision=precision, direct_gathers=direct))
            problems[(n, p)] = (pid, mesh.n_nodes)
        pid, nn = problems[(n, p)]
        trace.append((pid, synth.normal_rhs(nn, 50000 + i)))

    def run(reqs, arrivals):
        lat = [0.0] * len(reqs)
        status = [0] * len(reqs)
        rids = [None] * len(reqs)
        t_sub = [0.0] * len(reqs)
        ready = [threading.Event() for _ in reqs]

        def waiter():
            for i in range(len(reqs)):
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
                if (i + 1) % 100 == 0:
                    log(f"serving: {i + 1} of {len(reqs)} requests done "
                        f"({time.perf_counter() - t0:.1f} s)")
        th = threading.Thread(target=waiter, daemon=True)
        th.start()
        t0 = time.perf_counter()
        t_last = t0
        try:
            for i, (pid, b) in enumerate(reqs):
                if arrivals is not None:
                    delay = arrivals[i] - (time.perf_counter() - t0)
                    if delay > 0:
                        time.sleep(delay)
                rids[i] = srv.submit(pid, b)
                t_last = time.perf_counter()
                t_sub[i] = t_last - t0
                ready[i].set()
        finally:
            for e in ready:                # release the waiter whatever happened
                e.set()
            th.join()
        return time.perf_counter() - t0, t_last - t0, np.array(lat), status, np.array(t_sub)

    def open_loop(rate):
        reps = max(1, int(np.ceil(min_window_s * rate / len(trace))))
        reqs = trace * reps
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
        t_all, t_arr, lat, st, t_sub = run(reqs, arrivals)
        q = max(1, len(reqs) // 4)
        # steady window: the last three quarters of the arrival span, where
        # completions (submission + latency) are counted against arrivals;
        # served_rate over the whole run also counts the drain after the
        # last arrival
        a, b = 0.25 * t_arr, t_arr
        done_t = t_sub + lat * 1e-3
        w_arr = int(np.count_nonzero((t_sub >= a) & (t_sub <= b)))
        w_done = int(np.count_nonzero((done_t >= a) & (done_t <= b)))
        return {"offered_rate": round(rate, 2), "requests": len(reqs),
                "arrival_rate": round(len(reqs) / max(t_arr, 1e-9), 2),
                "served_rate": round(len(reqs) / t_all, 2),
                "window_arrival_rate": round(w_arr / max(b - a, 1e-9), 2),
                "window_served_rate": round(w_done / max(b - a, 1e-9), 2),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "first_quarter_p50_ms": round(float(np.median(lat[:q])), 3),
                "last_quarter_p50_ms": round(float(np.median(lat[-q:])), 3)}, st

    try:
        t_warm = run(trace, None)[0]             # warm-up: every hierarchy set up once
        log(f"serving: warm-up pass {t_warm:.2f} s ({len(problems)} hierarchies)")
        t_closed, _, lat_closed, st_closed, _ = run(trace, None)
        sat = len(trace) / t_closed
        log(f"serving: closed loop {sat:.1f} solves/s")
        o7, st7 = open_loop(0.7 * sat)
        log(f"serving: open loop at 0.7 S: {o7}")
        o4, st4 = open_loop(0.4 * sat)
        log(f"serving: open loop at 0.4 S: {o4}")
        stats = srv.stats()
    finally:
        srv.close()
    out = {"workload": f"{n_req} requests, n in {list(n_range)}, p in {list(p_range)}, "
                       f"{len(problems)} hierarchies, {precision}{', no staged tables' if direct else ''}, "
                       f"{slots} slots per hierarchy, "
                       f"{'admission hold ' + str(hold_ms) + ' ms, ' if hold_ms else ''}"
                       f"chunk {chunk}, HBM budget {budget / 1e9:.0f} GB",
           "saturation_solves_per_s": round(sat, 2),
           "closed_p50_ms": round(float(np.percentile(lat_closed, 50)), 3),
           "closed_p99_ms": round(float(np.percentile(lat_closed, 99)), 3),
           "p50_ms": o7["p50_ms"], "p99_ms": o7["p99_ms"],
           "open_loop_07": o7, "open_loop_04": o4,
           "warmup_s": round(t_warm, 2),
           "all_ok": all(s_ == 0 for s_ in list(st_closed) + list(st7) + list(st4)),
           "setups": stats["setups"], "evictions": stats["evictions"],
           "cache_hits": stats["cache_hits"], "peak_bytes": stats["peak_bytes"]}
    log(f"serving: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="helmholtz32_p4", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-modal", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the 16^3 p = 4 and manufactured-solution legs")
    ap.add_argument("--no-study", action="store_true",
                    help="skip the nodal parameter study at p = 5")
    ap.add_argument("--no-jacobi", action="store_true",
                    help="skip the diagonally preconditioned CG baseline")
    ap.add_argument("--study", action="store_true",
                    help="only run the parameter studies at p = 5 (Chebyshev degree x "
                         "p-schedule x basis, with breakdowns) and print them as one JSON line")
    ap.add_argument("--serving", default="small", choices=["small", "medium", "large", "full", "off"])
    ap.add_argument("--serving-slots", type=int, default=8,
                    help="right-hand sides batched per hierarchy in the serving leg")
    ap.add_argument("--serving-chunk", type=int, default=2,
                    help="CG iterations between admission points in the serving leg")
    ap.add_argument("--serving-hold", type=int, default=None,
                    help="serving: admission hold in ms (requests join a hierarchy once they fill its free "
                         "slots or the oldest has waited this long, or a hierarchy's last solve time "
                         "if shorter; 0 = at the next chunk boundary); default 10000")
    ap.add_argument("--serving-only", action="store_true",
                    help="only run the serving leg given by --serving and print it as one JSON line")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched leg (64 right-hand sides, 20^3 p = 3) and print "
                         "it as one JSON line (for kernel traces of the block products)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch a 1 GiB copy (3x) and the fine Chebyshev step (6x), "
                         "for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (the solve would "
              "shard by element slabs, one process per GPU, halos exchanged over RCCL)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_15121_amd import Solver, Options, read_bandwidth

    dev = torch.device("cuda:0")
    if args.study:
        print(json.dumps({"study": study(torch, Solver, Options)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_leg(torch, Solver, Options)}), flush=True)
        return
    if args.serving_only:
        from paper_2512_15121_amd import Server
        print(json.dumps({"serving": serving(torch, Server, Options, args.serving, args.serving_slots,
                                             args.serving_chunk, args.serving_hold)}), flush=True)
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
            f"({by:.0f} format bytes, {ms * 1e3:.1f} us each)")
        return
    log(f"workload {args.workload}: n={w['n']} p={w['p']} nodes={mesh.n_nodes} lambda={lam:.6g}")
    # a process's first setup also pays the runtime's one-time load of the
    # library's code objects (~0.15 s): a tiny hierarchy takes it first, so
    # setup_s is the hierarchy's own setup
    import synth
    tiny = synth.hex_mesh(2, 2, perturb=0.1, seed=1)
    t0 = time.perf_counter()
    Solver(tiny.coords, tiny.l2g, 2, 1.0, Options()).close()
    first_use_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    solver = Solver(mesh.coords, mesh.l2g, w["p"], lam, Options())
    setup_s = time.perf_counter() - t0
    levels = [solver.level(l) for l in range(solver.num_levels())]
    log(f"setup {setup_s:.2f} s; levels {[(d['kind'], d['order'], d['rows'], d['nnz_A']) for d in levels]}")
    bt = torch.from_numpy(b).to(dev)
    elapsed, infos, x, step_ms, step_launches = time_solves(torch, solver, bt, args.steps, args.warmup)
    iters = infos[-1].iters
    assert all(i.status == 0 and i.iters == iters for i in infos)
    true_rel = infos[-1].true_relres
    bytes_per_solve = infos[-1].bytes
    value = args.steps / elapsed
    ms_per_step = 1000.0 * elapsed / args.steps
    log(f"fp64: {value:.2f} solves/s, {iters} iterations, true relres {true_rel:.2e}")

    # dominant kernel: the fused Chebyshev step on the fine operator, timed in
    # the timed solves above; algorithmic bytes from the operator's sizes
    n0, nnz0 = levels[0]["rows"], levels[0]["nnz_A"]
    alg_bytes = cheb_step_algorithmic_bytes(nnz0, n0, 8)
    iso_ms, fmt_bytes = solver.time_kernel("cheb_step", level=0, reps=50)
    achieved = alg_bytes / (step_ms * 1e-3) / 1e9
    stream_gbs = read_bandwidth(4 << 30, 10)
    traffic = traffic_entry(args.workload)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic,
                "kernel": "spmv_stream_kernel<double, SPMV_CHEB_STEP, 16, 1> (staged gathers) "
                          "on the fine level",
                "bytes_per_launch": alg_bytes,
                "ms_per_launch": round(step_ms, 5),
                "launches_timed": step_launches,
                "format_bytes_per_launch": fmt_bytes,
                "format_gbs": round(fmt_bytes / (step_ms * 1e-3) / 1e9, 1),
                "traffic_gbs": (round(traffic / (step_ms * 1e-3) / 1e9, 1) if traffic else None),
                "read_stream_gbs": round(stream_gbs, 1),
                "frac_of_read_stream": round(achieved / stream_gbs, 4),
                "isolated_ms_per_launch": round(iso_ms, 5)}
    log(f"cheb_step fine: {step_ms * 1e3:.1f} us in the solves ({step_launches} launches), "
        f"{achieved:.0f} GB/s algorithmic = {achieved / PEAK_HBM_GBS:.3f} of 8 TB/s; "
        f"isolated {iso_ms * 1e3:.1f} us; read stream {stream_gbs:.0f} GB/s")

    extra = {"iterations": iters, "true_relres": true_rel,
             "solve_gbs": round(bytes_per_solve / (ms_per_step * 1e-3) / 1e9, 1),
             "solve_bytes": bytes_per_solve,
             "setup_s": round(setup_s, 3), "setup_ms": solver.setup_times(),
             "first_use_s": round(first_use_s, 3),
             "levels": levels}
    for kname in ("spmv", "restrict", "prolong"):
        kms, kb = solver.time_kernel(kname, level=0, reps=20)
        extra[f"{kname}_fine_format_gbs"] = round(kb / (kms * 1e-3) / 1e9, 1)
    extra["breakdown_fp64"] = breakdown(torch, solver, bt)
    log(f"breakdown fp64: {extra['breakdown_fp64']['ms_per_solve']}")

    if not args.no_mixed:
        sm = Solver(mesh.coords, mesh.l2g, w["p"], lam, Options(precision="mixed"))
        el_m, inf_m, xm, step32_ms, _ = time_solves(torch, sm, bt, args.steps, args.warmup)
        err = (torch.linalg.norm(xm - x) / torch.linalg.norm(x)).item()
        alg32 = cheb_step_algorithmic_bytes(nnz0, n0, 4)
        extra["mixed"] = {"solves_per_s": round(args.steps / el_m, 3),
                          "speedup_vs_fp64": round(el_m and elapsed / el_m, 3),
                          "iterations": inf_m[-1].iters, "true_relres": inf_m[-1].true_relres,
                          "rel_diff_vs_fp64": err,
                          "solve_gbs": round(inf_m[-1].bytes / (el_m / args.steps) / 1e9, 1),
                          "cheb_step_fp32_us": round(step32_ms * 1e3, 2),
                          "cheb_step_fp32_algorithmic_gbs": round(alg32 / (step32_ms * 1e-3) / 1e9, 1),
                          "cheb_step_fp32_frac": round(alg32 / (step32_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        extra["breakdown_mixed"] = breakdown(torch, sm, bt)
        log(f"mixed: {args.steps / el_m:.2f} solves/s, {inf_m[-1].iters} iterations")
        sm.close()
    if not args.no_jacobi:
        extra["jacobi_pcg"] = jacobi_leg(torch, Solver, Options, mesh, lam, w, bt)
    if not args.no_small:
        extra.update(small_legs(torch, Solver, Options))
    if not args.no_modal:
        extra["modal"] = modal_leg(torch, Solver, Options, WORKLOADS["helmholtz16_p4"], 10.0)
    if not args.no_batched:
        extra["batched"] = batched_leg(torch, Solver, Options)
    if not args.no_study:
        extra["study_nodal_p5"] = study(torch, Solver, Options, reps=1, bases=("nodal",))
    if args.serving != "off":
        from paper_2512_15121_amd import Server
        extra["serving"] = serving(torch, Server, Options, args.serving, args.serving_slots,
                                   args.serving_chunk, args.serving_hold)

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle builds a 16^3, p = 4 hierarchy in about ten seconds; the
        # headline 32^3 one (8x the elements) does not fit a bench run
        cmesh, cb, clam, cw = problem("helmholtz16_p4")
        cpu = cpu_baseline(cmesh, cb, clam, cw, extra.get("helmholtz16_p4", {}).get("fp64", {}).get("iterations"),
                           "helmholtz16_p4")
    solver.close()

    out = {
        "metric": "GIAMG-PCG solves/s at 1e-10 relative residual (FP64; mixed precision in extra.mixed)",
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


def serving(torch, Server, Options, size, slots=8, chunk=2, hold_ms=None):
    """The serving trace of the chosen size (small: 200 requests, n <= 8,
    p <= 4; medium: 2000 requests, n <= 16, p <= 6, ~78 GB of hierarchies;
    large: 2000 requests, n <= 20, p <= 6, ~187 GB, the largest n range
    whose hierarchies all fit one MI355X's HBM; full: n <= 24, ~381 GB of
    hierarchies in mixed precision, so the full trace runs in FP64 without
    staged-gather tables, ~15 B per fine nonzero, within a 270 GB budget)."""
    if hold_ms is None:   # admission in batches, held at most one solve's time (or 10 s)
        hold_ms = 10000
    try:
        if size == "full":
            return serving_leg(torch, Server, Options, n_req=2000, n_range=(4, 24), p_range=(2, 6),
                               budget=270e9, slots=slots, chunk=chunk, precision="fp64", direct=True,
                               hold_ms=hold_ms)
        if size == "large":
            return serving_leg(torch, Server, Options, n_req=2000, n_range=(4, 20), p_range=(2, 6),
                               budget=250e9, slots=slots, chunk=chunk, hold_ms=hold_ms)
        if size == "medium":
            return serving_leg(torch, Server, Options, n_req=2000, n_range=(4, 16), p_range=(2, 6),
                               slots=slots, chunk=chunk, hold_ms=hold_ms)
        return serving_leg(torch, Server, Options, slots=slots, chunk=chunk, hold_ms=hold_ms)
    except Exception as e:
        log(f"serving leg failed: {e}")
        return {"error": str(e)}


if __name__ == "__main__":
    main()
