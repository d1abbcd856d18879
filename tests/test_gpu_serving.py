"""Continuous batching and serving through the C ABI.

* a right-hand side that joins a session while other columns are mid-solve
  gives the same bits as solved alone (giamg_solve_batch with k = 1);
* the server batches requests of different hierarchies, returns the same
  bits as the alone solves, matches the oracle, and evicts idle hierarchies
  under a small HBM budget without changing any result.
"""
import numpy as np
import pytest

import synth
from oracle import hierarchy, krylov

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2512_15121_amd import giamg
    giamg.library()
    return torch, torch.device("cuda:0")


PROBLEMS = [(4, 2, 1.0, 7), (5, 3, 2.5, 8), (3, 4, 0.7, 9)]


def _alone(torch, dev, m, p, lam, b, precision="mixed"):
    from paper_2512_15121_amd import Solver, Options
    s = Solver(m.coords, m.l2g, p, lam, Options(precision=precision))
    X, inf = s.solve_batch(torch.from_numpy(b[:, None].copy()).to(dev), tol=1e-10)
    s.close()
    return X[:, 0].cpu().numpy(), inf[0]


def test_session_join_midflight_bitwise(torch_dev):
    torch, dev = torch_dev
    from paper_2512_15121_amd import Solver, Options, Session
    n, p, lam, seed = PROBLEMS[1]
    m = synth.hex_mesh(n, p, perturb=0.1, seed=seed)
    s = Solver(m.coords, m.l2g, p, lam, Options(precision="mixed"))
    sess = Session(s, 4, tol=1e-10)
    bs = [synth.normal_rhs(m.n_nodes, 30 + i) for i in range(3)]
    bt = [torch.from_numpy(b).to(dev) for b in bs]
    sess.admit([0], [bt[0]])
    sess.step(3)
    sess.admit([2], [bt[1]])          # joins while slot 0 is mid-solve
    assign = {0: 0, 2: 1}             # slot -> right-hand side
    results = {}
    for _ in range(300):
        sess.step(1)
        running, infos = sess.poll()
        for slot, idx in list(assign.items()):
            if running[slot]:
                continue
            results[idx] = (sess.retire(slot, torch.zeros_like(bt[0])).cpu().numpy(), infos[slot])
            del assign[slot]
            if idx == 0:
                sess.admit([0], [bt[2]])   # reuse the freed slot while slot 2 runs
                assign[0] = 2
        if len(results) == 3:
            break
    sess.close()
    s.close()
    assert len(results) == 3
    for key, b in enumerate(bs):
        x, info = results[key]
        xa, ia = _alone(torch, dev, m, p, lam, b)
        assert info.iters == ia.iters and info.status == 0
        assert np.array_equal(x, xa), key


def test_server_mixed_hierarchies(torch_dev):
    torch, dev = torch_dev
    from paper_2512_15121_amd import Server, Options
    meshes = [synth.hex_mesh(n, p, perturb=0.1, seed=sd) for n, p, lam, sd in PROBLEMS]
    srv = Server(hbm_budget=8 << 30, slots=4, chunk=2, tol=1e-10)
    pids = [srv.add_problem(m.coords, m.l2g, p, lam, Options(precision="mixed"))
            for m, (n, p, lam, sd) in zip(meshes, PROBLEMS)]
    reqs = []
    for i in range(12):
        j = i % 3
        b = synth.normal_rhs(meshes[j].n_nodes, 100 + i)
        reqs.append((srv.submit(pids[j], b), j, b))
    results = [(srv.wait(r), j, b) for r, j, b in reqs]
    st = srv.stats()
    srv.close()
    assert st["completed"] == 12 and st["setups"] == 3
    for (x, info, lat), j, b in results:
        n, p, lam, sd = PROBLEMS[j]
        assert info.status == 0 and lat > 0
        xa, ia = _alone(torch, dev, meshes[j], p, lam, b)
        assert np.array_equal(x, xa)
        H = hierarchy.build(meshes[j].coords, meshes[j].l2g, p, lam)
        ref = krylov.giamg_pcg(H, b, tol=1e-10)
        assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_server_fp64_without_staged_tables(torch_dev):
    """The configuration of the largest serving trace: FP64 hierarchies
    built with direct gathers (no staged-gather tables kept; the server's
    block products never read them).  Results are bitwise those of the same
    right-hand side solved alone on a default FP64 handle, and match the
    oracle."""
    torch, dev = torch_dev
    from paper_2512_15121_amd import Server, Options
    meshes = [synth.hex_mesh(n, p, perturb=0.1, seed=sd) for n, p, lam, sd in PROBLEMS]
    srv = Server(hbm_budget=8 << 30, slots=4, chunk=2, tol=1e-10)
    pids = [srv.add_problem(m.coords, m.l2g, p, lam, Options(precision="fp64", direct_gathers=True))
            for m, (n, p, lam, sd) in zip(meshes, PROBLEMS)]
    reqs = []
    for i in range(9):
        j = i % 3
        b = synth.normal_rhs(meshes[j].n_nodes, 200 + i)
        reqs.append((srv.submit(pids[j], b), j, b))
    results = [(srv.wait(r), j, b) for r, j, b in reqs]
    st = srv.stats()
    srv.close()
    assert st["completed"] == 9 and st["setups"] == 3
    for (x, info, lat), j, b in results:
        n, p, lam, sd = PROBLEMS[j]
        assert info.status == 0
        xa, ia = _alone(torch, dev, meshes[j], p, lam, b, precision="fp64")
        assert info.iters == ia.iters and np.array_equal(x, xa)
        H = hierarchy.build(meshes[j].coords, meshes[j].l2g, p, lam)
        ref = krylov.giamg_pcg(H, b, tol=1e-10)
        assert abs(info.iters - ref.iters) <= 1
        assert np.linalg.norm(x - ref.x) <= 1e-9 * np.linalg.norm(ref.x)


def test_server_admission_hold(torch_dev):
    """With an admission hold, requests that do not fill a hierarchy's free
    slots join once the oldest has waited the hold -- the full hold_ms
    before any request has finished there (the first request below waits at
    least that long), afterwards at most the last request's solve time (the
    next ones finish far sooner than hold_ms).  Every result is bitwise the
    solve alone."""
    torch, dev = torch_dev
    from paper_2512_15121_amd import Server, Options
    n, p, lam, sd = PROBLEMS[1]
    m = synth.hex_mesh(n, p, perturb=0.1, seed=sd)
    hold = 1500
    srv = Server(hbm_budget=8 << 30, slots=4, chunk=2, tol=1e-10, hold_ms=hold)
    pid = srv.add_problem(m.coords, m.l2g, p, lam, Options(precision="mixed"))
    b0 = synth.normal_rhs(m.n_nodes, 299)
    first = srv.wait(srv.submit(pid, b0))            # 1 of 4 slots: the full hold
    bs = [synth.normal_rhs(m.n_nodes, 300 + i) for i in range(3)]   # 3 < 4 free slots
    out = [srv.wait(r) for r in [srv.submit(pid, b) for b in bs]]
    # then more than the free slots
    bs2 = [synth.normal_rhs(m.n_nodes, 310 + i) for i in range(6)]
    out2 = [srv.wait(r) for r in [srv.submit(pid, b) for b in bs2]]
    srv.close()
    assert first[2] >= hold
    assert max(lat for _, _, lat in out) < hold
    for (x, info, lat), b in zip([first] + out + out2, [b0] + bs + bs2):
        assert info.status == 0
        xa, ia = _alone(torch, dev, m, p, lam, b)
        assert info.iters == ia.iters and np.array_equal(x, xa)


def test_server_budget_evicts_and_stays_exact(torch_dev):
    torch, dev = torch_dev
    from paper_2512_15121_amd import Server, Options
    probs = PROBLEMS[1:]
    meshes = [synth.hex_mesh(n, p, perturb=0.1, seed=sd) for n, p, lam, sd in probs]
    # measure each group's device footprint with an ample budget
    sizes = []
    for m, (n, p, lam, sd) in zip(meshes, probs):
        s0 = Server(hbm_budget=8 << 30, slots=2, chunk=2, tol=1e-10)
        pid = s0.add_problem(m.coords, m.l2g, p, lam, Options(precision="mixed"))
        s0.wait(s0.submit(pid, synth.normal_rhs(m.n_nodes, 1)))
        sizes.append(s0.stats()["resident_bytes"])
        s0.close()
    # room for either group, never both
    budget = sum(sizes) - 1
    srv = Server(hbm_budget=budget, slots=2, chunk=2, tol=1e-10)
    pids = [srv.add_problem(m.coords, m.l2g, p, lam, Options(precision="mixed"))
            for m, (n, p, lam, sd) in zip(meshes, probs)]
    out = []
    for i in range(6):
        j = i % 2
        b = synth.normal_rhs(meshes[j].n_nodes, 200 + i)
        r = srv.submit(pids[j], b)
        out.append((srv.wait(r), j, b))
    st = srv.stats()
    srv.close()
    assert st["evictions"] >= 4 and st["completed"] == 6
    assert st["peak_bytes"] <= budget
    for (x, info, lat), j, b in out:
        n, p, lam, sd = probs[j]
        xa, _ = _alone(torch, dev, meshes[j], p, lam, b)
        assert np.array_equal(x, xa)


def test_server_queues_more_requests_than_slots(torch_dev):
    """Requests beyond the free slots wait for the running chunk to end
    (regression: a queued request must not produce an empty admission)."""
    torch, dev = torch_dev
    from paper_2512_15121_amd import Server, Options
    n, p, lam, sd = PROBLEMS[0]
    m = synth.hex_mesh(n, p, perturb=0.1, seed=sd)
    srv = Server(hbm_budget=1 << 30, slots=2, chunk=1, tol=1e-10)
    pid = srv.add_problem(m.coords, m.l2g, p, lam, Options(precision="mixed"))
    bs = [synth.normal_rhs(m.n_nodes, 300 + i) for i in range(10)]
    rids = [srv.submit(pid, b) for b in bs]
    res = [srv.wait(r) for r in rids]
    st = srv.stats()
    srv.close()
    assert st["completed"] == 10 and st["setups"] == 1
    for (x, info, lat), b in zip(res, bs):
        xa, ia = _alone(torch, dev, m, p, lam, b)
        assert info.status == 0 and np.array_equal(x, xa)


def test_server_rejects_invalid_problem(torch_dev):
    """A registered problem passes the same mesh and option checks as
    giamg_setup, at registration (not later on the setup worker)."""
    from paper_2512_15121_amd import Server, Options, GiamgError, giamg
    m = synth.hex_mesh(2, 2, perturb=0.1, seed=3)
    srv = Server(hbm_budget=1 << 30, slots=2, chunk=2, tol=1e-10)
    bad_l2g = m.l2g.copy()
    bad_l2g[0, 0] = m.n_nodes
    cases = [(m.l2g, 2, 0.0, Options(degree=0), "degree"),
             (m.l2g, 2, float("inf"), Options(), "lambda"),
             (bad_l2g, 2, 0.0, Options(), "l2g"),
             (m.l2g, 2, 0.0, Options(schedule=[2]), "schedule")]
    for l2g, p, lam, opts, word in cases:
        with pytest.raises(GiamgError) as e:
            srv.add_problem(m.coords, l2g, p, lam, opts)
        assert e.value.code == giamg.EINVAL and word in str(e.value), word
    pid = srv.add_problem(m.coords, m.l2g, 2, 0.0, Options())
    x, info, _ = srv.wait(srv.submit(pid, synth.normal_rhs(m.n_nodes, 5)))
    assert info.status == 0 and np.isfinite(x).all()
    srv.close()
