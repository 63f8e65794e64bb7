"""GPU tests of the continuous-batching server.

Each request's result in the mix must equal the same request solved alone (the same kernels
on the same data: bitwise equality is expected, and at worst the solver tolerance) and the
CPU FP64 oracle's solution of its system (FP64 <= 1e-12, refined split-BF16 <= 1e-10); the
device-workspace budget is respected at every instant; requests overlap in time when the
budget and slots allow it, and are serialised when the budget admits only one at a time.
Right-hand sides come from the seeded generators of workloads.py.
"""
import numpy as np
import pytest

import workloads
from oracle import solvers

pytestmark = pytest.mark.gpu

GRIDS = ((24, 20, 28), (32, 32, 32), (40, 24, 16), (17, 33, 21))
BIG_GRIDS = ((64, 64, 64), (96, 64, 80), (128, 128, 128))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2461_amd import load
    load()
    return t


def _requests(torch, n, seed, grids=GRIDS):
    reqs = workloads.serving_requests(seed, n, rate_hz=1000.0, grids=grids)
    out = []
    for r in reqs:
        prob = workloads.serving_problem(r)
        f = torch.from_numpy(workloads.rhs_normal(r["rhs_seed"], r["nrhs"], prob.shape_xyz)).to("cuda")
        out.append((r, prob, f))
    return out


def _oracle_err(prob, f, u):
    """Largest per-RHS relative 2-norm error of u against the oracle's sparse-LU solution."""
    fn = f.cpu().numpy()
    ref, _ = solvers.solve_problem(prob.faces, prob.sigma, fn, prob.loc, prob.bc_lo, prob.bc_hi, method="splu")
    un = u.cpu().numpy()
    return max(solvers.rel_err(un[r], ref[r]) for r in range(fn.shape[0]))


def _run_server(torch, reqs, precision, budget, slots, warm=True):
    """Submit every request back to back (after a first pass that fills the plan cache)."""
    from paper_1107_2461_amd import Server
    srv = Server(budget, slots=slots, precision=precision, max_bypass_ms=20.0)
    outs, recs = {}, []
    for _ in range(2 if warm else 1):
        outs = {}
        for r, prob, f in reqs:
            u = torch.empty_like(f)
            outs[r["rid"]] = u
            srv.submit(r["rid"], prob.faces, f, u, [prob.sigma] * f.shape[0], prob.bc_lo, prob.bc_hi)
        srv.drain()
        recs = srv.poll(max_records=len(reqs) + 8)
    srv.close()
    torch.cuda.synchronize()
    return outs, recs


def _alone(torch, prob, f, precision):
    from paper_1107_2461_amd import Plan
    plan = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, precision=precision)
    u = plan.solve(f)
    torch.cuda.synchronize()
    return u


def _same(torch, a, b):
    return torch.equal(a, b) or float((a - b).norm() / a.norm()) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "bf16x3_ir"])
def test_mix_equals_alone_and_overlaps(torch, precision):
    budget = 2 << 30
    reqs = _requests(torch, 24, seed=5, grids=BIG_GRIDS)
    outs, recs = _run_server(torch, reqs, precision, budget=budget, slots=4)
    assert len(recs) == len(reqs)
    assert all(r["status"] == 0 for r in recs), recs
    bitwise = 0
    for r, prob, f in reqs:
        ua = _alone(torch, prob, f, precision)
        um = outs[r["rid"]]
        bitwise += int(torch.equal(ua, um))
        assert _same(torch, ua, um), r
    print(f"{precision}: {bitwise}/{len(reqs)} results bitwise identical alone and in the mix")
    # budget and slots respected at every admission instant; some requests ran concurrently
    for t in sorted({x["t_admit"] for x in recs}):
        # requests solved together share one solve (slot, completion time) and its footprint
        live = {(x["slot"], x["t_done"]): x["footprint"] for x in recs if x["t_admit"] <= t < x["t_done"]}
        assert sum(live.values()) <= budget
        assert len(live) <= 4
    overl = sum(1 for a in recs for b in recs
                if a["id"] < b["id"] and a["t_admit"] < b["t_done"] and b["t_admit"] < a["t_done"])
    print(f"{precision}: {overl} overlapping request pairs")
    assert overl > 0
    for x in recs:
        assert x["t_submit"] <= x["t_admit"] <= x["t_done"]
    # cold plans, ragged grids, mixed walls, Laplace requests: each served result equals the
    # request alone and the oracle's solution
    small = _requests(torch, 16, seed=7)
    outs_s, _ = _run_server(torch, small, precision, budget=64 << 20, slots=4, warm=False)
    tol = 1e-12 if precision == "fp64" else 1e-10
    worst = 0.0
    for r, prob, f in small:
        assert _same(torch, _alone(torch, prob, f, precision), outs_s[r["rid"]]), r
        err = _oracle_err(prob, f, outs_s[r["rid"]])
        worst = max(worst, err)
        assert err <= tol, (r, err)
    print(f"{precision}: served small-grid mix vs oracle, worst relative error {worst:.2e}")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3_ir", 1e-10)])
def test_same_plan_requests_ride_along(torch, precision, tol):
    # one slot: while the first request of a plan runs, the next ones queue and are then solved
    # together as one multi-RHS solve, each with its own shifts; every result must equal the
    # request solved alone, and the budget counts the batch (with its staging) once
    from paper_1107_2461_amd import Server
    n = (48, 40, 36)
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(1, 0, 0), bc_hi=(0, 0, 1), sigma=1.0)
    shapes = [(1, [0.5]), (3, [10.0, 0.01, 3.0]), (2, [1.0, 200.0]), (1, [0.2]), (2, [7.0, 7.0])]
    fs = [torch.from_numpy(workloads.rhs_uniform(80 + i, k, prob.shape_xyz)).to("cuda")
          for i, (k, _) in enumerate(shapes)]
    budget = 1 << 30
    srv = Server(budget, slots=1, precision=precision, max_bypass_ms=1000.0)
    for rnd in range(2):   # the first round builds the plan; the second runs with it resident
        us = [torch.empty_like(f) for f in fs]
        for i, ((k, sig), f) in enumerate(zip(shapes, fs)):
            srv.submit(10 * rnd + i, prob.faces, f, us[i], sig, prob.bc_lo, prob.bc_hi)
        srv.drain()
        recs = srv.poll(max_records=64)
    srv.close()
    torch.cuda.synchronize()
    assert len(recs) == len(shapes) and all(r["status"] == 0 for r in recs), recs
    assert max(r["batch"] for r in recs) >= 2, recs
    solves = {(r["slot"], r["t_done"]): r["footprint"] for r in recs}
    assert all(fp <= budget for fp in solves.values())
    from paper_1107_2461_amd import Plan
    for i, ((k, sig), f) in enumerate(zip(shapes, fs)):
        plan = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, precision=precision)
        ua = plan.solve(f, sigma=sig)
        torch.cuda.synchronize()
        assert float((ua - us[i]).norm() / ua.norm()) <= tol, (i, precision)
        fn = f.cpu().numpy()
        un = us[i].cpu().numpy()
        for r in range(k):   # each right-hand side with its own shift, against the oracle
            ref, _ = solvers.solve_problem(prob.faces, sig[r], fn[r:r + 1], prob.loc, prob.bc_lo, prob.bc_hi,
                                           method="splu")
            assert solvers.rel_err(un[r], ref[0]) <= tol, (i, r, precision)


def test_tight_budget_serialises(torch):
    from paper_1107_2461_amd import Plan
    reqs = _requests(torch, 8, seed=6, grids=BIG_GRIDS)
    foot = 0
    for r, prob, f in reqs:
        p = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma)
        foot = max(foot, p.workspace_bytes(f.shape[0]))
    outs, recs = _run_server(torch, reqs, "fp64", budget=foot, slots=4)
    for a in recs:
        for b in recs:
            if a["id"] < b["id"] and a["footprint"] + b["footprint"] > foot:
                # two requests that do not fit together never run at the same time
                assert a["t_done"] <= b["t_admit"] + 1e-9 or b["t_done"] <= a["t_admit"] + 1e-9
    for r, prob, f in reqs:
        assert _same(torch, _alone(torch, prob, f, "fp64"), outs[r["rid"]])


def test_submit_rejects_request_larger_than_budget(torch):
    from paper_1107_2461_amd import HelmError, Server
    prob = workloads.box_problem(32, 1.5, 1.0)
    f = torch.zeros((1, 32, 32, 32), dtype=torch.float64, device="cuda")
    srv = Server(1024, slots=1)
    with pytest.raises(HelmError, match="EINVAL"):
        srv.submit(1, prob.faces, f, torch.empty_like(f), [1.0])
    srv.close()


def test_plan_cache_counters(torch):
    """Every submit is one plan lookup: a miss builds the plan (counted with its setup time),
    and repeats of a grid/wall combination hit the resident plan."""
    from paper_1107_2461_amd import Server
    reqs = _requests(torch, 12, seed=8)
    keys = {(tuple(np.round(np.concatenate(prob.faces), 15)), tuple(prob.bc_lo), tuple(prob.bc_hi))
            for _, prob, _ in reqs}
    srv = Server(1 << 30, slots=2)
    for _ in range(2):
        for r, prob, f in reqs:
            srv.submit(r["rid"], prob.faces, f, torch.empty_like(f), [prob.sigma] * f.shape[0], prob.bc_lo,
                       prob.bc_hi)
        srv.drain()
    st = srv.stats()
    srv.close()
    assert st["submitted"] == st["completed"] == 2 * len(reqs)
    assert st["plan_hits"] + st["plan_misses"] == 2 * len(reqs)
    assert st["plan_misses"] == len(keys)
    assert st["setup_seconds"] > 0.0


def test_resident_plans_bounded_lru(torch):
    """Beyond 2048 resident plans the least recently used is evicted: after 2100 distinct grids,
    the first grid misses again (rebuilt) while the most recent one hits."""
    from paper_1107_2461_amd import Server
    n = 8
    f = torch.randn((1, n, n, n), device="cuda", dtype=torch.float64)
    N = 2100
    grids = [tuple(workloads.stretched_faces(n, 1.0 + 0.0004 * k) for _ in range(3)) for k in range(N)]
    srv = Server(1 << 30, slots=2)
    outs = []
    for k, faces in enumerate(grids):
        u = torch.empty_like(f)
        outs.append(u)
        srv.submit(k, faces, f, u, [1.0])
    srv.drain()
    st = srv.stats()
    assert st["plan_misses"] == N and st["plan_hits"] == 0
    srv.submit(1000, grids[-1], f, torch.empty_like(f), [1.0])    # resident
    srv.submit(1001, grids[0], f, torch.empty_like(f), [1.0])     # evicted long ago
    srv.drain()
    recs = srv.poll(max_records=N + 8)
    st = srv.stats()
    srv.close()
    assert st["plan_hits"] == 1 and st["plan_misses"] == N + 1
    assert len(recs) == N + 2 and all(r["status"] == 0 for r in recs)


def test_submit_waits_for_the_callers_stream(torch):
    """f is written by a long torch kernel on the caller's stream right before submit; the
    solve must see the written values (the server waits for an event recorded at submit)."""
    from paper_1107_2461_amd import Server
    prob = workloads.box_problem((96, 80, 64), 1.5, 2.0)
    nx, ny, nz = prob.shape_xyz
    src = torch.from_numpy(workloads.rhs_normal(91, 2, prob.shape_xyz)).to("cuda")
    big = torch.randn((4096, 4096), dtype=torch.float64, device="cuda")
    srv = Server(1 << 30, slots=2)
    outs = []
    for rep in range(3):
        f = torch.zeros_like(src)
        # queue a few large products, then the write of f, all on the current stream; nothing
        # is synchronized before submit
        acc = big
        for _ in range(4):
            acc = acc @ big / 4096.0
        f.copy_(src + 0.0 * acc[0, 0])
        u = torch.empty_like(f)
        srv.submit(rep, prob.faces, f, u, [2.0, 2.0])
        outs.append((f, u))
    srv.drain()
    srv.close()
    torch.cuda.synchronize()
    ua = _alone(torch, prob, src, "fp64")
    for f, u in outs:
        assert torch.equal(u, ua) or float((u - ua).norm() / ua.norm()) <= 1e-12


def test_server_holds_exactly_its_budget(torch):
    """The workspace arena is the budget, taken once from the allocator at creation: a stream of
    requests of several sizes allocates nothing more, and destroying the server returns it."""
    from paper_1107_2461_amd import Server, torch_allocator
    al = torch_allocator()
    reqs = _requests(torch, 12, seed=9)
    budget = 48 << 20
    torch.cuda.synchronize()
    m0, b0 = torch.cuda.memory_allocated(), al.blocks()
    srv = Server(budget, slots=3, allocator=al)
    m1 = torch.cuda.memory_allocated()
    assert al.blocks() == b0 + 1 and m1 - m0 >= budget
    for rnd in range(2):
        outs = {}
        for r, prob, f in reqs:
            u = torch.empty_like(f)
            outs[r["rid"]] = u
            srv.submit(r["rid"], prob.faces, f, u, [prob.sigma] * f.shape[0], prob.bc_lo, prob.bc_hi)
        srv.drain()
        recs = srv.poll(max_records=64)
        assert len(recs) == len(reqs) and all(x["status"] == 0 for x in recs)
        # device memory beyond the arena: only the plans' eigenbases (shared per axis, resident)
        if rnd == 0:
            m_plans = torch.cuda.memory_allocated()
        else:
            assert torch.cuda.memory_allocated() == m_plans
    for r, prob, f in reqs:
        assert _same(torch, _alone(torch, prob, f, "fp64"), outs[r["rid"]])
    srv.close()
    del outs, u                   # the outputs were allocated after m0 was taken
    torch.cuda.synchronize()
    assert al.blocks() == b0 and torch.cuda.memory_allocated() == m0


def test_plan_memory_from_torch_allocator(torch):
    """A plan built with the torch allocator keeps its device memory in torch's caching allocator
    (memory_allocated rises by at least its FP64 eigenbases) and solves exactly as a plan on
    hipMalloc memory; destroying it returns the memory."""
    from paper_1107_2461_amd import Plan, torch_allocator
    al = torch_allocator()
    n = (40, 36, 44)
    faces = tuple(workloads.stretched_faces(n[d], 1.3 + 0.1 * d) for d in range(3))
    f = torch.from_numpy(workloads.rhs_uniform(93, 2, n)).to("cuda")
    import gc
    for precision in ("fp64", "bf16x3_ir"):
        torch.cuda.synchronize()
        m0, b0 = torch.cuda.memory_allocated(), al.blocks()
        plan = Plan(faces, (0, 1, 0), (0, 0, 1), 0.5, precision=precision, allocator=al)
        m1 = torch.cuda.memory_allocated()
        assert al.blocks() > b0
        assert m1 - m0 >= sum(2 * k * k * 8 for k in n), (m1 - m0)
        u = plan.solve(f)
        ref = Plan(faces, (0, 1, 0), (0, 0, 1), 0.5, precision=precision).solve(f)
        torch.cuda.synchronize()
        assert torch.equal(u, ref)
        plan._ws.clear()          # the binding's cached solve workspace (a torch tensor of its own)
        torch.cuda.synchronize()
        m2 = torch.cuda.memory_allocated()
        del plan
        gc.collect()
        torch.cuda.synchronize()
        # destroying the plan returns exactly what building it took (other tensors stay)
        assert al.blocks() == b0 and m2 - torch.cuda.memory_allocated() == m1 - m0


def test_one_big_solve_at_a_time(torch):
    """Solves of 2^23 or more unknowns x right-hand sides run one at a time: with eight such
    requests queued (on 256^3 grids, 1 or 2 RHS, different stretching, so that riders cannot
    join a 2-RHS head within 2^25) and four slots, no two big solves overlap in time, while the
    small requests submitted behind them are solved beside them; every big result matches the
    same request solved alone."""
    from paper_1107_2461_amd import Plan, Server
    n = 256
    gen = torch.Generator(device="cuda").manual_seed(11)
    big = []
    for q in range(8):
        beta = 1.0 + 0.1 * q
        prob = workloads.box_problem(n, beta, 1.0)
        f = torch.randn((1 + q % 2, n, n, n), generator=gen, device="cuda", dtype=torch.float64)
        big.append((prob, f))
    small = _requests(torch, 12, 31)
    srv = Server(8 << 30, slots=4, precision="fp64", max_bypass_ms=1000.0)
    outs = {}
    torch.cuda.synchronize()
    for q, (prob, f) in enumerate(big):
        outs[q] = torch.empty_like(f)
        srv.submit(q, prob.faces, f, outs[q], [prob.sigma] * f.shape[0], prob.bc_lo, prob.bc_hi)
    for r, prob, f in small:
        u = torch.empty_like(f)
        outs[100 + r["rid"]] = u
        srv.submit(100 + r["rid"], prob.faces, f, u, [prob.sigma] * f.shape[0], prob.bc_lo, prob.bc_hi)
    srv.drain()
    recs = srv.poll(max_records=64)
    srv.close()
    assert len(recs) == len(big) + len(small) and all(r["status"] == 0 for r in recs)
    solves = {}  # one entry per big solve (riders share their head's slot and completion time)
    for r in recs:
        if r["id"] < 100:
            solves.setdefault((r["slot"], r["t_done"]), []).append(r)
    spans = sorted((min(x["t_admit"] for x in v), max(x["t_done"] for x in v)) for v in solves.values())
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0, ("two big solves overlap", spans)
    beside = [r for r in recs if r["id"] >= 100 and any(a <= r["t_admit"] < d for a, d in spans)]
    print(f"big solves {len(spans)}, small requests admitted while a big one ran: {len(beside)} of {len(small)}")
    for q, (prob, f) in enumerate(big):
        ref = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma).solve(f)
        torch.cuda.synchronize()
        d = float((outs[q] - ref).abs().max() / ref.abs().max())
        assert d <= 1e-12, (q, d)
