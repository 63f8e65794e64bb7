"""GPU tests of the grouped solve (helm_solve_group): the right-hand sides of several plans of
one shape but their own grids (stretching, walls, shifts) solved together, one launch per stage
of eqs. 25-29.

Every right-hand side must match its plan solved alone (same kernels and summation order:
bitwise equality expected, the solver tolerance at worst) and the CPU FP64 oracle's sparse-LU
solution of its own system (FP64 <= 1e-12, refined split-BF16 <= 1e-10, relative 2-norm).
Right-hand sides come from the seeded generators of workloads.py.
"""
import numpy as np
import pytest

import workloads
from oracle import solvers

pytestmark = pytest.mark.gpu

D, N = workloads.DIRICHLET, workloads.NEUMANN


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2461_amd import load
    load()
    return t


# one shape, three grids: own stretch per axis, own walls, own shift
SHAPE = (32, 16, 32)
MEMBERS = (
    dict(beta=(1.5, 1.0, 2.0), lo=(D, D, D), hi=(D, D, D), sigma=10.0),
    dict(beta=(0.0, 1.75, 1.25), lo=(N, D, N), hi=(D, N, N), sigma=0.5),
    dict(beta=(2.0, 0.0, 1.5), lo=(N, N, D), hi=(N, N, D), sigma=0.0),
)


def _problem(m, shape=SHAPE):
    faces = tuple(workloads.stretched_faces(shape[d], m["beta"][d]) for d in range(3))
    return workloads.Problem(faces=faces, bc_lo=m["lo"], bc_hi=m["hi"], sigma=m["sigma"])


def _plans(precision, members=MEMBERS, shape=SHAPE, **kw):
    from paper_1107_2461_amd import Plan
    probs = [_problem(m, shape) for m in members]
    plans = [Plan(p.faces, p.bc_lo, p.bc_hi, p.sigma, precision=precision, **kw) for p in probs]
    return probs, plans


def _oracle(prob, f):
    ref, _ = solvers.solve_problem(prob.faces, prob.sigma, f, prob.loc, prob.bc_lo, prob.bc_hi, method="splu")
    return ref


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3_ir", 1e-10), ("bf16x3", 1e-5)])
def test_group_matches_alone_and_oracle(torch, precision, tol):
    from paper_1107_2461_amd import solve_group
    probs, plans = _plans(precision)
    nrhs = [1, 2, 1]
    fs = [workloads.rhs_normal(40 + i, n, SHAPE) for i, n in enumerate(nrhs)]
    f = torch.from_numpy(np.concatenate(fs)).to("cuda")
    info = {}
    u = solve_group(plans, f, nrhs, info=info)
    torch.cuda.synchronize()
    un = u.cpu().numpy()
    o = 0
    worst_alone, worst_oracle = 0.0, 0.0
    for i, (prob, plan, n) in enumerate(zip(probs, plans, nrhs)):
        alone = plan.solve(torch.from_numpy(fs[i]).to("cuda")).cpu().numpy()
        ref = _oracle(prob, fs[i])
        for r in range(n):
            worst_alone = max(worst_alone, solvers.rel_err(un[o + r], alone[r]))
            worst_oracle = max(worst_oracle, solvers.rel_err(un[o + r], ref[r]))
        o += n
    print(f"{precision}: group vs alone {worst_alone:.1e}, vs oracle {worst_oracle:.1e}, sweeps {info['sweeps']}")
    assert worst_oracle <= tol
    assert worst_alone <= (1e-13 if precision == "fp64" else tol)


def test_group_per_rhs_shifts(torch):
    """Shifts given per right-hand side override each plan's own."""
    from paper_1107_2461_amd import solve_group
    probs, plans = _plans("fp64")
    nrhs = [2, 1, 1]
    sig = [3.0, 0.25, 1e3, 7.5]
    fs = [workloads.rhs_uniform(50 + i, n, SHAPE) for i, n in enumerate(nrhs)]
    u = solve_group(plans, torch.from_numpy(np.concatenate(fs)).to("cuda"), nrhs, sigma=sig).cpu().numpy()
    o = 0
    for i, (prob, n) in enumerate(zip(probs, nrhs)):
        for r in range(n):
            ref, _ = solvers.solve_problem(prob.faces, sig[o + r], fs[i][r:r + 1], prob.loc, prob.bc_lo, prob.bc_hi,
                                           method="splu")
            assert solvers.rel_err(u[o + r], ref[0]) <= 1e-12
        o += n


def test_group_of_one_plan_is_multi_rhs(torch):
    from paper_1107_2461_amd import solve_group
    probs, plans = _plans("bf16x3_ir", members=MEMBERS[:1])
    p = plans[0]
    f = torch.from_numpy(workloads.rhs_normal(60, 3, SHAPE)).to("cuda")
    u = solve_group([p, p], f, [1, 2])
    ref = p.solve(f)
    assert torch.equal(u, ref)


def test_group_refusals(torch):
    from paper_1107_2461_amd import HelmError, Plan, solve_group
    probs, plans = _plans("fp64")
    f = torch.zeros((2,) + SHAPE[::-1], dtype=torch.float64, device="cuda")
    # different shapes
    other = Plan(tuple(workloads.stretched_faces(n, 1.0) for n in (32, 16, 16)), sigma=1.0)
    with pytest.raises(HelmError):
        solve_group([plans[0], other], f, [1, 1])
    # the Thomas method is not grouped
    tpt = Plan(probs[0].faces, probs[0].bc_lo, probs[0].bc_hi, 1.0, method="tpt")
    with pytest.raises(HelmError):
        solve_group([plans[0], tpt], f, [1, 1])
    # a tiling that cannot keep each workgroup inside one right-hand side
    ragged = [Plan(tuple(workloads.stretched_faces(n, b) for n in (20, 12, 10)), sigma=1.0) for b in (1.0, 1.5)]
    fr = torch.zeros((2, 10, 12, 20), dtype=torch.float64, device="cuda")
    with pytest.raises(HelmError):
        solve_group(ragged, fr, [1, 1])
    # a low-precision group with a singular (all-Neumann, sigma = 0) right-hand side
    sing = dict(beta=(1.0, 1.0, 1.0), lo=(N, N, N), hi=(N, N, N), sigma=0.0)
    _, lp = _plans("bf16x3_ir", members=(MEMBERS[0], sing))
    with pytest.raises(HelmError):
        solve_group(lp, f, [1, 1])
    torch.cuda.synchronize()


def test_group_fp64_singular_member(torch):
    """An all-Neumann Laplace member in an FP64 group: projected like a solve of its own."""
    from paper_1107_2461_amd import solve_group
    sing = dict(beta=(1.25, 1.5, 1.0), lo=(N, N, N), hi=(N, N, N), sigma=0.0)
    members = (MEMBERS[0], sing)
    probs, plans = _plans("fp64", members=members)
    fs = [workloads.rhs_uniform(70, 1, SHAPE), workloads.remove_weighted_mean(workloads.rhs_uniform(71, 1, SHAPE),
                                                                            probs[1].faces)]
    u = solve_group(plans, torch.from_numpy(np.concatenate(fs)).to("cuda"), [1, 1]).cpu().numpy()
    for i, prob in enumerate(probs):
        ref = _oracle(prob, fs[i])
        assert solvers.rel_err(u[i], ref[0]) <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3_ir", 1e-10)])
def test_server_groups_grids_of_one_shape(torch, precision, tol):
    """One slot: while the first request runs, requests on other grids of the same shape queue
    and are then solved together as one grouped solve; each result must equal its request
    solved alone and the oracle's solution of its own system."""
    from paper_1107_2461_amd import Plan, Server
    betas = [(1.0, 1.5, 2.0), (1.25, 1.25, 1.25), (2.0, 1.0, 1.5), (1.75, 2.0, 1.0), (1.5, 1.75, 1.75),
             (1.0, 1.0, 1.0)]
    walls = [((D, D, D), (D, D, D)), ((N, D, D), (D, D, N)), ((D, N, D), (D, D, D)), ((D, D, N), (N, D, D)),
             ((D, D, D), (N, N, D)), ((N, D, N), (D, N, D))]
    sigmas = [[0.5], [10.0, 0.01], [1.0], [200.0, 3.0], [0.2], [7.0]]
    probs, fs = [], []
    for i, (b, (lo, hi), sg) in enumerate(zip(betas, walls, sigmas)):
        probs.append(_problem(dict(beta=b, lo=lo, hi=hi, sigma=sg[0])))
        fs.append(torch.from_numpy(workloads.rhs_uniform(90 + i, len(sg), SHAPE)).to("cuda"))
    srv = Server(1 << 30, slots=1, precision=precision, max_bypass_ms=1000.0)
    for rnd in range(2):   # the first round builds the plans; the second runs with them resident
        us = [torch.empty_like(f) for f in fs]
        for i, (prob, f) in enumerate(zip(probs, fs)):
            srv.submit(10 * rnd + i, prob.faces, f, us[i], sigmas[i], prob.bc_lo, prob.bc_hi)
        srv.drain()
        recs = srv.poll(max_records=64)
    srv.close()
    torch.cuda.synchronize()
    assert len(recs) == len(probs) and all(r["status"] == 0 for r in recs), recs
    assert max(r["batch"] for r in recs) >= 3, recs
    worst_alone, worst_oracle = 0.0, 0.0
    for i, (prob, f) in enumerate(zip(probs, fs)):
        plan = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, precision=precision)
        ua = plan.solve(f, sigma=sigmas[i])
        torch.cuda.synchronize()
        worst_alone = max(worst_alone, float((ua - us[i]).norm() / ua.norm()))
        fn, un = f.cpu().numpy(), us[i].cpu().numpy()
        for r in range(fn.shape[0]):
            ref, _ = solvers.solve_problem(prob.faces, sigmas[i][r], fn[r:r + 1], prob.loc, prob.bc_lo, prob.bc_hi,
                                           method="splu")
            worst_oracle = max(worst_oracle, solvers.rel_err(un[r], ref[0]))
    print(f"{precision}: batches {[r['batch'] for r in recs]}, vs alone {worst_alone:.1e}, vs oracle {worst_oracle:.1e}")
    assert worst_alone <= tol and worst_oracle <= tol
