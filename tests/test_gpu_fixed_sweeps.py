"""Refinement with a fixed sweep count (ir_tol = 0): the same sweeps as the adaptive stop, with
no norm read back, so the call only enqueues kernels.  Its result must equal the adaptive
solve's when both run the same number of sweeps, meet the refinement tolerance against the CPU
oracle, and, captured into a graph by the caller, replay to the same result every time (each
replay checked, with other GPU work and synchronisations between replays).
"""
import numpy as np
import pytest

import workloads
from oracle import fv, solvers

pytestmark = pytest.mark.gpu
D, N = fv.DIRICHLET, fv.NEUMANN


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2461_amd import load
    load()
    return t


def _setup(seed):
    n = (28, 24, 30)
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(D, N, D), bc_hi=(D, D, N), sigma=0.3)
    f = workloads.rhs_uniform(seed, 2, prob.shape_xyz)
    ref = np.stack([solvers.solve_problem(prob.faces, 0.3, f[r:r + 1], prob.loc, prob.bc_lo, prob.bc_hi,
                                          method="splu")[0] for r in range(2)])
    return prob, f, ref


@pytest.mark.parametrize("precision", ["bf16x3_ir", "fp32_ir"])
def test_fixed_sweeps_match_adaptive(torch, precision):
    from paper_1107_2461_amd import Plan
    prob, f, ref = _setup(91)
    fd = torch.from_numpy(f).cuda()
    adaptive = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, precision=precision)
    ua = adaptive.solve(fd)
    k = adaptive.last_info["sweeps"]
    fixed = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, precision=precision, ir_tol=0.0, max_sweeps=k)
    uf = fixed.solve(fd)
    torch.cuda.synchronize()
    assert fixed.last_info["sweeps"] == k and fixed.last_info["converged"] is None
    assert torch.equal(ua, uf)
    u = uf.cpu().numpy()
    assert max(solvers.rel_err(u[r], ref[r]) for r in range(2)) <= 1e-10


def test_fixed_sweeps_captured_in_graph(torch):
    from paper_1107_2461_amd import Plan
    prob, f, ref = _setup(92)
    plan = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, precision="bf16x3_ir", ir_tol=0.0, max_sweeps=2)
    fd = torch.from_numpy(f).cuda()
    u = torch.empty_like(fd)
    ws = plan.workspace(2, fd.device)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.solve(fd, out=u, workspace=ws)       # eager reference on the capture stream
    s.synchronize()
    eager = u.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.solve(fd, out=u, workspace=ws)
    for rep in range(4):
        u.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, eager), rep
        (torch.randn(1 << 16, device="cuda", dtype=torch.float64) * 3).sum().item()
    assert max(solvers.rel_err(u.cpu().numpy()[r], ref[r]) for r in range(2)) <= 1e-10
