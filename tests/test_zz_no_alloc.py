"""helm_solve_noalloc (the solve with the library's static per-GPU workspace) against helm_solve
through the C ABI: two calls in a row, the second with a smaller input, for FP64 TPF and TPT,
split-BF16 with a fixed refinement sweep count and the all-Neumann pressure Laplacian; each
result must match helm_solve's within the solver's tolerance (FP64 1e-12, refined 1e-10; the
same kernels on the same data are expected to agree bit for bit) and the oracle.  The host-side
refusals (workspace above the array, adaptive refinement, stage timing) return EINVAL before
anything is launched."""
import numpy as np
import pytest

import workloads
from oracle import solvers

pytestmark = pytest.mark.gpu
D, N = 0, 1


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2461_amd import load
    load()
    return t


def _case(n, seed, nrhs, bc_lo=(D, N, D), bc_hi=(N, D, D), beta=1.5):
    faces = tuple(workloads.stretched_faces(n[d], beta) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=bc_lo, bc_hi=bc_hi, sigma=0.7)
    return prob, workloads.rhs_uniform(seed, nrhs, prob.shape_xyz)


def _rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("precision,method,tol", [("fp64", "tpf", 1e-12), ("fp64", "tpt", 1e-12),
                                                  ("bf16x3_ir", "tpf", 1e-10)])
def test_noalloc_matches_solve_two_calls(torch, precision, method, tol):
    from paper_1107_2461_amd import Plan
    kw = dict(precision=precision, method=method)
    if precision.endswith("_ir"):
        kw.update(ir_tol=0.0, max_sweeps=3)
    # first call: 36 x 28 x 24 with three right-hand sides and their own shifts; second: smaller
    for n, nrhs, seed in (((36, 28, 24), 3, 101), ((20, 16, 12), 1, 102)):
        prob, f = _case(n, seed, nrhs)
        sig = [0.7, 30.0, 0.01][:nrhs]
        plan = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, **kw)
        fd = torch.from_numpy(f).to("cuda")
        u_na = plan.solve_noalloc(fd, sigma=sig)
        u_ws = plan.solve(fd, sigma=sig)
        torch.cuda.synchronize()
        print(n, nrhs, precision, method, "bitwise" if torch.equal(u_na, u_ws) else _rel(u_na, u_ws), flush=True)
        assert _rel(u_na, u_ws) <= tol
        un = u_na.cpu().numpy()
        for r in range(nrhs):
            ref, _ = solvers.solve_problem(prob.faces, sig[r], f[r:r + 1], prob.loc, prob.bc_lo, prob.bc_hi,
                                           method="splu")
            assert solvers.rel_err(un[r], ref[0]) <= tol, (n, r)


def test_noalloc_pressure_refined_fixed_sweeps(torch):
    # all-Neumann Laplace: the refined path ends with the volume-weighted mean removal, whose
    # partial sums live in the workspace
    from paper_1107_2461_amd import Plan
    for n, seed in (((28, 24, 32), 103), ((20, 16, 12), 104)):
        faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
        f = workloads.remove_weighted_mean(workloads.rhs_uniform(seed, 1, n), faces)
        plan = Plan(faces, pressure=True, precision="bf16x3_ir", ir_tol=0.0, max_sweeps=3)
        fd = torch.from_numpy(f).to("cuda")
        u_na = plan.solve_noalloc(fd)
        u_ws = plan.solve(fd)
        torch.cuda.synchronize()
        assert _rel(u_na, u_ws) <= 1e-10
        ref, _ = solvers.solve_problem(faces, 0.0, f, bc_lo=(N,) * 3, bc_hi=(N,) * 3, method="splu")
        assert solvers.rel_err(u_na.cpu().numpy(), ref) <= 1e-10


def test_noalloc_refusals(torch):
    from paper_1107_2461_amd import HelmError, Plan
    from paper_1107_2461_amd._lib import NOALLOC_MAX_WORKSPACE
    prob, f = _case((128, 128, 128), 105, 1)
    plan = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma)
    # 128^3 FP64 with 17 right-hand sides needs 17 x 16 MiB > 256 MiB: refused on the host
    assert plan.workspace_bytes(17) > NOALLOC_MAX_WORKSPACE >= plan.workspace_bytes(16)
    big = torch.zeros((17, 128, 128, 128), dtype=torch.float64, device="cuda")
    with pytest.raises(HelmError, match="EINVAL"):
        plan.solve_noalloc(big)
    del big
    small = torch.from_numpy(f).to("cuda")
    adaptive = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, precision="bf16x3_ir")
    with pytest.raises(HelmError, match="EINVAL"):
        adaptive.solve_noalloc(small)               # adaptive refinement reads norms back
    plan.profile(True)
    with pytest.raises(HelmError, match="EINVAL"):
        plan.solve_noalloc(small)                   # stage timing creates events
    plan.profile(False)
    u = plan.solve_noalloc(small)                   # and the plain call still works afterwards
    torch.cuda.synchronize()
    assert _rel(u, plan.solve(small)) <= 1e-12
