"""GPU parity: the HIP solve path (through the C ABI) against the CPU FP64 oracle.

Tolerances (relative 2-norm error against the oracle, per the accuracy targets of the
solver): FP64 TPF/TPT <= 1e-12; refined FP32/BF16 <= 1e-10; unrefined FP32 <= 1e-5;
unrefined BF16 <= 1e-2.  All-Neumann Laplace solutions are compared in the zero
volume-weighted-mean gauge (the solution is defined up to a constant, eq. 28 discussion).
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


def _gpu(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _solve(torch, prob, f, sigma=None, **kw):
    from paper_1107_2461_amd import Plan
    plan = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, loc=prob.loc, **kw)
    u = plan.solve(_gpu(torch, f), sigma=sigma)
    torch.cuda.synchronize()
    return u.cpu().numpy(), plan


def _oracle(prob, f, sigma=None, method="auto"):
    if sigma is None:
        u, _ = solvers.solve_problem(prob.faces, prob.sigma, f, prob.loc, prob.bc_lo, prob.bc_hi, method=method)
        return u
    out = np.empty_like(f)
    for r in range(f.shape[0]):
        out[r], _ = solvers.solve_problem(prob.faces, sigma[r], f[r:r + 1], prob.loc, prob.bc_lo, prob.bc_hi,
                                          method=method)
    return out


def _per_rhs_err(u, ref):
    return max(solvers.rel_err(u[r], ref[r]) for r in range(ref.shape[0]))


def test_small_dirichlet_tpf_fp64(torch):
    prob, f = workloads.workload_small_dirichlet()
    u, _ = _solve(torch, prob, f)
    ref = _oracle(prob, f, method="splu")
    assert _per_rhs_err(u, ref) <= 1e-12


def test_small_dirichlet_tpt_fp64(torch):
    prob, f = workloads.workload_small_dirichlet()
    u, _ = _solve(torch, prob, f, method="tpt")
    u2, _ = _solve(torch, prob, f, method="tpf")
    ref = _oracle(prob, f, method="splu")
    assert _per_rhs_err(u, ref) <= 1e-12
    assert _per_rhs_err(u, u2) <= 1e-12      # TPF and TPT agree (Section 5.1: >= 10 digits)


RAGGED = [
    # (n, betas, bc_lo, bc_hi, loc)  -- several tiles plus ragged tails on every axis
    ((19, 23, 17), (1.5, 1.0, 2.0), (D, N, D), (N, D, D), (fv.CELL,) * 3),
    ((37, 18, 21), (2.0, 1.5, 1.0), (D, D, N), (D, D, D), fv.velocity_loc(0)),
    ((16, 33, 20), (1.25, 1.5, 1.75), (N, D, D), (D, D, N), fv.velocity_loc(1)),
    ((24, 14, 35), (1.0, 2.0, 1.5), (D, D, D), (D, D, D), fv.velocity_loc(2)),
    ((65, 7, 9), (1.5, 1.5, 1.5), (D, N, N), (D, N, N), (fv.CELL,) * 3),
]


@pytest.mark.parametrize("case", range(len(RAGGED)))
@pytest.mark.parametrize("method", ["tpf", "tpt"])
def test_ragged_mixed_bc_fp64(torch, case, method):
    n, betas, lo, hi, loc = RAGGED[case]
    faces = tuple(workloads.stretched_faces(n[d], betas[d]) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=lo, bc_hi=hi, loc=loc, sigma=0.7)
    sig = [0.7, 3.0e2, 0.0]
    f = workloads.rhs_uniform(11 + case, 3, prob.shape_xyz)
    u, _ = _solve(torch, prob, f, sigma=sig, method=method)
    ref = _oracle(prob, f, sigma=sig, method="splu")
    assert _per_rhs_err(u, ref) <= 1e-12


def _gauge(x, faces):
    return workloads.remove_weighted_mean(x, faces)


@pytest.mark.parametrize("method", ["tpf", "tpt"])
def test_all_neumann_laplace_projection(torch, method):
    n = (20, 17, 26)
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(N,) * 3, bc_hi=(N,) * 3, sigma=0.0)
    f = workloads.rhs_uniform(21, 2, prob.shape_xyz)       # not mean-free: the solver projects it
    u, _ = _solve(torch, prob, f, method=method)
    ref = _oracle(prob, f, method="splu")
    assert _per_rhs_err(u, ref) <= 1e-12                      # u has zero weighted mean already
    assert _per_rhs_err(_gauge(u, faces), ref) <= 1e-12
    # the FP64 path has no projection pass: the zeroed null coefficient alone leaves the
    # weighted mean at the rounding level
    for r in range(2):
        assert np.abs(u[r] - _gauge(u, faces)[r]).max() <= 1e-14 * np.abs(u[r]).max()
    # eq. 28 option: zero denominator replaced by 1 -> differs from the projection by a constant
    u28, _ = _solve(torch, prob, f, method=method, null_mode=1)
    d = u28 - u
    for r in range(2):
        assert np.ptp(d[r]) <= 1e-11 * np.abs(u[r]).max()


def test_pressure_plan_entry_point(torch):
    from paper_1107_2461_amd import Plan
    n = (24, 20, 28)
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(N,) * 3, bc_hi=(N,) * 3, sigma=0.0)
    f = workloads.remove_weighted_mean(workloads.rhs_uniform(4, 1, prob.shape_xyz), faces)
    plan = Plan(faces, pressure=True)
    u = plan.solve(_gpu(torch, f)).cpu().numpy()
    ref = _oracle(prob, f, method="splu")
    assert _per_rhs_err(u, ref) <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 1e-2), ("bf16x3", 1e-5), ("fp32_ir", 1e-10),
                                           ("bf16_ir", 1e-10), ("bf16x3_ir", 1e-10)])
def test_low_precision_and_refinement(torch, precision, tol):
    prob = workloads.box_problem((40, 36, 44), 1.5, sigma=0.1)
    f = workloads.rhs_normal(3, 2, prob.shape_xyz)
    u, plan = _solve(torch, prob, f, precision=precision)
    ref = _oracle(prob, f, method="splu")
    err = _per_rhs_err(u, ref)
    print(precision, err, plan.last_info)
    assert err <= tol


@pytest.mark.parametrize("case", range(len(RAGGED)))
def test_ragged_mixed_bc_split_bf16_refined(torch, case):
    """Split-BF16 products with refinement on ragged, staggered, multi-RHS problems (tails of
    every tile, rows not multiple of 8, per-RHS shifts including a Laplace RHS)."""
    n, betas, lo, hi, loc = RAGGED[case]
    faces = tuple(workloads.stretched_faces(n[d], betas[d]) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=lo, bc_hi=hi, loc=loc, sigma=0.7)
    sig = [0.7, 3.0e2, 0.0]
    f = workloads.rhs_uniform(31 + case, 3, prob.shape_xyz)
    u, plan = _solve(torch, prob, f, sigma=sig, precision="bf16x3_ir")
    ref = _oracle(prob, f, sigma=sig, method="splu")
    assert plan.last_info["converged"]
    assert _per_rhs_err(u, ref) <= 1e-10


@pytest.mark.parametrize("precision", ["bf16_ir", "bf16x3_ir", "fp32_ir"])
def test_refinement_neumann_laplace(torch, precision):
    n = (32, 28, 36)
    faces = tuple(workloads.stretched_faces(n[d], 2.0) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(N,) * 3, bc_hi=(N,) * 3, sigma=0.0)
    f = workloads.remove_weighted_mean(workloads.rhs_uniform(5, 1, prob.shape_xyz), faces)
    u, plan = _solve(torch, prob, f, precision=precision)
    ref = _oracle(prob, f, method="splu")
    assert plan.last_info["converged"]
    assert _per_rhs_err(u, ref) <= 1e-10          # the solver returns the zero-mean gauge


def test_apply_matches_oracle_operator(torch):
    n, betas, lo, hi, loc = RAGGED[1]
    faces = tuple(workloads.stretched_faces(n[d], betas[d]) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=lo, bc_hi=hi, loc=loc, sigma=2.5)
    from paper_1107_2461_amd import Plan
    plan = Plan(faces, lo, hi, 2.5, loc=loc)
    u = workloads.rhs_uniform(7, 2, prob.shape_xyz)
    hu = plan.apply(_gpu(torch, u)).cpu().numpy()
    ref = solvers.apply_operator(faces, 2.5, u, loc, lo, hi)
    assert _per_rhs_err(hu, ref) <= 1e-14


def test_error_paths(torch):
    from paper_1107_2461_amd import HelmError, Plan
    prob = workloads.box_problem(12, 1.0, sigma=1.0)
    lam, _, _ = Plan(prob.faces, sigma=1.0).eigen(0)
    lam_y, _, _ = Plan(prob.faces, sigma=1.0).eigen(1)
    lam_z, _, _ = Plan(prob.faces, sigma=1.0).eigen(2)
    bad_sigma = -(lam[3] + lam_y[1] + lam_z[0])
    with pytest.raises(HelmError, match="ESINGULAR"):
        Plan(prob.faces, sigma=bad_sigma)
    plan = Plan(prob.faces, sigma=1.0, precision="bf16_ir")
    f = _gpu(torch, workloads.rhs_normal(1, 1, prob.shape_xyz))
    with pytest.raises(HelmError, match="EINVAL"):
        plan.solve(f, out=f)                     # refinement needs f intact
    plan2 = Plan(prob.faces, sigma=1.0, precision="bf16_ir", max_sweeps=1, ir_tol=1e-14)
    with pytest.raises(HelmError, match="ENOTCONVERGED"):
        plan2.solve(f)
    fn = f.clone()
    fn.view(-1)[5] = float("nan")
    with pytest.raises(HelmError, match="ENONFINITE"):
        Plan(prob.faces, sigma=1.0, precision="fp32_ir").solve(fn)
