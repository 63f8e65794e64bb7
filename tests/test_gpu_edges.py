"""GPU edge cases of the solve path against the CPU FP64 oracle: the longest axis the plans
take (512 unknowns), the shortest ones (2 cells; a face-located axis with 2 unknowns), z lines
of every length class for the two-ended Thomas solve, the largest batch (64 right-hand sides,
each with its own shift), and the bounds that are refused.
Tolerances as in test_gpu_parity.py: FP64 <= 1e-12, refined <= 1e-10.
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


def _run(torch, prob, f, sigma=None, **kw):
    from paper_1107_2461_amd import Plan
    plan = Plan(prob.faces, prob.bc_lo, prob.bc_hi, prob.sigma, loc=prob.loc, **kw)
    u = plan.solve(_gpu(torch, f), sigma=sigma)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def _oracle(prob, f, sigma):
    out = np.empty_like(f)
    for r in range(f.shape[0]):
        out[r], _ = solvers.solve_problem(prob.faces, sigma[r], f[r:r + 1], prob.loc, prob.bc_lo, prob.bc_hi,
                                          method="splu")
    return out


def _err(u, ref):
    return max(solvers.rel_err(u[r], ref[r]) for r in range(ref.shape[0]))


@pytest.mark.parametrize("axis", [0, 2])
def test_longest_axis_512(torch, axis):
    n = [5, 4, 3]
    n[axis] = 512
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(D, N, D), bc_hi=(N, D, D), sigma=0.3)
    f = workloads.rhs_uniform(31 + axis, 2, prob.shape_xyz)
    ref = _oracle(prob, f, [0.3, 0.3])
    assert _err(_run(torch, prob, f), ref) <= 1e-12
    assert _err(_run(torch, prob, f, method="tpt"), ref) <= 1e-12
    assert _err(_run(torch, prob, f, precision="bf16x3_ir"), ref) <= 1e-10


@pytest.mark.parametrize("n", [(256, 6, 5), (5, 6, 256), (7, 256, 3)])
def test_long_axis_few_rows_split_bf16(torch, n):
    # a 256-long axis with few rows to transform: the split-BF16 launcher shrinks its tiles to
    # 16 rows so the launch still spreads over the chip (one GPU's slab in a sharded solve)
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(D, N, D), bc_hi=(D, D, N), sigma=0.2)
    f = workloads.rhs_uniform(71, 3, prob.shape_xyz)
    sig = [0.2, 5.0, 0.01]
    ref = _oracle(prob, f, sig)
    assert _err(_run(torch, prob, f, sigma=sig, precision="bf16x3_ir"), ref) <= 1e-10
    assert _err(_run(torch, prob, f, sigma=sig, precision="bf16x3"), ref) <= 1e-5


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3_ir", 1e-10), ("fp32_ir", 1e-10)])
def test_shortest_axes(torch, precision, tol):
    # two cells per axis, and a face-located axis with two interior unknowns (n = 3)
    for n, loc in (((2, 2, 2), (fv.CELL,) * 3), ((3, 2, 4), fv.velocity_loc(0))):
        faces = tuple(workloads.stretched_faces(n[d], 1.25) for d in range(3))
        prob = workloads.Problem(faces=faces, bc_lo=(D, D, N), bc_hi=(D, D, D), loc=loc, sigma=1.0)
        f = workloads.rhs_uniform(41, 3, prob.shape_xyz)
        ref = _oracle(prob, f, [1.0] * 3)
        assert _err(_run(torch, prob, f, precision=precision), ref) <= tol, (n, precision)


@pytest.mark.parametrize("nz,loc_z", [(2, fv.CELL), (3, fv.CELL), (3, fv.FACE), (33, fv.CELL), (34, fv.CELL),
                                       (65, fv.CELL)])
def test_tpt_z_lengths(torch, nz, loc_z):
    # the z lines split at the middle row into a part eliminated from each end: two unknowns
    # (one side empty), odd and even lengths, and lengths one past a 16-step segment
    n = (7, 5, nz)
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(D, N, D), bc_hi=(D, D, N), loc=(fv.CELL, fv.CELL, loc_z),
                             sigma=0.5)
    sig = [0.5, 1e-3, 40.0]
    f = workloads.rhs_uniform(61 + nz, 3, prob.shape_xyz)
    ref = _oracle(prob, f, sig)
    assert _err(_run(torch, prob, f, sigma=sig, method="tpt"), ref) <= 1e-12


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3_ir", 1e-10)])
def test_64_rhs_each_with_its_shift(torch, precision, tol):
    # the largest batch; shifts span five decades so every RHS has a different denominator,
    # and the split-BF16 tiles straddle RHS boundaries (P = 10 x 9 per z plane)
    n = (10, 9, 8)
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(D, D, D), bc_hi=(N, D, D), sigma=1.0)
    f = workloads.rhs_uniform(51, 64, prob.shape_xyz)
    sig = list(np.logspace(-2, 3, 64))
    ref = _oracle(prob, f, sig)
    assert _err(_run(torch, prob, f, sigma=sig, precision=precision), ref) <= tol


def test_refused_bounds(torch):
    from paper_1107_2461_amd import HelmError, Plan
    faces = tuple(workloads.stretched_faces(k, 1.0) for k in (8, 8, 513))
    with pytest.raises(HelmError, match="EINVAL"):
        Plan(faces, sigma=1.0)                                   # an axis longer than 512
    faces = tuple(workloads.stretched_faces(k, 1.0) for k in (8, 8, 1))
    with pytest.raises(HelmError, match="EINVAL"):
        Plan(faces, sigma=1.0)                                   # fewer than two cells
    faces = tuple(workloads.stretched_faces(k, 1.0) for k in (6, 5, 4))
    plan = Plan(faces, sigma=1.0)
    with pytest.raises(HelmError, match="EINVAL"):
        plan.solve(torch.zeros((65, 4, 5, 6), dtype=torch.float64, device="cuda"))   # more than 64 RHS


@pytest.mark.parametrize("precision,method,tol", [("fp64", "tpf", 1e-12), ("fp64", "tpt", 1e-12),
                                                  ("bf16x3_ir", "tpf", 1e-10)])
def test_face_located_neumann_axes(torch, precision, method, tol):
    # face-located unknowns next to a Neumann wall (the oracle's reading, pinned by the hand
    # fixture and the uniform-grid DCT-II closed form): x face-located with Neumann at both
    # ends, z face-located with Dirichlet below and Neumann above (the Thomas axis)
    n = (21, 18, 23)
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(N, D, D), bc_hi=(N, D, N), loc=(fv.FACE, fv.CELL, fv.FACE),
                             sigma=0.8)
    f = workloads.rhs_uniform(81, 2, prob.shape_xyz)
    sig = [0.8, 25.0]
    ref = _oracle(prob, f, sig)
    assert _err(_run(torch, prob, f, sigma=sig, precision=precision, method=method), ref) <= tol


@pytest.mark.parametrize("n,nrhs", [((256, 16, 16), 64), ((256, 32, 16), 64)])
def test_split_bf16_taller_tiles_few_rows(torch, n, nrhs):
    # a 256-long x axis with 16384 (resp. 32768) rows in all: the split-BF16 x products run with
    # tiles of 32 (resp. 64) rows per workgroup, the largest height that still gives 512
    # workgroups; every right-hand side against the oracle
    faces = tuple(workloads.stretched_faces(n[d], 1.5) for d in range(3))
    prob = workloads.Problem(faces=faces, bc_lo=(D, N, D), bc_hi=(D, D, N), sigma=0.2)
    f = workloads.rhs_uniform(72 + n[1], nrhs, prob.shape_xyz)
    ref, _ = solvers.solve_problem(prob.faces, prob.sigma, f, prob.loc, prob.bc_lo, prob.bc_hi, method="splu")
    assert _err(_run(torch, prob, f, precision="bf16x3_ir"), ref) <= 1e-10
