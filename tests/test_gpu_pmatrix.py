"""GPU parity of the pressure matrix C (eq. 9) and its preconditioned FGMRES inverse.

The oracle builds C column by column from sparse-LU velocity solves on the cell-by-cell
assembled staggered operators and solves C p = b with the zero-mean gauge by a bordered
dense system.  Iteration counts are only compared between the preconditioned and plain
iteration: the paper's counts (Section 2: 2-4 and 6-8 BiCGstab(2) iterations) are for a 2D
problem and another Krylov method, so they are context, not a pin.
"""
import numpy as np
import pytest

import workloads
from oracle import pressure, solvers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2461_amd import load
    load()
    return t


def _faces(n, betas=(1.5, 1.0, 2.0)):
    return tuple(workloads.stretched_faces(n[d], betas[d]) for d in range(3))


@pytest.mark.parametrize("method", ["tpf", "tpt"])
@pytest.mark.parametrize("n,tau", [((9, 7, 11), 1e2), ((12, 10, 8), 1e-2), ((6, 13, 7), 1.0)])
def test_pmatrix_apply_matches_oracle(torch, n, tau, method):
    from paper_1107_2461_amd import PressureMatrix
    faces = _faces(n)
    pm = PressureMatrix(faces, tau, method=method)
    orc = pressure.PressureMatrix(faces, 1.0 / tau)
    rng = np.random.default_rng(8)
    for _ in range(2):
        p = rng.uniform(-1, 1, (n[2], n[1], n[0]))
        y = pm.apply(torch.from_numpy(p).cuda()).cpu().numpy().ravel()
        ref = orc.matvec(p.ravel())
        assert solvers.rel_err(y, ref) <= 1e-12


@pytest.mark.parametrize("precision,method", [("fp64", "tpf"), ("fp64", "tpt"), ("bf16_ir", "tpf")])
def test_pmatrix_fgmres_matches_dense_oracle(torch, precision, method):
    from paper_1107_2461_amd import PressureMatrix
    n = (10, 8, 12)
    faces = _faces(n)
    tau = 1e2
    b = workloads.remove_weighted_mean(workloads.rhs_uniform(4, 1, n), faces)[0]
    orc = pressure.PressureMatrix(faces, 1.0 / tau)
    ref, mu = orc.solve_dense_gauged(b.ravel())
    assert abs(mu) < 1e-8
    pm = PressureMatrix(faces, tau, precision=precision, method=method)
    p = pm.solve(torch.from_numpy(b).cuda(), tol=1e-11, max_it=300, restart=30).cpu().numpy().ravel()
    info = pm.last_info
    assert info["converged"], info
    # gauge: zero volume-weighted mean, then compare
    pv = solvers.project(p, orc.vol)
    assert solvers.rel_err(pv, ref) <= 1e-8
    assert np.linalg.norm(orc.matvec(p) - b.ravel()) / np.linalg.norm(b) <= 1e-10


def test_pmatrix_preconditioners(torch):
    """Iteration counts of FGMRES on C with no preconditioner (0), the inverse pressure
    Laplacian of Section 2 (1) and I + (1/tau) A_p^{-1} (2): option 1 wins in the Chorin
    regime (1/tau far above the Laplacian's eigenvalues), option 2 never loses to plain GMRES."""
    from paper_1107_2461_amd import PressureMatrix
    n = (16, 14, 18)
    faces = _faces(n)
    b = workloads.remove_weighted_mean(workloads.rhs_uniform(4, 1, n), faces)[0]
    bt = torch.from_numpy(b).cuda()
    counts = {}
    for tau in (1e-6, 1e-2, 1e2):
        pm = PressureMatrix(faces, tau)
        row = {}
        for pc in (0, 1, 2):
            pm.solve(bt, tol=1e-10, max_it=600, restart=60, precondition=pc)
            info = pm.last_info
            row[pc] = info["iterations"] if info["converged"] else 10**6
        counts[tau] = row
    print("FGMRES iterations {tau: {preconditioner: its}}:", counts)
    assert counts[1e-6][1] < counts[1e-6][0]          # Chorin regime: the paper's preconditioner helps
    for tau in counts:
        assert counts[tau][2] <= counts[tau][0]
        assert counts[tau][2] < 10**6
