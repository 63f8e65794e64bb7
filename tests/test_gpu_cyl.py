"""GPU parity of the cylindrical-coordinate solve (Section 6, eqs. 41-44) through the C ABI
against the CPU FP64 oracle (oracle/cyl.py, assembled cell by cell from face fluxes):
full cylinders through the axis with a periodic theta axis (uniform and stretched),
annular sectors with walls, the singular all-Neumann Laplacian (projected), per-RHS
shifts, ragged sizes; the FP64 operator helm_apply against the oracle's operator.
Tolerances: FP64 solve <= 1e-12 (relative 2-norm per RHS), operator <= 1e-13.
"""
import numpy as np
import pytest

import workloads
from oracle import cyl, solvers

pytestmark = pytest.mark.gpu
D, N = cyl.DIRICHLET, cyl.NEUMANN


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2461_amd import load
    load()
    return t


def _faces(kind, n, beta, lo, hi):
    if kind == "uniform":
        return np.linspace(lo, hi, n + 1)
    return workloads.stretched_faces(n, beta, lo, hi)


# (name, r faces, theta faces, z faces, periodic, bc_r, bc_t, bc_z, sigma per RHS)
CASES = [
    ("cylinder_periodic_uniform", _faces("s", 24, 1.5, 0.0, 1.0), _faces("uniform", 32, 0, 0.0, 2 * np.pi),
     _faces("s", 20, 1.5, 0.0, 2.0), True, (N, D), None, (D, D), [1.0, 50.0]),
    ("annulus_sector_walls", _faces("s", 19, 2.0, 0.4, 1.3), _faces("s", 17, 1.25, 0.0, 2.0),
     _faces("s", 23, 1.0, -1.0, 1.0), False, (D, N), (N, D), (N, D), [0.3]),
    ("cylinder_periodic_stretched_theta", _faces("s", 21, 1.0, 0.0, 0.8), _faces("s", 27, 1.5, 0.0, 2 * np.pi),
     _faces("s", 18, 2.0, 0.0, 1.0), True, (N, D), None, (D, N), [5.0, 0.01, 200.0]),
    ("annulus_periodic_ragged", _faces("s", 37, 1.5, 0.5, 2.0), _faces("uniform", 19, 0, 0.0, 2 * np.pi),
     _faces("s", 23, 1.5, 0.0, 1.0), True, (D, D), None, (N, N), [0.7]),
]


def _plan(case, sigma0):
    from paper_1107_2461_amd import CylPlan
    _, rf, tf, zf, per, bc_r, bc_t, bc_z, _ = case
    bt = bc_t if bc_t is not None else (N, N)
    return CylPlan((rf, tf, zf), (bc_r[0], bt[0], bc_z[0]), (bc_r[1], bt[1], bc_z[1]), sigma0, theta_periodic=per)


def _shape(case):
    _, rf, tf, zf = case[:4]
    return len(rf) - 1, len(zf) - 1, len(tf) - 1


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_cyl_solve_matches_oracle(torch, case):
    name, rf, tf, zf, per, bc_r, bc_t, bc_z, sig = case
    nrhs = len(sig)
    seed = 300 + [c[0] for c in CASES].index(name)
    f = workloads.rhs_uniform(seed, nrhs, _shape(case)[::-1])   # (nrhs, n_r, n_z, n_theta)
    plan = _plan(case, sig[0])
    assert plan.shape_rtz == (len(rf) - 1, len(tf) - 1, len(zf) - 1)
    u = plan.solve(torch.from_numpy(f).to("cuda"), sigma=sig)
    torch.cuda.synchronize()
    un = u.cpu().numpy()
    worst = 0.0
    for r in range(nrhs):
        ref = cyl.solve(rf, tf, zf, sig[r], f[r:r + 1], bc_r, bc_t, bc_z, method="splu")
        worst = max(worst, solvers.rel_err(un[r], ref[0]))
    print(name, "relative error vs oracle", worst)
    assert worst <= 1e-12


def test_cyl_neumann_laplace_projected(torch):
    """No Dirichlet wall, sigma = 0: the projected solution (zero volume-weighted mean) of the
    oracle, for both null-mode options up to a constant."""
    from paper_1107_2461_amd import CylPlan, NULL_PAPER_EQ28
    rf = workloads.stretched_faces(20, 1.5, 0.0, 1.0)
    tf = np.linspace(0.0, 2 * np.pi, 25)
    zf = workloads.stretched_faces(16, 1.5)
    f = workloads.rhs_uniform(7, 2, (24, 16, 20))
    ref = cyl.solve(rf, tf, zf, 0.0, f, (N, N), None, (N, N), method="splu")
    vol = cyl.volumes(rf, tf, zf)
    for mode in (0, NULL_PAPER_EQ28):
        plan = CylPlan((rf, tf, zf), (N, N, N), (N, N, N), 0.0, theta_periodic=True, null_mode=mode)
        u = plan.solve(torch.from_numpy(f).to("cuda"))
        torch.cuda.synchronize()
        un = u.cpu().numpy()
        for r in range(2):
            ur = un[r].ravel()
            if mode != 0:
                ur = solvers.project(ur, vol)
            else:
                assert abs(solvers.weighted_mean(ur, vol)) <= 1e-12 * np.abs(ur).max()
            assert solvers.rel_err(ur, ref[r].ravel()) <= 1e-12


@pytest.mark.parametrize("case", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_cyl_apply_matches_oracle_operator(torch, case):
    name, rf, tf, zf, per, bc_r, bc_t, bc_z, sig = case
    u = workloads.rhs_uniform(11, 2, _shape(case)[::-1])
    plan = _plan(case, sig[0])
    hu = plan.apply(torch.from_numpy(u).to("cuda"), sigma=[sig[0], 3.0]).cpu().numpy()
    ref = np.stack([cyl.apply(rf, tf, zf, s, u[r:r + 1], bc_r, bc_t, bc_z)[0] for r, s in enumerate([sig[0], 3.0])])
    assert np.abs(hu - ref).max() <= 1e-13 * np.abs(ref).max()


def test_cyl_noalloc_matches_solve(torch):
    case = CASES[0]
    sig = case[-1]
    plan = _plan(case, sig[0])
    f = torch.from_numpy(workloads.rhs_uniform(13, 2, _shape(case)[::-1])).to("cuda")
    a = plan.solve(f, sigma=sig)
    b = plan.solve_noalloc(f, sigma=sig)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_cyl_refusals(torch):
    from paper_1107_2461_amd import CylPlan, HelmError
    rf, tf, zf = np.linspace(0, 1, 5), np.linspace(0, 2 * np.pi, 7), np.linspace(0, 1, 4)
    with pytest.raises(HelmError, match="EINVAL"):
        CylPlan((rf, tf, zf), sigma=-1.0)                                  # negative shift
    with pytest.raises(HelmError, match="EINVAL"):
        CylPlan((rf - 0.5, tf, zf), sigma=1.0)                             # negative radius
    with pytest.raises(HelmError, match="EINVAL"):
        CylPlan((rf, np.linspace(0, 1, 3), zf), sigma=1.0)                 # periodic with two cells
    plan = CylPlan((rf, tf, zf), sigma=1.0)
    with pytest.raises(HelmError, match="EINVAL"):
        plan.solve(torch.zeros((1, 4, 3, 6), dtype=torch.float64, device="cuda"), sigma=[-2.0])
