"""GPU parity of the Stokes solve (eq. 8 by the three steps of Section 2, helm_stokes_solve).

The oracle solves the assembled, bordered eq. 8 system by sparse LU.  The GPU result comes
from six velocity Helmholtz solves and FGMRES on the pressure matrix, so its error is the
FGMRES tolerance times the conditioning of C (plus the velocity solves' own error); the
bars below are derived that way: FGMRES to 1e-12 with FP64 solves gives errors near 1e-11
on these grids, and the refined split-BF16 velocity solves (1e-11 each) cap the reachable
FGMRES residual near 1e-11, so those run to 1e-10.
"""
import numpy as np
import pytest

import workloads
from oracle import solvers, stokes

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


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("precision,method,tol,bar", [("fp64", "tpt", 1e-12, 1e-9), ("fp64", "tpf", 1e-12, 1e-9),
                                                      ("bf16x3_ir", "tpf", 1e-10, 1e-7)])
@pytest.mark.parametrize("n,tau,with_g", [((13, 9, 11), 1e2, False), ((12, 10, 14), 1e-1, True)])
def test_stokes_matches_assembled_oracle(torch, precision, method, tol, bar, n, tau, with_g):
    from paper_1107_2461_amd import PressureMatrix
    faces = _faces(n)
    orc = stokes.StokesSystem(faces, 1.0 / tau)
    rng = np.random.default_rng(21)
    f = [rng.uniform(-1, 1, orc.shapes[d]) for d in range(3)]
    g = rng.uniform(-1, 1, (n[2], n[1], n[0])) if with_g else None   # keeps its mean: dropped by both
    ux, uy, uz, p, c = orc.solve(f, g)
    pm = PressureMatrix(faces, tau, precision=precision, method=method)
    assert pm.velocity_shapes() == tuple(orc.shapes)
    out = pm.stokes([torch.from_numpy(x).cuda() for x in f], None if g is None else torch.from_numpy(g).cuda(),
                    tol=tol, max_it=400, restart=40, precondition=2)
    info = pm.last_info
    assert info["converged"], info
    got = [t.cpu().numpy() for t in out]
    for d, ref in enumerate((ux, uy, uz)):
        assert _rel(got[d], ref) <= bar, (d, _rel(got[d], ref))
    assert _rel(got[3], p) <= bar
    assert abs(solvers.weighted_mean(got[3].ravel(), orc.vol)) <= 1e-12 * np.abs(p).max()
    # the rows of eq. 8 on the GPU result
    mom, div = orc.apply(got[:3], got[3])
    scale = max(np.abs(x).max() for x in f)
    for d in range(3):
        assert np.abs(mom[d] - f[d]).max() <= 10 * bar * scale
    gt = np.zeros_like(div) if g is None else g - solvers.weighted_mean(g.ravel(), orc.vol)
    assert np.abs(div - gt).max() <= 10 * bar * max(scale, np.abs(gt).max())


def test_stokes_pure_gradient_forcing(torch):
    """f = Grad q, g = 0: the pressure alone balances the forcing (u = 0, p = q - mean)."""
    from paper_1107_2461_amd import PressureMatrix
    n = (10, 12, 9)
    faces = _faces(n)
    orc = stokes.StokesSystem(faces, 1.0)
    q = np.random.default_rng(22).uniform(-1, 1, orc.np)
    f = [(orc.G[d] @ q).reshape(orc.shapes[d]) for d in range(3)]
    pm = PressureMatrix(faces, 1.0)
    out = pm.stokes([torch.from_numpy(x).cuda() for x in f], tol=1e-12, max_it=200, restart=30)
    assert pm.last_info["converged"], pm.last_info
    scale = max(np.abs(x).max() for x in f)
    for d in range(3):
        assert np.abs(out[d].cpu().numpy()).max() <= 1e-9 * scale
    q0 = solvers.project(q, orc.vol)
    assert _rel(out[3].cpu().numpy().ravel(), q0) <= 1e-9


def test_stokes_rejects_aliasing_and_shapes(torch):
    import ctypes as C
    from paper_1107_2461_amd import PressureMatrix, _lib, load
    n = (6, 5, 7)
    pm = PressureMatrix(_faces(n), 1.0)
    shapes = pm.velocity_shapes()
    f = [torch.zeros(s, dtype=torch.float64, device="cuda") for s in shapes]
    with pytest.raises(ValueError):
        pm.stokes([f[1], f[0], f[2]])
    lib = load()
    nb = C.c_size_t()
    assert lib.helm_stokes_workspace_size(pm._h, 30, C.byref(nb)) == _lib.HELM_OK
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    wsp = C.c_void_p((ws.data_ptr() + 255) // 256 * 256)
    p = torch.empty((n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
    fa = (C.c_void_p * 3)(*[x.data_ptr() for x in f])
    info = _lib.HelmInfo()
    # u aliasing f is refused before any launch
    st = lib.helm_stokes_solve(pm._h, fa, None, fa, C.c_void_p(p.data_ptr()), 1e-10, 10, 30, 2, wsp, None,
                               C.byref(info))
    assert st == _lib.HELM_EINVAL
    assert lib.helm_stokes_workspace_size(pm._h, 0, C.byref(nb)) == _lib.HELM_EINVAL


@pytest.mark.parametrize("precision,method,rel", [("fp64", "tpt", 1e-12), ("bf16x3_ir", "tpf", 1e-9)])
def test_stokes_rows_multi_tile(torch, precision, method, rel):
    """At a size spanning several 16-wide MFMA blocks with ragged tails (pressure 40 x 37 x 45),
    the rows of eq. 8 on the GPU result with the oracle's sparse blocks: the momentum rows as a
    backward error (the velocity solves' accuracy times the size of the terms), the continuity
    rows to the FGMRES tolerance times the size of the divergence terms."""
    from paper_1107_2461_amd import PressureMatrix
    n = (40, 37, 45)
    faces = _faces(n)
    tau, tol = 10.0, 1e-10
    orc = stokes.StokesSystem(faces, 1.0 / tau, factorize=False)
    rng = np.random.default_rng(23)
    f = [rng.uniform(-1, 1, orc.shapes[d]) for d in range(3)]
    pm = PressureMatrix(faces, tau, precision=precision, method=method)
    out = pm.stokes([torch.from_numpy(x).cuda() for x in f], tol=tol, max_it=400, restart=40, precondition=2)
    assert pm.last_info["converged"], pm.last_info
    got = [t.cpu().numpy() for t in out]
    mom, div = orc.apply(got[:3], got[3])
    pmax = np.abs(got[3]).max()
    for d in range(3):
        hn = abs(orc.H[d]).sum(axis=1).max()
        gn = abs(orc.G[d]).sum(axis=1).max()
        size = hn * np.abs(got[d]).max() + gn * pmax + np.abs(f[d]).max()
        assert np.abs(mom[d] - f[d]).max() <= rel * size, (d, np.abs(mom[d] - f[d]).max() / size)
    dsize = max(abs(orc.D[d]).sum(axis=1).max() * np.abs(got[d]).max() for d in range(3))
    assert np.abs(div).max() <= 10 * tol * dsize, np.abs(div).max() / dsize


def test_stokes_minimum_grid(torch):
    """Three pressure cells per axis (two velocity nodes along each velocity's own axis)."""
    from paper_1107_2461_amd import PressureMatrix
    n = (3, 3, 3)
    faces = _faces(n)
    orc = stokes.StokesSystem(faces, 0.5)
    rng = np.random.default_rng(24)
    f = [rng.uniform(-1, 1, orc.shapes[d]) for d in range(3)]
    ux, uy, uz, p, _ = orc.solve(f)
    pm = PressureMatrix(faces, 2.0)
    # unpreconditioned: the velocity solves at two and three unknowns per axis are the paths
    # exercised here (the shortest-axis and Thomas-length tests cover them on their own)
    out = pm.stokes([torch.from_numpy(x).cuda() for x in f], tol=1e-13, max_it=100, restart=20, precondition=0)
    assert pm.last_info["converged"], pm.last_info
    for d, ref in enumerate((ux, uy, uz)):
        assert _rel(out[d].cpu().numpy(), ref) <= 1e-10
    assert _rel(out[3].cpu().numpy(), p) <= 1e-10


def test_stokes_not_converged_reports_and_returns_finite(torch):
    """max_it = 1: the status says so, and u, p come from the best pressure found (finite;
    the velocities still satisfy the momentum rows for that pressure)."""
    import ctypes as C
    from paper_1107_2461_amd import PressureMatrix, _lib, load
    n = (12, 10, 14)
    faces = _faces(n)
    orc = stokes.StokesSystem(faces, 0.01, factorize=False)
    rng = np.random.default_rng(25)
    f = [rng.uniform(-1, 1, orc.shapes[d]) for d in range(3)]
    pm = PressureMatrix(faces, 100.0)
    ft = [torch.from_numpy(x).cuda() for x in f]
    out = pm.stokes(ft, tol=1e-14, max_it=1, restart=5, precondition=0)
    assert not pm.last_info["converged"] and pm.last_info["iterations"] == 1
    # six velocity solves of steps 1 and 3, three for the one action of C (no preconditioner)
    assert pm.last_info["helmholtz_solves"] == 9
    got = [t.cpu().numpy() for t in out]
    assert all(np.isfinite(g).all() for g in got)
    mom, _ = orc.apply(got[:3], got[3])
    for d in range(3):
        size = (abs(orc.H[d]).sum(axis=1).max() * np.abs(got[d]).max()
                + abs(orc.G[d]).sum(axis=1).max() * np.abs(got[3]).max() + np.abs(f[d]).max())
        assert np.abs(mom[d] - f[d]).max() <= 1e-12 * size
    # the C ABI reports the same through its status
    lib = load()
    nb = C.c_size_t()
    assert lib.helm_stokes_workspace_size(pm._h, 5, C.byref(nb)) == _lib.HELM_OK
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    u = [torch.empty_like(x) for x in ft]
    p = torch.empty((n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
    info = _lib.HelmInfo()
    st = lib.helm_stokes_solve(pm._h, (C.c_void_p * 3)(*[x.data_ptr() for x in ft]), None,
                               (C.c_void_p * 3)(*[x.data_ptr() for x in u]), C.c_void_p(p.data_ptr()), 1e-14, 1, 5,
                               0, C.c_void_p((ws.data_ptr() + 255) // 256 * 256), None, C.byref(info))
    torch.cuda.synchronize()
    assert st == _lib.HELM_ENOTCONVERGED and info.converged == 0 and info.iterations == 1 and info.sweeps == 9
