"""Pins of the CPU oracle against facts fixed by the paper and by mathematics (no GPU).

Each pin is independent of the oracle's own code path:
  * a hand-computed 1D operator on a non-uniform 3-cell grid (golden fixture),
  * closed-form eigenpairs of the uniform-grid operators (DST-I/II/IV, DCT-II/IV),
  * the uniform-grid 3D solve by scipy.fft sine/cosine transforms (a library routine),
  * the Kronecker-sum structure of eq. 29 (3D assembly vs 1D operators),
  * three independent linear solvers (dense LU, sparse LU, PCG) on tiny inputs,
  * O(h^2) convergence to a continuous trigonometric solution,
  * Neumann gauge invariants (eq. 28 discussion) and the MAC identities of eqs. 4/9.
"""
import json
import os

import numpy as np
import pytest
import scipy.fft as sfft
import scipy.sparse as sp

import workloads
from oracle import fv, pressure, solvers

GOLD = os.path.join(os.path.dirname(__file__), "golden")
D, N = fv.DIRICHLET, fv.NEUMANN


def _uniform_faces(n, L):
    return np.linspace(0.0, L, n + 1)


# ------------------------------------------------------------------ 1D operators

def test_operator_1d_hand_fixture():
    g = json.load(open(os.path.join(GOLD, "op1d_3cell.json")))
    faces = np.array(g["faces"])
    cases = {
        "cell_dirichlet": (fv.CELL, D, D),
        "cell_neumann": (fv.CELL, N, N),
        "cell_dirichlet_lo_neumann_hi": (fv.CELL, D, N),
        "face_dirichlet": (fv.FACE, D, D),
        "face_neumann": (fv.FACE, N, N),
        "face_dirichlet_lo_neumann_hi": (fv.FACE, D, N),
    }
    for key, (loc, lo, hi) in cases.items():
        K, vol = fv.operator_1d(faces, loc, lo, hi)
        np.testing.assert_allclose(K, np.array(g[key]["K"]), rtol=1e-14, atol=1e-14, err_msg=key)
        np.testing.assert_allclose(vol, np.array(g[key]["vol"]), rtol=1e-14, err_msg=key)


@pytest.mark.parametrize("bc", ["DD", "NN", "DN", "ND"])
def test_uniform_eigs_closed_form_cell(bc):
    n, L = 16, 0.7
    h = L / n
    lo = D if bc[0] == "D" else N
    hi = D if bc[1] == "D" else N
    K, vol = fv.operator_1d(_uniform_faces(n, L), fv.CELL, lo, hi)
    A = K / vol[:, None]
    k = np.arange(n)
    if bc == "DD":
        lam = 4 / h**2 * np.sin(np.pi * (k + 1) / (2 * n)) ** 2
        vec = lambda a: np.sin(np.pi * (a + 1) * (2 * k + 1) / (2 * n))
    elif bc == "NN":
        lam = 4 / h**2 * np.sin(np.pi * k / (2 * n)) ** 2
        vec = lambda a: np.cos(np.pi * a * (2 * k + 1) / (2 * n))
    elif bc == "DN":
        lam = 4 / h**2 * np.sin(np.pi * (2 * k + 1) / (4 * n)) ** 2
        vec = lambda a: np.sin(np.pi * (2 * a + 1) * (2 * k + 1) / (4 * n))
    else:
        lam = 4 / h**2 * np.sin(np.pi * (2 * k + 1) / (4 * n)) ** 2
        vec = lambda a: np.cos(np.pi * (2 * a + 1) * (2 * k + 1) / (4 * n))
    for a in range(n):
        v = vec(a)
        np.testing.assert_allclose(A @ v, lam[a] * v, rtol=0, atol=1e-10 * lam.max())
    np.testing.assert_allclose(np.sort(np.linalg.eigvals(A).real), np.sort(lam), rtol=1e-12, atol=1e-9)


def test_uniform_eigs_closed_form_face():
    n, L = 12, 1.3
    h = L / n
    K, vol = fv.operator_1d(_uniform_faces(n, L), fv.FACE, D, D)
    A = K / vol[:, None]
    i = np.arange(1, n)
    for a in range(1, n):
        v = np.sin(np.pi * a * i / n)
        lam = 4 / h**2 * np.sin(np.pi * a / (2 * n)) ** 2
        np.testing.assert_allclose(A @ v, lam * v, atol=1e-10 * 4 / h**2)


@pytest.mark.parametrize("bc", ["NN", "DN", "ND"])
def test_uniform_eigs_closed_form_face_neumann(bc):
    """Face-located nodes with a Neumann wall: on a uniform grid the m = n - 1 nodes have
    control volumes h and link conductances 1/h, a Dirichlet wall adds 1/h (wall value at
    distance h) and a Neumann wall nothing, so A = (1/h^2) tridiag(-1, 2, -1) with the end
    diagonals 1 (Neumann) -- the DCT-II matrix for NN, a DST-VII-type one for DN/ND."""
    n, L = 13, 0.9
    h = L / n
    m = n - 1
    lo = D if bc[0] == "D" else N
    hi = D if bc[1] == "D" else N
    K, vol = fv.operator_1d(_uniform_faces(n, L), fv.FACE, lo, hi)
    np.testing.assert_allclose(vol, np.full(m, h), rtol=1e-13)
    A = K / vol[:, None]
    i = np.arange(m)
    lam = []
    for a in range(m):
        if bc == "NN":
            v = np.cos(np.pi * a * (i + 0.5) / m)
            la = 4 / h**2 * np.sin(np.pi * a / (2 * m)) ** 2
        elif bc == "DN":
            v = np.sin(np.pi * (2 * a + 1) * (i + 1) / (2 * m + 1))
            la = 4 / h**2 * np.sin(np.pi * (2 * a + 1) / (2 * (2 * m + 1))) ** 2
        else:
            v = np.sin(np.pi * (2 * a + 1) * (m - i) / (2 * m + 1))
            la = 4 / h**2 * np.sin(np.pi * (2 * a + 1) / (2 * (2 * m + 1))) ** 2
        np.testing.assert_allclose(A @ v, la * v, rtol=0, atol=1e-10 * 4 / h**2)
        lam.append(la)
    np.testing.assert_allclose(np.sort(np.linalg.eigvals(A).real), np.sort(lam), rtol=1e-12, atol=1e-9)


# ------------------------------------------------------------------ 3D assembly

def _kron_sum(faces, loc, lo, hi, sigma):
    mats = []
    for d in range(3):
        K, vol = fv.operator_1d(faces[d], loc[d], lo[d], hi[d])
        mats.append(sp.csr_matrix(K / vol[:, None]))
    I = [sp.identity(m.shape[0]) for m in mats]
    Ax, Ay, Az = mats
    # x fastest: index = i + nx (j + ny k)  =>  kron(z, kron(y, x))
    H = (sp.kron(I[2], sp.kron(I[1], Ax)) + sp.kron(I[2], sp.kron(Ay, I[0]))
         + sp.kron(Az, sp.kron(I[1], I[0])))
    return H + sigma * sp.identity(H.shape[0])


@pytest.mark.parametrize("loc", [(fv.CELL,) * 3, fv.velocity_loc(0), fv.velocity_loc(1), fv.velocity_loc(2)])
def test_kronecker_identity(loc):
    faces = (workloads.stretched_faces(7, 1.5), workloads.stretched_faces(5, 2.0, 0, 2.0),
             workloads.stretched_faces(6, 1.0, 0, 0.5))
    lo, hi = (D, N, D), (N, D, N)
    sigma = 3.7
    H, _, _, _ = fv.helmholtz_matrix(faces, sigma, loc, lo, hi)
    Hk = _kron_sum(faces, loc, lo, hi, sigma)
    diff = abs(H - Hk).max()
    assert diff <= 1e-12 * abs(Hk).max(), diff


def _transform_solve(f, h, sigma, kinds):
    """Uniform-grid solve with scipy.fft transforms; kinds[d] = (transform, type, eig-function)."""
    g = f
    lam = 0.0
    for axis_arr, (tr, typ, eigf), hh in zip((2, 1, 0), kinds, h):
        n = f.shape[axis_arr]
        g = tr(g, type=typ, axis=axis_arr, norm="ortho")
        shape = [1, 1, 1]
        shape[axis_arr] = n
        lam = lam + eigf(np.arange(n), n, hh).reshape(shape)
    den = lam + sigma
    return g, den


def _dst2(g, type, axis, norm):
    return sfft.dst(g, type=type, axis=axis, norm=norm)


def test_uniform_dirichlet_solve_matches_dst():
    n = (10, 8, 6)
    L = (1.0, 2.0, 0.5)
    faces = tuple(_uniform_faces(n[d], L[d]) for d in range(3))
    h = [L[d] / n[d] for d in range(3)]
    sigma = 2.5
    rng = np.random.default_rng(0)
    f = rng.uniform(-1, 1, (n[2], n[1], n[0]))
    u, _ = solvers.solve_problem(faces, sigma, f[None], method="dense")
    eig = lambda k, m, hh: 4 / hh**2 * np.sin(np.pi * (k + 1) / (2 * m)) ** 2
    g = sfft.dstn(f, type=2, norm="ortho")
    lam = (eig(np.arange(n[0]), n[0], h[0])[None, None, :] + eig(np.arange(n[1]), n[1], h[1])[None, :, None]
           + eig(np.arange(n[2]), n[2], h[2])[:, None, None])
    ref = sfft.idstn(g / (lam + sigma), type=2, norm="ortho")
    assert solvers.rel_err(u[0], ref) < 1e-13


def test_uniform_mixed_bc_solve_matches_transforms():
    """x: Dirichlet-Neumann (DST-IV), y: Neumann-Neumann (DCT-II), z: Neumann-Dirichlet (DCT-IV)."""
    n = (9, 7, 8)
    L = (1.0, 0.6, 1.7)
    faces = tuple(_uniform_faces(n[d], L[d]) for d in range(3))
    h = [L[d] / n[d] for d in range(3)]
    sigma = 0.9
    rng = np.random.default_rng(1)
    f = rng.uniform(-1, 1, (n[2], n[1], n[0]))
    u, _ = solvers.solve_problem(faces, sigma, f[None], bc_lo=(D, N, N), bc_hi=(N, N, D), method="dense")
    g = sfft.dst(f, type=4, axis=2, norm="ortho")
    g = sfft.dct(g, type=2, axis=1, norm="ortho")
    g = sfft.dct(g, type=4, axis=0, norm="ortho")
    e4 = lambda m, hh: 4 / hh**2 * np.sin(np.pi * (2 * np.arange(m) + 1) / (4 * m)) ** 2
    e2 = lambda m, hh: 4 / hh**2 * np.sin(np.pi * np.arange(m) / (2 * m)) ** 2
    lam = e4(n[0], h[0])[None, None, :] + e2(n[1], h[1])[None, :, None] + e4(n[2], h[2])[:, None, None]
    g = g / (lam + sigma)
    g = sfft.idct(g, type=4, axis=0, norm="ortho")
    g = sfft.idct(g, type=2, axis=1, norm="ortho")
    ref = sfft.idst(g, type=4, axis=2, norm="ortho")
    assert solvers.rel_err(u[0], ref) < 1e-13


def test_uniform_neumann_laplace_matches_dct():
    n = (8, 10, 6)
    L = (1.0, 1.5, 0.8)
    faces = tuple(_uniform_faces(n[d], L[d]) for d in range(3))
    h = [L[d] / n[d] for d in range(3)]
    rng = np.random.default_rng(2)
    f = rng.uniform(-1, 1, (n[2], n[1], n[0]))
    u, _ = solvers.solve_problem(faces, 0.0, f[None], bc_lo=(N,) * 3, bc_hi=(N,) * 3)
    g = sfft.dctn(f, type=2, norm="ortho")
    e2 = lambda m, hh: 4 / hh**2 * np.sin(np.pi * np.arange(m) / (2 * m)) ** 2
    lam = e2(n[0], h[0])[None, None, :] + e2(n[1], h[1])[None, :, None] + e2(n[2], h[2])[:, None, None]
    lam[0, 0, 0] = 1.0
    g = g / lam
    g[0, 0, 0] = 0.0             # projection: the zero mode of f is removed, u has zero mean
    ref = sfft.idctn(g, type=2, norm="ortho")
    assert solvers.rel_err(u[0], ref) < 1e-12


def test_uniform_face_located_matches_dst1():
    n = (9, 6, 7)
    L = (1.0, 1.0, 2.0)
    faces = tuple(_uniform_faces(n[d], L[d]) for d in range(3))
    h = [L[d] / n[d] for d in range(3)]
    loc = fv.velocity_loc(0)
    sigma = 4.0
    rng = np.random.default_rng(3)
    f = rng.uniform(-1, 1, (n[2], n[1], n[0] - 1))
    u, _ = solvers.solve_problem(faces, sigma, f[None], loc=loc, method="dense")
    g = sfft.dst(f, type=1, axis=2, norm="ortho")
    g = sfft.dst(g, type=2, axis=1, norm="ortho")
    g = sfft.dst(g, type=2, axis=0, norm="ortho")
    e1 = 4 / h[0]**2 * np.sin(np.pi * np.arange(1, n[0]) / (2 * n[0])) ** 2
    e2 = lambda m, hh: 4 / hh**2 * np.sin(np.pi * (np.arange(m) + 1) / (2 * m)) ** 2
    lam = e1[None, None, :] + e2(n[1], h[1])[None, :, None] + e2(n[2], h[2])[:, None, None]
    g = g / (lam + sigma)
    g = sfft.idst(g, type=2, axis=0, norm="ortho")
    g = sfft.idst(g, type=2, axis=1, norm="ortho")
    ref = sfft.idst(g, type=1, axis=2, norm="ortho")
    assert solvers.rel_err(u[0], ref) < 1e-13


def test_uniform_face_located_neumann_matches_dct2():
    """x face-located with Neumann walls (DCT-II of length n - 1), y cell-centred Dirichlet
    (DST-II), z cell-centred Dirichlet-Neumann (DST-IV), against scipy.fft transforms."""
    n = (9, 6, 7)
    L = (1.0, 1.0, 2.0)
    faces = tuple(_uniform_faces(n[d], L[d]) for d in range(3))
    h = [L[d] / n[d] for d in range(3)]
    loc = fv.velocity_loc(0)
    sigma = 0.7
    rng = np.random.default_rng(13)
    f = rng.uniform(-1, 1, (n[2], n[1], n[0] - 1))
    u, _ = solvers.solve_problem(faces, sigma, f[None], loc=loc, bc_lo=(N, D, D), bc_hi=(N, D, N),
                                 method="dense")
    g = sfft.dct(f, type=2, axis=2, norm="ortho")
    g = sfft.dst(g, type=2, axis=1, norm="ortho")
    g = sfft.dst(g, type=4, axis=0, norm="ortho")
    m = n[0] - 1
    ex = 4 / h[0]**2 * np.sin(np.pi * np.arange(m) / (2 * m)) ** 2
    ey = 4 / h[1]**2 * np.sin(np.pi * (np.arange(n[1]) + 1) / (2 * n[1])) ** 2
    ez = 4 / h[2]**2 * np.sin(np.pi * (2 * np.arange(n[2]) + 1) / (4 * n[2])) ** 2
    lam = ex[None, None, :] + ey[None, :, None] + ez[:, None, None]
    g = g / (lam + sigma)
    g = sfft.idst(g, type=4, axis=0, norm="ortho")
    g = sfft.idst(g, type=2, axis=1, norm="ortho")
    ref = sfft.idct(g, type=2, axis=2, norm="ortho")
    assert solvers.rel_err(u[0], ref) < 1e-13


# ------------------------------------------------------------------ solvers

@pytest.mark.parametrize("bcs", [((D, D, D), (D, D, D)), ((D, N, N), (N, D, N))])
def test_three_solvers_agree_tiny(bcs):
    faces = (workloads.stretched_faces(10, 1.5), workloads.stretched_faces(11, 2.0),
             workloads.stretched_faces(12, 1.0))
    sigma = 0.3
    rng = np.random.default_rng(4)
    f = rng.uniform(-1, 1, (1, 12, 11, 10))
    ud, _ = solvers.solve_problem(faces, sigma, f, bc_lo=bcs[0], bc_hi=bcs[1], method="dense")
    us, _ = solvers.solve_problem(faces, sigma, f, bc_lo=bcs[0], bc_hi=bcs[1], method="splu")
    up, info = solvers.solve_problem(faces, sigma, f, bc_lo=bcs[0], bc_hi=bcs[1], method="pcg", tol=1e-15)
    assert solvers.rel_err(us, ud) < 1e-13
    assert solvers.rel_err(up, ud) < 1e-12
    assert info[0]["true_rel_residual"] < 1e-14


def test_operator_residual_of_solution():
    p, f = workloads.workload_small_dirichlet()
    f = f[:, :12, :12, :12].copy()
    faces = tuple(fc[:13] for fc in p.faces)
    u, _ = solvers.solve_problem(faces, p.sigma, f, method="dense")
    r = f - solvers.apply_operator(faces, p.sigma, u)
    assert np.linalg.norm(r) / np.linalg.norm(f) < 1e-13


@pytest.mark.parametrize("beta", [0.0, 1.5])
def test_continuous_solution_second_order(beta):
    """O(h^2) convergence to u = sin(pi x) sin(2 pi y) sin(3 pi z), Dirichlet, on [0,1]^3."""
    sigma = 1.0
    errs = []
    for n in (12, 24, 48):
        p = workloads.box_problem(n, beta, sigma)
        cx, cy, cz = (workloads.centres(f) for f in p.faces)
        ue = (np.sin(3 * np.pi * cz)[:, None, None] * np.sin(2 * np.pi * cy)[None, :, None]
              * np.sin(np.pi * cx)[None, None, :])
        f = (sigma + 14 * np.pi**2) * ue
        u, _ = solvers.solve_problem(p.faces, sigma, f[None], method="pcg", tol=1e-12)
        errs.append(np.abs(u[0] - ue).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    # pre-asymptotic on the coarsest stretched grid; the finest pair must be second order
    assert rates[0] > 1.5 and rates[-1] > 1.85, (errs, rates)


def test_neumann_gauge_and_invariance():
    faces = (workloads.stretched_faces(9, 1.5), workloads.stretched_faces(8, 1.0),
             workloads.stretched_faces(7, 2.0))
    rng = np.random.default_rng(5)
    f = rng.uniform(-1, 1, (1, 7, 8, 9))
    nb = dict(bc_lo=(N,) * 3, bc_hi=(N,) * 3)
    u1, _ = solvers.solve_problem(faces, 0.0, f, **nb)
    u2, _ = solvers.solve_problem(faces, 0.0, f + 3.25, **nb)
    up, info = solvers.solve_problem(faces, 0.0, f, method="pcg", tol=1e-15, **nb)
    K3, vol, _ = fv.assemble_3d(faces, bc_lo=(N,) * 3, bc_hi=(N,) * 3)
    assert abs(solvers.weighted_mean(u1[0].ravel(), vol)) < 1e-14
    assert solvers.rel_err(u2, u1) < 1e-12
    assert solvers.rel_err(up, u1) < 1e-11
    # -L_h u equals the projected f
    fp = solvers.project(f[0].ravel(), vol)
    r = fp - (K3 @ u1[0].ravel()) / vol
    assert np.linalg.norm(r) / np.linalg.norm(fp) < 1e-12


# ------------------------------------------------------------------ MAC / pressure matrix

def _mac_faces():
    return (workloads.stretched_faces(6, 1.5), workloads.stretched_faces(5, 1.0),
            workloads.stretched_faces(7, 2.0))


def test_mac_div_grad_is_neumann_laplacian():
    faces = _mac_faces()
    L = sum(fv.mac_div(faces, d) @ fv.mac_grad(faces, d) for d in range(3))
    Ap, vol = pressure.neumann_laplacian(faces)
    assert abs(L + Ap).max() < 1e-12 * abs(Ap).max()


def test_pressure_matrix_invariants_and_chorin_limit():
    faces = _mac_faces()
    Ap, vol = pressure.neumann_laplacian(faces)
    n = int(np.prod([len(f) - 1 for f in faces]))
    C = pressure.PressureMatrix(faces, 1e-2).dense()
    assert np.abs(C @ np.ones(n)).max() < 1e-10 * np.abs(C).max()
    assert np.abs(vol @ C).max() < 1e-10 * np.abs(C).max() * vol.max()
    # Chorin limit (end of Section 2): dt -> 0, C / dt -> -Div Grad = A_p
    errs = []
    for sigma in (1e5, 1e7):
        Cs = pressure.PressureMatrix(faces, sigma).dense()
        errs.append(np.abs(sigma * Cs - Ap.toarray()).max() / abs(Ap).max())
    assert errs[1] < errs[0] * 2e-2 and errs[1] < 1e-3, errs


def test_pressure_matrix_gauged_solve():
    faces = _mac_faces()
    pm = pressure.PressureMatrix(faces, 1e-2)
    rng = np.random.default_rng(6)
    b = workloads.remove_weighted_mean(rng.uniform(-1, 1, (1, 7, 5, 6)), faces)[0].ravel()
    p, mu = pm.solve_dense_gauged(b)
    assert abs(mu) < 1e-10
    assert np.linalg.norm(pm.matvec(p) - b) / np.linalg.norm(b) < 1e-11
    assert abs(solvers.weighted_mean(p, pm.vol)) < 1e-13


# ------------------------------------------------------------------ planted mistakes

def test_pins_catch_planted_mistakes(monkeypatch):
    """A plausible error in the oracle (wrong wall distance, dropped area, sign) fails a pin."""
    n = (6, 5, 4)
    L = (1.0, 2.0, 0.5)
    faces = tuple(_uniform_faces(n[d], L[d]) for d in range(3))
    h = [L[d] / n[d] for d in range(3)]
    rng = np.random.default_rng(7)
    f = rng.uniform(-1, 1, (n[2], n[1], n[0]))
    eig = lambda m, hh: 4 / hh**2 * np.sin(np.pi * (np.arange(m) + 1) / (2 * m)) ** 2
    lam = eig(n[0], h[0])[None, None, :] + eig(n[1], h[1])[None, :, None] + eig(n[2], h[2])[:, None, None]
    sigma = 1.5
    ref = sfft.idstn(sfft.dstn(f, type=2, norm="ortho") / (lam + sigma), type=2, norm="ortho")

    def err():
        u, _ = solvers.solve_problem(faces, sigma, f[None], method="dense")
        return solvers.rel_err(u[0], ref)

    assert err() < 1e-13
    orig_nodes = fv.axis_nodes

    def wall_full_cell(faces_, loc=fv.CELL):          # Dirichlet value at distance w instead of w/2
        pos, cv, dl, dh = orig_nodes(faces_, loc)
        return pos, cv, 2 * dl, 2 * dh
    monkeypatch.setattr(fv, "axis_nodes", wall_full_cell)
    assert err() > 1e-3
    monkeypatch.setattr(fv, "axis_nodes", orig_nodes)

    def swapped_cv(faces_, loc=fv.CELL):             # control volume taken from the wrong axis size
        pos, cv, dl, dh = orig_nodes(faces_, loc)
        return pos, np.full_like(cv, 0.25), dl, dh
    monkeypatch.setattr(fv, "axis_nodes", swapped_cv)
    assert err() > 1e-3
    monkeypatch.setattr(fv, "axis_nodes", orig_nodes)

    orig_h = fv.helmholtz_matrix

    def wrong_sign(faces_, sigma_, *a, **k):
        return orig_h(faces_, -sigma_, *a, **k)
    monkeypatch.setattr(fv, "helmholtz_matrix", wrong_sign)
    assert err() > 1e-3


def test_oracle_floor_recorded():
    """The mutual difference of two independent FP64 oracles (tests/golden/oracle_floor.json,
    written by make_oracle_samples.py --floor) lies under every FP64 parity tolerance (1e-12)
    for each full-size configuration, so those tolerances test the solver, not the oracle."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_floor.json")
    data = json.load(open(path))
    for name in ("c1", "c2_tau0.001", "c2_tau1", "c2_tau100", "c3", "c4_pressure"):
        assert name in data, name
        for row in data[name]["rhs"]:
            assert row["rel_inf"] <= 1e-12, (name, row)
