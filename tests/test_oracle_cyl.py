"""Pins of the cylindrical-coordinate oracle (Section 6, eq. 41) against facts fixed by the
geometry and the mathematics (no GPU):
  * hand-computed conductances and volumes on a 2 x 3 x 2 grid with the axis, a periodic
    theta wrap and Dirichlet walls (golden fixture),
  * the exact volume of an annular sector,
  * conservation: with no Dirichlet wall the assembled fluxes sum to zero,
  * the closed-form eigenvalue of a uniform periodic theta axis acting with the 1/r^2 metric,
  * the Cartesian limit of a thin annulus far from the axis,
  * O(h^2) convergence to a continuous solution of eq. 41 (through the axis),
  * three independent solvers on a tiny stretched sector, the Neumann gauge,
  * planted mistakes in the metric and the areas fail a pin.
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import cyl, fv, solvers

GOLD = os.path.join(os.path.dirname(__file__), "golden")
D, N = cyl.DIRICHLET, cyl.NEUMANN


def _idx(shape, i, j, k):
    nr, nz, nt = shape
    return j + nt * (k + nz * i)


def test_hand_fixture():
    g = json.load(open(os.path.join(GOLD, "cyl_2x3x2.json")))
    K3, vol, shape = cyl.assemble(g["r_faces"], g["t_faces"], g["z_faces"], (D, D), None, (D, D))
    K = K3.toarray()
    for e in g["entries"]:
        (i1, j1, k1), (i2, j2, k2) = e["cells"]
        v = K[_idx(shape, i1, j1, k1), _idx(shape, i2, j2, k2)]
        assert abs(v - e["value"]) <= 1e-14 * max(1.0, abs(e["value"])), e["what"]
    for e in g["volumes"]:
        i, j, k = e["cell"]
        assert abs(vol[_idx(shape, i, j, k)] - e["value"]) <= 1e-14, e["what"]
    assert np.allclose(K, K.T, rtol=0, atol=1e-15)


def test_volume_of_annular_sector():
    rf = workloads.stretched_faces(7, 1.5, 0.3, 1.7)
    tf = workloads.stretched_faces(5, 1.0, 0.0, 2.2)
    zf = workloads.stretched_faces(4, 2.0, -1.0, 0.5)
    vol = cyl.volumes(rf, tf, zf)
    assert abs(vol.sum() - 0.5 * (1.7**2 - 0.3**2) * 2.2 * 1.5) <= 1e-14 * vol.sum()


@pytest.mark.parametrize("r0", [0.0, 0.4])
def test_conservation_without_dirichlet_walls(r0):
    rf = workloads.stretched_faces(6, 1.5, r0, 1.0)
    tf = np.linspace(0.0, 2 * np.pi, 9)
    zf = workloads.stretched_faces(5, 1.2)
    K3, vol, _ = cyl.assemble(rf, tf, zf, (N, N), None, (N, N))
    ones = np.ones(K3.shape[0])
    assert np.abs(K3 @ ones).max() <= 1e-13 * abs(K3).max()
    assert cyl.is_singular(rf, (N, N), None, (N, N))
    # a Dirichlet wall with nonzero area breaks the null space; the axis does not
    assert not cyl.is_singular(rf, (N, D), None, (N, N))
    assert cyl.is_singular(workloads.stretched_faces(6, 1.5, 0.0, 1.0), (D, N), None, (N, N))


@pytest.mark.parametrize("m", [1, 2, 5])
def test_periodic_theta_closed_form_eigenvalue(m):
    """On a uniform periodic theta axis of M cells, cos(m t_j) is an eigenvector of the discrete
    second difference with eigenvalue (4 / h^2) sin^2(pi m / M); through the metric of eq. 41
    the operator on a(r) cos(m t) b(z) differs from the operator on a(r) b(z) (m = 0) times
    cos(m t) by exactly lambda_m / rc^2 times the field."""
    M = 12
    h = 2 * np.pi / M
    rf = workloads.stretched_faces(6, 1.5, 0.0, 1.3)
    tf = np.linspace(0.0, 2 * np.pi, M + 1)
    zf = workloads.stretched_faces(5, 1.0, 0.0, 0.8)
    rc, _, tc, _, zc, _ = cyl.cell_geometry(rf, tf, zf)
    rng = np.random.default_rng(1)
    a = rng.uniform(0.5, 1.5, len(rc))
    b = rng.uniform(-1, 1, len(zc))
    cm = np.cos(m * tc)
    u_m = a[:, None, None] * b[None, :, None] * cm[None, None, :]
    u_0 = a[:, None, None] * b[None, :, None] * np.ones_like(tc)[None, None, :]
    sigma = 0.7
    Hm = cyl.apply(rf, tf, zf, sigma, u_m, (D, D), None, (D, D))
    H0 = cyl.apply(rf, tf, zf, sigma, u_0, (D, D), None, (D, D))
    lam = 4 / h**2 * np.sin(np.pi * m / M) ** 2
    expect = H0 * cm[None, None, :] + lam / rc[:, None, None] ** 2 * u_m
    assert np.abs(Hm - expect).max() <= 1e-12 * np.abs(Hm).max()


def test_cartesian_limit_thin_annulus():
    """Far from the axis a thin sector is a box: r in [R, R+1], theta in [0, 1/R] (arc length 1),
    z in [0, 1].  The cylindrical operator tends to the Cartesian one (x along the arc, y = z,
    z = r - R) with a difference of order 1/R."""
    n = (5, 4, 6)   # (theta, z, r) cells
    diffs = []
    for R in (1e2, 1e3):
        tf = workloads.stretched_faces(n[0], 1.5, 0.0, 1.0 / R)
        zf = workloads.stretched_faces(n[1], 1.0)
        rf = workloads.stretched_faces(n[2], 2.0, R, R + 1.0)
        bc_t, bc_z, bc_r = (D, N), (N, D), (D, D)
        K3, vol, _ = cyl.assemble(rf, tf, zf, bc_r, bc_t, bc_z)
        Hc = (K3.multiply(1.0 / vol[:, None])).toarray()
        H, _, _, _ = fv.helmholtz_matrix((tf * R, zf, rf - R), 0.0, bc_lo=(bc_t[0], bc_z[0], bc_r[0]),
                                         bc_hi=(bc_t[1], bc_z[1], bc_r[1]))
        Hx = H.toarray()          # Cartesian index x + nx (y + ny z) = theta + nt (z + nz r): same order
        diffs.append(np.abs(Hc - Hx).max() / np.abs(Hx).max())
    assert diffs[0] < 5e-2 and diffs[1] < 0.2 * diffs[0], diffs


def test_continuous_solution_second_order_through_the_axis():
    """u = (r^2 - r^4) cos(2 t) sin(pi z) on the full cylinder r <= 1 (periodic theta, Dirichlet
    at r = 1 and z = 0, 1): D_rr u + u_tt / r^2 = -12 r^2 cos(2 t) sin(pi z) and u_zz = -pi^2 u."""
    sigma = 1.0
    errs = []
    for n in (8, 16, 32):
        rf = np.linspace(0.0, 1.0, n + 1)
        tf = np.linspace(0.0, 2 * np.pi, n + 1)
        zf = workloads.stretched_faces(n, 1.5)
        rc, _, tc, _, zc, _ = cyl.cell_geometry(rf, tf, zf)
        R, Z, T = np.meshgrid(rc, zc, tc, indexing="ij")
        g = R**2 - R**4
        ue = g * np.cos(2 * T) * np.sin(np.pi * Z)
        f = (sigma * g + 12 * R**2 + np.pi**2 * g) * np.cos(2 * T) * np.sin(np.pi * Z)
        u = cyl.solve(rf, tf, zf, sigma, f[None], (N, D), None, (D, D), method="splu")
        errs.append(np.abs(u[0] - ue).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 1.8, (errs, rates)


def test_three_solvers_agree_tiny_sector():
    rf = workloads.stretched_faces(7, 1.5, 0.2, 1.0)
    tf = workloads.stretched_faces(6, 1.25, 0.0, 1.5)
    zf = workloads.stretched_faces(8, 2.0)
    rng = np.random.default_rng(2)
    f = rng.uniform(-1, 1, (1, 7, 8, 6))
    kw = dict(bc_r=(D, N), bc_t=(N, D), bc_z=(D, N))
    ud = cyl.solve(rf, tf, zf, 0.3, f, method="dense", **kw)
    us = cyl.solve(rf, tf, zf, 0.3, f, method="splu", **kw)
    up = cyl.solve(rf, tf, zf, 0.3, f, method="pcg", tol=1e-15, **kw)
    assert solvers.rel_err(us, ud) < 1e-13 and solvers.rel_err(up, ud) < 1e-12
    r = f - cyl.apply(rf, tf, zf, 0.3, ud, **kw)
    assert np.linalg.norm(r) / np.linalg.norm(f) < 1e-13


def test_neumann_gauge():
    rf = workloads.stretched_faces(6, 1.5, 0.0, 1.0)
    tf = np.linspace(0.0, 2 * np.pi, 8)
    zf = workloads.stretched_faces(5, 1.0)
    rng = np.random.default_rng(3)
    f = rng.uniform(-1, 1, (1, 6, 5, 7))
    kw = dict(bc_r=(N, N), bc_t=None, bc_z=(N, N))
    u1 = cyl.solve(rf, tf, zf, 0.0, f, **kw)
    u2 = cyl.solve(rf, tf, zf, 0.0, f + 2.5, **kw)
    up = cyl.solve(rf, tf, zf, 0.0, f, method="pcg", tol=1e-15, **kw)
    vol = cyl.volumes(rf, tf, zf)
    assert abs(solvers.weighted_mean(u1[0].ravel(), vol)) < 1e-14
    assert solvers.rel_err(u2, u1) < 1e-12 and solvers.rel_err(up, u1) < 1e-11


def test_pins_catch_planted_mistakes(monkeypatch):
    """Radial nodes off the cell midpoints, or theta nodes off theirs (which also moves the
    periodic wrap distance), each fail the hand fixture."""
    g = json.load(open(os.path.join(GOLD, "cyl_2x3x2.json")))

    def fixture_ok():
        K3, vol, shape = cyl.assemble(g["r_faces"], g["t_faces"], g["z_faces"], (D, D), None, (D, D))
        K = K3.toarray()
        return all(abs(K[_idx(shape, *e["cells"][0]), _idx(shape, *e["cells"][1])] - e["value"])
                   <= 1e-12 * max(1.0, abs(e["value"])) for e in g["entries"])

    assert fixture_ok()
    orig = cyl.cell_geometry

    def outer_centres(rf, tf, zf):               # radial nodes moved a tenth of a cell outward
        rc, dr, tc, dt, zc, dz = orig(rf, tf, zf)
        return rc + 0.1 * dr, dr, tc, dt, zc, dz
    monkeypatch.setattr(cyl, "cell_geometry", outer_centres)
    assert not fixture_ok()
    monkeypatch.setattr(cyl, "cell_geometry", orig)

    def shifted_theta(rf, tf, zf):               # theta centres off by a quarter cell
        rc, dr, tc, dt, zc, dz = orig(rf, tf, zf)
        return rc, dr, tc + 0.25 * dt, dt, zc, dz
    monkeypatch.setattr(cyl, "cell_geometry", shifted_theta)
    assert not fixture_ok()
    monkeypatch.setattr(cyl, "cell_geometry", orig)
    assert fixture_ok()
