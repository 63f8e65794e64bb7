"""Pins of the Stokes-system oracle (Section 2, eq. 8) on the CPU.

The monolithic bordered solve of oracle/stokes.py is checked against what fixes it
independently: a closed-form case (a pure pressure-gradient forcing is balanced by the
pressure alone), the three-step factorization of Section 2 computed with the dense
pressure matrix of oracle/pressure.py (itself pinned by its invariants and the Chorin
limit), the continuity rows, and planted mistakes that must fail these pins.
"""
import numpy as np
import pytest

import workloads
from oracle import fv, pressure, solvers, stokes


def _faces():
    return (workloads.stretched_faces(6, 1.5), workloads.stretched_faces(5, 1.0),
            workloads.stretched_faces(7, 2.0))


def _rand_forcing(sysm, seed):
    rng = np.random.default_rng(seed)
    f = [rng.uniform(-1, 1, sysm.shapes[d]) for d in range(3)]
    g = rng.uniform(-1, 1, (sysm.n[2], sysm.n[1], sysm.n[0]))
    return f, g


def test_pure_gradient_forcing_closed_form():
    # f_d = Grad_d q, g = 0  =>  u = 0 and p = q up to the gauge (zero volume-weighted mean)
    faces = _faces()
    sysm = stokes.StokesSystem(faces, 3.0)
    q = np.random.default_rng(11).uniform(-1, 1, sysm.np)
    f = [(sysm.G[d] @ q).reshape(sysm.shapes[d]) for d in range(3)]
    ux, uy, uz, p, c = sysm.solve(f)
    for u in (ux, uy, uz):
        assert np.abs(u).max() < 1e-12
    q0 = solvers.project(q, sysm.vol)
    assert np.abs(p.ravel() - q0).max() < 1e-12 * np.abs(q0).max()
    assert abs(c) < 1e-12


@pytest.mark.parametrize("sigma_v", [1e-2, 1.0, 1e3])
def test_matches_three_step_factorization(sigma_v):
    # Section 2: u^ = H^-1 f; C p = g - Div u^ (C = -sum Div H^-1 Grad); u = u^ - H^-1 Grad p
    faces = _faces()
    sysm = stokes.StokesSystem(faces, sigma_v)
    f, g = _rand_forcing(sysm, 12)
    g = workloads.remove_weighted_mean(g[None], faces)[0]
    pm = pressure.PressureMatrix(faces, sigma_v)
    uh = [pm.velocity_solve(d, f[d].ravel()) for d in range(3)]
    b = g.ravel() - sum(pm.div[d] @ uh[d] for d in range(3))
    p3, mu = pm.solve_dense_gauged(b)
    assert abs(mu) < 1e-9 * np.abs(b).max()
    u3 = [uh[d] - pm.velocity_solve(d, pm.grad[d] @ p3) for d in range(3)]
    ux, uy, uz, p, c = sysm.solve(f, g)
    for d, u in enumerate((ux, uy, uz)):
        assert np.abs(u.ravel() - u3[d]).max() < 1e-10 * np.abs(u3[d]).max()
    assert np.abs(p.ravel() - p3).max() < 1e-10 * np.abs(p3).max()
    assert abs(c) < 1e-12


def test_continuity_and_border_multiplier():
    faces = _faces()
    sysm = stokes.StokesSystem(faces, 0.5)
    f, g = _rand_forcing(sysm, 13)          # g keeps its volume-weighted mean
    ux, uy, uz, p, c = sysm.solve(f, g)
    mom, div = sysm.apply((ux, uy, uz), p)
    for d in range(3):
        assert np.abs(mom[d] - f[d]).max() < 1e-11
    gm = solvers.weighted_mean(g.ravel(), sysm.vol)
    assert abs(c - gm) < 1e-12               # the incompatible part of g is what the border drops
    assert np.abs(div.ravel() - (g.ravel() - gm)).max() < 1e-11
    assert abs(solvers.weighted_mean(p.ravel(), sysm.vol)) < 1e-13


def test_pins_catch_planted_mistakes(monkeypatch):
    faces = _faces()
    orig_grad = fv.mac_grad
    monkeypatch.setattr(fv, "mac_grad", lambda fc, d: -orig_grad(fc, d))   # gradient sign
    sysm = stokes.StokesSystem(faces, 3.0)
    monkeypatch.setattr(fv, "mac_grad", orig_grad)
    q = np.random.default_rng(11).uniform(-1, 1, sysm.np)
    f = [(orig_grad(faces, d) @ q).reshape(sysm.shapes[d]) for d in range(3)]
    p = sysm.solve(f)[3]
    assert np.abs(p.ravel() - solvers.project(q, sysm.vol)).max() > 1e-3

    orig_div = fv.mac_div
    monkeypatch.setattr(fv, "mac_div", lambda fc, d: orig_div(fc, d) * (0.5 if d == 1 else 1.0))  # dropped area
    bad = stokes.StokesSystem(faces, 1.0)
    monkeypatch.setattr(fv, "mac_div", orig_div)
    good = stokes.StokesSystem(faces, 1.0)
    f, g = _rand_forcing(good, 14)
    g = workloads.remove_weighted_mean(g[None], faces)[0]
    ub = bad.solve(f, g)
    _, div = good.apply(ub[:3], ub[3])
    assert np.abs(div - g).max() > 1e-3
