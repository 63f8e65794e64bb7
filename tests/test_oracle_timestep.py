"""Pins of the time-step oracle (Section 5, eqs. 37-40; oracle/timestep.py), no GPU:
  * the corrected velocity is discretely divergence-free (what eqs. 39-40 construct);
  * a fluid at rest with the linear conduction profile between the heated walls keeps that
    temperature exactly (a steady solution of eq. 37);
  * on a uniform grid the conservative advection terms reproduce the exact derivative of a
    linear field in the interior, and conserve T (the fluxes telescope);
  * the same step with dense LU, sparse LU and PCG inner solves agrees;
  * planted mistakes (a dropped dt in the correction, the wrong sign of the wall term) fail a pin.
"""
import numpy as np
import pytest

import workloads
from oracle import fv, timestep

D, N = fv.DIRICHLET, fv.NEUMANN


def _faces(n, beta=1.5):
    return tuple(workloads.stretched_faces(n[d], beta) for d in range(3))


def _state(faces, seed, amp=0.1):
    return workloads.timestep_state(seed, tuple(len(f) - 1 for f in faces), amp)


def test_corrected_velocity_is_divergence_free():
    faces = _faces((9, 8, 10))
    T0, Tm, v0, vm, p0 = _state(faces, 1)
    T1, v1, p1, dp = timestep.step(faces, 0.71, 1e5, 1e-2, T0, Tm, v0, vm, p0)
    div = timestep.divergence(faces, v1)
    scale = max(np.abs(v).max() for v in v1) / min(np.diff(f).min() for f in faces)
    assert np.abs(div).max() <= 1e-11 * scale


def test_conduction_state_is_steady():
    faces = _faces((10, 7, 8))
    n = [len(f) - 1 for f in faces]
    cx = workloads.centres(faces[0])
    Ts = np.broadcast_to((0.5 - cx)[None, None, :], (n[2], n[1], n[0])).copy()   # T_lo = 0.5, T_hi = -0.5
    zero = [np.zeros(tuple(n[2 - a] - (1 if 2 - a == d else 0) for a in range(3))) for d in range(3)]
    T1, v1, p1, dp = timestep.step(faces, 0.71, 1e5, 1e-2, Ts, Ts, zero, zero, np.zeros_like(Ts))
    assert np.abs(T1 - Ts).max() <= 1e-13


def test_advection_exact_for_linear_fields_on_uniform_grid():
    n = (12, 10, 9)
    faces = tuple(np.linspace(0.0, L, k + 1) for k, L in zip(n, (1.0, 0.8, 1.3)))
    cx, cy, cz = (workloads.centres(f) for f in faces)
    U, a = 0.7, 2.5
    shp = [(n[2], n[1], n[0] - 1), (n[2], n[1] - 1, n[0]), (n[2] - 1, n[1], n[0])]
    v = [np.full(shp[0], U), np.zeros(shp[1]), np.zeros(shp[2])]
    T = np.broadcast_to(a * cx[None, None, :], (n[2], n[1], n[0]))
    A = timestep.advect_T(faces, v, T)
    assert np.abs(A[:, :, 1:-1] - U * a).max() <= 1e-12          # U dT/dx away from the x walls
    vol = np.diff(faces[2])[:, None, None] * np.diff(faces[1])[None, :, None] * np.diff(faces[0])[None, None, :]
    rng = np.random.default_rng(2)
    vr = [rng.standard_normal(s) for s in shp]
    Tr = rng.standard_normal((n[2], n[1], n[0]))
    assert abs((timestep.advect_T(faces, vr, Tr) * vol).sum()) <= 1e-12 * np.abs(Tr).max() * 10
    # u = U + b y in the interior rows: (v . grad) u = 0 there (v = w = 0, du/dx = 0)
    uy = np.broadcast_to((U + 0.3 * cy)[None, :, None], shp[0]).copy()
    Au = timestep.advect_vel(faces, [uy, v[1], v[2]], 0)
    assert np.abs(Au[:, 1:-1, 1:-1]).max() <= 1e-12


def test_inner_solvers_agree():
    faces = _faces((6, 5, 7))
    st = _state(faces, 3)
    a = timestep.step(faces, 0.71, 1e5, 1e-2, *st, method="dense")
    b = timestep.step(faces, 0.71, 1e5, 1e-2, *st, method="splu")
    c = timestep.step(faces, 0.71, 1e5, 1e-2, *st, method="pcg")
    for x, y, z in ((a[0], b[0], c[0]), (a[2], b[2], c[2])):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max() and np.abs(x - z).max() <= 1e-10 * np.abs(x).max()
    for d in range(3):
        assert np.abs(a[1][d] - b[1][d]).max() <= 1e-12 * np.abs(a[1][d]).max()


def test_pins_catch_planted_mistakes(monkeypatch):
    faces = _faces((9, 8, 10))
    T0, Tm, v0, vm, p0 = _state(faces, 4)
    orig_grad = fv.mac_grad
    calls = {"n": 0}

    def grad_missing_dt_in_correction(f, d):     # the correction's gradient scaled wrongly
        calls["n"] += 1
        G = orig_grad(f, d)
        return G if calls["n"] <= 3 else 0.5 * G
    monkeypatch.setattr(fv, "mac_grad", grad_missing_dt_in_correction)
    _, v1, _, _ = timestep.step(faces, 0.71, 1e5, 1e-2, T0, Tm, v0, vm, p0)
    monkeypatch.setattr(fv, "mac_grad", orig_grad)
    assert np.abs(timestep.divergence(faces, v1)).max() > 1e-6

    orig_wall = timestep.wall_term
    monkeypatch.setattr(timestep, "wall_term", lambda f, lo, hi: -orig_wall(f, lo, hi))
    n = [len(f) - 1 for f in faces]
    Ts = np.broadcast_to((0.5 - workloads.centres(faces[0]))[None, None, :], (n[2], n[1], n[0])).copy()
    zero = [np.zeros_like(v) for v in v0]
    T1, _, _, _ = timestep.step(faces, 0.71, 1e5, 1e-2, Ts, Ts, zero, zero, np.zeros_like(Ts))
    assert np.abs(T1 - Ts).max() > 1e-3
