"""One step of the paper's time integration (Section 5, eqs. 37-40) on the MAC grid, for the CPU
oracle (test infrastructure only).

Boussinesq convection in a box (eqs. 34-36), Prandtl number Pr, Grashof number Gr, time step
dt: temperature T and pressure p at cell centres, the velocity component v_d on the interior
d-faces (no-slip walls), T = T_lo at x = 0 and T_hi at x = 1, adiabatic elsewhere.  With
kappa = 1 / (Pr sqrt(Gr)) and nu = 1 / sqrt(Gr), one step is
  (37)  (3/(2 dt) - kappa Lap) T1 = (4 T0 - Tm)/(2 dt) - A_T(v0, T0)           (wall values of T
        enter through the boundary flux of Lap)
  (38)  (3/(2 dt) - nu Lap) vs_d = (4 v0_d - vm_d)/(2 dt) - A_d(v0) - Grad_d p0 + [d = z] T1 at
        the z-faces
  (39)  -Lap dp = (1/dt) Div vs
  (40)  v1_d = vs_d + dt Grad_d dp,   p1 = p0 - dp.
Readings (the paper gives the scheme, not its discretization): Lap is the FV Laplacian of the
oracle (oracle.fv); A_T and A_d are the conservative central advection terms
  A_T = sum_d ((v_d Tbar)_{hi face} - (v_d Tbar)_{lo face}) / w_d   (Tbar: mean of the two cells),
  A_d on the d-velocity control volume [c_{i-1}, c_i]: along d the flux ubar^2 at the cell
  centres (ubar: mean of the cell's two d-faces, wall faces 0) over c_i - c_{i-1}; along e != d
  the flux vbar_e * utilde_d at the e-faces (vbar_e: mean of the e-velocity of the two cells
  beside the d-face; utilde_d: mean of v_d in the two cells beside the e-face; zero on e-walls)
  over the cell width w_e;
and T1 at a z-face is the mean of its two cells.  Eq. 40 as printed adds dp to p; with the
gradient sign of eq. 38 and the correction of eq. 40 the consistent update subtracts it, which
is the reading used.  Arrays are [nz, ny, nx] (x fastest) on their own grids.
"""
from __future__ import annotations

import numpy as np

from . import fv, solvers

D, N = fv.DIRICHLET, fv.NEUMANN
T_BC_LO = (D, N, N)
T_BC_HI = (D, N, N)


def _geom(faces):
    x = [np.asarray(f, dtype=np.float64) for f in faces]
    c = [0.5 * (a[1:] + a[:-1]) for a in x]
    w = [np.diff(a) for a in x]
    return x, c, w


def _pad(v, d):
    """Velocity on all faces along d (wall faces 0): shape with n[d] + 1 entries along d."""
    ax = 2 - d                       # array axis of direction d in [z, y, x] order
    pad = [(0, 0)] * 3
    pad[ax] = (1, 1)
    return np.pad(v, pad)


def _sl(d, a, b):
    s = [slice(None)] * 3
    s[2 - d] = slice(a, b)
    return tuple(s)


def wall_term(faces, t_lo, t_hi):
    """Lap of the Dirichlet wall values of T (x walls) as a cell field: the part of the FV
    Laplacian that the homogeneous operator leaves out."""
    x, c, w = _geom(faces)
    nx, ny, nz = (len(a) - 1 for a in x)
    g = np.zeros((nz, ny, nx))
    g[:, :, 0] += t_lo / ((c[0][0] - x[0][0]) * w[0][0])
    g[:, :, -1] += t_hi / ((x[0][-1] - c[0][-1]) * w[0][-1])
    return g


def advect_T(faces, v, T):
    """A_T(v, T) at cell centres (conservative central form)."""
    _, _, w = _geom(faces)
    out = np.zeros_like(T)
    for d in range(3):
        vf = _pad(v[d], d)                                   # all d-faces
        Tp = np.pad(T, [(1, 1) if ax == 2 - d else (0, 0) for ax in range(3)], mode="edge")
        Tbar = 0.5 * (Tp[_sl(d, 0, -1)] + Tp[_sl(d, 1, None)])   # on all d-faces
        F = vf * Tbar
        shape = [1, 1, 1]
        shape[2 - d] = -1
        out += (F[_sl(d, 1, None)] - F[_sl(d, 0, -1)]) / w[d].reshape(shape)
    return out


def advect_vel(faces, v, d):
    """A_d(v) on the interior d-faces (conservative central form, means as in the module note)."""
    _, c, w = _geom(faces)
    ud = v[d]
    ufull = _pad(ud, d)                                       # d-faces incl. walls
    # along d: flux ubar^2 at the cell centres, over the distance between neighbouring centres
    ubar = 0.5 * (ufull[_sl(d, 0, -1)] + ufull[_sl(d, 1, None)])   # at the cells
    F = ubar * ubar
    shape = [1, 1, 1]
    shape[2 - d] = -1
    out = (F[_sl(d, 1, None)] - F[_sl(d, 0, -1)]) / np.diff(c[d]).reshape(shape)
    for e in range(3):
        if e == d:
            continue
        ve = _pad(v[e], e)                                    # e-velocity on all e-faces (cells along d)
        vbar = 0.5 * (ve[_sl(d, 0, -1)] + ve[_sl(d, 1, None)])    # beside the d-face: cells i-1, i along d
        up = np.pad(ud, [(1, 1) if ax == 2 - e else (0, 0) for ax in range(3)], mode="edge")
        util = 0.5 * (up[_sl(e, 0, -1)] + up[_sl(e, 1, None)])    # v_d on the e-faces
        G = vbar * util                                       # zero on e-walls through vbar
        she = [1, 1, 1]
        she[2 - e] = -1
        out = out + (G[_sl(e, 1, None)] - G[_sl(e, 0, -1)]) / w[e].reshape(she)
    return out


def step(faces, Pr, Gr, dt, T0, Tm, v0, vm, p0, t_lo=0.5, t_hi=-0.5, method="splu"):
    """One step of eqs. 37-40; returns (T1, v1 (three arrays), p1, dp)."""
    kappa = 1.0 / (Pr * np.sqrt(Gr))
    nu = 1.0 / np.sqrt(Gr)
    b = 1.5 / dt                                              # 3 / (2 dt)
    n = [len(f) - 1 for f in faces]
    # (37): temperature, homogeneous operator plus the wall term
    rhs = (4.0 * T0 - Tm) / (2.0 * dt) - advect_T(faces, v0, T0) + kappa * wall_term(faces, t_lo, t_hi)
    T1, _ = solvers.solve_problem(faces, b / kappa, rhs[None] / kappa, bc_lo=T_BC_LO, bc_hi=T_BC_HI,
                                  method=method)
    T1 = T1[0]
    # (38): velocities
    vs = []
    for d in range(3):
        G = (fv.mac_grad(faces, d) @ p0.ravel()).reshape(v0[d].shape)
        rhs = (4.0 * v0[d] - vm[d]) / (2.0 * dt) - advect_vel(faces, v0, d) - G
        if d == 2:
            rhs = rhs + 0.5 * (T1[1:] + T1[:-1])
        sol, _ = solvers.solve_problem(faces, b / nu, rhs[None] / nu, loc=fv.velocity_loc(d), method=method)
        vs.append(sol[0])
    # (39): pressure correction
    div = sum(fv.mac_div(faces, d) @ vs[d].ravel() for d in range(3)).reshape(n[2], n[1], n[0])
    dp, _ = solvers.solve_problem(faces, 0.0, div[None] / dt, bc_lo=(N,) * 3, bc_hi=(N,) * 3, method=method)
    dp = dp[0]
    # (40)
    v1 = [vs[d] + dt * (fv.mac_grad(faces, d) @ dp.ravel()).reshape(vs[d].shape) for d in range(3)]
    return T1, v1, p0 - dp, dp


def divergence(faces, v):
    n = [len(f) - 1 for f in faces]
    return sum(fv.mac_div(faces, d) @ v[d].ravel() for d in range(3)).reshape(n[2], n[1], n[0])
