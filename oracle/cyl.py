"""Finite-volume Helmholtz operator in cylindrical coordinates for the CPU oracle
(test infrastructure only).

Section 6, eq. 41: the Laplacian in (r, theta, z) is
    D_rr u + (1/r^2) D_theta_theta u + D_zz u,   D_rr = (1/r) d/dr (r d/dr).
Discretization (the paper gives the equation, not the scheme; the reading used here is the
cell-centred finite-volume scheme of the Cartesian oracle, written in cylindrical
coordinates): cells [r_i, r_{i+1}] x [t_j, t_{j+1}] x [z_k, z_{k+1}], unknowns at the cell
midpoints (rc_i, tc_j, zc_k), volume (r_{i+1}^2 - r_i^2)/2 * dt_j * dz_k.  The Laplacian of a
cell is (1/volume) * the sum over its faces of face area times the normal derivative:
  * r-face at r_{i+1}: area r_{i+1} dt dz, derivative (u_{i+1} - u_i) / (rc_{i+1} - rc_i);
    a Dirichlet wall at r_0 > 0 or r_n uses the wall value 0 at the wall radius; a wall
    at r_0 = 0 (the axis) has zero area and carries no flux; Neumann walls carry none;
  * theta-face at t_{j+1}: area dr dz, derivative (u_{j+1} - u_j) / (rc_i (tc_{j+1} - tc_j));
    a periodic theta axis couples the last and the first cell across t_n = t_0 + period;
    a walled theta axis (a sector) uses the Dirichlet / Neumann rule of the other walls;
  * z-face: area rc_i dr_i dt_j, derivative (u_{k+1} - u_k) / (zc_{k+1} - zc_k).
The library solves (sigma I - Lap_h) u = f.  After multiplying by the volumes this is the
symmetric system (K3 + sigma Vol) u = Vol f, solved by the same plain solvers as the
Cartesian oracle.

Array layout of grid functions: [..., nr, nz, nt] (theta fastest, r slowest), index
t + nt * (k + nz * i).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fv, solvers

DIRICHLET = fv.DIRICHLET
NEUMANN = fv.NEUMANN


def cell_geometry(r_faces, t_faces, z_faces):
    """Cell midpoints and widths per axis: (rc, dr, tc, dt, zc, dz)."""
    r = np.asarray(r_faces, dtype=np.float64)
    t = np.asarray(t_faces, dtype=np.float64)
    z = np.asarray(z_faces, dtype=np.float64)
    return (0.5 * (r[1:] + r[:-1]), np.diff(r), 0.5 * (t[1:] + t[:-1]), np.diff(t),
            0.5 * (z[1:] + z[:-1]), np.diff(z))


def volumes(r_faces, t_faces, z_faces):
    """Cell volumes (r_{i+1}^2 - r_i^2)/2 * dt_j * dz_k in the [nr, nz, nt] layout, flattened."""
    r = np.asarray(r_faces, dtype=np.float64)
    ring = 0.5 * (r[1:] ** 2 - r[:-1] ** 2)
    dt = np.diff(np.asarray(t_faces, dtype=np.float64))
    dz = np.diff(np.asarray(z_faces, dtype=np.float64))
    return (ring[:, None, None] * dz[None, :, None] * dt[None, None, :]).ravel()


def assemble(r_faces, t_faces, z_faces, bc_r=(DIRICHLET, DIRICHLET), bc_t=None, bc_z=(DIRICHLET, DIRICHLET)):
    """Assemble the cylindrical FV operator cell by cell from face fluxes.

    bc_t None means a periodic theta axis.  Returns (K3, vol, shape) with K3 the symmetric
    sparse conductance matrix (sum over each cell's faces of area / distance couplings, the
    theta distance measured along the arc at the cell's radius) and vol the cell volumes,
    so that -Lap_h = diag(1/vol) K3.  shape = (nr, nz, nt).
    """
    rf = np.asarray(r_faces, dtype=np.float64)
    tf = np.asarray(t_faces, dtype=np.float64)
    zf = np.asarray(z_faces, dtype=np.float64)
    rc, dr, tc, dt, zc, dz = cell_geometry(rf, tf, zf)
    nr, nt, nz = len(rc), len(tc), len(zc)
    N = nr * nz * nt
    ii, kk, jj = np.meshgrid(np.arange(nr), np.arange(nz), np.arange(nt), indexing="ij")
    idx = jj + nt * (kk + nz * ii)
    diag = np.zeros(N)
    rows, cols, vals = [], [], []

    def link(p, q, g):
        np.add.at(diag, p, g)
        np.add.at(diag, q, g)
        rows.extend([p, q])
        cols.extend([q, p])
        vals.extend([-g, -g])

    # radial faces between cells i and i+1: area r_{i+1} dt dz
    sel = ii < nr - 1
    i = ii[sel]
    link(idx[sel], idx[sel] + nt * nz, rf[i + 1] * dt[jj[sel]] * dz[kk[sel]] / (rc[i + 1] - rc[i]))
    # radial walls: the inner wall has area r_0 dt dz (zero on the axis)
    if bc_r[0] == DIRICHLET and rf[0] > 0.0:
        sel = ii == 0
        np.add.at(diag, idx[sel], rf[0] * dt[jj[sel]] * dz[kk[sel]] / (rc[0] - rf[0]))
    if bc_r[1] == DIRICHLET:
        sel = ii == nr - 1
        np.add.at(diag, idx[sel], rf[-1] * dt[jj[sel]] * dz[kk[sel]] / (rf[-1] - rc[-1]))
    # theta faces: area dr dz, arc distance rc_i * (tc_{j+1} - tc_j)
    sel = jj < nt - 1
    j = jj[sel]
    link(idx[sel], idx[sel] + 1, dr[ii[sel]] * dz[kk[sel]] / (rc[ii[sel]] * (tc[j + 1] - tc[j])))
    if bc_t is None:
        # periodic: the last cell's upper face is the first cell's lower face
        dwrap = (tf[-1] - tc[-1]) + (tc[0] - tf[0])
        sel = jj == nt - 1
        link(idx[sel], idx[sel] - (nt - 1), dr[ii[sel]] * dz[kk[sel]] / (rc[ii[sel]] * dwrap))
    else:
        if bc_t[0] == DIRICHLET:
            sel = jj == 0
            np.add.at(diag, idx[sel], dr[ii[sel]] * dz[kk[sel]] / (rc[ii[sel]] * (tc[0] - tf[0])))
        if bc_t[1] == DIRICHLET:
            sel = jj == nt - 1
            np.add.at(diag, idx[sel], dr[ii[sel]] * dz[kk[sel]] / (rc[ii[sel]] * (tf[-1] - tc[-1])))
    # axial faces: area rc dr dt
    sel = kk < nz - 1
    k = kk[sel]
    link(idx[sel], idx[sel] + nt, rc[ii[sel]] * dr[ii[sel]] * dt[jj[sel]] / (zc[k + 1] - zc[k]))
    if bc_z[0] == DIRICHLET:
        sel = kk == 0
        np.add.at(diag, idx[sel], rc[ii[sel]] * dr[ii[sel]] * dt[jj[sel]] / (zc[0] - zf[0]))
    if bc_z[1] == DIRICHLET:
        sel = kk == nz - 1
        np.add.at(diag, idx[sel], rc[ii[sel]] * dr[ii[sel]] * dt[jj[sel]] / (zf[-1] - zc[-1]))
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    K3 = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    K3.sum_duplicates()
    return K3, volumes(rf, tf, zf), (nr, nz, nt)


def is_singular(r_faces, bc_r, bc_t, bc_z):
    """True when the constant is in the null space: no Dirichlet wall with nonzero area."""
    inner_open = bc_r[0] == NEUMANN or float(r_faces[0]) == 0.0
    return (inner_open and bc_r[1] == NEUMANN and (bc_t is None or tuple(bc_t) == (NEUMANN, NEUMANN))
            and tuple(bc_z) == (NEUMANN, NEUMANN))


def solve(r_faces, t_faces, z_faces, sigma, f, bc_r=(DIRICHLET, DIRICHLET), bc_t=None,
          bc_z=(DIRICHLET, DIRICHLET), method="splu", tol=1e-14):
    """Solve (sigma I - Lap_h) u = f for every RHS in f[(nrhs,) nr, nz, nt].

    method "dense", "splu" or "pcg".  The singular Laplace problem (sigma = 0 with no Dirichlet
    wall) is solved in the projected gauge (volume-weighted mean of f removed, u with zero
    volume-weighted mean), as the Cartesian oracle does.
    """
    K3, vol, shape = assemble(r_faces, t_faces, z_faces, bc_r, bc_t, bc_z)
    N = K3.shape[0]
    f = np.asarray(f, dtype=np.float64)
    fr = f.reshape(-1, N)
    singular = sigma == 0.0 and is_singular(r_faces, bc_r, bc_t, bc_z)
    H = (sp.diags(1.0 / vol) @ K3 + sigma * sp.identity(N)).tocsr()
    out = np.empty_like(fr)
    lu = None
    for q in range(fr.shape[0]):
        if singular and method != "pcg":
            out[q] = solvers.project(solvers.solve_neumann_bordered(K3, vol, fr[q]), vol)
        elif method == "dense":
            out[q] = solvers.solve_dense(H, fr[q])
        elif method == "splu":
            if lu is None:
                import scipy.sparse.linalg as spla
                lu = spla.splu(H.tocsc())
            out[q] = lu.solve(fr[q])
        elif method == "pcg":
            out[q], _ = solvers.solve_pcg(K3, vol, sigma, fr[q], tol=tol, neumann=singular)
        else:
            raise ValueError(method)
    return out.reshape(f.shape)


def apply(r_faces, t_faces, z_faces, sigma, u, bc_r=(DIRICHLET, DIRICHLET), bc_t=None,
          bc_z=(DIRICHLET, DIRICHLET)):
    """(sigma I - Lap_h) u with the assembled operator, for every RHS in u[..., nr, nz, nt]."""
    K3, vol, shape = assemble(r_faces, t_faces, z_faces, bc_r, bc_t, bc_z)
    N = K3.shape[0]
    ur = np.asarray(u, dtype=np.float64).reshape(-1, N)
    return np.stack([K3 @ x / vol + sigma * x for x in ur]).reshape(np.shape(u))
