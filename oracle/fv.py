"""Finite-volume geometry and operators for the CPU oracle (test infrastructure only).

Discretization (the paper cites its finite-volume scheme without stating it; the
reading used throughout is written out here, Section 3 eq. 23 and Section 5.1):

* Cell-centred unknowns: node i sits at the cell centre c_i, its control volume is
  the cell [x_i, x_{i+1}] of width w_i.  Between two nodes the face flux is
  (u_{i+1} - u_i) / (c_{i+1} - c_i).  At a Dirichlet wall the flux uses the wall
  value 0 at distance c_0 - x_0 (resp. x_n - c_{n-1}); at a Neumann wall it is 0.
* Face-located unknowns (a staggered velocity in its own direction): nodes at the
  interior faces x_1..x_{n-1}, control volume [c_{i-1}, c_i]; a Dirichlet wall
  value 0 sits on the wall face, at distance x_1 - x_0 (resp. x_n - x_{n-1}); at a
  Neumann wall the outer end of the first (last) control volume, the cell centre
  c_0 (c_{n-1}), carries no flux.
* The FV Laplacian is (1/vol) * sum over the control volume's faces of
  area * flux; the library solves (sigma I - Laplacian_h) u = f.

Lexicographic order is x fastest: index = i + nx * (j + ny * k).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

DIRICHLET = 0
NEUMANN = 1
CELL = 0
FACE = 1


def axis_nodes(faces, loc=CELL):
    """Node positions, control-volume widths and wall distances along one axis.

    Returns (pos, cv, d_lo, d_hi): pos[m] node coordinates, cv[m] control-volume
    widths, d_lo/d_hi the distance from the first/last node to the point where a
    Dirichlet wall value is imposed.
    """
    x = np.asarray(faces, dtype=np.float64)
    c = 0.5 * (x[1:] + x[:-1])
    if loc == CELL:
        pos = c
        cv = x[1:] - x[:-1]
        d_lo = c[0] - x[0]
        d_hi = x[-1] - c[-1]
    elif loc == FACE:
        pos = x[1:-1]
        cv = c[1:] - c[:-1]
        d_lo = x[1] - x[0]
        d_hi = x[-1] - x[-2]
    else:
        raise ValueError("loc")
    return pos, cv, d_lo, d_hi


def operator_1d(faces, loc=CELL, bc_lo=DIRICHLET, bc_hi=DIRICHLET):
    """Dense 1D matrices (K, vol) with A = diag(1/vol) K = minus the FV second derivative.

    K is the symmetric conductance matrix: each link between consecutive nodes with
    distance d adds 1/d to both diagonals and -1/d to both off-diagonals; a Dirichlet
    wall adds 1/d_wall to its node's diagonal.  This is the paper's D_xx up to sign
    (eq. 23): D_xx = -diag(1/vol) K.
    """
    pos, cv, d_lo, d_hi = axis_nodes(faces, loc)
    m = len(pos)
    K = np.zeros((m, m))
    for i in range(m - 1):
        g = 1.0 / (pos[i + 1] - pos[i])
        K[i, i] += g
        K[i + 1, i + 1] += g
        K[i, i + 1] -= g
        K[i + 1, i] -= g
    if bc_lo == DIRICHLET:
        K[0, 0] += 1.0 / d_lo
    if bc_hi == DIRICHLET:
        K[m - 1, m - 1] += 1.0 / d_hi
    return K, cv.copy()


def assemble_3d(faces, loc=(CELL,) * 3, bc_lo=(DIRICHLET,) * 3, bc_hi=(DIRICHLET,) * 3):
    """Assemble the 3D FV operator cell by cell from face fluxes.

    Returns (K3, vol, shape) where K3 is the symmetric sparse conductance matrix
    (sum over control-volume faces of area / distance couplings) and vol the
    control-volume volumes, so that -Laplacian_h = diag(1/vol) K3.  The assembly
    walks the 3D links of each direction directly (it does not use Kronecker
    products), so that the Kronecker-sum structure of eq. 29 is a property to test.
    """
    axes = [axis_nodes(faces[d], loc[d]) for d in range(3)]
    n = [len(a[0]) for a in axes]
    nx, ny, nz = n
    N = nx * ny * nz
    cv = [a[1] for a in axes]
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = ii + nx * (jj + ny * kk)
    vol = (cv[2][kk] * cv[1][jj] * cv[0][ii]).ravel()

    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    coord = (ii, jj, kk)
    for d in range(3):
        pos, _, d_lo, d_hi = axes[d]
        # face area of a d-directed flux through the control volume at (i, j, k)
        others = [e for e in range(3) if e != d]
        area = cv[others[0]][coord[others[0]]] * cv[others[1]][coord[others[1]]]
        c_d = coord[d]
        # interior links between node c and c+1 along d
        sel = c_d < n[d] - 1
        p = idx[sel]
        step = (1, nx, nx * ny)[d]
        q = p + step
        g = area[sel] / (pos[c_d[sel] + 1] - pos[c_d[sel]])
        np.add.at(diag, p, g)
        np.add.at(diag, q, g)
        rows += [p, q]
        cols += [q, p]
        vals += [-g, -g]
        # walls
        if bc_lo[d] == DIRICHLET:
            sel = c_d == 0
            np.add.at(diag, idx[sel], area[sel] / d_lo)
        if bc_hi[d] == DIRICHLET:
            sel = c_d == n[d] - 1
            np.add.at(diag, idx[sel], area[sel] / d_hi)
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    K3 = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(N, N))
    K3.sum_duplicates()
    return K3, vol, (nx, ny, nz)


def helmholtz_matrix(faces, sigma, loc=(CELL,) * 3, bc_lo=(DIRICHLET,) * 3, bc_hi=(DIRICHLET,) * 3):
    """H = sigma I - Laplacian_h = sigma I + diag(1/vol) K3, as a sparse CSR matrix."""
    K3, vol, shape = assemble_3d(faces, loc, bc_lo, bc_hi)
    H = sp.diags(1.0 / vol) @ K3 + sigma * sp.identity(K3.shape[0])
    return H.tocsr(), K3, vol, shape


# ---------------------------------------------------------------------------------
# Staggered (MAC) first-derivative operators for the pressure matrix (eqs. 4, 9, 30-31).
# Pressure at cell centres (nx, ny, nz); the d-velocity at the interior d-faces.
# ---------------------------------------------------------------------------------

def _shape_with(n, d, m):
    s = list(n)
    s[d] = m
    return s


def mac_grad(faces, d):
    """Pressure gradient along d at interior d-faces: (p_i - p_{i-1}) / (c_i - c_{i-1}).

    It uses no pressure boundary value (the paper's condition (ii) in Section 2).
    Maps the pressure grid to the d-velocity grid (one fewer node along d).
    """
    n = [len(f) - 1 for f in faces]
    nv = _shape_with(n, d, n[d] - 1)
    c = 0.5 * (np.asarray(faces[d])[1:] + np.asarray(faces[d])[:-1])
    kk, jj, ii = np.meshgrid(np.arange(nv[2]), np.arange(nv[1]), np.arange(nv[0]), indexing="ij")
    coord = [ii, jj, kk]
    row = (ii + nv[0] * (jj + nv[1] * kk)).ravel()
    f = coord[d].ravel() + 1                # face index 1..n-1 separating cells f-1 and f
    cp = [ii.ravel(), jj.ravel(), kk.ravel()]
    hi = cp.copy(); hi[d] = f
    lo = cp.copy(); lo[d] = f - 1
    col_hi = hi[0] + n[0] * (hi[1] + n[1] * hi[2])
    col_lo = lo[0] + n[0] * (lo[1] + n[1] * lo[2])
    inv = 1.0 / (c[f] - c[f - 1])
    G = sp.csr_matrix((np.concatenate([inv, -inv]),
                       (np.concatenate([row, row]), np.concatenate([col_hi, col_lo]))),
                      shape=(int(np.prod(nv)), int(np.prod(n))))
    return G


def mac_div(faces, d):
    """d-part of the divergence at cell centres: (v_{i+1/2} - v_{i-1/2}) / w_i, wall values 0."""
    n = [len(f) - 1 for f in faces]
    nv = _shape_with(n, d, n[d] - 1)
    w = np.diff(np.asarray(faces[d], dtype=np.float64))
    kk, jj, ii = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    cp = [ii.ravel(), jj.ravel(), kk.ravel()]
    row = cp[0] + n[0] * (cp[1] + n[1] * cp[2])
    cell = cp[d]
    rows, cols, vals = [], [], []
    # face above the cell (interior face index cell+1 -> velocity node index cell)
    sel = cell < n[d] - 1
    v = [c[sel] for c in cp]
    v[d] = cell[sel]
    rows.append(row[sel]); cols.append(v[0] + nv[0] * (v[1] + nv[1] * v[2])); vals.append(1.0 / w[cell[sel]])
    # face below the cell (interior face index cell -> velocity node index cell-1)
    sel = cell > 0
    v = [c[sel] for c in cp]
    v[d] = cell[sel] - 1
    rows.append(row[sel]); cols.append(v[0] + nv[0] * (v[1] + nv[1] * v[2])); vals.append(-1.0 / w[cell[sel]])
    D = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(int(np.prod(n)), int(np.prod(nv))))
    return D


def velocity_loc(d):
    loc = [CELL, CELL, CELL]
    loc[d] = FACE
    return tuple(loc)
