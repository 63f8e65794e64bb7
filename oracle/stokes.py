"""The Stokes system of Section 2 solved as one assembled matrix (test infrastructure only).

Eq. 8 couples the three staggered velocity components and the pressure on a MAC grid.
The paper writes the momentum rows with H = Laplacian - I/dt and the right-hand sides
R_d; with the library's positive Helmholtz form H_d = sigma_v I - Laplacian_h on the
d-velocity grid (sigma_v = 1/dt), multiplying those rows by -1 gives

    H_d u_d + Grad_d p = f_d          (d = x, y, z;  f_d = -R_d)
    sum_d Div_d u_d    = g            (g = 0 in the paper)

with no-slip (zero Dirichlet) velocities on every wall and a pressure gradient that
uses no pressure boundary value.  The pressure is fixed only up to a constant, and the
divergence of any wall-bounded velocity has zero volume-weighted mean, so the oracle
borders the matrix: one extra unknown (a constant added to the continuity rows, which
absorbs the incompatible part of g) and one extra row (zero volume-weighted mean of p).
For a compatible g the extra unknown is zero.

This is the definition written out: the blocks come from the cell-by-cell assembled
operators of fv.py and the bordered matrix is factorised by sparse LU.  It does not use
the three-step factorization of eqs. 2 and 8; the tests check the two against each other.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fv


class StokesSystem:
    """Assembled, bordered Stokes matrix of eq. 8 for a pressure grid and shift sigma_v.

    factorize=False keeps only the blocks (for apply() at sizes where the sparse LU of the
    bordered matrix would be too large)."""

    def __init__(self, faces, sigma_v, factorize=True):
        self.faces = tuple(np.asarray(f, dtype=np.float64) for f in faces)
        self.sigma_v = float(sigma_v)
        self.n = tuple(len(f) - 1 for f in self.faces)          # pressure cells (nx, ny, nz)
        self.np = int(np.prod(self.n))
        self.shapes = []                                          # velocity grids, (nz, ny, nx) order
        self.H, self.G, self.D = [], [], []
        for d in range(3):
            H, _, _, _ = fv.helmholtz_matrix(self.faces, self.sigma_v, fv.velocity_loc(d))
            self.H.append(H.tocsr())
            self.G.append(fv.mac_grad(self.faces, d))
            self.D.append(fv.mac_div(self.faces, d))
            nv = list(self.n)
            nv[d] -= 1
            self.shapes.append((nv[2], nv[1], nv[0]))
        self.nv = [H.shape[0] for H in self.H]
        _, self.vol, _ = fv.assemble_3d(self.faces, bc_lo=(fv.NEUMANN,) * 3, bc_hi=(fv.NEUMANN,) * 3)
        Z = [[None] * 4 for _ in range(4)]
        for d in range(3):
            Z[d][d] = self.H[d]
            Z[d][3] = self.G[d]
            Z[3][d] = self.D[d]
        Z[3][3] = sp.csr_matrix((self.np, self.np))
        self.S = sp.bmat(Z, format="csr")                         # eq. 8 in the library's signs
        self._lu = None
        if not factorize:
            return
        nt = self.S.shape[0]
        ones_p = np.zeros(nt)
        ones_p[nt - self.np:] = 1.0                               # constant in the continuity rows
        vol_p = np.zeros(nt)
        vol_p[nt - self.np:] = self.vol                           # gauge: sum vol * p = 0
        B = sp.bmat([[self.S, sp.csr_matrix(ones_p[:, None])],
                     [sp.csr_matrix(vol_p[None, :]), None]], format="csc")
        self._lu = spla.splu(B)

    def solve(self, f, g=None):
        """(u_x, u_y, u_z, p, c): velocities on their grids (nz, ny, nx order), p on the cells,
        and the border multiplier c (the volume-weighted mean of g that was dropped)."""
        rhs = [np.asarray(f[d], dtype=np.float64).ravel() for d in range(3)]
        rhs.append(np.zeros(self.np) if g is None else np.asarray(g, dtype=np.float64).ravel())
        x = self._lu.solve(np.concatenate(rhs + [np.zeros(1)]))
        out, o = [], 0
        for d in range(3):
            out.append(x[o:o + self.nv[d]].reshape(self.shapes[d]))
            o += self.nv[d]
        p = x[o:o + self.np].reshape(self.n[2], self.n[1], self.n[0])
        return out[0], out[1], out[2], p, float(x[-1])

    def apply(self, u, p):
        """(H_d u_d + Grad_d p for d, sum_d Div_d u_d): the rows of eq. 8 in the library's signs."""
        pv = np.asarray(p, dtype=np.float64).ravel()
        mom = [(self.H[d] @ np.asarray(u[d]).ravel() + self.G[d] @ pv).reshape(self.shapes[d]) for d in range(3)]
        div = sum(self.D[d] @ np.asarray(u[d]).ravel() for d in range(3))
        return mom, div.reshape(self.n[2], self.n[1], self.n[0])
