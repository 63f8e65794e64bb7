"""The pressure matrix C of the Stokes-operator factorization (test infrastructure only).

Eq. 9 (Section 2) defines C = sum_d Grad-to-div products through the inverse
velocity Helmholtz operators.  The paper writes H = Laplacian - I/dt (negative
definite); with the library's positive form H_d = sigma_v I - Laplacian_h on the
d-velocity grid (sigma_v = 1/dt), the paper's C becomes

    C p = - sum_d Div_d H_d^{-1} Grad_d p,

on a MAC grid with no-slip (Dirichlet) velocities and no pressure boundary values.
For small dt, H_d ~ sigma_v I and C ~ dt * (-Div Grad), i.e. dt times the Neumann
pressure Laplacian (the Chorin limit stated at the end of Section 2).

The velocity solves here use sparse LU (or PCG at large sizes) on the cell-by-cell
assembled velocity operators of fv.assemble_3d.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fv, solvers


class PressureMatrix:
    """Action and (small-size) dense form of C for a pressure grid and velocity shift sigma_v."""

    def __init__(self, faces, sigma_v, method="splu"):
        self.faces = tuple(np.asarray(f, dtype=np.float64) for f in faces)
        self.sigma_v = float(sigma_v)
        self.method = method
        self.n = tuple(len(f) - 1 for f in self.faces)
        self.grad = [fv.mac_grad(self.faces, d) for d in range(3)]
        self.div = [fv.mac_div(self.faces, d) for d in range(3)]
        self.H = []
        self.lu = []
        self.spd = []
        for d in range(3):
            H, K3, vol, _ = fv.helmholtz_matrix(self.faces, self.sigma_v, fv.velocity_loc(d))
            self.H.append(H)
            self.spd.append((K3, vol))
            self.lu.append(spla.splu(H.tocsc()) if method == "splu" else None)
        _, self.vol = fv.assemble_3d(self.faces, bc_lo=(fv.NEUMANN,) * 3, bc_hi=(fv.NEUMANN,) * 3)[0:2]

    def velocity_solve(self, d, r):
        if self.lu[d] is not None:
            return self.lu[d].solve(r)
        K3, vol = self.spd[d]
        x, _ = solvers.solve_pcg(K3, vol, self.sigma_v, r, tol=1e-15)
        return x

    def matvec(self, p):
        p = np.asarray(p, dtype=np.float64).ravel()
        out = np.zeros_like(p)
        for d in range(3):
            out -= self.div[d] @ self.velocity_solve(d, self.grad[d] @ p)
        return out

    def dense(self):
        N = int(np.prod(self.n))
        C = np.empty((N, N))
        e = np.zeros(N)
        for j in range(N):
            e[j] = 1.0
            C[:, j] = self.matvec(e)
            e[j] = 0.0
        return C

    def solve_dense_gauged(self, b):
        """Solve C p = b with zero volume-weighted-mean p via the bordered system.

        C annihilates constants and its range is volume-weighted-mean free, so
        [[C, 1], [vol^T, 0]] is nonsingular; for a consistent b the border multiplier is 0.
        """
        C = self.dense()
        N = C.shape[0]
        M = np.zeros((N + 1, N + 1))
        M[:N, :N] = C
        M[:N, N] = 1.0
        M[N, :N] = self.vol
        rhs = np.concatenate([np.asarray(b, dtype=np.float64).ravel(), [0.0]])
        x = np.linalg.solve(M, rhs)
        return x[:N], x[N]


def neumann_laplacian(faces):
    """-Laplacian_h on the cell-centred all-Neumann grid, as diag(1/vol) K3 (sparse)."""
    K3, vol, _ = fv.assemble_3d(faces, bc_lo=(fv.NEUMANN,) * 3, bc_hi=(fv.NEUMANN,) * 3)
    return (sp.diags(1.0 / vol) @ K3).tocsr(), vol
