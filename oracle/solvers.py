"""Plain FP64 CPU solvers for the assembled FV system (test infrastructure only).

The system (sigma I - Laplacian_h) u = f is, after multiplying by the control
volumes, the symmetric positive (semi)definite system (K3 + sigma Vol) u = Vol f
with K3 the conductance matrix of fv.assemble_3d.  Solvers:

  solve_dense     numpy dense LU (brute force, <= 12^3 unknowns)
  solve_splu      scipy sparse LU (<= 32^3)
  solve_pcg       Jacobi-preconditioned conjugate gradients on the SPD form, any size

The all-Neumann Laplace problem (sigma = 0, every wall Neumann) is singular: its
null space is the constant.  Following the paper's Neumann discussion (Section 3,
eq. 28) and the projection reading, the right-hand side is projected onto the
range (its volume-weighted mean removed) and the solution is gauge-fixed to zero
volume-weighted mean.
"""
from __future__ import annotations

import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fv


def is_all_neumann(bc_lo, bc_hi):
    return all(b == fv.NEUMANN for b in bc_lo) and all(b == fv.NEUMANN for b in bc_hi)


def weighted_mean(x, vol):
    return float((x * vol).sum() / vol.sum())


def project(x, vol):
    """Remove the volume-weighted mean (solvability projection / gauge fix)."""
    return x - weighted_mean(x, vol)


def solve_dense(H, f):
    """Dense LU solve of H u = f (brute force for tiny grids)."""
    return np.linalg.solve(H.toarray(), f)


def solve_splu(H, f):
    return spla.splu(H.tocsc()).solve(f)


def solve_neumann_bordered(K3, vol, f):
    """All-Neumann Laplace by the bordered system [[K3, vol], [vol^T, 0]] (sparse LU).

    The border enforces the zero-volume-weighted-mean gauge; the RHS is projected first.
    """
    N = K3.shape[0]
    fp = project(f, vol)
    b = np.concatenate([vol * fp, [0.0]])
    v = sp.csr_matrix(vol.reshape(-1, 1))
    M = sp.bmat([[K3, v], [v.T, None]]).tocsc()
    x = spla.splu(M).solve(b)
    return x[:N]


def solve_pcg(K3, vol, sigma, f, tol=1e-14, maxit=100000, neumann=False, x0=None, verbose=False,
              max_restarts=4):
    """Jacobi-preconditioned CG on (K3 + sigma Vol) u = Vol f.

    Runs CG until the recursively updated residual drops below tol * ||b||, then
    recomputes the true residual b - S x; while that is still above tol * ||b||, CG is
    restarted from the current iterate (residual replacement, at most max_restarts
    times), because in floating point the recursive residual keeps shrinking after the
    true one has stalled.  Returns (u, info) with the total iteration count, the true
    relative residual, the number of restarts and the wall time.
    """
    t0 = time.perf_counter()
    S = (K3 + sp.diags(sigma * vol)).tocsr()
    if neumann:
        f = project(f, vol)
    b = vol * f
    dinv = 1.0 / S.diagonal()
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    it = 0
    restarts = 0
    while True:
        r = b - S @ x
        if neumann:
            r -= r.sum() / r.size      # keep the residual in the range (constant null vector)
        if np.linalg.norm(r) <= tol * bn or it >= maxit:
            break
        if restarts > max_restarts:
            break
        z = dinv * r
        p = z.copy()
        rz = r @ z
        while it < maxit:
            if np.linalg.norm(r) <= tol * bn:
                break
            q = S @ p
            alpha = rz / (p @ q)
            x += alpha * p
            r -= alpha * q
            z = dinv * r
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
            it += 1
            if verbose and it % 100 == 0:
                print(f"  pcg it {it} rel {np.linalg.norm(r) / bn:.3e}", flush=True)
        restarts += 1
    if neumann:
        x = project(x, vol)
    true_rel = np.linalg.norm(b - S @ x) / bn
    info = dict(iterations=it, true_rel_residual=float(true_rel), restarts=restarts - 1,
                seconds=time.perf_counter() - t0)
    return x, info


def solve_problem(faces, sigma, f, loc=(fv.CELL,) * 3, bc_lo=(fv.DIRICHLET,) * 3,
                  bc_hi=(fv.DIRICHLET,) * 3, method="auto", tol=1e-14):
    """Solve (sigma I - Laplacian_h) u = f for every RHS in f[(nrhs,) nz, ny, nx].

    method: "dense", "splu", "pcg" or "auto" (dense <= 1728 unknowns, splu <= 40^3,
    PCG otherwise).  All-Neumann with sigma = 0 is solved in the projected gauge.
    Returns (u, info list).
    """
    H, K3, vol, shape = fv.helmholtz_matrix(faces, sigma, loc, bc_lo, bc_hi)
    nx, ny, nz = shape
    N = nx * ny * nz
    neumann = sigma == 0.0 and is_all_neumann(bc_lo, bc_hi)
    f = np.asarray(f, dtype=np.float64)
    fr = f.reshape(-1, N)
    if method == "auto":
        method = "dense" if N <= 1728 else ("splu" if N <= 64000 else "pcg")
    out = np.empty_like(fr)
    infos = []
    lu = None
    for r in range(fr.shape[0]):
        t0 = time.perf_counter()
        if neumann and method != "pcg":
            out[r] = project(solve_neumann_bordered(K3, vol, fr[r]), vol)
            infos.append(dict(method="bordered-splu", seconds=time.perf_counter() - t0))
        elif method == "dense":
            out[r] = solve_dense(H, fr[r])
            infos.append(dict(method="dense", seconds=time.perf_counter() - t0))
        elif method == "splu":
            if lu is None:
                lu = spla.splu(H.tocsc())
            out[r] = lu.solve(fr[r])
            infos.append(dict(method="splu", seconds=time.perf_counter() - t0))
        elif method == "pcg":
            out[r], info = solve_pcg(K3, vol, sigma, fr[r], tol=tol, neumann=neumann)
            info["method"] = "pcg"
            infos.append(info)
        else:
            raise ValueError(method)
    return out.reshape(f.shape), infos


def apply_operator(faces, sigma, u, loc=(fv.CELL,) * 3, bc_lo=(fv.DIRICHLET,) * 3,
                   bc_hi=(fv.DIRICHLET,) * 3):
    """H u with the cell-by-cell assembled operator, for every RHS in u[..., nz, ny, nx]."""
    H, _, _, shape = fv.helmholtz_matrix(faces, sigma, loc, bc_lo, bc_hi)
    N = int(np.prod(shape))
    ur = np.asarray(u, dtype=np.float64).reshape(-1, N)
    return np.stack([H @ x for x in ur]).reshape(np.shape(u))


def rel_err(u, ref):
    u = np.asarray(u).ravel()
    ref = np.asarray(ref).ravel()
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
