"""Writes sampled CPU-oracle solutions of the full-size workloads to tests/golden/*.json.

Calls only the oracle (oracle/) and the seeded input generators (workloads.py).  Each file
holds the oracle's solution at 2048 seeded random grid points per right-hand side, its
2-norm and max-norm, and the PCG statistics, so that GPU tests and the benchmark can
check full-size solves without re-running a minutes-long CPU solve.

    python tests/golden/make_oracle_samples.py [c2|c3|c4 ...]
    python tests/golden/make_oracle_samples.py --floor [c1|c2|c3|c4 ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import fv, solvers  # noqa: E402

NSAMPLE = 2048


def _sample(u, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(u.size, size=min(NSAMPLE, u.size), replace=False))
    return idx


def _record(name, prob, f, tol, extra):
    K3, vol, shape = fv.assemble_3d(prob.faces, prob.loc, prob.bc_lo, prob.bc_hi)
    neumann = prob.sigma == 0.0 and solvers.is_all_neumann(prob.bc_lo, prob.bc_hi)
    out = dict(name=name, shape_xyz=list(shape), sigma=prob.sigma, nrhs=int(f.shape[0]), rhs=[], **extra)
    for r in range(f.shape[0]):
        t0 = time.perf_counter()
        u, info = solvers.solve_pcg(K3, vol, prob.sigma, f[r].ravel(), tol=tol, maxit=50000, neumann=neumann)
        idx = _sample(u, 1000 + r)
        out["rhs"].append(dict(idx=idx.tolist(), u=u[idx].tolist(), norm2=float(np.linalg.norm(u)),
                               norminf=float(np.abs(u).max()), pcg_iterations=info["iterations"],
                               pcg_true_rel_residual=info["true_rel_residual"],
                               seconds=time.perf_counter() - t0))
        print(f"{name} rhs {r}: {info['iterations']} it, res {info['true_rel_residual']:.2e}, "
              f"{time.perf_counter() - t0:.1f}s", flush=True)
    path = os.path.join(HERE, f"oracle_samples_{name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path, flush=True)


def make(which):
    if which == "c2":
        for tau in (1e-3, 1.0, 1e2):
            prob, f = workloads.workload_multirhs_128(tau)
            _record(f"c2_tau{tau:g}", prob, f, 1e-15, dict(tau=tau, workload=prob.name))
    elif which == "c3":
        prob, f = workloads.workload_mixed_256()
        _record("c3", prob, f, 1e-15, dict(workload=prob.name))
    elif which == "c4":
        prob, f = workloads.workload_pressure()
        _record("c4_pressure", prob, f, 1e-15, dict(workload=prob.name))
    else:
        raise SystemExit(f"unknown workload {which}")


def _second_solve(prob, f, neumann):
    """An independently coded FP64 solve of the same SPD system (K3 + sigma Vol) u = Vol f:
    scipy's conjugate-gradient routine with a Jacobi preconditioner (a library routine, not
    the oracle's own PCG).  Neumann: f projected first, the result gauge-fixed afterwards."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    K3, vol, _ = fv.assemble_3d(prob.faces, prob.loc, prob.bc_lo, prob.bc_hi)
    S = (K3 + sp.diags(prob.sigma * vol)).tocsr()
    dinv = 1.0 / S.diagonal()
    M = spla.LinearOperator(S.shape, matvec=lambda x: dinv * x)
    out = []
    for r in range(f.shape[0]):
        fr = f[r].ravel()
        if neumann:
            fr = solvers.project(fr, vol)
        b = vol * fr
        it = [0]
        t0 = time.perf_counter()
        u, code = spla.cg(S, b, rtol=1e-14, atol=0.0, maxiter=50000, M=M,
                          callback=lambda xk: it.__setitem__(0, it[0] + 1))
        if neumann:
            u = solvers.project(u, vol)
        res = float(np.linalg.norm(b - S @ u) / np.linalg.norm(b))
        out.append((u, dict(iterations=it[0], true_rel_residual=res, code=int(code),
                            seconds=time.perf_counter() - t0)))
    return out


def floor(which):
    """Mutual difference of two independent FP64 oracles at the stored sample points (the
    floor under every parity tolerance), written to tests/golden/oracle_floor.json."""
    path = os.path.join(HERE, "oracle_floor.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    if which == "c1":
        prob, f = workloads.workload_small_dirichlet()
        K3, vol, _ = fv.assemble_3d(prob.faces, prob.loc, prob.bc_lo, prob.bc_hi)
        H = fv.helmholtz_matrix(prob.faces, prob.sigma, prob.loc, prob.bc_lo, prob.bc_hi)[0]
        ua = solvers.solve_splu(H, f[0].ravel())
        ub, info = solvers.solve_pcg(K3, vol, prob.sigma, f[0].ravel(), tol=1e-15, maxit=50000)
        d = float(np.abs(ua - ub).max() / np.abs(ua).max())
        data["c1"] = dict(solvers=["oracle sparse LU", "oracle Jacobi-PCG (1e-15)"], rhs=[dict(rel_inf=d)],
                          note="all points")
        print(f"c1: floor {d:.2e}", flush=True)
    else:
        names = {"c2": [f"c2_tau{t:g}" for t in (1e-3, 1.0, 1e2)], "c3": ["c3"], "c4": ["c4_pressure"]}[which]
        for name in names:
            g = json.load(open(os.path.join(HERE, f"oracle_samples_{name}.json")))
            if which == "c2":
                prob, f = workloads.workload_multirhs_128(g["tau"])
            elif which == "c3":
                prob, f = workloads.workload_mixed_256()
            else:
                prob, f = workloads.workload_pressure()
            neumann = prob.sigma == 0.0 and solvers.is_all_neumann(prob.bc_lo, prob.bc_hi)
            rows = []
            for r, (u, info) in enumerate(_second_solve(prob, f, neumann)):
                gr = g["rhs"][r]
                idx = np.array(gr["idx"])
                d = float(np.abs(u[idx] - np.array(gr["u"])).max() / gr["norminf"])
                rows.append(dict(rel_inf=d, second_iterations=info["iterations"],
                                 second_true_rel_residual=info["true_rel_residual"]))
                print(f"{name} rhs {r}: floor {d:.2e} ({info['iterations']} it, res "
                      f"{info['true_rel_residual']:.1e}, {info['seconds']:.0f}s)", flush=True)
            data[name] = dict(solvers=["oracle Jacobi-PCG (1e-15, residual replacement)",
                                       "scipy.sparse.linalg.cg, Jacobi, rtol 1e-14"],
                              rhs=rows, note=f"max over the {NSAMPLE} stored sample points, relative to max|u|")
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--floor":
        for w in (args[1:] or ["c1", "c2", "c3", "c4"]):
            floor(w)
    else:
        for w in (args or ["c2", "c3", "c4"]):
            make(w)
