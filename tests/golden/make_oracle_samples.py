"""Writes sampled CPU-oracle solutions of the full-size workloads to tests/golden/*.json.

Calls only the oracle (oracle/) and the seeded input generators (workloads.py).  Each file
holds the oracle's solution at 2048 seeded random grid points per right-hand side, its
2-norm and max-norm, and the PCG statistics, so that GPU tests and the benchmark can
check full-size solves without re-running a minutes-long CPU solve.

    python tests/golden/make_oracle_samples.py [c2|c3|c4 ...]
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


if __name__ == "__main__":
    for w in (sys.argv[1:] or ["c2", "c3", "c4"]):
        make(w)
