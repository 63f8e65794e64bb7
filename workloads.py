"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU oracle.

This module holds no step of the solver's arithmetic: it only produces grids
(face coordinates) and right-hand sides.  Both sides of every parity check take
their inputs from here, so the GPU library and the oracle see identical bytes.

Grid recipe (the paper only says the finite-volume grid is "stretched near the
boundaries", Section 5.1): faces of a tanh-stretched grid on [lo, hi],

    x_i = lo + (hi - lo) * (1 + tanh(beta * (2 i / n - 1)) / tanh(beta)) / 2,  i = 0..n,

which clusters cells toward both walls; beta = 0 is read as a uniform grid.

Right-hand-side recipe: numpy.random.default_rng(seed), arrays drawn in C order
with shape (nrhs, nz, ny, nx) (x fastest), float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Boundary-condition codes (same numeric values as the library's C enum).
DIRICHLET = 0
NEUMANN = 1
# Unknown location along an axis (same numeric values as the library's C enum).
CELL = 0
FACE = 1


def stretched_faces(n: int, beta: float, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n + 1 strictly increasing face coordinates, tanh-clustered toward both ends."""
    if n < 1:
        raise ValueError("n must be >= 1")
    s = np.arange(n + 1, dtype=np.float64) / n
    if beta == 0.0:
        t = s
    else:
        t = 0.5 * (1.0 + np.tanh(beta * (2.0 * s - 1.0)) / math.tanh(beta))
    x = lo + (hi - lo) * t
    x[0], x[-1] = lo, hi
    return x


def centres(faces: np.ndarray) -> np.ndarray:
    faces = np.asarray(faces, dtype=np.float64)
    return 0.5 * (faces[1:] + faces[:-1])


@dataclass
class Problem:
    """One Helmholtz/Laplace problem: (sigma I - Laplacian_h) u = f on a box grid."""
    faces: tuple                      # (fx, fy, fz) host float64 arrays
    bc_lo: tuple = (DIRICHLET,) * 3   # per axis, low face
    bc_hi: tuple = (DIRICHLET,) * 3   # per axis, high face
    loc: tuple = (CELL,) * 3          # unknown location per axis
    sigma: float = 0.0
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def shape_xyz(self):
        n = []
        for f, l in zip(self.faces, self.loc):
            n.append(len(f) - 1 if l == CELL else len(f) - 2)
        return tuple(n)

    @property
    def npts(self) -> int:
        nx, ny, nz = self.shape_xyz
        return nx * ny * nz


def box_problem(n, beta, sigma, bc=DIRICHLET, name=""):
    """Cube [0,1]^3 with n = (nx, ny, nz) cells, same stretch and BC on every face."""
    if isinstance(n, int):
        n = (n, n, n)
    if not isinstance(beta, (tuple, list)):
        beta = (beta,) * 3
    faces = tuple(stretched_faces(n[d], beta[d]) for d in range(3))
    bcs = (bc,) * 3
    return Problem(faces=faces, bc_lo=bcs, bc_hi=bcs, sigma=sigma, name=name)


def rhs_uniform(seed: int, nrhs: int, shape_xyz, lo=-1.0, hi=1.0) -> np.ndarray:
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nrhs, nz, ny, nx))


def rhs_normal(seed: int, nrhs: int, shape_xyz) -> np.ndarray:
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(nrhs, nz, ny, nx))


def rhs_manufactured_noise(seed: int, nrhs: int, faces, amp=1e-3) -> np.ndarray:
    """sin(pi x) sin(2 pi y) sin(3 pi z) at cell centres plus U[-amp, amp] noise per RHS."""
    cx, cy, cz = (centres(f) for f in faces)
    s = (np.sin(3 * np.pi * cz)[:, None, None] * np.sin(2 * np.pi * cy)[None, :, None]
         * np.sin(np.pi * cx)[None, None, :])
    rng = np.random.default_rng(seed)
    noise = rng.uniform(-amp, amp, size=(nrhs,) + s.shape)
    return s[None] + noise


def remove_weighted_mean(f: np.ndarray, faces) -> np.ndarray:
    """Subtract the cell-volume-weighted mean over each RHS (the all-Neumann solvability condition)."""
    wx, wy, wz = (np.diff(np.asarray(fc, dtype=np.float64)) for fc in faces)
    vol = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
    out = np.array(f, dtype=np.float64, copy=True)
    for r in range(out.shape[0]):
        out[r] -= (out[r] * vol).sum() / vol.sum()
    return out


# ----------------------------------------------------------------------------------
# The five benchmark workloads (sizes, stretch, shifts, seeds).
# ----------------------------------------------------------------------------------

def workload_small_dirichlet():
    """32^3 stretched cells (beta 1.5), Dirichlet, tau = 0.1 (sigma = 10), f ~ U[-1,1], seed 1."""
    p = box_problem(32, 1.5, sigma=10.0, name="helmholtz_32cube_dirichlet_tau0.1")
    f = rhs_uniform(1, 1, p.shape_xyz)
    return p, f / 0.1          # (I - tau L) u = f  <=>  (1/tau - L) u = f / tau


def workload_multirhs_128(tau: float):
    """128^3 stretched cells, Dirichlet, 3 RHS = manufactured field + U[-1e-3,1e-3] noise, seed 2."""
    p = box_problem(128, 1.5, sigma=1.0 / tau, name=f"helmholtz_128cube_3rhs_tau{tau:g}")
    f = rhs_manufactured_noise(2, 3, p.faces)
    return p, f / tau


def workload_mixed_256():
    """256^3 stretched cells, Dirichlet, tau = 10 (sigma = 0.1), f ~ N(0,1), seed 3."""
    p = box_problem(256, 1.5, sigma=0.1, name="helmholtz_256cube_tau10")
    f = rhs_normal(3, 1, p.shape_xyz)
    return p, f / 10.0


def workload_pressure():
    """Pressure Laplacian, 192x160x224 cells, beta 1.5, all Neumann, f ~ U[-1,1] V-mean removed, seed 4."""
    n = (192, 160, 224)
    faces = tuple(stretched_faces(n[d], 1.5) for d in range(3))
    p = Problem(faces=faces, bc_lo=(NEUMANN,) * 3, bc_hi=(NEUMANN,) * 3, sigma=0.0,
                name="pressure_192x160x224_neumann")
    f = remove_weighted_mean(rhs_uniform(4, 1, p.shape_xyz), faces)
    return p, f


SERVING_GRIDS = ((64, 64, 64), (96, 128, 64), (128, 128, 128), (192, 192, 192), (256, 256, 256))
SERVING_BETAS = (1.0, 1.25, 1.5, 1.75, 2.0)


def serving_requests(seed: int, count: int, rate_hz: float, grids=SERVING_GRIDS):
    """Poisson-arrival request stream: grid, per-axis stretch, per-face BC, sigma, nrhs.

    tau = 10^U(-3, 2); 20% of requests are Laplace (sigma = 0); each face is Dirichlet or
    Neumann with probability 1/2; nrhs is 1 or 3.  Right-hand sides are drawn lazily from
    a per-request seed so that the stream itself stays small.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate_hz)
        g = grids[rng.integers(len(grids))]
        betas = tuple(float(SERVING_BETAS[rng.integers(len(SERVING_BETAS))]) for _ in range(3))
        lo = tuple(int(rng.integers(2)) for _ in range(3))
        hi = tuple(int(rng.integers(2)) for _ in range(3))
        laplace = rng.random() < 0.2
        tau = 10.0 ** rng.uniform(-3.0, 2.0)
        sigma = 0.0 if laplace else 1.0 / tau
        nrhs = 1 if rng.random() < 0.5 else 3
        out.append(dict(rid=rid, arrival=t, n=g, beta=betas, bc_lo=lo, bc_hi=hi,
                        sigma=sigma, nrhs=nrhs, rhs_seed=int(rng.integers(1 << 31))))
    return out


def serving_problem(req) -> Problem:
    faces = tuple(stretched_faces(req["n"][d], req["beta"][d]) for d in range(3))
    return Problem(faces=faces, bc_lo=tuple(req["bc_lo"]), bc_hi=tuple(req["bc_hi"]),
                   sigma=req["sigma"], name=f"serve_{req['rid']}")


def timestep_state(seed: int, n_xyz, amp: float = 0.1):
    """Seeded fields of two time levels for one step of eqs. 37-40 on the MAC grid of n_xyz
    pressure cells: (T0, Tm, v0, vm, p0) with T ~ U[-0.5, 0.5] at the cells, each velocity
    component amp * N(0,1) on its interior faces, p ~ N(0,1) at the cells; arrays [nz, ny, nx]."""
    nx, ny, nz = n_xyz
    n = (nx, ny, nz)
    rng = np.random.default_rng(seed)
    cell = (nz, ny, nx)
    vel = [tuple(n[2 - a] - (1 if 2 - a == d else 0) for a in range(3)) for d in range(3)]
    T0, Tm = rng.uniform(-0.5, 0.5, cell), rng.uniform(-0.5, 0.5, cell)
    v0 = [amp * rng.standard_normal(s) for s in vel]
    vm = [amp * rng.standard_normal(s) for s in vel]
    p0 = rng.standard_normal(cell)
    return T0, Tm, v0, vm, p0
