"""MI355X fast-diagonalization Helmholtz/Laplace solver (Vitoshkin & Gelfgat, Section 3).

Thin Python binding over libhelm.so (include/helm.h): argument marshalling only.  Every
step of a solve runs in the library's HIP kernels; PyTorch supplies device memory and
streams.  There is no CPU fallback: a missing library raises.

    from paper_1107_2461_amd import Plan
    plan = Plan(faces=(fx, fy, fz), bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), sigma=10.0)
    u = plan.solve(f)          # f: float64 CUDA tensor [nrhs, nz, ny, nx]
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (BF16, BF16_IR, CELL, DIRICHLET, FACE, FP32, FP32_IR, FP64, NEUMANN, NULL_PAPER_EQ28,
                   NULL_PROJECT, TPF, TPT_Z, HelmError, check, load)

__all__ = ["Plan", "CylPlan", "TimeStepper", "solve_group", "group_workspace_bytes", "host_operator_cyl", "host_eigen_cyl", "PressureMatrix", "Server", "TorchAllocator", "torch_allocator", "sched_simulate", "load", "HelmError", "host_operator_1d", "host_eigen_1d", "DIRICHLET",
           "NEUMANN", "CELL", "FACE", "FP64", "FP32", "BF16", "FP32_IR", "BF16_IR", "TPF", "TPT_Z",
           "NULL_PROJECT", "NULL_PAPER_EQ28"]


def _torch():
    import torch
    return torch


def _grid(faces, loc):
    arrs = [np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in faces]
    g = _lib.HelmGrid()
    for d in range(3):
        g.n[d] = len(arrs[d]) - 1
        g.faces[d] = arrs[d].ctypes.data_as(_lib.DP)
        g.loc[d] = int(loc[d])
    return g, arrs


class TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator (helm_opts.alloc).

    Each block the library asks for is a torch uint8 tensor kept here until the library
    releases it, so torch.cuda.memory_allocated() counts the library's plans, pressure-matrix
    vectors and server arenas.  The library synchronizes the device before it releases a
    block, so the caching allocator may hand the memory out again at once.  Use the shared
    instance from torch_allocator(): it must outlive every object built with it."""

    def __init__(self):
        import threading
        self._blocks = {}
        self._lock = threading.Lock()
        self._fn_alloc = _lib.ALLOC_FN(self._alloc)
        self._fn_free = _lib.FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        torch = _torch()
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=torch.device("cuda", torch.cuda.current_device()))
        except RuntimeError:
            return None
        with self._lock:
            self._blocks[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, nbytes, ctx):
        with self._lock:
            self._blocks.pop(ptr, None)

    def blocks(self):
        """Number of live blocks held for the library."""
        with self._lock:
            return len(self._blocks)

    def fill(self, opts):
        opts.alloc = self._fn_alloc
        opts.dealloc = self._fn_free
        opts.alloc_ctx = None


_TORCH_ALLOCATOR = None


def torch_allocator():
    """The process-wide TorchAllocator (created on first use, never released)."""
    global _TORCH_ALLOCATOR
    if _TORCH_ALLOCATOR is None:
        _TORCH_ALLOCATOR = TorchAllocator()
    return _TORCH_ALLOCATOR


def _opts(precision, method, ir_tol, max_sweeps, null_mode, allocator=None):
    o = _lib.HelmOpts()
    load().helm_default_opts(C.byref(o))
    if allocator is not None:
        allocator.fill(o)
    o.precision = _lib.PRECISIONS.get(precision, precision) if isinstance(precision, str) else int(precision)
    o.method = _lib.METHODS.get(method, method) if isinstance(method, str) else int(method)
    if ir_tol is not None:
        o.ir_tol = float(ir_tol)
    if max_sweeps is not None:
        o.max_sweeps = int(max_sweeps)
    o.null_mode = int(null_mode)
    return o


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Plan:
    """A solve plan for (sigma I - Lap_h) u = f (helm_setup).

    precision: "fp64", "fp32", "bf16", "bf16x3" or their "_ir" forms (refined in FP64);
    method: "tpf" or "tpt" (Thomas in z, FP64); ir_tol / max_sweeps: refinement stop (the
    library's defaults when None); ir_tol = 0 runs exactly max_sweeps sweeps without reading
    norms back, so a solve only enqueues kernels and may be captured in a CUDA graph."""

    def __init__(self, faces, bc_lo=(DIRICHLET,) * 3, bc_hi=(DIRICHLET,) * 3, sigma=0.0, loc=(CELL,) * 3,
                 precision="fp64", method="tpf", ir_tol=None, max_sweeps=None, null_mode=NULL_PROJECT,
                 pressure=False, allocator=None, _handle=None):
        lib = load()
        if _handle is not None:            # built by a subclass's own setup call
            self._h = _handle
            self.sigma = float(sigma)
            self.pressure = False
            self.shape_xyz = tuple(self.eigen(d)[0].shape[0] for d in range(3))
            self._ws = {}
            self.last_info = None
            return
        g, self._faces = _grid(faces, loc)
        opts = _opts(precision, method, ir_tol, max_sweeps, null_mode, allocator)
        h = C.c_void_p()
        if pressure:
            check(lib.helm_pressure_setup(C.byref(g), C.byref(opts), C.byref(h)), "helm_pressure_setup")
        else:
            bc = _lib.HelmBC()
            for d in range(3):
                bc.lo[d] = int(bc_lo[d])
                bc.hi[d] = int(bc_hi[d])
            check(lib.helm_setup(C.byref(g), C.byref(bc), float(sigma), C.byref(opts), C.byref(h)), "helm_setup")
        self._h = h
        self.sigma = 0.0 if pressure else float(sigma)
        self.pressure = pressure
        self.shape_xyz = tuple(self.eigen(d)[0].shape[0] for d in range(3))
        self._ws = {}
        self.last_info = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                load().helm_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, nrhs):
        n = C.c_size_t()
        check(load().helm_workspace_size(self._h, int(nrhs), C.byref(n)), "helm_workspace_size")
        return n.value

    def workspace(self, nrhs, device=None):
        torch = _torch()
        key = (nrhs, device)
        ws = self._ws.get(key)
        if ws is None:
            ws = torch.empty(max(self.workspace_bytes(nrhs), 1) + 256, dtype=torch.uint8,
                             device=device or "cuda")
            self._ws[key] = ws
        return ws

    @staticmethod
    def _aligned(ws):
        p = ws.data_ptr()
        return C.c_void_p((p + 255) // 256 * 256)

    def solve(self, f, out=None, sigma=None, stream=None, workspace=None, allow_unconverged=False):
        """u = H^{-1} f for f: float64 CUDA tensor [nrhs, nz, ny, nx] (or [nz, ny, nx])."""
        torch = _torch()
        squeeze = f.dim() == 3
        f4 = f.unsqueeze(0) if squeeze else f
        if f4.dtype != torch.float64 or not f4.is_cuda or not f4.is_contiguous():
            raise ValueError("f must be a contiguous float64 CUDA tensor")
        nrhs = f4.shape[0]
        if tuple(f4.shape[1:]) != self.shape_xyz[::-1]:
            raise ValueError(f"f shape {tuple(f4.shape)} does not match the plan grid {self.shape_xyz[::-1]}")
        u = torch.empty_like(f4) if out is None else (out.unsqueeze(0) if out.dim() == 3 else out)
        ws = workspace if workspace is not None else self.workspace(nrhs, f4.device)
        sig = None
        if sigma is not None:
            sarr = (C.c_double * nrhs)(*[float(s) for s in np.broadcast_to(np.asarray(sigma, float), (nrhs,))])
            sig = C.cast(sarr, _lib.DP)
        info = _lib.HelmInfo()
        fn = load().helm_pressure_solve if self.pressure else load().helm_solve
        if self.pressure:
            st = fn(self._h, C.c_void_p(f4.data_ptr()), C.c_void_p(u.data_ptr()), nrhs, self._aligned(ws),
                    _stream_ptr(stream), C.byref(info))
        else:
            st = fn(self._h, C.c_void_p(f4.data_ptr()), C.c_void_p(u.data_ptr()), nrhs, sig, self._aligned(ws),
                    _stream_ptr(stream), C.byref(info))
        # converged: None when not checked (ir_tol = 0, a fixed sweep count)
        self.last_info = dict(sweeps=info.sweeps, last_correction=info.last_correction,
                              converged=None if info.converged < 0 else bool(info.converged))
        if not (allow_unconverged and st == _lib.HELM_ENOTCONVERGED):
            check(st, "helm_solve")
        return u[0] if squeeze else u

    def solve_noalloc(self, f, out=None, sigma=None, stream=None):
        """helm_solve_noalloc: the solve with the library's static per-GPU workspace (no
        allocation by the library; refined plans need ir_tol = 0).  out must be given by callers
        that cannot allocate; None allocates it here with torch."""
        torch = _torch()
        squeeze = f.dim() == 3
        f4 = f.unsqueeze(0) if squeeze else f
        if f4.dtype != torch.float64 or not f4.is_cuda or not f4.is_contiguous():
            raise ValueError("f must be a contiguous float64 CUDA tensor")
        nrhs = f4.shape[0]
        if tuple(f4.shape[1:]) != self.shape_xyz[::-1]:
            raise ValueError(f"f shape {tuple(f4.shape)} does not match the plan grid {self.shape_xyz[::-1]}")
        u = torch.empty_like(f4) if out is None else (out.unsqueeze(0) if out.dim() == 3 else out)
        sig = None
        if sigma is not None:
            sarr = (C.c_double * nrhs)(*[float(s) for s in np.broadcast_to(np.asarray(sigma, float), (nrhs,))])
            sig = C.cast(sarr, _lib.DP)
        info = _lib.HelmInfo()
        st = load().helm_solve_noalloc(self._h, C.c_void_p(f4.data_ptr()), C.c_void_p(u.data_ptr()), nrhs, sig,
                                       _stream_ptr(stream), C.byref(info))
        self.last_info = dict(sweeps=info.sweeps, last_correction=info.last_correction,
                              converged=None if info.converged < 0 else bool(info.converged))
        check(st, "helm_solve_noalloc")
        return u[0] if squeeze else u

    def apply(self, u, sigma=None, stream=None):
        """Hu with the FP64 7-point operator (helm_apply)."""
        torch = _torch()
        u4 = u.unsqueeze(0) if u.dim() == 3 else u
        if u4.dtype != torch.float64 or not u4.is_cuda or not u4.is_contiguous():
            raise ValueError("u must be a contiguous float64 CUDA tensor")
        out = torch.empty_like(u4)
        nrhs = u4.shape[0]
        sig = None
        if sigma is not None:
            sarr = (C.c_double * nrhs)(*[float(s) for s in np.broadcast_to(np.asarray(sigma, float), (nrhs,))])
            sig = C.cast(sarr, _lib.DP)
        check(load().helm_apply(self._h, C.c_void_p(u4.data_ptr()), C.c_void_p(out.data_ptr()), nrhs, sig,
                                _stream_ptr(stream)), "helm_apply")
        return out[0] if u.dim() == 3 else out

    def profile(self, enable=True, stages=None):
        """Enable/disable per-launch stage timing (helm_profile_enable); `stages` (names from
        STAGES) restricts it to those stages (helm_profile_stages), None times all of them."""
        lib = load()
        mask = ~0 & 0xFFFFFFFF
        if stages is not None:
            mask = 0
            for name in stages:
                mask |= 1 << _lib.STAGES.index(name)
        check(lib.helm_profile_stages(self._h, C.c_uint(mask)), "helm_profile_stages")
        check(lib.helm_profile_enable(self._h, int(bool(enable))), "helm_profile_enable")

    def profile_read(self):
        """{stage: (milliseconds, launches)} accumulated since the last read (helm_profile_read)."""
        ms = (C.c_double * len(_lib.STAGES))()
        n = (C.c_int * len(_lib.STAGES))()
        check(load().helm_profile_read(self._h, ms, n), "helm_profile_read")
        return {name: (ms[i], n[i]) for i, name in enumerate(_lib.STAGES) if n[i]}

    def fast_axes(self):
        """Axes (0 = x, 1 = y, 2 = z) transformed by the fast sine/cosine transform (helm_fast_axes)."""
        m = C.c_int()
        check(load().helm_fast_axes(self._h, C.byref(m)), "helm_fast_axes")
        return tuple(d for d in range(3) if (m.value >> d) & 1)

    def eigen(self, axis):
        lib = load()
        n = C.c_int()
        check(lib.helm_get_eigen(self._h, axis, C.byref(n), None, None, None), "helm_get_eigen")
        m = n.value
        lam = np.empty(m)
        E = np.empty((m, m))
        Ei = np.empty((m, m))
        check(lib.helm_get_eigen(self._h, axis, C.byref(n), lam.ctypes.data_as(_lib.DP), E.ctypes.data_as(_lib.DP),
                                 Ei.ctypes.data_as(_lib.DP)), "helm_get_eigen")
        return lam, E, Ei


class CylPlan(Plan):
    """Cylindrical-coordinate plan (helm_cyl_setup; Section 6, eqs. 41-44): FP64, transforms in
    theta and z and one Thomas solve per radial line.  Grid functions are float64 CUDA tensors
    [nrhs, n_r, n_z, n_theta] (theta fastest); solve / solve_noalloc / apply as for Plan.

    faces = (r_faces, theta_faces, z_faces); bc_lo / bc_hi = (r, theta, z) walls (the inner r
    wall is ignored on the axis r_0 = 0, the theta walls when theta_periodic)."""

    def __init__(self, faces, bc_lo=(DIRICHLET,) * 3, bc_hi=(DIRICHLET,) * 3, sigma=0.0, theta_periodic=True,
                 null_mode=NULL_PROJECT, allocator=None):
        lib = load()
        arrs = [np.ascontiguousarray(np.asarray(f, dtype=np.float64)) for f in faces]
        g = _lib.HelmCylGrid()
        for d in range(3):
            g.n[d] = len(arrs[d]) - 1
            g.faces[d] = arrs[d].ctypes.data_as(_lib.DP)
        g.theta_periodic = int(bool(theta_periodic))
        bc = _lib.HelmBC()
        for d in range(3):
            bc.lo[d] = int(bc_lo[d])
            bc.hi[d] = int(bc_hi[d])
        opts = _opts("fp64", "tpt", None, None, null_mode, allocator)
        h = C.c_void_p()
        check(lib.helm_cyl_setup(C.byref(g), C.byref(bc), float(sigma), C.byref(opts), C.byref(h)), "helm_cyl_setup")
        self._faces = arrs
        super().__init__(None, sigma=sigma, _handle=h)
        # plan axes are (theta, z, r); the tensor shape is (nrhs, n_r, n_z, n_theta)
        self.shape_rtz = (self.shape_xyz[2], self.shape_xyz[0], self.shape_xyz[1])


def host_operator_cyl(kind, faces, bc_lo=DIRICHLET, bc_hi=DIRICHLET):
    """Rows (lower, diag, upper) of A = V^{-1} K and control volumes of a cylindrical axis from the
    library's host code: kind 0 = radial (volumes rc dr), 1 = periodic theta (lower[0] and
    upper[-1] couple the two ends)."""
    lib = load()
    fa = np.ascontiguousarray(np.asarray(faces, dtype=np.float64))
    n = len(fa) - 1
    out = [np.zeros(n) for _ in range(4)]
    m = C.c_int()
    check(lib.helm_host_operator_cyl(int(kind), n, fa.ctypes.data_as(_lib.DP), bc_lo, bc_hi, C.byref(m),
                                     *[o.ctypes.data_as(_lib.DP) for o in out]), "helm_host_operator_cyl")
    return tuple(o[:m.value] for o in out)


def host_eigen_cyl(kind, faces, bc_lo=DIRICHLET, bc_hi=DIRICHLET):
    """(lam, E, Einv) of a cylindrical axis (kind 0 radial, 1 periodic) from the library's host code."""
    lib = load()
    fa = np.ascontiguousarray(np.asarray(faces, dtype=np.float64))
    n = len(fa) - 1
    lam = np.zeros(n)
    E = np.zeros(n * n)
    Ei = np.zeros(n * n)
    m = C.c_int()
    check(lib.helm_host_eigen_cyl(int(kind), n, fa.ctypes.data_as(_lib.DP), bc_lo, bc_hi, C.byref(m),
                                  lam.ctypes.data_as(_lib.DP), E.ctypes.data_as(_lib.DP),
                                  Ei.ctypes.data_as(_lib.DP)), "helm_host_eigen_cyl")
    mm = m.value
    return lam[:mm], E[:mm * mm].reshape(mm, mm), Ei[:mm * mm].reshape(mm, mm)


def host_operator_1d(faces, loc=CELL, bc_lo=DIRICHLET, bc_hi=DIRICHLET):
    """Rows (lower, diag, upper) of A = V^{-1} K and control volumes, computed by the library's host code."""
    lib = load()
    fa = np.ascontiguousarray(np.asarray(faces, dtype=np.float64))
    n = len(fa) - 1
    out = [np.zeros(n) for _ in range(4)]
    m = C.c_int()
    check(lib.helm_host_operator_1d(n, fa.ctypes.data_as(_lib.DP), loc, bc_lo, bc_hi, C.byref(m),
                                    *[o.ctypes.data_as(_lib.DP) for o in out]), "helm_host_operator_1d")
    return tuple(o[:m.value] for o in out)


def host_eigen_1d(faces, loc=CELL, bc_lo=DIRICHLET, bc_hi=DIRICHLET):
    """(lam, E, Einv) of one axis from the library's host eigensolver."""
    lib = load()
    fa = np.ascontiguousarray(np.asarray(faces, dtype=np.float64))
    n = len(fa) - 1
    lam = np.zeros(n)
    E = np.zeros(n * n)
    Ei = np.zeros(n * n)
    m = C.c_int()
    check(lib.helm_host_eigen_1d(n, fa.ctypes.data_as(_lib.DP), loc, bc_lo, bc_hi, C.byref(m),
                                 lam.ctypes.data_as(_lib.DP), E.ctypes.data_as(_lib.DP), Ei.ctypes.data_as(_lib.DP)),
          "helm_host_eigen_1d")
    mm = m.value
    return lam[:mm], E[:mm * mm].reshape(mm, mm), Ei[:mm * mm].reshape(mm, mm)


class PressureMatrix:
    """Pressure matrix C of eq. 9 with FGMRES solve (helm_pmatrix_*)."""

    def __init__(self, faces, tau, precision="fp64", method=None, allocator=None):
        """method: "tpf" or "tpt" (FP64 only) for the velocity and pressure-preconditioner solves;
        None picks the Thomas variant in FP64 (the faster one there) and "tpf" otherwise."""
        lib = load()
        g, self._faces = _grid(faces, (CELL,) * 3)
        if method is None:
            method = "tpt" if precision == "fp64" else "tpf"
        opts = _opts(precision, method, None, None, NULL_PROJECT, allocator)
        h = C.c_void_p()
        check(lib.helm_pmatrix_setup(C.byref(g), float(tau), C.byref(opts), C.byref(h)), "helm_pmatrix_setup")
        self._h = h
        self.shape_xyz = tuple(len(f) - 1 for f in faces)
        self._ws = {}
        self.last_info = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                load().helm_pmatrix_destroy(h)
            except Exception:
                pass
            self._h = None

    def _workspace(self, restart, device):
        torch = _torch()
        ws = self._ws.get(restart)
        if ws is None:
            n = C.c_size_t()
            check(load().helm_pmatrix_workspace_size(self._h, int(restart), C.byref(n)), "workspace")
            ws = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
            self._ws[restart] = ws
        return Plan._aligned(ws)

    def apply(self, p, stream=None):
        torch = _torch()
        y = torch.empty_like(p)
        check(load().helm_pmatrix_apply(self._h, C.c_void_p(p.data_ptr()), C.c_void_p(y.data_ptr()),
                                        self._workspace(30, p.device), _stream_ptr(stream)), "helm_pmatrix_apply")
        return y

    def solve(self, b, tol=1e-10, max_it=500, restart=30, precondition=2, stream=None):
        """p with C p = b by FGMRES; precondition: 0 none, 1 pressure Laplacian, 2 I + (1/tau) A_p^{-1}."""
        torch = _torch()
        p = torch.empty_like(b)
        info = _lib.HelmInfo()
        st = load().helm_pmatrix_solve(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(p.data_ptr()), float(tol),
                                       int(max_it), int(restart), int(precondition),
                                       self._workspace(restart, b.device), _stream_ptr(stream), C.byref(info))
        self.last_info = dict(iterations=info.iterations, residual=info.residual, converged=st == _lib.HELM_OK,
                              helmholtz_solves=info.sweeps)
        if st not in (_lib.HELM_OK, _lib.HELM_ENOTCONVERGED):
            check(st, "helm_pmatrix_solve")
        return p

    def velocity_shapes(self):
        """(nz, ny, nx) of the x-, y- and z-velocity grids (one fewer node along their own axis)."""
        nx, ny, nz = self.shape_xyz
        return (nz, ny, nx - 1), (nz, ny - 1, nx), (nz - 1, ny, nx)

    def stokes(self, f, g=None, tol=1e-10, max_it=500, restart=30, precondition=2, stream=None):
        """Stokes system of eq. 8 by its three-step factorization (helm_stokes_solve):
        H_d u_d + Grad_d p = f[d], sum_d Div_d u_d = g (None: 0).  f: three contiguous float64
        CUDA tensors on the velocity grids (velocity_shapes()); returns (u_x, u_y, u_z, p) with p
        of zero volume-weighted mean."""
        torch = _torch()
        lib = load()
        for fd, shp in zip(f, self.velocity_shapes()):
            if tuple(fd.shape) != shp or fd.dtype != torch.float64 or not fd.is_contiguous():
                raise ValueError(f"velocity right-hand side must be contiguous float64 of shape {shp}")
        if g is not None and (tuple(g.shape) != tuple(reversed(self.shape_xyz)) or g.dtype != torch.float64
                              or not g.is_contiguous()):
            raise ValueError("g must be a contiguous float64 field on the pressure cells (nz, ny, nx)")
        key = ("stokes", restart)
        ws = self._ws.get(key)
        if ws is None:
            n = C.c_size_t()
            check(lib.helm_stokes_workspace_size(self._h, int(restart), C.byref(n)), "workspace")
            ws = torch.empty(n.value + 256, dtype=torch.uint8, device=f[0].device)
            self._ws[key] = ws
        nx, ny, nz = self.shape_xyz
        u = [torch.empty_like(fd) for fd in f]
        p = torch.empty((nz, ny, nx), dtype=torch.float64, device=f[0].device)
        fa = (C.c_void_p * 3)(*[fd.data_ptr() for fd in f])
        ua = (C.c_void_p * 3)(*[ud.data_ptr() for ud in u])
        info = _lib.HelmInfo()
        st = lib.helm_stokes_solve(self._h, fa, C.c_void_p(g.data_ptr() if g is not None else None), ua,
                                   C.c_void_p(p.data_ptr()), float(tol), int(max_it), int(restart), int(precondition),
                                   Plan._aligned(ws), _stream_ptr(stream), C.byref(info))
        self.last_info = dict(iterations=info.iterations, residual=info.residual, converged=st == _lib.HELM_OK,
                              helmholtz_solves=info.sweeps)
        if st not in (_lib.HELM_OK, _lib.HELM_ENOTCONVERGED):
            check(st, "helm_stokes_solve")
        return u[0], u[1], u[2], p


class Server:
    """Continuous-batching solve server (helm_server_*): submit requests, poll completions."""

    def __init__(self, budget_bytes, slots=4, precision="fp64", max_bypass_ms=50.0, method="tpf", allocator=None):
        lib = load()
        opts = _opts(precision, method, None, None, NULL_PROJECT, allocator)
        h = C.c_void_p()
        check(lib.helm_server_create(int(budget_bytes), int(slots), float(max_bypass_ms), C.byref(opts), C.byref(h)),
              "helm_server_create")
        self._h = h
        self._live = {}

    def submit(self, rid, faces, f, u, sigma, bc_lo=(DIRICHLET,) * 3, bc_hi=(DIRICHLET,) * 3, loc=(CELL,) * 3,
               stream=None):
        """Queue one request; f, u: contiguous float64 CUDA tensors [nrhs, nz, ny, nx]; sigma: nrhs shifts.
        The solve waits on the device for the work enqueued on `stream` (torch's current stream
        when None) before reading f."""
        g, arrs = _grid(faces, loc)
        bc = _lib.HelmBC()
        for d in range(3):
            bc.lo[d] = int(bc_lo[d])
            bc.hi[d] = int(bc_hi[d])
        nrhs = f.shape[0]
        sig = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (nrhs,)))
        self._live[int(rid)] = (f, u)
        st = load().helm_server_submit(self._h, C.byref(g), C.byref(bc), sig.ctypes.data_as(_lib.DP), int(nrhs),
                                       C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), int(rid),
                                       _stream_ptr(stream))
        if st != _lib.HELM_OK:
            self._live.pop(int(rid), None)
            check(st, "helm_server_submit")

    def poll(self, max_records=256, wait_ms=0):
        recs = (_lib.HelmRequestRecord * max_records)()
        n = C.c_int()
        check(load().helm_server_poll(self._h, recs, max_records, C.byref(n), int(wait_ms)), "helm_server_poll")
        out = []
        for i in range(n.value):
            r = recs[i]
            self._live.pop(r.id, None)
            out.append(dict(id=r.id, status=r.status, sweeps=r.sweeps, last_correction=r.last_correction,
                            t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done, footprint=r.footprint,
                            slot=r.slot, batch=r.batch))
        return out

    def drain(self):
        check(load().helm_server_drain(self._h), "helm_server_drain")

    def now(self):
        return load().helm_server_now(self._h)

    def stats(self):
        """Counters since creation (helm_server_stats): submitted, completed, plan_hits,
        plan_misses, setup_seconds."""
        st = _lib.HelmServerStats()
        check(load().helm_server_stats(self._h, C.byref(st)), "helm_server_stats")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().helm_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TimeStepper:
    """One step of the paper's time integration (helm_ts_*; Section 5, eqs. 37-40) on the MAC
    grid of the pressure cells `faces`: right-hand sides from the previous fields (time
    derivative, advection, pressure gradient, buoyancy, heated walls T_lo at x = 0 and T_hi at
    x = 1), one temperature, three velocity and one pressure solve, correction and update.
    Fields are contiguous float64 CUDA tensors: cells (nz, ny, nx), velocities on
    velocity_shapes()."""

    def __init__(self, faces, Pr, Gr, dt, T_lo=0.5, T_hi=-0.5, precision="fp64", method="tpf", allocator=None):
        lib = load()
        g, self._faces = _grid(faces, (CELL,) * 3)
        opts = _opts(precision, method, None, None, NULL_PROJECT, allocator)
        h = C.c_void_p()
        check(lib.helm_ts_create(C.byref(g), float(Pr), float(Gr), float(dt), float(T_lo), float(T_hi),
                                 C.byref(opts), C.byref(h)), "helm_ts_create")
        self._h = h
        self.shape_xyz = tuple(len(f) - 1 for f in faces)
        self._ws = None
        self.last_info = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                load().helm_ts_destroy(h)
            except Exception:
                pass
            self._h = None

    def cell_shape(self):
        nx, ny, nz = self.shape_xyz
        return (nz, ny, nx)

    def velocity_shapes(self):
        nx, ny, nz = self.shape_xyz
        return (nz, ny, nx - 1), (nz, ny - 1, nx), (nz - 1, ny, nx)

    def step(self, T0, Tm, v0, vm, p0, T1=None, v1=None, p1=None, server=None, stream=None):
        """(T1, v1, p1) of eqs. 37-40 from the fields at steps n (T0, v0, p0) and n - 1 (Tm, vm).
        server: a Server dedicated to this stepper, through which the five solves are run."""
        torch = _torch()
        for t, shp in [(T0, self.cell_shape()), (Tm, self.cell_shape()), (p0, self.cell_shape())] + \
                list(zip(v0, self.velocity_shapes())) + list(zip(vm, self.velocity_shapes())):
            if tuple(t.shape) != shp or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"field must be a contiguous float64 CUDA tensor of shape {shp}")
        T1 = torch.empty_like(T0) if T1 is None else T1
        v1 = [torch.empty_like(v) for v in v0] if v1 is None else list(v1)
        p1 = torch.empty_like(p0) if p1 is None else p1
        if self._ws is None:
            n = C.c_size_t()
            check(load().helm_ts_workspace_size(self._h, C.byref(n)), "helm_ts_workspace_size")
            self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=T0.device)
        fl = _lib.HelmTsFields()
        fl.T0, fl.Tm, fl.p0 = T0.data_ptr(), Tm.data_ptr(), p0.data_ptr()
        fl.T1, fl.p1 = T1.data_ptr(), p1.data_ptr()
        for d in range(3):
            fl.v0[d], fl.vm[d], fl.v1[d] = v0[d].data_ptr(), vm[d].data_ptr(), v1[d].data_ptr()
        info = _lib.HelmInfo()
        check(load().helm_ts_step(self._h, C.byref(fl), server._h if server is not None else None,
                                  Plan._aligned(self._ws), _stream_ptr(stream), C.byref(info)), "helm_ts_step")
        self.last_info = dict(solves=info.sweeps)
        return T1, v1, p1


def _group_args(plans, nrhs):
    hs = (C.c_void_p * len(plans))(*[p._h for p in plans])
    ns = (C.c_int * len(plans))(*[int(n) for n in nrhs])
    return C.cast(hs, C.POINTER(C.c_void_p)), C.cast(ns, _lib.IP)


def group_workspace_bytes(plans, nrhs):
    """helm_group_workspace_size for nrhs[i] right-hand sides of plans[i]."""
    hs, ns = _group_args(plans, nrhs)
    n = C.c_size_t()
    check(load().helm_group_workspace_size(hs, len(plans), ns, C.byref(n)), "helm_group_workspace_size")
    return n.value


def solve_group(plans, f, nrhs=None, out=None, sigma=None, stream=None, workspace=None, info=None):
    """helm_solve_group: the right-hand sides of several plans of one shape in one solve (one
    launch per stage).  f: float64 CUDA tensor [sum nrhs, nz, ny, nx], the right-hand sides of
    plans[0] first; nrhs: per plan (default 1 each); sigma: one shift per right-hand side
    (default: each plan's own).  Returns u (and fills `info`, a dict, when given)."""
    torch = _torch()
    plans = list(plans)
    nrhs = [1] * len(plans) if nrhs is None else [int(n) for n in nrhs]
    if len(nrhs) != len(plans):
        raise ValueError("nrhs must give one count per plan")
    total = sum(nrhs)
    if f.dtype != torch.float64 or not f.is_cuda or not f.is_contiguous() or f.dim() != 4 or f.shape[0] != total:
        raise ValueError("f must be a contiguous float64 CUDA tensor [sum nrhs, nz, ny, nx]")
    u = torch.empty_like(f) if out is None else out
    hs, ns = _group_args(plans, nrhs)
    if workspace is None:
        workspace = torch.empty(group_workspace_bytes(plans, nrhs) + 256, dtype=torch.uint8, device=f.device)
    sig = None
    if sigma is not None:
        sarr = (C.c_double * total)(*[float(s) for s in np.broadcast_to(np.asarray(sigma, float), (total,))])
        sig = C.cast(sarr, _lib.DP)
    hi = _lib.HelmInfo()
    st = load().helm_solve_group(hs, len(plans), ns, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), sig,
                                 Plan._aligned(workspace), _stream_ptr(stream), C.byref(hi))
    if info is not None:
        info.update(sweeps=hi.sweeps, last_correction=hi.last_correction,
                    converged=None if hi.converged < 0 else bool(hi.converged))
    check(st, "helm_solve_group")
    return u


def sched_simulate(arrival, service, footprint, slots, budget, max_bypass_ms=0.0, big=None):
    """Admission policy of the server on a virtual clock (host only): returns (admit, done) times.
    big: per request, whether its solve is of the big class (at most one runs at a time)."""
    lib = load()
    arr = np.ascontiguousarray(np.asarray(arrival, dtype=np.float64))
    srv = np.ascontiguousarray(np.asarray(service, dtype=np.float64))
    ft = np.ascontiguousarray(np.asarray(footprint, dtype=np.uint64))
    n = len(arr)
    bg = None if big is None else np.ascontiguousarray(np.asarray(big, dtype=np.int32))
    if bg is not None and len(bg) != n:
        raise ValueError("big: one flag per request")
    admit = np.zeros(n)
    done = np.zeros(n)
    check(lib.helm_sched_simulate(n, arr.ctypes.data_as(_lib.DP), srv.ctypes.data_as(_lib.DP),
                                  ft.ctypes.data_as(C.POINTER(C.c_size_t)),
                                  None if bg is None else bg.ctypes.data_as(C.POINTER(C.c_int)), int(slots), int(budget),
                                  float(max_bypass_ms), admit.ctypes.data_as(_lib.DP), done.ctypes.data_as(_lib.DP)),
          "helm_sched_simulate")
    return admit, done
