"""ctypes declarations of libhelm.so (include/helm.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhelm.so")

NOALLOC_MAX_WORKSPACE = 256 << 20   # HELM_NOALLOC_MAX_WORKSPACE
HELM_OK, HELM_EINVAL, HELM_ESINGULAR, HELM_ENOMEM, HELM_EDEVICE, HELM_ENOTCONVERGED, HELM_ENONFINITE = range(7)
DIRICHLET, NEUMANN = 0, 1
CELL, FACE = 0, 1
FP64, FP32, BF16, FP32_IR, BF16_IR, BF16X3, BF16X3_IR = range(7)
TPF, TPT_Z, FFT = 0, 1, 2
NULL_PROJECT, NULL_PAPER_EQ28 = 0, 1
STAGES = ("x_fwd", "y_fwd", "z_fwd_div", "z_inv", "y_inv", "x_inv", "thomas", "null_line", "residual", "convert",
          "apply", "other", "update", "x_fwd_rhs", "z_inv_u")

PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp32_ir": FP32_IR, "bf16_ir": BF16_IR, "bf16x3": BF16X3,
              "bf16x3_ir": BF16X3_IR}
METHODS = {"tpf": TPF, "tpt": TPT_Z, "fft": FFT}


class HelmGrid(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("faces", C.POINTER(C.c_double) * 3), ("loc", C.c_int * 3)]


class HelmCylGrid(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("faces", C.POINTER(C.c_double) * 3), ("theta_periodic", C.c_int)]


class HelmTsFields(C.Structure):
    _fields_ = [("T0", C.c_void_p), ("Tm", C.c_void_p), ("v0", C.c_void_p * 3), ("vm", C.c_void_p * 3),
                ("p0", C.c_void_p), ("T1", C.c_void_p), ("v1", C.c_void_p * 3), ("p1", C.c_void_p)]


class HelmBC(C.Structure):
    _fields_ = [("lo", C.c_int * 3), ("hi", C.c_int * 3)]


# helm_alloc_fn / helm_free_fn
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class HelmOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("method", C.c_int), ("ir_tol", C.c_double), ("max_sweeps", C.c_int),
                ("null_mode", C.c_int), ("alloc", ALLOC_FN), ("dealloc", FREE_FN), ("alloc_ctx", C.c_void_p)]


class HelmInfo(C.Structure):
    _fields_ = [("sweeps", C.c_int), ("last_correction", C.c_double), ("converged", C.c_int),
                ("iterations", C.c_int), ("residual", C.c_double)]


class HelmRequestRecord(C.Structure):
    _fields_ = [("id", C.c_longlong), ("status", C.c_int), ("sweeps", C.c_int), ("last_correction", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double), ("footprint", C.c_size_t),
                ("slot", C.c_int), ("batch", C.c_int)]


class HelmServerStats(C.Structure):
    _fields_ = [("submitted", C.c_longlong), ("completed", C.c_longlong), ("plan_hits", C.c_longlong),
                ("plan_misses", C.c_longlong), ("setup_seconds", C.c_double)]


P = C.c_void_p
DP = C.POINTER(C.c_double)
IP = C.POINTER(C.c_int)

# name -> (restype, argtypes)
SIGNATURES = {
    "helm_default_opts": (None, [C.POINTER(HelmOpts)]),
    "helm_status_str": (C.c_char_p, [C.c_int]),
    "helm_setup": (C.c_int, [C.POINTER(HelmGrid), C.POINTER(HelmBC), C.c_double, C.POINTER(HelmOpts),
                             C.POINTER(P)]),
    "helm_workspace_size": (C.c_int, [P, C.c_int, C.POINTER(C.c_size_t)]),
    "helm_solve": (C.c_int, [P, P, P, C.c_int, DP, P, P, C.POINTER(HelmInfo)]),
    "helm_solve_noalloc": (C.c_int, [P, P, P, C.c_int, DP, P, C.POINTER(HelmInfo)]),
    "helm_apply": (C.c_int, [P, P, P, C.c_int, DP, P]),
    "helm_fast_axes": (C.c_int, [P, IP]),
    "helm_group_workspace_size": (C.c_int, [C.POINTER(P), C.c_int, IP, C.POINTER(C.c_size_t)]),
    "helm_solve_group": (C.c_int, [C.POINTER(P), C.c_int, IP, P, P, DP, P, P, C.POINTER(HelmInfo)]),
    "helm_get_eigen": (C.c_int, [P, C.c_int, IP, DP, DP, DP]),
    "helm_destroy": (None, [P]),
    "helm_pressure_setup": (C.c_int, [C.POINTER(HelmGrid), C.POINTER(HelmOpts), C.POINTER(P)]),
    "helm_pressure_solve": (C.c_int, [P, P, P, C.c_int, P, P, C.POINTER(HelmInfo)]),
    "helm_pmatrix_setup": (C.c_int, [C.POINTER(HelmGrid), C.c_double, C.POINTER(HelmOpts), C.POINTER(P)]),
    "helm_pmatrix_workspace_size": (C.c_int, [P, C.c_int, C.POINTER(C.c_size_t)]),
    "helm_pmatrix_apply": (C.c_int, [P, P, P, P, P]),
    "helm_pmatrix_solve": (C.c_int, [P, P, P, C.c_double, C.c_int, C.c_int, C.c_int, P, P,
                                     C.POINTER(HelmInfo)]),
    "helm_pmatrix_destroy": (None, [P]),
    "helm_stokes_workspace_size": (C.c_int, [P, C.c_int, C.POINTER(C.c_size_t)]),
    "helm_stokes_solve": (C.c_int, [P, C.POINTER(P), P, C.POINTER(P), P, C.c_double, C.c_int, C.c_int, C.c_int, P, P,
                                    C.POINTER(HelmInfo)]),
    "helm_profile_enable": (C.c_int, [P, C.c_int]),
    "helm_profile_read": (C.c_int, [P, DP, IP]),
    "helm_profile_stages": (C.c_int, [P, C.c_uint]),
    "helm_probe_mfma": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, P, P, DP]),
    "helm_probe_copy": (C.c_int, [P, P, C.c_longlong, P]),
    "helm_server_create": (C.c_int, [C.c_size_t, C.c_int, C.c_double, C.POINTER(HelmOpts), C.POINTER(P)]),
    "helm_server_submit": (C.c_int, [P, C.POINTER(HelmGrid), C.POINTER(HelmBC), DP, C.c_int, P, P, C.c_longlong,
                                     P]),
    "helm_server_poll": (C.c_int, [P, C.POINTER(HelmRequestRecord), C.c_int, IP, C.c_int]),
    "helm_server_drain": (C.c_int, [P]),
    "helm_server_now": (C.c_double, [P]),
    "helm_server_stats": (C.c_int, [P, C.POINTER(HelmServerStats)]),
    "helm_server_destroy": (None, [P]),
    "helm_sched_simulate": (C.c_int, [C.c_int, DP, DP, C.POINTER(C.c_size_t), C.POINTER(C.c_int), C.c_int,
                                      C.c_size_t, C.c_double, DP,
                                      DP]),
    "helm_cyl_setup": (C.c_int, [C.POINTER(HelmCylGrid), C.POINTER(HelmBC), C.c_double, C.POINTER(HelmOpts),
                                 C.POINTER(P)]),
    "helm_host_operator_cyl": (C.c_int, [C.c_int, C.c_int, DP, C.c_int, C.c_int, IP, DP, DP, DP, DP]),
    "helm_host_eigen_cyl": (C.c_int, [C.c_int, C.c_int, DP, C.c_int, C.c_int, IP, DP, DP, DP]),
    "helm_ts_create": (C.c_int, [C.POINTER(HelmGrid), C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                 C.POINTER(HelmOpts), C.POINTER(P)]),
    "helm_ts_workspace_size": (C.c_int, [P, C.POINTER(C.c_size_t)]),
    "helm_ts_step": (C.c_int, [P, C.POINTER(HelmTsFields), P, P, P, C.POINTER(HelmInfo)]),
    "helm_ts_destroy": (None, [P]),
    "helm_host_operator_1d": (C.c_int, [C.c_int, DP, C.c_int, C.c_int, C.c_int, IP, DP, DP, DP, DP]),
    "helm_host_eigen_1d": (C.c_int, [C.c_int, DP, C.c_int, C.c_int, C.c_int, IP, DP, DP, DP]),
}

_lib = None


def load(path: str | None = None):
    """Load libhelm.so (built in-tree by paper_1107_2461_amd.build); raise if it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run `python -m paper_1107_2461_amd.build` "
                           "(the HIP library is required; there is no fallback)")
    lib = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


class HelmError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = load().helm_status_str(status).decode()
        super().__init__(f"{what}: {msg}" if what else msg)


def check(status, what=""):
    if status != HELM_OK:
        raise HelmError(status, what)
