"""Host-side checks of the C-ABI library that need no GPU.

* the shared library loads and exports every function include/helm.h declares;
* the library's host setup stage (1D FV operators and the FP64 tridiagonal eigensolver,
  Section 3 eqs. 23-24) agrees with the oracle's independent 1D operator and with scipy;
* argument validation of the host entry points.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.linalg as sl

import workloads
from oracle import fv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1107_2461_amd import _lib as L
    return L.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "helm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(helm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib()
    names = declared_functions()
    assert len(names) >= 15, names
    missing = [n for n in names if getattr(lib, n, None) is None]
    assert not missing, missing


def test_status_strings():
    lib = _lib()
    for s in range(7):
        assert lib.helm_status_str(s).startswith(b"HELM_")


CASES = [
    (workloads.stretched_faces(17, 1.5), fv.CELL, fv.DIRICHLET, fv.DIRICHLET),
    (workloads.stretched_faces(23, 2.0), fv.CELL, fv.NEUMANN, fv.NEUMANN),
    (workloads.stretched_faces(9, 1.0, 0.0, 3.0), fv.CELL, fv.DIRICHLET, fv.NEUMANN),
    (workloads.stretched_faces(12, 1.25), fv.FACE, fv.DIRICHLET, fv.DIRICHLET),
    (np.linspace(0, 1, 33), fv.CELL, fv.NEUMANN, fv.DIRICHLET),
]


@pytest.mark.parametrize("faces,loc,lo,hi", CASES)
def test_host_operator_matches_oracle(faces, loc, lo, hi):
    from paper_1107_2461_amd import host_operator_1d
    lower, diag, upper, vol = host_operator_1d(faces, loc, lo, hi)
    K, vo = fv.operator_1d(faces, loc, lo, hi)
    A = K / vo[:, None]
    m = len(vo)
    np.testing.assert_allclose(vol, vo, rtol=1e-15)
    np.testing.assert_allclose(diag, np.diag(A), rtol=1e-14)
    np.testing.assert_allclose(upper[:-1], np.diag(A, 1), rtol=1e-14)
    np.testing.assert_allclose(lower[1:], np.diag(A, -1), rtol=1e-14)
    assert upper[m - 1] == 0.0 and lower[0] == 0.0


@pytest.mark.parametrize("faces,loc,lo,hi", CASES)
def test_host_eigen_matches_scipy(faces, loc, lo, hi):
    from paper_1107_2461_amd import host_eigen_1d
    lam, E, Ei = host_eigen_1d(faces, loc, lo, hi)
    K, vol = fv.operator_1d(faces, loc, lo, hi)
    A = K / vol[:, None]
    ref = sl.eigh(K, np.diag(vol), eigvals_only=True)
    scale = ref.max()
    np.testing.assert_allclose(lam, ref, rtol=0, atol=1e-12 * scale)
    m = len(lam)
    # eq. 24: A = E diag(lam) E^{-1}, with E^{-1} E = I and E^T V E = I
    np.testing.assert_allclose(A @ E, E * lam[None, :], atol=1e-11 * scale)
    np.testing.assert_allclose(Ei @ E, np.eye(m), atol=1e-13)
    np.testing.assert_allclose(E.T @ (vol[:, None] * E), np.eye(m), atol=1e-13)
    if lo == fv.NEUMANN and hi == fv.NEUMANN:
        assert lam[0] == 0.0
        c = E[:, 0]
        assert np.ptp(c) <= 1e-15 * abs(c).max()     # exact constant null vector


def test_host_uniform_dirichlet_closed_form():
    from paper_1107_2461_amd import host_eigen_1d
    n, L = 64, 2.0
    h = L / n
    lam, _, _ = host_eigen_1d(np.linspace(0, L, n + 1))
    ref = 4 / h**2 * np.sin(np.pi * np.arange(1, n + 1) / (2 * n)) ** 2
    np.testing.assert_allclose(lam, ref, rtol=1e-12)


def test_host_argument_validation():
    from paper_1107_2461_amd import _lib as L
    lib = _lib()
    m = C.c_int()
    bad = np.array([0.0, 0.5, 0.4, 1.0])
    st = lib.helm_host_operator_1d(3, bad.ctypes.data_as(L.DP), 0, 0, 0, C.byref(m), None, None, None, None)
    assert st == L.HELM_EINVAL
    ok = np.linspace(0, 1, 5)
    assert lib.helm_host_operator_1d(4, ok.ctypes.data_as(L.DP), 7, 0, 0, C.byref(m), None, None, None,
                                     None) == L.HELM_EINVAL
    assert lib.helm_host_operator_1d(4, ok.ctypes.data_as(L.DP), 0, 0, 3, C.byref(m), None, None, None,
                                     None) == L.HELM_EINVAL
    assert lib.helm_host_operator_1d(1, ok.ctypes.data_as(L.DP), 0, 0, 0, C.byref(m), None, None, None,
                                     None) == L.HELM_EINVAL
    nanf = np.array([0.0, np.nan, 1.0])
    assert lib.helm_host_operator_1d(2, nanf.ctypes.data_as(L.DP), 0, 0, 0, C.byref(m), None, None, None,
                                     None) == L.HELM_EINVAL
    assert lib.helm_setup(None, None, 0.0, None, None) == L.HELM_EINVAL
