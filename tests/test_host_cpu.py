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


# ------------------------------------------------------------------ cylindrical axes (Section 6)

def _dense_rows(lower, diag, upper, periodic=False):
    m = len(diag)
    A = np.diag(diag) + np.diag(lower[1:], -1) + np.diag(upper[:-1], 1)
    if periodic:
        A[0, m - 1] += lower[0]
        A[m - 1, 0] += upper[m - 1]
    return A


@pytest.mark.parametrize("r0,lo,hi", [(0.0, fv.NEUMANN, fv.DIRICHLET), (0.3, fv.DIRICHLET, fv.NEUMANN),
                                      (0.3, fv.NEUMANN, fv.NEUMANN)])
def test_host_radial_operator_matches_oracle(r0, lo, hi):
    """The library's radial operator equals the oracle's cylindrical assembly on an (n_r, 1, 1)
    sector whose theta and z walls are Neumann (no theta or z coupling remains)."""
    from oracle import cyl
    from paper_1107_2461_amd import host_operator_cyl
    rf = workloads.stretched_faces(11, 1.5, r0, 1.4)
    lower, diag, upper, vol = host_operator_cyl(0, rf, lo, hi)
    K3, v3, _ = cyl.assemble(rf, [0.0, 0.7], [0.0, 0.4], (lo, hi), (fv.NEUMANN, fv.NEUMANN),
                             (fv.NEUMANN, fv.NEUMANN))
    A = K3.toarray() / v3[:, None]
    assert np.abs(_dense_rows(lower, diag, upper) - A).max() <= 1e-13 * np.abs(A).max()
    np.testing.assert_allclose(vol * 0.7 * 0.4, v3, rtol=1e-14)


def test_host_periodic_operator_matches_oracle():
    """The library's periodic theta operator times 1 / rc^2 equals the oracle's assembly on a
    one-cell annulus [1, 2] (Neumann radial and axial walls)."""
    from oracle import cyl
    from paper_1107_2461_amd import host_operator_cyl
    tf = workloads.stretched_faces(13, 1.25, 0.0, 2 * np.pi)
    lower, diag, upper, vol = host_operator_cyl(1, tf)
    K3, v3, _ = cyl.assemble([1.0, 2.0], tf, [0.0, 0.5], (fv.NEUMANN, fv.NEUMANN), None, (fv.NEUMANN, fv.NEUMANN))
    A = K3.toarray() / v3[:, None]
    assert np.abs(_dense_rows(lower, diag, upper, periodic=True) / 1.5**2 - A).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("M", [3, 8, 13])
def test_host_periodic_eigen(M):
    """Uniform periodic axis: eigenvalues (4 / h^2) sin^2(pi m / M), m = 0..M-1 (pairs m, M - m
    coincide); A E = E diag(lam), Einv E = I, lam_0 = 0 exactly.  Stretched: the same invariants
    and the eigenvalues of the dense matrix by scipy."""
    from paper_1107_2461_amd import host_eigen_cyl, host_operator_cyl
    for tf in (np.linspace(0.0, 2 * np.pi, M + 1), workloads.stretched_faces(M, 1.5, 0.0, 2 * np.pi)):
        lam, E, Ei = host_eigen_cyl(1, tf)
        lower, diag, upper, vol = host_operator_cyl(1, tf)
        A = _dense_rows(lower, diag, upper, periodic=True)
        assert lam[0] == 0.0
        assert np.abs(A @ E - E * lam[None, :]).max() <= 1e-12 * np.abs(A).max()
        assert np.abs(Ei @ E - np.eye(M)).max() <= 1e-12
        ref = np.sort(np.linalg.eigvals(A).real)
        assert np.abs(np.sort(lam) - ref).max() <= 1e-11 * np.abs(A).max()
    h = 2 * np.pi / M
    lam, _, _ = host_eigen_cyl(1, np.linspace(0.0, 2 * np.pi, M + 1))
    closed = np.sort(4 / h**2 * np.sin(np.pi * np.arange(M) / M) ** 2)
    assert np.abs(lam - closed).max() <= 1e-12 * closed.max()


def test_host_radial_eigen_generalized():
    from paper_1107_2461_amd import host_eigen_cyl, host_operator_cyl
    rf = workloads.stretched_faces(20, 1.5, 0.0, 1.0)
    lam, E, Ei = host_eigen_cyl(0, rf, fv.NEUMANN, fv.NEUMANN)
    A = _dense_rows(*host_operator_cyl(0, rf, fv.NEUMANN, fv.NEUMANN)[:3])
    assert lam[0] == 0.0 and lam[1] > 0
    assert np.abs(A @ E - E * lam[None, :]).max() <= 1e-11 * np.abs(A).max()
    assert np.abs(Ei @ E - np.eye(20)).max() <= 1e-12


def test_host_cyl_refusals():
    from paper_1107_2461_amd import HelmError, host_operator_cyl
    with pytest.raises(HelmError, match="EINVAL"):
        host_operator_cyl(0, [-0.1, 0.5, 1.0])          # negative radius
    with pytest.raises(HelmError, match="EINVAL"):
        host_operator_cyl(1, [0.0, 1.0, 2.0])           # periodic axis with two cells
    with pytest.raises(HelmError, match="EINVAL"):
        host_operator_cyl(2, [0.0, 1.0, 2.0, 3.0])      # unknown kind
