// Host setup stage: 1D FV operators (Section 3, eq. 23) and their eigen-decomposition (eq. 24).
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

namespace helm {

std::string build_operator_1d(int n, const double* faces, int loc, int bc_lo, int bc_hi, Axis1D& ax) {
  if (!faces) return "faces pointer is NULL";
  if (loc != 0 && loc != 1) return "loc must be HELM_CELL or HELM_FACE";
  if ((bc_lo != 0 && bc_lo != 1) || (bc_hi != 0 && bc_hi != 1)) return "bad boundary code";
  if (n < 2 || (loc == 1 && n < 3)) return "too few cells on an axis";
  for (int i = 0; i < n; ++i)
    if (!(faces[i + 1] > faces[i]) || !std::isfinite(faces[i]) || !std::isfinite(faces[i + 1]))
      return "faces must be finite and strictly increasing";
  ax.faces.assign(faces, faces + n + 1);
  ax.loc = loc;
  ax.bc_lo = bc_lo;
  ax.bc_hi = bc_hi;
  std::vector<double> c(n);
  for (int i = 0; i < n; ++i) c[i] = 0.5 * (faces[i] + faces[i + 1]);
  // Node positions, control volumes and the distances to the Dirichlet wall values.
  std::vector<double> pos;
  double d_lo, d_hi;
  if (loc == 0) {
    pos = c;
    ax.vol.resize(n);
    for (int i = 0; i < n; ++i) ax.vol[i] = faces[i + 1] - faces[i];
    d_lo = c[0] - faces[0];
    d_hi = faces[n] - c[n - 1];
  } else {
    pos.assign(faces + 1, faces + n);  // interior faces
    ax.vol.resize(n - 1);
    for (int i = 0; i < n - 1; ++i) ax.vol[i] = c[i + 1] - c[i];
    d_lo = faces[1] - faces[0];
    d_hi = faces[n] - faces[n - 1];
  }
  const int m = static_cast<int>(pos.size());
  ax.m = m;
  ax.k_diag.assign(m, 0.0);
  ax.k_off.assign(m > 1 ? m - 1 : 0, 0.0);
  for (int i = 0; i + 1 < m; ++i) {
    const double g = 1.0 / (pos[i + 1] - pos[i]);
    ax.k_off[i] = -g;
    ax.k_diag[i] += g;
    ax.k_diag[i + 1] += g;
  }
  if (bc_lo == 0) ax.k_diag[0] += 1.0 / d_lo;
  if (bc_hi == 0) ax.k_diag[m - 1] += 1.0 / d_hi;
  ax.null_mode = (bc_lo == 1 && bc_hi == 1);
  ax.lower.assign(m, 0.0);
  ax.diag.assign(m, 0.0);
  ax.upper.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    ax.diag[i] = ax.k_diag[i] / ax.vol[i];
    if (i > 0) ax.lower[i] = ax.k_off[i - 1] / ax.vol[i];
    if (i + 1 < m) ax.upper[i] = ax.k_off[i] / ax.vol[i];
  }
  return "";
}

namespace {

// Implicit QL with shifts on a symmetric tridiagonal matrix (d: diagonal, e: off-diagonal,
// e[i] couples i and i + 1), accumulating the rotations into Z (row-major, Z[k][a] =
// component k of vector a).  On return d holds the eigenvalues in ascending order.
template <typename R>
bool tridiag_ql(int m, std::vector<R>& d, std::vector<R>& e, std::vector<R>& Z) {
  Z.assign(static_cast<size_t>(m) * m, R(0));
  for (int i = 0; i < m; ++i) Z[static_cast<size_t>(i) * m + i] = R(1);
  e.resize(m);
  e[m - 1] = R(0);
  const R eps = std::numeric_limits<R>::epsilon();
  for (int l = 0; l < m; ++l) {
    int iter = 0;
    for (;;) {
      // Look for a negligible off-diagonal element splitting the matrix at or below l.
      int s = l;
      for (; s < m - 1; ++s) {
        const R dd = std::fabs(d[s]) + std::fabs(d[s + 1]);
        if (std::fabs(e[s]) <= eps * dd) break;
      }
      if (s == l) break;
      if (++iter > 60) return false;
      // Shift from the leading 2x2 block (Wilkinson-type), then chase the bulge upward
      // from s to l with plane rotations, accumulating them into Z.
      R g = (d[l + 1] - d[l]) / (R(2) * e[l]);
      R r = std::hypot(g, R(1));
      g = d[s] - d[l] + e[l] / (g + (g >= R(0) ? r : -r));
      R sn = R(1), cs = R(1), p = R(0);
      int i = s - 1;
      bool underflow = false;
      for (; i >= l; --i) {
        R f = sn * e[i];
        const R b = cs * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == R(0)) {
          d[i + 1] -= p;
          e[s] = R(0);
          underflow = true;
          break;
        }
        sn = f / r;
        cs = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * sn + R(2) * cs * b;
        p = sn * r;
        d[i + 1] = g + p;
        g = cs * r - b;
        for (int k = 0; k < m; ++k) {
          R* zk = &Z[static_cast<size_t>(k) * m];
          f = zk[i + 1];
          zk[i + 1] = sn * zk[i] + cs * f;
          zk[i] = cs * zk[i] - sn * f;
        }
      }
      if (underflow) continue;
      d[l] -= p;
      e[l] = g;
      e[s] = R(0);
    }
  }
  // Sort ascending, permuting the eigenvector columns alongside.
  std::vector<int> order(m);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  std::vector<R> d2(m), Z2(static_cast<size_t>(m) * m);
  for (int a = 0; a < m; ++a) {
    d2[a] = d[order[a]];
    for (int k = 0; k < m; ++k) Z2[static_cast<size_t>(k) * m + a] = Z[static_cast<size_t>(k) * m + order[a]];
  }
  d.swap(d2);
  Z.swap(Z2);
  return true;
}

}  // namespace

bool tridiag_eigen(int m, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Z) {
  return tridiag_ql<double>(m, d, e, Z);
}

// The decomposition is computed in extended precision (x86 80-bit long double, epsilon ~1e-19)
// from the FP64 operator entries and rounded to FP64 at the end.  A QL sweep is accurate to
// epsilon * lambda_max in absolute terms; on stretched grids lambda_max / lambda_1 reaches
// ~2e5, so in FP64 the smallest eigenvalues (which dominate the solution for small sigma) and
// their vectors carry relative errors near 1e-11.  The extended sweep brings them to the FP64
// rounding of the exact decomposition of the FP64 operator.
std::string eigen_1d(Axis1D& ax) {
  using R = long double;
  const int m = ax.m;
  std::vector<R> sv(m), d(m), e(m, R(0)), Q;
  for (int i = 0; i < m; ++i) sv[i] = std::sqrt(static_cast<R>(ax.vol[i]));
  for (int i = 0; i < m; ++i) d[i] = static_cast<R>(ax.k_diag[i]) / static_cast<R>(ax.vol[i]);
  for (int i = 0; i + 1 < m; ++i) e[i] = static_cast<R>(ax.k_off[i]) / (sv[i] * sv[i + 1]);
  if (!tridiag_ql<R>(m, d, e, Q)) return "tridiagonal eigensolver did not converge";
  // Neumann at both walls: the constant is an exact null vector of K, so the smallest
  // eigenpair is set exactly: lambda_0 = 0, q_0 = V^{1/2} 1 / ||V^{1/2} 1||; the other
  // vectors are re-orthogonalized against it.
  if (ax.null_mode) {
    R nrm = 0;
    for (int i = 0; i < m; ++i) nrm += static_cast<R>(ax.vol[i]);
    nrm = std::sqrt(nrm);
    std::vector<R> q0(m);
    R dot = 0;
    for (int i = 0; i < m; ++i) {
      q0[i] = sv[i] / nrm;
      dot += q0[i] * Q[static_cast<size_t>(i) * m];
    }
    const R sgn = dot >= R(0) ? R(1) : R(-1);
    for (int i = 0; i < m; ++i) Q[static_cast<size_t>(i) * m] = sgn * q0[i];
    d[0] = R(0);
    for (int a = 1; a < m; ++a) {
      R h = 0, nn = 0;
      for (int i = 0; i < m; ++i) h += q0[i] * Q[static_cast<size_t>(i) * m + a];
      for (int i = 0; i < m; ++i) {
        R& z = Q[static_cast<size_t>(i) * m + a];
        z -= h * q0[i];
        nn += z * z;
      }
      nn = R(1) / std::sqrt(nn);
      for (int i = 0; i < m; ++i) Q[static_cast<size_t>(i) * m + a] *= nn;
    }
  }
  ax.lam.resize(m);
  for (int a = 0; a < m; ++a) ax.lam[a] = static_cast<double>(d[a]);
  ax.E.assign(static_cast<size_t>(m) * m, 0.0);
  ax.Einv.assign(static_cast<size_t>(m) * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int a = 0; a < m; ++a) {
      const R q = Q[static_cast<size_t>(i) * m + a];
      ax.E[static_cast<size_t>(i) * m + a] = static_cast<double>(q / sv[i]);
      ax.Einv[static_cast<size_t>(a) * m + i] = static_cast<double>(q * sv[i]);
    }
  return "";
}

}  // namespace helm
