// Host setup stage: 1D FV operators (Section 3, eq. 23) and their eigen-decomposition (eq. 24).
#include "setup.hpp"

#include <algorithm>
#include <cmath>
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

bool tridiag_eigen(int m, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Z) {
  Z.assign(static_cast<size_t>(m) * m, 0.0);
  for (int i = 0; i < m; ++i) Z[static_cast<size_t>(i) * m + i] = 1.0;
  e.resize(m);
  e[m - 1] = 0.0;
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < m; ++l) {
    int iter = 0;
    for (;;) {
      // Look for a negligible off-diagonal element splitting the matrix at or below l.
      int s = l;
      for (; s < m - 1; ++s) {
        const double dd = std::fabs(d[s]) + std::fabs(d[s + 1]);
        if (std::fabs(e[s]) <= eps * dd) break;
      }
      if (s == l) break;
      if (++iter > 60) return false;
      // Shift from the leading 2x2 block (Wilkinson-type), then chase the bulge upward
      // from s to l with plane rotations, accumulating them into Z.
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[s] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double sn = 1.0, cs = 1.0, p = 0.0;
      int i = s - 1;
      bool underflow = false;
      for (; i >= l; --i) {
        double f = sn * e[i];
        const double b = cs * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[s] = 0.0;
          underflow = true;
          break;
        }
        sn = f / r;
        cs = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * sn + 2.0 * cs * b;
        p = sn * r;
        d[i + 1] = g + p;
        g = cs * r - b;
        for (int k = 0; k < m; ++k) {
          double* zk = &Z[static_cast<size_t>(k) * m];
          f = zk[i + 1];
          zk[i + 1] = sn * zk[i] + cs * f;
          zk[i] = cs * zk[i] - sn * f;
        }
      }
      if (underflow) continue;
      d[l] -= p;
      e[l] = g;
      e[s] = 0.0;
    }
  }
  // Sort ascending, permuting the eigenvector columns alongside.
  std::vector<int> order(m);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  std::vector<double> d2(m), Z2(static_cast<size_t>(m) * m);
  for (int a = 0; a < m; ++a) {
    d2[a] = d[order[a]];
    for (int k = 0; k < m; ++k) Z2[static_cast<size_t>(k) * m + a] = Z[static_cast<size_t>(k) * m + order[a]];
  }
  d.swap(d2);
  Z.swap(Z2);
  return true;
}

std::string eigen_1d(Axis1D& ax) {
  const int m = ax.m;
  std::vector<double> sv(m), d(m), e(m, 0.0), Q;
  for (int i = 0; i < m; ++i) sv[i] = std::sqrt(ax.vol[i]);
  for (int i = 0; i < m; ++i) d[i] = ax.k_diag[i] / ax.vol[i];
  for (int i = 0; i + 1 < m; ++i) e[i] = ax.k_off[i] / (sv[i] * sv[i + 1]);
  if (!tridiag_eigen(m, d, e, Q)) return "tridiagonal eigensolver did not converge";
  // Neumann at both walls: the constant is an exact null vector of K, so the smallest
  // eigenpair is set exactly: lambda_0 = 0, q_0 = V^{1/2} 1 / ||V^{1/2} 1||; the other
  // vectors are re-orthogonalized against it.
  if (ax.null_mode) {
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += ax.vol[i];
    nrm = std::sqrt(nrm);
    std::vector<double> q0(m);
    double dot = 0.0;
    for (int i = 0; i < m; ++i) {
      q0[i] = sv[i] / nrm;
      dot += q0[i] * Q[static_cast<size_t>(i) * m];
    }
    const double sgn = dot >= 0.0 ? 1.0 : -1.0;
    for (int i = 0; i < m; ++i) Q[static_cast<size_t>(i) * m] = sgn * q0[i];
    d[0] = 0.0;
    for (int a = 1; a < m; ++a) {
      double h = 0.0, nn = 0.0;
      for (int i = 0; i < m; ++i) h += q0[i] * Q[static_cast<size_t>(i) * m + a];
      for (int i = 0; i < m; ++i) {
        double& z = Q[static_cast<size_t>(i) * m + a];
        z -= h * q0[i];
        nn += z * z;
      }
      nn = 1.0 / std::sqrt(nn);
      for (int i = 0; i < m; ++i) Q[static_cast<size_t>(i) * m + a] *= nn;
    }
  }
  ax.lam = d;
  ax.E.assign(static_cast<size_t>(m) * m, 0.0);
  ax.Einv.assign(static_cast<size_t>(m) * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int a = 0; a < m; ++a) {
      const double q = Q[static_cast<size_t>(i) * m + a];
      ax.E[static_cast<size_t>(i) * m + a] = q / sv[i];
      ax.Einv[static_cast<size_t>(a) * m + i] = q * sv[i];
    }
  return "";
}

}  // namespace helm
