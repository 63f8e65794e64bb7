// Host setup stage: 1D FV operators (Section 3, eq. 23) and their eigen-decomposition (eq. 24).
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <system_error>
#include <thread>
#include <vector>

namespace helm {

namespace {

// Rows of A = V^{-1} K from K and V (periodic axes also couple the first and last node).
void fill_rows(Axis1D& ax) {
  const int m = ax.m;
  ax.lower.assign(m, 0.0);
  ax.diag.assign(m, 0.0);
  ax.upper.assign(m, 0.0);
  for (int i = 0; i < m; ++i) {
    ax.diag[i] = ax.k_diag[i] / ax.vol[i];
    if (i > 0) ax.lower[i] = ax.k_off[i - 1] / ax.vol[i];
    if (i + 1 < m) ax.upper[i] = ax.k_off[i] / ax.vol[i];
  }
  if (ax.periodic) {
    ax.lower[0] = ax.k_wrap / ax.vol[0];
    ax.upper[m - 1] = ax.k_wrap / ax.vol[m - 1];
  }
}

bool faces_ok(int n, const double* faces) {
  for (int i = 0; i < n; ++i)
    if (!(faces[i + 1] > faces[i]) || !std::isfinite(faces[i]) || !std::isfinite(faces[i + 1])) return false;
  return true;
}

}  // namespace

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
  fill_rows(ax);
  return "";
}


std::string build_operator_radial(int n, const double* faces, int bc_lo, int bc_hi, Axis1D& ax) {
  if (!faces) return "faces pointer is NULL";
  if ((bc_lo != 0 && bc_lo != 1) || (bc_hi != 0 && bc_hi != 1)) return "bad boundary code";
  if (n < 2) return "too few cells on an axis";
  if (!faces_ok(n, faces)) return "faces must be finite and strictly increasing";
  if (!(faces[0] >= 0.0)) return "radial faces must start at r >= 0";
  ax.faces.assign(faces, faces + n + 1);
  ax.loc = 0;
  const bool axis = faces[0] == 0.0;
  ax.bc_lo = axis ? 1 : bc_lo;
  ax.bc_hi = bc_hi;
  ax.m = n;
  std::vector<double> rc(n);
  for (int i = 0; i < n; ++i) rc[i] = 0.5 * (faces[i] + faces[i + 1]);
  ax.vol.resize(n);
  ax.gdiag.resize(n);
  ax.inv_r2.resize(n);
  for (int i = 0; i < n; ++i) {
    const double dr = faces[i + 1] - faces[i];
    ax.vol[i] = rc[i] * dr;
    ax.gdiag[i] = dr / rc[i];
    ax.inv_r2[i] = 1.0 / (rc[i] * rc[i]);
  }
  ax.k_diag.assign(n, 0.0);
  ax.k_off.assign(n - 1, 0.0);
  for (int i = 0; i + 1 < n; ++i) {
    const double g = faces[i + 1] / (rc[i + 1] - rc[i]);
    ax.k_off[i] = -g;
    ax.k_diag[i] += g;
    ax.k_diag[i + 1] += g;
  }
  if (!axis && bc_lo == 0) ax.k_diag[0] += faces[0] / (rc[0] - faces[0]);
  if (bc_hi == 0) ax.k_diag[n - 1] += faces[n] / (faces[n] - rc[n - 1]);
  ax.null_mode = ax.bc_lo == 1 && bc_hi == 1;
  fill_rows(ax);
  return "";
}

std::string build_operator_periodic(int n, const double* faces, Axis1D& ax) {
  if (!faces) return "faces pointer is NULL";
  if (n < 3) return "a periodic axis needs at least three cells";
  if (!faces_ok(n, faces)) return "faces must be finite and strictly increasing";
  ax.faces.assign(faces, faces + n + 1);
  ax.loc = 0;
  ax.bc_lo = ax.bc_hi = 1;
  ax.periodic = true;
  ax.m = n;
  std::vector<double> c(n);
  for (int i = 0; i < n; ++i) c[i] = 0.5 * (faces[i] + faces[i + 1]);
  ax.vol.resize(n);
  for (int i = 0; i < n; ++i) ax.vol[i] = faces[i + 1] - faces[i];
  ax.k_diag.assign(n, 0.0);
  ax.k_off.assign(n - 1, 0.0);
  for (int i = 0; i + 1 < n; ++i) {
    const double g = 1.0 / (c[i + 1] - c[i]);
    ax.k_off[i] = -g;
    ax.k_diag[i] += g;
    ax.k_diag[i + 1] += g;
  }
  const double gw = 1.0 / ((faces[n] - c[n - 1]) + (c[0] - faces[0]));
  ax.k_wrap = -gw;
  ax.k_diag[0] += gw;
  ax.k_diag[n - 1] += gw;
  ax.null_mode = true;  // no wall: the constant is in the null space
  fill_rows(ax);
  return "";
}

namespace {

// Rows [k0, k1) of an m x m row-major matrix through work(k0, k1), split between host threads
// (the caller's thread takes the first range; a range whose thread cannot be made runs on the
// caller's): for updates in which every row sees the same sequence of operations.
template <typename F>
void split_rows(int m, F&& work) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nt = static_cast<int>(std::min<unsigned>(std::min(hw, 16u), static_cast<unsigned>(m / 32)));
  if (nt <= 1) {
    work(0, m);
    return;
  }
  std::vector<std::thread> pool;
  const int per = (m + nt - 1) / nt;
  for (int t = 1; t < nt; ++t) {
    if (t * per >= m) break;
    try {
      pool.emplace_back(work, t * per, std::min(m, (t + 1) * per));
    } catch (const std::system_error&) {
      work(t * per, std::min(m, (t + 1) * per));
    }
  }
  work(0, std::min(m, per));
  for (auto& th : pool) th.join();
}

// Householder reduction of a dense symmetric matrix A (m x m row-major) to tridiagonal form
// T = Q^T A Q (Golub & Van Loan, Section 8.3.1): d, e receive the diagonal and off-diagonal of
// T, Q (row-major) the accumulated orthogonal transform.  The reflectors are kept and applied
// to Q at the end, each row of Q taking them in order (split_rows): the same operations per
// row as accumulating them one by one.
template <typename R>
void householder_tridiag(int m, std::vector<R> A, std::vector<R>& d, std::vector<R>& e, std::vector<R>& Q) {
  auto at = [&](int i, int j) -> R& { return A[static_cast<size_t>(i) * m + j]; };
  Q.assign(static_cast<size_t>(m) * m, R(0));
  for (int i = 0; i < m; ++i) Q[static_cast<size_t>(i) * m + i] = R(1);
  std::vector<R> v(m), p(m), w(m);
  struct Reflector {
    int k;
    R beta;
    std::vector<R> v;  // entries k + 1 .. m - 1
  };
  std::vector<Reflector> refl;
  for (int k = 0; k + 2 < m; ++k) {
    // reflector H = I - 2 v v^T / (v^T v) mapping A[k+1.., k] onto a multiple of e_{k+1}
    R alpha = 0;
    for (int i = k + 1; i < m; ++i) alpha += at(i, k) * at(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == R(0)) continue;
    if (at(k + 1, k) > 0) alpha = -alpha;
    std::fill(v.begin(), v.end(), R(0));
    for (int i = k + 1; i < m; ++i) v[i] = at(i, k);
    v[k + 1] -= alpha;
    R vv = 0;
    for (int i = k + 1; i < m; ++i) vv += v[i] * v[i];
    if (vv == R(0)) continue;
    const R beta = R(2) / vv;
    // A <- H A H on the trailing block: p = beta A v, w = p - (beta/2)(v^T p) v, A -= v w^T + w v^T
    for (int i = k; i < m; ++i) {
      R s = 0;
      for (int j = k + 1; j < m; ++j) s += at(i, j) * v[j];
      p[i] = beta * s;
    }
    R vp = 0;
    for (int i = k + 1; i < m; ++i) vp += v[i] * p[i];
    for (int i = k; i < m; ++i) w[i] = p[i] - R(0.5) * beta * vp * v[i];
    for (int i = k; i < m; ++i)
      for (int j = k; j < m; ++j) at(i, j) -= v[i] * w[j] + w[i] * v[j];
    refl.push_back({k, beta, std::vector<R>(v.begin() + k + 1, v.end())});
  }
  // Q <- Q H_0 H_1 ...
  split_rows(m, [&](int r0, int r1) {
    for (int r = r0; r < r1; ++r) {
      R* q = &Q[static_cast<size_t>(r) * m];
      for (const Reflector& h : refl) {
        const R* vk = h.v.data();  // vk[j - k - 1] = v[j] for j > k
        R* qk = q + h.k + 1;
        const int len = m - h.k - 1;
        R s = 0;
        for (int j = 0; j < len; ++j) s += qk[j] * vk[j];
        s *= h.beta;
        for (int j = 0; j < len; ++j) qk[j] -= s * vk[j];
      }
    }
  });
  d.resize(m);
  e.assign(m, R(0));
  for (int i = 0; i < m; ++i) d[i] = at(i, i);
  for (int i = 0; i + 1 < m; ++i) e[i] = at(i + 1, i);
}

// One plane rotation of the QL sweep: columns i and i + 1 of Z become
// (cs z_i - sn z_{i+1}, sn z_i + cs z_{i+1}).
template <typename R>
struct PlaneRot {
  int i;
  R cs, sn;
};

// Z <- Z G_1 G_2 ... (the rotations in the order the sweep made them).  Each row of Z sees
// the whole sequence independently of the others, so rows are split between threads and
// taken 16 at a time, each block staying in cache while the rotation list streams past it;
// every element gets the same operations in the same order as a rotation-by-rotation update.
template <typename R>
void apply_rotations(int m, std::vector<R>& Z, const std::vector<PlaneRot<R>>& rots) {
  constexpr int kRows = 16;
  split_rows(m, [&](int k0, int k1) {
    for (int b = k0; b < k1; b += kRows) {
      const int b1 = std::min(k1, b + kRows);
      for (const PlaneRot<R>& g : rots)
        for (int k = b; k < b1; ++k) {
          R* zk = &Z[static_cast<size_t>(k) * m];
          const R f = zk[g.i + 1];
          zk[g.i + 1] = g.sn * zk[g.i] + g.cs * f;
          zk[g.i] = g.cs * zk[g.i] - g.sn * f;
        }
    }
  });
}

// Implicit QL with shifts on a symmetric tridiagonal matrix (d: diagonal, e: off-diagonal,
// e[i] couples i and i + 1), accumulating the rotations into Z (row-major, Z[k][a] =
// component k of vector a).  On return d holds the eigenvalues in ascending order.
// keep_z: Z holds an orthogonal basis on entry (a Householder transform) and the rotations
// are applied to it, so the columns become eigenvectors of the matrix that was reduced.
// The sweeps record their rotations, which are applied to Z at the end (apply_rotations).
template <typename R>
bool tridiag_ql(int m, std::vector<R>& d, std::vector<R>& e, std::vector<R>& Z, bool keep_z = false) {
  if (!keep_z) {
    Z.assign(static_cast<size_t>(m) * m, R(0));
    for (int i = 0; i < m; ++i) Z[static_cast<size_t>(i) * m + i] = R(1);
  }
  std::vector<PlaneRot<R>> rots;
  rots.reserve(static_cast<size_t>(m) * m);
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
        rots.push_back({i, cs, sn});
      }
      if (underflow) continue;
      d[l] -= p;
      e[l] = g;
      e[s] = R(0);
    }
  }
  apply_rotations(m, Z, rots);
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
  if (ax.periodic) {
    // V^{-1/2} K V^{-1/2} is cyclic: reduce the dense symmetric matrix to tridiagonal form first
    std::vector<R> T(static_cast<size_t>(m) * m, R(0));
    for (int i = 0; i < m; ++i) T[static_cast<size_t>(i) * m + i] = d[i];
    for (int i = 0; i + 1 < m; ++i)
      T[static_cast<size_t>(i) * m + i + 1] = T[static_cast<size_t>(i + 1) * m + i] = e[i];
    const R w = static_cast<R>(ax.k_wrap) / (sv[0] * sv[m - 1]);
    T[static_cast<size_t>(m - 1)] += w;
    T[static_cast<size_t>(m - 1) * m] += w;
    householder_tridiag<R>(m, T, d, e, Q);
    if (!tridiag_ql<R>(m, d, e, Q, true)) return "tridiagonal eigensolver did not converge";
  } else if (!tridiag_ql<R>(m, d, e, Q)) {
    return "tridiagonal eigensolver did not converge";
  }
  // Neumann at both walls (or no wall, periodic): the constant is an exact null vector of K,
  // so the smallest eigenpair is set exactly: lambda_0 = 0, q_0 = V^{1/2} 1 / ||V^{1/2} 1||;
  // the other vectors are re-orthogonalized against it.
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
