// Host-side setup stage: 1D finite-volume operators and their FP64 eigen-decomposition.
//
// Section 3, eq. 23: along each axis the FV second derivative is a three-point operator
// D_dd.  Here A = -D_dd = V^{-1} K, with K the symmetric conductance matrix (link
// conductance 1/distance between neighbouring nodes, wall conductance 1/(distance to the
// wall value) at a Dirichlet wall, none at a Neumann wall) and V the control-volume widths.
// Eq. 24: A = E diag(lambda) E^{-1}, computed once per axis.  A is similar to the symmetric
// tridiagonal T = V^{-1/2} K V^{-1/2} = Q diag(lambda) Q^T, so E = V^{-1/2} Q and
// E^{-1} = Q^T V^{1/2}: real eigenpairs, no explicit inversion.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

namespace helm {

struct Axis1D {
  int m = 0;                       // number of unknowns on this axis
  int loc = 0, bc_lo = 0, bc_hi = 0;
  std::vector<double> faces;       // n + 1 faces as given
  std::vector<double> vol;         // control-volume widths, m
  std::vector<double> k_diag;      // K diagonal, m
  std::vector<double> k_off;       // K off-diagonal between node i and i+1, m - 1 (negative)
  std::vector<double> lower, diag, upper;  // rows of A = V^{-1} K
  std::vector<double> lam;         // eigenvalues, ascending, m
  std::vector<double> E, Einv;     // m x m row-major: E[i*m + a] = component i of vector a
  bool null_mode = false;          // Neumann at both ends (or periodic): lambda_0 = 0 exactly
  // Cylindrical axes (Section 6, eq. 41).
  bool periodic = false;           // theta axis closed on itself: node m-1 couples to node 0
  double k_wrap = 0.0;             // K entry of that coupling (negative)
  std::vector<double> gdiag;       // radial axis: dr_i / rc_i, the metric weight of the theta
                                   // term in the K form (its V^{-1} form is 1 / rc_i^2)
  std::vector<double> inv_r2;      // radial axis: 1 / rc_i^2
};

// Builds the 1D operator; returns an empty string on success, else a message.
std::string build_operator_1d(int n, const double* faces, int loc, int bc_lo, int bc_hi, Axis1D& ax);

// Symmetric tridiagonal eigen-decomposition by the implicit QL method with shifts
// (Bowdler, Martin, Reinsch & Wilkinson 1968; Golub & Van Loan, Section 8.3).
// d[m] diagonal, e[m] with e[i] coupling i and i+1 (e[m-1] unused).  On return d holds
// the eigenvalues ascending and Z (m x m row-major) the orthonormal eigenvectors as
// columns.  Returns false if an eigenvalue failed to converge.
bool tridiag_eigen(int m, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Z);

// Eigen-decomposition of an operator built by one of the builders here (fills lam, E, Einv).
// A periodic axis (a cyclic tridiagonal K) is reduced to tridiagonal form by Householder
// reflections before the QL iteration.
std::string eigen_1d(Axis1D& ax);

// Radial axis of the cylindrical operator (Section 6, eq. 41, the D_rr part): cells
// [r_i, r_{i+1}] with midpoints rc_i, r_0 >= 0.  K has link conductance r_{i+1} / (rc_{i+1} -
// rc_i) (face area per unit angle and height over the node distance), a Dirichlet wall adds
// r_wall / (distance to the wall), an axis (r_0 = 0, zero area) and a Neumann wall nothing;
// V = rc_i (r_{i+1} - r_i).  Also fills gdiag and inv_r2.  bc_lo is ignored when r_0 = 0.
std::string build_operator_radial(int n, const double* faces, int bc_lo, int bc_hi, Axis1D& ax);

// Periodic axis (the cylindrical theta direction closed on itself): cell-centred nodes, the
// last cell's upper face is the first cell's lower face, so node n-1 couples to node 0 across
// the distance (t_n - tc_{n-1}) + (tc_0 - t_0).  n >= 3.
std::string build_operator_periodic(int n, const double* faces, Axis1D& ax);

}  // namespace helm
