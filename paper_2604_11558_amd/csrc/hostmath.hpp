// Host-side FP64 set-up of the split exponential Euler method: grids, the
// one-dimensional finite-difference operators of Table 1 (paper Section 3),
// their real eigen-decompositions (Proposition 1) and the dense phi_1 / exp
// factors applied as mu-mode products (Section 4).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace tg {

// Tridiagonal 1D operator.  Row r couples (r-1, r, r+1); for the periodic
// theta operator row 0 couples to n-1 and row n-1 to 0 through lo[0] and
// up[n-1].  For non-periodic operators lo[0] = up[n-1] = 0.
struct Tridiag {
  int n = 0;
  bool periodic = false;
  std::vector<double> lo, dg, up;  // A[r][r-1], A[r][r], A[r][r+1]
  std::vector<double> dense() const;  // row-major n x n
};

// Real diagonalisation A = V diag(lam) Vinv (row-major n x n matrices).
struct Eig {
  int n = 0;
  std::vector<double> lam, V, Vinv;
};

// RHO_LAMBDA: the radial part of the anomalous operator Delta_lambda with
// Dirichlet data at rho_* (Section 5.3, eq. (A_lambda)); its lambda is the
// extra argument below.
enum Coord { RHO2 = 0, RHO3 = 1, THETA = 2, PHI = 3, ZED = 4, RHO_LAMBDA = 5 };

// Grid points of one coordinate (paper eqs. (A_theta), (disk_discr),
// (ball_discr), (A_phi), (A_z), (A_lambda)).
std::vector<double> coord_grid(Coord c, int n, double extent, double lam = 0.0);
// The matching tridiagonal operator.
Tridiag coord_operator(Coord c, int n, double extent, double lam = 0.0);
// Quadrature weight of each grid point along one coordinate: the measure,
// in that coordinate's factor of the volume element (rho for RHO2 and
// RHO_LAMBDA, rho^2 for RHO3, sin(phi) for PHI, 1 for THETA and ZED), of the
// cell between the midpoints to its neighbours, the end cells closed by the
// ends of the coordinate's range.  The weights sum to the coordinate's
// factor of the domain measure.
std::vector<double> coord_weights(Coord c, int n, double extent, double lam = 0.0);
// sigma of system (syscn): root in (0, 1/2) (Appendix A).
double sigma_phi(int n);

// Eigen-decomposition of a non-periodic tridiagonal operator through the
// diagonal symmetriser Xi (A Xi = Xi S, S symmetric), and the implicit QL
// iteration with Wilkinson shifts on S.
Eig eig_tridiag(const Tridiag& A);
// Orthonormal real Fourier eigenbasis of the circulant theta operator
// (closed form; Q is orthogonal so Vinv = Q^T).
Eig eig_theta(int n);

// phi_1(c A) and e^{c A} from an eigen-decomposition (row-major n x n).
std::vector<double> phi1_from_eig(const Eig& e, double c);
std::vector<double> dphi1_from_eig(const Eig& e, double c);  // (e^{cA} - phi_1(cA)) / d-scaling helper
double phi1(double x);
double phi2(double x);

// Symmetric tridiagonal eigen-solver (implicit QL, Wilkinson shift).
// d (n) diagonal, e (n-1) off-diagonal; on return d holds the eigenvalues
// and Z (row-major n x n, column j = eigenvector j) the orthonormal vectors.
bool symtridiag_ql(std::vector<double>& d, std::vector<double> e, std::vector<double>& Z);

}  // namespace tg
