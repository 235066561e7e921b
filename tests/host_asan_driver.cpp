// Exercises the library's host-side FP64 set-up (grids, operators,
// quadrature weights, sigma, eigen-decompositions, phi_1 factors) for every
// coordinate at small, odd and large sizes; built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Exit status
// 0 and "host set-up ok" on success; a residual check catches a wrong
// decomposition, the sanitizers any out-of-bounds access or undefined
// arithmetic.
#include <cmath>
#include <cstdio>
#include <vector>

#include "hostmath.hpp"

int main() {
  using namespace tg;
  const Coord coords[] = {RHO2, RHO3, THETA, PHI, ZED, RHO_LAMBDA};
  const int sizes[] = {3, 4, 7, 64, 129, 512};
  double worst = 0.0;
  for (Coord c : coords) {
    for (int n : sizes) {
      const double extent = c == ZED ? 2.5 : 1.3;
      const double lam = c == RHO_LAMBDA ? -1.95 : 0.0;
      std::vector<double> x = coord_grid(c, n, extent, lam);
      std::vector<double> w = coord_weights(c, n, extent, lam);
      Tridiag A = coord_operator(c, n, extent, lam);
      if (static_cast<int>(x.size()) != n || static_cast<int>(w.size()) != n || A.n != n) return 2;
      Eig e = c == THETA ? eig_theta(n) : eig_tridiag(A);
      std::vector<double> D = A.dense();
      double scale = 0.0, res = 0.0;
      for (double v : D) scale = std::fmax(scale, std::fabs(v));
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          double av = 0.0;
          for (int k = 0; k < n; ++k) av += D[i * n + k] * e.V[k * n + j];
          res = std::fmax(res, std::fabs(av - e.V[i * n + j] * e.lam[j]));
        }
      worst = std::fmax(worst, res / (scale * std::sqrt(static_cast<double>(n))));
      for (double cc : {1e-5, 3e-3, 0.4}) {
        std::vector<double> P = phi1_from_eig(e, cc);
        std::vector<double> dP = dphi1_from_eig(e, cc);
        if (static_cast<int>(P.size()) != n * n || static_cast<int>(dP.size()) != n * n) return 3;
        for (double v : P)
          if (!std::isfinite(v)) return 4;
      }
    }
  }
  for (int n : {3, 8, 65, 2049}) {
    const double s = sigma_phi(n);
    if (!(s > 0.0 && s < 0.5)) return 5;
  }
  for (double v : {0.0, 1e-12, -1e-3, -3.0, -700.0}) {
    if (!std::isfinite(phi1(v)) || !std::isfinite(phi2(v))) return 6;
  }
  std::printf("host set-up ok, worst eigen residual %.3e\n", worst);
  return worst < 1e-11 ? 0 : 7;
}
