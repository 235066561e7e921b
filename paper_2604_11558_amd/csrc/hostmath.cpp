// Host-side FP64 set-up: grids, 1D operators, eigen-decompositions, phi_1.
#include "hostmath.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <stdexcept>

namespace tg {

static const double kPi = 3.14159265358979323846264338327950288;

std::vector<double> Tridiag::dense() const {
  std::vector<double> A(static_cast<size_t>(n) * n, 0.0);
  for (int r = 0; r < n; ++r) {
    A[r * n + r] += dg[r];
    if (r > 0) A[r * n + r - 1] += lo[r];
    if (r + 1 < n) A[r * n + r + 1] += up[r];
  }
  if (periodic) {
    A[0 * n + (n - 1)] += lo[0];
    A[(n - 1) * n + 0] += up[n - 1];
  }
  return A;
}

// Appendix A: f(x) = cot(x pi / (n-1+2x)) - 2 (n-1+2x) / pi is strictly
// decreasing on (0, 1/2), +inf at 0+ and negative at 1/2; bisect to the
// last representable interval.
double sigma_phi(int n) {
  auto f = [n](double x) {
    const double m = (n - 1) + 2.0 * x;
    return 1.0 / std::tan(x * kPi / m) - 2.0 * m / kPi;
  };
  double a = 1e-300, b = 0.5;
  for (int it = 0; it < 2000; ++it) {
    const double c = 0.5 * (a + b);
    if (c <= a || c >= b) break;
    if (f(c) > 0.0) a = c; else b = c;
  }
  return std::fabs(f(a)) < std::fabs(f(b)) ? a : b;
}

std::vector<double> coord_grid(Coord c, int n, double extent, double lam) {
  std::vector<double> g(n);
  switch (c) {
    case RHO2: {  // half-point grid, h = rho_* / (n - 1/2)
      const double h = extent / (n - 0.5);
      for (int i = 0; i < n; ++i) g[i] = 0.5 * h + i * h;
      break;
    }
    case RHO3: {  // rho_i = i h, h = rho_* / n
      const double h = extent / n;
      for (int i = 0; i < n; ++i) g[i] = (i + 1) * h;
      break;
    }
    case RHO_LAMBDA: {  // rho_i = (1 - lambda) h / 2 + (i - 1) h, h = rho_* / (n + (1 - lambda) / 2)
      const double s = 0.5 * (1.0 - lam);
      const double h = extent / (n + s);
      for (int i = 0; i < n; ++i) g[i] = (s + i) * h;
      break;
    }
    case THETA: {  // theta_j = j h, h = 2 pi / n
      const double h = 2.0 * kPi / n;
      for (int i = 0; i < n; ++i) g[i] = (i + 1) * h;
      break;
    }
    case PHI: {  // phi_k = (sigma + k - 1) h, h = pi / (n - 1 + 2 sigma)
      const double s = sigma_phi(n);
      const double h = kPi / (n - 1 + 2.0 * s);
      for (int i = 0; i < n; ++i) g[i] = (s + i) * h;
      break;
    }
    case ZED: {  // z_k = (k - 1) h, h = z_* / n
      const double h = extent / n;
      for (int i = 0; i < n; ++i) g[i] = i * h;
      break;
    }
  }
  return g;
}

std::vector<double> coord_weights(Coord c, int n, double extent, double lam) {
  std::vector<double> w(n);
  if (c == THETA) {
    for (int i = 0; i < n; ++i) w[i] = 2.0 * kPi / n;
    return w;
  }
  const auto g = coord_grid(c, n, extent, lam);
  const double hi = c == PHI ? kPi : extent;  // every other range starts at 0
  // integral of the volume-element factor from 0 to x
  auto prim = [c](double x) {
    switch (c) {
      case RHO2:
      case RHO_LAMBDA: return 0.5 * x * x;
      case RHO3: return x * x * x / 3.0;
      case PHI: return 1.0 - std::cos(x);
      default: return x;
    }
  };
  double left = 0.0;
  for (int i = 0; i < n; ++i) {
    const double right = i + 1 < n ? 0.5 * (g[i] + g[i + 1]) : hi;
    w[i] = prim(right) - prim(left);
    left = right;
  }
  return w;
}

Tridiag coord_operator(Coord c, int n, double extent, double lam) {
  if (n < 3) throw std::invalid_argument("grid needs at least 3 points per coordinate");
  Tridiag T;
  T.n = n;
  T.lo.assign(n, 0.0);
  T.dg.assign(n, 0.0);
  T.up.assign(n, 0.0);
  // b(l), c(l) below use the paper's 1-based l = 1..n-1:
  // A[l][l+1] = b_l (row l-1 here, "up"), A[l+1][l] = c_l (row l here, "lo").
  auto set_bc = [&](auto b, auto cc, double a) {
    for (int r = 0; r < n; ++r) T.dg[r] = a;
    for (int l = 1; l <= n - 1; ++l) {
      T.up[l - 1] = b(l);
      T.lo[l] = cc(l);
    }
  };
  switch (c) {
    case RHO2: {
      const double h = extent / (n - 0.5), h2 = h * h;
      set_bc([&](int l) { return 2.0 * l / ((2.0 * l - 1.0) * h2); },
             [&](int l) { return l == n - 1 ? 2.0 / h2 : 2.0 * l / ((2.0 * l + 1.0) * h2); },
             -2.0 / h2);
      break;
    }
    case RHO_LAMBDA: {
      // eq. (A_lambda), 1-based l: a_l = -2 / ((s+l-1)^lam h^(2+lam)),
      // b_l = (1-lam+l-1) / ((s+l-1)^(1+lam) h^(2+lam)), c_l = l / ((s+l)^(1+lam) h^(2+lam))
      const double s = 0.5 * (1.0 - lam);
      const double h = extent / (n + s), hp = std::pow(h, 2.0 + lam);
      for (int r = 0; r < n; ++r) T.dg[r] = -2.0 / (std::pow(s + r, lam) * hp);
      for (int l = 1; l <= n - 1; ++l) {
        T.up[l - 1] = (1.0 - lam + l - 1.0) / (std::pow(s + l - 1.0, 1.0 + lam) * hp);
        T.lo[l] = l / (std::pow(s + l, 1.0 + lam) * hp);
      }
      break;
    }
    case RHO3: {
      const double h = extent / n, h2 = h * h;
      set_bc([&](int l) { return (l + 1.0) / (l * h2); },
             [&](int l) { return l == n - 1 ? 2.0 / h2 : l / ((l + 1.0) * h2); }, -2.0 / h2);
      break;
    }
    case PHI: {
      const double s = sigma_phi(n);
      const double h = kPi / (n - 1 + 2.0 * s), h2 = h * h;
      auto b = [&](int l) { return 1.0 / h2 + 1.0 / std::tan((s + l - 1) * h) / (2.0 * h); };
      set_bc(b, [&](int l) { return b(n - l); }, -2.0 / h2);
      break;
    }
    case ZED: {
      const double h = extent / n, h2 = h * h;
      set_bc([&](int l) { return l == 1 ? 2.0 / h2 : 1.0 / h2; }, [&](int) { return 1.0 / h2; },
             -2.0 / h2);
      break;
    }
    case THETA: {
      const double h = 2.0 * kPi / n, h2 = h * h;
      T.periodic = true;
      for (int r = 0; r < n; ++r) {
        T.dg[r] = -2.0 / h2;
        T.lo[r] = 1.0 / h2;
        T.up[r] = 1.0 / h2;
      }
      break;
    }
  }
  return T;
}

// Implicit QL on a symmetric tridiagonal matrix: repeatedly pick the
// leading unreduced block [l, m], apply a Wilkinson-shifted QL sweep of
// Givens rotations chased from the bottom of the block upwards, and
// accumulate the rotations into Z.  This is the published implicit QL
// algorithm with Wilkinson shifts of Bowdler, Martin, Reinsch and
// Wilkinson ("The QR and QL algorithms for symmetric matrices", Numer.
// Math. 11 (1968); the tql2 procedure of the Handbook for Automatic
// Computation, vol. II, and of EISPACK), restated here.
bool symtridiag_ql(std::vector<double>& d, std::vector<double> e, std::vector<double>& Z) {
  const int n = static_cast<int>(d.size());
  e.resize(n, 0.0);
  e[n - 1] = 0.0;
  Z.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) Z[i * n + i] = 1.0;
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (iter > 100) return false;
      // Wilkinson shift from the leading 2x2 block
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        const double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {  // underflow: split the block here
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          const double zf = Z[k * n + i + 1];
          Z[k * n + i + 1] = s * Z[k * n + i] + c * zf;
          Z[k * n + i] = c * Z[k * n + i] - s * zf;
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

Eig eig_tridiag(const Tridiag& A) {
  if (A.periodic) throw std::invalid_argument("eig_tridiag: periodic operator");
  const int n = A.n;
  // Proposition 1: xi_1 = 1, xi_{l+1} = xi_l sqrt(c_l / b_l); S = Xi^-1 A Xi has
  // diagonal a_l and symmetric off-diagonal sqrt(b_l c_l).
  std::vector<double> xi(n, 1.0), d(A.dg), e(n, 0.0);
  for (int l = 0; l + 1 < n; ++l) {
    const double b = A.up[l], c = A.lo[l + 1];
    xi[l + 1] = xi[l] * std::sqrt(c / b);
    e[l] = std::sqrt(b * c);
  }
  std::vector<double> Q;
  if (!symtridiag_ql(d, e, Q)) throw std::runtime_error("eigen-solver did not converge");
  // Zero row sums (Neumann and pole-free ends): the constants are an exact
  // eigenvector with eigenvalue 0, which the iteration returns only to
  // O(eps ||A||); scaled by tau d / rho^2 that residue would perturb the
  // constant mode, so the eigenvalue nearest 0 is set to 0 exactly.
  double amax = 0.0, rmax = 0.0;
  for (int r = 0; r < n; ++r) {
    amax = std::max(amax, std::fabs(A.dg[r]));
    rmax = std::max(rmax, std::fabs(A.lo[r] + A.dg[r] + A.up[r]));
  }
  if (rmax <= 1e-12 * amax) {
    int k = 0;
    for (int j = 1; j < n; ++j)
      if (std::fabs(d[j]) < std::fabs(d[k])) k = j;
    if (std::fabs(d[k]) <= 1e-10 * amax) d[k] = 0.0;
  }
  Eig out;
  out.n = n;
  out.lam = d;
  out.V.resize(static_cast<size_t>(n) * n);
  out.Vinv.resize(static_cast<size_t>(n) * n);
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < n; ++j) {
      out.V[r * n + j] = xi[r] * Q[r * n + j];
      out.Vinv[j * n + r] = Q[r * n + j] / xi[r];
    }
  return out;
}

// Circulant A_theta: eigenvectors cos(m theta_j), sin(m theta_j) with
// eigenvalue -(4/h^2) sin^2(m pi / n), plus the constant and, for even n,
// the alternating vector.
Eig eig_theta(int n) {
  const double h = 2.0 * kPi / n;
  Eig out;
  out.n = n;
  out.lam.assign(n, 0.0);
  out.V.assign(static_cast<size_t>(n) * n, 0.0);
  int col = 0;
  auto lam_of = [&](int m) {
    const double s = std::sin(m * kPi / n);
    return -4.0 / (h * h) * s * s;
  };
  const double c0 = 1.0 / std::sqrt(static_cast<double>(n));
  const double c1 = std::sqrt(2.0 / n);
  for (int j = 0; j < n; ++j) out.V[j * n + col] = c0;
  out.lam[col++] = 0.0;
  for (int m = 1; 2 * m < n; ++m) {
    for (int j = 0; j < n; ++j) {
      // theta_j = (j+1) h; reduce the angle index mod n for accuracy
      const long idx = (static_cast<long>(m) * (j + 1)) % n;
      const double a = 2.0 * kPi * idx / n;
      out.V[j * n + col] = c1 * std::cos(a);
      out.V[j * n + col + 1] = c1 * std::sin(a);
    }
    out.lam[col] = out.lam[col + 1] = lam_of(m);
    col += 2;
  }
  if (n % 2 == 0) {
    for (int j = 0; j < n; ++j) out.V[j * n + col] = ((j + 1) % 2 == 0) ? c0 : -c0;
    out.lam[col++] = -4.0 / (h * h);
  }
  out.Vinv.resize(static_cast<size_t>(n) * n);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) out.Vinv[c * n + r] = out.V[r * n + c];
  return out;
}

double phi1(double x) { return x == 0.0 ? 1.0 : std::expm1(x) / x; }

double phi2(double x) {
  if (std::fabs(x) < 1e-3) return 0.5 + x / 6.0 + x * x / 24.0 + x * x * x / 120.0;
  return (std::expm1(x) - x) / (x * x);
}

static std::vector<double> sandwich(const Eig& e, const std::vector<double>& diag) {
  const int n = e.n;
  std::vector<double> out(static_cast<size_t>(n) * n, 0.0);
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < n; ++j) {
      const double v = e.V[r * n + j] * diag[j];
      if (v == 0.0) continue;
      const double* vi = &e.Vinv[static_cast<size_t>(j) * n];
      double* o = &out[static_cast<size_t>(r) * n];
      for (int c = 0; c < n; ++c) o[c] += v * vi[c];
    }
  return out;
}

std::vector<double> phi1_from_eig(const Eig& e, double c) {
  std::vector<double> dg(e.n);
  for (int j = 0; j < e.n; ++j) dg[j] = phi1(c * e.lam[j]);
  return sandwich(e, dg);
}

// d/dd phi_1(d c A) = c A (phi_1 - phi_2)(d c A); here c is the full
// multiplier (tau d) and the result is scaled by c/d outside.
std::vector<double> dphi1_from_eig(const Eig& e, double c) {
  std::vector<double> dg(e.n);
  for (int j = 0; j < e.n; ++j) {
    const double x = c * e.lam[j];
    dg[j] = e.lam[j] * (phi1(x) - phi2(x));
  }
  return sandwich(e, dg);
}

}  // namespace tg
