// C interface: grids, plans (FP64 factor precompute + upload) and the step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <exception>
#include <limits>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tgexp.h"
#include "plan.hpp"

namespace {

thread_local std::string g_last_error = "no error";

struct Fail : std::runtime_error {
  int code;
  Fail(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define TG_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) throw Fail((code), (msg)); \
  } while (0)

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  // the runtime also keeps the error as the thread's last error, which the
  // next launch's hipGetLastError would report again: read it off here
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory)
    throw Fail(TG_ENOMEM, std::string(what) + ": " + hipGetErrorString(e));
  throw Fail(TG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Fail& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return TG_ENOMEM;
  } catch (const std::invalid_argument& e) {
    g_last_error = e.what();
    return TG_EINVAL;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return TG_EINVAL;
  }
}

// Host staging of the plan's small device arrays and factors: every block
// is 256-byte aligned inside one allocation.
struct Arena {
  std::vector<char> bytes;
  size_t add(const void* src, size_t n) {
    size_t off = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(off + n);
    if (n) std::memcpy(bytes.data() + off, src, n);
    return off;
  }
  size_t add_d(const std::vector<double>& v) { return add(v.data(), v.size() * sizeof(double)); }
  template <typename T>
  size_t add_t(const std::vector<double>& v) {
    std::vector<T> t(v.begin(), v.end());
    return add(t.data(), t.size() * sizeof(T));
  }
};

// Round to the nearest bf16 (ties to even); returns the 16-bit pattern.
uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
double bf16_value(uint16_t b) {
  uint32_t u = static_cast<uint32_t>(b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

int bf16_terms(int precision) { return precision == TG_BF16X2 ? 2 : (precision == TG_BF16X3 ? 3 : 0); }

}  // namespace

// ---------------------------------------------------------------------------
double tg_grid_s::extent_of(int mode) const {
  switch (coord[mode]) {
    case tg::RHO2:
    case tg::RHO3:
    case tg::RHO_LAMBDA: return extent[0];
    case tg::ZED: return extent[1];
    default: return 1.0;
  }
}
tg::Tridiag tg_grid_s::op(int mode) const { return tg::coord_operator(coord[mode], n[mode], extent_of(mode), lam); }
std::vector<double> tg_grid_s::coords(int mode) const {
  return tg::coord_grid(coord[mode], n[mode], extent_of(mode), lam);
}
tg::Eig tg_grid_s::eig(int mode) const {
  if (coord[mode] == tg::THETA) return tg::eig_theta(n[mode]);
  return tg::eig_tridiag(op(mode));
}

extern "C" {

const char* tg_last_error(void) { return g_last_error.c_str(); }
int tg_version(void) { return 1; }

int tg_grid_create(int32_t geometry, const int32_t* n, const double* extent, tg_grid* out) {
  return guarded([&] {
    TG_REQUIRE(n && out, TG_EINVAL, "tg_grid_create: null pointer");
    TG_REQUIRE(geometry != TG_DISK_LAMBDA || extent, TG_EINVAL,
               "tg_grid_create: the anomalous disk needs extent = (rho_*, lambda)");
    auto g = new tg_grid_s();
    g->geometry = geometry;
    switch (geometry) {
      case TG_DISK: g->ndim = 2; g->coord[0] = tg::RHO2; g->coord[1] = tg::THETA; break;
      case TG_SPHERE: g->ndim = 2; g->coord[0] = tg::THETA; g->coord[1] = tg::PHI; break;
      case TG_BALL: g->ndim = 3; g->coord[0] = tg::RHO3; g->coord[1] = tg::THETA; g->coord[2] = tg::PHI; break;
      case TG_CYLINDER: g->ndim = 3; g->coord[0] = tg::RHO2; g->coord[1] = tg::THETA; g->coord[2] = tg::ZED; break;
      case TG_DISK_LAMBDA: g->ndim = 2; g->coord[0] = tg::RHO_LAMBDA; g->coord[1] = tg::THETA; break;
      default: delete g; throw Fail(TG_EINVAL, "tg_grid_create: unknown geometry");
    }
    for (int m = 0; m < g->ndim; ++m) {
      if (n[m] < 3 || n[m] > 65536) {
        delete g;
        throw Fail(TG_EINVAL, "tg_grid_create: each n must be in [3, 65536]");
      }
      g->n[m] = n[m];
    }
    if (geometry == TG_DISK_LAMBDA) {
      // extent = (rho_*, lambda); the grid needs (1 - lambda) / 2 > 0
      if (!(extent[0] > 0.0) || !(extent[1] < 1.0) || !std::isfinite(extent[1])) {
        delete g;
        throw Fail(TG_EINVAL, "tg_grid_create: anomalous disk needs rho_* > 0 and lambda < 1");
      }
      g->extent[0] = extent[0];
      g->lam = extent[1];
    } else if (extent) {
      if (!(extent[0] > 0.0) || !(extent[1] > 0.0)) {
        delete g;
        throw Fail(TG_EINVAL, "tg_grid_create: extents must be positive");
      }
      g->extent[0] = extent[0];
      g->extent[1] = extent[1];
    }
    *out = g;
    return TG_OK;
  });
}

int tg_grid_destroy(tg_grid g) {
  delete g;
  return TG_OK;
}

int tg_grid_dims(tg_grid g, int32_t* ndim, int32_t* n) {
  return guarded([&] {
    TG_REQUIRE(g && ndim && n, TG_EINVAL, "tg_grid_dims: null pointer");
    *ndim = g->ndim;
    for (int m = 0; m < 3; ++m) n[m] = g->n[m];
    return TG_OK;
  });
}

static int check_mode(tg_grid g, int32_t mode) {
  TG_REQUIRE(g, TG_EINVAL, "null grid");
  TG_REQUIRE(mode >= 1 && mode <= g->ndim, TG_EINVAL, "mode out of range");
  return mode - 1;
}

int tg_grid_coords(tg_grid g, int32_t mode, double* out) {
  return guarded([&] {
    const int m = check_mode(g, mode);
    TG_REQUIRE(out, TG_EINVAL, "null output");
    auto c = g->coords(m);
    std::memcpy(out, c.data(), c.size() * sizeof(double));
    return TG_OK;
  });
}

int tg_grid_operator(tg_grid g, int32_t mode, double* lo, double* diag, double* up) {
  return guarded([&] {
    const int m = check_mode(g, mode);
    TG_REQUIRE(lo && diag && up, TG_EINVAL, "null output");
    auto T = g->op(m);
    std::memcpy(lo, T.lo.data(), T.n * sizeof(double));
    std::memcpy(diag, T.dg.data(), T.n * sizeof(double));
    std::memcpy(up, T.up.data(), T.n * sizeof(double));
    return TG_OK;
  });
}

int tg_grid_eig(tg_grid g, int32_t mode, double* lam, double* V, double* Vinv) {
  return guarded([&] {
    const int m = check_mode(g, mode);
    TG_REQUIRE(lam && V && Vinv, TG_EINVAL, "null output");
    auto e = g->eig(m);
    std::memcpy(lam, e.lam.data(), e.n * sizeof(double));
    std::memcpy(V, e.V.data(), e.V.size() * sizeof(double));
    std::memcpy(Vinv, e.Vinv.data(), e.Vinv.size() * sizeof(double));
    return TG_OK;
  });
}

int tg_grid_phi1(tg_grid g, int32_t mode, double c, double* out) {
  return guarded([&] {
    const int m = check_mode(g, mode);
    TG_REQUIRE(out && std::isfinite(c), TG_EINVAL, "bad argument");
    auto P = tg::phi1_from_eig(g->eig(m), c);
    std::memcpy(out, P.data(), P.size() * sizeof(double));
    return TG_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
namespace {

std::vector<double> default_reference(int reaction, int ns, const double* rp) {
  std::vector<double> w(ns, 0.0);
  if (reaction == TG_REACT_SCHNAKENBERG || reaction == TG_REACT_SCHNAKENBERG_SCALED) {
    const double a = rp[0], b = rp[1];
    w[0] = a + b;
    w[1] = b / ((a + b) * (a + b));
  } else if (reaction == TG_REACT_AIS3) {
    const double a = rp[0], b = rp[1], kap = rp[2];
    const double ue = (-1.0 + std::sqrt(1.0 + 4.0 * kap * (a + b))) / (2.0 * kap);
    w[0] = ue;
    w[1] = b / (ue * ue);
    w[2] = ue;
  } else if (reaction == TG_REACT_LINEAR) {
    for (int s = 0; s < ns; ++s) w[s] = rp[2 * s + 1];
  } else if (reaction == TG_REACT_DIB) {
    w[0] = 0.0;
    w[1] = rp[4];
  }
  return w;
}

std::vector<double> reaction_at(int reaction, int ns, const double* rp, const double* w) {
  std::vector<double> g(ns, 0.0);
  if (reaction == TG_REACT_SCHNAKENBERG) {
    const double u2v = w[0] * w[0] * w[1];
    g[0] = rp[0] - w[0] + u2v;
    g[1] = rp[1] - u2v;
  } else if (reaction == TG_REACT_SCHNAKENBERG_SCALED) {
    const double u2v = w[0] * w[0] * w[1];
    g[0] = rp[2] * (rp[0] - w[0] + u2v);
    g[1] = rp[2] * (rp[1] - u2v);
  } else if (reaction == TG_REACT_AIS3) {
    const double u2v = w[0] * w[0] * w[1];
    g[0] = rp[0] - w[0] + u2v - rp[2] * w[0] * w[2];
    g[1] = rp[1] - u2v;
    g[2] = rp[3] * (w[0] - w[2]);
  }
  // TG_REACT_LINEAR and TG_REACT_DIB: the stencil launch evaluates the whole
  // kinetics at w_ref + deviation, so no value at the reference is kept
  return g;
}

constexpr size_t kLdsLimit = 160 * 1024;

// an autotuning candidate replaces the current choice only when it is at
// least 2% faster, so that timing noise does not flip between near-equal ones
constexpr double kTuneGain = 0.98;

// Launch-timing hook (tg_run_timed): when set, an event is recorded on the
// launch stream before every kernel launch of a step.
struct LaunchEvents {
  std::vector<hipEvent_t> ev;
  size_t next = 0;
};
thread_local LaunchEvents* g_launch_events = nullptr;
inline void mark_launch(hipStream_t st) {
  if (!g_launch_events) return;
  TG_REQUIRE(g_launch_events->next < g_launch_events->ev.size(), TG_EINVAL, "launch timing: too many launches");
  hip_check(hipEventRecord(g_launch_events->ev[g_launch_events->next++], st), "event record");
}

// Pick the GEMM tile: the largest tile that still gives about two
// workgroups per compute unit, else the smallest.
int pick_tile(int M, int N, int64_t batches) {
  const int64_t want = 512;
  const int tms[4] = {64, 32, 64, 32}, tns[4] = {64, 64, 32, 32};
  for (int t = 0; t < 4; ++t) {
    const int64_t wg = static_cast<int64_t>((M + tms[t] - 1) / tms[t]) * ((N + tns[t] - 1) / tns[t]) * batches;
    if (wg >= want) return t;
  }
  return 3;
}

template <typename T>
void build_plan(tg_plan_s* P) {
  const tg_grid_s& G = P->grid;
  const int nd = G.ndim;
  int dev = 0, num_cus = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  hip_check(hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
  num_cus = std::max(num_cus, 1);
  const int n1 = G.n[0], n2 = G.n[1], n3 = nd == 3 ? G.n[2] : 1;
  const int nslab = P->nslab;
  const double tau = P->tau;
  Arena ar;
  // stencil coefficients and scales: [3 modes][3][nmax]
  const int nmax = std::max(n1, std::max(n2, n3));
  P->nmax = nmax;
  std::vector<double> coef(9 * nmax, 0.0), scale(9 * nmax, 1.0);
  P->periodic_mask = 0;
  for (int m = 0; m < nd; ++m) {
    auto T_ = G.op(m);
    if (T_.periodic) P->periodic_mask |= 1 << m;
    for (int r = 0; r < T_.n; ++r) {
      coef[(m * 3 + 0) * nmax + r] = T_.lo[r];
      coef[(m * 3 + 1) * nmax + r] = T_.dg[r];
      coef[(m * 3 + 2) * nmax + r] = T_.up[r];
    }
  }
  P->scale_mask = 0;
  auto set_scale = [&](int mode, int coord, const std::vector<double>& v) {
    for (size_t r = 0; r < v.size(); ++r) scale[(mode * 3 + coord) * nmax + r] *= v[r];
    P->scale_mask |= 1 << (3 * mode + coord);
  };
  auto inv2 = [](const std::vector<double>& x) {
    std::vector<double> y(x.size());
    for (size_t i = 0; i < x.size(); ++i) y[i] = 1.0 / (x[i] * x[i]);
    return y;
  };
  auto sininv2 = [](const std::vector<double>& x, double s) {
    std::vector<double> y(x.size());
    for (size_t i = 0; i < x.size(); ++i) {
      const double si = std::sin(x[i]);
      y[i] = s / (si * si);
    }
    return y;
  };
  // per-slab tau * d_s
  std::vector<double> cs(nslab);
  for (int s = 0; s < nslab; ++s) cs[s] = tau * P->diff[s];
  // distinct factors: per species if every instance shares d, else per slab
  bool shared = true;
  for (int b = 1; b < P->batch && shared; ++b)
    for (int s = 0; s < P->ns; ++s)
      if (P->diff[b * P->ns + s] != P->diff[s]) shared = false;
  const int fmod = shared ? P->ns : nslab;
  auto per_slab_factor = [&](const tg::Eig& e, double extra) {
    std::vector<double> all;
    all.reserve(static_cast<size_t>(fmod) * e.n * e.n);
    for (int f = 0; f < fmod; ++f) {
      auto Pm = tg::phi1_from_eig(e, cs[f] * extra);
      all.insert(all.end(), Pm.begin(), Pm.end());
    }
    return all;
  };

  struct PendingOp {
    int mode, epi, fmod;
    size_t L, pm = SIZE_MAX, pn = SIZE_MAX, pb = SIZE_MAX;
    size_t LT = SIZE_MAX, dL = SIZE_MAX;
  };
  // transposed blocks of a factor stack (n x n blocks)
  auto add_transposed = [&](const std::vector<double>& stack, int n) {
    std::vector<double> t(stack.size());
    const size_t sq = static_cast<size_t>(n) * n;
    for (size_t b = 0; b < stack.size() / sq; ++b)
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) t[b * sq + c * n + r] = stack[b * sq + r * n + c];
    return ar.add_t<T>(t);
  };
  // d/dd phi_1(tau d extra A) per block = tau extra V diag(lam (phi_1 - phi_2)(c lam)) V^-1
  auto per_slab_dfactor = [&](const tg::Eig& e, double extra) {
    std::vector<double> all;
    for (int f = 0; f < fmod; ++f) {
      auto D = tg::dphi1_from_eig(e, cs[f] * extra);
      for (double& x : D) x *= tau * extra;
      all.insert(all.end(), D.begin(), D.end());
    }
    return all;
  };
  std::vector<PendingOp> ops;
  const double s2 = (G.geometry == TG_SPHERE) ? 1.0 / (G.extent[0] * G.extent[0]) : 1.0;

  // Fused route: factors zero-padded to a multiple of 128 in both dimensions
  // so that 16-wide vector loads over the padded k range stay in bounds.
  struct PadF {
    size_t off = SIZE_MAX;
    int ld = 0, fmod = 1;
  };
  const int nterms = bf16_terms(P->precision);
  auto addpad = [&](const std::vector<double>& stack, int n, int blocks) {
    PadF f;
    f.ld = (n + 127) / 128 * 128;
    f.fmod = blocks;
    std::vector<double> pad(static_cast<size_t>(blocks) * f.ld * f.ld, 0.0);
    for (int b = 0; b < blocks; ++b)
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c)
          pad[(static_cast<size_t>(b) * f.ld + r) * f.ld + c] = stack[(static_cast<size_t>(b) * n + r) * n + c];
    if (nterms == 0) {
      f.off = ar.add_t<T>(pad);
      return f;
    }
    // split-bf16 stack: block b, term t at (b * nterms + t) * ld * ld
    const size_t sq = static_cast<size_t>(f.ld) * f.ld;
    std::vector<uint16_t> bf(static_cast<size_t>(blocks) * nterms * sq);
    for (int b = 0; b < blocks; ++b)
      for (size_t e = 0; e < sq; ++e) {
        double r = pad[b * sq + e];
        for (int t = 0; t < nterms; ++t) {
          const uint16_t h = bf16_bits(static_cast<float>(r));
          bf[(static_cast<size_t>(b) * nterms + t) * sq + e] = h;
          r -= bf16_value(h);
        }
      }
    f.off = ar.add(bf.data(), bf.size() * sizeof(uint16_t));
    return f;
  };
  struct FSpec {
    int kind = 0, mode = 1, nm = 0, na = 1, nb = 1, rows = 0;
    int sandwich = 0, phi = 0, stencil = 0, plane = 0;
    PadF L1, L2, Pf;
    size_t pm = SIZE_MAX, pn = SIZE_MAX, pb = SIZE_MAX;
  };
  std::vector<FSpec> fspecs;

  if (G.geometry == TG_DISK || G.geometry == TG_DISK_LAMBDA) {  // eq. (ee_disk)
    // D_rho: rho^-2, or rho^(-2-lambda) for the anomalous operator (Section 5.3)
    auto rinv2 = inv2(G.coords(0));
    if (G.geometry == TG_DISK_LAMBDA) {
      const auto r = G.coords(0);
      for (size_t i = 0; i < rinv2.size(); ++i) rinv2[i] = std::pow(r[i], -2.0 - G.lam);
    }
    set_scale(1, 0, rinv2);
    auto et = G.eig(1);
    auto er = G.eig(0);
    PendingOp o1{2, tg::EPI_PHI, 1, ar.add_t<T>(et.Vinv)};
    o1.pm = ar.add_d(et.lam);
    o1.pn = ar.add_d(rinv2);
    PendingOp o2{2, tg::EPI_STORE, 1, ar.add_t<T>(et.V)};
    auto Pr = per_slab_factor(er, 1.0);
    PendingOp o3{1, tg::EPI_UPDATE, fmod, ar.add_t<T>(Pr)};
    o1.LT = add_transposed(et.Vinv, n2);
    o2.LT = add_transposed(et.V, n2);
    o3.LT = add_transposed(Pr, n1);
    o3.dL = ar.add_t<T>(per_slab_dfactor(er, 1.0));
    ops = {o1, o2, o3};
    FSpec a;  // theta sandwich with the stencil, then rho (plane tail when it fits)
    a.mode = 2; a.nm = n2; a.na = n1; a.nb = 1;
    a.sandwich = 1; a.phi = 1; a.stencil = 1; a.plane = 1;
    a.L1 = addpad(et.Vinv, n2, 1); a.L2 = addpad(et.V, n2, 1); a.Pf = addpad(Pr, n1, fmod);
    a.pm = o1.pm; a.pn = o1.pn;
    fspecs = {a};
  } else if (G.geometry == TG_SPHERE) {  // eq. (ee_sphere)
    auto sph = sininv2(G.coords(1), s2);
    set_scale(0, 1, sph);
    set_scale(1, 0, std::vector<double>(n1, s2));
    auto et = G.eig(0);
    auto ep = G.eig(1);
    auto Pp = per_slab_factor(ep, s2);
    PendingOp o1{2, tg::EPI_STORE, fmod, ar.add_t<T>(Pp)};
    PendingOp o2{1, tg::EPI_PHI, 1, ar.add_t<T>(et.Vinv)};
    o2.pm = ar.add_d(sph);
    o2.pn = ar.add_d(et.lam);
    PendingOp o3{1, tg::EPI_UPDATE, 1, ar.add_t<T>(et.V)};
    o1.LT = add_transposed(Pp, n2);
    o1.dL = ar.add_t<T>(per_slab_dfactor(ep, s2));
    o2.LT = add_transposed(et.Vinv, n1);
    o3.LT = add_transposed(et.V, n1);
    ops = {o1, o2, o3};
    FSpec a;  // phi product with the stencil
    a.mode = 2; a.nm = n2; a.na = n1; a.nb = 1; a.stencil = 1;
    a.L1 = addpad(per_slab_factor(ep, s2), n2, fmod);
    FSpec b;  // theta sandwich + update
    b.kind = 1; b.mode = 1; b.nm = n1; b.rows = n2; b.sandwich = 1; b.phi = 1;
    b.L1 = addpad(et.Vinv, n1, 1); b.L2 = addpad(et.V, n1, 1);
    b.pm = o2.pm; b.pn = o2.pn;
    fspecs = {a, b};
  } else if (G.geometry == TG_BALL) {  // eq. (ee_ball)
    auto rinv2 = inv2(G.coords(0));
    auto sph = sininv2(G.coords(2), 1.0);
    set_scale(1, 0, rinv2);
    set_scale(1, 2, sph);
    set_scale(2, 0, rinv2);
    auto er = G.eig(0);
    auto et = G.eig(1);
    auto ep = G.eig(2);
    std::vector<double> rinv2_a(static_cast<size_t>(n1) * n2);
    for (int j = 0; j < n2; ++j)
      for (int i = 0; i < n1; ++i) rinv2_a[j * n1 + i] = rinv2[i];
    PendingOp o1{3, tg::EPI_PHI, 1, ar.add_t<T>(ep.Vinv)};
    o1.pm = ar.add_d(ep.lam);
    o1.pn = ar.add_d(rinv2_a);
    PendingOp o2{3, tg::EPI_STORE, 1, ar.add_t<T>(ep.V)};
    PendingOp o3{2, tg::EPI_PHI, 1, ar.add_t<T>(et.Vinv)};
    o3.pm = ar.add_d(et.lam);
    o3.pn = ar.add_d(rinv2);
    o3.pb = ar.add_d(sph);
    PendingOp o4{2, tg::EPI_STORE, 1, ar.add_t<T>(et.V)};
    auto Pr = per_slab_factor(er, 1.0);
    PendingOp o5{1, tg::EPI_UPDATE, fmod, ar.add_t<T>(Pr)};
    o1.LT = add_transposed(ep.Vinv, n3);
    o2.LT = add_transposed(ep.V, n3);
    o3.LT = add_transposed(et.Vinv, n2);
    o4.LT = add_transposed(et.V, n2);
    o5.LT = add_transposed(Pr, n1);
    o5.dL = ar.add_t<T>(per_slab_dfactor(er, 1.0));
    ops = {o1, o2, o3, o4, o5};
    FSpec a;  // phi sandwich with the stencil
    a.mode = 3; a.nm = n3; a.na = n1 * n2; a.nb = 1;
    a.sandwich = 1; a.phi = 1; a.stencil = 1;
    a.L1 = addpad(ep.Vinv, n3, 1); a.L2 = addpad(ep.V, n3, 1);
    a.pm = o1.pm; a.pn = o1.pn;
    FSpec b;  // theta sandwich + rho product + update over (rho, theta) planes
    b.mode = 2; b.nm = n2; b.na = n1; b.nb = n3;
    b.sandwich = 1; b.phi = 1; b.plane = 1;
    b.L1 = addpad(et.Vinv, n2, 1); b.L2 = addpad(et.V, n2, 1); b.Pf = addpad(Pr, n1, fmod);
    b.pm = o3.pm; b.pn = o3.pn; b.pb = o3.pb;
    fspecs = {a, b};
  } else {  // TG_CYLINDER, eq. (ee_cylinder)
    auto rinv2 = inv2(G.coords(0));
    set_scale(1, 0, rinv2);
    auto er = G.eig(0);
    auto et = G.eig(1);
    auto ez = G.eig(2);
    auto Pz = per_slab_factor(ez, 1.0);
    auto Pr = per_slab_factor(er, 1.0);
    PendingOp o1{3, tg::EPI_STORE, fmod, ar.add_t<T>(Pz)};
    PendingOp o2{2, tg::EPI_PHI, 1, ar.add_t<T>(et.Vinv)};
    o2.pm = ar.add_d(et.lam);
    o2.pn = ar.add_d(rinv2);
    PendingOp o3{2, tg::EPI_STORE, 1, ar.add_t<T>(et.V)};
    PendingOp o4{1, tg::EPI_UPDATE, fmod, ar.add_t<T>(Pr)};
    o1.LT = add_transposed(Pz, n3);
    o1.dL = ar.add_t<T>(per_slab_dfactor(ez, 1.0));
    o2.LT = add_transposed(et.Vinv, n2);
    o3.LT = add_transposed(et.V, n2);
    o4.LT = add_transposed(Pr, n1);
    o4.dL = ar.add_t<T>(per_slab_dfactor(er, 1.0));
    ops = {o1, o2, o3, o4};
    FSpec a;  // z product with the stencil
    a.mode = 3; a.nm = n3; a.na = n1 * n2; a.nb = 1; a.stencil = 1;
    a.L1 = addpad(Pz, n3, fmod);
    FSpec b;  // theta sandwich + rho product + update over (rho, theta) planes
    b.mode = 2; b.nm = n2; b.na = n1; b.nb = n3;
    b.sandwich = 1; b.phi = 1; b.plane = 1;
    b.L1 = addpad(et.Vinv, n2, 1); b.L2 = addpad(et.V, n2, 1); b.Pf = addpad(Pr, n1, fmod);
    b.pm = o2.pm; b.pn = o2.pn;
    fspecs = {a, b};
  }

  // transposed operators: (A^T)[r][r-1] = A[r-1][r], (A^T)[r][r+1] = A[r+1][r]
  std::vector<double> coefT(coef.size(), 0.0);
  for (int m = 0; m < nd; ++m) {
    const int nmu = G.n[m];
    const bool per = (P->periodic_mask >> m) & 1;
    const double* lo = &coef[(m * 3 + 0) * nmax];
    const double* dg = &coef[(m * 3 + 1) * nmax];
    const double* up = &coef[(m * 3 + 2) * nmax];
    for (int r = 0; r < nmu; ++r) {
      coefT[(m * 3 + 1) * nmax + r] = dg[r];
      coefT[(m * 3 + 0) * nmax + r] = r > 0 ? up[r - 1] : (per ? up[nmu - 1] : 0.0);
      coefT[(m * 3 + 2) * nmax + r] = r + 1 < nmu ? lo[r + 1] : (per ? lo[0] : 0.0);
    }
  }
  std::vector<double> rd(nslab), tv(nslab, tau), trd(nslab);
  for (int q = 0; q < nslab; ++q) {
    rd[q] = 1.0 / P->diff[q];
    trd[q] = tau / P->diff[q];
  }
  const size_t o_coefT = ar.add_d(coefT), o_rd = ar.add_d(rd), o_tv = ar.add_d(tv), o_trd = ar.add_d(trd);
  const size_t o_coef = ar.add_d(coef), o_scale = ar.add_d(scale);
  const size_t o_diff = ar.add_d(P->diff), o_rp = ar.add_d(P->rparams);
  const size_t o_wref = ar.add_d(P->wref), o_g0 = ar.add_d(P->g0), o_cs = ar.add_d(cs);
  // quadrature weights of the steady-state indicators (Section 5.2)
  std::vector<double> w1 = tg::coord_weights(G.coord[0], n1, G.extent_of(0), G.lam);
  if (G.geometry == TG_SPHERE)
    for (auto& v : w1) v *= G.extent[0] * G.extent[0];
  const auto w2 = tg::coord_weights(G.coord[1], n2, G.extent_of(1), G.lam);
  const auto w3 = nd == 3 ? tg::coord_weights(G.coord[2], n3, G.extent_of(2), G.lam) : std::vector<double>(1, 1.0);
  std::vector<double> w23(static_cast<size_t>(n2) * n3);
  for (int k = 0; k < n3; ++k)
    for (int j = 0; j < n2; ++j) w23[static_cast<size_t>(k) * n2 + j] = w2[j] * w3[k];
  double s1 = 0.0, s23 = 0.0;
  for (double v : w1) s1 += v;
  for (double v : w23) s23 += v;
  P->wsum_inv = 1.0 / (s1 * s23);
  const size_t o_w1 = ar.add_d(w1), o_w23 = ar.add_d(w23);

  hip_check(hipMalloc(reinterpret_cast<void**>(&P->dmem), ar.bytes.size()), "hipMalloc(plan)");
  hip_check(hipMemcpy(P->dmem, ar.bytes.data(), ar.bytes.size(), hipMemcpyHostToDevice), "hipMemcpy(plan)");
  auto D = [&](size_t off) { return reinterpret_cast<const double*>(P->dmem + off); };
  P->d_coef = D(o_coef);
  P->d_scale = D(o_scale);
  P->d_diff = D(o_diff);
  P->d_rparams = D(o_rp);
  P->d_wref = D(o_wref);
  P->d_g0 = D(o_g0);
  P->d_cs = D(o_cs);
  P->d_coefT = D(o_coefT);
  P->d_rd = D(o_rd);
  P->d_tau = D(o_tv);
  P->d_taurd = D(o_trd);
  P->d_w1 = D(o_w1);
  P->d_w23 = D(o_w23);
  const int nn[3] = {n1, n2, n3};
  for (const auto& o : ops) {
    tg::ChainOp c;
    c.mode = o.mode;
    c.L = P->dmem + o.L;
    c.fmod = o.fmod;
    c.epi = o.epi;
    c.pm = o.pm == SIZE_MAX ? nullptr : D(o.pm);
    c.pn = o.pn == SIZE_MAX ? nullptr : D(o.pn);
    c.pb = o.pb == SIZE_MAX ? nullptr : D(o.pb);
    c.LT = o.LT == SIZE_MAX ? nullptr : P->dmem + o.LT;
    c.dL = o.dL == SIZE_MAX ? nullptr : P->dmem + o.dL;
    int64_t na = 1, nb = 1;
    for (int m = 0; m < o.mode - 1; ++m) na *= nn[m];
    for (int m = o.mode; m < 3; ++m) nb *= nn[m];
    const int nm = nn[o.mode - 1];
    if (o.mode == 1) c.tile = pick_tile(static_cast<int>(nb), nm, nslab);
    else c.tile = pick_tile(nm, static_cast<int>(na), nb * nslab);
    c.flops = 2.0 * nm * static_cast<double>(P->state_elems);
    P->chain.push_back(c);
  }
  // Fused route: resolve the specs, choose tile widths, check LDS budgets.
  {
    auto mkF = [&](const PadF& f) {
      tg::Factor F{};
      F.L = f.off == SIZE_MAX ? nullptr : P->dmem + f.off;
      F.ld = f.ld;
      F.fstride = static_cast<int64_t>(f.ld) * f.ld * (nterms ? nterms : 1);
      F.fmod = f.fmod;
      return F;
    };
    auto strided_lds = [&](int nm, int na, int tn, int sandwich, int plane, int stencil) {
      return nterms ? tg::strided_bf16_lds_bytes(nterms, nm, na, tn, sandwich, plane)
                    : tg::strided_lds_bytes<T>(nm, tn, sandwich, plane, stencil);
    };
    auto first_lds = [&](int nm, int tm, int sandwich) {
      return nterms ? tg::first_bf16_lds_bytes(nterms, nm, tm, sandwich) : tg::first_lds_bytes<T>(nm, tm, sandwich);
    };
    auto Dp = [&](size_t off) { return off == SIZE_MAX ? nullptr : D(off); };
    auto first_op = [&](int nm, int rows, const PadF& L1, const PadF& L2, int sandwich, int in) {
      tg::FusedOp op;
      op.kind = 1;
      op.mode = 1;
      tg::FirstArgs& fa = op.fa;
      fa.nm = nm;
      fa.rows = rows;
      fa.nslab = nslab;
      fa.sandwich = sandwich;
      fa.L1 = mkF(L1);
      if (sandwich) fa.L2 = mkF(L2);
      fa.update = 1;
      fa.alpha = tau;
      fa.flag = P->dflag;
      const int64_t wg32 = static_cast<int64_t>((rows + 31) / 32) * nslab;
      fa.tm = wg32 >= 512 ? 32 : 16;
      op.in = in;
      op.out = -1;
      op.updates_state = true;
      op.flops = (sandwich ? 2.0 : 1.0) * 2.0 * nm * static_cast<double>(P->state_elems);
      return op;
    };
    std::vector<tg::FusedOp> out;
    bool ok = true;
    int buf = 0, prev = -1;
    for (const auto& f : fspecs) {
      if (f.kind == 1) {
        auto op = first_op(f.nm, f.rows, f.L1, f.L2, f.sandwich, prev);
        op.fa.ph = {P->d_cs, Dp(f.pm), Dp(f.pn), nullptr};
        if (first_lds(f.nm, op.fa.tm, f.sandwich) > kLdsLimit) { ok = false; break; }
        out.push_back(op);
        prev = -1;
        continue;
      }
      tg::FusedOp op;
      op.kind = 0;
      op.mode = f.mode;
      tg::StridedArgs& sa = op.sa;
      sa.nm = f.nm;
      sa.na = f.na;
      sa.nb = f.nb;
      sa.nslab = nslab;
      sa.sandwich = f.sandwich;
      sa.phi = f.phi;
      sa.stencil = f.stencil;
      sa.L1 = mkF(f.L1);
      if (f.sandwich) sa.L2 = mkF(f.L2);
      sa.ph = {P->d_cs, Dp(f.pm), Dp(f.pn), Dp(f.pb)};
      sa.alpha = tau;
      sa.flag = P->dflag;
      sa.update = 1;
      bool plane = f.plane != 0;
      if (plane) {
        sa.tn = (f.na + 31) / 32 * 32;
        const size_t lds = strided_lds(f.nm, f.na, sa.tn, f.sandwich, 1, f.stencil);
        if (lds > kLdsLimit) {
          plane = false;
        } else {
          // 3D grids: whole planes that take two rounds of workgroups, the
          // second less than half full, run slower than the split tail
          // (sandwich launch, then the mode-1 launch): the 100^3 cylinder's
          // 300 planes of 135-139 KB (one per CU) on 256 CUs.  The disk
          // (one plane per slab) keeps its plane launch at any batch: its
          // resident route is built from it.
          const int64_t slots = std::max<int64_t>(1, static_cast<int64_t>(kLdsLimit / lds)) * num_cus;
          const int64_t wgs = static_cast<int64_t>(f.nb) * nslab;
          if (f.nb > 1 && wgs > slots && wgs - slots < slots / 2) plane = false;
        }
      }
      if (!plane) {
        // 32-wide column tiles when that still gives ~512 workgroups, and
        // 16-wide ones where the wider tile does not fit in LDS
        const int64_t wg32 = static_cast<int64_t>((f.na + 31) / 32) * f.nb * nslab;
        sa.tn = wg32 >= 512 ? 32 : 16;
        if (sa.tn == 32 && strided_lds(f.nm, f.na, 32, f.sandwich, 0, f.stencil) > kLdsLimit) sa.tn = 16;
        if (strided_lds(f.nm, f.na, sa.tn, f.sandwich, 0, f.stencil) > kLdsLimit) { ok = false; break; }
      }
      sa.plane = plane ? 1 : 0;
      if (plane) sa.P = mkF(f.Pf);
      op.flops = ((f.sandwich ? 2.0 : 1.0) * 2.0 * f.nm + (plane ? 2.0 * f.na : 0.0)) *
                 static_cast<double>(P->state_elems);
      op.in = prev;
      if (plane) {
        op.out = -1;
        op.updates_state = true;
        prev = -1;
      } else {
        op.out = buf;
        prev = buf;
        buf ^= 1;
      }
      out.push_back(op);
      if (f.plane && !plane) {  // split tail: mode-1 product + update
        auto t = first_op(n1, static_cast<int>(P->npts / n1), f.Pf, f.Pf, 0, prev);
        if (first_lds(n1, t.fa.tm, 0) > kLdsLimit) { ok = false; break; }
        out.push_back(t);
        prev = -1;
      }
    }
    P->fused_ok = ok && !out.empty() && out.back().updates_state;
    if (P->fused_ok) P->fused = out;
    TG_REQUIRE(P->fused_ok || nterms == 0, TG_ENOTSUP,
               "tg_plan_create: split-bf16 precision needs the fused route, which does not fit this grid");
  }
  const size_t bytes = static_cast<size_t>(P->state_elems) * sizeof(T);
  for (int i = 0; i < 2; ++i) hip_check(hipMalloc(&P->scratch[i], bytes), "hipMalloc(scratch)");
  hip_check(hipMalloc(reinterpret_cast<void**>(&P->dflag), sizeof(int)), "hipMalloc(flag)");
  hip_check(hipMemset(P->dflag, 0, sizeof(int)), "hipMemset(flag)");
}

// Launch one chain op reading X and writing Y (or updating Y += tau * acc).
// Fusions for the adjoint: Y2 also receives the same product through epi2;
// with L2 and X2 the product runs over the concatenated contraction,
// Y = L X + L2 X2 (L2 a factor of the same shape as c.L); with X2 and Y2
// (no L2; modes >= 2) a second product Y2 = L X2 shares the factor tiles.
struct OpExtra {
  void* Y2 = nullptr;
  int epi2 = tg::EPI_STORE;
  const void* L2 = nullptr;
  const void* X2 = nullptr;
};
template <typename T>
void launch_op(const tg_plan_s* P, const tg::ChainOp& c, const void* X, void* Y, int epi, hipStream_t st,
               double alpha = -1.0, const tg::DiagArgs* dg = nullptr, const OpExtra& ex = OpExtra{}) {
  const int nd = P->grid.ndim;
  const int nn[3] = {P->grid.n[0], P->grid.n[1], nd == 3 ? P->grid.n[2] : 1};
  int64_t na = 1, nb = 1;
  for (int m = 0; m < c.mode - 1; ++m) na *= nn[m];
  for (int m = c.mode; m < 3; ++m) nb *= nn[m];
  const int nm = nn[c.mode - 1];
  tg::GemmArgs g{};
  g.nslab = P->nslab;
  g.epi = epi;
  g.alpha = alpha < 0.0 ? P->tau : alpha;
  g.cs = P->d_cs;
  g.pm = c.pm;
  g.pn = c.pn;
  g.pb = c.pb;
  g.tile = c.tile;
  g.flag = P->dflag;
  g.rd = P->d_rd;
  const int64_t slab = P->npts;
  const int big = std::numeric_limits<int>::max();
  if (c.slice) {
    TG_REQUIRE(!ex.Y2 && !ex.L2, TG_ENOTSUP, "product fusions need a per-mode op");
    // per slice i (grid y) and slab: C_i (nm x ncol) = P_i (nm x nm) X_i, where
    // X_i[k][n] = X[k sk + n sn + i]
    g.A = c.L; g.B = X; g.C = Y;
    g.M = nm; g.N = c.ncol; g.K = nm; g.nbatch = nn[0];
    g.lda = nm; g.ldb = c.sk; g.ldc = c.sk;
    g.b_ncol = c.sn; g.c_ncol = c.sn;
    g.a_bstride = static_cast<int64_t>(nm) * nm; g.b_bstride = 1; g.c_bstride = 1;
    g.a_sstride = static_cast<int64_t>(nn[0]) * nm * nm; g.a_smod = c.fmod;
    g.b_sstride = slab; g.b_smod = big;
    g.c_sstride = slab;
    g.b_kcontig = 0;
    TG_REQUIRE(!dg, TG_ENOTSUP, "indicators need a first-mode update");
    mark_launch(st);
    hip_check(tg::launch_mode_gemm<T>(g, st), "per-slice product launch");
    return;
  }
  TG_REQUIRE(!(ex.X2 && !ex.L2) || (ex.Y2 && c.mode >= 2), TG_ENOTSUP, "dual product needs mode >= 2");
  if (c.mode == 1) {
    // C (nb x nm) = X (nb x nm, K-contiguous) * L^T
    g.A = X; g.B = c.L; g.C = Y;
    if (ex.L2) { g.A2 = ex.X2; g.B2 = ex.L2; }
    g.M = static_cast<int>(nb); g.N = nm; g.K = nm; g.nbatch = 1;
    g.lda = nm; g.ldb = nm; g.ldc = nm;
    g.a_sstride = slab; g.a_smod = big;
    g.b_sstride = static_cast<int64_t>(nm) * nm; g.b_smod = c.fmod;
    g.c_sstride = slab;
    g.b_kcontig = 1;
  } else {
    // per b: C (nm x na) = L (nm x nm) * X_b (nm x na)
    g.A = c.L; g.B = X; g.C = Y;
    if (ex.L2) { g.A2 = ex.L2; g.B2 = ex.X2; }
    else if (ex.X2) g.B2 = ex.X2;  // dual product into Y2
    g.M = nm; g.N = static_cast<int>(na); g.K = nm; g.nbatch = static_cast<int>(nb);
    g.lda = nm; g.ldb = na; g.ldc = na;
    g.a_bstride = 0; g.b_bstride = nm * na; g.c_bstride = nm * na;
    g.a_sstride = static_cast<int64_t>(nm) * nm; g.a_smod = c.fmod;
    g.b_sstride = slab; g.b_smod = big;
    g.c_sstride = slab;
    g.b_kcontig = 0;
  }
  if (dg) {
    TG_REQUIRE(c.mode == 1 && epi == tg::EPI_UPDATE, TG_ENOTSUP, "indicators need a first-mode update");
    g.dg = *dg;
  }
  g.C2 = ex.Y2;
  g.epi2 = ex.epi2;
  mark_launch(st);
  hip_check(tg::launch_mode_gemm<T>(g, st), "mode product launch");
}

template <typename T>
void launch_stencil_stage(const tg_plan_s* P, const void* W, void* F, int what, hipStream_t st, void* F2 = nullptr) {
  tg::StencilArgs a{};
  a.W = W;
  a.F = F;
  a.F2 = F2;
  a.ndim = P->grid.ndim;
  a.n[0] = P->grid.n[0];
  a.n[1] = P->grid.n[1];
  a.n[2] = P->grid.ndim == 3 ? P->grid.n[2] : 1;
  a.nspecies = P->ns;
  a.batch = P->batch;
  a.what = what;
  a.coef = P->d_coef;
  a.scale = P->d_scale;
  a.nmax = P->nmax;
  a.periodic_mask = P->periodic_mask;
  a.scale_mask = P->scale_mask;
  a.diff = P->d_diff;
  a.reaction = P->reaction;
  a.rparams = P->d_rparams;
  a.wref = P->d_wref;
  a.g0 = P->d_g0;
  mark_launch(st);
  hip_check(tg::launch_stencil<T>(a, st), "stencil launch");
}

tg::StencilArgs stencil_args(const tg_plan_s* P, const void* W, void* F, int what) {
  tg::StencilArgs a{};
  a.W = W;
  a.F = F;
  a.ndim = P->grid.ndim;
  a.n[0] = P->grid.n[0];
  a.n[1] = P->grid.n[1];
  a.n[2] = P->grid.ndim == 3 ? P->grid.n[2] : 1;
  a.nspecies = P->ns;
  a.batch = P->batch;
  a.what = what;
  a.coef = P->d_coef;
  a.scale = P->d_scale;
  a.nmax = P->nmax;
  a.periodic_mask = P->periodic_mask;
  a.scale_mask = P->scale_mask;
  a.diff = P->d_diff;
  a.reaction = P->reaction;
  a.rparams = P->d_rparams;
  a.wref = P->d_wref;
  a.g0 = P->d_g0;
  return a;
}

// Concrete arguments of one fused op.  src: input tile data (or, for the
// stencil op, the state W it is computed from); dst: output buffer, or the
// state / target of the final product; update: add tau * result to dst
// instead of storing.
tg::StridedArgs strided_args_for(const tg_plan_s* P, const tg::FusedOp& op, const void* src, void* dst,
                                 bool update, bool from_state) {
  tg::StridedArgs a = op.sa;
  a.flag = P->dflag;  // allocated after the ops are built
  if (!from_state) a.stencil = 0;
  if (a.stencil) {
    a.st = stencil_args(P, src, nullptr, TG_APPLY_F);
    a.X = nullptr;
  } else {
    a.X = src;
  }
  if (a.plane) {
    a.W = dst;
    a.Y = nullptr;
    a.update = update ? 1 : 0;
  } else {
    a.Y = dst;
  }
  return a;
}

tg::FirstArgs first_args_for(const tg_plan_s* P, const tg::FusedOp& op, const void* src, void* dst, bool update) {
  tg::FirstArgs a = op.fa;
  a.flag = P->dflag;  // allocated after the ops are built
  a.X = src;
  a.Y = dst;
  a.update = update ? 1 : 0;
  return a;
}

template <typename T>
void launch_fused(const tg_plan_s* P, const tg::FusedOp& op, const void* src, void* dst, bool update,
                  bool from_state, hipStream_t st, const tg::DiagArgs* dg = nullptr) {
  const int nt = bf16_terms(P->precision);
  TG_REQUIRE(!dg || update, TG_ENOTSUP, "indicators need an update launch");
  if (op.kind == 0) {
    tg::StridedArgs a = strided_args_for(P, op, src, dst, update, from_state);
    if (dg) {
      TG_REQUIRE(a.plane, TG_ENOTSUP, "indicators need a plane-tail update");
      a.dg = *dg;
    }
    mark_launch(st);
    hip_check(nt ? tg::launch_strided_bf16(nt, a, st) : tg::launch_strided<T>(a, st), "fused strided launch");
  } else {
    tg::FirstArgs a = first_args_for(P, op, src, dst, update);
    if (dg) a.dg = *dg;
    mark_launch(st);
    hip_check(nt ? tg::launch_first_bf16(nt, a, st) : tg::launch_first<T>(a, st), "fused first-mode launch");
  }
}

// in / out buffers of fused op i of a step on `state` (route 0 or 2)
struct FusedIO {
  const void* in;
  void* out;
  bool update;
  bool from_state;
};
FusedIO fused_io(const tg_plan_s* P, size_t i, void* state, bool apart) {
  const auto& op = P->fused[i];
  const void* src = apart ? P->scratch[1] : state;
  const bool last = i + 1 == P->fused.size();
  return FusedIO{op.in < 0 ? src : P->scratch[op.in], last ? state : P->scratch[op.out], last, !apart};
}

// Run the fused chain: the first op reads `src` (the state when it carries
// the stencil), intermediate results go to scratch, the last op updates or
// stores `dst`.
template <typename T>
void run_fused(const tg_plan_s* P, const void* src, void* dst, bool update, bool from_state, hipStream_t st,
               const tg::DiagArgs* dg = nullptr) {
  for (size_t i = 0; i < P->fused.size(); ++i) {
    const auto& op = P->fused[i];
    const void* in = op.in < 0 ? src : P->scratch[op.in];
    const bool last = i + 1 == P->fused.size();
    void* out = last ? dst : P->scratch[op.out];
    launch_fused<T>(P, op, in, out, last ? update : false, from_state, st, last ? dg : nullptr);
  }
}

// Apply the split chain to `in`.  final_update: last op does state += tau*acc
// on `out`; otherwise the last op stores into `out`.
// The per-mode chain of the active route: route 3 replaces the scaled
// mode's eigen-basis sandwich by per-slice dense factors.
const std::vector<tg::ChainOp>& chain_of(const tg_plan_s* P) {
  return P->route == 3 && !P->slice_chain.empty() ? P->slice_chain : P->chain;
}

bool slice_capable(const tg_plan_s* P) {
  return (P->grid.geometry == TG_BALL || P->grid.geometry == TG_CYLINDER) && !bf16_terms(P->precision);
}

// Per-slice factors of the scaled mode, phi_1(tau d_s rho_i^-2 A) for each
// slab s and radial index i (the ball's phi mode, the cylinder's theta mode),
// from the mode's eigen-decomposition; the chain of route 1 with that mode's
// sandwich replaced by one per-slice product.
template <typename T>
void build_slice_chain(tg_plan_s* P) {
  const tg_grid_s& G = P->grid;
  const int n1 = G.n[0], n2 = G.n[1], n3 = G.n[2];
  const bool ball = G.geometry == TG_BALL;
  const int mode = ball ? 3 : 2;
  const size_t first = ball ? 0 : 1;  // the sandwich pair in the route-1 chain
  TG_REQUIRE(P->chain.size() > first + 1 && P->chain[first].mode == mode && P->chain[first + 1].mode == mode &&
                 P->chain[first].epi == tg::EPI_PHI,
             TG_ENOTSUP, "per-slice route: unexpected chain");
  const int nm = G.n[mode - 1];
  const tg::Eig e = G.eig(mode - 1);
  const auto r = G.coords(0);
  const int fmod = P->nslab;
  const size_t blk = static_cast<size_t>(nm) * nm;
  std::vector<T> host(static_cast<size_t>(fmod) * n1 * blk);
  for (int f = 0; f < fmod; ++f)
    for (int i = 0; i < n1; ++i) {
      const auto Pm = tg::phi1_from_eig(e, P->tau * P->diff[f] / (r[i] * r[i]));
      T* dst = host.data() + (static_cast<size_t>(f) * n1 + i) * blk;
      for (size_t q = 0; q < blk; ++q) dst[q] = static_cast<T>(Pm[q]);
    }
  void* mem = nullptr;
  hip_check(hipMalloc(&mem, host.size() * sizeof(T)), "hipMalloc(per-slice factors)");
  hipError_t err = hipMemcpy(mem, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(mem);
    hip_check(err, "hipMemcpy(per-slice factors)");
  }
  tg::ChainOp op = P->chain[first];
  op.slice = 1;
  op.L = mem;
  op.fmod = fmod;
  op.epi = tg::EPI_STORE;
  op.pm = op.pn = op.pb = nullptr;
  op.LT = op.dL = nullptr;
  op.sk = ball ? static_cast<int64_t>(n1) * n2 : n1;
  op.sn = ball ? n1 : static_cast<int64_t>(n1) * n2;
  op.ncol = ball ? n2 : n3;
  op.tile = pick_tile(nm, op.ncol, static_cast<int64_t>(n1) * P->nslab);
  op.flops = 2.0 * nm * static_cast<double>(P->state_elems);
  std::vector<tg::ChainOp> chain(P->chain.begin(), P->chain.begin() + first);
  chain.push_back(op);
  chain.insert(chain.end(), P->chain.begin() + first + 2, P->chain.end());
  P->slice_mem = mem;
  P->slice_chain = std::move(chain);
}

void ensure_slice_chain(tg_plan_s* P) {
  TG_REQUIRE(slice_capable(P), TG_ENOTSUP,
             "per-slice route: ball and cylinder plans in FP64 or FP32 only");
  TG_REQUIRE(P->grid.n[0] <= 65535, TG_ENOTSUP, "per-slice route: too many radial slices");
  if (!P->slice_chain.empty()) return;
  if (P->precision == TG_FP64) build_slice_chain<double>(P);
  else build_slice_chain<float>(P);
}

template <typename T>
void run_chain(const tg_plan_s* P, const void* in, void* out, bool final_update, hipStream_t st,
               const tg::DiagArgs* dg = nullptr) {
  const auto& chain = chain_of(P);
  const size_t nops = chain.size();
  const void* X = in;
  int buf = (in == P->scratch[0]) ? 1 : 0;
  for (size_t o = 0; o < nops; ++o) {
    const auto& c = chain[o];
    const bool last = (o + 1 == nops);
    void* Y = last ? out : P->scratch[buf];
    int epi = c.epi;
    if (last) epi = final_update ? tg::EPI_UPDATE : tg::EPI_STORE;
    launch_op<T>(P, c, X, Y, epi, st, -1.0, last ? dg : nullptr);
    X = Y;
    buf ^= 1;
  }
}

// 0: fused with the stencil in the first tile load; 2: fused products after
// a separate stencil launch; 1: one launch per mode product; 3: as 1 with
// per-slice dense factors for the scaled mode (ball, cylinder).
// Route 4 (resident): the step is one fused strided op with the stencil, the
// sandwich and the plane-tail update on a 2D grid (the disk), and the tiles
// of every species of an instance fit in LDS together.
bool resident_ok(const tg_plan_s* P) {
  if (bf16_terms(P->precision) || !P->fused_ok || P->fused.size() != 1 || P->grid.ndim != 2) return false;
  if (P->reaction >= TG_REACT_LINEAR) return false;  // kinetics of the stencil launch only
  const tg::FusedOp& op = P->fused.front();
  if (op.kind != 0) return false;
  const tg::StridedArgs& a = op.sa;
  if (!a.stencil || !a.sandwich || !a.phi || !a.plane || a.nb != 1 || P->batch > 65535) return false;
  const size_t b = P->precision == TG_FP64 ? tg::resident_lds_bytes<double>(P->ns, a.nm, a.na)
                                           : tg::resident_lds_bytes<float>(P->ns, a.nm, a.na);
  return b > 0 && b <= kLdsLimit;
}

int active_route(const tg_plan_s* P) {
  if (P->route == 4) return resident_ok(P) ? 4 : 0;
  if (bf16_terms(P->precision)) return P->route == 2 ? 2 : 0;  // split-bf16 runs fused only
  if (P->route == 3) return P->slice_chain.empty() ? 1 : 3;
  return P->fused_ok && P->route != 1 ? P->route : 1;
}
bool use_fused(const tg_plan_s* P) {
  const int r = active_route(P);
  return r == 0 || r == 2;
}

// Whether a fused plan computes F in a stencil launch of its own before the
// products (route 2) instead of inside the first product's tile load
// (route 0).  Route 0 keeps it in the tile load except where that launch
// also updates the state in place (the disk's single plane launch) and the
// plan has several species: there the workgroup of one species could
// overwrite values that the workgroup of another, started later, has still
// to read for the reaction.
bool stencil_apart(const tg_plan_s* P) {
  const int r = active_route(P);
  if (r != 0) return r == 2;
  if (P->reaction >= TG_REACT_LINEAR) return true;  // kinetics of the stencil launch only
  const auto& op = P->fused.front();
  return P->ns > 1 && op.kind == 0 && op.sa.stencil && op.sa.plane;
}

// Whether the active route computes F inside the first fused op's tile
// load, which then needs LDS for the stencil's neighbours as well.
bool in_tile_stencil(const tg_plan_s* P) { return active_route(P) == 0 && !stencil_apart(P); }

// LDS bytes of fused op `op` at tile width (kind 0: columns, kind 1: rows)
// `t`, as the active route launches it.
size_t fused_lds_bytes(const tg_plan_s* P, const tg::FusedOp& op, int t) {
  const int nt = bf16_terms(P->precision);
  if (op.kind == 1) {
    const auto& a = op.fa;
    return nt ? tg::first_bf16_lds_bytes(nt, a.nm, t, a.sandwich)
              : (P->precision == TG_FP64 ? tg::first_lds_bytes<double>(a.nm, t, a.sandwich)
                                         : tg::first_lds_bytes<float>(a.nm, t, a.sandwich));
  }
  const auto& a = op.sa;
  const int st = a.stencil && in_tile_stencil(P) ? 1 : 0;
  return nt ? tg::strided_bf16_lds_bytes(nt, a.nm, a.na, t, a.sandwich, a.plane)
            : (P->precision == TG_FP64 ? tg::strided_lds_bytes<double>(a.nm, t, a.sandwich, a.plane, st)
                                       : tg::strided_lds_bytes<float>(a.nm, t, a.sandwich, a.plane, st));
}
bool fused_tile_fits(const tg_plan_s* P, const tg::FusedOp& op, int t) {
  const size_t b = fused_lds_bytes(P, op, t);
  return b > 0 && b <= kLdsLimit;
}

// After a route change: column tiles chosen for a route without the
// in-tile stencil that do not fit with it go back to 16 columns (which
// the plan's construction checked with the stencil).
void fit_tiles_to_route(tg_plan_s* P) {
  for (auto& op : P->fused)
    if (op.kind == 0 && !op.sa.plane && op.sa.tn != 16 && !fused_tile_fits(P, op, op.sa.tn)) op.sa.tn = 16;
}

// Launches of one step of the active route.
int step_launches(const tg_plan_s* P) {
  const int r = active_route(P);
  if (r == 4) return 1;
  if (r == 0 || r == 2) return static_cast<int>(P->fused.size()) + (stencil_apart(P) ? 1 : 0);
  return static_cast<int>(chain_of(P).size()) + 1;
}

// `steps` steps of a route-4 plan: resident launches of at most
// kResidentChunk steps each.
constexpr int64_t kResidentChunk = 1024;
template <typename T>
void run_resident(tg_plan_s* P, void* state, int64_t steps, hipStream_t st) {
  tg::ResidentArgs r{};
  r.a = strided_args_for(P, P->fused.front(), state, state, true, true);
  r.np = tg::resident_np(r.a.nm, r.a.na);
  r.tn = tg::resident_tn(r.a.nm, r.a.na);
  r.ninst = P->batch;
  for (int64_t done = 0; done < steps; done += kResidentChunk) {
    r.steps = static_cast<int>(std::min<int64_t>(kResidentChunk, steps - done));
    mark_launch(st);
    hip_check(tg::launch_resident<T>(r, st), "resident launch");
  }
}
void run_resident_any(tg_plan_s* P, void* state, int64_t steps, hipStream_t st) {
  if (P->precision == TG_FP64) run_resident<double>(P, state, steps, st);
  else run_resident<float>(P, state, steps, st);
}

template <typename T>
void step_impl(tg_plan_s* P, void* state, hipStream_t st, const tg::DiagArgs* dg = nullptr) {
  const int r = active_route(P);
  if (r == 4 && !dg) {
    run_resident<T>(P, state, 1, st);
    return;
  }
  if (r == 0 && !stencil_apart(P)) {
    // the first fused op computes F from the state inside its tile load
    run_fused<T>(P, state, state, true, true, st, dg);
    return;
  }
  if (r == 0 || r == 2 || r == 4) {  // (route 4 with indicators: the fused launches)
    launch_stencil_stage<T>(P, state, P->scratch[1], TG_APPLY_F, st);
    run_fused<T>(P, P->scratch[1], state, true, false, st, dg);
    return;
  }
  launch_stencil_stage<T>(P, state, P->scratch[0], TG_APPLY_F, st);
  run_chain<T>(P, P->scratch[0], state, true, st, dg);
}

// One reverse step of the discrete adjoint (see tg_adjoint_step).
template <typename T>
void adjoint_impl(tg_plan_s* P, const void* state, void* lam, double* grad, hipStream_t st) {
  const size_t bytes = static_cast<size_t>(P->state_elems) * sizeof(T);
  // the gradient's partial sums: three per species and block of 256 points
  const size_t pbytes = sizeof(double) * 3 * static_cast<size_t>(P->nslab) * static_cast<size_t>((P->npts + 255) / 256);
  if (!P->adj_ws) hip_check(hipMalloc(&P->adj_ws, 8 * bytes + pbytes), "hipMalloc(adjoint workspace)");
  char* w = static_cast<char*>(P->adj_ws);
  double* part = reinterpret_cast<double*>(w + 8 * bytes);
  void* F = w;
  void* DMW = w + bytes;
  void* xbuf[2] = {w + 2 * bytes, w + 3 * bytes};
  void* tbuf[2] = {w + 4 * bytes, w + 5 * bytes};
  void* MU = w + 6 * bytes;
  void* MTMU = w + 7 * bytes;
  const int64_t npts = P->npts;

  // F = d M W + g(W) and d M W at step n (one launch)
  launch_stencil_stage<T>(P, state, F, 3, st, DMW);

  // tangent of the split action along d: t = (dS/dd) F, carried through the
  // chain next to x = partial products of S F
  const void* x = F;
  const void* t = nullptr;
  int xb = 0, tb = 0;
  const size_t nops = P->chain.size();
  for (size_t o = 0; o < nops; ++o) {
    const auto& c = P->chain[o];
    const bool need_x = o + 1 < nops;  // S F itself is not needed, only its tangent
    void* xn = xbuf[xb];
    void* tn = tbuf[tb];
    bool t_written = false;
    if (c.epi == tg::EPI_PHI) {  // y = Phi o (L x): t' = Phi o (L t) + dPhi/dd o (L x)
      // dPhi/dd o (L x) and, from the same product, y itself
      OpExtra ex;
      if (need_x) {
        ex.Y2 = xn;
        ex.epi2 = tg::EPI_PHI;
      }
      launch_op<T>(P, c, x, tn, tg::EPI_DPHI, st, -1.0, nullptr, ex);
      if (t) launch_op<T>(P, c, t, tn, tg::EPI_PHI_ACC, st);
      t_written = true;
    } else if (c.dL) {  // y = L(d) x: t' = (dL/dd) x + L t, one contraction over both pairs
      tg::ChainOp cd = c;
      cd.L = c.dL;
      OpExtra ex;
      if (t) {
        ex.L2 = c.L;
        ex.X2 = t;
      }
      launch_op<T>(P, cd, x, tn, tg::EPI_STORE, st, -1.0, nullptr, ex);
      if (need_x) launch_op<T>(P, c, x, xn, tg::EPI_STORE, st);
      t_written = true;
    } else if (t && need_x && c.mode >= 2) {  // L t and L x from shared factor tiles
      OpExtra ex;
      ex.X2 = x;
      ex.Y2 = xn;
      launch_op<T>(P, c, t, tn, tg::EPI_STORE, st, -1.0, nullptr, ex);
      t_written = true;
    } else {
      if (t) {
        launch_op<T>(P, c, t, tn, tg::EPI_STORE, st);
        t_written = true;
      }
      if (need_x) launch_op<T>(P, c, x, xn, tg::EPI_STORE, st);
    }
    x = xn;
    xb ^= 1;
    if (t_written) {
      t = tn;
      tb ^= 1;
    }
  }
  TG_REQUIRE(t != nullptr, TG_EINVAL, "adjoint: chain without a d-dependent factor");

  // mu = S^T lambda: transposed factors in reverse order; each Hadamard
  // factor moves to the product that precedes it in the reversed chain
  const void* y = lam;
  int yb = 0;
  const int n = static_cast<int>(P->chain.size());
  for (int j = n - 1; j >= 0; --j) {
    tg::ChainOp ct = P->chain[j];
    ct.L = P->chain[j].LT;
    int epi = tg::EPI_STORE;
    ct.pm = ct.pn = ct.pb = nullptr;
    if (j >= 1 && P->chain[j - 1].epi == tg::EPI_PHI) {
      epi = tg::EPI_PHI;
      ct.pm = P->chain[j - 1].pm;
      ct.pn = P->chain[j - 1].pn;
      ct.pb = P->chain[j - 1].pb;
    }
    void* out = j == 0 ? MU : xbuf[yb];
    launch_op<T>(P, ct, y, out, epi, st);
    y = out;
    yb ^= 1;
  }
  // lambda += tau (d M^T mu + J^T mu)
  tg::StencilArgs a = stencil_args(P, MU, MTMU, TG_APPLY_DIFFUSION);
  a.coef = P->d_coefT;
  hip_check(tg::launch_stencil<T>(a, st), "adjoint stencil");
  tg::AdjointArgs aa{};
  aa.state = state;
  aa.mu = MU;
  aa.mtmu = MTMU;
  aa.lam = lam;
  // dL/dd_s += tau <lambda_s, (dS/dd) F_s> + (tau / d_s) <mu_s, d_s M W_s>;
  // dL/dc_s += tau sum mu_s (old lambda: read before the update)
  aa.tang = t;
  aa.dmw = DMW;
  aa.part = part;
  aa.grad = grad;
  aa.tau_s = P->d_tau;
  aa.taurd_s = P->d_taurd;
  aa.npts = npts;
  aa.nspecies = P->ns;
  aa.batch = P->batch;
  aa.reaction = P->reaction;
  aa.tau = P->tau;
  aa.rparams = P->d_rparams;
  aa.wref = P->d_wref;
  hip_check(tg::launch_adjoint_combine<T>(aa, st), "adjoint combine");
}

void step_any(tg_plan_s* P, void* state, hipStream_t st, const tg::DiagArgs* dg = nullptr) {
  if (P->precision == TG_FP64) step_impl<double>(P, state, st, dg);
  else step_impl<float>(P, state, st, dg);
}

// Indicator arguments writing to out ([nslab][2] doubles); allocates the
// partial-sum buffer on first use.  Every n >= 3 and tiles are at least 16
// wide, so a slab has at most npts / 48 + npts / 9 + 1 tiles in any launch
// configuration: npts / 8 + 64 slots per slab (the launchers check it).
tg::DiagArgs diag_args(tg_plan_s* P, double* out) {
  if (!P->diag_part) {
    const int64_t cap = P->npts / 8 + 64;
    TG_REQUIRE(cap < (int64_t(1) << 30), TG_EINVAL, "indicators: grid too large");
    hip_check(hipMalloc(reinterpret_cast<void**>(&P->diag_part), sizeof(double) * 2 * cap * P->nslab),
              "hipMalloc(indicator partials)");
    P->diag_cap = static_cast<int>(cap);
  }
  tg::DiagArgs d{};
  d.part = P->diag_part;
  d.out = out;
  d.w1 = P->d_w1;
  d.w23 = P->d_w23;
  d.wref = P->d_wref;
  d.wsum_inv = P->wsum_inv;
  d.cap = P->diag_cap;
  return d;
}

constexpr int kStepsPerGraph = 8;
// plan runs replay a graph of kLongGraph steps first (fewer graph launches:
// measured 33.8 -> 33.3 us per FP32 step of the 64 x 64 x 128 ball)
constexpr int kLongGraph = 32;

// A HIP graph of `steps` consecutive steps on `state`, captured once per
// (state pointer, steps) on the plan's private stream and replayed on the
// caller's.
hipGraphExec_t step_graph(tg_plan_s* P, void* state, int steps) {
  const std::pair<void*, int> key(state, steps);
  auto it = P->graphs.find(key);
  if (it != P->graphs.end()) return it->second;
  if (!P->capture_stream)
    hip_check(hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking), "capture stream");
  hipGraph_t graph = nullptr;
  hip_check(hipStreamBeginCapture(P->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    for (int i = 0; i < steps; ++i) step_any(P, state, P->capture_stream);
  } catch (...) {
    (void)hipStreamEndCapture(P->capture_stream, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  hip_check(hipStreamEndCapture(P->capture_stream, &graph), "end capture");
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  hip_check(e, "graph instantiate");
  P->graphs[key] = ex;
  return ex;
}

// ---------------------------------------------------------------------------
// Bulk-surface step (Section 5.5): both stencil launches read the states at
// t_n (each with the other's values at the interface), then each side runs
// its own split products from its F.  Route 0 computes F inside the first
// product's tile, which knows no partner, so its plans take route 2 here.
struct Coupled {
  tg_plan_s* bulk;
  tg_plan_s* surf;
  double c[5];  // ball + sphere: zeta1, zeta2, zeta3, eta1, eta2; cylinder + disk: alpha3, beta3
};

template <typename T>
void coupled_impl(const Coupled& C, void* ub, void* us, hipStream_t st) {
  tg_plan_s* B = C.bulk;
  tg_plan_s* S = C.surf;
  void* fb = !use_fused(B) ? B->scratch[0] : B->scratch[1];
  void* fs = !use_fused(S) ? S->scratch[0] : S->scratch[1];
  tg::StencilArgs ab = stencil_args(B, ub, fb, TG_APPLY_F);
  tg::StencilArgs as = stencil_args(S, us, fs, TG_APPLY_F);
  tg::CoupleArgs cb{}, cs{};
  if (B->grid.geometry == TG_CYLINDER) {  // Section 5.6: flux through the z = 0 row's ghost point
    const double hz = B->grid.extent[1] / B->grid.n[2];
    cb = tg::CoupleArgs{3, us, S->d_wref, 0, 2.0 / hz, C.c[0], C.c[1], 0.0, 0.0, 0.0, S->d_rparams};
    cs = tg::CoupleArgs{4, ub, B->d_wref, B->grid.n[2], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, nullptr};
  } else {  // Section 5.5: Robin terms through the ball's boundary row
    const double h = B->grid.extent[0] / B->grid.n[0];
    cb = tg::CoupleArgs{1, us, S->d_wref, B->grid.n[0], (2.0 / h) * (1.0 + h / B->grid.extent[0]),
                        C.c[0], C.c[1], C.c[2], C.c[3], C.c[4], nullptr};
    cs = cb;
    cs.kind = 2;
    cs.other = ub;
    cs.oref = B->d_wref;
  }
  ab.cp = cb;
  as.cp = cs;
  mark_launch(st);
  hip_check(tg::launch_stencil<T>(ab, st), "bulk stencil launch");
  mark_launch(st);
  hip_check(tg::launch_stencil<T>(as, st), "surface stencil launch");
  if (!use_fused(B)) run_chain<T>(B, fb, ub, true, st);
  else run_fused<T>(B, fb, ub, true, false, st);
  if (!use_fused(S)) run_chain<T>(S, fs, us, true, st);
  else run_fused<T>(S, fs, us, true, false, st);
}

void coupled_any(const Coupled& C, void* ub, void* us, hipStream_t st) {
  if (C.bulk->precision == TG_FP64) coupled_impl<double>(C, ub, us, st);
  else coupled_impl<float>(C, ub, us, st);
}

// Device buffers are read and written as 4-element vectors.
bool aligned(const tg_plan_s* p, const void* ptr) {
  return reinterpret_cast<uintptr_t>(ptr) % (4u * static_cast<unsigned>(p->esize)) == 0;
}

void drop_graphs(tg_plan_s* P) {
  for (auto& kv : P->graphs) (void)hipGraphExecDestroy(kv.second);
  P->graphs.clear();
  ++P->version;
}

}  // namespace

// ---------------------------------------------------------------------------
// Grouped runs: several plans (e.g. batches on different grids) stepped
// together.  With equal precision (FP64 or FP32), route and fused-op
// structure, fused op k of every member runs in ONE persistent launch
// (tg::launch_*_group); otherwise each member's launches follow each other.
// Either way, steps are replayed from one captured graph.
struct tg_group_s {
  std::vector<tg_plan_s*> plans;
  std::vector<void*> states;
  bool grouped = false;
  int route = 0;
  bool apart = false;                     // a stencil launch per member first
  std::vector<int> kind;                  // per fused op
  std::vector<tg::GroupLaunch> launch;    // per fused op
  std::vector<size_t> offset;             // byte offset of op k's group in dev
  void* dev = nullptr;
  hipGraphExec_t graph = nullptr;
  hipStream_t capture = nullptr;
  ~tg_group_s() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (capture) (void)hipStreamDestroy(capture);
    if (dev) (void)hipFree(dev);
  }
  int launches_per_step() const {
    if (!grouped) {
      int n = 0;
      for (auto* P : plans) n += step_launches(P);
      return n;
    }
    return static_cast<int>(kind.size()) + (apart ? static_cast<int>(plans.size()) : 0);
  }
};

namespace {

template <typename T>
bool build_group_launches(tg_group_s* G) {
  const size_t nops = G->plans[0]->fused.size();
  std::vector<tg::StridedGroup> sg(nops);
  std::vector<tg::FirstGroup> fg(nops);
  G->kind.assign(nops, 0);
  G->launch.assign(nops, tg::GroupLaunch{});
  const int n = static_cast<int>(G->plans.size());
  for (size_t k = 0; k < nops; ++k) {
    G->kind[k] = G->plans[0]->fused[k].kind;
    if (G->kind[k] == 0) {
      tg::StridedGroup& g = sg[k];
      g = tg::StridedGroup{};
      g.map.n = n;
      bool wide = false;
      for (int q = 0; q < n; ++q) {
        const FusedIO io = fused_io(G->plans[q], k, G->states[q], G->apart);
        g.a[q] = strided_args_for(G->plans[q], G->plans[q]->fused[k], io.in, io.out, io.update, io.from_state);
        wide |= g.a[q].tn % 32 == 0;
      }
      // one variant for all members: 32-wide (or wider) column tiles, else
      // all 16-wide (tiles that cover whole planes keep their width)
      tg::StridedGroup g16 = g;
      if (wide)
        for (int q = 0; q < n; ++q)
          if (g.a[q].tn == 16) g.a[q].tn = 32;
      if (tg::plan_strided_group<T>(g, G->launch[k]) != hipSuccess) {
        for (int q = 0; q < n; ++q)
          if (!g16.a[q].plane) g16.a[q].tn = 16;
        if (tg::plan_strided_group<T>(g16, G->launch[k]) != hipSuccess) return false;
        g = g16;
      }
    } else {
      tg::FirstGroup& g = fg[k];
      g = tg::FirstGroup{};
      g.map.n = n;
      int tm = 16;
      for (int q = 0; q < n; ++q) {
        const FusedIO io = fused_io(G->plans[q], k, G->states[q], G->apart);
        g.a[q] = first_args_for(G->plans[q], G->plans[q]->fused[k], io.in, io.out, io.update);
        tm = std::max(tm, g.a[q].tm);
      }
      for (int q = 0; q < n; ++q) g.a[q].tm = tm;
      if (tg::plan_first_group<T>(g, G->launch[k]) != hipSuccess) return false;
    }
  }
  // one device block with every op's group descriptor
  size_t bytes = 0;
  G->offset.assign(nops, 0);
  for (size_t k = 0; k < nops; ++k) {
    G->offset[k] = bytes;
    bytes += ((G->kind[k] == 0 ? sizeof(tg::StridedGroup) : sizeof(tg::FirstGroup)) + 255) / 256 * 256;
  }
  std::vector<unsigned char> host(bytes, 0);
  for (size_t k = 0; k < nops; ++k) {
    if (G->kind[k] == 0) std::memcpy(host.data() + G->offset[k], &sg[k], sizeof(tg::StridedGroup));
    else std::memcpy(host.data() + G->offset[k], &fg[k], sizeof(tg::FirstGroup));
  }
  hip_check(hipMalloc(&G->dev, bytes), "hipMalloc(group)");
  hip_check(hipMemcpy(G->dev, host.data(), bytes, hipMemcpyHostToDevice), "group upload");
  return true;
}

bool groupable(const std::vector<tg_plan_s*>& plans) {
  const tg_plan_s* P0 = plans[0];
  if (bf16_terms(P0->precision) || !use_fused(P0)) return false;
  for (const auto* P : plans) {
    if (P->precision != P0->precision || active_route(P) != active_route(P0)) return false;
    if (stencil_apart(P) != stencil_apart(P0)) return false;
    if (P->fused.size() != P0->fused.size()) return false;
    for (size_t k = 0; k < P->fused.size(); ++k)
      if (P->fused[k].kind != P0->fused[k].kind) return false;
  }
  return true;
}

template <typename T>
void group_step(tg_group_s* G, hipStream_t st) {
  if (!G->grouped) {
    for (size_t q = 0; q < G->plans.size(); ++q) step_any(G->plans[q], G->states[q], st);
    return;
  }
  if (G->apart)
    for (size_t q = 0; q < G->plans.size(); ++q)
      launch_stencil_stage<T>(G->plans[q], G->states[q], G->plans[q]->scratch[1], TG_APPLY_F, st);
  for (size_t k = 0; k < G->kind.size(); ++k) {
    const void* d = static_cast<char*>(G->dev) + G->offset[k];
    if (G->kind[k] == 0)
      hip_check(tg::launch_strided_group<T>(G->launch[k], static_cast<const tg::StridedGroup*>(d), st),
                "grouped strided launch");
    else
      hip_check(tg::launch_first_group<T>(G->launch[k], static_cast<const tg::FirstGroup*>(d), st),
                "grouped first-mode launch");
  }
}

void group_step_any(tg_group_s* G, hipStream_t st) {
  if (G->plans[0]->precision == TG_FP64) group_step<double>(G, st);
  else group_step<float>(G, st);
}

tg_group_s* find_group(const tg_plan* plans, int32_t n_plans, void* const* states) {
  TG_REQUIRE(plans && states && n_plans >= 1 && n_plans <= tg::kMaxGroup, TG_EINVAL,
             "group: 1 to 4 plans and their states");
  std::vector<tg_plan_s*> ps(plans, plans + n_plans);
  std::vector<void*> ss(states, states + n_plans);
  std::vector<uint64_t> key;
  for (int q = 0; q < n_plans; ++q) {
    TG_REQUIRE(ps[q] && ss[q], TG_EINVAL, "group: null plan or state");
    TG_REQUIRE(aligned(ps[q], ss[q]), TG_EINVAL, "group: states must be aligned to 4 elements");
    for (int r = 0; r < q; ++r) TG_REQUIRE(ss[r] != ss[q], TG_EINVAL, "group: states must be distinct");
    key.push_back(ps[q]->serial);
    key.push_back(ps[q]->version);
    key.push_back(reinterpret_cast<uintptr_t>(ss[q]));
  }
  tg_plan_s* P0 = ps[0];
  auto it = P0->groups.find(key);
  if (it != P0->groups.end()) return it->second;
  auto* G = new tg_group_s();
  try {
    G->plans = ps;
    G->states = ss;
    G->route = active_route(P0);
    G->apart = use_fused(P0) && stencil_apart(P0);
    if (groupable(ps)) {
      G->grouped = P0->precision == TG_FP64 ? build_group_launches<double>(G) : build_group_launches<float>(G);
      if (!G->grouped && G->dev) {
        (void)hipFree(G->dev);
        G->dev = nullptr;
      }
    }
    hip_check(hipStreamCreateWithFlags(&G->capture, hipStreamNonBlocking), "capture stream");
    hipGraph_t graph = nullptr;
    hip_check(hipStreamBeginCapture(G->capture, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      for (int i = 0; i < kStepsPerGraph; ++i) group_step_any(G, G->capture);
    } catch (...) {
      (void)hipStreamEndCapture(G->capture, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    hip_check(hipStreamEndCapture(G->capture, &graph), "end capture");
    hipError_t e = hipGraphInstantiate(&G->graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(e, "graph instantiate");
  } catch (...) {
    delete G;
    throw;
  }
  P0->groups[key] = G;
  return G;
}

}  // namespace

extern "C" {

int tg_plan_create(tg_grid g, int32_t n_species, int32_t batch, const double* diff, int32_t reaction,
                   int32_t n_params, const double* params, const double* w_ref, double tau,
                   int32_t precision, tg_plan* out) {
  tg_plan_s* P = nullptr;
  int rc = guarded([&] {
    TG_REQUIRE(g && diff && out, TG_EINVAL, "tg_plan_create: null pointer");
    TG_REQUIRE(batch >= 1 && batch <= 65535, TG_EINVAL, "tg_plan_create: batch out of range");
    TG_REQUIRE(std::isfinite(tau) && tau > 0.0, TG_EINVAL, "tg_plan_create: tau must be positive");
    TG_REQUIRE(precision == TG_FP64 || precision == TG_FP32 || precision == TG_BF16X2 ||
                   precision == TG_BF16X3,
               TG_EINVAL, "tg_plan_create: unknown precision");
    int need_ns = 0, need_np = 0;
    switch (reaction) {
      case TG_REACT_NONE: need_ns = -1; need_np = 0; break;
      case TG_REACT_SCHNAKENBERG: need_ns = 2; need_np = 2; break;
      case TG_REACT_AIS3: need_ns = 3; need_np = 4; break;
      case TG_REACT_SCHNAKENBERG_SCALED: need_ns = 2; need_np = 3; break;
      case TG_REACT_LINEAR: need_ns = -1; need_np = 2 * n_species; break;
      case TG_REACT_DIB: need_ns = 2; need_np = 10; break;
      default: throw Fail(TG_EINVAL, "tg_plan_create: unknown reaction");
    }
    TG_REQUIRE(n_species >= 1 && n_species <= 3, TG_EINVAL, "tg_plan_create: 1 to 3 species");
    TG_REQUIRE(need_ns < 0 || n_species == need_ns, TG_EINVAL, "tg_plan_create: species count does not match reaction");
    TG_REQUIRE(n_params >= need_np && (n_params == 0 || params), TG_EINVAL, "tg_plan_create: missing reaction parameters");
    P = new tg_plan_s();
    static std::atomic<uint64_t> next_serial{1};
    P->serial = next_serial++;
    P->grid = *g;
    P->ns = n_species;
    P->batch = batch;
    P->nslab = n_species * batch;
    TG_REQUIRE(P->nslab <= 65535, TG_EINVAL, "tg_plan_create: too many instances");
    P->reaction = reaction;
    P->precision = precision;
    P->tau = tau;
    P->esize = precision == TG_FP64 ? 8 : 4;
    P->npts = static_cast<int64_t>(g->n[0]) * g->n[1] * (g->ndim == 3 ? g->n[2] : 1);
    P->state_elems = P->npts * P->nslab;
    P->diff.assign(diff, diff + P->nslab);
    for (double d : P->diff) TG_REQUIRE(std::isfinite(d) && d > 0.0, TG_EINVAL, "tg_plan_create: diffusion must be positive");
    TG_REQUIRE(n_params <= tg::kRParams, TG_EINVAL, "tg_plan_create: too many reaction parameters");
    TG_REQUIRE(reaction != TG_REACT_LINEAR || n_species <= 3, TG_EINVAL,
               "tg_plan_create: linear kinetics take at most three species");
    P->rparams.assign(static_cast<size_t>(batch) * tg::kRParams, 0.0);
    for (int b = 0; b < batch; ++b)
      for (int q = 0; q < n_params; ++q) P->rparams[b * tg::kRParams + q] = params[b * n_params + q];
    for (double v : P->rparams) TG_REQUIRE(std::isfinite(v), TG_EINVAL, "tg_plan_create: non-finite reaction parameter");
    P->wref.resize(P->nslab);
    P->g0.resize(P->nslab);
    for (int b = 0; b < batch; ++b) {
      std::vector<double> w = w_ref ? std::vector<double>(w_ref + b * n_species, w_ref + (b + 1) * n_species)
                                    : default_reference(reaction, n_species, &P->rparams[b * tg::kRParams]);
      auto g0 = reaction_at(reaction, n_species, &P->rparams[b * tg::kRParams], w.data());
      for (int s = 0; s < n_species; ++s) {
        P->wref[b * n_species + s] = w[s];
        P->g0[b * n_species + s] = g0[s];
      }
    }
    if (precision == TG_FP64) build_plan<double>(P);
    else build_plan<float>(P);
    *out = P;
    return TG_OK;
  });
  if (rc != TG_OK && P) tg_plan_destroy(P);
  return rc;
}

int tg_plan_destroy(tg_plan p) {
  if (!p) return TG_OK;
  for (auto& kv : p->groups) delete kv.second;
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->dmem) (void)hipFree(p->dmem);
  for (auto& s : p->scratch)
    if (s) (void)hipFree(s);
  if (p->dflag) (void)hipFree(p->dflag);
  if (p->adj_ws) (void)hipFree(p->adj_ws);
  if (p->diag_part) (void)hipFree(p->diag_part);
  if (p->slice_mem) (void)hipFree(p->slice_mem);
  for (auto& kv : p->coupled_graphs) (void)hipGraphExecDestroy(kv.second);
  delete p;
  return TG_OK;
}

int tg_plan_state_size(tg_plan p, int64_t* elems, int32_t* elem_bytes) {
  return guarded([&] {
    TG_REQUIRE(p && elems && elem_bytes, TG_EINVAL, "null pointer");
    *elems = p->state_elems;
    *elem_bytes = p->esize;
    return TG_OK;
  });
}

int tg_plan_reference(tg_plan p, double* w_ref) {
  return guarded([&] {
    TG_REQUIRE(p && w_ref, TG_EINVAL, "null pointer");
    std::memcpy(w_ref, p->wref.data(), p->wref.size() * sizeof(double));
    return TG_OK;
  });
}


int tg_step(tg_plan p, void* state, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && state, TG_EINVAL, "tg_step: null pointer");
    TG_REQUIRE(aligned(p, state), TG_EINVAL, "tg_step: state must be aligned to 4 elements");
    step_any(p, state, static_cast<hipStream_t>(stream));
    return TG_OK;
  });
}

// n plain steps: resident launches on route 4; else replays of the
// kLongGraph-step graph, then of the kStepsPerGraph-step one, then single
// steps.  The first call that replays a graph captures both, so a warm-up
// of kStepsPerGraph steps keeps the captures out of a later timed run.
static void run_plain(tg_plan_s* p, void* state, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  if (active_route(p) == 4) {
    run_resident_any(p, state, n, st);
    return;
  }
  int64_t left = n;
  if (n >= kStepsPerGraph) {
    hipGraphExec_t g_short = step_graph(p, state, kStepsPerGraph);
    hipGraphExec_t g_long = step_graph(p, state, kLongGraph);
    for (; left >= kLongGraph; left -= kLongGraph) hip_check(hipGraphLaunch(g_long, st), "graph launch");
    for (; left >= kStepsPerGraph; left -= kStepsPerGraph) hip_check(hipGraphLaunch(g_short, st), "graph launch");
    // the rest (fewer than kStepsPerGraph steps) from graphs of 4, 2 and 1
    // steps, captured with the others
    for (int k = kStepsPerGraph / 2; k >= 1; k /= 2) {
      hipGraphExec_t g = step_graph(p, state, k);
      if (left >= k) {
        hip_check(hipGraphLaunch(g, st), "graph launch");
        left -= k;
      }
    }
  }
  for (; left > 0; --left) step_any(p, state, st);
}

int tg_run(tg_plan p, void* state, int64_t n_steps, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && state && n_steps >= 0, TG_EINVAL, "tg_run: bad argument");
    TG_REQUIRE(aligned(p, state), TG_EINVAL, "tg_run: state must be aligned to 4 elements");
    hipStream_t st = static_cast<hipStream_t>(stream);
    run_plain(p, state, n_steps, st);
    int flag = 0;
    hip_check(hipMemcpyAsync(&flag, p->dflag, sizeof(int), hipMemcpyDeviceToHost, st), "tg_run: flag copy");
    hip_check(hipStreamSynchronize(st), "tg_run: synchronize");
    if (flag) {
      hip_check(hipMemset(p->dflag, 0, sizeof(int)), "tg_run: flag reset");
      throw Fail(TG_ENONFINITE, "tg_run: non-finite value in the state");
    }
    return TG_OK;
  });
}

int tg_run_history(tg_plan p, void* state, int64_t n_steps, void* history, int32_t history_fp64, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && state && history && n_steps >= 0, TG_EINVAL, "tg_run_history: bad argument");
    TG_REQUIRE(aligned(p, state), TG_EINVAL, "tg_run_history: state must be aligned to 4 elements");
    const bool f64 = p->precision == TG_FP64;
    const bool widen = history_fp64 != 0 && !f64;
    const size_t bytes = static_cast<size_t>(p->state_elems) * (f64 ? 8 : 4);
    const size_t hslot = static_cast<size_t>(p->state_elems) * (f64 || widen ? 8 : 4);
    const char* s0 = static_cast<const char*>(state);
    const char* h0 = static_cast<const char*>(history);
    const size_t hbytes = hslot * static_cast<size_t>(n_steps);
    TG_REQUIRE(h0 + hbytes <= s0 || s0 + bytes <= h0, TG_EINVAL, "tg_run_history: history overlaps the state");
    TG_REQUIRE(!widen || (reinterpret_cast<uintptr_t>(history) & 15) == 0, TG_EINVAL,
               "tg_run_history: an FP64 history must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* h = static_cast<char*>(history);
    for (int64_t k = 0; k < n_steps; ++k) {
      void* slot = h + static_cast<size_t>(k) * hslot;
      if (widen)
        hip_check(tg::launch_widen(static_cast<const float*>(state), static_cast<double*>(slot), p->state_elems, st),
                  "tg_run_history: widen");
      else
        hip_check(hipMemcpyAsync(slot, state, bytes, hipMemcpyDeviceToDevice, st), "tg_run_history: copy");
      step_any(p, state, st);
    }
    int flag = 0;
    hip_check(hipMemcpyAsync(&flag, p->dflag, sizeof(int), hipMemcpyDeviceToHost, st), "tg_run_history: flag copy");
    hip_check(hipStreamSynchronize(st), "tg_run_history: synchronize");
    if (flag) {
      hip_check(hipMemset(p->dflag, 0, sizeof(int)), "tg_run_history: flag reset");
      throw Fail(TG_ENONFINITE, "tg_run_history: non-finite value in the state");
    }
    return TG_OK;
  });
}

int tg_run_prepare(tg_plan p, void* state) {
  return guarded([&] {
    TG_REQUIRE(p && state, TG_EINVAL, "tg_run_prepare: null pointer");
    TG_REQUIRE(aligned(p, state), TG_EINVAL, "tg_run_prepare: state must be aligned to 4 elements");
    if (active_route(p) != 4) {
      (void)step_graph(p, state, kStepsPerGraph);
      (void)step_graph(p, state, kLongGraph);
      for (int k = kStepsPerGraph / 2; k >= 1; k /= 2) (void)step_graph(p, state, k);
    }
    return TG_OK;
  });
}

int tg_sync_status(tg_plan p, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p, TG_EINVAL, "tg_sync_status: null plan");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int flag = 0;
    hip_check(hipMemcpyAsync(&flag, p->dflag, sizeof(int), hipMemcpyDeviceToHost, st), "tg_sync_status: flag copy");
    hip_check(hipStreamSynchronize(st), "tg_sync_status: synchronize");
    if (flag) {
      hip_check(hipMemset(p->dflag, 0, sizeof(int)), "tg_sync_status: flag reset");
      throw Fail(TG_ENONFINITE, "tg_sync_status: non-finite value in the state");
    }
    return TG_OK;
  });
}

int tg_step_diag(tg_plan p, void* state, double* diag, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && state && diag, TG_EINVAL, "tg_step_diag: null pointer");
    TG_REQUIRE(aligned(p, state), TG_EINVAL, "tg_step_diag: state must be aligned to 4 elements");
    const tg::DiagArgs d = diag_args(p, diag);
    step_any(p, state, static_cast<hipStream_t>(stream), &d);
    return TG_OK;
  });
}

int tg_step_diag_noalloc(tg_plan p, void* state, double* diag, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && state && diag, TG_EINVAL, "tg_step_diag_noalloc: null pointer");
    TG_REQUIRE(aligned(p, state), TG_EINVAL, "tg_step_diag_noalloc: state must be aligned to 4 elements");
    // the same partial-sum layout as tg_step_diag: cap slots of two doubles
    // per slab, every slot a launch reads written by that launch (nothing
    // has to start at zero)
    const int64_t cap = p->npts / 8 + 64;
    const int64_t need = 2 * cap * static_cast<int64_t>(p->nslab) * static_cast<int64_t>(sizeof(double));
    TG_REQUIRE(need <= static_cast<int64_t>(tg::kStaticScratchBytes), TG_EINVAL,
               "tg_step_diag_noalloc: the plan needs " + std::to_string(need) +
                   " bytes of indicator partial sums, more than the static scratch of " +
                   std::to_string(tg::kStaticScratchBytes) + " bytes (use tg_step_diag)");
    void* part = nullptr;
    hip_check(tg::static_scratch(&part), "tg_step_diag_noalloc: static scratch address");
    tg::DiagArgs d{};
    d.part = static_cast<double*>(part);
    d.out = diag;
    d.w1 = p->d_w1;
    d.w23 = p->d_w23;
    d.wref = p->d_wref;
    d.wsum_inv = p->wsum_inv;
    d.cap = static_cast<int>(cap);
    step_any(p, state, static_cast<hipStream_t>(stream), &d);
    return TG_OK;
  });
}

int tg_run_diag(tg_plan p, void* state, int64_t n_steps, int32_t every, double* diag, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && state && n_steps >= 0 && every >= 1, TG_EINVAL, "tg_run_diag: bad argument");
    TG_REQUIRE(diag || n_steps / every == 0, TG_EINVAL, "tg_run_diag: null record buffer");
    TG_REQUIRE(aligned(p, state), TG_EINVAL, "tg_run_diag: state must be aligned to 4 elements");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t records = n_steps / every;
    tg::DiagArgs d = records > 0 ? diag_args(p, diag) : tg::DiagArgs{};
    int64_t done = 0;
    for (int64_t r = 0; r < records; ++r) {
      // every - 1 plain steps (run_plain), then the recorded step
      run_plain(p, state, every - 1, st);
      d.out = diag + 2 * static_cast<int64_t>(p->nslab) * r;
      step_any(p, state, st, &d);
      done += every;
    }
    run_plain(p, state, n_steps - done, st);
    int flag = 0;
    hip_check(hipMemcpyAsync(&flag, p->dflag, sizeof(int), hipMemcpyDeviceToHost, st), "tg_run_diag: flag copy");
    hip_check(hipStreamSynchronize(st), "tg_run_diag: synchronize");
    if (flag) {
      hip_check(hipMemset(p->dflag, 0, sizeof(int)), "tg_run_diag: flag reset");
      throw Fail(TG_ENONFINITE, "tg_run_diag: non-finite value in the state");
    }
    return TG_OK;
  });
}

static Coupled check_coupled(tg_plan bulk, tg_plan surface, void* ub, void* us, const double* coupling) {
  TG_REQUIRE(bulk && surface && ub && us && coupling, TG_EINVAL, "bulk-surface step: null pointer");
  const bool ball = bulk->grid.geometry == TG_BALL && surface->grid.geometry == TG_SPHERE;
  const bool cyl = bulk->grid.geometry == TG_CYLINDER && surface->grid.geometry == TG_DISK;
  TG_REQUIRE(ball || cyl, TG_EINVAL,
             "bulk-surface step: needs a ball plan and a sphere plan, or a cylinder plan and a disk plan");
  TG_REQUIRE(bulk->ns == 2 && surface->ns == 2, TG_EINVAL, "bulk-surface step: two species on each side");
  TG_REQUIRE(bulk->batch == surface->batch, TG_EINVAL, "bulk-surface step: batch sizes differ");
  TG_REQUIRE(bulk->precision == surface->precision, TG_EINVAL, "bulk-surface step: precisions differ");
  if (ball) {
    TG_REQUIRE(bulk->grid.n[1] == surface->grid.n[0] && bulk->grid.n[2] == surface->grid.n[1], TG_EINVAL,
               "bulk-surface step: the sphere grid must be the ball's (theta, phi) grid");
    TG_REQUIRE(bulk->grid.extent[0] == surface->grid.extent[0], TG_EINVAL,
               "bulk-surface step: the sphere's radius must be the ball's");
  } else {
    TG_REQUIRE(bulk->grid.n[0] == surface->grid.n[0] && bulk->grid.n[1] == surface->grid.n[1], TG_EINVAL,
               "bulk-surface step: the disk grid must be the cylinder's (rho, theta) grid");
    TG_REQUIRE(bulk->grid.extent[0] == surface->grid.extent[0], TG_EINVAL,
               "bulk-surface step: the disk's radius must be the cylinder's");
    TG_REQUIRE(surface->reaction == TG_REACT_DIB, TG_EINVAL,
               "bulk-surface step: the bottom disk needs the DIB kinetics (their p, q are the exchange)");
  }
  TG_REQUIRE(bulk != surface && ub != us, TG_EINVAL, "bulk-surface step: distinct plans and states");
  TG_REQUIRE(aligned(bulk, ub) && aligned(surface, us), TG_EINVAL,
             "bulk-surface step: states must be aligned to 4 elements");
  for (int q = 0; q < 5; ++q)
    TG_REQUIRE(std::isfinite(coupling[q]), TG_EINVAL, "bulk-surface step: non-finite coupling constant");
  Coupled C{bulk, surface, {coupling[0], coupling[1], coupling[2], coupling[3], coupling[4]}};
  return C;
}

int tg_coupled_step(tg_plan bulk, tg_plan surface, void* bulk_state, void* surface_state, const double* coupling,
                    void* stream) {
  return guarded([&] {
    const Coupled C = check_coupled(bulk, surface, bulk_state, surface_state, coupling);
    coupled_any(C, bulk_state, surface_state, static_cast<hipStream_t>(stream));
    return TG_OK;
  });
}

int tg_coupled_run(tg_plan bulk, tg_plan surface, void* bulk_state, void* surface_state, const double* coupling,
                   int64_t n_steps, void* stream) {
  return guarded([&] {
    TG_REQUIRE(n_steps >= 0, TG_EINVAL, "tg_coupled_run: negative step count");
    const Coupled C = check_coupled(bulk, surface, bulk_state, surface_state, coupling);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t full = n_steps / kStepsPerGraph;
    if (full > 0) {
      std::vector<uint64_t> key = {surface->serial, surface->version, bulk->version,
                                   reinterpret_cast<uint64_t>(bulk_state), reinterpret_cast<uint64_t>(surface_state)};
      for (double v : C.c) {
        uint64_t b;
        std::memcpy(&b, &v, sizeof(b));
        key.push_back(b);
      }
      hipGraphExec_t ex = nullptr;
      auto it = bulk->coupled_graphs.find(key);
      if (it != bulk->coupled_graphs.end()) {
        ex = it->second;
      } else {
        if (!bulk->capture_stream)
          hip_check(hipStreamCreateWithFlags(&bulk->capture_stream, hipStreamNonBlocking), "capture stream");
        hipGraph_t graph = nullptr;
        hip_check(hipStreamBeginCapture(bulk->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        try {
          for (int i = 0; i < kStepsPerGraph; ++i) coupled_any(C, bulk_state, surface_state, bulk->capture_stream);
        } catch (...) {
          (void)hipStreamEndCapture(bulk->capture_stream, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          throw;
        }
        hip_check(hipStreamEndCapture(bulk->capture_stream, &graph), "end capture");
        hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        hip_check(e, "graph instantiate");
        bulk->coupled_graphs[key] = ex;
      }
      for (int64_t i = 0; i < full; ++i) hip_check(hipGraphLaunch(ex, st), "tg_coupled_run: graph launch");
    }
    for (int64_t i = full * kStepsPerGraph; i < n_steps; ++i) coupled_any(C, bulk_state, surface_state, st);
    int flag[2] = {0, 0};
    hip_check(hipMemcpyAsync(&flag[0], bulk->dflag, sizeof(int), hipMemcpyDeviceToHost, st), "flag copy");
    hip_check(hipMemcpyAsync(&flag[1], surface->dflag, sizeof(int), hipMemcpyDeviceToHost, st), "flag copy");
    hip_check(hipStreamSynchronize(st), "tg_coupled_run: synchronize");
    if (flag[0] || flag[1]) {
      hip_check(hipMemset(bulk->dflag, 0, sizeof(int)), "flag reset");
      hip_check(hipMemset(surface->dflag, 0, sizeof(int)), "flag reset");
      throw Fail(TG_ENONFINITE, "tg_coupled_run: non-finite value in a state");
    }
    return TG_OK;
  });
}

int tg_apply_chain_op(tg_plan p, int32_t op, const void* in, void* out, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && in && out && in != out, TG_EINVAL, "tg_apply_chain_op: bad pointers");
    TG_REQUIRE(aligned(p, in) && aligned(p, out), TG_EINVAL, "tg_apply_chain_op: buffers must be aligned to 4 elements");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (use_fused(p) || active_route(p) == 4) {
      TG_REQUIRE(op >= 0 && op < static_cast<int32_t>(p->fused.size()), TG_EINVAL, "tg_apply_chain_op: op out of range");
      const bool from_state = active_route(p) != 2;
      if (p->precision == TG_FP64) launch_fused<double>(p, p->fused[op], in, out, false, from_state, st);
      else launch_fused<float>(p, p->fused[op], in, out, false, from_state, st);
      return TG_OK;
    }
    const auto& chain = chain_of(p);
    TG_REQUIRE(op >= 0 && op < static_cast<int32_t>(chain.size()), TG_EINVAL, "tg_apply_chain_op: op out of range");
    const auto& c = chain[op];
    const int epi = c.epi == tg::EPI_UPDATE ? tg::EPI_STORE : c.epi;
    if (p->precision == TG_FP64) launch_op<double>(p, c, in, out, epi, st);
    else launch_op<float>(p, c, in, out, epi, st);
    return TG_OK;
  });
}

int tg_plan_set_route(tg_plan p, int32_t route) {
  return guarded([&] {
    TG_REQUIRE(p && route >= 0 && route <= 4, TG_EINVAL, "tg_plan_set_route: bad argument");
    TG_REQUIRE(!((route == 1 || route == 3) && bf16_terms(p->precision)), TG_ENOTSUP,
               "tg_plan_set_route: split-bf16 plans have no per-mode route");
    if (route == 3) ensure_slice_chain(p);
    TG_REQUIRE(route != 4 || resident_ok(p), TG_ENOTSUP,
               "tg_plan_set_route: the resident route needs a disk plan in FP64 or FP32 whose species fit in LDS");
    if (route != p->route) {
      drop_graphs(p);
      p->route = route;
      fit_tiles_to_route(p);
    }
    return TG_OK;
  });
}

int tg_plan_route(tg_plan p, int32_t* route) {
  return guarded([&] {
    TG_REQUIRE(p && route, TG_EINVAL, "tg_plan_route: null pointer");
    *route = active_route(p);
    return TG_OK;
  });
}

int tg_plan_chain(tg_plan p, int32_t* n_ops, int32_t* modes, double* flops) {
  return guarded([&] {
    TG_REQUIRE(p && n_ops, TG_EINVAL, "tg_plan_chain: null pointer");
    if (use_fused(p) || active_route(p) == 4) {
      *n_ops = static_cast<int32_t>(p->fused.size());
      for (size_t i = 0; i < p->fused.size(); ++i) {
        if (modes) modes[i] = p->fused[i].mode;
        if (flops) flops[i] = p->fused[i].flops;
      }
    } else {
      const auto& chain = chain_of(p);
      *n_ops = static_cast<int32_t>(chain.size());
      for (size_t i = 0; i < chain.size(); ++i) {
        if (modes) modes[i] = chain[i].mode;
        if (flops) flops[i] = chain[i].flops;
      }
    }
    return TG_OK;
  });
}

int tg_adjoint_step(tg_plan p, const void* state_n, void* lambda, double* grad, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && state_n && lambda && grad && state_n != lambda, TG_EINVAL, "tg_adjoint_step: bad pointers");
    TG_REQUIRE(aligned(p, state_n) && aligned(p, lambda), TG_EINVAL, "tg_adjoint_step: buffers must be aligned");
    TG_REQUIRE(p->reaction <= TG_REACT_SCHNAKENBERG_SCALED, TG_ENOTSUP,
               "tg_adjoint_step: no adjoint for the linear and DIB kinetics");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->precision == TG_FP64) adjoint_impl<double>(p, state_n, lambda, grad, st);
    else adjoint_impl<float>(p, state_n, lambda, grad, st);
    return TG_OK;
  });
}

int tg_apply_operator(tg_plan p, const void* in, void* out, int32_t what, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && in && out && in != out, TG_EINVAL, "tg_apply_operator: bad pointers");
    TG_REQUIRE(what >= 0 && what <= 2, TG_EINVAL, "tg_apply_operator: bad selector");
    const size_t bytes = static_cast<size_t>(p->state_elems) * p->esize;
    const char* ib = static_cast<const char*>(in);
    const char* ob = static_cast<const char*>(out);
    TG_REQUIRE(ib + bytes <= ob || ob + bytes <= ib, TG_EINVAL, "tg_apply_operator: in and out overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->precision == TG_FP64) launch_stencil_stage<double>(p, in, out, what, st);
    else launch_stencil_stage<float>(p, in, out, what, st);
    return TG_OK;
  });
}

int tg_apply_split_phi1(tg_plan p, const void* in, void* out, void* stream) {
  return guarded([&] {
    TG_REQUIRE(p && in && out && in != out, TG_EINVAL, "tg_apply_split_phi1: bad pointers");
    TG_REQUIRE(aligned(p, in) && aligned(p, out), TG_EINVAL, "tg_apply_split_phi1: buffers must be aligned to 4 elements");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (use_fused(p)) {
      if (p->precision == TG_FP64) run_fused<double>(p, in, out, false, false, st);
      else run_fused<float>(p, in, out, false, false, st);
    } else {
      if (p->precision == TG_FP64) run_chain<double>(p, in, out, false, st);
      else run_chain<float>(p, in, out, false, st);
    }
    return TG_OK;
  });
}

int tg_group_run(const tg_plan* plans, int32_t n_plans, void* const* states, int64_t n_steps, void* stream) {
  return guarded([&] {
    TG_REQUIRE(n_steps >= 0, TG_EINVAL, "tg_group_run: negative step count");
    tg_group_s* G = find_group(plans, n_plans, states);
    hipStream_t st = static_cast<hipStream_t>(stream);
    bool resident = false;
    for (auto* P : G->plans) resident = resident || active_route(P) == 4;
    if (resident) {
      // members on route 4 run all their steps in resident launches, the
      // others their own graph replays (the members are independent)
      for (size_t q = 0; q < G->plans.size(); ++q) run_plain(G->plans[q], G->states[q], n_steps, st);
    } else {
      const int64_t full = n_steps / kStepsPerGraph;
      for (int64_t it = 0; it < full; ++it) hip_check(hipGraphLaunch(G->graph, st), "tg_group_run: graph launch");
      for (int64_t it = full * kStepsPerGraph; it < n_steps; ++it) group_step_any(G, st);
    }
    std::vector<int> flags(G->plans.size(), 0);
    for (size_t q = 0; q < G->plans.size(); ++q)
      hip_check(hipMemcpyAsync(&flags[q], G->plans[q]->dflag, sizeof(int), hipMemcpyDeviceToHost, st),
                "tg_group_run: flag copy");
    hip_check(hipStreamSynchronize(st), "tg_group_run: synchronize");
    bool bad = false;
    for (size_t q = 0; q < G->plans.size(); ++q)
      if (flags[q]) {
        hip_check(hipMemset(G->plans[q]->dflag, 0, sizeof(int)), "tg_group_run: flag reset");
        bad = true;
      }
    if (bad) throw Fail(TG_ENONFINITE, "tg_group_run: non-finite value in a state");
    return TG_OK;
  });
}

int tg_group_autotune(const tg_plan* plans, int32_t n_plans, void* const* states, int32_t iters, void* stream,
                      double* best_us) {
  std::vector<void*> tmp;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  tg_plan_s* P0 = (plans && n_plans >= 1) ? plans[0] : nullptr;
  int rc = guarded([&] {
    TG_REQUIRE(plans && states && n_plans >= 1 && n_plans <= tg::kMaxGroup && iters >= 1 && iters <= 10000,
               TG_EINVAL, "tg_group_autotune: bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<tg_plan_s*> ps(plans, plans + n_plans);
    bool fused_all = true;
    for (int q = 0; q < n_plans; ++q) {
      TG_REQUIRE(ps[q] && states[q] && aligned(ps[q], states[q]), TG_EINVAL, "tg_group_autotune: bad plan or state");
      fused_all = fused_all && ps[q]->fused_ok;
      void* t = nullptr;
      const size_t bytes = static_cast<size_t>(ps[q]->state_elems) * ps[q]->esize;
      hip_check(hipMalloc(&t, bytes), "hipMalloc(group autotune state)");
      tmp.push_back(t);
      hip_check(hipMemcpyAsync(t, states[q], bytes, hipMemcpyDeviceToDevice, st), "group autotune copy");
    }
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    std::vector<int> routes = fused_all ? std::vector<int>{0, 2} : std::vector<int>{};
    if (routes.empty()) {
      if (best_us) *best_us = 0.0;
      return TG_OK;  // nothing to choose: the plans run their own routes
    }
    auto set_route = [&](int r) {
      for (auto* P : ps)
        if (P->route != r) {
          drop_graphs(P);
          P->route = r;
          fit_tiles_to_route(P);
        }
    };
    // each member's column tiles; on the stencil-apart route the products
    // without a plane tail may also take 32 columns where only the in-tile
    // stencil kept them at 16 (whole 128-byte lines of an FP32 row)
    std::vector<std::vector<int>> tn0(n_plans);
    auto save_tiles = [&]() {
      for (int q = 0; q < n_plans; ++q) {
        tn0[q].clear();
        for (const auto& op : ps[q]->fused) tn0[q].push_back(op.kind == 0 ? op.sa.tn : 0);
      }
    };
    auto set_wide = [&](bool wide) {
      for (int q = 0; q < n_plans; ++q) {
        bool changed = false;
        for (size_t k = 0; k < ps[q]->fused.size(); ++k) {
          auto& op = ps[q]->fused[k];
          if (op.kind != 0 || op.sa.plane) continue;
          const int t = wide && tn0[q][k] == 16 && fused_tile_fits(ps[q], op, 32) ? 32 : tn0[q][k];
          changed = changed || t != op.sa.tn;
          op.sa.tn = t;
        }
        if (changed) drop_graphs(ps[q]);
      }
    };
    std::vector<std::pair<int, bool>> configs;
    for (int r : routes) {
      configs.push_back({r, false});
      if (r == 2) configs.push_back({r, true});
    }
    double best = std::numeric_limits<double>::infinity();
    int best_route = routes[0];
    bool best_wide = false;
    for (const auto& [r, wide] : configs) {
      set_route(r);
      if (!wide) save_tiles();
      set_wide(wide);
      tg_group_s* G = find_group(plans, n_plans, tmp.data());
      for (int w = 0; w < 2; ++w) group_step_any(G, st);
      hip_check(hipEventRecord(e0, st), "event record");
      for (int it = 0; it < iters; ++it) group_step_any(G, st);
      hip_check(hipEventRecord(e1, st), "event record");
      hip_check(hipEventSynchronize(e1), "event sync");
      float ms = 0.0f;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
      const double us = 1e3 * static_cast<double>(ms) / iters;
      if (us < (std::isfinite(best) ? kTuneGain * best : best)) {
        best = us;
        best_route = r;
        best_wide = wide;
      }
      set_wide(false);
    }
    set_route(best_route);
    save_tiles();
    set_wide(best_wide);
    if (best_us) *best_us = best;
    return TG_OK;
  });
  // drop the groups built on the private copies, then the copies
  if (P0 && !tmp.empty()) {
    (void)hipDeviceSynchronize();
    for (auto it = P0->groups.begin(); it != P0->groups.end();) {
      bool uses_tmp = false;
      for (size_t k = 2; k < it->first.size(); k += 3)
        for (void* t : tmp) uses_tmp = uses_tmp || it->first[k] == reinterpret_cast<uintptr_t>(t);
      if (uses_tmp) {
        delete it->second;
        it = P0->groups.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (void* t : tmp) (void)hipFree(t);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

int tg_group_info(const tg_plan* plans, int32_t n_plans, void* const* states, int32_t* grouped,
                  int32_t* launches_per_step) {
  return guarded([&] {
    tg_group_s* G = find_group(plans, n_plans, states);
    if (grouped) *grouped = G->grouped ? 1 : 0;
    if (launches_per_step) *launches_per_step = G->launches_per_step();
    return TG_OK;
  });
}

int tg_plan_tiles(tg_plan p, int32_t* n_ops, int32_t* tiles) {
  return guarded([&] {
    TG_REQUIRE(p && n_ops, TG_EINVAL, "tg_plan_tiles: null pointer");
    *n_ops = static_cast<int32_t>(p->fused.size());
    if (tiles)
      for (size_t k = 0; k < p->fused.size(); ++k)
        tiles[k] = p->fused[k].kind == 0 ? p->fused[k].sa.tn : p->fused[k].fa.tm;
    return TG_OK;
  });
}

int tg_plan_set_tiles(tg_plan p, int32_t n_ops, const int32_t* tiles) {
  return guarded([&] {
    TG_REQUIRE(p && tiles && n_ops == static_cast<int32_t>(p->fused.size()), TG_EINVAL,
               "tg_plan_set_tiles: one tile width per fused launch");
    for (int k = 0; k < n_ops; ++k) {
      const auto& op = p->fused[k];
      const int t = tiles[k];
      if (op.kind == 1) {
        TG_REQUIRE(t == 16 || t == 32, TG_EINVAL, "tg_plan_set_tiles: first-mode tiles are 16 or 32 rows");
      } else {
        TG_REQUIRE(t == 16 || (t > 0 && t % 32 == 0), TG_EINVAL, "tg_plan_set_tiles: 16 or a multiple of 32 columns");
        TG_REQUIRE(!op.sa.plane || t == op.sa.tn, TG_EINVAL, "tg_plan_set_tiles: a plane launch keeps its width");
      }
      // as the active route launches it (the in-tile stencil's LDS only
      // where that route computes F in the tile load)
      TG_REQUIRE(fused_tile_fits(p, op, t), TG_EINVAL, "tg_plan_set_tiles: tile does not fit in LDS");
    }
    for (int k = 0; k < n_ops; ++k) {
      if (p->fused[k].kind == 1) p->fused[k].fa.tm = tiles[k];
      else p->fused[k].sa.tn = tiles[k];
    }
    drop_graphs(p);
    return TG_OK;
  });
}

int tg_plan_autotune(tg_plan p, const void* state, int32_t iters, void* stream, double* best_us) {
  void* tmp = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = guarded([&] {
    TG_REQUIRE(p && state && iters >= 1 && iters <= 10000, TG_EINVAL, "tg_plan_autotune: bad argument");
    TG_REQUIRE(aligned(p, state), TG_EINVAL, "tg_plan_autotune: state must be aligned to 4 elements");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t bytes = static_cast<size_t>(p->state_elems) * p->esize;
    hip_check(hipMalloc(&tmp, bytes), "hipMalloc(autotune state)");
    hip_check(hipMemcpyAsync(tmp, state, bytes, hipMemcpyDeviceToDevice, st), "autotune copy");
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    const int nt = bf16_terms(p->precision);
    auto lds_ok = [&](const tg::FusedOp& op) {
      return fused_tile_fits(p, op, op.kind == 0 ? op.sa.tn : op.fa.tm);
    };
    // time `iters` steps of the current configuration (+inf if it cannot
    // run): direct launches, or on route 4 one resident launch of `iters`
    // steps, as tg_run takes them
    auto measure = [&]() {
      try {
        const bool res = active_route(p) == 4;
        if (res) run_resident_any(p, tmp, 2, st);
        else
          for (int w = 0; w < 2; ++w) step_any(p, tmp, st);
        hip_check(hipEventRecord(e0, st), "event record");
        if (res) run_resident_any(p, tmp, iters, st);
        else
          for (int it = 0; it < iters; ++it) step_any(p, tmp, st);
        hip_check(hipEventRecord(e1, st), "event record");
        hip_check(hipEventSynchronize(e1), "event sync");
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
        return 1e3 * static_cast<double>(ms) / iters;
      } catch (const Fail&) {
        (void)hipStreamSynchronize(st);
        return std::numeric_limits<double>::infinity();
      }
    };
    std::vector<int> routes;
    if (p->fused_ok) routes = {0, 2};
    if (!nt) routes.push_back(1);
    if (slice_capable(p)) {
      ensure_slice_chain(p);
      routes.push_back(3);
    }
    if (resident_ok(p)) routes.push_back(4);
    const int saved_route = p->route;
    double best = std::numeric_limits<double>::infinity();
    int best_route = saved_route;
    std::vector<int> best_tiles;
    auto tiles_now = [&]() {
      std::vector<int> t;
      for (const auto& op : p->fused) t.push_back(op.kind == 0 ? op.sa.tn : op.fa.tm);
      return t;
    };
    auto set_tiles = [&](const std::vector<int>& t) {
      for (size_t k = 0; k < p->fused.size(); ++k) {
        if (p->fused[k].kind == 0) p->fused[k].sa.tn = t[k];
        else p->fused[k].fa.tm = t[k];
      }
    };
    const std::vector<int> start_tiles = tiles_now();
    for (int r : routes) {
      p->route = r;
      set_tiles(start_tiles);
      fit_tiles_to_route(p);
      double cur = measure();
      if (r == 0 || r == 2) {
        // coordinate descent over the fused ops' tile sizes
        for (size_t k = 0; k < p->fused.size(); ++k) {
          tg::FusedOp& op = p->fused[k];
          std::vector<int> cand;
          if (op.kind == 1) cand = {16, 32};
          else if (op.sa.plane) cand = {op.sa.tn};  // whole planes: fixed width
          else cand = {16, 32, 64};
          int keep = op.kind == 0 ? op.sa.tn : op.fa.tm;
          for (int c : cand) {
            if (c == keep) continue;
            const int old = keep;
            if (op.kind == 0) op.sa.tn = c;
            else op.fa.tm = c;
            double t = lds_ok(op) ? measure() : std::numeric_limits<double>::infinity();
            if (t < kTuneGain * cur) {
              cur = t;
              keep = c;
            } else {
              if (op.kind == 0) op.sa.tn = old;
              else op.fa.tm = old;
            }
          }
        }
      }
      if (cur < (best_tiles.empty() ? best : kTuneGain * best)) {
        best = cur;
        best_route = r;
        best_tiles = tiles_now();
      }
    }
    p->route = best_route;
    set_tiles(best_tiles.empty() ? start_tiles : best_tiles);
    fit_tiles_to_route(p);
    (void)saved_route;
    drop_graphs(p);
    if (best_us) *best_us = best;
    TG_REQUIRE(std::isfinite(best), TG_EHIP, "tg_plan_autotune: no configuration ran");
    return TG_OK;
  });
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (tmp) {
    (void)hipDeviceSynchronize();
    (void)hipFree(tmp);
  }
  return rc;
}

int tg_run_timed(tg_plan p, void* state, int64_t n_steps, void* stream, int32_t max_launches, int32_t* n_launches,
                 double* launch_us) {
  LaunchEvents le;
  int rc = guarded([&] {
    TG_REQUIRE(p && state && n_launches && launch_us && n_steps >= 1 && n_steps <= 100000 && max_launches >= 1,
               TG_EINVAL, "tg_run_timed: bad argument");
    TG_REQUIRE(aligned(p, state), TG_EINVAL, "tg_run_timed: state must be aligned to 4 elements");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int L = step_launches(p);
    TG_REQUIRE(L <= max_launches, TG_EINVAL, "tg_run_timed: more launches per step than max_launches");
    le.ev.resize(static_cast<size_t>(n_steps) * (L + 1), nullptr);
    for (auto& e : le.ev) hip_check(hipEventCreate(&e), "event create");
    for (int64_t it = 0; it < n_steps; ++it) {
      g_launch_events = &le;
      try {
        step_any(p, state, st);
      } catch (...) {
        g_launch_events = nullptr;
        throw;
      }
      g_launch_events = nullptr;
      hip_check(hipEventRecord(le.ev[le.next++], st), "event record");  // end of the step's last launch
    }
    hip_check(hipStreamSynchronize(st), "tg_run_timed: synchronize");
    TG_REQUIRE(le.next == le.ev.size(), TG_EINVAL, "tg_run_timed: unexpected launch count");
    std::vector<double> acc(L, 0.0);
    for (int64_t it = 0; it < n_steps; ++it)
      for (int l = 0; l < L; ++l) {
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, le.ev[it * (L + 1) + l], le.ev[it * (L + 1) + l + 1]), "event time");
        acc[l] += ms;
      }
    *n_launches = L;
    for (int l = 0; l < L; ++l) launch_us[l] = 1e3 * acc[l] / static_cast<double>(n_steps);
    return TG_OK;
  });
  g_launch_events = nullptr;
  for (auto& e : le.ev)
    if (e) (void)hipEventDestroy(e);
  return rc;
}

}  // extern "C"
