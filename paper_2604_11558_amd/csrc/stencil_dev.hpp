// Device evaluation of F = d_s M W + g(W) at one grid point (deviation form).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tg {

// p(ub, r, s) and q(vb, r, s) of the DIB kinetics (eq. (bulkcylnl); with
// ub = vb = 1 the surface-only model of eq. (DIBnl)); rp = (zeta1, ...,
// zeta5, eta1, ..., eta5).
__device__ __forceinline__ void dib_pq(const double* rp, double ub, double vb, double r, double s, double& p,
                                       double& q) {
  p = rp[1] * ub * (1.0 - s) * r - rp[2] * r * r * r - rp[3] * (s - rp[4]);
  q = rp[5] * vb * (1.0 + rp[6] * r) * (1.0 - s) * (1.0 - rp[7] * (1.0 - s)) -
      rp[8] * (1.0 + rp[9] * r) * s * (1.0 + rp[7] * s);
}

// Kinetics that only the stencil launch evaluates (plans with them compute
// F in a launch of its own): linear relaxation g_s = -k_s (w_s - c_s),
// constants (k_0, c_0, k_1, c_1, ...), and the DIB kinetics zeta1 (p, q) of
// two surface species with the bulk values set to 1.
__device__ __forceinline__ void reaction_ext(const StencilArgs& a, int inst, double d0, double d1, double d2,
                                             double& G0, double& G1, double& G2) {
  const int ns = a.nspecies;
  const double* rp = a.rparams + inst * kRParams;
  const double* wr = a.wref + inst * ns;
  G0 = G1 = G2 = 0.0;
  if (a.reaction == 4) {
    G0 = -rp[0] * ((wr[0] - rp[1]) + d0);
    if (ns > 1) G1 = -rp[2] * ((wr[1] - rp[3]) + d1);
    if (ns > 2) G2 = -rp[4] * ((wr[2] - rp[5]) + d2);
  } else if (a.reaction == 5) {
    double p, q;
    dib_pq(rp, 1.0, 1.0, wr[0] + d0, wr[1] + d1, p, q);
    G0 = rp[0] * p;
    G1 = rp[0] * q;
  }
}

// The reaction terms of all species at a point, expanded around the
// reference state w_ref so that no O(1) terms cancel: with deviations
// (p, q, r) from (u_r, v_r, w_r),
//   u^2 v - u_r^2 v_r = u_r^2 q + 2 u_r v_r p + 2 u_r p q + v_r p^2 + p^2 q.
__device__ __forceinline__ void reaction3(const StencilArgs& a, int inst, double dp, double dq, double dr,
                                          double& G0, double& G1, double& G2) {
  if (a.reaction >= 4) {
    reaction_ext(a, inst, dp, dq, dr, G0, G1, G2);
    return;
  }
  const int ns = a.nspecies;
  const double* rp = a.rparams + inst * kRParams;
  const double* wr = a.wref + inst * ns;
  const double* g0 = a.g0 + inst * ns;
  const double ur = wr[0], vr = wr[1];
  const double N = ur * ur * dq + 2.0 * ur * vr * dp + 2.0 * ur * dp * dq + vr * dp * dp + dp * dp * dq;
  if (a.reaction == 1 || a.reaction == 3) {  // (gamma times) Schnakenberg: a - u + u^2 v,  b - u^2 v
    const double gam = a.reaction == 3 ? rp[2] : 1.0;
    G0 = g0[0] + gam * (N - dp);
    G1 = g0[1] - gam * N;
    G2 = 0.0;
  } else {  // a - u + u^2 v - kappa u w,  b - u^2 v,  mu (u - w)
    const double kap = rp[2], mu = rp[3];
    const double wrr = wr[2];
    G0 = g0[0] - dp + N - kap * (ur * dr + wrr * dp + dp * dr);
    G1 = g0[1] - N;
    G2 = g0[2] + mu * (dp - dr);
  }
}

// The reaction constants of one instance, read once (uniform values) so that
// their loads are issued together at the start of a kernel.
struct ReactConst {
  int reaction;
  double ur, vr, wr, g0, g1, g2, kap, mu, gam;
};

__device__ __forceinline__ ReactConst react_const(const StencilArgs& a, int inst) {
  ReactConst c;
  c.reaction = a.reaction;
  const int ns = a.nspecies;
  const double* rp = a.rparams + inst * kRParams;
  const double* wr = a.wref + inst * ns;
  const double* g0 = a.g0 + inst * ns;
  c.ur = wr[0];
  c.vr = ns > 1 ? wr[1] : 0.0;
  c.wr = ns > 2 ? wr[2] : 0.0;
  c.g0 = g0[0];
  c.g1 = ns > 1 ? g0[1] : 0.0;
  c.g2 = ns > 2 ? g0[2] : 0.0;
  c.kap = rp[2];
  c.mu = rp[3];
  c.gam = c.reaction == 3 ? rp[2] : 1.0;
  return c;
}

// reaction3 with the constants already loaded
__device__ __forceinline__ void reaction3c(const ReactConst& c, double dp, double dq, double dr, double& G0,
                                           double& G1, double& G2) {
  const double ur = c.ur, vr = c.vr;
  const double N = ur * ur * dq + 2.0 * ur * vr * dp + 2.0 * ur * dp * dq + vr * dp * dp + dp * dp * dq;
  if (c.reaction == 1 || c.reaction == 3) {
    G0 = c.g0 + c.gam * (N - dp);
    G1 = c.g1 - c.gam * N;
    G2 = 0.0;
  } else {
    G0 = c.g0 - dp + N - c.kap * (ur * dr + c.wr * dp + dp * dr);
    G1 = c.g1 - N;
    G2 = c.g2 + c.mu * (dp - dr);
  }
}

__device__ __forceinline__ void reaction_dev(const StencilArgs& a, int inst, const double* w, double* G) {
  reaction3(a, inst, w[0], w[1], w[2], G[0], G[1], G[2]);
}

// d_s * sum_mu scale_mu(i,j,k) * (A_mu W)(i,j,k) for species sp at point
// (i, j, k) = p of one instance; Wi points at the instance's species 0.
template <typename T>
__device__ __forceinline__ double diffusion_dev(const StencilArgs& a, const T* Wi, int inst, int sp,
                                                int64_t p, int i, int j, int k) {
  const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
  const int64_t npts = static_cast<int64_t>(n1) * n2 * n3;
  const T* Ws = Wi + sp * npts;
  const int idx[3] = {i, j, k};
  const int64_t stride[3] = {1, n1, static_cast<int64_t>(n1) * n2};
  const int nm = a.nmax;
  const double w0 = static_cast<double>(Ws[p]);
  double acc = 0.0;
  for (int mu = 0; mu < a.ndim; ++mu) {
    const int x = idx[mu];
    const int nmu = a.n[mu];
    const double* cf = a.coef + mu * 3 * nm;
    const double lo = cf[x], dg = cf[nm + x], up = cf[2 * nm + x];
    const bool per = (a.periodic_mask >> mu) & 1;
    int xm = x - 1, xp = x + 1;
    if (xm < 0) xm = per ? nmu - 1 : -1;
    if (xp >= nmu) xp = per ? 0 : -1;
    const double wm = xm >= 0 ? static_cast<double>(Ws[p + (xm - x) * stride[mu]]) : 0.0;
    const double wp = xp >= 0 ? static_cast<double>(Ws[p + (xp - x) * stride[mu]]) : 0.0;
    const double* sc = a.scale + mu * 3 * nm;
    const double scl = sc[i] * sc[nm + j] * sc[2 * nm + k];
    acc += scl * (lo * wm + dg * w0 + up * wp);
  }
  return a.diff[inst * a.nspecies + sp] * acc;
}

// Same as diffusion_dev with 32-bit indexing and the mode count fixed at
// compile time (point index p < 2^31 is checked by the launchers).
template <typename T, int NDIM>
__device__ __forceinline__ double diffusion_fast(const StencilArgs& a, const T* Ws, double w0, int sp,
                                                 int inst, int p, int i, int j, int k) {
  const int n1 = a.n[0], n2 = a.n[1];
  const int stride[3] = {1, n1, n1 * n2};
  const int idx[3] = {i, j, k};
  const int nm = a.nmax;
  double acc = 0.0;
#pragma unroll
  for (int mu = 0; mu < NDIM; ++mu) {
    const int x = idx[mu];
    const int nmu = a.n[mu];
    const double* cf = a.coef + mu * 3 * nm;
    const bool per = (a.periodic_mask >> mu) & 1;
    const int dm = x > 0 ? -stride[mu] : (per ? (nmu - 1) * stride[mu] : 0);
    const int dp = x + 1 < nmu ? stride[mu] : (per ? -(nmu - 1) * stride[mu] : 0);
    // non-periodic ends have zero lo / up coefficients; the offset 0 then
    // just re-reads the centre value
    const double wm = static_cast<double>(Ws[p + dm]);
    const double wp = static_cast<double>(Ws[p + dp]);
    const double* sc = a.scale + mu * 3 * nm;
    const int sm = a.scale_mask >> (3 * mu);
    double scl = 1.0;  // unit scale vectors are not loaded
    if (sm & 1) scl *= sc[i];
    if (sm & 2) scl *= sc[nm + j];
    if (sm & 4) scl *= sc[2 * nm + k];
    acc += scl * (cf[x] * wm + cf[nm + x] * w0 + cf[2 * nm + x] * wp);
  }
  return a.diff[inst * a.nspecies + sp] * acc;
}

// F_sp at the point with coordinates (i, j, k), index p (32-bit); both the
// diffusion of species sp and the coupled reaction.
template <typename T>
__device__ __forceinline__ double stencil_point_ijk(const StencilArgs& a, int inst, int sp, int p, int i,
                                                    int j, int k) {
  const int npts = a.n[0] * a.n[1] * a.n[2];
  const int ns = a.nspecies;
  const T* Wi = static_cast<const T*>(a.W) + static_cast<int64_t>(inst) * ns * npts;
  // scalars selected by value: no dynamically indexed local arrays, which
  // would live in scratch memory
  const double w0 = static_cast<double>(Wi[p]);
  const double w1 = ns > 1 ? static_cast<double>(Wi[npts + p]) : 0.0;
  const double w2 = ns > 2 ? static_cast<double>(Wi[2 * npts + p]) : 0.0;
  const double wsp = sp == 0 ? w0 : (sp == 1 ? w1 : w2);
  double f = 0.0;
  if (a.what != 2) {
    f = a.ndim == 3 ? diffusion_fast<T, 3>(a, Wi + sp * npts, wsp, sp, inst, p, i, j, k)
                    : diffusion_fast<T, 2>(a, Wi + sp * npts, wsp, sp, inst, p, i, j, k);
  }
  if (a.what != 1 && a.reaction != 0) {
    double G0, G1, G2;
    reaction3(a, inst, w0, w1, w2, G0, G1, G2);
    f += sp == 0 ? G0 : (sp == 1 ? G1 : G2);
  }
  return f;
}

// F_sp at point p (what: 0 = operator + reaction, 1 = operator, 2 = reaction)
template <typename T>
__device__ __forceinline__ double stencil_point(const StencilArgs& a, int inst, int sp, int64_t p) {
  const int n1 = a.n[0], n2 = a.n[1];
  const int64_t npts = static_cast<int64_t>(n1) * n2 * a.n[2];
  const int i = static_cast<int>(p % n1);
  const int j = static_cast<int>((p / n1) % n2);
  const int k = static_cast<int>(p / (static_cast<int64_t>(n1) * n2));
  const int ns = a.nspecies;
  const T* Wi = static_cast<const T*>(a.W) + static_cast<int64_t>(inst) * ns * npts;
  double f = 0.0;
  if (a.what != 2) f = diffusion_dev<T>(a, Wi, inst, sp, p, i, j, k);
  if (a.what != 1 && a.reaction != 0) {
    double w[3] = {0, 0, 0}, G[3] = {0, 0, 0};
    for (int q = 0; q < ns && q < 3; ++q) w[q] = static_cast<double>(Wi[q * npts + p]);
    reaction_dev(a, inst, w, G);
    f += G[sp];
  }
  return f;
}

}  // namespace tg
