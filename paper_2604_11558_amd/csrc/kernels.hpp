// Device kernels of the split exponential Euler step and their launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tg {

// EPI_DPHI: C = acc * d/dd phi_1(x) with x = d c (= (x / d)(phi_1 - phi_2)(x));
// EPI_PHI_ACC: C += acc * phi_1(x).
enum Epilogue : int { EPI_STORE = 0, EPI_PHI = 1, EPI_UPDATE = 2, EPI_DPHI = 3, EPI_PHI_ACC = 4 };

// Steady-state indicators gathered in the update epilogue of a step's last
// launch.  Each workgroup sums, over the points it updates, w * W_new and
// w * (W_new - W_old)^2 with w = w1[i] * w23[j + n2 k] the quadrature weight
// of point (i, j, k), and stores the two sums in part[2 * (slab * tiles +
// tile) + {0, 1}] (no atomics: the sums are reproducible).  A finishing
// launch adds up each slab's partial sums in a fixed order and writes
// out[2 * slab] = wref[slab] + wsum_inv * sum(w W_new) (the integral mean of
// the full value) and out[2 * slab + 1] = sqrt(sum(w dW^2)).
struct DiagArgs {
  double* part;         // null: no indicators
  double* out;
  const double* w1;     // [n1]
  const double* w23;    // [n2 * n3]
  const double* wref;   // [nslab]
  double wsum_inv;
  int tiles;            // partial slots per slab (set by the launcher)
  int cap;              // slots per slab available in part
};

// Sum each slab's `tiles` partial pairs and write the indicators.
hipError_t launch_diag_finish(const DiagArgs& d, int nslab, hipStream_t s);

// The library's static device scratch (a file-scope array of
// kStaticScratchBytes, one copy per GPU, held until the process ends), for
// entry points that allocate nothing.  Returns the current device's address
// of the array, resolved once per device (with that device current) and
// cached.  Host code must use this address, never the array's name.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
hipError_t static_scratch(void** out);

// One mu-mode product over a batch of "slabs" (species x instances), as a
// GEMM C = A * B per (slab, batch b):
//   strided mode (mu >= 2):  A = factor L (M x K, row-major), B = X_b (K x N,
//                            row-major, N = product of faster modes), C = Y_b.
//   first mode  (mu == 1):   A = X (M x K row-major, M = slower points),
//                            B(k, n) = L[n][k] (factor stored N x K), C = Y.
// Epilogues: EPI_STORE C = acc; EPI_PHI C = acc * phi_1(cs[s] pm[m] pn[n] pb[b])
// (any of pm/pn/pb may be null = 1); EPI_UPDATE C += alpha * acc.
// Two fusions for the adjoint: with A2 and B2 set (same shapes, strides and
// slab moduli as A and B) the contraction runs over both pairs,
// acc = A B + A2 B2; with C2 set (B2 null) the same product is also written
// to C2 through epilogue epi2 (EPI_STORE or EPI_PHI; no indicators).
struct GemmArgs {
  const void* A;
  const void* B;
  void* C;
  const void* A2;
  const void* B2;
  void* C2;
  int epi2;
  int M, N, K;
  int nbatch;   // b range (strided mode); 1 otherwise
  int nslab;
  int64_t lda, ldb, ldc;
  int64_t a_bstride, b_bstride, c_bstride;  // per b
  int64_t a_sstride, b_sstride, c_sstride;  // per slab (times slab % *_smod)
  int a_smod, b_smod;                       // modulus of slab index for factors
  int b_kcontig;                            // B stored N x K (first-mode form)
  int64_t b_ncol, c_ncol;                   // column strides of B (not k-contiguous) and C; 0 means 1
  int epi;
  double alpha;
  const double* cs;                // per slab phi_1 argument multiplier (tau d_s)
  const double* pm;                // per row
  const double* pn;                // per column
  const double* pb;                // per batch b
  int tile;                        // 0: 64x64, 1: 32x64, 2: 64x32, 3: 32x32
  int* flag;                       // EPI_UPDATE: set to 1 if a non-finite value is written
  const double* rd;                // per slab 1 / d_s (EPI_DPHI)
  DiagArgs dg;                     // EPI_UPDATE of a first-mode product only
};

template <typename T>
hipError_t launch_mode_gemm(const GemmArgs& g, hipStream_t s);

// Bulk-surface exchange added to F by the stencil launch (two species on
// each side; both states in deviation form around their references):
//   bulk (ball) boundary layer i = n1 - 1, above surface point q = j + n2 k:
//     F_u += kappa z1 (z2 r - z3 u),   F_v += kappa z1 (e1 s - e2 v)
//   surface point q:   F_r -= z1 (z2 r - z3 u_b),   F_s -= z1 (e1 s - e2 v_b)
// with u_b, v_b the bulk values at (n_rho - 1, q).
// Reaction constants per instance (stride of StencilArgs::rparams).
constexpr int kRParams = 12;

// Bulk-surface exchange, added to F by the stencil launch.
//   kind 1 / 2: ball / its sphere (Section 5.5): Robin terms with kappa =
//     (2 / h)(1 + h / rho_*) and (z1, z2, z3, e1, e2) = (zeta1, zeta2,
//     zeta3, eta1, eta2); on1 = n_rho of the ball (sphere side).
//   kind 3 / 4: cylinder / its bottom disk (Section 5.6): on the cylinder's
//     z = 0 layer F_s -= kappa d_s zeta1 c_s (p, q)(u, v, r, s) with kappa =
//     2 / h_z, (c_u, c_v) = (z1, z2) = (alpha3, beta3) and zeta1, p, q from
//     the disk plan's DIB constants (orp); on the disk the DIB kinetics take
//     the cylinder's z = 0 values (u, v) instead of 1; on1 = n_z (disk side).
struct CoupleArgs {
  int kind;               // 0 none, 1 ball, 2 sphere, 3 cylinder, 4 bottom disk
  const void* other;      // partner state (same element type) [batch][2][...]
  const double* oref;     // partner reference [batch][2]
  int on1;                // n_rho of the ball (kind 2), n_z of the cylinder (kind 4)
  double kappa, z1, z2, z3, e1, e2;
  const double* orp;      // partner reaction constants [batch][kRParams] (kind 3)
};

// F = d_s * M W (+ G(W)) pointwise stencil over all modes, deviation form.
struct StencilArgs {
  const void* W;
  void* F;
  int ndim;
  int n[3];
  int nspecies;
  int batch;
  int what;                 // 0: operator + reaction, 1: operator only, 2: reaction only,
                            // 3: operator + reaction into F and the operator alone into F2
  const double* coef;       // [3 modes][3][nmax]: lo, dg, up of each mode's operator
  const double* scale;      // [3 modes][3 coords][nmax]: per-coordinate scale factors
  int nmax;
  int periodic_mask;        // bit mu-1 set: mode mu wraps around
  int scale_mask;           // bit 3 mu + c set: scale[mu][c] is not all ones
  const double* diff;       // [batch][nspecies]
  int reaction;             // 0 none, 1 Schnakenberg, 2 AIS3
  const double* rparams;    // [batch][4]
  const double* wref;       // [batch][nspecies] reference state (deviation origin)
  const double* g0;         // [batch][nspecies] reaction at the reference state
  CoupleArgs cp;            // bulk-surface exchange (separate stencil launch only)
  void* F2;                 // what == 3 only
};

template <typename T>
hipError_t launch_stencil(const StencilArgs& a, hipStream_t s);

// Adjoint combination per point, all species of an instance:
//   lam_s += tau * (mtmu_s + sum_r dG_r/dw_s (W) mu_r)
// with W = w_ref + state (the reaction Jacobian at step n).
// The same launch gathers, per block of 256 points and species s, the
// partial sums of lam_s tang_s (the old lam), mu_s dmw_s and mu_s into
// part[batch][blocks][3 * nspecies]; a second launch adds each slab's
// partials by a fixed tree over the blocks and accumulates
//   grad[s] += tau[s] <lam_s, tang_s> + taurd[s] <mu_s, dmw_s>,
//   grad[nslab + s] += tau[s] sum mu_s
// (no atomics: repeated sweeps give identical gradients).
struct AdjointArgs {
  const void* state;
  const void* mu;     // S^T lambda (unscaled)
  const void* mtmu;   // d_s M^T mu
  void* lam;
  const void* tang;   // (dS/dd) F of the step
  const void* dmw;    // d_s M W of the step
  double* part;       // [batch][blocks][3 * nspecies], blocks = ceil(npts / 256)
  double* grad;       // [2 * batch * nspecies], accumulated
  const double* tau_s;    // [nslab] tau
  const double* taurd_s;  // [nslab] tau / d_s
  int64_t npts;
  int nspecies, batch, reaction;
  double tau;
  const double* rparams;
  const double* wref;
};
template <typename T>
hipError_t launch_adjoint_combine(const AdjointArgs& a, hipStream_t s);

// dst[i] = (double) src[i], i < n (FP32 states kept in FP64).
hipError_t launch_widen(const float* src, double* dst, int64_t n, hipStream_t s);

}  // namespace tg
