// Grid and plan objects behind the C interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <utility>
#include <string>
#include <vector>

#include "hostmath.hpp"
#include "fused.hpp"
#include "kernels.hpp"

struct tg_grid_s {
  int geometry = 0;
  int ndim = 0;
  int n[3] = {1, 1, 1};
  double extent[2] = {1.0, 1.0};
  double lam = 0.0;  // lambda of the anomalous disk (TG_DISK_LAMBDA)
  tg::Coord coord[3] = {tg::RHO2, tg::THETA, tg::PHI};
  double extent_of(int mode) const;          // 0-based mode
  tg::Tridiag op(int mode) const;            // 0-based mode, unscaled
  std::vector<double> coords(int mode) const;
  tg::Eig eig(int mode) const;
};

namespace tg {

// One mu-mode product of the split chain, resolved to device pointers.
struct ChainOp {
  int mode = 1;            // 1-based mode index mu
  const void* L = nullptr; // factor(s): fmod blocks of n_mu x n_mu, row-major (T)
  int fmod = 1;            // slab s uses factor block s % fmod
  int epi = EPI_STORE;     // EPI_UPDATE is replaced by EPI_STORE for the test hook
  const double* pm = nullptr;
  const double* pn = nullptr;
  const double* pb = nullptr;
  int tile = 0;
  double flops = 0.0;
  const void* LT = nullptr;  // transposed factor blocks (adjoint)
  const void* dL = nullptr;  // d/dd of the factor blocks, or null if L does not depend on d
  // per-slice product (slice != 0): one dense factor per (factor block, slice
  // i = mode-1 index), [fmod][n1][n_mu][n_mu]; the product runs over the
  // other columns (ncol of them, stride sn) with rows of stride sk
  int slice = 0;
  int64_t sk = 0, sn = 0;
  int ncol = 0;
};

// One fused launch of the step (see fused.hpp).  in / out name the
// buffers: -1 = the state, 0 / 1 = plan scratch buffers.
struct FusedOp {
  int kind = 0;            // 0 strided (mode >= 2), 1 first mode
  int mode = 1;
  StridedArgs sa{};
  FirstArgs fa{};
  int in = -1, out = -1;
  bool updates_state = false;
  double flops = 0.0;      // algorithmic flops of one launch (2 n_mu per output of each product)
};

}  // namespace tg

struct tg_group_s;  // grouped runs of several plans (api.cpp)

struct tg_plan_s {
  tg_grid_s grid;
  int ns = 0, batch = 0, nslab = 0;
  int reaction = 0, precision = 0;
  double tau = 0.0;
  int64_t npts = 0, state_elems = 0;
  int esize = 8;
  std::vector<double> diff, rparams, wref, g0;
  // device memory
  char* dmem = nullptr;      // all small arrays and factors
  void* scratch[2] = {nullptr, nullptr};
  int* dflag = nullptr;
  // device pointers into dmem
  const double* d_coef = nullptr;
  const double* d_scale = nullptr;
  const double* d_diff = nullptr;
  const double* d_rparams = nullptr;
  const double* d_wref = nullptr;
  const double* d_g0 = nullptr;
  const double* d_cs = nullptr;
  const double* d_coefT = nullptr;   // transposed 1D operators (adjoint stencil)
  const double* d_rd = nullptr;      // 1 / d per slab
  const double* d_tau = nullptr;     // tau per slab
  const double* d_taurd = nullptr;   // tau / d per slab
  void* adj_ws = nullptr;            // adjoint workspace: 8 state-sized buffers
  // steady-state indicators: quadrature weights w1 [n1], w23 [n2 n3] (the
  // sphere's rho_*^2 folded into w1), 1 / sum of all weights, and the
  // per-tile partial sums (allocated on first use, diag_cap slots per slab)
  const double* d_w1 = nullptr;
  const double* d_w23 = nullptr;
  double wsum_inv = 0.0;
  double* diag_part = nullptr;
  int diag_cap = 0;
  int nmax = 0;
  int periodic_mask = 0;
  int scale_mask = 0;
  std::vector<tg::ChainOp> chain;   // generic route: one launch per mode product
  std::vector<tg::ChainOp> slice_chain;  // per-slice route (ball, cylinder), built on first use
  void* slice_mem = nullptr;             // its per-slice factors
  std::vector<tg::FusedOp> fused;   // fused route
  bool fused_ok = false;
  int route = 0;                     // 0 fused (when available), 1 generic
  // captured step graphs keyed by (state pointer, steps per graph)
  std::map<std::pair<void*, int>, hipGraphExec_t> graphs;
  hipStream_t capture_stream = nullptr;
  // unique id, and a counter bumped whenever the launch configuration
  // (route, tiles) changes; grouped runs are keyed on both
  uint64_t serial = 0;
  uint64_t version = 0;
  // grouped runs led by this plan, keyed by (serial, version, state) of members
  std::map<std::vector<uint64_t>, tg_group_s*> groups;
  // captured bulk-surface steps led by this (bulk) plan, keyed by the
  // partner's (serial, version), both states and the coupling constants
  std::map<std::vector<uint64_t>, hipGraphExec_t> coupled_graphs;
};
