// Fused mu-mode product kernels: the data tile of a workgroup (all of the
// contracted index for a block of the other indices) sits in LDS for the
// whole contraction; factors stream from L2 as 4-wide vectors along k.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace tg {

// Phi argument of an eigen-basis Hadamard factor:
// x = cs[slab] * pm[row] * pn[col] * pb[b]   (null arrays mean 1).
struct PhiArgs {
  const double* cs;
  const double* pm;
  const double* pn;
  const double* pb;
};

// A padded factor stack: block f of fmod blocks is at L + f * fstride, row-
// major with leading dimension ld; rows and columns beyond n are zero.
struct Factor {
  const void* L;
  int ld;
  int64_t fstride;
  int fmod;
};

// Strided mode (mu >= 2) product over the view [nb][nm][na] of every slab:
//   Y_b = L2 (Phi o (L1 X_b))   (sandwich)    or    Y_b = Phi? o (L1 X_b)
// A workgroup owns `tn` consecutive columns a of one (b, slab) and all nm
// rows.  With `stencil` set, X is not read: the tile is computed from the
// state as F = d M W + g(W) (the first product of a step).
// With `plane` set (na == tile width), the result is multiplied along mode 1
// by the factor `P` and added to the state: W += alpha * (Y x_1 P).
struct StridedArgs {
  const void* X;
  void* Y;
  int nm, na, nb, nslab;
  int tn;          // columns per workgroup (multiple of 16)
  int sandwich;
  int phi;         // apply the Phi factor after the first product
  Factor L1, L2;
  PhiArgs ph;
  int stencil;
  StencilArgs st;  // valid when stencil != 0 (W = state)
  int plane;
  Factor P;        // mode-1 factor for the plane tail
  void* W;         // state updated by the plane tail
  int update;      // plane tail: 1 = W += alpha * Z, 0 = W = Z
  double alpha;
  int* flag;
  DiagArgs dg;     // plane-tail updates only (row j + n2 k, column i)
};

// First mode product over rows r (all slower points) of every slab:
//   Y = (Phi o (X L1^T)) L2^T  (sandwich)   or   Y = X L1^T
// epilogue: store into Y, or W += alpha * result (update).
struct FirstArgs {
  const void* X;
  void* Y;
  int nm, rows, nslab;
  int tm;          // rows per workgroup (multiple of 16)
  int sandwich;
  Factor L1, L2;
  PhiArgs ph;      // x = cs[s] pm[row] pn[col]
  int update;
  double alpha;
  int* flag;
  DiagArgs dg;     // updates only (row = slower points j + n2 k, column i)
};

// Grouped persistent launch of up to kMaxGroup launches of one kind (the
// same chain op of plans on grids of different sizes).  Member q owns the
// logical tiles start[q] .. start[q+1]; its tile index decomposes as
// x + nbx[q] * (y + nby[q] * z).  span = 8 * per_xcd >= total.
constexpr int kMaxGroup = 4;
struct GroupMap {
  int n, total, span, per_xcd;
  int start[kMaxGroup + 1];
  int nbx[kMaxGroup], nby[kMaxGroup];
};
struct StridedGroup {
  GroupMap map;
  StridedArgs a[kMaxGroup];
};
struct FirstGroup {
  GroupMap map;
  FirstArgs a[kMaxGroup];
};
// One kernel variant, its LDS bytes and the persistent grid size.
struct GroupLaunch {
  int variant = -1;
  size_t lds = 0;
  int grid = 0;
};
// Host side: check the members a[0 .. map.n), fill the tile map and pick
// one kernel variant for all of them (the runtime-K one when their
// contraction lengths need different unrolled ones).  hipErrorInvalidValue
// when they cannot share a launch.  Queries the current device's occupancy.
template <typename T>
hipError_t plan_strided_group(StridedGroup& g, GroupLaunch& L);
template <typename T>
hipError_t plan_first_group(FirstGroup& g, GroupLaunch& L);
// `dev` holds a copy of the planned group in device memory.
template <typename T>
hipError_t launch_strided_group(const GroupLaunch& L, const StridedGroup* dev, hipStream_t s);
template <typename T>
hipError_t launch_first_group(const GroupLaunch& L, const FirstGroup* dev, hipStream_t s);

template <typename T>
hipError_t launch_strided(const StridedArgs& a, hipStream_t s);
template <typename T>
hipError_t launch_first(const FirstArgs& a, hipStream_t s);
// LDS bytes a launch would need (0 if the shape is not supported).
template <typename T>
size_t strided_lds_bytes(int nm, int tn, int sandwich, int plane, int stencil = 0);
template <typename T>
size_t first_lds_bytes(int nm, int tm, int sandwich);

// Several split steps of a plan whose step is one fused strided op with the
// stencil, the sandwich, its phi factor and the plane-tail update, on a 2D
// grid (the disk), in one launch: one workgroup per instance keeps every
// species' state in LDS for all `steps` steps.  a.W == a.st.W is the state
// (read, then updated in place); np, tn: resident_np / resident_tn.
struct ResidentArgs {
  StridedArgs a;
  int np, tn;
  int ninst;
  int steps;
};
template <typename T>
hipError_t launch_resident(const ResidentArgs& r, hipStream_t s);
int resident_np(int nm, int na);
int resident_tn(int nm, int na);
// LDS bytes of the resident launch (0 if the shape is not supported).
template <typename T>
size_t resident_lds_bytes(int ns, int nm, int na);

// Split-bf16 variants (FP32 state and accumulation; nterms = 2 or 3 bf16
// terms per operand).  Factors are NT-term bf16 stacks: term t of block f at
// (bf16*) L + f * fstride + t * ld * ld.  A plane launch needs a sandwich
// and tn == na rounded up to 32.
// Workgroups of `kernel` (with `threads` threads and `lds` bytes of dynamic
// LDS) that fit on the current device at once: the occupancy per CU times
// the CU count, queried once per kernel, shape and device (thread-safe);
// 0 when the query fails.  Multi-tile launches size their grids with it.
int resident_workgroups(const void* kernel, int threads, size_t lds);

hipError_t launch_strided_bf16(int nterms, const StridedArgs& a, hipStream_t s);
hipError_t launch_first_bf16(int nterms, const FirstArgs& a, hipStream_t s);
size_t strided_bf16_lds_bytes(int nterms, int nm, int na, int tn, int sandwich, int plane);
size_t first_bf16_lds_bytes(int nterms, int nm, int tm, int sandwich);

}  // namespace tg
