// Fused mu-mode product kernels (see fused.hpp).
//
// Both kernels run 256 threads = 4 waves.  The workgroup's data tile holds
// the whole contracted index in LDS; each wave computes 16FM x 16FN output
// sub-tiles with 16x16x4 MFMAs.  Factor operands are read from global
// memory (L2 resident: a few hundred KB at most) four consecutive k at a
// time; to make that a single vector load the k index of MFMA step t in
// lane group g is k0 + 4 g + t instead of k0 + 4 t + g (any assignment of
// k to (step, group) is valid as long as both operands use the same one).
#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

#include "fused.hpp"
#include "diag_dev.hpp"
#include "phi_dev.hpp"
#include "stencil_dev.hpp"

namespace tg {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct M16;
template <> struct M16<double> {
  using acc = f64x4;
  using v4 = f64x4;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element r of lane group g is row g + 4 r (FP64 layout)
  static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
  static __device__ __forceinline__ double phi1(double x) { return x == 0.0 ? 1.0 : expm1(x) / x; }
};
template <> struct M16<float> {
  using acc = f32x4;
  using v4 = f32x4;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element r of lane group g is row 4 g + r (FP32 layout)
  static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
  static __device__ __forceinline__ float phi1(float x) { return phi1_f32(x); }
};

static inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// q = x / d, r = x % d for 0 <= x < 2^24 and 0 < d < 2^12 (the quotient
// estimate from the float reciprocal is off by at most one, then fixed):
// integer division by a runtime divisor costs dozens of instructions.
struct Div {
  int d;
  float inv;
  __device__ __forceinline__ explicit Div(int dd) : d(dd), inv(1.0f / static_cast<float>(dd)) {}
  __device__ __forceinline__ int quot(int x, int& r) const {
    int q = static_cast<int>(static_cast<float>(x) * inv);
    r = x - q * d;
    if (r < 0) { --q; r += d; }
    if (r >= d) { ++q; r -= d; }
    return q;
  }
};

// LDS row pitch (elements).  With w a multiple of 16, w + 4 puts the rows
// read by lane groups 0 and 1 of a 16-wide access in different halves of
// the 32 banks (FP32), and gives the 16-byte (FP32) / 32-byte (FP64) row
// vectors read by 8 / 4 consecutive lanes distinct banks.
template <typename T>
__host__ __device__ inline int pitch_kmajor(int w) { return w + 4; }
template <typename T>
__host__ __device__ inline int pitch_rowvec(int w) { return w + 4; }

// acc[f][j] += sum_{k < K} A[r0 + 16 f + li][k] * sB[k][c0 + 16 j + li]
// A: zero-padded factor rows in global memory; sB: k-major LDS tile.
template <typename T, int FM, int FN>
__device__ __forceinline__ void gemm_gA_sB(typename M16<T>::acc (&acc)[FM][FN], const T* __restrict__ A,
                                           int lda, int r0, const T* sB, int ldb, int c0, int K, int lane) {
  using v4 = typename M16<T>::v4;
  const int li = lane & 15, g = lane >> 4;
  const T* arow[FM];
#pragma unroll
  for (int f = 0; f < FM; ++f) arow[f] = A + static_cast<int64_t>(r0 + 16 * f + li) * lda + 4 * g;
  // factor vectors are fetched two k-chunks ahead of their use
  v4 cur[FM], nx1[FM];
#pragma unroll
  for (int f = 0; f < FM; ++f) {
    cur[f] = *reinterpret_cast<const v4*>(arow[f]);
    if (K > 16) nx1[f] = *reinterpret_cast<const v4*>(arow[f] + 16);
  }
  for (int k0 = 0; k0 < K; k0 += 16) {
    v4 nx2[FM];
    const bool more = k0 + 32 < K;
#pragma unroll
    for (int f = 0; f < FM; ++f)
      if (more) nx2[f] = *reinterpret_cast<const v4*>(arow[f] + k0 + 32);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T* brow = sB + (k0 + 4 * g + t) * ldb + c0 + li;
      T b[FN];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = brow[16 * j];
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[f][j] = M16<T>::mac(cur[f][t], b[j], acc[f][j]);
    }
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      cur[f] = nx1[f];
      if (more) nx1[f] = nx2[f];
    }
  }
}

// acc[f][j] += sum_{k < K} sA[r0 + 16 f + li][k] * B[c0 + 16 j + li][k]
// sA: row-major LDS tile; B: zero-padded factor rows (= output columns).
template <typename T, int FM, int FN>
__device__ __forceinline__ void gemm_sA_gB(typename M16<T>::acc (&acc)[FM][FN], const T* sA, int lda,
                                           int r0, const T* __restrict__ B, int ldb, int c0, int K,
                                           int lane) {
  using v4 = typename M16<T>::v4;
  const int li = lane & 15, g = lane >> 4;
  const T* brow[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) brow[j] = B + static_cast<int64_t>(c0 + 16 * j + li) * ldb + 4 * g;
  v4 cur[FN], nx1[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    cur[j] = *reinterpret_cast<const v4*>(brow[j]);
    if (K > 16) nx1[j] = *reinterpret_cast<const v4*>(brow[j] + 16);
  }
  for (int k0 = 0; k0 < K; k0 += 16) {
    v4 nx2[FN];
    const bool more = k0 + 32 < K;
#pragma unroll
    for (int j = 0; j < FN; ++j)
      if (more) nx2[j] = *reinterpret_cast<const v4*>(brow[j] + k0 + 32);
    v4 a[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f)
      a[f] = *reinterpret_cast<const v4*>(sA + (r0 + 16 * f + li) * lda + k0 + 4 * g);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[f][j] = M16<T>::mac(a[f][t], cur[j][t], acc[f][j]);
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      cur[j] = nx1[j];
      if (more) nx1[j] = nx2[j];
    }
  }
}

// Fully unrolled variants for K = 16 KCH: every factor vector of the wave's
// rows is requested before the first MFMA, so the loads overlap each other
// and a single wait covers them (the runtime-K loops above are used for
// larger contractions).
template <typename T, int FM, int FN, int KCH>
__device__ __forceinline__ void gemm_gA_sB_u(typename M16<T>::acc (&acc)[FM][FN], const T* __restrict__ A,
                                             int lda, int r0, const T* sB, int ldb, int c0, int lane) {
  using v4 = typename M16<T>::v4;
  const int li = lane & 15, g = lane >> 4;
  v4 av[FM][KCH];
#pragma unroll
  for (int f = 0; f < FM; ++f) {
    const T* arow = A + static_cast<int64_t>(r0 + 16 * f + li) * lda + 4 * g;
#pragma unroll
    for (int c = 0; c < KCH; ++c) av[f][c] = *reinterpret_cast<const v4*>(arow + 16 * c);
  }
#pragma unroll
  for (int c = 0; c < KCH; ++c)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T* brow = sB + (16 * c + 4 * g + t) * ldb + c0 + li;
      T b[FN];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = brow[16 * j];
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[f][j] = M16<T>::mac(av[f][c][t], b[j], acc[f][j]);
    }
}

template <typename T, int FM, int FN, int KCH>
__device__ __forceinline__ void gemm_sA_gB_u(typename M16<T>::acc (&acc)[FM][FN], const T* sA, int lda,
                                             int r0, const T* __restrict__ B, int ldb, int c0, int lane) {
  using v4 = typename M16<T>::v4;
  const int li = lane & 15, g = lane >> 4;
  v4 bv[FN][KCH];
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const T* brow = B + static_cast<int64_t>(c0 + 16 * j + li) * ldb + 4 * g;
#pragma unroll
    for (int c = 0; c < KCH; ++c) bv[j][c] = *reinterpret_cast<const v4*>(brow + 16 * c);
  }
#pragma unroll
  for (int c = 0; c < KCH; ++c) {
    v4 a[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f)
      a[f] = *reinterpret_cast<const v4*>(sA + (r0 + 16 * f + li) * lda + 16 * c + 4 * g);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[f][j] = M16<T>::mac(a[f][t], bv[j][c][t], acc[f][j]);
  }
}

// Split forms of the unrolled products: the factor vectors of a wave's rows
// (columns) are loaded by one call and consumed by another, so that the
// loads of the next product can be issued while the current one runs.
template <typename T, int FM, int KCH>
__device__ __forceinline__ void load_rows_u(typename M16<T>::v4 (&av)[FM][KCH], const T* __restrict__ A, int lda,
                                            int r0, int lane) {
  using v4 = typename M16<T>::v4;
  const int li = lane & 15, g = lane >> 4;
#pragma unroll
  for (int f = 0; f < FM; ++f) {
    const T* arow = A + static_cast<int64_t>(r0 + 16 * f + li) * lda + 4 * g;
#pragma unroll
    for (int c = 0; c < KCH; ++c) av[f][c] = *reinterpret_cast<const v4*>(arow + 16 * c);
  }
}

template <typename T, int FM, int FN, int KCH>
__device__ __forceinline__ void mma_rows_sB(typename M16<T>::acc (&acc)[FM][FN],
                                            const typename M16<T>::v4 (&av)[FM][KCH], const T* sB, int ldb, int c0,
                                            int lane) {
  const int li = lane & 15, g = lane >> 4;
#pragma unroll
  for (int c = 0; c < KCH; ++c)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T* brow = sB + (16 * c + 4 * g + t) * ldb + c0 + li;
      T b[FN];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = brow[16 * j];
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[f][j] = M16<T>::mac(av[f][c][t], b[j], acc[f][j]);
    }
}

template <typename T, int FN, int KCH>
__device__ __forceinline__ void load_cols_u(typename M16<T>::v4 (&bv)[FN][KCH], const T* __restrict__ B, int ldb,
                                            int c0, int lane) {
  using v4 = typename M16<T>::v4;
  const int li = lane & 15, g = lane >> 4;
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const T* brow = B + static_cast<int64_t>(c0 + 16 * j + li) * ldb + 4 * g;
#pragma unroll
    for (int c = 0; c < KCH; ++c) bv[j][c] = *reinterpret_cast<const v4*>(brow + 16 * c);
  }
}

template <typename T, int FM, int FN, int KCH>
__device__ __forceinline__ void mma_sA_cols(typename M16<T>::acc (&acc)[FM][FN], const T* sA, int lda, int r0,
                                            const typename M16<T>::v4 (&bv)[FN][KCH], int lane) {
  using v4 = typename M16<T>::v4;
  const int li = lane & 15, g = lane >> 4;
#pragma unroll
  for (int c = 0; c < KCH; ++c) {
    v4 a[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f)
      a[f] = *reinterpret_cast<const v4*>(sA + (r0 + 16 * f + li) * lda + 16 * c + 4 * g);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[f][j] = M16<T>::mac(a[f][t], bv[j][c][t], acc[f][j]);
  }
}

// Dispatch on the compile-time chunk count (KCH == 0: runtime K).
template <typename T, int FM, int FN, int KCH>
__device__ __forceinline__ void mm_gA_sB(typename M16<T>::acc (&acc)[FM][FN], const T* A, int lda, int r0,
                                         const T* sB, int ldb, int c0, int K, int lane) {
  if constexpr (KCH > 0) gemm_gA_sB_u<T, FM, FN, KCH>(acc, A, lda, r0, sB, ldb, c0, lane);
  else gemm_gA_sB<T, FM, FN>(acc, A, lda, r0, sB, ldb, c0, K, lane);
}
template <typename T, int FM, int FN, int KCH>
__device__ __forceinline__ void mm_sA_gB(typename M16<T>::acc (&acc)[FM][FN], const T* sA, int lda, int r0,
                                         const T* B, int ldb, int c0, int K, int lane) {
  if constexpr (KCH > 0) {
    if (K == 16 * KCH) {
      gemm_sA_gB_u<T, FM, FN, KCH>(acc, sA, lda, r0, B, ldb, c0, lane);
      return;
    }
  }
  gemm_sA_gB<T, FM, FN>(acc, sA, lda, r0, B, ldb, c0, K, lane);
}

template <typename T, int FM, int FN>
__device__ __forceinline__ void zero(typename M16<T>::acc (&acc)[FM][FN]) {
#pragma unroll
  for (int f = 0; f < FM; ++f)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[f][j] = typename M16<T>::acc{0, 0, 0, 0};
}

__device__ __forceinline__ double phi_arg(const PhiArgs& p, int s, int row, int col, int b) {
  double x = p.cs[s];
  if (p.pm) x *= p.pm[row];
  if (p.pn) x *= p.pn[col];
  if (p.pb) x *= p.pb[b];
  return x;
}

template <typename T>
__device__ __forceinline__ const T* factor_of(const Factor& F, int s) {
  return static_cast<const T*>(F.L) + static_cast<int64_t>(s % F.fmod) * F.fstride;
}

// Tile loads.  Rows of the source are contiguous; when the row length is a
// multiple of 4 every thread moves 4-element vectors, eight of them in
// flight before the LDS stores.
constexpr int kBatch = 8;

// sX[k][c] = X[k * na + a0 + c] for k < nm, a0 + c < na, else 0 (k < NP, c < TN);
// NT threads
template <typename T, int NT>
__device__ __forceinline__ void load_tile_kmajor(const T* __restrict__ X, int na, int nm, int a0, int NP,
                                                 int TN, T* sX, int ld, int tid) {
  using v4 = typename M16<T>::v4;
  const Div dtn(TN);
  if (na % 4 == 0) {
    const int nvec = NP * TN / 4;
    if (nvec <= 2 * NT) {  // the usual small tile: at most two vectors per thread
      v4 r[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int v = tid + NT * q;
        int c;
        const int k = dtn.quot(4 * v, c);
        r[q] = v4{0, 0, 0, 0};
        if (v < nvec && k < nm && a0 + c < na)
          r[q] = *reinterpret_cast<const v4*>(X + static_cast<int64_t>(k) * na + a0 + c);
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int v = tid + NT * q;
        if (v < nvec) {
          int c;
          const int k = dtn.quot(4 * v, c);
          *reinterpret_cast<v4*>(sX + k * ld + c) = r[q];
        }
      }
      return;
    }
    for (int v0 = 0; v0 < nvec; v0 += NT * kBatch) {
      v4 r[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int v = v0 + tid + NT * q;
        int c;
        const int k = dtn.quot(4 * v, c);
        r[q] = v4{0, 0, 0, 0};
        if (v < nvec && k < nm && a0 + c < na)
          r[q] = *reinterpret_cast<const v4*>(X + static_cast<int64_t>(k) * na + a0 + c);
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int v = v0 + tid + NT * q;
        if (v < nvec) {
          int c;
          const int k = dtn.quot(4 * v, c);
          *reinterpret_cast<v4*>(sX + k * ld + c) = r[q];
        }
      }
    }
    return;
  }
  for (int e = tid; e < NP * TN; e += NT) {
    int c;
    const int k = dtn.quot(e, c);
    sX[k * ld + c] = (k < nm && a0 + c < na) ? X[static_cast<int64_t>(k) * na + a0 + c] : T(0);
  }
}

// sX[r][c] = X[(rt0 + r) * nm + c] for rt0 + r < rows, c < nm, else 0 (r < TM, c < NP)
template <typename T, int NT>
__device__ __forceinline__ void load_tile_rows(const T* __restrict__ X, int nm, int rows, int rt0, int TM,
                                               int NP, T* sX, int ld, int tid) {
  using v4 = typename M16<T>::v4;
  const Div dnp(NP);
  if (nm % 4 == 0) {
    const int nvec = TM * NP / 4;
    if (nvec <= 2 * NT) {  // the usual small tile: at most two vectors per thread
      v4 r[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int v = tid + NT * q;
        int c;
        const int rr = dnp.quot(4 * v, c);
        r[q] = v4{0, 0, 0, 0};
        if (v < nvec && c < nm && rt0 + rr < rows)
          r[q] = *reinterpret_cast<const v4*>(X + static_cast<int64_t>(rt0 + rr) * nm + c);
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int v = tid + NT * q;
        if (v < nvec) {
          int c;
          const int rr = dnp.quot(4 * v, c);
          *reinterpret_cast<v4*>(sX + rr * ld + c) = r[q];
        }
      }
      return;
    }
    for (int v0 = 0; v0 < nvec; v0 += NT * kBatch) {
      v4 r[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int v = v0 + tid + NT * q;
        int c;
        const int rr = dnp.quot(4 * v, c);
        r[q] = v4{0, 0, 0, 0};
        if (v < nvec && c < nm && rt0 + rr < rows)
          r[q] = *reinterpret_cast<const v4*>(X + static_cast<int64_t>(rt0 + rr) * nm + c);
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int v = v0 + tid + NT * q;
        if (v < nvec) {
          int c;
          const int rr = dnp.quot(4 * v, c);
          *reinterpret_cast<v4*>(sX + rr * ld + c) = r[q];
        }
      }
    }
    return;
  }
  for (int e = tid; e < TM * NP; e += NT) {
    int c;
    const int r = dnp.quot(e, c);
    sX[r * ld + c] = (c < nm && rt0 + r < rows) ? X[static_cast<int64_t>(rt0 + r) * nm + c] : T(0);
  }
}

// ---------------------------------------------------------------------------
// Epilogue helpers.  Every lane owns FM x FN x 4 accumulator elements: rows
// r0 + 16 f + row(g, r), columns c0 + 16 j + li.  Loads that feed an
// epilogue (phi_1 argument factors, the state of an update) are issued with
// clamped indices before the product, so they overlap it and each other;
// only the final store is predicated.
template <typename T, int FM>
__device__ __forceinline__ void row_factors(double (&fr)[FM][4], const double* pm, int r0, int g, int lim,
                                            int off) {
#pragma unroll
  for (int f = 0; f < FM; ++f)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + 16 * f + M16<T>::row(g, r);
      fr[f][r] = pm ? pm[off + min(row, lim - 1)] : 1.0;
    }
}

template <int FN>
__device__ __forceinline__ void col_factors(double (&fc)[FN], const double* pn, int c0, int li, int lim, int off) {
#pragma unroll
  for (int j = 0; j < FN; ++j) fc[j] = pn ? pn[off + min(c0 + 16 * j + li, lim - 1)] : 1.0;
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// F = d_sp M W + g(W) for a stencil tile, staged through LDS.
//
// The tile's rows k are the slowest grid coordinate (mode 3 in 3D, mode 2
// in 2D; all nm of them are in the tile), its columns the faster ones
// (a = i + n1 j in 3D, a = i in 2D).  The centre values of species sp are
// loaded as a plain tile into `stage` (row neighbours come from there);
// the other species and the column neighbours of each element are loaded
// into registers, several elements per thread and pass, all requests
// issued before any is used.  The operator is evaluated as
//   d ( sum_m rs_m(k) (A_m w(a-) + B_m w + C_m w(a+)) + cs_r(c) (L(k) w(k-1) + D(k) w + U(k) w(k+1)) )
// over the column modes m, with the column factors A_m = cs_m lo_m, ...
// (cs_m the column part of mode m's scale) and the row factors L = rs_r lo_r,
// ... (rs the row parts), all in FP64: next to the axis and the poles the
// terms exceed F by orders of magnitude, and FP32 arithmetic there costs
// about an order of magnitude of the FP32 path's accuracy.
template <int NT>
constexpr int stencil_batch() { return NT >= 512 ? 4 : 8; }

__host__ __device__ inline int stencil_coef_doubles(int NP, int TN) { return NP * 5 + TN * 7; }

// DIM (2 or 3) and NSP (species) fix the grid's mode and species counts at
// compile time; 0 reads them from the arguments.
template <typename T, int NT, int DIM = 0, int NSP = 0>
__device__ __forceinline__ void stencil_tile(const StencilArgs& st, int inst, int sp, int a0, int NP, int TN, int nm,
                                             int na, T* sX, T* stage, int ld, double* cfd, int tid) {
  const int ns = NSP ? NSP : st.nspecies;
  const int ndim = DIM ? DIM : st.ndim;
  const bool three = ndim == 3;
  const int n1 = st.n[0], n2 = st.n[1];
  const int nmx = st.nmax;
  const int64_t plane = static_cast<int64_t>(nm) * na;
  const T* Wi = static_cast<const T*>(st.W) + static_cast<int64_t>(inst) * ns * plane;
  const T* Ws = Wi + sp * plane;
  const int rmode = three ? 2 : 1;          // mode whose coordinate is the row
  const int rslot = three ? 2 : 1;          // scale slot of the row coordinate
  const Div dtn(TN), dn1(n1);
  const bool per0 = st.periodic_mask & 1;
  const bool per1 = (st.periodic_mask >> 1) & 1;
  const bool perr = (st.periodic_mask >> rmode) & 1;
  const int total = NP * TN;
  constexpr int kB = stencil_batch<NT>();
  // uniform constants first: their loads overlap everything below
  const double d = st.diff[inst * ns + sp];
  const ReactConst rcst = react_const(st, inst);
  const bool react = st.what != 1 && st.reaction != 0;
  const bool diffuse = st.what != 2;
  // LDS: rows [NP][5] = rs_0, rs_1, L, D, U;  cols [TN][7] = A_0, B_0, C_0, A_1, B_1, C_1, cs_r
  double* rc = cfd;
  double* cc = rc + NP * 5;
  // column geometry of an element: its neighbours' offsets a-, a+ (mode 1)
  // and a-, a+ along mode 2 (3D)
  struct Col {
    int aa, im, ip, jm, jp;
  };
  auto col_of = [&](int c) {
    Col q;
    q.aa = a0 + c;
    const int aa = min(q.aa, na - 1);
    int i = aa, j = 0;
    if (three) j = dn1.quot(aa, i);
    q.im = i > 0 ? aa - 1 : (per0 ? aa + n1 - 1 : aa);
    q.ip = i + 1 < n1 ? aa + 1 : (per0 ? aa - (n1 - 1) : aa);
    q.jm = !three ? aa : (j > 0 ? aa - n1 : (per1 ? aa + (n2 - 1) * n1 : aa));
    q.jp = !three ? aa : (j + 1 < n2 ? aa + n1 : (per1 ? aa - (n2 - 1) * n1 : aa));
    return q;
  };
  // a thread keeps one column when NT is a multiple of TN
  const bool colfix = NT % TN == 0;
  int c_fix;
  const int k_fix = dtn.quot(tid, c_fix);
  const int kstep = NT / TN;  // rows between a thread's elements when colfix
  const Col cf0 = col_of(c_fix);

  T oth[kB][2], c0m[kB], c0p[kB], c1m[kB], c1p[kB];
  auto elem = [&](int e, int& k, int& c) {
    if (colfix) {
      c = c_fix;
      k = k_fix + (e - tid) / NT * kstep;  // e = e0 + tid + NT q, e0 a multiple of NT
    } else {
      k = dtn.quot(e, c);
    }
  };
  // species read by the reaction besides sp (index clamped for fewer species)
  const int o0s = ns > 1 ? (sp == 0 ? 1 : 0) : 0;
  const int o1s = ns > 2 ? (sp == 2 ? 1 : 2) : 0;
  // Every address below is clamped into the slab (row min(k, nm - 1), the
  // column's clamped neighbours), so the loads carry no conditions and the
  // compiler issues them back to back.
  auto request = [&](int e0) {
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int e = e0 + tid + NT * q;
      int k, c;
      elem(e, k, c);
      const Col g = colfix ? cf0 : col_of(c);
      const int64_t p = static_cast<int64_t>(min(k, nm - 1)) * na;
      const int ac = min(g.aa, na - 1);
      // (the compute phase reads these only for elements inside the tile,
      // and each only where its term exists; with the mode and species
      // counts fixed, the loads of absent terms are left out)
      c0m[q] = Ws[p + g.im];
      c0p[q] = Ws[p + g.ip];
      if (DIM == 0 || DIM == 3) {
        c1m[q] = Ws[p + g.jm];
        c1p[q] = Ws[p + g.jp];
      } else {
        c1m[q] = c1p[q] = T(0);
      }
      oth[q][0] = Wi[o0s * plane + p + ac];
      oth[q][1] = NSP == 0 || NSP > 2 ? Wi[o1s * plane + p + ac] : T(0);
    }
  };
  // Operator coefficients: the row (k = tid) and column (c = tid) entries
  // are requested first (every index is below nmax and the tables hold
  // 3 x 3 x nmax entries), so one round trip serves all.
  // (only the threads that own a row or a column load; whole waves past
  // them skip the loads)
  const double* rcoef = st.coef + rmode * 3 * nmx;
  double rsv[3] = {1.0, 1.0, 1.0}, rcv[3] = {0.0, 0.0, 0.0};
  if (tid < NP) {
    const int kkr = min(tid, nm - 1);
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) rsv[mu] = st.scale[mu * 3 * nmx + rslot * nmx + kkr];
#pragma unroll
    for (int x = 0; x < 3; ++x) rcv[x] = rcoef[x * nmx + kkr];
  }
  double csv[3][2] = {{1.0, 1.0}, {1.0, 1.0}, {1.0, 1.0}}, ccv[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  if (tid < TN) {
    const int acq = min(a0 + tid, na - 1);
    int ci = acq, cj = 0;
    if (three) cj = dn1.quot(acq, ci);
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      csv[mu][0] = st.scale[mu * 3 * nmx + ci];
      csv[mu][1] = st.scale[mu * 3 * nmx + nmx + cj];
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int x = 0; x < 3; ++x) ccv[m][x] = st.coef[m * 3 * nmx + x * nmx + (m == 0 ? ci : cj)];
  }
  request(0);
  // row table: rs_0, rs_1, L, D, U = rs_r * (lo, dg, up) of the row mode
  auto put_row = [&](int k, const double (&rs_)[3], const double (&c_)[3]) {
    double rs[3];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const bool on = mu < ndim && ((st.scale_mask >> (3 * mu + rslot)) & 1);
      rs[mu] = on ? rs_[mu] : 1.0;
    }
    const double rr = three ? rs[2] : rs[1];
    rc[k * 5 + 0] = rs[0];
    rc[k * 5 + 1] = three ? rs[1] : 0.0;
    rc[k * 5 + 2] = rr * c_[0];
    rc[k * 5 + 3] = rr * c_[1];
    rc[k * 5 + 4] = rr * c_[2];
  };
  if (tid < NP) put_row(tid, rsv, rcv);
  for (int k = tid + NT; k < NP; k += NT) {  // only when NP > NT
    const int kk = min(k, nm - 1);
    double a_[3], b_[3];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) a_[mu] = st.scale[mu * 3 * nmx + rslot * nmx + kk];
#pragma unroll
    for (int x = 0; x < 3; ++x) b_[x] = rcoef[x * nmx + kk];
    put_row(k, a_, b_);
  }
  // column table: A_m, B_m, C_m = cs_m * (lo, dg, up) of column mode m, and
  // cs_r (the row mode's column scale)
  auto put_col = [&](int c, const double (&cs_)[3][2], const double (&q_)[2][3]) {
    double cs[3];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      double f = 1.0;
      if (mu < ndim) {
        const int sm = st.scale_mask >> (3 * mu);
        if (sm & 1) f *= cs_[mu][0];
        if (three && (sm & 2)) f *= cs_[mu][1];
      }
      cs[mu] = f;
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const bool col_mode = m == 0 || three;
      cc[c * 7 + 3 * m + 0] = col_mode ? cs[m] * q_[m][0] : 0.0;
      cc[c * 7 + 3 * m + 1] = col_mode ? cs[m] * q_[m][1] : 0.0;
      cc[c * 7 + 3 * m + 2] = col_mode ? cs[m] * q_[m][2] : 0.0;
    }
    cc[c * 7 + 6] = three ? cs[2] : cs[1];
  };
  if (tid < TN) put_col(tid, csv, ccv);
  for (int c = tid + NT; c < TN; c += NT) {  // only when TN > NT
    const int aa = min(a0 + c, na - 1);
    int i = aa, j = 0;
    if (three) j = dn1.quot(aa, i);
    double a_[3][2], b_[2][3];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      a_[mu][0] = st.scale[mu * 3 * nmx + i];
      a_[mu][1] = st.scale[mu * 3 * nmx + nmx + j];
    }
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int x = 0; x < 3; ++x) b_[m][x] = st.coef[m * 3 * nmx + x * nmx + (m == 0 ? i : j)];
    put_col(c, a_, b_);
  }
  load_tile_kmajor<T, NT>(Ws, na, nm, a0, NP, TN, stage, ld, tid);
  __syncthreads();  // staged centres and coefficients
  double cr[7];
  if (colfix) {
#pragma unroll
    for (int x = 0; x < 7; ++x) cr[x] = cc[c_fix * 7 + x];
  }
  for (int e0 = 0; e0 < total; e0 += NT * kB) {
    if (e0 > 0) request(e0);
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int e = e0 + tid + NT * q;
      if (e >= total) break;
      int k, c;
      elem(e, k, c);
      double v = 0.0;
      if (k < nm && a0 + c < na) {
        const double w0 = static_cast<double>(stage[k * ld + c]);
        double f = 0.0;
        if (diffuse) {
          double c7[7];
#pragma unroll
          for (int x = 0; x < 7; ++x) c7[x] = colfix ? cr[x] : cc[c * 7 + x];
          const double* r5 = rc + k * 5;
          const int km = k > 0 ? k - 1 : (perr ? nm - 1 : k);
          const int kp = k + 1 < nm ? k + 1 : (perr ? 0 : k);
          const double wkm = static_cast<double>(stage[km * ld + c]);
          const double wkp = static_cast<double>(stage[kp * ld + c]);
          f = c7[6] * (r5[2] * wkm + r5[3] * w0 + r5[4] * wkp);
          f += r5[0] * (c7[0] * static_cast<double>(c0m[q]) + c7[1] * w0 + c7[2] * static_cast<double>(c0p[q]));
          if (three)
            f += r5[1] * (c7[3] * static_cast<double>(c1m[q]) + c7[4] * w0 + c7[5] * static_cast<double>(c1p[q]));
          f *= d;
        }
        if (react) {
          const double dw0 = w0;
          const double o0 = static_cast<double>(oth[q][0]), o1 = static_cast<double>(oth[q][1]);
          const double u = sp == 0 ? dw0 : o0;
          const double vv = sp == 1 ? dw0 : (sp == 0 ? o0 : o1);
          const double w = sp == 2 ? dw0 : o1;
          double G0, G1, G2;
          reaction3c(rcst, u, vv, w, G0, G1, G2);
          f += sp == 0 ? G0 : (sp == 1 ? G1 : G2);
        }
        v = f;
      }
      sX[k * ld + c] = static_cast<T>(v);
    }
  }
}

// One tile of a strided launch: columns bx * tn .., view row block by, slab bz.
//
// Latency plan (unrolled products, KCH > 0): the factor rows of a wave's
// first sub-tile for the first product, its phi_1 argument factors and,
// for an update, its state values are requested before the tile load; the
// factor rows of the next product (and of the plane tail) are requested
// right after the MFMAs of the current one, so each product finds its
// operands in registers after the barrier.  Waves with more than one
// sub-tile load the later ones in place.
template <typename T, int FM, int FN, int KCH, int NW, bool DG = true>
__device__ __forceinline__ void strided_tile(const StridedArgs& a, int bx, int by, int bz, unsigned char* smem) {
  constexpr int NT = 64 * NW;
  using acc_t = typename M16<T>::acc;
  using v4 = typename M16<T>::v4;
  constexpr int KR = KCH > 0 ? KCH : 1;  // register prefetch extent
  // cross-product prefetch only where two factor register sets fit
  // (FP64 with 128-long contractions keeps one set, loaded per product)
  constexpr bool kPre = KCH > 0 && (NW == 4 || FM > 1) && sizeof(T) * FM * KCH * 4 <= (sizeof(T) == 8 ? 128 : 256);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int nm = a.nm, na = a.na, TN = a.tn;
  const int NP = KCH > 0 ? 16 * KCH : (nm + 16 * FM - 1) / (16 * FM) * (16 * FM);
  const int ld = pitch_kmajor<T>(TN);
  T* sX = reinterpret_cast<T*>(smem);
  T* sT = sX + NP * ld;
  const int a0 = bx * TN, b = by, s = bz;
  const int64_t slab = static_cast<int64_t>(nm) * na * a.nb;
  const int64_t base = static_cast<int64_t>(s) * slab + static_cast<int64_t>(b) * nm * na;

  const int nrt = NP / (16 * FM), nct = TN / (16 * FN);
  const int nsub = nrt * nct;
  const bool keep = a.sandwich || a.plane;  // result of the first product stays in LDS
  const T* L1 = factor_of<T>(a.L1, s);
  const T* L2 = a.sandwich ? factor_of<T>(a.L2, s) : nullptr;
  const T* P = a.plane ? factor_of<T>(a.P, s) : nullptr;
  T* Y = static_cast<T*>(a.Y) + base;
  T* W = a.plane ? static_cast<T*>(a.W) + base : nullptr;
  const double cb = a.phi ? a.ph.cs[s] * (a.ph.pb ? a.ph.pb[b] : 1.0) : 0.0;
  const int KP = (na + 15) / 16 * 16;
  const bool plane_u = KCH > 0 && KP == 16 * KCH;  // plane tail unrolled too

  // 0. requests for this wave's first sub-tile, issued before the tile load
  const int r00 = (wave / nct) * 16 * FM, c00 = (wave % nct) * 16 * FN;
  v4 fv[FM][KR];
  double fr[FM][4], fc[FN];
  if constexpr (kPre)
    if (wave < nsub) load_rows_u<T, FM, KCH>(fv, L1, a.L1.ld, r00, lane);
  if (a.phi) {
    row_factors<T, FM>(fr, a.ph.pm, r00, g, nm, 0);
    col_factors<FN>(fc, a.ph.pn, c00, li, na - a0, a0);
  }

  // 1. data tile: rows k < NP (zero beyond nm), columns a0 .. a0 + TN
  if (a.stencil) {
    // The stencil launch is always the last mode (nb == 1): the column a
    // holds the faster coordinates, the row k the slowest one.
    double* cfs = reinterpret_cast<double*>(sT + NP * ld);
    const int sns = a.st.nspecies, inst = s / sns, sp = s % sns;
    // the common shapes with their mode and species counts fixed (fewer
    // branches and live scalars in the staging and arithmetic)
    if (a.st.ndim == 3 && sns == 2)
      stencil_tile<T, NT, 3, 2>(a.st, inst, sp, a0, NP, TN, nm, na, sX, sT, ld, cfs, tid);
    else if (a.st.ndim == 2 && sns == 2)
      stencil_tile<T, NT, 2, 2>(a.st, inst, sp, a0, NP, TN, nm, na, sX, sT, ld, cfs, tid);
    else
      stencil_tile<T, NT>(a.st, inst, sp, a0, NP, TN, nm, na, sX, sT, ld, cfs, tid);
  } else {
    load_tile_kmajor<T, NT>(static_cast<const T*>(a.X) + base, na, nm, a0, NP, TN, sX, ld, tid);
  }
  __syncthreads();

  // 2. first product (and the phi_1 factor)
  for (int sub = wave; sub < nsub; sub += NW) {
    const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
    const bool first = sub == wave;
    if (!first && a.phi) {
      row_factors<T, FM>(fr, a.ph.pm, r0, g, nm, 0);
      col_factors<FN>(fc, a.ph.pn, c0, li, na - a0, a0);
    }
    acc_t acc[FM][FN];
    zero<T, FM, FN>(acc);
    if constexpr (KCH > 0) {
      if (!first || !kPre) load_rows_u<T, FM, KCH>(fv, L1, a.L1.ld, r0, lane);
      mma_rows_sB<T, FM, FN, KCH>(acc, fv, sX, ld, c0, lane);
      // next product's factor rows for this wave's first sub-tile
      if (kPre && sub + NW >= nsub && a.sandwich) load_rows_u<T, FM, KCH>(fv, L2, a.L2.ld, r00, lane);
    } else {
      gemm_gA_sB<T, FM, FN>(acc, L1, a.L1.ld, r0, sX, ld, c0, NP, lane);
    }
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + 16 * f + M16<T>::row(g, r), col = c0 + 16 * j + li;
          T v = acc[f][j][r];
          const bool in = row < nm && a0 + col < na;
          if (a.phi) v *= M16<T>::phi1(static_cast<T>(cb * fr[f][r] * fc[j]));
          if (keep) sT[row * ld + col] = in ? v : T(0);
          else if (in) Y[static_cast<int64_t>(row) * na + a0 + col] = v;
        }
  }
  if (!keep) return;

  // requests of the plane tail for this wave's first sub-tile: the state
  // values of the update and (without a sandwich) the factor columns
  v4 pv[FN][KR];
  T wv[FM][FN][4];
  auto plane_requests = [&](int r0, int c0) {
    if constexpr (KCH > 0)
      if (plane_u) load_cols_u<T, FN, KCH>(pv, P, a.P.ld, c0, lane);
    if (a.update) {
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = min(r0 + 16 * f + M16<T>::row(g, r), nm - 1);
            const int col = min(c0 + 16 * j + li, na - 1);
            wv[f][j][r] = W[static_cast<int64_t>(row) * na + col];
          }
    }
  };
  if (kPre && a.plane && !a.sandwich && wave < nsub) plane_requests(r00, c00);
  __syncthreads();

  // 3. second product of the sandwich (into LDS for the plane tail)
  if (a.sandwich) {
    for (int sub = wave; sub < nsub; sub += NW) {
      const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
      const bool first = sub == wave;
      acc_t acc[FM][FN];
      zero<T, FM, FN>(acc);
      if constexpr (KCH > 0) {
        if (!first || !kPre) load_rows_u<T, FM, KCH>(fv, L2, a.L2.ld, r0, lane);
        mma_rows_sB<T, FM, FN, KCH>(acc, fv, sT, ld, c0, lane);
      } else {
        gemm_gA_sB<T, FM, FN>(acc, L2, a.L2.ld, r0, sT, ld, c0, NP, lane);
      }
      if (kPre && a.plane && sub + NW >= nsub) plane_requests(r00, c00);
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + 16 * f + M16<T>::row(g, r), col = c0 + 16 * j + li;
            const T v = acc[f][j][r];
            const bool in = row < nm && a0 + col < na;
            if (a.plane) sX[row * ld + col] = in ? v : T(0);
            else if (in) Y[static_cast<int64_t>(row) * na + a0 + col] = v;
          }
    }
    if (!a.plane) return;
    __syncthreads();
  }

  // 4. plane tail: Z[row][i'] = sum_i T[row][i] P[i'][i];  W += alpha Z
  const T* Tin = a.sandwich ? sX : sT;
  const T alpha = static_cast<T>(a.alpha);
  const bool diag = DG && a.dg.part != nullptr;  // grouped launches carry none
  double ds0 = 0.0, ds1 = 0.0;
  for (int sub = wave; sub < nsub; sub += NW) {
    const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
    if (sub != wave || !kPre) plane_requests(r0, c0);
    acc_t acc[FM][FN];
    zero<T, FM, FN>(acc);
    bool done = false;
    if constexpr (KCH > 0) {
      if (plane_u) {
        mma_sA_cols<T, FM, FN, KCH>(acc, Tin, ld, r0, pv, lane);
        done = true;
      }
    }
    if (!done) gemm_sA_gB<T, FM, FN>(acc, Tin, ld, r0, P, a.P.ld, c0, KP, lane);
    bool bad = false;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + 16 * f + M16<T>::row(g, r), col = c0 + 16 * j + li;
          const T nv = a.update ? wv[f][j][r] + alpha * acc[f][j][r] : acc[f][j][r];
          if (row < nm && col < na) {
            W[static_cast<int64_t>(row) * na + col] = nv;
            bad |= !isfinite(nv);
            if (diag)
              diag_point(a.dg, b * nm + row, col, static_cast<double>(nv),
                         a.update ? static_cast<double>(wv[f][j][r]) : 0.0, ds0, ds1);
          }
        }
    if (bad && a.flag) atomicOr(a.flag, 1);
  }
  if (diag) {
    const int nbx = (na + TN - 1) / TN;
    diag_flush<NW>(a.dg, ds0, ds1, static_cast<int64_t>(s) * a.dg.tiles + static_cast<int64_t>(b) * nbx + bx,
                   reinterpret_cast<double*>(smem));
  }
}

// 8-wave FP32 workgroups with one-row sub-tiles (many workgroups) are held
// to 128 VGPRs (4 waves per SIMD) so that two share a CU, and the other
// 8-wave ones and the FP32 runtime-K ones to 256 registers (2 waves per
// SIMD: the runtime-K variant otherwise lands just above and runs at one);
// the others may use more.
template <typename T, int FM, int FN, int NW, int KCH>
constexpr int waves_per_eu() {
  if (NW == 8) return (sizeof(T) == 4 && FM == 1) ? 4 : 2;
  if (sizeof(T) == 4) return KCH == 0 ? 2 : 1;
  // FP64: the variants that fit 256 registers (spilling at most a few bytes)
  return (FM == 2 && KCH > 0 && !(FN == 2 && KCH == 8)) ? 2 : 1;
}
// The persistent grouped kernels carry more live state: FP64 ones keep the
// uncapped register budget.
template <typename T, int FM, int FN, int NW, int KCH>
constexpr int group_waves_per_eu() { return sizeof(T) == 8 && NW == 4 ? 1 : waves_per_eu<T, FM, FN, NW, KCH>(); }

template <typename T, int FM, int FN, int KCH, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(waves_per_eu<T, FM, FN, NW, KCH>())))
void strided_kernel(StridedArgs a) {
  extern __shared__ __align__(256) unsigned char smem[];
  // 1D grid of 8 * per_xcd workgroups, dispatched round-robin over the 8
  // XCDs: XCD x takes logical tiles x * per_xcd .. (x + 1) * per_xcd.  The
  // logical order runs over the species of an instance first, then the
  // column tiles, so that a tile, its neighbours in the next-slower
  // coordinate and the other species' tiles of the same columns (read by
  // the in-tile stencil) share an XCD and its L2.
  const int nbx = (a.na + a.tn - 1) / a.tn;
  const int total = nbx * a.nb * a.nslab;
  const int per_xcd = (total + 7) / 8;
  const int L = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (L >= total) return;
  const int ns = a.stencil ? a.st.nspecies : 1;
  const int sp = L % ns;
  int rest = L / ns;
  const int bx = rest % nbx;
  rest /= nbx;
  const int by = rest % a.nb;
  const int inst = rest / a.nb;
  strided_tile<T, FM, FN, KCH, NW>(a, bx, by, inst * ns + sp, smem);
}

// ---------------------------------------------------------------------------
// Multi-tile form of the strided launches without an in-tile stencil or a
// plane tail (the same products and rounding as strided_tile): a tile is a
// few microseconds of load and barrier latency around a fraction of a
// microsecond of MFMA work, so a workgroup walks a run of consecutive tiles
// (row block b fastest, then the column tile, then the slab), loading the
// next tile into registers while the current one is multiplied; the factor
// rows of a wave stay in registers while the slab is unchanged, and the
// phi_1 factors while the column tile is (unless they depend on b).  Wave w
// owns rows 16 w .. 16 w + 15 (NP = 16 KCH rows, KCH waves) and all
// TN = 16 FN columns; a thread loads EPT = 4 FN rows of one column.  The data
// tile is double-buffered: one barrier per tile for a single product, two
// for a sandwich.
template <typename T, int KCH, int FN, int SW>
__global__ __launch_bounds__(64 * KCH) void strided_mt_kernel(StridedArgs a) {
  constexpr int NP = 16 * KCH, TN = 16 * FN, EPT = 4 * FN, LD = TN + 4;  // KCH waves
  using acc_t = typename M16<T>::acc;
  using v4 = typename M16<T>::v4;
  extern __shared__ __align__(256) unsigned char smem[];
  T* const sX = reinterpret_cast<T*>(smem);  // two buffers of NP x LD
  T* const sT = sX + 2 * NP * LD;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int nm = a.nm, na = a.na, nb = a.nb;
  const int nbx = (na + TN - 1) / TN;
  const int per_slab = nbx * nb;
  const int64_t total = static_cast<int64_t>(per_slab) * a.nslab;
  // logical workgroup w is XCD-major (blockIdx round-robins over the 8
  // XCDs), so one XCD's runs are adjacent; run w = [total w / G, total (w + 1) / G)
  const int G = gridDim.x, per_xcd = G / 8;
  const int w = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  const int lo = static_cast<int>(total * w / G), hi = static_cast<int>(total * (w + 1) / G);
  if (lo >= hi) return;
  const int lc = tid % TN, lk = (tid / TN) * EPT;
  const int r0 = 16 * wave;
  const T* X = static_cast<const T*>(a.X);
  T* Y = static_cast<T*>(a.Y);
  const int64_t slab = static_cast<int64_t>(nm) * na * nb;

  T pre[EPT];
  auto fetch = [&](int L) {
    const int s = L / per_slab, rest = L % per_slab, b = rest % nb, a0 = (rest / nb) * TN;
    const T* x = X + s * slab + static_cast<int64_t>(b) * nm * na + a0 + lc;
    const bool col = a0 + lc < na;
#pragma unroll
    for (int i = 0; i < EPT; ++i) pre[i] = (col && lk + i < nm) ? x[static_cast<int64_t>(lk + i) * na] : T(0);
  };
  fetch(lo);

  v4 f1[1][KCH], f2[1][SW ? KCH : 1];
  double fr[1][4];
  if (a.phi) row_factors<T, 1>(fr, a.ph.pm, r0, g, nm, 0);
  T ph[FN][4];
  int scur = -1, phs = -1, pha = -1;
  int buf = 0;
  for (int L = lo; L < hi; ++L, buf ^= 1) {
    const int s = L / per_slab, rest = L % per_slab, b = rest % nb, a0 = (rest / nb) * TN;
    T* const sb = sX + buf * NP * LD;
#pragma unroll
    for (int i = 0; i < EPT; ++i) sb[(lk + i) * LD + lc] = pre[i];
    if (L + 1 < hi) fetch(L + 1);
    if (s != scur) {
      scur = s;
      load_rows_u<T, 1, KCH>(f1, factor_of<T>(a.L1, s), a.L1.ld, r0, lane);
      if constexpr (SW) load_rows_u<T, 1, KCH>(f2, factor_of<T>(a.L2, s), a.L2.ld, r0, lane);
    }
    // phi_1 factors: the same for every row block b unless pb scales them
    if (a.phi && (s != phs || a0 != pha || a.ph.pb)) {
      phs = s;
      pha = a0;
      double fc[FN];
      const double cb = a.ph.cs[s] * (a.ph.pb ? a.ph.pb[b] : 1.0);
      col_factors<FN>(fc, a.ph.pn, 0, li, na - a0, a0);
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) ph[j][r] = M16<T>::phi1(static_cast<T>(cb * fr[0][r] * fc[j]));
    }
    __syncthreads();

    acc_t acc[1][FN];
    zero<T, 1, FN>(acc);
    mma_rows_sB<T, 1, FN, KCH>(acc, f1, sb, LD, 0, lane);
    T* const y = Y + s * slab + static_cast<int64_t>(b) * nm * na + a0;
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + M16<T>::row(g, r), col = 16 * j + li;
        T v = acc[0][j][r];
        const bool in = row < nm && a0 + col < na;
        if (a.phi) v *= ph[j][r];
        if (SW) sT[row * LD + col] = in ? v : T(0);
        else if (in) y[static_cast<int64_t>(row) * na + col] = v;
      }
    if constexpr (SW) {
      __syncthreads();
      zero<T, 1, FN>(acc);
      mma_rows_sB<T, 1, FN, KCH>(acc, f2, sT, LD, 0, lane);
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + M16<T>::row(g, r), col = 16 * j + li;
          if (row < nm && a0 + col < na) y[static_cast<int64_t>(row) * na + col] = acc[0][j][r];
        }
    }
  }
}

// ---------------------------------------------------------------------------
// One tile of a first-mode launch: rows bx * tm .., slab by.
template <typename T, int FM, int FN, int KCH, bool DG = true>
__device__ __forceinline__ void first_tile(const FirstArgs& a, int bx, int by, unsigned char* smem) {
  using acc_t = typename M16<T>::acc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int nm = a.nm, TM = a.tm;
  const int NP = KCH > 0 ? 16 * KCH : (nm + 16 * FN - 1) / (16 * FN) * (16 * FN);
  const int ld = pitch_rowvec<T>(NP);
  T* sX = reinterpret_cast<T*>(smem);
  T* sT = sX + TM * ld;
  const int rt0 = bx * TM, s = by;
  const int64_t base = static_cast<int64_t>(s) * a.rows * nm;

  load_tile_rows<T, 256>(static_cast<const T*>(a.X) + base, nm, a.rows, rt0, TM, NP, sX, ld, tid);
  __syncthreads();

  const int nrt = TM / (16 * FM), nct = NP / (16 * FN);
  const int nsub = nrt * nct;
  T* Y = static_cast<T*>(a.Y) + base;
  const T alpha = static_cast<T>(a.alpha);
  const bool diag = DG && a.dg.part != nullptr;  // grouped launches carry none
  double ds0 = 0.0, ds1 = 0.0;
  // final epilogue of a sub-tile: store, or add alpha * result to the target
  auto finish = [&](int r0, int c0, const acc_t (&acc)[FM][FN], const T (&yv)[FM][FN][4]) {
    bool bad = false;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rg = rt0 + r0 + 16 * f + M16<T>::row(g, r), col = c0 + 16 * j + li;
          const T nv = a.update ? yv[f][j][r] + alpha * acc[f][j][r] : acc[f][j][r];
          if (rg < a.rows && col < nm) {
            Y[static_cast<int64_t>(rg) * nm + col] = nv;
            bad |= !isfinite(nv);
            if (diag)
              diag_point(a.dg, rg, col, static_cast<double>(nv), a.update ? static_cast<double>(yv[f][j][r]) : 0.0,
                         ds0, ds1);
          }
        }
    if (bad && a.update && a.flag) atomicOr(a.flag, 1);
  };
  auto flush = [&]() {
    if (diag)
      diag_flush<4>(a.dg, ds0, ds1, static_cast<int64_t>(s) * a.dg.tiles + bx, reinterpret_cast<double*>(smem));
  };
  auto prefetch = [&](int r0, int c0, T (&yv)[FM][FN][4]) {
    if (!a.update) return;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rg = min(rt0 + r0 + 16 * f + M16<T>::row(g, r), a.rows - 1);
          const int col = min(c0 + 16 * j + li, nm - 1);
          yv[f][j][r] = Y[static_cast<int64_t>(rg) * nm + col];
        }
  };
  const T* L1 = factor_of<T>(a.L1, s);
  const double cs = a.sandwich ? a.ph.cs[s] : 0.0;
  for (int sub = wave; sub < nsub; sub += 4) {
    const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
    T yv[FM][FN][4];
    T ph[FM][FN][4];
    if (a.sandwich) {
      double fr[FM][4], fc[FN];
      row_factors<T, FM>(fr, a.ph.pm, r0, g, a.rows - rt0, rt0);
      col_factors<FN>(fc, a.ph.pn, c0, li, nm, 0);
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) ph[f][j][r] = M16<T>::phi1(static_cast<T>(cs * fr[f][r] * fc[j]));
    } else {
      prefetch(r0, c0, yv);
    }
    acc_t acc[FM][FN];
    zero<T, FM, FN>(acc);
    mm_sA_gB<T, FM, FN, KCH>(acc, sX, ld, r0, L1, a.L1.ld, c0, NP, lane);
    if (!a.sandwich) {
      finish(r0, c0, acc, yv);
      continue;
    }
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + 16 * f + M16<T>::row(g, r), col = c0 + 16 * j + li;
          const bool in = col < nm && rt0 + row < a.rows;
          const T v = acc[f][j][r] * ph[f][j][r];
          sT[row * ld + col] = in ? v : T(0);
        }
  }
  if (!a.sandwich) {
    flush();
    return;
  }
  __syncthreads();
  const T* L2 = factor_of<T>(a.L2, s);
  for (int sub = wave; sub < nsub; sub += 4) {
    const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
    T yv[FM][FN][4];
    prefetch(r0, c0, yv);
    acc_t acc[FM][FN];
    zero<T, FM, FN>(acc);
    mm_sA_gB<T, FM, FN, KCH>(acc, sT, ld, r0, L2, a.L2.ld, c0, NP, lane);
    finish(r0, c0, acc, yv);
  }
  flush();
}

// Multi-tile form of the single first-mode product (no sandwich, no
// indicators), with or without the update W += alpha Z: the same products
// and rounding as first_tile.  A workgroup walks a run of consecutive row
// tiles; the next tile's rows (and the state values its update adds to)
// are loaded into registers while the current one is multiplied, and each
// wave keeps the factor rows of its 32 output columns in registers while
// the slab is unchanged.  TM = 16 FM rows per tile, NP = 16 KCH columns,
// KCH / 2 waves.
template <typename T, int KCH, int FM>
__global__ __launch_bounds__(32 * KCH) void first_mt_kernel(FirstArgs a) {
  constexpr int FN = 2, NW = KCH / 2, NTH = 64 * NW, NP = 16 * KCH, TM = 16 * FM, LD = NP + 4;
  constexpr int VPT = TM * NP / 4 / NTH;  // 4-element groups per thread
  using acc_t = typename M16<T>::acc;
  using v4 = typename M16<T>::v4;
  extern __shared__ __align__(256) unsigned char smem[];
  T* const sX = reinterpret_cast<T*>(smem);  // two buffers of TM x LD
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int nm = a.nm, rows = a.rows;
  const int nrt = (rows + TM - 1) / TM;
  const int64_t total = static_cast<int64_t>(nrt) * a.nslab;
  const int G = gridDim.x, per_xcd = G / 8;
  const int w = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  const int lo = static_cast<int>(total * w / G), hi = static_cast<int>(total * (w + 1) / G);
  if (lo >= hi) return;
  const int c0 = 32 * wave;
  const bool vec = nm % 4 == 0;
  const T* X = static_cast<const T*>(a.X);
  T* Y = static_cast<T*>(a.Y);
  const T alpha = static_cast<T>(a.alpha);
  const int64_t slab = static_cast<int64_t>(rows) * nm;

  v4 pre[VPT];
  T yn[FM][FN][4];
  auto fetch = [&](int L) {
    const int s = L / nrt, rt0 = (L % nrt) * TM;
    const T* x = X + s * slab;
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int e = 4 * (tid + NTH * q), r = e / NP, c = e % NP;
      const int64_t off = static_cast<int64_t>(rt0 + r) * nm + c;
      const bool rin = rt0 + r < rows;
      if (vec) {
        pre[q] = (rin && c < nm) ? *reinterpret_cast<const v4*>(x + off) : v4{0, 0, 0, 0};
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) pre[q][u] = (rin && c + u < nm) ? x[off + u] : T(0);
      }
    }
    if (a.update) {
      const T* y = Y + s * slab;
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rg = min(rt0 + 16 * f + M16<T>::row(g, r), rows - 1);
            const int col = min(c0 + 16 * j + li, nm - 1);
            yn[f][j][r] = y[static_cast<int64_t>(rg) * nm + col];
          }
    }
  };
  fetch(lo);

  v4 fb[FN][KCH];
  int scur = -1;
  int buf = 0;
  for (int L = lo; L < hi; ++L, buf ^= 1) {
    const int s = L / nrt, rt0 = (L % nrt) * TM;
    T* const sb = sX + buf * TM * LD;
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int e = 4 * (tid + NTH * q), r = e / NP, c = e % NP;
      *reinterpret_cast<v4*>(sb + r * LD + c) = pre[q];
    }
    T yv[FM][FN][4];
    if (a.update) {
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) yv[f][j][r] = yn[f][j][r];
    }
    if (L + 1 < hi) fetch(L + 1);
    if (s != scur) {
      scur = s;
      load_cols_u<T, FN, KCH>(fb, factor_of<T>(a.L1, s), a.L1.ld, c0, lane);
    }
    __syncthreads();

    acc_t acc[FM][FN];
    zero<T, FM, FN>(acc);
    mma_sA_cols<T, FM, FN, KCH>(acc, sb, LD, 0, fb, lane);
    T* const y = Y + s * slab;
    bool bad = false;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rg = rt0 + 16 * f + M16<T>::row(g, r), col = c0 + 16 * j + li;
          const T nv = a.update ? yv[f][j][r] + alpha * acc[f][j][r] : acc[f][j][r];
          if (rg < rows && col < nm) {
            y[static_cast<int64_t>(rg) * nm + col] = nv;
            bad |= !isfinite(nv);
          }
        }
    if (bad && a.update && a.flag) atomicOr(a.flag, 1);
  }
}

template <typename T, int FM, int FN, int KCH>
__global__ __launch_bounds__(256) void first_kernel(FirstArgs a) {
  extern __shared__ __align__(256) unsigned char smem[];
  first_tile<T, FM, FN, KCH>(a, blockIdx.x, blockIdx.y, smem);
}

// ---------------------------------------------------------------------------
// Grouped persistent launches: the tiles of up to kMaxGroup launches of the
// same kind (e.g. the same chain op of plans on different grids) in one
// grid.  Workgroups are dispatched round-robin over the 8 XCDs, so the grid
// size is a multiple of 8 and tile t of the strided loop is remapped so that
// each XCD walks a contiguous range of logical tiles (consecutive tiles
// share a slab and its factors, which then stay in that XCD's L2).
__device__ __forceinline__ int group_member(const GroupMap& m, int L, int& local) {
  int q = 0;
  while (q + 1 < m.n && L >= m.start[q + 1]) ++q;
  local = L - m.start[q];
  return q;
}

template <typename T, int FM, int FN, int KCH, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(group_waves_per_eu<T, FM, FN, NW, KCH>())))
void strided_group_kernel(const StridedGroup* __restrict__ grp) {
  extern __shared__ __align__(256) unsigned char smem[];
  const GroupMap& m = grp->map;
  for (int t = blockIdx.x; t < m.span; t += gridDim.x) {
    const int L = (t & 7) * m.per_xcd + (t >> 3);
    if (L >= m.total) continue;
    int local;
    const int q = group_member(m, L, local);
    const int nbx = m.nbx[q], nby = m.nby[q];
    strided_tile<T, FM, FN, KCH, NW, false>(grp->a[q], local % nbx, (local / nbx) % nby, local / (nbx * nby),
                                            smem);
    __syncthreads();  // the next tile reuses the LDS
  }
}

template <typename T, int FM, int FN, int KCH>
__global__ __launch_bounds__(256) void first_group_kernel(const FirstGroup* __restrict__ grp) {
  extern __shared__ __align__(256) unsigned char smem[];
  const GroupMap& m = grp->map;
  for (int t = blockIdx.x; t < m.span; t += gridDim.x) {
    const int L = (t & 7) * m.per_xcd + (t >> 3);
    if (L >= m.total) continue;
    int local;
    const int q = group_member(m, L, local);
    const int nbx = m.nbx[q];
    first_tile<T, FM, FN, KCH, false>(grp->a[q], local % nbx, local / nbx, smem);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Host launchers.  FM / FN are picked from the shape: FM covers the rows of
// a wave sub-tile (16 FM), FN its columns (16 FN).

// Contractions up to 128 run fully unrolled with the padded extent
// NP = 16 KCH (KCH = 4 or 8) and FM = 2; longer ones use the runtime loop
// with FM = 4 and NP = nm rounded up to 64.
static int pick_kch(int nm) { return nm <= 64 ? 4 : (nm <= 128 ? 8 : 0); }
static int strided_np(int nm) {
  const int kch = pick_kch(nm);
  return kch ? 16 * kch : round_up(nm, 64);
}
static int first_np(int nm) {
  const int kch = pick_kch(nm);
  return kch ? 16 * kch : round_up(nm, 32);
}

template <typename T>
size_t strided_lds_bytes(int nm, int tn, int sandwich, int plane, int stencil) {
  const int NP = strided_np(nm);
  const int ld = pitch_kmajor<T>(tn);
  const int bufs = (sandwich || plane || stencil) ? 2 : 1;
  return static_cast<size_t>(bufs) * NP * ld * sizeof(T) +
         (stencil ? sizeof(double) * stencil_coef_doubles(NP, tn) : 0);
}

template <typename T>
size_t first_lds_bytes(int nm, int tm, int sandwich) {
  const int NP = first_np(nm);
  const int ld = pitch_rowvec<T>(NP);
  return static_cast<size_t>(sandwich ? 2 : 1) * tm * ld * sizeof(T);
}

static constexpr size_t kMaxLds = 160 * 1024;

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

// Strided kernel variants (FM, FN, KCH, NW).  Contractions up to 128 use
// the unrolled products; in FP32, with at least 8 sub-tiles a workgroup
// runs 8 waves (more waves per SIMD to overlap the latencies of loads, LDS
// and the phi_1 epilogue), otherwise 4.
struct SVar {
  int fm, fn, kch, nw;
};
static constexpr SVar kSVar[10] = {{2, 1, 4, 4}, {2, 2, 4, 4}, {2, 1, 8, 4}, {2, 2, 8, 4}, {4, 1, 0, 4},
                                   {4, 2, 0, 4}, {1, 1, 4, 8}, {2, 1, 4, 8}, {1, 1, 8, 8}, {2, 1, 8, 8}};

static int strided_variant(int kch, int NP, int TN, bool wide_ok) {
  if (kch > 0 && wide_ok) {
    const int nct1 = TN / 16;
    const int base = kch == 4 ? 0 : 2;
    if ((NP / 32) * nct1 >= 8) return kch == 4 ? 7 : 9;
    if ((NP / 16) * nct1 >= 8) return kch == 4 ? 6 : 8;
    return base + (TN % 32 == 0 ? 1 : 0);
  }
  if (kch > 0) return (kch == 4 ? 0 : 2) + (TN % 32 == 0 ? 1 : 0);
  return TN % 32 == 0 ? 5 : 4;
}

static bool variant_fits(int v, int NP, int TN) {
  const SVar& x = kSVar[v];
  return NP % (16 * x.fm) == 0 && TN % (16 * x.fn) == 0 && (x.kch == 0 || NP == 16 * x.kch);
}

// Call f.template operator()<FM, FN, KCH, NW>() for variant v.
template <typename F>
static hipError_t with_svar(int v, F&& f) {
  switch (v) {
    case 0: return f.template operator()<2, 1, 4, 4>();
    case 1: return f.template operator()<2, 2, 4, 4>();
    case 2: return f.template operator()<2, 1, 8, 4>();
    case 3: return f.template operator()<2, 2, 8, 4>();
    case 4: return f.template operator()<4, 1, 0, 4>();
    case 5: return f.template operator()<4, 2, 0, 4>();
    case 6: return f.template operator()<1, 1, 4, 8>();
    case 7: return f.template operator()<2, 1, 4, 8>();
    case 8: return f.template operator()<1, 1, 8, 8>();
    case 9: return f.template operator()<2, 1, 8, 8>();
    default: return hipErrorInvalidValue;
  }
}

int resident_workgroups(const void* kernel, int threads, size_t lds) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, int, size_t>, int> known;
  const auto key = std::make_tuple(kernel, dev, threads, lds);
  std::lock_guard<std::mutex> hold(mu);
  const auto it = known.find(key);
  if (it != known.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 0;
  return known[key] = per_cu * cus;
}

// Multi-tile launches: as many workgroups as fit on the device at once (at
// most one per tile), a multiple of 8 for the XCD-major run order.
template <typename T, int KCH, int FN, int SW>
static hipError_t go_strided_mt(const StridedArgs& a, hipStream_t s) {
  auto k = strided_mt_kernel<T, KCH, FN, SW>;
  constexpr int threads = 64 * KCH;
  constexpr size_t lds = static_cast<size_t>(2 + SW) * 16 * KCH * (16 * FN + 4) * sizeof(T);
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  const int fit = resident_workgroups(reinterpret_cast<const void*>(k), threads, lds);
  if (fit < 1) return hipErrorInvalidValue;
  const int64_t total = static_cast<int64_t>((a.na + 16 * FN - 1) / (16 * FN)) * a.nb * a.nslab;
  if (total >= (int64_t(1) << 30)) return hipErrorInvalidValue;
  const int grid = static_cast<int>((std::min<int64_t>(fit, total) + 7) / 8 * 8);
  hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_strided(const StridedArgs& a, hipStream_t s) {
  if (a.nm <= 0 || a.na <= 0 || a.nb <= 0 || a.nslab <= 0 || a.nb > 65535 || a.nslab > 65535)
    return hipErrorInvalidValue;
  if (a.tn != 16 && a.tn % 32 != 0) return hipErrorInvalidValue;
  if (a.plane && a.tn < a.na) return hipErrorInvalidValue;  // plane needs whole rows
  const int NP = strided_np(a.nm);
  if (a.L1.ld < NP || (a.sandwich && a.L2.ld < NP) || (a.plane && a.P.ld < round_up(a.na, 32)))
    return hipErrorInvalidValue;
  const size_t lds = strided_lds_bytes<T>(a.nm, a.tn, a.sandwich, a.plane, a.stencil);
  if (lds > kMaxLds) return hipErrorInvalidValue;
  // 8-wave workgroups for FP32 only (measured: FP64 is faster with 4)
  const int v = strided_variant(pick_kch(a.nm), NP, a.tn, sizeof(T) == 4);
  StridedArgs b = a;
  if (b.dg.part) {  // indicators: plane-tail updates, one partial pair per tile
    b.dg.tiles = (a.na + a.tn - 1) / a.tn * a.nb;
    if (!a.plane || !a.update || b.dg.tiles > b.dg.cap) return hipErrorInvalidValue;
  }
  if (!a.stencil && !a.plane && !b.dg.part && pick_kch(a.nm) > 0 && (a.tn == 16 || a.tn == 32)) {
    const bool k8 = pick_kch(a.nm) == 8;
    if (a.tn == 16)
      return a.sandwich ? (k8 ? go_strided_mt<T, 8, 1, 1>(a, s) : go_strided_mt<T, 4, 1, 1>(a, s))
                        : (k8 ? go_strided_mt<T, 8, 1, 0>(a, s) : go_strided_mt<T, 4, 1, 0>(a, s));
    return a.sandwich ? (k8 ? go_strided_mt<T, 8, 2, 1>(a, s) : go_strided_mt<T, 4, 2, 1>(a, s))
                      : (k8 ? go_strided_mt<T, 8, 2, 0>(a, s) : go_strided_mt<T, 4, 2, 0>(a, s));
  }
  hipError_t e = with_svar(v, [&]<int FM, int FN, int KCH, int NW>() -> hipError_t {
    auto k = strided_kernel<T, FM, FN, KCH, NW>;
    hipError_t e = allow_lds(k, lds);
    if (e != hipSuccess) return e;
    const int64_t total = static_cast<int64_t>((a.na + a.tn - 1) / a.tn) * a.nb * a.nslab;
    if (total >= (int64_t(1) << 30)) return hipErrorInvalidValue;
    const int per_xcd = static_cast<int>((total + 7) / 8);
    hipLaunchKernelGGL(k, dim3(8 * per_xcd), dim3(64 * NW), lds, s, b);
    return hipGetLastError();
  });
  if (e != hipSuccess || !b.dg.part) return e;
  return launch_diag_finish(b.dg, b.nslab, s);
}

template <typename T, int FM, int FN, int KCH>
static hipError_t go_first(const FirstArgs& a, size_t lds, hipStream_t s) {
  auto k = first_kernel<T, FM, FN, KCH>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  dim3 grid((a.rows + a.tm - 1) / a.tm, a.nslab);
  hipLaunchKernelGGL(k, grid, dim3(256), lds, s, a);
  return hipGetLastError();
}

template <typename T, int KCH, int FM>
static hipError_t go_first_mt(const FirstArgs& a, hipStream_t s) {
  auto k = first_mt_kernel<T, KCH, FM>;
  constexpr int threads = 32 * KCH;
  constexpr size_t lds = static_cast<size_t>(2) * 16 * FM * (16 * KCH + 4) * sizeof(T);
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  const int fit = resident_workgroups(reinterpret_cast<const void*>(k), threads, lds);
  if (fit < 1) return hipErrorInvalidValue;
  const int64_t total = static_cast<int64_t>((a.rows + 16 * FM - 1) / (16 * FM)) * a.nslab;
  if (total >= (int64_t(1) << 30)) return hipErrorInvalidValue;
  const int grid = static_cast<int>((std::min<int64_t>(fit, total) + 7) / 8 * 8);
  hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_first(const FirstArgs& a, hipStream_t s) {
  if (a.nm <= 0 || a.rows <= 0 || a.nslab <= 0 || a.nslab > 65535) return hipErrorInvalidValue;
  if (a.tm != 16 && a.tm != 32) return hipErrorInvalidValue;
  const int NP = first_np(a.nm);
  if (a.L1.ld < NP || (a.sandwich && a.L2.ld < NP)) return hipErrorInvalidValue;
  const size_t lds = first_lds_bytes<T>(a.nm, a.tm, a.sandwich);
  if (lds > kMaxLds) return hipErrorInvalidValue;
  FirstArgs b = a;
  if (b.dg.part) {  // indicators: one partial pair per row block
    b.dg.tiles = (a.rows + a.tm - 1) / a.tm;
    if (!a.update || b.dg.tiles > b.dg.cap) return hipErrorInvalidValue;
  }
  const int kch = pick_kch(a.nm);
  // multi-tile for FP32 only (measured: the FP64 single-tile kernel with
  // 32-row tiles is faster than either multi-tile FP64 form)
  if constexpr (sizeof(T) == 4) {
    if (!a.sandwich && !b.dg.part && kch > 0) {
      if (a.tm == 16) return kch == 4 ? go_first_mt<T, 4, 1>(a, s) : go_first_mt<T, 8, 1>(a, s);
      return kch == 4 ? go_first_mt<T, 4, 2>(a, s) : go_first_mt<T, 8, 2>(a, s);
    }
  }
  hipError_t e;
  if (a.tm == 16) {
    if (kch == 4) e = go_first<T, 1, 2, 4>(b, lds, s);
    else if (kch == 8) e = go_first<T, 1, 2, 8>(b, lds, s);
    else e = go_first<T, 1, 2, 0>(b, lds, s);
  } else {
    if (kch == 4) e = go_first<T, 2, 2, 4>(b, lds, s);
    else if (kch == 8) e = go_first<T, 2, 2, 8>(b, lds, s);
    else e = go_first<T, 2, 2, 0>(b, lds, s);
  }
  if (e != hipSuccess || !b.dg.part) return e;
  return launch_diag_finish(b.dg, b.nslab, s);
}

// ---------------------------------------------------------------------------
// Grouped launches
static int round8(int x) { return (x + 7) / 8 * 8; }

template <typename K>
static hipError_t group_grid(K kernel, int block, size_t lds, int span, int& grid) {
  hipError_t e = allow_lds(kernel, lds);
  if (e != hipSuccess) return e;
  int per_cu = 0, dev = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds);
  if (e != hipSuccess) return e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidValue;
  grid = std::min(round8(per_cu * cus), span);  // span is a multiple of 8
  return hipSuccess;
}

template <typename T>
hipError_t plan_strided_group(StridedGroup& g, GroupLaunch& L) {
  GroupMap& m = g.map;
  if (m.n < 1 || m.n > kMaxGroup) return hipErrorInvalidValue;
  int kch = pick_kch(g.a[0].nm);
  for (int q = 0; q < m.n; ++q) {
    const StridedArgs& a = g.a[q];
    if (a.nm <= 0 || a.na <= 0 || a.nb <= 0 || a.nslab <= 0) return hipErrorInvalidValue;
    if (a.tn != 16 && a.tn % 32 != 0) return hipErrorInvalidValue;
    if (a.plane && a.tn < a.na) return hipErrorInvalidValue;
    if (pick_kch(a.nm) != kch) kch = 0;
  }
  size_t lds = 0;
  int64_t most = -1;
  int v = -1;
  for (int q = 0; q < m.n; ++q) {
    const StridedArgs& a = g.a[q];
    const int NP = kch ? 16 * kch : round_up(a.nm, 64);
    if (a.L1.ld < NP || (a.sandwich && a.L2.ld < NP) || (a.plane && a.P.ld < round_up(a.na, 32)))
      return hipErrorInvalidValue;
    const size_t b = static_cast<size_t>((a.sandwich || a.plane || a.stencil) ? 2 : 1) * NP * pitch_kmajor<T>(a.tn) *
                         sizeof(T) + (a.stencil ? sizeof(double) * stencil_coef_doubles(NP, a.tn) : 0);
    lds = std::max(lds, b);
    m.nbx[q] = (a.na + a.tn - 1) / a.tn;
    m.nby[q] = a.nb;
    const int64_t tiles = static_cast<int64_t>(m.nbx[q]) * a.nb * a.nslab;
    if (tiles > (1 << 30)) return hipErrorInvalidValue;
    if (tiles > most) {  // the variant the member with the most tiles prefers
      most = tiles;
      v = strided_variant(kch, NP, a.tn, sizeof(T) == 4);
    }
  }
  if (lds > kMaxLds) return hipErrorInvalidValue;
  for (int q = 0; q < m.n; ++q) {
    const int NP = kch ? 16 * kch : round_up(g.a[q].nm, 64);
    if (!variant_fits(v, NP, g.a[q].tn)) v = kch == 4 ? 6 : (kch == 8 ? 8 : 4);  // (1, 1) or (4, 1) fit all
  }
  for (int q = 0; q < m.n; ++q) {
    const int NP = kch ? 16 * kch : round_up(g.a[q].nm, 64);
    if (!variant_fits(v, NP, g.a[q].tn)) return hipErrorInvalidValue;
  }
  m.start[0] = 0;
  for (int q = 0; q < m.n; ++q) m.start[q + 1] = m.start[q] + m.nbx[q] * m.nby[q] * g.a[q].nslab;
  m.total = m.start[m.n];
  m.per_xcd = (m.total + 7) / 8;
  m.span = 8 * m.per_xcd;
  L.variant = v;
  L.lds = lds;
  return with_svar(v, [&]<int FM, int FN, int KCH, int NW>() -> hipError_t {
    return group_grid(strided_group_kernel<T, FM, FN, KCH, NW>, 64 * NW, lds, m.span, L.grid);
  });
}

template <typename T>
hipError_t launch_strided_group(const GroupLaunch& L, const StridedGroup* dev, hipStream_t s) {
  if (!dev || L.grid <= 0 || L.grid % 8 != 0) return hipErrorInvalidValue;
  return with_svar(L.variant, [&]<int FM, int FN, int KCH, int NW>() -> hipError_t {
    hipLaunchKernelGGL((strided_group_kernel<T, FM, FN, KCH, NW>), dim3(L.grid), dim3(64 * NW), L.lds, s, dev);
    return hipGetLastError();
  });
}

// first-mode variants: 0 (1,2,4) 1 (1,2,8) 2 (1,2,0) 3 (2,2,4) 4 (2,2,8) 5 (2,2,0)
template <typename T>
hipError_t plan_first_group(FirstGroup& g, GroupLaunch& L) {
  GroupMap& m = g.map;
  if (m.n < 1 || m.n > kMaxGroup) return hipErrorInvalidValue;
  int kch = pick_kch(g.a[0].nm);
  const int tm = g.a[0].tm;
  if (tm != 16 && tm != 32) return hipErrorInvalidValue;
  for (int q = 0; q < m.n; ++q) {
    const FirstArgs& a = g.a[q];
    if (a.nm <= 0 || a.rows <= 0 || a.nslab <= 0 || a.tm != tm) return hipErrorInvalidValue;
    if (pick_kch(a.nm) != kch) kch = 0;
  }
  size_t lds = 0;
  for (int q = 0; q < m.n; ++q) {
    const FirstArgs& a = g.a[q];
    const int NP = kch ? 16 * kch : round_up(a.nm, 32);
    if (a.L1.ld < NP || (a.sandwich && a.L2.ld < NP)) return hipErrorInvalidValue;
    lds = std::max(lds, static_cast<size_t>(a.sandwich ? 2 : 1) * tm * pitch_rowvec<T>(NP) * sizeof(T));
    m.nbx[q] = (a.rows + tm - 1) / tm;
    m.nby[q] = 1;
    if (static_cast<int64_t>(m.nbx[q]) * a.nslab > (1 << 30)) return hipErrorInvalidValue;
  }
  if (lds > kMaxLds) return hipErrorInvalidValue;
  m.start[0] = 0;
  for (int q = 0; q < m.n; ++q) m.start[q + 1] = m.start[q] + m.nbx[q] * g.a[q].nslab;
  m.total = m.start[m.n];
  m.per_xcd = (m.total + 7) / 8;
  m.span = 8 * m.per_xcd;
  L.variant = (tm == 16 ? 0 : 3) + (kch == 4 ? 0 : kch == 8 ? 1 : 2);
  L.lds = lds;
  switch (L.variant) {
    case 0: return group_grid(first_group_kernel<T, 1, 2, 4>, 256, lds, m.span, L.grid);
    case 1: return group_grid(first_group_kernel<T, 1, 2, 8>, 256, lds, m.span, L.grid);
    case 2: return group_grid(first_group_kernel<T, 1, 2, 0>, 256, lds, m.span, L.grid);
    case 3: return group_grid(first_group_kernel<T, 2, 2, 4>, 256, lds, m.span, L.grid);
    case 4: return group_grid(first_group_kernel<T, 2, 2, 8>, 256, lds, m.span, L.grid);
    default: return group_grid(first_group_kernel<T, 2, 2, 0>, 256, lds, m.span, L.grid);
  }
}

template <typename T>
hipError_t launch_first_group(const GroupLaunch& L, const FirstGroup* dev, hipStream_t s) {
  if (!dev || L.grid <= 0 || L.grid % 8 != 0) return hipErrorInvalidValue;
  const dim3 grid(L.grid), block(256);
  switch (L.variant) {
    case 0: hipLaunchKernelGGL((first_group_kernel<T, 1, 2, 4>), grid, block, L.lds, s, dev); break;
    case 1: hipLaunchKernelGGL((first_group_kernel<T, 1, 2, 8>), grid, block, L.lds, s, dev); break;
    case 2: hipLaunchKernelGGL((first_group_kernel<T, 1, 2, 0>), grid, block, L.lds, s, dev); break;
    case 3: hipLaunchKernelGGL((first_group_kernel<T, 2, 2, 4>), grid, block, L.lds, s, dev); break;
    case 4: hipLaunchKernelGGL((first_group_kernel<T, 2, 2, 8>), grid, block, L.lds, s, dev); break;
    case 5: hipLaunchKernelGGL((first_group_kernel<T, 2, 2, 0>), grid, block, L.lds, s, dev); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Several split steps in one launch for a plan whose step is a single fused
// op (stencil, sandwich with its phi_1 factor, plane tail with the update:
// the disk, eq. (ee_disk)).  One workgroup per instance keeps the state, F
// and the sandwich intermediate of every species in LDS, so the steps cost
// no launches and no HBM round trips, and the reaction reads the other
// species from the same workgroup's LDS.
//
// LDS: sW, sF, sT = [ns][NP][ld] (row k: mode 2, the sandwich's coordinate;
// column c: mode 1), then the operator tables rc [NP][5] (rs_0, 0, L, D, U
// of the row mode, as in stencil_tile) and cc [TN][4] (A, B, C of the column
// mode, cs_r) in FP64.  Padding rows and columns of sF and sT stay zero.
//
// KR > 0: NP = 16 KR, TN = 16 KC and NW = KR KC waves, so each wave owns one
// 16 x 16 output position of every product for all species and keeps, for
// all the steps, its factor rows (V^-1, V), its factor columns (P of each
// species) and its phi_1 values in registers: a step then reads nothing
// but LDS.  KR == 0: any padded shape, factors read from L2 per product
// and phi_1 evaluated per step.
template <typename T, int NW, int KR, int KC>
__global__ __launch_bounds__(64 * NW) void resident_kernel(ResidentArgs r) {
  // species held in registers by the register-resident form
  constexpr int NSR = KR > 0 ? 2 : 3;
  extern __shared__ __align__(256) unsigned char smem[];
  constexpr int NT = 64 * NW;
  using acc_t = typename M16<T>::acc;
  const StridedArgs& a = r.a;
  const StencilArgs& st = a.st;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int ns = st.nspecies, inst = blockIdx.x;
  const int nm = a.nm, na = a.na, NP = r.np, TN = r.tn;
  const int ld = pitch_kmajor<T>(TN), tile = NP * ld;
  T* sW = reinterpret_cast<T*>(smem);
  T* sF = sW + ns * tile;
  T* sT = sF + ns * tile;
  double* rc = reinterpret_cast<double*>(sT + ns * tile);
  double* cc = rc + 5 * NP;
  const int64_t plane = static_cast<int64_t>(nm) * na;
  T* Wg = static_cast<T*>(a.W) + static_cast<int64_t>(inst) * ns * plane;
  const Div dld(ld), dna(na);

  // 1. the state of every species; padding and work tiles zeroed
  for (int s = 0; s < ns; ++s)
    for (int e = tid; e < tile; e += NT) {
      int c;
      const int k = dld.quot(e, c);
      const bool in = k < nm && c < na;
      sW[s * tile + e] = in ? Wg[s * plane + static_cast<int64_t>(k) * na + c] : T(0);
      sF[s * tile + e] = T(0);
      sT[s * tile + e] = T(0);
    }
  // operator tables (2D: the row mode is mode 2, the column mode mode 1)
  const int nmx = st.nmax;
  for (int k = tid; k < NP; k += NT) {
    const int kk = min(k, nm - 1);
    const double rs0 = ((st.scale_mask >> 1) & 1) ? st.scale[nmx + kk] : 1.0;
    const double rs1 = ((st.scale_mask >> 4) & 1) ? st.scale[3 * nmx + nmx + kk] : 1.0;
    const double* rcoef = st.coef + 3 * nmx;
    rc[k * 5 + 0] = rs0;
    rc[k * 5 + 1] = 0.0;
    rc[k * 5 + 2] = rs1 * rcoef[kk];
    rc[k * 5 + 3] = rs1 * rcoef[nmx + kk];
    rc[k * 5 + 4] = rs1 * rcoef[2 * nmx + kk];
  }
  for (int c = tid; c < TN; c += NT) {
    const int ci = min(c, na - 1);
    const double cs0 = (st.scale_mask & 1) ? st.scale[ci] : 1.0;
    const double cs1 = ((st.scale_mask >> 3) & 1) ? st.scale[3 * nmx + ci] : 1.0;
    cc[c * 4 + 0] = cs0 * st.coef[ci];
    cc[c * 4 + 1] = cs0 * st.coef[nmx + ci];
    cc[c * 4 + 2] = cs0 * st.coef[2 * nmx + ci];
    cc[c * 4 + 3] = cs1;
  }
  double dif[3] = {0.0, 0.0, 0.0}, cphi[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < ns; ++s) {
    dif[s] = st.diff[inst * ns + s];
    cphi[s] = a.ph.cs[inst * ns + s];
  }
  const ReactConst rcst = react_const(st, inst);
  const bool react = st.reaction != 0;
  const bool per_c = st.periodic_mask & 1;         // mode 1 wraps around
  const bool per_r = (st.periodic_mask >> 1) & 1;  // mode 2 wraps around
  const int nct = TN / 16, nsub1 = (NP / 16) * nct, nsub = ns * nsub1;
  const T alpha = static_cast<T>(a.alpha);
  // register-resident operands of this wave's output position (KR > 0)
  using v4 = typename M16<T>::v4;
  // KR > 0: wave w owns output position w % (KR KC) and the species
  // w / (KR KC), w / (KR KC) + SPW, ... (SPW = NW / (KR KC) waves per
  // position), NJ = NSR / SPW of them
  constexpr int KRr = KR > 0 ? KR : 1, KCr = KC > 0 ? KC : 1;
  constexpr int SPW = KR > 0 ? NW / (KR * KC) : 1, NJ = NSR / SPW;
  static_assert(KR == 0 || (SPW >= 1 && NJ >= 1 && NJ * SPW == NSR), "resident: waves per position");
  const int pos = wave % (KRr * KCr), s0 = wave / (KRr * KCr);
  const int wr0 = KR > 0 ? (pos / KCr) * 16 : 0, wc0 = KR > 0 ? (pos % KCr) * 16 : 0;
  v4 f1[1][KRr], f2[1][KRr], fp[NJ][1][KCr];
  T ph[NJ][4];
  if constexpr (KR > 0) {
    load_rows_u<T, 1, KR>(f1, factor_of<T>(a.L1, inst * ns), a.L1.ld, wr0, lane);
    load_rows_u<T, 1, KR>(f2, factor_of<T>(a.L2, inst * ns), a.L2.ld, wr0, lane);
    const int col = wc0 + li;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int s = s0 + j * SPW;
      if (s < ns) load_cols_u<T, 1, KC>(fp[j], factor_of<T>(a.P, inst * ns + s), a.P.ld, wc0, lane);
      double cp = 0.0;
#pragma unroll
      for (int q = 0; q < NSR; ++q)
        if (q == s) cp = cphi[q];
      const double fc = cp * (a.ph.pn ? a.ph.pn[min(col, na - 1)] : 1.0);
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const int row = wr0 + M16<T>::row(g, q4);
        const double fr = a.ph.pm ? a.ph.pm[min(row, nm - 1)] : 1.0;
        ph[j][q4] = (s < ns && row < nm && col < na) ? M16<T>::phi1(static_cast<T>(fc * fr)) : T(0);
      }
    }
  }
  __syncthreads();

  for (int step = 0; step < r.steps; ++step) {
    // a. F = d M W + g(W), every species
    for (int e = tid; e < nm * na; e += NT) {
      int c;
      const int k = dna.quot(e, c);
      const int km = k > 0 ? k - 1 : (per_r ? nm - 1 : k);
      const int kp = k + 1 < nm ? k + 1 : (per_r ? 0 : k);
      const int cm = c > 0 ? c - 1 : (per_c ? na - 1 : c);
      const int cp = c + 1 < na ? c + 1 : (per_c ? 0 : c);
      const double* r5 = rc + k * 5;
      const double* c4 = cc + c * 4;
      double wv[3] = {0.0, 0.0, 0.0}, G[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < NSR; ++s)
        if (s < ns) wv[s] = static_cast<double>(sW[s * tile + k * ld + c]);
      if (react) reaction3c(rcst, wv[0], wv[1], wv[2], G[0], G[1], G[2]);
#pragma unroll
      for (int s = 0; s < NSR; ++s) {
        if (s >= ns) break;
        const T* w = sW + s * tile;
        const double w0 = wv[s];
        double f = c4[3] * (r5[2] * static_cast<double>(w[km * ld + c]) + r5[3] * w0 +
                            r5[4] * static_cast<double>(w[kp * ld + c]));
        f += r5[0] * (c4[0] * static_cast<double>(w[k * ld + cm]) + c4[1] * w0 +
                      c4[2] * static_cast<double>(w[k * ld + cp]));
        sF[s * tile + k * ld + c] = static_cast<T>(dif[s] * f + G[s]);
      }
    }
    __syncthreads();
    if constexpr (KR > 0) {
      const int col = wc0 + li;
      // b. sT = Phi o (V^-1 F)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int s = s0 + j * SPW;
        if (s >= ns) break;
        acc_t acc[1][1];
        zero<T, 1, 1>(acc);
        mma_rows_sB<T, 1, 1, KR>(acc, f1, sF + s * tile, ld, wc0, lane);
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
          sT[s * tile + (wr0 + M16<T>::row(g, q4)) * ld + col] = acc[0][0][q4] * ph[j][q4];
      }
      __syncthreads();
      // c. sF = V sT
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int s = s0 + j * SPW;
        if (s >= ns) break;
        acc_t acc[1][1];
        zero<T, 1, 1>(acc);
        mma_rows_sB<T, 1, 1, KR>(acc, f2, sT + s * tile, ld, wc0, lane);
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int row = wr0 + M16<T>::row(g, q4);
          sF[s * tile + row * ld + col] = (row < nm && col < na) ? acc[0][0][q4] : T(0);
        }
      }
      __syncthreads();
      // d. sW += alpha (sF x_1 P)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int s = s0 + j * SPW;
        if (s >= ns) break;
        acc_t acc[1][1];
        zero<T, 1, 1>(acc);
        mma_sA_cols<T, 1, 1, KC>(acc, sF + s * tile, ld, wr0, fp[j], lane);
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int row = wr0 + M16<T>::row(g, q4);
          if (row < nm && col < na) {
            T* w = sW + s * tile + row * ld + col;
            *w = *w + alpha * acc[0][0][q4];
          }
        }
      }
      __syncthreads();
      continue;
    }
    // b. sT = Phi o (V^-1 F)
    for (int sub = wave; sub < nsub; sub += NW) {
      const int s = sub / nsub1, q = sub - s * nsub1;
      const int r0 = (q / nct) * 16, c0 = (q % nct) * 16, col = c0 + li;
      acc_t acc[1][1];
      zero<T, 1, 1>(acc);
      gemm_gA_sB<T, 1, 1>(acc, factor_of<T>(a.L1, inst * ns + s), a.L1.ld, r0, sF + s * tile, ld, c0, NP, lane);
      const double fc = cphi[s] * (a.ph.pn ? a.ph.pn[min(col, na - 1)] : 1.0);
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const int row = r0 + M16<T>::row(g, q4);
        const double fr = a.ph.pm ? a.ph.pm[min(row, nm - 1)] : 1.0;
        const T v = acc[0][0][q4] * M16<T>::phi1(static_cast<T>(fc * fr));
        sT[s * tile + row * ld + col] = (row < nm && col < na) ? v : T(0);
      }
    }
    __syncthreads();
    // c. sF = V sT
    for (int sub = wave; sub < nsub; sub += NW) {
      const int s = sub / nsub1, q = sub - s * nsub1;
      const int r0 = (q / nct) * 16, c0 = (q % nct) * 16, col = c0 + li;
      acc_t acc[1][1];
      zero<T, 1, 1>(acc);
      gemm_gA_sB<T, 1, 1>(acc, factor_of<T>(a.L2, inst * ns + s), a.L2.ld, r0, sT + s * tile, ld, c0, NP, lane);
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const int row = r0 + M16<T>::row(g, q4);
        sF[s * tile + row * ld + col] = (row < nm && col < na) ? acc[0][0][q4] : T(0);
      }
    }
    __syncthreads();
    // d. sW += alpha (sF x_1 P)
    for (int sub = wave; sub < nsub; sub += NW) {
      const int s = sub / nsub1, q = sub - s * nsub1;
      const int r0 = (q / nct) * 16, c0 = (q % nct) * 16, col = c0 + li;
      acc_t acc[1][1];
      zero<T, 1, 1>(acc);
      gemm_sA_gB<T, 1, 1>(acc, sF + s * tile, ld, r0, factor_of<T>(a.P, inst * ns + s), a.P.ld, c0, TN, lane);
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const int row = r0 + M16<T>::row(g, q4);
        if (row < nm && col < na) {
          T* w = sW + s * tile + row * ld + col;
          *w = *w + alpha * acc[0][0][q4];
        }
      }
    }
    __syncthreads();
  }

  // 2. the state back
  bool bad = false;
  for (int s = 0; s < ns; ++s)
    for (int e = tid; e < nm * na; e += NT) {
      int c;
      const int k = dna.quot(e, c);
      const T v = sW[s * tile + k * ld + c];
      Wg[s * plane + e] = v;
      bad |= !isfinite(v);
    }
  if (bad && a.flag) atomicOr(a.flag, 1);
}

// Padded rows and columns of the resident tiles: 64 x 32 (the register-
// resident form) for grids up to that size, else nm and na rounded up to 16.
int resident_np(int nm, int na) { return nm <= 64 && na <= 32 ? 64 : round_up(nm, 16); }
int resident_tn(int nm, int na) { return nm <= 64 && na <= 32 ? 32 : round_up(na, 16); }

// Waves of the register-resident form: FP32, 16 (one per position and
// species; measured 5.9 against 6.7 us per step on the 32 x 64 disk); FP64,
// 8 (one per position, both species: at 16 waves the 128-register budget
// spills and a step takes 10.4 against 9.5 us).
template <typename T>
constexpr int resident_reg_waves() { return sizeof(T) == 4 ? 16 : 8; }

template <typename T>
size_t resident_lds_bytes(int ns, int nm, int na) {
  if (ns < 1 || ns > 3 || nm < 1 || na < 1) return 0;
  const int NP = resident_np(nm, na), TN = resident_tn(nm, na);
  return static_cast<size_t>(3 * ns) * NP * pitch_kmajor<T>(TN) * sizeof(T) + sizeof(double) * (5 * NP + 4 * TN);
}

template <typename T>
hipError_t launch_resident(const ResidentArgs& r, hipStream_t s) {
  const StridedArgs& a = r.a;
  const int ns = a.st.nspecies;
  if (!a.stencil || !a.sandwich || !a.phi || !a.plane || !a.update || a.nb != 1 || a.st.ndim != 2)
    return hipErrorInvalidValue;
  if (ns < 1 || ns > 3 || r.ninst < 1 || r.ninst > 65535 || a.nslab != ns * r.ninst || r.steps < 1)
    return hipErrorInvalidValue;
  if (a.nm != a.st.n[1] || a.na != a.st.n[0] || a.W != a.st.W || !a.W) return hipErrorInvalidValue;
  if (r.np != resident_np(a.nm, a.na) || r.tn != resident_tn(a.nm, a.na)) return hipErrorInvalidValue;
  if (a.L1.ld < r.np || a.L2.ld < r.np || a.P.ld < r.tn) return hipErrorInvalidValue;
  const size_t lds = resident_lds_bytes<T>(ns, a.nm, a.na);
  if (lds == 0 || lds > kMaxLds) return hipErrorInvalidValue;
  // the register-resident form for 64 x 32 padded tiles (8 waves) and up
  // to two species, the general one otherwise
  const bool reg = r.np == 64 && r.tn == 32 && a.L1.fmod == 1 && a.L2.fmod == 1 && ns <= 2;
  constexpr int RW = resident_reg_waves<T>();
  auto k = reg ? resident_kernel<T, RW, 4, 2> : resident_kernel<T, 8, 0, 0>;
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(r.ninst), dim3(reg ? 64 * RW : 512), lds, s, r);
  return hipGetLastError();
}

template hipError_t plan_strided_group<double>(StridedGroup&, GroupLaunch&);
template hipError_t plan_strided_group<float>(StridedGroup&, GroupLaunch&);
template hipError_t plan_first_group<double>(FirstGroup&, GroupLaunch&);
template hipError_t plan_first_group<float>(FirstGroup&, GroupLaunch&);
template hipError_t launch_strided_group<double>(const GroupLaunch&, const StridedGroup*, hipStream_t);
template hipError_t launch_strided_group<float>(const GroupLaunch&, const StridedGroup*, hipStream_t);
template hipError_t launch_first_group<double>(const GroupLaunch&, const FirstGroup*, hipStream_t);
template hipError_t launch_first_group<float>(const GroupLaunch&, const FirstGroup*, hipStream_t);

template hipError_t launch_strided<double>(const StridedArgs&, hipStream_t);
template hipError_t launch_strided<float>(const StridedArgs&, hipStream_t);
template hipError_t launch_first<double>(const FirstArgs&, hipStream_t);
template hipError_t launch_first<float>(const FirstArgs&, hipStream_t);
template size_t strided_lds_bytes<double>(int, int, int, int, int);
template size_t strided_lds_bytes<float>(int, int, int, int, int);
template size_t first_lds_bytes<double>(int, int, int);
template size_t first_lds_bytes<float>(int, int, int);
template hipError_t launch_resident<double>(const ResidentArgs&, hipStream_t);
template hipError_t launch_resident<float>(const ResidentArgs&, hipStream_t);
template size_t resident_lds_bytes<double>(int, int, int);
template size_t resident_lds_bytes<float>(int, int, int);

}  // namespace tg
