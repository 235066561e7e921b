// Split-bf16 variants of the fused mu-mode product kernels (FP32 state,
// FP32 accumulation).  Every operand x is carried as NT bf16 terms,
// x ~ t0 + t1 (+ t2) with t_i = bf16(x - t_0 - ... - t_{i-1}), and a product
// keeps the term pairs (i, j) with i + j < NT:
//   NT = 2: t0 s0 + t0 s1 + t1 s0           (3 MFMAs, ~2^-16 relative)
//   NT = 3: adds t0 s2 + t1 s1 + t2 s0      (6 MFMAs, ~2^-24 relative)
// Factors are split on the host; data tiles are split once when they enter
// LDS, stored k-contiguous so that each MFMA operand (8 consecutive k) is a
// single 16-byte read.  MFMA: v_mfma_f32_16x16x32_bf16, operand A(i, k) in
// lane i + 16 (k / 8) element k % 8, B(k, j) in lane j + 16 (k / 8) element
// k % 8, accumulator element r of lane l is D(4 (l / 16) + r, l % 16)
// (checked on gfx950 with a one-wave probe).
#include <algorithm>

#include "fused.hpp"
#include "diag_dev.hpp"
#include "phi_dev.hpp"
#include "stencil_dev.hpp"

namespace tg {

typedef float fx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ fx4 mfma_bf16(bx8 a, bx8 b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int NT>
__device__ __forceinline__ void split_terms(float x, __bf16 (&t)[NT]) {
  float r = x;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    t[i] = static_cast<__bf16>(r);
    r -= static_cast<float>(t[i]);
  }
}

__device__ __forceinline__ float phi1f(float x) { return phi1_f32(x); }

// LDS pitch (bf16 elements) of a k-contiguous row of NP values: the byte
// stride 2 NP + 16 puts 8 consecutive rows on distinct 16-byte bank groups.
__host__ __device__ constexpr int pitch_k(int np) { return np + 8; }

// acc[f][j] += sum_k A(r0 + 16 f + li, k) B(k, c0 + 16 j + li) over the
// term pairs i + j < NT.  A: rows of a split factor in global memory
// (term t at A + t * tstride, leading dimension lda).  B: LDS tile, term t
// at sB + t * bstride, column c stored k-contiguous at c * ldb.
template <int NT, int FM, int FN, int KB>
__device__ __forceinline__ void gemm_fac_lds(fx4 (&acc)[FM][FN], const __bf16* __restrict__ A, int64_t tstride,
                                             int lda, int r0, const __bf16* sB, int bstride, int ldb, int c0,
                                             int kblocks, int lane) {
  const int li = lane & 15, g = lane >> 4;
  const int nkb = KB > 0 ? KB : kblocks;
#pragma unroll
  for (int kb = 0; kb < (KB > 0 ? KB : 1); ++kb) {
    for (int kk = (KB > 0 ? kb : 0); kk < (KB > 0 ? kb + 1 : nkb); ++kk) {
      const int k0 = 32 * kk + 8 * g;
      bx8 a[FM][NT], b[FN][NT];
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          a[f][t] = *reinterpret_cast<const bx8*>(A + t * tstride + static_cast<int64_t>(r0 + 16 * f + li) * lda + k0);
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          b[j][t] = *reinterpret_cast<const bx8*>(sB + t * bstride + (c0 + 16 * j + li) * ldb + k0);
#pragma unroll
      for (int ta = 0; ta < NT; ++ta)
#pragma unroll
        for (int tb = 0; tb < NT - ta; ++tb)
#pragma unroll
          for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[f][j] = mfma_bf16(a[f][ta], b[j][tb], acc[f][j]);
    }
  }
}

// acc[f][j] += sum_k sA(r0 + 16 f + li, k) B(c0 + 16 j + li, k): A from an
// LDS tile (rows k-contiguous), B = rows of a split factor (output columns).
template <int NT, int FM, int FN, int KB>
__device__ __forceinline__ void gemm_lds_fac(fx4 (&acc)[FM][FN], const __bf16* sA, int astride, int lda, int r0,
                                             const __bf16* __restrict__ B, int64_t tstride, int ldb, int c0,
                                             int kblocks, int lane) {
  const int li = lane & 15, g = lane >> 4;
  const int nkb = KB > 0 ? KB : kblocks;
#pragma unroll
  for (int kb = 0; kb < (KB > 0 ? KB : 1); ++kb) {
    for (int kk = (KB > 0 ? kb : 0); kk < (KB > 0 ? kb + 1 : nkb); ++kk) {
      const int k0 = 32 * kk + 8 * g;
      bx8 a[FM][NT], b[FN][NT];
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          b[j][t] = *reinterpret_cast<const bx8*>(B + t * tstride + static_cast<int64_t>(c0 + 16 * j + li) * ldb + k0);
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          a[f][t] = *reinterpret_cast<const bx8*>(sA + t * astride + (r0 + 16 * f + li) * lda + k0);
#pragma unroll
      for (int ta = 0; ta < NT; ++ta)
#pragma unroll
        for (int tb = 0; tb < NT - ta; ++tb)
#pragma unroll
          for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[f][j] = mfma_bf16(a[f][ta], b[j][tb], acc[f][j]);
    }
  }
}

template <int FM, int FN>
__device__ __forceinline__ void zero_acc(fx4 (&acc)[FM][FN]) {
#pragma unroll
  for (int f = 0; f < FM; ++f)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[f][j] = fx4{0, 0, 0, 0};
}

__device__ __forceinline__ const __bf16* bf_factor(const Factor& F, int s) {
  return static_cast<const __bf16*>(F.L) + static_cast<int64_t>(s % F.fmod) * F.fstride;
}

// Stores NT split terms of 4 values that are consecutive along k of LDS
// column `col` starting at k = k0 (8-byte stores).
template <int NT>
__device__ __forceinline__ void put4_kcontig(__bf16* s, int stride, int ld, int col, int k0, const float (&v)[4]) {
  __bf16 t[4][NT];
#pragma unroll
  for (int r = 0; r < 4; ++r) split_terms<NT>(v[r], t[r]);
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    bx4 w = {t[0][q], t[1][q], t[2][q], t[3][q]};
    *reinterpret_cast<bx4*>(s + q * stride + col * ld + k0) = w;
  }
}

template <int NT>
__device__ __forceinline__ void put1(__bf16* s, int stride, int off, float v) {
  __bf16 t[NT];
  split_terms<NT>(v, t);
#pragma unroll
  for (int q = 0; q < NT; ++q) s[q * stride + off] = t[q];
}

// ---------------------------------------------------------------------------
// Strided mode (mu >= 2): data tile column c (k-contiguous) of NT terms.
template <int NT, int FM, int FN, int KB, int NW>
__global__ __launch_bounds__(64 * NW) void strided_bf16_kernel(StridedArgs a) {
  extern __shared__ __align__(256) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int nm = a.nm, na = a.na, TN = a.tn;
  const int NP = KB > 0 ? 32 * KB : (nm + 63) / 64 * 64;
  const int ldk = pitch_k(NP);
  const int tstr = TN * ldk;                 // one term of one tile
  // plane tail operand: NP rows (i contiguous) per term, in the data
  // tile's space once the first product has consumed it
  const int ldr = pitch_k((na + 31) / 32 * 32);
  const int rstr = NP * ldr;
  const int xsz = a.plane ? max(NT * tstr, NT * rstr) : NT * tstr;
  __bf16* sX = reinterpret_cast<__bf16*>(smem);
  __bf16* sT = sX + xsz;
  // 1D grid of 8 * per_xcd workgroups, dispatched round-robin over the 8
  // XCDs: XCD x takes logical tiles x * per_xcd .. (x + 1) * per_xcd, in
  // the order species, column tile, row block, instance, so that a tile's
  // stencil neighbours and its other species share an XCD's L2
  const int nbx = (na + TN - 1) / TN;
  const int total = nbx * a.nb * a.nslab;
  const int per_xcd = (total + 7) / 8;
  const int L = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (L >= total) return;
  const int nsp = a.stencil ? a.st.nspecies : 1;
  int rest = L / nsp;
  const int bx = rest % nbx;
  rest /= nbx;
  const int a0 = bx * TN, b = rest % a.nb, s = (rest / a.nb) * nsp + L % nsp;
  const int64_t slab = static_cast<int64_t>(nm) * na * a.nb;
  const int64_t base = static_cast<int64_t>(s) * slab + static_cast<int64_t>(b) * nm * na;

  // 1. data tile (k < NP rows, zero beyond nm), split into terms
  if (a.stencil) {
    const int inst = s / a.st.nspecies, sp = s % a.st.nspecies;
    const int n1 = a.st.n[0];
    const bool three = a.st.ndim == 3;
    // four points per thread in flight (their loads overlap)
#pragma unroll 4
    for (int e = tid; e < NP * TN; e += 64 * NW) {
      const int k = e / TN, c = e % TN;
      const int aa = a0 + c;
      float v = 0.0f;
      if (k < nm && aa < na) {
        const int i = three ? aa % n1 : aa;
        const int j = three ? aa / n1 : k;
        const int kk = three ? k : 0;
        v = static_cast<float>(stencil_point_ijk<float>(a.st, inst, sp, k * na + aa, i, j, kk));
      }
      put1<NT>(sX, tstr, c * ldk + k, v);
    }
  } else {
    const float* X = static_cast<const float*>(a.X) + base;
    for (int e = tid; e < NP * TN; e += 64 * NW) {
      const int k = e / TN, c = e % TN;
      const float v = (k < nm && a0 + c < na) ? X[static_cast<int64_t>(k) * na + a0 + c] : 0.0f;
      put1<NT>(sX, tstr, c * ldk + k, v);
    }
  }
  __syncthreads();

  const int nrt = NP / (16 * FM), nct = TN / (16 * FN);
  const int nsub = nrt * nct;
  const bool keep = a.sandwich || a.plane;
  const __bf16* L1 = bf_factor(a.L1, s);
  const int64_t t1 = static_cast<int64_t>(a.L1.ld) * a.L1.ld;
  float* Y = static_cast<float*>(a.Y) + base;
  const double cb = a.phi ? a.ph.cs[s] * (a.ph.pb ? a.ph.pb[b] : 1.0) : 0.0;
  const int kblocks = NP / 32;

  // 2. first product and the phi_1 factor
  for (int sub = wave; sub < nsub; sub += NW) {
    const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
    float ph[FM][FN][4];
    if (a.phi) {
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = min(r0 + 16 * f + 4 * g + r, nm - 1), col = min(a0 + c0 + 16 * j + li, na - 1);
            double x = cb;
            if (a.ph.pm) x *= a.ph.pm[row];
            if (a.ph.pn) x *= a.ph.pn[col];
            ph[f][j][r] = phi1f(static_cast<float>(x));
          }
    }
    fx4 acc[FM][FN];
    zero_acc<FM, FN>(acc);
    gemm_fac_lds<NT, FM, FN, KB>(acc, L1, t1, a.L1.ld, r0, sX, tstr, ldk, c0, kblocks, lane);
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int col = c0 + 16 * j + li;
        const int rb = r0 + 16 * f + 4 * g;
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const bool in = rb + r < nm && a0 + col < na;
          v[r] = acc[f][j][r] * (a.phi ? ph[f][j][r] : 1.0f);
          if (!in) v[r] = 0.0f;
          if (!keep && in) Y[static_cast<int64_t>(rb + r) * na + a0 + col] = v[r];
        }
        if (keep) put4_kcontig<NT>(sT, tstr, ldk, col, rb, v);
      }
  }
  if (!keep) return;
  __syncthreads();

  // 3. second product of the sandwich; for the plane tail the result goes
  //    to LDS rows (row-major, i contiguous) for the mode-1 product
  if (a.sandwich) {
    const __bf16* L2 = bf_factor(a.L2, s);
    const int64_t t2 = static_cast<int64_t>(a.L2.ld) * a.L2.ld;
    for (int sub = wave; sub < nsub; sub += NW) {
      const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
      fx4 acc[FM][FN];
      zero_acc<FM, FN>(acc);
      gemm_fac_lds<NT, FM, FN, KB>(acc, L2, t2, a.L2.ld, r0, sT, tstr, ldk, c0, kblocks, lane);
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + 16 * f + 4 * g + r, col = c0 + 16 * j + li;
            const bool in = row < nm && a0 + col < na;
            const float v = in ? acc[f][j][r] : 0.0f;
            if (a.plane) put1<NT>(sX, rstr, row * ldr + col, v);
            else if (in) Y[static_cast<int64_t>(row) * na + a0 + col] = v;
          }
    }
    if (!a.plane) return;
    __syncthreads();
  }

  // 4. plane tail: Z[row][i'] = sum_i T[row][i] P[i'][i];  W += alpha Z
  //    (a plane launch always has a sandwich, so T is in sX as rows)
  const __bf16* P = bf_factor(a.P, s);
  const int64_t tp = static_cast<int64_t>(a.P.ld) * a.P.ld;
  float* W = static_cast<float*>(a.W) + base;
  const int kbt = (na + 31) / 32;
  const float alpha = static_cast<float>(a.alpha);
  const bool diag = a.dg.part != nullptr;
  double ds0 = 0.0, ds1 = 0.0;
  for (int sub = wave; sub < nsub; sub += NW) {
    const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
    float wv[FM][FN][4];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(r0 + 16 * f + 4 * g + r, nm - 1), col = min(c0 + 16 * j + li, na - 1);
          wv[f][j][r] = a.update ? W[static_cast<int64_t>(row) * na + col] : 0.0f;
        }
    fx4 acc[FM][FN];
    zero_acc<FM, FN>(acc);
    gemm_lds_fac<NT, FM, FN, 0>(acc, sX, rstr, ldr, r0, P, tp, a.P.ld, c0, kbt, lane);
    bool bad = false;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + 16 * f + 4 * g + r, col = c0 + 16 * j + li;
          const float nv = a.update ? wv[f][j][r] + alpha * acc[f][j][r] : acc[f][j][r];
          if (row < nm && col < na) {
            W[static_cast<int64_t>(row) * na + col] = nv;
            bad |= !isfinite(nv);
            if (diag) diag_point(a.dg, b * nm + row, col, nv, wv[f][j][r], ds0, ds1);
          }
        }
    if (bad && a.flag) atomicOr(a.flag, 1);
  }
  if (diag)
    diag_flush<NW>(a.dg, ds0, ds1, static_cast<int64_t>(s) * a.dg.tiles + static_cast<int64_t>(b) * nbx + bx,
                  reinterpret_cast<double*>(smem));
}

// ---------------------------------------------------------------------------
// Strided mode, multi-tile form for launches without an in-tile stencil or
// plane tail (the same products, the same rounding as strided_bf16_kernel).
// A tile of one of these launches is a few microseconds of latency and a
// fraction of a microsecond of MFMA work, so here a workgroup walks a run of
// consecutive tiles (row block b fastest, then the column tile, then the
// slab): the next tile's values are loaded into registers while the current
// one is multiplied, the factor rows a wave multiplies stay in registers
// while the slab does not change, and so do the phi_1 factors while the
// column tile does not (unless they depend on b).  Wave w owns rows
// 16 w .. 16 w + 15 of every product and all TN = 16 FN columns; a thread
// loads EPT = 4 FN consecutive rows of one column and stores their terms
// with one LDS write per term.  The data tile is double-buffered (one
// barrier per tile for a single product, two for a sandwich).
template <int NT, int KB, int FN, int SW>
__global__ __launch_bounds__(128 * KB) void strided_bf16_mt_kernel(StridedArgs a) {
  constexpr int NP = 32 * KB, TN = 16 * FN, EPT = 4 * FN;  // 2 KB waves
  constexpr int LDK = NP + 8, TSTR = TN * LDK;
  extern __shared__ __align__(256) unsigned char smem[];
  __bf16* const sX = reinterpret_cast<__bf16*>(smem);  // two buffers of NT terms
  __bf16* const sT = sX + 2 * NT * TSTR;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int nm = a.nm, na = a.na, nb = a.nb;
  const int nbx = (na + TN - 1) / TN;
  const int per_slab = nbx * nb;
  const int64_t total = static_cast<int64_t>(per_slab) * a.nslab;
  // logical workgroup w = XCD-major (blockIdx round-robins over 8 XCDs), so
  // the runs of one XCD are adjacent tiles; run w = [total w / G, total (w+1) / G)
  const int G = gridDim.x, per_xcd = G / 8;
  const int w = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  const int lo = static_cast<int>(total * w / G), hi = static_cast<int>(total * (w + 1) / G);
  if (lo >= hi) return;
  const int lc = tid % TN, lk = (tid / TN) * EPT;  // this thread's loads
  const int r0 = 16 * wave;                          // this wave's rows
  const float* X = static_cast<const float*>(a.X);
  float* Y = static_cast<float*>(a.Y);
  const int64_t slab = static_cast<int64_t>(nm) * na * nb;

  float pre[EPT];
  auto fetch = [&](int L) {
    const int s = L / per_slab, rest = L % per_slab, b = rest % nb, a0 = (rest / nb) * TN;
    const float* x = X + s * slab + static_cast<int64_t>(b) * nm * na + a0 + lc;
    const bool col = a0 + lc < na;
#pragma unroll
    for (int i = 0; i < EPT; ++i) pre[i] = (col && lk + i < nm) ? x[static_cast<int64_t>(lk + i) * na] : 0.0f;
  };
  fetch(lo);

  bx8 f1[KB][NT], f2[SW ? KB : 1][NT];
  double pmr[4];
  float ph[FN][4];
  int scur = -1, phs = -1, pha = -1;
  double csl = 0.0;
  int buf = 0;
  for (int L = lo; L < hi; ++L, buf ^= 1) {
    const int s = L / per_slab, rest = L % per_slab, b = rest % nb, a0 = (rest / nb) * TN;
    __bf16* const sb = sX + buf * NT * TSTR;
    {  // the prefetched rows lk .. lk + EPT - 1 of column lc, one write per term
      __bf16 t[EPT][NT];
#pragma unroll
      for (int i = 0; i < EPT; ++i) split_terms<NT>(pre[i], t[i]);
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        if constexpr (EPT == 4) {
          bx4 v = {t[0][q], t[1][q], t[2][q], t[3][q]};
          *reinterpret_cast<bx4*>(sb + q * TSTR + lc * LDK + lk) = v;
        } else {
          bx8 v = {t[0][q], t[1][q], t[2][q], t[3][q], t[4][q], t[5][q], t[6][q], t[7][q]};
          *reinterpret_cast<bx8*>(sb + q * TSTR + lc * LDK + lk) = v;
        }
      }
    }
    if (L + 1 < hi) fetch(L + 1);
    if (s != scur) {  // this slab's factor rows r0 + li, k = 32 kb + 8 g .. + 7
      scur = s;
      const __bf16* A1 = bf_factor(a.L1, s);
      const int64_t t1 = static_cast<int64_t>(a.L1.ld) * a.L1.ld;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          f1[kb][t] = *reinterpret_cast<const bx8*>(A1 + t * t1 + static_cast<int64_t>(r0 + li) * a.L1.ld + 32 * kb + 8 * g);
      if constexpr (SW) {
        const __bf16* A2 = bf_factor(a.L2, s);
        const int64_t t2 = static_cast<int64_t>(a.L2.ld) * a.L2.ld;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            f2[kb][t] =
                *reinterpret_cast<const bx8*>(A2 + t * t2 + static_cast<int64_t>(r0 + li) * a.L2.ld + 32 * kb + 8 * g);
      }
      if (a.phi) {
        csl = a.ph.cs[s];
#pragma unroll
        for (int r = 0; r < 4; ++r) pmr[r] = a.ph.pm ? a.ph.pm[min(r0 + 4 * g + r, nm - 1)] : 1.0;
      }
    }
    // phi_1 factors: the same for every row block b unless pb scales them
    if (a.phi && (s != phs || a0 != pha || a.ph.pb)) {
      phs = s;
      pha = a0;
      const double cb = csl * (a.ph.pb ? a.ph.pb[b] : 1.0);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const double pn = a.ph.pn ? a.ph.pn[min(a0 + 16 * j + li, na - 1)] : 1.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double x = cb;
          if (a.ph.pm) x *= pmr[r];
          if (a.ph.pn) x *= pn;
          ph[j][r] = phi1f(static_cast<float>(x));
        }
      }
    }
    __syncthreads();

    fx4 acc[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[j] = fx4{0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      bx8 v[FN][NT];
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          v[j][t] = *reinterpret_cast<const bx8*>(sb + t * TSTR + (16 * j + li) * LDK + 32 * kb + 8 * g);
#pragma unroll
      for (int ta = 0; ta < NT; ++ta)
#pragma unroll
        for (int tb = 0; tb < NT - ta; ++tb)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[j] = mfma_bf16(f1[kb][ta], v[j][tb], acc[j]);
    }
    float* const y = Y + s * slab + static_cast<int64_t>(b) * nm * na + a0;
    const int rb = r0 + 4 * g;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = 16 * j + li;
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool in = rb + r < nm && a0 + col < na;
        v[r] = acc[j][r] * (a.phi ? ph[j][r] : 1.0f);
        if (!in) v[r] = 0.0f;
        if (!SW && in) y[static_cast<int64_t>(rb + r) * na + col] = v[r];
      }
      if (SW) put4_kcontig<NT>(sT, TSTR, LDK, col, rb, v);
    }
    if constexpr (SW) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[j] = fx4{0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        bx8 v[FN][NT];
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            v[j][t] = *reinterpret_cast<const bx8*>(sT + t * TSTR + (16 * j + li) * LDK + 32 * kb + 8 * g);
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
          for (int tb = 0; tb < NT - ta; ++tb)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[j] = mfma_bf16(f2[kb][ta], v[j][tb], acc[j]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * j + li;
          if (rb + r < nm && a0 + col < na) y[static_cast<int64_t>(rb + r) * na + col] = acc[j][r];
        }
    }
  }
}

// ---------------------------------------------------------------------------
// First mode: data tile rows (k-contiguous) of NT terms.
template <int NT, int FM, int FN, int KB>
__global__ __launch_bounds__(256) void first_bf16_kernel(FirstArgs a) {
  extern __shared__ __align__(256) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int nm = a.nm, TM = a.tm;
  const int NP = KB > 0 ? 32 * KB : (nm + 31) / 32 * 32;
  const int ldk = pitch_k(NP);
  const int tstr = TM * ldk;
  __bf16* sX = reinterpret_cast<__bf16*>(smem);
  __bf16* sT = sX + NT * tstr;
  const int rt0 = blockIdx.x * TM, s = blockIdx.y;
  const int64_t base = static_cast<int64_t>(s) * a.rows * nm;
  const float* X = static_cast<const float*>(a.X) + base;
  for (int e = tid; e < TM * NP; e += 256) {
    const int r = e / NP, c = e % NP;
    const float v = (c < nm && rt0 + r < a.rows) ? X[static_cast<int64_t>(rt0 + r) * nm + c] : 0.0f;
    put1<NT>(sX, tstr, r * ldk + c, v);
  }
  __syncthreads();

  const int nrt = TM / (16 * FM), nct = NP / (16 * FN);
  const int nsub = nrt * nct;
  float* Y = static_cast<float*>(a.Y) + base;
  const float alpha = static_cast<float>(a.alpha);
  const int kblocks = NP / 32;
  const bool diag = a.dg.part != nullptr;
  double ds0 = 0.0, ds1 = 0.0;
  auto finish = [&](int r0, int c0, const fx4 (&acc)[FM][FN]) {
    bool bad = false;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rg = rt0 + r0 + 16 * f + 4 * g + r, col = c0 + 16 * j + li;
          if (rg < a.rows && col < nm) {
            float* dst = Y + static_cast<int64_t>(rg) * nm + col;
            const float ov = a.update ? *dst : 0.0f;
            const float nv = a.update ? ov + alpha * acc[f][j][r] : acc[f][j][r];
            *dst = nv;
            bad |= !isfinite(nv);
            if (diag) diag_point(a.dg, rg, col, nv, ov, ds0, ds1);
          }
        }
    if (bad && a.update && a.flag) atomicOr(a.flag, 1);
  };
  auto flush = [&]() {
    if (diag)
      diag_flush<4>(a.dg, ds0, ds1, static_cast<int64_t>(s) * a.dg.tiles + blockIdx.x,
                    reinterpret_cast<double*>(smem));
  };
  const __bf16* L1 = bf_factor(a.L1, s);
  const int64_t t1 = static_cast<int64_t>(a.L1.ld) * a.L1.ld;
  const double cs = a.sandwich ? a.ph.cs[s] : 0.0;
  for (int sub = wave; sub < nsub; sub += 4) {
    const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
    float ph[FM][FN][4];
    if (a.sandwich) {
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rg = min(rt0 + r0 + 16 * f + 4 * g + r, a.rows - 1), col = min(c0 + 16 * j + li, nm - 1);
            double x = cs;
            if (a.ph.pm) x *= a.ph.pm[rg];
            if (a.ph.pn) x *= a.ph.pn[col];
            ph[f][j][r] = phi1f(static_cast<float>(x));
          }
    }
    fx4 acc[FM][FN];
    zero_acc<FM, FN>(acc);
    gemm_lds_fac<NT, FM, FN, KB>(acc, sX, tstr, ldk, r0, L1, t1, a.L1.ld, c0, kblocks, lane);
    if (!a.sandwich) {
      finish(r0, c0, acc);
      continue;
    }
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + 16 * f + 4 * g + r, col = c0 + 16 * j + li;
          const bool in = col < nm && rt0 + row < a.rows;
          put1<NT>(sT, tstr, row * ldk + col, in ? acc[f][j][r] * ph[f][j][r] : 0.0f);
        }
  }
  if (!a.sandwich) {
    flush();
    return;
  }
  __syncthreads();
  const __bf16* L2 = bf_factor(a.L2, s);
  const int64_t t2 = static_cast<int64_t>(a.L2.ld) * a.L2.ld;
  for (int sub = wave; sub < nsub; sub += 4) {
    const int r0 = (sub / nct) * 16 * FM, c0 = (sub % nct) * 16 * FN;
    fx4 acc[FM][FN];
    zero_acc<FM, FN>(acc);
    gemm_lds_fac<NT, FM, FN, KB>(acc, sT, tstr, ldk, r0, L2, t2, a.L2.ld, c0, kblocks, lane);
    finish(r0, c0, acc);
  }
  flush();
}

// Multi-tile form of the single first-mode product (no sandwich, no
// indicators), with or without the update: the same products and rounding
// as first_bf16_kernel.  A workgroup walks a run of consecutive row tiles,
// loading the next tile's rows and the state values of its update into
// registers while the current one is multiplied; each wave keeps the split
// factor rows of its 32 output columns in registers while the slab is
// unchanged.  TM = 16 FM rows, NP = 32 KB columns, KB waves.
template <int NT, int KB, int FM>
__global__ __launch_bounds__(64 * KB) void first_bf16_mt_kernel(FirstArgs a) {
  constexpr int FN = 2, NW = KB, NTH = 64 * NW, NP = 32 * KB, TM = 16 * FM, LDK = NP + 8, TSTR = TM * LDK;
  constexpr int VPT = TM * NP / 4 / NTH;  // 4-element groups per thread
  extern __shared__ __align__(256) unsigned char smem[];
  __bf16* const sX = reinterpret_cast<__bf16*>(smem);  // two buffers of NT terms
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
  const float* X = static_cast<const float*>(a.X);
  float* Y = static_cast<float*>(a.Y);
  const float alpha = static_cast<float>(a.alpha);
  const int64_t slab = static_cast<int64_t>(rows) * nm;

  fx4 pre[VPT];
  float yn[FM][FN][4];
  auto fetch = [&](int L) {
    const int s = L / nrt, rt0 = (L % nrt) * TM;
    const float* x = X + s * slab;
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int e = 4 * (tid + NTH * q), r = e / NP, c = e % NP;
      const int64_t off = static_cast<int64_t>(rt0 + r) * nm + c;
      const bool rin = rt0 + r < rows;
      if (vec) {
        pre[q] = (rin && c < nm) ? *reinterpret_cast<const fx4*>(x + off) : fx4{0, 0, 0, 0};
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) pre[q][u] = (rin && c + u < nm) ? x[off + u] : 0.0f;
      }
    }
    if (a.update) {
      const float* y = Y + s * slab;
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rg = min(rt0 + 16 * f + 4 * g + r, rows - 1);
            const int col = min(c0 + 16 * j + li, nm - 1);
            yn[f][j][r] = y[static_cast<int64_t>(rg) * nm + col];
          }
    }
  };
  fetch(lo);

  bx8 fb[KB][FN][NT];
  int scur = -1;
  int buf = 0;
  for (int L = lo; L < hi; ++L, buf ^= 1) {
    const int s = L / nrt, rt0 = (L % nrt) * TM;
    __bf16* const sb = sX + buf * NT * TSTR;
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int e = 4 * (tid + NTH * q), r = e / NP, c = e % NP;
      __bf16 t[4][NT];
#pragma unroll
      for (int u = 0; u < 4; ++u) split_terms<NT>(pre[q][u], t[u]);
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        bx4 v = {t[0][k], t[1][k], t[2][k], t[3][k]};
        *reinterpret_cast<bx4*>(sb + k * TSTR + r * LDK + c) = v;
      }
    }
    float yv[FM][FN][4];
    if (a.update) {
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) yv[f][j][r] = yn[f][j][r];
    }
    if (L + 1 < hi) fetch(L + 1);
    if (s != scur) {  // factor rows c0 + 16 j + li, k = 32 kb + 8 g .. + 7
      scur = s;
      const __bf16* B = bf_factor(a.L1, s);
      const int64_t t1 = static_cast<int64_t>(a.L1.ld) * a.L1.ld;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            fb[kb][j][t] = *reinterpret_cast<const bx8*>(B + t * t1 + static_cast<int64_t>(c0 + 16 * j + li) * a.L1.ld +
                                                         32 * kb + 8 * g);
    }
    __syncthreads();

    fx4 acc[FM][FN];
    zero_acc<FM, FN>(acc);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      bx8 av[FM][NT];
#pragma unroll
      for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          av[f][t] = *reinterpret_cast<const bx8*>(sb + t * TSTR + (16 * f + li) * LDK + 32 * kb + 8 * g);
#pragma unroll
      for (int ta = 0; ta < NT; ++ta)
#pragma unroll
        for (int tb = 0; tb < NT - ta; ++tb)
#pragma unroll
          for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[f][j] = mfma_bf16(av[f][ta], fb[kb][j][tb], acc[f][j]);
    }
    float* const y = Y + s * slab;
    bool bad = false;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rg = rt0 + 16 * f + 4 * g + r, col = c0 + 16 * j + li;
          const float nv = a.update ? yv[f][j][r] + alpha * acc[f][j][r] : acc[f][j][r];
          if (rg < rows && col < nm) {
            y[static_cast<int64_t>(rg) * nm + col] = nv;
            bad |= !isfinite(nv);
          }
        }
    if (bad && a.update && a.flag) atomicOr(a.flag, 1);
  }
}

// ---------------------------------------------------------------------------
static int bf_np_strided(int nm) { return nm <= 64 ? 64 : (nm <= 128 ? 128 : (nm + 63) / 64 * 64); }
static int bf_np_first(int nm) { return nm <= 64 ? 64 : (nm <= 128 ? 128 : (nm + 31) / 32 * 32); }
static int bf_kb(int nm) { return nm <= 64 ? 2 : (nm <= 128 ? 4 : 0); }

size_t strided_bf16_lds_bytes(int nterms, int nm, int na, int tn, int sandwich, int plane) {
  const int NP = bf_np_strided(nm);
  const size_t tile = static_cast<size_t>(nterms) * tn * pitch_k(NP);
  const size_t rows = plane ? static_cast<size_t>(nterms) * NP * pitch_k((na + 31) / 32 * 32) : 0;
  const size_t x = std::max(tile, rows);
  return 2 * ((sandwich || plane) ? x + tile : x);
}

size_t first_bf16_lds_bytes(int nterms, int nm, int tm, int sandwich) {
  const int NP = bf_np_first(nm);
  return static_cast<size_t>(sandwich ? 2 : 1) * nterms * tm * pitch_k(NP) * 2;
}

template <typename K>
static hipError_t bf_allow(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

template <int NT, int FM, int FN, int KB, int NW = 4>
static hipError_t go_sbf(const StridedArgs& a, size_t lds, hipStream_t s) {
  auto k = strided_bf16_kernel<NT, FM, FN, KB, NW>;
  hipError_t e = bf_allow(k, lds);
  if (e != hipSuccess) return e;
  const int64_t total = static_cast<int64_t>((a.na + a.tn - 1) / a.tn) * a.nb * a.nslab;
  if (total >= (int64_t(1) << 30)) return hipErrorInvalidValue;
  const int per_xcd = static_cast<int>((total + 7) / 8);
  hipLaunchKernelGGL(k, dim3(8 * per_xcd), dim3(64 * NW), lds, s, a);
  return hipGetLastError();
}

// Multi-tile launches: as many workgroups as fit on the device at once (at
// most one per tile), a multiple of 8 for the XCD-major run order.
template <int NT, int KB, int FN, int SW>
static hipError_t go_sbf_mt(const StridedArgs& a, hipStream_t s) {
  auto k = strided_bf16_mt_kernel<NT, KB, FN, SW>;
  constexpr int threads = 128 * KB;
  constexpr size_t lds = static_cast<size_t>(2 + SW) * NT * 16 * FN * pitch_k(32 * KB) * 2;
  hipError_t e = bf_allow(k, lds);
  if (e != hipSuccess) return e;
  const int fit = resident_workgroups(reinterpret_cast<const void*>(k), threads, lds);
  if (fit < 1) return hipErrorInvalidValue;
  const int64_t total = static_cast<int64_t>((a.na + 16 * FN - 1) / (16 * FN)) * a.nb * a.nslab;
  if (total >= (int64_t(1) << 30)) return hipErrorInvalidValue;
  const int grid = static_cast<int>((std::min<int64_t>(fit, total) + 7) / 8 * 8);
  hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <int NT, int KB>
static hipError_t sbf_mt(const StridedArgs& a, hipStream_t s) {
  if (a.tn == 16) return a.sandwich ? go_sbf_mt<NT, KB, 1, 1>(a, s) : go_sbf_mt<NT, KB, 1, 0>(a, s);
  return a.sandwich ? go_sbf_mt<NT, KB, 2, 1>(a, s) : go_sbf_mt<NT, KB, 2, 0>(a, s);
}

template <int NT>
static hipError_t sbf_dispatch(const StridedArgs& a, size_t lds, hipStream_t s) {
  const int kb = bf_kb(a.nm);
  if (!a.stencil && !a.plane && !a.dg.part && (a.tn == 16 || a.tn == 32) && kb > 0)
    return kb == 2 ? sbf_mt<NT, 2>(a, s) : sbf_mt<NT, 4>(a, s);
  const bool fn2 = a.tn % 32 == 0;
  // 8 waves where a tile has 8 or more 16-wide sub-tiles (more waves per
  // SIMD to overlap the latencies of the few workgroups of these launches)
  // (NP = 32 kb rows: kb tn / 16 sub-tiles of 32 x 16, twice as many of 16 x 16)
  const int c16 = a.tn / 16;
  if (kb > 0 && kb * c16 >= 8)
    return kb == 2 ? go_sbf<NT, 2, 1, 2, 8>(a, lds, s) : go_sbf<NT, 2, 1, 4, 8>(a, lds, s);
  if (kb > 0 && 2 * kb * c16 >= 8)
    return kb == 2 ? go_sbf<NT, 1, 1, 2, 8>(a, lds, s) : go_sbf<NT, 1, 1, 4, 8>(a, lds, s);
  if (kb == 2) return fn2 ? go_sbf<NT, 2, 2, 2>(a, lds, s) : go_sbf<NT, 2, 1, 2>(a, lds, s);
  if (kb == 4) return fn2 ? go_sbf<NT, 2, 2, 4>(a, lds, s) : go_sbf<NT, 2, 1, 4>(a, lds, s);
  return fn2 ? go_sbf<NT, 4, 2, 0>(a, lds, s) : go_sbf<NT, 4, 1, 0>(a, lds, s);
}

hipError_t launch_strided_bf16(int nterms, const StridedArgs& a, hipStream_t s) {
  if (a.nm <= 0 || a.na <= 0 || a.nb <= 0 || a.nslab <= 0 || a.nb > 65535 || a.nslab > 65535)
    return hipErrorInvalidValue;
  if (a.tn != 16 && a.tn % 32 != 0) return hipErrorInvalidValue;
  if (a.plane && (a.tn != (a.na + 31) / 32 * 32 || !a.sandwich)) return hipErrorInvalidValue;
  const int NP = bf_np_strided(a.nm);
  if (a.L1.ld < NP || (a.sandwich && a.L2.ld < NP) || (a.plane && a.P.ld < (a.na + 31) / 32 * 32))
    return hipErrorInvalidValue;
  const size_t lds = strided_bf16_lds_bytes(nterms, a.nm, a.na, a.tn, a.sandwich, a.plane);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (nterms != 2 && nterms != 3) return hipErrorInvalidValue;
  StridedArgs b = a;
  if (b.dg.part) {  // indicators: plane-tail updates, one partial pair per tile
    b.dg.tiles = (a.na + a.tn - 1) / a.tn * a.nb;
    if (!a.plane || !a.update || b.dg.tiles > b.dg.cap) return hipErrorInvalidValue;
  }
  const hipError_t e = nterms == 2 ? sbf_dispatch<2>(b, lds, s) : sbf_dispatch<3>(b, lds, s);
  if (e != hipSuccess || !b.dg.part) return e;
  return launch_diag_finish(b.dg, b.nslab, s);
}

template <int NT, int FM, int FN, int KB>
static hipError_t go_fbf(const FirstArgs& a, size_t lds, hipStream_t s) {
  auto k = first_bf16_kernel<NT, FM, FN, KB>;
  hipError_t e = bf_allow(k, lds);
  if (e != hipSuccess) return e;
  dim3 grid((a.rows + a.tm - 1) / a.tm, a.nslab);
  hipLaunchKernelGGL(k, grid, dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int NT, int KB, int FM>
static hipError_t go_fbf_mt(const FirstArgs& a, hipStream_t s) {
  auto k = first_bf16_mt_kernel<NT, KB, FM>;
  constexpr int threads = 64 * KB;
  constexpr size_t lds = static_cast<size_t>(2) * NT * 16 * FM * pitch_k(32 * KB) * 2;
  hipError_t e = bf_allow(k, lds);
  if (e != hipSuccess) return e;
  const int fit = resident_workgroups(reinterpret_cast<const void*>(k), threads, lds);
  if (fit < 1) return hipErrorInvalidValue;
  const int64_t total = static_cast<int64_t>((a.rows + 16 * FM - 1) / (16 * FM)) * a.nslab;
  if (total >= (int64_t(1) << 30)) return hipErrorInvalidValue;
  const int grid = static_cast<int>((std::min<int64_t>(fit, total) + 7) / 8 * 8);
  hipLaunchKernelGGL(k, dim3(grid), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <int NT>
static hipError_t fbf_dispatch(const FirstArgs& a, size_t lds, hipStream_t s) {
  const int kb = bf_kb(a.nm);
  if (!a.sandwich && !a.dg.part && kb > 0) {
    if (a.tm == 16) return kb == 2 ? go_fbf_mt<NT, 2, 1>(a, s) : go_fbf_mt<NT, 4, 1>(a, s);
    return kb == 2 ? go_fbf_mt<NT, 2, 2>(a, s) : go_fbf_mt<NT, 4, 2>(a, s);
  }
  if (a.tm == 16) {
    if (kb == 2) return go_fbf<NT, 1, 2, 2>(a, lds, s);
    if (kb == 4) return go_fbf<NT, 1, 2, 4>(a, lds, s);
    return go_fbf<NT, 1, 2, 0>(a, lds, s);
  }
  if (kb == 2) return go_fbf<NT, 2, 2, 2>(a, lds, s);
  if (kb == 4) return go_fbf<NT, 2, 2, 4>(a, lds, s);
  return go_fbf<NT, 2, 2, 0>(a, lds, s);
}

hipError_t launch_first_bf16(int nterms, const FirstArgs& a, hipStream_t s) {
  if (a.nm <= 0 || a.rows <= 0 || a.nslab <= 0 || a.nslab > 65535) return hipErrorInvalidValue;
  if (a.tm != 16 && a.tm != 32) return hipErrorInvalidValue;
  const int NP = bf_np_first(a.nm);
  if (a.L1.ld < NP || (a.sandwich && a.L2.ld < NP)) return hipErrorInvalidValue;
  const size_t lds = first_bf16_lds_bytes(nterms, a.nm, a.tm, a.sandwich);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (nterms != 2 && nterms != 3) return hipErrorInvalidValue;
  FirstArgs b = a;
  if (b.dg.part) {  // indicators: one partial pair per row block
    b.dg.tiles = (a.rows + a.tm - 1) / a.tm;
    if (!a.update || b.dg.tiles > b.dg.cap) return hipErrorInvalidValue;
  }
  const hipError_t e = nterms == 2 ? fbf_dispatch<2>(b, lds, s) : fbf_dispatch<3>(b, lds, s);
  if (e != hipSuccess || !b.dg.part) return e;
  return launch_diag_finish(b.dg, b.nslab, s);
}

}  // namespace tg
