// Device kernels: MFMA mu-mode products with fused epilogues, and the
// stencil + reaction stage of the split exponential Euler step.
#include "kernels.hpp"
#include "diag_dev.hpp"
#include "stencil_dev.hpp"

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <vector>

// Static device scratch of the entry points that allocate nothing (partial
// sums of the indicators).  In host code `scratch` names a host-side stand-in,
// not device memory: its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[tg::kStaticScratchBytes / sizeof(double)];

namespace tg {

hipError_t static_scratch(void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;  // per device ordinal
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (static_cast<size_t>(dev) >= addr.size()) addr.resize(static_cast<size_t>(dev) + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// 16x16 output MFMA with K = 4 per instruction (FP64 and FP32).  Operand
// layout per 64-lane wave (both types): A(i, k) in lane i + 16 k, B(k, j)
// in lane j + 16 k.  Accumulator element r of lane l holds D(row, l % 16)
// with row = 4 (l / 16) + r for FP32 but row = l / 16 + 4 r for FP64
// (checked on gfx950 with a one-wave probe).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using acc_t = dbl4;
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma<float> {
  using acc_t = flt4;
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

__device__ __forceinline__ double phi1_t(double x) { return x == 0.0 ? 1.0 : expm1(x) / x; }
__device__ __forceinline__ float phi1_t(float x) { return x == 0.0f ? 1.0f : expm1f(x) / x; }
// phi_2(x) = (e^x - 1 - x) / x^2, Taylor series near 0
__device__ __forceinline__ double phi2_t(double x) {
  if (fabs(x) < 1e-3) return 0.5 + x / 6.0 + x * x / 24.0 + x * x * x / 120.0;
  return (expm1(x) - x) / (x * x);
}
__device__ __forceinline__ float phi2_t(float x) {
  if (fabsf(x) < 1e-2f) return 0.5f + x / 6.0f + x * x / 24.0f + x * x * x / 120.0f;
  return (expm1f(x) - x) / (x * x);
}

// Workgroup of 4 SK waves computes a TM x TN tile of C; wave w owns the
// (TM/2) x (TN/2) quarter w % 4 of the tile, made of 16x16 MFMA blocks, over
// the (w / 4)-th of SK contiguous ranges of K.  The K range is walked in chunks of
// KC staged through LDS (k-major so MFMA operand reads are unit-stride
// across lanes); the global loads of the next chunk are issued before the
// MFMAs of the current one, so their latency overlaps the products instead
// of adding to every chunk.  SK > 1 is for grids with few tiles: a single
// wave per SIMD leaves every load, LDS and MFMA latency exposed, SK waves
// per quarter hide them for one another.  Their partial quarters are summed
// through LDS (over the staging tiles) in the fixed order 0, 1, ..., SK - 1,
// so results are reproducible.
//   FUSE = 0: plain product; 1: also C2 through epi2; 2: the contraction
//   concatenated with A2 B2; 3: a second product A B2 (sharing A's tiles)
//   into C2 through epi2.
template <typename T, int TM, int TN, int KC, int SK, int FUSE>
__global__ __launch_bounds__(256 * SK) void mode_gemm_kernel(GemmArgs g) {
  using acc_t = typename Mfma<T>::acc_t;
  constexpr int NT = 256 * SK;
  constexpr int WM = TM / 2, WN = TN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LA = TM * KC / NT, LB = TN * KC / NT;
  static_assert(LA >= 1 && LB >= 1 && LA * NT == TM * KC && LB * NT == TN * KC, "tile does not fit the threads");
  static_assert(KC % (4 * SK) == 0, "K chunk not a multiple of the k-step split");
  constexpr bool dual = FUSE == 3;
  constexpr int NACC = dual ? 2 : 1;
  __shared__ union {
    struct {
      T a[KC][TM + 4];
      T b[NACC][KC][TN + 4];
    } st;
    acc_t red[SK > 1 ? SK - 1 : 1][NACC * 4 * FM * FN][64];
  } sm;
  auto& sA = sm.st.a;
  auto& sB = sm.st.b[0];
  auto& sB2 = sm.st.b[NACC - 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int quarter = SK > 1 ? wave & 3 : wave, kq = SK > 1 ? wave >> 2 : 0;
  const int wm = quarter >> 1, wn = quarter & 1;
  const int tiles_n = (g.N + TN - 1) / TN;
  const int m0 = (blockIdx.x / tiles_n) * TM;
  const int n0 = (blockIdx.x % tiles_n) * TN;
  const int b = blockIdx.y, s = blockIdx.z;
  const T* A = static_cast<const T*>(g.A) + b * g.a_bstride +
               static_cast<int64_t>(s % g.a_smod) * g.a_sstride;
  const T* B = static_cast<const T*>(g.B) + b * g.b_bstride +
               static_cast<int64_t>(s % g.b_smod) * g.b_sstride;
  T* C = static_cast<T*>(g.C) + b * g.c_bstride + static_cast<int64_t>(s) * g.c_sstride;
  // second pair of the concatenated contraction (k >= K), same offsets
  constexpr bool cat = FUSE == 2;
  const T* A2 = cat ? static_cast<const T*>(g.A2) + (A - static_cast<const T*>(g.A)) : nullptr;
  const T* B2 = (cat || dual) ? static_cast<const T*>(g.B2) + (B - static_cast<const T*>(g.B)) : nullptr;
  const int Kt = cat ? 2 * g.K : g.K;
  const int64_t bcol = g.b_ncol ? g.b_ncol : 1, ccol = g.c_ncol ? g.c_ncol : 1;

  acc_t acc[FM][FN], acc2[dual ? FM : 1][dual ? FN : 1];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  if constexpr (dual) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc2[i][j] = acc_t{0, 0, 0, 0};
  }

  const int li = lane & 15, lk = lane >> 4;
  T ra[LA], rb[LB], rb2[dual ? LB : 1];
  // The split takes contiguous K ranges of Kq (a multiple of the k-step)
  // per wave group, so each partial sums neighbouring terms in order as the
  // unsplit product does (operands such as stencil differences cancel
  // locally; interleaved partials would grow and then cancel).  Row c of a
  // chunk's LDS tile holds k = (c / KCQ) Kq + t KCQ + c % KCQ of chunk t.
  constexpr int KCQ = KC / SK;
  const int Kq = SK == 1 ? Kt : (Kt + 4 * SK - 1) / (4 * SK) * 4;
  auto kmap = [&](int t, int c, int& gk) {
    const int kl = t * KCQ + c % KCQ;
    gk = (c / KCQ) * Kq + kl;
    return kl < Kq && gk < Kt;
  };
  {
    auto gload = [&](int t) {
#pragma unroll
      for (int e = 0; e < LA; ++e) {
        const int idx = tid + NT * e;
        const int r = idx / KC, c = idx % KC;
        const int gm = m0 + r;
        int gk;
        const bool ok = kmap(t, c, gk) && gm < g.M;
        const bool hi = cat && gk >= g.K;
        ra[e] = ok ? (hi ? A2 : A)[gm * g.lda + (hi ? gk - g.K : gk)] : T(0);
      }
#pragma unroll
      for (int e = 0; e < LB; ++e) {
        const int idx = tid + NT * e;
        int gk;
        if (g.b_kcontig) {
          const int nn = idx / KC, kk = idx % KC;
          const int gn = n0 + nn;
          const bool ok = kmap(t, kk, gk) && gn < g.N;
          const bool hi = cat && gk >= g.K;
          rb[e] = ok ? (hi ? B2 : B)[gn * g.ldb + (hi ? gk - g.K : gk)] : T(0);
          if constexpr (dual) rb2[e] = ok ? B2[gn * g.ldb + gk] : T(0);
        } else {
          const int kk = idx / TN, nn = idx % TN;
          const int gn = n0 + nn;
          const bool ok = kmap(t, kk, gk) && gn < g.N;
          const bool hi = cat && gk >= g.K;
          rb[e] = ok ? (hi ? B2 : B)[(hi ? gk - g.K : gk) * g.ldb + gn * bcol] : T(0);
          if constexpr (dual) rb2[e] = ok ? B2[gk * g.ldb + gn * bcol] : T(0);
        }
      }
    };
    gload(0);
    for (int t = 0; t * KCQ < Kq; ++t) {
      __syncthreads();  // the previous chunk's products have read the LDS tiles
#pragma unroll
      for (int e = 0; e < LA; ++e) {
        const int idx = tid + NT * e;
        sA[idx % KC][idx / KC] = ra[e];
      }
#pragma unroll
      for (int e = 0; e < LB; ++e) {
        const int idx = tid + NT * e;
        if (g.b_kcontig) sB[idx % KC][idx / KC] = rb[e];
        else sB[idx / TN][idx % TN] = rb[e];
        if constexpr (dual) {
          if (g.b_kcontig) sB2[idx % KC][idx / KC] = rb2[e];
          else sB2[idx / TN][idx % TN] = rb2[e];
        }
      }
      __syncthreads();
      if ((t + 1) * KCQ < Kq) gload(t + 1);  // in flight during this chunk's MFMAs
#pragma unroll
      for (int kk = kq * KCQ; kk < (kq + 1) * KCQ; kk += 4) {
        T av[FM], bv[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) av[i] = sA[kk + lk][wm * WM + i * 16 + li];
#pragma unroll
        for (int j = 0; j < FN; ++j) bv[j] = sB[kk + lk][wn * WN + j * 16 + li];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = Mfma<T>::mac(av[i], bv[j], acc[i][j]);
        if constexpr (dual) {
#pragma unroll
          for (int j = 0; j < FN; ++j) bv[j] = sB2[kk + lk][wn * WN + j * 16 + li];
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc2[i][j] = Mfma<T>::mac(av[i], bv[j], acc2[i][j]);
        }
      }
    }
  };
  if constexpr (SK > 1) {
    auto& red = sm.red;
    __syncthreads();  // every wave is done with the staging tiles
    constexpr int NB = 4 * FM * FN;  // blocks of one accumulator set
    if (kq > 0) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          red[kq - 1][(quarter * FM + i) * FN + j][lane] = acc[i][j];
          if constexpr (dual) red[kq - 1][NB + (quarter * FM + i) * FN + j][lane] = acc2[i][j];
        }
    }
    __syncthreads();
    if (kq == 0) {
#pragma unroll
      for (int p = 0; p < SK - 1; ++p)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            acc[i][j] = acc[i][j] + red[p][(quarter * FM + i) * FN + j][lane];
            if constexpr (dual) acc2[i][j] = acc2[i][j] + red[p][NB + (quarter * FM + i) * FN + j][lane];
          }
    }
  }

  T* C2 = (FUSE == 1 || dual) ? static_cast<T*>(g.C2) + (C - static_cast<T*>(g.C)) : nullptr;
  const bool phi_epi =
      g.epi == EPI_PHI || g.epi == EPI_DPHI || g.epi == EPI_PHI_ACC || ((FUSE == 1 || dual) && g.epi2 == EPI_PHI);
  const double cs = phi_epi ? g.cs[s] : 0.0;
  const double pbv = (phi_epi && g.pb) ? g.pb[b] : 1.0;
  const bool diag = g.dg.part != nullptr;  // EPI_UPDATE of a first-mode product
  double ds0 = 0.0, ds1 = 0.0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + Mfma<T>::row(lk, r);
        const int col = n0 + wn * WN + j * 16 + li;
        if ((SK == 1 || kq == 0) && row < g.M && col < g.N) {
          T v = acc[i][j][r];
          const int64_t off = static_cast<int64_t>(row) * g.ldc + col * ccol;
          T* dst = C + off;
          double x = 0.0;
          if (phi_epi) {
            x = cs * pbv;
            if (g.pm) x *= g.pm[row];
            if (g.pn) x *= g.pn[col];
          }
          if constexpr (FUSE == 1 || dual) {
            const T v2 = dual ? acc2[dual ? i : 0][dual ? j : 0][r] : v;
            C2[off] = g.epi2 == EPI_PHI ? v2 * phi1_t(static_cast<T>(x)) : v2;
          }
          if (g.epi == EPI_PHI || g.epi == EPI_DPHI || g.epi == EPI_PHI_ACC) {
            const T xt = static_cast<T>(x);
            if (g.epi == EPI_PHI) {
              *dst = v * phi1_t(xt);
            } else if (g.epi == EPI_PHI_ACC) {
              *dst = *dst + v * phi1_t(xt);
            } else {  // d/dd phi_1(d c) = (x / d) (phi_1 - phi_2)(x)
              *dst = v * static_cast<T>(x * g.rd[s]) * (phi1_t(xt) - phi2_t(xt));
            }
          } else if (g.epi == EPI_UPDATE) {
            const T ov = *dst;
            const T nv = ov + static_cast<T>(g.alpha) * v;
            *dst = nv;
            if (!isfinite(nv) && g.flag) atomicOr(g.flag, 1);
            if (diag) diag_point(g.dg, row, col, static_cast<double>(nv), static_cast<double>(ov), ds0, ds1);
          } else {
            *dst = v;
          }
        }
      }
  if (diag)
    diag_flush<4 * SK>(g.dg, ds0, ds1, static_cast<int64_t>(s) * g.dg.tiles + blockIdx.x,
                  reinterpret_cast<double*>(&sm));
}

template <typename T, int TM, int TN, int SK, int FUSE>
static hipError_t launch_tile_sk(const GemmArgs& g, hipStream_t s) {
  constexpr int KC = SK > 2 ? 64 : 32;
  const int tiles = ((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN);
  GemmArgs h = g;
  if (h.dg.part) {  // indicators: first-mode updates, one partial pair per tile
    h.dg.tiles = tiles;
    if (g.epi != EPI_UPDATE || !g.b_kcontig || g.nbatch != 1 || tiles > h.dg.cap) return hipErrorInvalidValue;
  }
  dim3 grid(tiles, g.nbatch, g.nslab);
  hipLaunchKernelGGL((mode_gemm_kernel<T, TM, TN, KC, SK, FUSE>), grid, dim3(256 * SK), 0, s, h);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !h.dg.part) return e;
  return launch_diag_finish(h.dg, g.nslab, s);
}

// LDS of one workgroup: the staging tiles, or the partial quarters of the
// split, whichever is larger (two B tiles and two accumulator sets for the
// dual product).
template <typename T, int TM, int TN, int SK, int FUSE>
constexpr size_t gemm_lds() {
  constexpr int KC = SK > 2 ? 64 : 32;
  constexpr int nacc = FUSE == 3 ? 2 : 1;
  const size_t st = static_cast<size_t>(KC) * (TM + 4 + nacc * (TN + 4)) * sizeof(T);
  const size_t red = static_cast<size_t>(nacc) * (SK - 1) * TM * TN * sizeof(T);
  return st > red ? st : red;
}

// Waves per SIMD: SK = 4 while the tiles give at most one workgroup of
// 4 waves per compute unit, SK = 2 while they give at most two, else 1
// (each within 64 KB of LDS).
template <typename T, int TM, int TN, int FUSE>
static hipError_t launch_tile(const GemmArgs& g, hipStream_t s) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) ==
                                                hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  const int64_t wgs = static_cast<int64_t>((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN) * g.nbatch * g.nslab;
  if constexpr (gemm_lds<T, TM, TN, 4, FUSE>() <= 65536)
    if (wgs <= cus) return launch_tile_sk<T, TM, TN, 4, FUSE>(g, s);
  if constexpr (gemm_lds<T, TM, TN, 2, FUSE>() <= 65536)
    if (wgs <= 2 * cus) return launch_tile_sk<T, TM, TN, 2, FUSE>(g, s);
  static_assert(gemm_lds<T, TM, TN, 1, FUSE>() <= 65536, "GEMM tile exceeds 64 KB of LDS");
  return launch_tile_sk<T, TM, TN, 1, FUSE>(g, s);
}

template <typename T, int TM, int TN>
static hipError_t launch_tile_fused(const GemmArgs& g, hipStream_t s) {
  if (g.A2) return launch_tile<T, TM, TN, 2>(g, s);
  if (g.C2 && g.B2) return launch_tile<T, TM, TN, 3>(g, s);
  if (g.C2) return launch_tile<T, TM, TN, 1>(g, s);
  return launch_tile<T, TM, TN, 0>(g, s);
}

template <typename T>
hipError_t launch_mode_gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.nbatch <= 0 || g.nslab <= 0) return hipErrorInvalidValue;
  if ((g.A2 && (!g.B2 || g.C2)) || (g.B2 && !g.A2 && !g.C2)) return hipErrorInvalidValue;
  if (g.C2 && (g.dg.part || (g.epi2 != EPI_STORE && g.epi2 != EPI_PHI))) return hipErrorInvalidValue;
  if (g.C2 && g.B2 && (g.epi == EPI_UPDATE || g.epi == EPI_PHI_ACC)) return hipErrorInvalidValue;
  if (g.nbatch > 65535 || g.nslab > 65535) return hipErrorInvalidValue;
  switch (g.tile) {
    case 1: return launch_tile_fused<T, 32, 64>(g, s);
    case 2: return launch_tile_fused<T, 64, 32>(g, s);
    case 3: return launch_tile_fused<T, 32, 32>(g, s);
    default: return launch_tile_fused<T, 64, 64>(g, s);
  }
}

template hipError_t launch_mode_gemm<double>(const GemmArgs&, hipStream_t);
template hipError_t launch_mode_gemm<float>(const GemmArgs&, hipStream_t);

// ---------------------------------------------------------------------------
// Stencil + reaction (stencil_fast_kernel below): one thread per grid point
// of one instance; all species of the point are handled together because
// the reaction couples them.

// Bulk-surface exchange terms (see CoupleArgs) at point p = i + n1 q of this
// side; du, dv are this side's deviations there.
template <typename T>
__device__ __forceinline__ void exchange(const StencilArgs& a, int inst, int p, int i, int npts, double du,
                                         double dv, double& G0, double& G1) {
  const CoupleArgs& c = a.cp;
  const T* other = static_cast<const T*>(c.other);
  const double* wr = a.wref + inst * 2;
  const double* orf = c.oref + inst * 2;
  if (c.kind == 3) {  // cylinder: the z = 0 layer takes the bottom disk's flux
    const int64_t m = static_cast<int64_t>(a.n[0]) * a.n[1];  // points per z layer
    if (p >= m) return;
    const double* orp = c.orp + inst * kRParams;
    const double r = orf[0] + static_cast<double>(other[(inst * 2) * m + p]);
    const double s = orf[1] + static_cast<double>(other[(inst * 2 + 1) * m + p]);
    double pp, qq;
    dib_pq(orp, wr[0] + du, wr[1] + dv, r, s, pp, qq);
    const double* dd = a.diff + inst * 2;
    G0 -= c.kappa * dd[0] * orp[0] * c.z1 * pp;
    G1 -= c.kappa * dd[1] * orp[0] * c.z2 * qq;
    return;
  }
  if (c.kind == 4) {  // bottom disk: the DIB kinetics see the cylinder's z = 0 values
    const int64_t nb = static_cast<int64_t>(c.on1) * npts;  // cylinder points per species
    const double ub1 = (orf[0] - 1.0) + static_cast<double>(other[(inst * 2) * nb + p]);  // u - 1
    const double vb1 = (orf[1] - 1.0) + static_cast<double>(other[(inst * 2 + 1) * nb + p]);
    const double* rp = a.rparams + inst * kRParams;
    const double r = wr[0] + du, s = wr[1] + dv;
    // the plain DIB kinetics were evaluated with u = v = 1: add the difference
    G0 += rp[0] * rp[1] * ub1 * (1.0 - s) * r;
    G1 += rp[0] * rp[5] * vb1 * (1.0 + rp[6] * r) * (1.0 - s) * (1.0 - rp[7] * (1.0 - s));
    return;
  }
  if (c.kind == 1) {  // bulk: only the boundary layer exchanges
    const int n1 = a.n[0];
    if (i != n1 - 1) return;
    const int64_t m = npts / n1, q = p / n1;
    const double dr = static_cast<double>(other[(inst * 2) * m + q]);
    const double ds = static_cast<double>(other[(inst * 2 + 1) * m + q]);
    const double fu = (c.z2 * orf[0] - c.z3 * wr[0]) + (c.z2 * dr - c.z3 * du);
    const double fv = (c.e1 * orf[1] - c.e2 * wr[1]) + (c.e1 * ds - c.e2 * dv);
    G0 += c.kappa * c.z1 * fu;
    G1 += c.kappa * c.z1 * fv;
  } else {  // surface point p sits above the bulk point (on1 - 1, p)
    const int64_t nb = static_cast<int64_t>(c.on1) * npts;
    const int64_t b = static_cast<int64_t>(c.on1) * p + (c.on1 - 1);
    const double dub = static_cast<double>(other[(inst * 2) * nb + b]);
    const double dvb = static_cast<double>(other[(inst * 2 + 1) * nb + b]);
    const double fu = (c.z2 * wr[0] - c.z3 * orf[0]) + (c.z2 * du - c.z3 * dub);
    const double fv = (c.e1 * wr[1] - c.e2 * orf[1]) + (c.e1 * dv - c.e2 * dvb);
    G0 -= c.z1 * fu;
    G1 -= c.z1 * fv;
  }
}

// Same computation with the mode count and species count fixed at compile
// time, in three stages: every load of the point (its value and its two
// neighbours along each mode for every species, the operator coefficients
// and the scale factors of its coordinates) is issued before any
// arithmetic, then F is evaluated, then stored.  Unscaled coordinates keep
// the factor 1 without a load (multiplying by it is exact, as skipping it
// was).  W does not overlap F or F2 (the launcher checks), so no store has
// to precede a later load.
// DUAL: also the operator part alone into F2 (what == 3).
template <typename T, int NDIM, int NS, bool DUAL>
__global__ __launch_bounds__(256) void stencil_fast_kernel(StencilArgs a) {
  const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
  const int npts = n1 * n2 * n3;
  // XCD-major block order: the grid's x extent is a multiple of 8 and
  // workgroups go round-robin over the 8 XCDs, so XCD x takes the blocks
  // x * per_xcd .. (x + 1) * per_xcd, a contiguous range of slowest-mode
  // layers whose neighbours along that mode stay in its L2
  const int per_xcd = gridDim.x >> 3;
  const int blk = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  const int64_t pl = static_cast<int64_t>(blk) * 256 + threadIdx.x;
  const int inst = blockIdx.y;
  if (pl >= npts) return;
  const int p = static_cast<int>(pl);
  const int q = p / n1;
  const int i = p - q * n1;
  const int k = q / n2;
  const int j = q - k * n2;
  const T* __restrict__ Wi = static_cast<const T*>(a.W) + static_cast<int64_t>(inst) * NS * npts;
  T* __restrict__ F = static_cast<T*>(a.F) + static_cast<int64_t>(inst) * NS * npts;
  const ReactConst rc = react_const(a, inst);  // uniform constants, requested first
  const int nm = a.nmax;
  const int idx[3] = {i, j, k};
  const int stride[3] = {1, n1, n1 * n2};

  // 1. loads
  T wc[NS], wlo[NS][NDIM], wup[NS][NDIM];
  double clo[NDIM], cdg[NDIM], cup[NDIM], sc0[NDIM], sc1[NDIM], sc2[NDIM];
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) wc[sp] = Wi[sp * npts + p];
#pragma unroll
  for (int mu = 0; mu < NDIM; ++mu) {
    const int x = idx[mu];
    const int nmu = a.n[mu];
    const bool per = (a.periodic_mask >> mu) & 1;
    // non-periodic ends have zero lo / up coefficients; the offset 0 then
    // just re-reads the centre value
    const int dm = x > 0 ? -stride[mu] : (per ? (nmu - 1) * stride[mu] : 0);
    const int dp = x + 1 < nmu ? stride[mu] : (per ? -(nmu - 1) * stride[mu] : 0);
#pragma unroll
    for (int sp = 0; sp < NS; ++sp) {
      wlo[sp][mu] = Wi[sp * npts + p + dm];
      wup[sp][mu] = Wi[sp * npts + p + dp];
    }
    const double* cf = a.coef + mu * 3 * nm;
    clo[mu] = cf[x];
    cdg[mu] = cf[nm + x];
    cup[mu] = cf[2 * nm + x];
    const double* sc = a.scale + mu * 3 * nm;
    const int sm = a.scale_mask >> (3 * mu);
    sc0[mu] = (sm & 1) ? sc[i] : 1.0;
    sc1[mu] = (sm & 2) ? sc[nm + j] : 1.0;
    sc2[mu] = (sm & 4) ? sc[2 * nm + k] : 1.0;
  }

  // 2. arithmetic
  double w[3] = {0, 0, 0};
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) w[sp] = static_cast<double>(wc[sp]);
  double G[3] = {0, 0, 0};
  if (a.what != 1 && a.reaction != 0) {
    if (a.reaction >= 4) reaction_ext(a, inst, w[0], w[1], w[2], G[0], G[1], G[2]);
    else reaction3c(rc, w[0], w[1], w[2], G[0], G[1], G[2]);
  }
  if constexpr (NS == 2) {
    if (a.cp.kind != 0 && a.what != 1) exchange<T>(a, inst, p, i, npts, w[0], w[1], G[0], G[1]);
  }
  double f[NS];
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) {
    double acc = 0.0;
#pragma unroll
    for (int mu = 0; mu < NDIM; ++mu) {
      double scl = 1.0;
      scl *= sc0[mu];
      scl *= sc1[mu];
      scl *= sc2[mu];
      acc += scl * (clo[mu] * static_cast<double>(wlo[sp][mu]) + cdg[mu] * w[sp] +
                    cup[mu] * static_cast<double>(wup[sp][mu]));
    }
    f[sp] = a.what != 2 ? a.diff[inst * a.nspecies + sp] * acc : 0.0;
  }

  // 3. stores
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) {
    if constexpr (DUAL)
      static_cast<T*>(a.F2)[static_cast<int64_t>(inst) * NS * npts + sp * npts + p] = static_cast<T>(f[sp]);
    F[sp * npts + p] = static_cast<T>(a.what != 1 ? f[sp] + G[sp] : f[sp]);
  }
}

template <typename T, int NDIM, bool DUAL>
static hipError_t go_stencil(const StencilArgs& a, dim3 grid, hipStream_t s) {
  switch (a.nspecies) {
    case 1: hipLaunchKernelGGL((stencil_fast_kernel<T, NDIM, 1, DUAL>), grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((stencil_fast_kernel<T, NDIM, 2, DUAL>), grid, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((stencil_fast_kernel<T, NDIM, 3, DUAL>), grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const StencilArgs& a, hipStream_t s) {
  const int64_t npts = static_cast<int64_t>(a.n[0]) * a.n[1] * a.n[2];
  if (npts <= 0 || npts >= (int64_t(1) << 31) || a.batch <= 0 || a.batch > 65535) return hipErrorInvalidValue;
  if (a.what < 0 || a.what > 3 || (a.what == 3 && (!a.F2 || a.cp.kind != 0))) return hipErrorInvalidValue;
  // the kernel reads W through a restrict-qualified pointer: W must not
  // overlap F or F2
  const size_t span = static_cast<size_t>(npts) * a.nspecies * a.batch * sizeof(T);
  auto overlap = [&](const void* x, const void* y) {
    const char* u = static_cast<const char*>(x);
    const char* v = static_cast<const char*>(y);
    return u < v + span && v < u + span;
  };
  if (overlap(a.W, a.F) || (a.F2 && overlap(a.W, a.F2))) return hipErrorInvalidValue;
  dim3 grid(static_cast<unsigned>((npts + 2047) / 2048 * 8), a.batch);
  if (a.what == 3) return a.ndim == 3 ? go_stencil<T, 3, true>(a, grid, s) : go_stencil<T, 2, true>(a, grid, s);
  return a.ndim == 3 ? go_stencil<T, 3, false>(a, grid, s) : go_stencil<T, 2, false>(a, grid, s);
}

template hipError_t launch_stencil<double>(const StencilArgs&, hipStream_t);
template hipError_t launch_stencil<float>(const StencilArgs&, hipStream_t);

// ---------------------------------------------------------------------------
// Steady-state indicators: each slab's partial pairs summed in a fixed order.
__global__ __launch_bounds__(256) void diag_finish_kernel(DiagArgs d) {
  __shared__ double r0[256], r1[256];
  const int s = blockIdx.x, t = threadIdx.x;
  const double* part = d.part + 2 * static_cast<int64_t>(s) * d.tiles;
  double a = 0.0, b = 0.0;
  for (int i = t; i < d.tiles; i += 256) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  r0[t] = a;
  r1[t] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      r0[t] += r0[t + w];
      r1[t] += r1[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    d.out[2 * s] = d.wref[s] + d.wsum_inv * r0[0];
    d.out[2 * s + 1] = sqrt(r1[0]);
  }
}

hipError_t launch_diag_finish(const DiagArgs& d, int nslab, hipStream_t s) {
  if (!d.part || !d.out || nslab <= 0 || nslab > 65535 || d.tiles <= 0 || d.tiles > d.cap)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(diag_finish_kernel, dim3(nslab), dim3(256), 0, s, d);
  return hipGetLastError();
}

// lam_s += tau (mtmu_s + sum_r J[r][s] mu_r), J = dG/dW at W = w_ref + state.
template <typename T>
__global__ __launch_bounds__(256) void adjoint_combine_kernel(AdjointArgs a) {
  __shared__ double red[4][9];
  const int64_t p = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int inst = blockIdx.y;
  const bool in = p < a.npts;
  const int ns = a.nspecies;
  const int64_t base = static_cast<int64_t>(inst) * ns * a.npts + (in ? p : 0);
  const T* st = static_cast<const T*>(a.state) + base;
  const T* mu = static_cast<const T*>(a.mu) + base;
  const T* mt = static_cast<const T*>(a.mtmu) + base;
  const T* tg = static_cast<const T*>(a.tang) + base;
  const T* dm = static_cast<const T*>(a.dmw) + base;
  T* lam = static_cast<T*>(a.lam) + base;
  const double* wr = a.wref + inst * ns;
  double m[3] = {0, 0, 0}, jt[3] = {0, 0, 0}, d[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (in) {
    for (int q = 0; q < ns && q < 3; ++q) m[q] = static_cast<double>(mu[q * a.npts]);
    if (a.reaction == 1 || a.reaction == 3) {  // (gamma times) g_u = a - u + u^2 v,  g_v = b - u^2 v
      const double gam = a.reaction == 3 ? a.rparams[inst * kRParams + 2] : 1.0;
      const double u = wr[0] + static_cast<double>(st[0]);
      const double v = wr[1] + static_cast<double>(st[a.npts]);
      jt[0] = gam * ((-1.0 + 2.0 * u * v) * m[0] - 2.0 * u * v * m[1]);
      jt[1] = gam * (u * u * m[0] - u * u * m[1]);
    } else if (a.reaction == 2) {  // + kappa u w and mu (u - w) terms
      const double* rp = a.rparams + inst * kRParams;
      const double kap = rp[2], mup = rp[3];
      const double u = wr[0] + static_cast<double>(st[0]);
      const double v = wr[1] + static_cast<double>(st[a.npts]);
      const double w = wr[2] + static_cast<double>(st[2 * a.npts]);
      jt[0] = (-1.0 + 2.0 * u * v - kap * w) * m[0] - 2.0 * u * v * m[1] + mup * m[2];
      jt[1] = u * u * m[0] - u * u * m[1];
      jt[2] = -kap * u * m[0] - mup * m[2];
    }
    for (int q = 0; q < ns && q < 3; ++q) {
      const double l = static_cast<double>(lam[q * a.npts]);
      d[3 * q] = l * static_cast<double>(tg[q * a.npts]);
      d[3 * q + 1] = m[q] * static_cast<double>(dm[q * a.npts]);
      d[3 * q + 2] = m[q];
      const double add = a.tau * (static_cast<double>(mt[q * a.npts]) + jt[q]);
      lam[q * a.npts] = static_cast<T>(l + add);
    }
  }
  // block partials of the three sums per species: butterfly within each
  // wave, then the four waves in order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d[k] += __shfl_xor(d[k], off, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) red[wave][k] = d[k];
  }
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < 3 * ns) {
    const int k = threadIdx.x;
    const double v = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    a.part[(static_cast<int64_t>(inst) * gridDim.x + blockIdx.x) * (3 * ns) + k] = v;
  }
}

// One block per (species, instance): the three sums of the slab over the
// combine launch's blocks, by a fixed tree, into the gradient.
__global__ __launch_bounds__(256) void adjoint_dots_kernel(const double* __restrict__ part, int blocks, int ns,
                                                           const double* tau_s, const double* taurd_s,
                                                           double* grad, int nslab) {
  __shared__ double red[3][256];
  const int q = blockIdx.x, inst = blockIdx.y, t = threadIdx.x;
  double v[3] = {0, 0, 0};
  for (int bl = t; bl < blocks; bl += 256)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] += part[(static_cast<int64_t>(inst) * blocks + bl) * (3 * ns) + 3 * q + c];
#pragma unroll
  for (int c = 0; c < 3; ++c) red[c][t] = v[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int c = 0; c < 3; ++c) red[c][t] += red[c][t + w];
    __syncthreads();
  }
  if (t == 0) {
    const int s = inst * ns + q;
    grad[s] += red[0][0] * tau_s[s];
    grad[s] += red[1][0] * taurd_s[s];
    grad[nslab + s] += red[2][0] * tau_s[s];
  }
}

template <typename T>
hipError_t launch_adjoint_combine(const AdjointArgs& a, hipStream_t s) {
  if (a.npts <= 0 || a.batch <= 0 || a.batch > 65535 || a.nspecies < 1 || a.nspecies > 3) return hipErrorInvalidValue;
  if (!a.tang || !a.dmw || !a.part || !a.grad || !a.tau_s || !a.taurd_s) return hipErrorInvalidValue;
  const int64_t blocks = (a.npts + 255) / 256;
  if (blocks > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
  dim3 grid(static_cast<unsigned>(blocks), a.batch);
  hipLaunchKernelGGL(adjoint_combine_kernel<T>, grid, dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adjoint_dots_kernel, dim3(a.nspecies, a.batch), dim3(256), 0, s, a.part, static_cast<int>(blocks),
                     a.nspecies, a.tau_s, a.taurd_s, a.grad, a.batch * a.nspecies);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void widen_kernel(const float4* __restrict__ src, double* __restrict__ dst,
                                                    int64_t n4) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n4) return;
  const float4 v = src[i];
  double2* d = reinterpret_cast<double2*>(dst + 4 * i);
  d[0] = double2{v.x, v.y};
  d[1] = double2{v.z, v.w};
}

hipError_t launch_widen(const float* src, double* dst, int64_t n, hipStream_t s) {
  // states are padded to whole float4 groups and 16-byte aligned
  if (n <= 0 || n % 4 != 0 || (reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15))
    return hipErrorInvalidValue;
  const int64_t n4 = n / 4;
  hipLaunchKernelGGL(widen_kernel, dim3(static_cast<unsigned>((n4 + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(src), dst, n4);
  return hipGetLastError();
}

template hipError_t launch_adjoint_combine<double>(const AdjointArgs&, hipStream_t);
template hipError_t launch_adjoint_combine<float>(const AdjointArgs&, hipStream_t);

}  // namespace tg
