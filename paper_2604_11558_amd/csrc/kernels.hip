// Device kernels: MFMA mu-mode products with fused epilogues, and the
// stencil + reaction stage of the split exponential Euler step.
#include "kernels.hpp"
#include "stencil_dev.hpp"

#include <cstdio>

namespace tg {

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

// Workgroup of 4 waves computes a TM x TN tile of C; each wave a
// (TM/2) x (TN/2) quarter made of 16x16 MFMA blocks.  The K range is walked
// in chunks of KC staged through LDS (k-major so MFMA operand reads are
// unit-stride across lanes).
template <typename T, int TM, int TN, int KC>
__global__ __launch_bounds__(256) void mode_gemm_kernel(GemmArgs g) {
  using acc_t = typename Mfma<T>::acc_t;
  constexpr int WM = TM / 2, WN = TN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int LA = TM * KC / 256, LB = TN * KC / 256;
  static_assert(LA >= 1 && LB >= 1, "tile too small for 256 threads");
  __shared__ T sA[KC][TM + 4];
  __shared__ T sB[KC][TN + 4];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int tiles_n = (g.N + TN - 1) / TN;
  const int m0 = (blockIdx.x / tiles_n) * TM;
  const int n0 = (blockIdx.x % tiles_n) * TN;
  const int b = blockIdx.y, s = blockIdx.z;
  const T* A = static_cast<const T*>(g.A) + b * g.a_bstride +
               static_cast<int64_t>(s % g.a_smod) * g.a_sstride;
  const T* B = static_cast<const T*>(g.B) + b * g.b_bstride +
               static_cast<int64_t>(s % g.b_smod) * g.b_sstride;
  T* C = static_cast<T*>(g.C) + b * g.c_bstride + static_cast<int64_t>(s) * g.c_sstride;

  acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  const int li = lane & 15, lk = lane >> 4;
  for (int k0 = 0; k0 < g.K; k0 += KC) {
    T ra[LA], rb[LB];
#pragma unroll
    for (int e = 0; e < LA; ++e) {
      const int idx = tid + 256 * e;
      const int r = idx / KC, c = idx % KC;
      const int gm = m0 + r, gk = k0 + c;
      ra[e] = (gm < g.M && gk < g.K) ? A[gm * g.lda + gk] : T(0);
    }
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      const int idx = tid + 256 * e;
      if (g.b_kcontig) {
        const int nn = idx / KC, kk = idx % KC;
        const int gn = n0 + nn, gk = k0 + kk;
        rb[e] = (gn < g.N && gk < g.K) ? B[gn * g.ldb + gk] : T(0);
      } else {
        const int kk = idx / TN, nn = idx % TN;
        const int gn = n0 + nn, gk = k0 + kk;
        rb[e] = (gn < g.N && gk < g.K) ? B[gk * g.ldb + gn] : T(0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < LA; ++e) {
      const int idx = tid + 256 * e;
      sA[idx % KC][idx / KC] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      const int idx = tid + 256 * e;
      if (g.b_kcontig) sB[idx % KC][idx / KC] = rb[e];
      else sB[idx / TN][idx % TN] = rb[e];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T av[FM], bv[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) av[i] = sA[kk + lk][wm * WM + i * 16 + li];
#pragma unroll
      for (int j = 0; j < FN; ++j) bv[j] = sB[kk + lk][wn * WN + j * 16 + li];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = Mfma<T>::mac(av[i], bv[j], acc[i][j]);
    }
  }

  const double cs = (g.epi == EPI_PHI) ? g.cs[s] : 0.0;
  const double pbv = (g.epi == EPI_PHI && g.pb) ? g.pb[b] : 1.0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * WM + i * 16 + Mfma<T>::row(lk, r);
        const int col = n0 + wn * WN + j * 16 + li;
        if (row < g.M && col < g.N) {
          T v = acc[i][j][r];
          T* dst = C + static_cast<int64_t>(row) * g.ldc + col;
          if (g.epi == EPI_PHI) {
            double x = cs * pbv;
            if (g.pm) x *= g.pm[row];
            if (g.pn) x *= g.pn[col];
            v *= phi1_t(static_cast<T>(x));
            *dst = v;
          } else if (g.epi == EPI_UPDATE) {
            const T nv = *dst + static_cast<T>(g.alpha) * v;
            *dst = nv;
            if (!isfinite(nv) && g.flag) atomicOr(g.flag, 1);
          } else {
            *dst = v;
          }
        }
      }
}

template <typename T, int TM, int TN>
static hipError_t launch_tile(const GemmArgs& g, hipStream_t s) {
  constexpr int KC = 16;
  const int tiles = ((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN);
  dim3 grid(tiles, g.nbatch, g.nslab);
  hipLaunchKernelGGL((mode_gemm_kernel<T, TM, TN, KC>), grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mode_gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.nbatch <= 0 || g.nslab <= 0) return hipErrorInvalidValue;
  if (g.nbatch > 65535 || g.nslab > 65535) return hipErrorInvalidValue;
  switch (g.tile) {
    case 1: return launch_tile<T, 32, 64>(g, s);
    case 2: return launch_tile<T, 64, 32>(g, s);
    case 3: return launch_tile<T, 32, 32>(g, s);
    default: return launch_tile<T, 64, 64>(g, s);
  }
}

template hipError_t launch_mode_gemm<double>(const GemmArgs&, hipStream_t);
template hipError_t launch_mode_gemm<float>(const GemmArgs&, hipStream_t);

// ---------------------------------------------------------------------------
// Stencil + reaction: one thread per grid point of one instance; all species
// of the point are handled together because the reaction couples them.
template <typename T>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs a) {
  const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
  const int npts = n1 * n2 * n3;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int inst = blockIdx.y;
  if (p >= npts) return;
  const int i = p % n1;
  const int j = (p / n1) % n2;
  const int k = p / (n1 * n2);
  const int ns = a.nspecies;
  const T* Wi = static_cast<const T*>(a.W) + static_cast<int64_t>(inst) * ns * npts;
  T* F = static_cast<T*>(a.F) + static_cast<int64_t>(inst) * ns * npts;
  double G[3] = {0, 0, 0};
  if (a.what != 1 && a.reaction != 0) {
    double w[3] = {0, 0, 0};
    for (int sp = 0; sp < ns && sp < 3; ++sp) w[sp] = static_cast<double>(Wi[sp * npts + p]);
    reaction_dev(a, inst, w, G);
  }
  for (int sp = 0; sp < ns; ++sp) {
    double f = a.what != 2 ? diffusion_dev<T>(a, Wi, inst, sp, p, i, j, k) : 0.0;
    if (a.what != 1 && sp < 3) f += G[sp];
    F[sp * npts + p] = static_cast<T>(f);
  }
}

// Same computation with the mode count and species count fixed at compile
// time: every neighbour load of every species is issued before use.
template <typename T, int NDIM, int NS>
__global__ __launch_bounds__(256) void stencil_fast_kernel(StencilArgs a) {
  const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
  const int npts = n1 * n2 * n3;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int inst = blockIdx.y;
  if (p >= npts) return;
  const int q = p / n1;
  const int i = p - q * n1;
  const int k = q / n2;
  const int j = q - k * n2;
  const T* Wi = static_cast<const T*>(a.W) + static_cast<int64_t>(inst) * NS * npts;
  T* F = static_cast<T*>(a.F) + static_cast<int64_t>(inst) * NS * npts;
  double w[3] = {0, 0, 0};
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) w[sp] = static_cast<double>(Wi[sp * npts + p]);
  double G[3] = {0, 0, 0};
  if (a.what != 1 && a.reaction != 0) reaction_dev(a, inst, w, G);
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) {
    double f = a.what != 2 ? diffusion_fast<T, NDIM>(a, Wi + sp * npts, w[sp], sp, inst, p, i, j, k) : 0.0;
    if (a.what != 1) f += G[sp];
    F[sp * npts + p] = static_cast<T>(f);
  }
}

template <typename T, int NDIM>
static hipError_t go_stencil(const StencilArgs& a, dim3 grid, hipStream_t s) {
  switch (a.nspecies) {
    case 1: hipLaunchKernelGGL((stencil_fast_kernel<T, NDIM, 1>), grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((stencil_fast_kernel<T, NDIM, 2>), grid, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((stencil_fast_kernel<T, NDIM, 3>), grid, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const StencilArgs& a, hipStream_t s) {
  const int64_t npts = static_cast<int64_t>(a.n[0]) * a.n[1] * a.n[2];
  if (npts <= 0 || npts >= (int64_t(1) << 31) || a.batch <= 0 || a.batch > 65535) return hipErrorInvalidValue;
  dim3 grid(static_cast<unsigned>((npts + 255) / 256), a.batch);
  return a.ndim == 3 ? go_stencil<T, 3>(a, grid, s) : go_stencil<T, 2>(a, grid, s);
}

template hipError_t launch_stencil<double>(const StencilArgs&, hipStream_t);
template hipError_t launch_stencil<float>(const StencilArgs&, hipStream_t);

}  // namespace tg
