// Block GEMM tile on MFMA (FP64 / FP32 / BF16 operands) and its operand views:
// the building block of the batched GEMM jobs (gemm_jobs.h) and of the zip-up
// contractions (kernels.hip).
#pragma once
#include "internal.h"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int TILE = 64;          // output tile of the block GEMM (64 x 64, 256 threads)

// ---------------------------------------------------------------------------
// block GEMM tile on MFMA
//   C(m, n) = alpha * sum_{k0 <= k < k1} A(m, k) B(k, n) + beta * C(m, n)
//   for m0 <= m < m0 + TS, n0 <= n < n0 + TS (clipped to M, N), TS = 64 or 32.
// Operands are strided views: A(m, k) = A.p[m*A.rs + k*A.cs]. Values outside the
// bounds read as zero. MODE 0: FP64 MFMA 16x16x4 (FP64 accumulate); MODE 1: FP32
// MFMA 16x16x4; MODE 2: BF16 MFMA 16x16x32 (FP32 accumulate).
// Operand lane layout (all three): lane l holds A[l%16][k-group l/16] and
// B[k-group l/16][l%16]. Result layout: FP64 D[l/16 + 4v][l%16], FP32/BF16
// D[4(l/16) + v][l%16].
// ---------------------------------------------------------------------------
struct View { const double* p; long rs, cs; };

// Explicit global-address-space views of device pointers: loads through them are
// global_load (vector memory counter only), not flat loads, which the hardware
// also counts against the LDS counter and which would therefore make every LDS
// wait also wait for the prefetched tile.
typedef const __attribute__((address_space(1))) double* gcdp;
typedef __attribute__((address_space(1))) double* gdp;
__device__ __forceinline__ gcdp as_global(const double* p) { return (gcdp)p; }
__device__ __forceinline__ gdp as_global(double* p) { return (gdp)p; }

template <int MODE> struct Cfg;
template <> struct Cfg<0> { using T = double; using Acc = v4d; static constexpr int BK = 32; static constexpr int PAD = 1; };
template <> struct Cfg<1> { using T = float;  using Acc = v4f; static constexpr int BK = 32; static constexpr int PAD = 1; };
template <> struct Cfg<2> { using T = __bf16; using Acc = v4f; static constexpr int BK = 64; static constexpr int PAD = 8; };

template <int MODE>
__device__ __forceinline__ typename Cfg<MODE>::T to_t(double v) {
  if constexpr (MODE == 2) return (__bf16)(float)v;
  else return (typename Cfg<MODE>::T)v;
}

// The K loop keeps the next K-block's global loads in flight (in registers)
// while the MFMAs of the current block run from LDS: with the small grids of
// the bond-dimension GEMMs the tile time is dominated by load latency.
// TS: output tile edge, 64 (each of the four waves owns 32 x 32, four MFMA
// blocks) or 32 (each wave owns one 16 x 16 block): the small tile puts four
// times as many workgroups, each with a quarter of the dependent MFMA chain, on
// a product whose 64 x 64 grid would leave most of the chip idle.
template <int MODE, int TS = TILE>
__device__ __forceinline__ void gemm_tile(int M, int N, int k0, int k1, View A, View B, double* C, long crs, long ccs,
                                          double alpha, double beta, int m0, int n0) {
  static_assert(TS == 64 || TS == 32, "tile edge");
  using T = typename Cfg<MODE>::T;
  using Acc = typename Cfg<MODE>::Acc;
  constexpr int BK = Cfg<MODE>::BK;
  constexpr int PAD = Cfg<MODE>::PAD;
  constexpr int PER = TS * BK / 256;       // elements of each operand per thread and K-block
  constexpr int WB = TS / 32;              // 16 x 16 MFMA blocks per wave and dimension
  __shared__ __attribute__((aligned(16))) T As[TS][BK + PAD];
  __shared__ __attribute__((aligned(16))) T Bs[TS][BK + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (TS / 2), wn = (wave & 1) * (TS / 2);
  const int li = lane & 15, lk = lane >> 4;
  const bool a_kfast = (A.cs == 1), b_nfast = (B.cs == 1);
  const gcdp Ap = as_global(A.p), Bp = as_global(B.p);
  const gdp Cg = as_global(C);
  Acc acc[WB][WB];
  for (int a = 0; a < WB; ++a)
    for (int b = 0; b < WB; ++b) acc[a][b] = Acc{0, 0, 0, 0};
  T ra[PER], rb[PER];
  auto load = [&](int kb) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      int i, kk;
      if (a_kfast) { i = e / BK; kk = e % BK; } else { i = e % TS; kk = e / TS; }
      const int gm = m0 + i, gk = kb + kk;
      ra[q] = to_t<MODE>((gm < M && gk < k1) ? Ap[(long)gm * A.rs + (long)gk * A.cs] : 0.0);
      int j;
      if (b_nfast) { j = e % TS; kk = e / TS; } else { kk = e % BK; j = e / BK; }
      const int gn = n0 + j;
      const int gk2 = kb + kk;
      rb[q] = to_t<MODE>((gn < N && gk2 < k1) ? Bp[(long)gk2 * B.rs + (long)gn * B.cs] : 0.0);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      int i, kk;
      if (a_kfast) { i = e / BK; kk = e % BK; } else { i = e % TS; kk = e / TS; }
      As[i][kk] = ra[q];
      int j;
      if (b_nfast) { j = e % TS; kk = e / TS; } else { kk = e % BK; j = e / BK; }
      Bs[j][kk] = rb[q];
    }
  };
  if (k0 < k1) load(k0);
  for (int kb = k0; kb < k1; kb += BK) {
    store();
    __syncthreads();
    if (kb + BK < k1) load(kb + BK);
    if constexpr (MODE == 0) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double av[WB], bv[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) { av[u] = As[wm + 16 * u + li][kk + lk]; bv[u] = Bs[wn + 16 * u + li][kk + lk]; }
#pragma unroll
        for (int u = 0; u < WB; ++u)
#pragma unroll
          for (int v = 0; v < WB; ++v) acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[v], acc[u][v], 0, 0, 0);
      }
    } else if constexpr (MODE == 1) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float av[WB], bv[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) { av[u] = As[wm + 16 * u + li][kk + lk]; bv[u] = Bs[wn + 16 * u + li][kk + lk]; }
#pragma unroll
        for (int u = 0; u < WB; ++u)
#pragma unroll
          for (int v = 0; v < WB; ++v) acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv[v], acc[u][v], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 32) {
        v8bf av[WB], bv[WB];
#pragma unroll
        for (int u = 0; u < WB; ++u) {
          av[u] = *reinterpret_cast<const v8bf*>(&As[wm + 16 * u + li][kk + 8 * lk]);
          bv[u] = *reinterpret_cast<const v8bf*>(&Bs[wn + 16 * u + li][kk + 8 * lk]);
        }
#pragma unroll
        for (int u = 0; u < WB; ++u)
#pragma unroll
          for (int v = 0; v < WB; ++v) acc[u][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[u], bv[v], acc[u][v], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  for (int bi = 0; bi < WB; ++bi)
    for (int bj = 0; bj < WB; ++bj)
      for (int v = 0; v < 4; ++v) {
        const int r = (MODE == 0) ? (lk + 4 * v) : (4 * lk + v);
        const int gm = m0 + wm + bi * 16 + r, gn = n0 + wn + bj * 16 + li;
        if (gm < M && gn < N) {
          double val = alpha * (double)acc[bi][bj][v];
          const gdp cp = Cg + (long)gm * crs + (long)gn * ccs;
          if (beta != 0.0) val += beta * (*cp);
          *cp = val;
        }
      }
}

#define DISPATCH_MODE(mode, KERNEL, ...)                        \
  do {                                                          \
    if ((mode) == 0) KERNEL<0>(__VA_ARGS__);                    \
    else if ((mode) == 1) KERNEL<1>(__VA_ARGS__);               \
    else KERNEL<2>(__VA_ARGS__);                                \
  } while (0)

}  // namespace
