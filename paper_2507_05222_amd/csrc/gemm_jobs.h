// Batched GEMM jobs whose sizes, strides and batch counts are products of bond
// dimensions read on the device ("bond expressions"), shared by the variational
// solver (solve.hip) and the variational fit (fit.hip).
#pragma once
#include "device_common.h"

namespace {
constexpr int GB = 4;   // jobs per launch (kernel-argument table)

// value = mul * p1[i1] * p2[i2] + add   (a null pointer counts as 1)
struct IE {
  const int* p1; const int* p2; int i1, i2, mul, add;
};
__device__ __forceinline__ int ev(const IE& e) {
  int v = e.mul;
  if (e.p1) v *= e.p1[e.i1];
  if (e.p2) v *= e.p2[e.i2];
  return v + e.add;
}
inline IE C_(int v) { return IE{nullptr, nullptr, 0, 0, 0, v}; }
inline IE B1(const int* p, int i, int mul = 1, int add = 0) { return IE{p, nullptr, i, 0, mul, add}; }
inline IE B2(const int* p, int i, const int* q, int j, int mul = 1) { return IE{p, q, i, j, mul, 0}; }

struct GemmJob {
  const double* A; IE ars, acs;
  const double* B; IE brs, bcs;
  double* C; IE crs, ccs;
  IE M, N, K;
  IE nb, sa, sb, sc;        // batch count and batch strides
  const double* skip;       // if non-null and *skip != 0, the job is skipped
  double alpha, beta;       // C = alpha A B + beta C
};
struct GemmBatch {
  int n, maxb;
  double* cnt;              // measurement counters or null
  GemmJob j[GB];
};

template <int MODE>
__global__ void __launch_bounds__(256) k_gemm_jobs(GemmBatch gb) {
  const int ci = blockIdx.z / gb.maxb, bi = blockIdx.z % gb.maxb;
  if (ci >= gb.n) return;
  const GemmJob& j = gb.j[ci];
  if (j.skip && *j.skip != 0.0) return;
  if (bi >= ev(j.nb)) return;
  const int M = ev(j.M), N = ev(j.N), K = ev(j.K);
  if (gb.cnt && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && M > 0 && N > 0 && K > 0) {
    atomicAdd(gb.cnt, 2.0 * M * N * K);
    atomicAdd(gb.cnt + 1, 8.0 * ((double)M * K + (double)K * N + (double)M * N));
  }
  const int m0 = blockIdx.y * TILE, n0 = blockIdx.x * TILE;
  if (m0 >= M || n0 >= N) return;
  View A{j.A + (long)bi * ev(j.sa), ev(j.ars), ev(j.acs)};
  View B{j.B + (long)bi * ev(j.sb), ev(j.brs), ev(j.bcs)};
  gemm_tile<MODE>(M, N, 0, K, A, B, j.C + (long)bi * ev(j.sc), ev(j.crs), ev(j.ccs), j.alpha, j.beta, m0, n0);
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

void run_jobs(const GemmBatch& gb0, int maxM, int maxN, int mode, hipStream_t s) {
  GemmBatch gb = gb0;
  gb.cnt = qttk::tcount(KC_JOBS);
  dim3 grid(cdiv(maxN, TILE), cdiv(maxM, TILE), gb.n * gb.maxb);
  qttk::tmark(KC_JOBS, s);
  if (mode == 0) hipLaunchKernelGGL(k_gemm_jobs<0>, grid, dim3(256), 0, s, gb);
  else if (mode == 1) hipLaunchKernelGGL(k_gemm_jobs<1>, grid, dim3(256), 0, s, gb);
  else hipLaunchKernelGGL(k_gemm_jobs<2>, grid, dim3(256), 0, s, gb);
  qttk::tmark(KC_JOBS, s);
}

}  // namespace
