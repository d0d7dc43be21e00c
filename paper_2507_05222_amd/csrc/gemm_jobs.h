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
__device__ const int g_ie_one = 1;
// Branch-free: a null pointer is replaced by the address of a constant 1, so the
// loads of all expressions of a job are unconditional and issue back to back
// (a branch per expression would serialise one memory round trip each).
__device__ __forceinline__ int ev(const IE& e) {
  const int* a = e.p1 ? e.p1 + e.i1 : &g_ie_one;
  const int* b = e.p2 ? e.p2 + e.i2 : &g_ie_one;
  return e.mul * (*a) * (*b) + e.add;
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
  double* part;             // split-K: raw partial tiles ([tile][split][64][64])
  unsigned* ctr;            // split-K: one arrival counter per output tile, zero between launches;
                            // null: every split adds its product to C with atomic adds (C must
                            // hold zeros; the order of the additions is not fixed)
};
struct GemmBatch {
  int n, maxb;
  int ksplit;               // K-splits per output tile (1: none; jobs must then have nb == 1)
  double* cnt;              // measurement counters or null
  GemmJob j[GB];
};

template <int MODE, int TS>
__global__ void __launch_bounds__(256) k_gemm_jobs(GemmBatch gb) {
  const int S = gb.ksplit;
  const int zz = blockIdx.z / S, sp = blockIdx.z % S;
  const int ci = zz / gb.maxb, bi = zz % gb.maxb;
  if (ci >= gb.n) return;
  const GemmJob& j = gb.j[ci];
  if (j.skip && *j.skip != 0.0) return;
  if (bi >= ev(j.nb)) return;
  const int M = ev(j.M), N = ev(j.N), K = ev(j.K);
  if (gb.cnt && blockIdx.x == 0 && blockIdx.y == 0 && sp == 0 && threadIdx.x == 0 && M > 0 && N > 0 && K > 0) {
    atomicAdd(gb.cnt, 2.0 * M * N * K);
    atomicAdd(gb.cnt + 1, 8.0 * ((double)M * K + (double)K * N + (double)M * N));
  }
  const int m0 = blockIdx.y * TS, n0 = blockIdx.x * TS;
  if (m0 >= M || n0 >= N) return;
  View A{j.A + (long)bi * ev(j.sa), ev(j.ars), ev(j.acs)};
  View B{j.B + (long)bi * ev(j.sb), ev(j.brs), ev(j.bcs)};
  if (S == 1) {
    gemm_tile<MODE, false, TS>(M, N, 0, K, A, B, j.C + (long)bi * ev(j.sc), ev(j.crs), ev(j.ccs), j.alpha, j.beta,
                               m0, n0);
    return;
  }
  // Split-K without arrival counters: each split adds alpha times its partial
  // product to C (zeroed by the caller) with FP64 atomic adds.
  constexpr int BKr = Cfg<MODE>::BK;
  if (!j.ctr) {
    const int kc = ((K + S - 1) / S + BKr - 1) / BKr * BKr;
    const int k0 = min(K, sp * kc), k1 = min(K, k0 + kc);
    if (k0 < k1)
      gemm_tile<MODE, true, TS>(M, N, k0, k1, A, B, j.C + (long)bi * ev(j.sc), ev(j.crs), ev(j.ccs), j.alpha, 0.0,
                                m0, n0);
    return;
  }
  if constexpr (TS != TILE) return;   // ordered finish: 64 x 64 tiles only (the launcher's choice)
  // Split-K: each split writes its raw partial tile; the last split to arrive
  // (arrival counter, no waiting) adds the partials in split order, so the result
  // does not depend on which workgroup finishes last.
  constexpr int BK = Cfg<MODE>::BK;
  const int tile = blockIdx.y * gridDim.x + blockIdx.x;
  const int kc = ((K + S - 1) / S + BK - 1) / BK * BK;
  const int k0 = min(K, sp * kc), k1 = min(K, k0 + kc);
  double* P = j.part + (size_t)tile * S * TILE * TILE;
  gemm_tile<MODE>(M, N, k0, k1, A, B, P + (size_t)sp * TILE * TILE - ((long)m0 * TILE + n0), TILE, 1, 1.0, 0.0, m0, n0);
  __threadfence();
  __syncthreads();
  __shared__ int last;
  if (threadIdx.x == 0) last = (atomicAdd(j.ctr + tile, 1u) == (unsigned)(S - 1));
  __syncthreads();
  if (!last) return;
  __threadfence();
  const long crs = ev(j.crs), ccs = ev(j.ccs);
  const gdp C = as_global(j.C);
  const gcdp Pg = as_global((const double*)P);
  // four elements per thread and pass, all partial loads issued before any add
  for (int e0 = threadIdx.x; e0 < TILE * TILE; e0 += 4 * 256) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    double pv[4][8];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 8; ++q) pv[u][q] = (q < S) ? Pg[(size_t)q * TILE * TILE + e0 + u * 256] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[u] += pv[u][q];
      const int e = e0 + u * 256;
      const int gm = m0 + e / TILE, gn = n0 + e % TILE;
      if (gm < M && gn < N) {
        const gdp cp = C + (long)gm * crs + (long)gn * ccs;
        double r = v[u] * j.alpha;
        if (j.beta != 0.0) r += j.beta * (*cp);
        *cp = r;
      }
    }
  }
  if (threadIdx.x == 0) j.ctr[tile] = 0u;
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

constexpr int SPLIT_SLOTS = 32;   // partial tiles per chain workspace (tiles * splits)
constexpr int SPLIT_CTRS = 128;   // arrival counters per chain workspace
// K-splits for a GEMM with few output tiles and a long K: aim at ~24 workgroups
// per job, at least 64 of K per split.
inline int ksplit_for(int maxM, int maxN, int Kmax) {
  const int tiles = cdiv(maxM, TILE) * cdiv(maxN, TILE);
  int S = std::min(24 / std::max(tiles, 1), Kmax / 64);
  S = std::max(1, std::min(S, 8));
  while (S > 1 && tiles * S > SPLIT_SLOTS) --S;
  if (tiles > SPLIT_CTRS) S = 1;
  return S;
}

// Launches with fewer than SMALL_GRID workgroups of 64 x 64 tiles use 32 x 32 tiles.
constexpr long SMALL_GRID = 64;

template <int TS>
void launch_jobs(const GemmBatch& gb, int maxM, int maxN, int mode, hipStream_t s) {
  dim3 grid(cdiv(maxN, TS), cdiv(maxM, TS), gb.n * gb.maxb * gb.ksplit);
  if (mode == 0) hipLaunchKernelGGL((k_gemm_jobs<0, TS>), grid, dim3(256), 0, s, gb);
  else if (mode == 1) hipLaunchKernelGGL((k_gemm_jobs<1, TS>), grid, dim3(256), 0, s, gb);
  else hipLaunchKernelGGL((k_gemm_jobs<2, TS>), grid, dim3(256), 0, s, gb);
}

void run_jobs(const GemmBatch& gb0, int maxM, int maxN, int mode, hipStream_t s) {
  GemmBatch gb = gb0;
  if (gb.ksplit < 1) gb.ksplit = 1;
  bool ordered = false;     // split-K with arrival counters works on 64 x 64 tiles
  for (int i = 0; i < gb.n; ++i) ordered = ordered || (gb.ksplit > 1 && gb.j[i].ctr);
  const long wg64 = (long)cdiv(maxN, TILE) * cdiv(maxM, TILE) * gb.n * gb.maxb * gb.ksplit;
  const int kc = (mode == 0) ? KC_JOBS : KC_JOBS_LP;
  qttk::tmark(kc, s);
  gb.cnt = qttk::tcount(kc);   // after the mark: a launch is counted only if it is timed
  if (!ordered && wg64 < SMALL_GRID) launch_jobs<32>(gb, maxM, maxN, mode, s);
  else launch_jobs<TILE>(gb, maxM, maxN, mode, s);
  qttk::tmark(kc, s);
}

}  // namespace
