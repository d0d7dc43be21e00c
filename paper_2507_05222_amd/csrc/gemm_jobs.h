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
  double alpha, beta;       // C = alpha A B + beta C; split over K: C += alpha A B
};
// Split over K (ksplit > 1): split sp stores alpha times its partial product (beta
// ignored, zeros for an empty K range) at C + sp * slab, a slab of its own; the
// caller sums the slabs in a fixed order (k_slab_sum), so the result does not
// depend on the order in which the workgroups run.
struct GemmBatch {
  int n, maxb;
  int ksplit;               // K-splits per output tile (1: none; jobs must then have nb == 1)
  long slab;                // doubles between the slabs of consecutive splits
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
    gemm_tile<MODE, TS>(M, N, 0, K, A, B, j.C + (long)bi * ev(j.sc), ev(j.crs), ev(j.ccs), j.alpha, j.beta,
                               m0, n0);
    return;
  }
  const int kc = ((K + S - 1) / S + Cfg<MODE>::BK - 1) / Cfg<MODE>::BK * Cfg<MODE>::BK;
  const int k0 = min(K, sp * kc), k1 = min(K, k0 + kc);
  gemm_tile<MODE, TS>(M, N, k0, k1, A, B, j.C + (long)bi * ev(j.sc) + (long)sp * gb.slab, ev(j.crs), ev(j.ccs),
                             j.alpha, 0.0, m0, n0);
}

// Fixed-order sum of split-product slabs into core k of a train: for chain i,
// dst_i[(a, s, c)] = sum_{q < nq} src_i[q * slab + (a, s, c)] for a < bond[k],
// c < bond[k + 1] (layout [a][2][cap]), and zero elsewhere in the slot.
struct SlabSum {
  int n, nq, k, cap;
  long slab;
  double* dst[QTT_BMAX];
  const double* src[QTT_BMAX];
  const int* bond[QTT_BMAX];
};
__global__ void k_slab_sum(SlabSum z) {
  const int i = blockIdx.y;
  if (i >= z.n) return;
  const int nl = z.bond[i][z.k], nr = z.bond[i][z.k + 1];
  const int S = 2 * z.cap * z.cap;
  const gcdp src = as_global(z.src[i]);
  const gdp dst = as_global(z.dst[i]);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < S; e += gridDim.x * blockDim.x) {
    const int a = e / (2 * z.cap), c = e % z.cap;
    double v = 0.0;
    if (a < nl && c < nr)
      for (int q0 = 0; q0 < z.nq; q0 += 8) {       // eight loads in flight, added in slab order
        double t[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) t[q] = (q0 + q < z.nq) ? src[(long)(q0 + q) * z.slab + e] : 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) v += t[q];
      }
    dst[e] = v;
  }
}
void slab_sum(const SlabSum& z, hipStream_t s) {
  if (z.n > 0)
    hipLaunchKernelGGL(k_slab_sum, dim3((unsigned)std::max(1, std::min(32, (2 * z.cap * z.cap + 255) / 256)), z.n),
                       dim3(256), 0, s, z);
}

// Zero fill of up to QTT_BMAX buffers of len doubles (outputs of split products).
struct ZeroList {
  int n;
  long len;
  double* p[QTT_BMAX];
};
__global__ void k_zero_list(ZeroList z) {
  if ((int)blockIdx.y >= z.n) return;
  const gdp p = as_global(z.p[blockIdx.y]);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < z.len; e += (long)gridDim.x * blockDim.x) p[e] = 0.0;
}
void zero_list(const ZeroList& z, hipStream_t s) {
  if (z.n > 0 && z.len > 0)
    hipLaunchKernelGGL(k_zero_list, dim3((unsigned)std::min<long>(16, (z.len + 1023) / 1024), z.n), dim3(256), 0, s, z);
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// K-splits for a GEMM with few output tiles and a long K: aim at ~24 workgroups
// of 64 x 64 tiles per job, at least 64 of K per split, at most KSPLIT_MAX.
constexpr int KSPLIT_MAX = 8;
inline int ksplit_for(int maxM, int maxN, int Kmax) {
  const int tiles = cdiv(maxM, TILE) * cdiv(maxN, TILE);
  const int S = std::min(24 / std::max(tiles, 1), Kmax / 64);
  return std::max(1, std::min(S, KSPLIT_MAX));
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
  const long wg64 = (long)cdiv(maxN, TILE) * cdiv(maxM, TILE) * gb.n * gb.maxb * gb.ksplit;
  const int kc = (mode == 0) ? KC_JOBS : KC_JOBS_LP;
  qttk::tmark(kc, s);
  gb.cnt = qttk::tcount(kc);   // after the mark: a launch is counted only if it is timed
  if (wg64 < SMALL_GRID) launch_jobs<32>(gb, maxM, maxN, mode, s);
  else launch_jobs<TILE>(gb, maxM, maxN, mode, s);
  qttk::tmark(kc, s);
}

}  // namespace
