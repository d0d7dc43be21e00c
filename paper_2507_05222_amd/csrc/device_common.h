// Device building blocks shared by the kernel translation units: wavefront
// reductions, one-sided Jacobi and Householder QR for one workgroup (the MFMA
// block-GEMM tile is in gemm_tile.h). Everything here has internal linkage.
#pragma once
#include "gemm_tile.h"

namespace {

constexpr int FACT_THREADS = 1024; // threads of the one-workgroup factorisation kernels
constexpr int MAXN = 512;         // max columns handled by the factorisation kernels


__host__ __device__ inline size_t align64(size_t x) { return (x + 63) & ~size_t(63); }

// ---------------------------------------------------------------------------
// wavefront / workgroup helpers
// ---------------------------------------------------------------------------
// Lane shift of a double through DPP (two 32-bit moves); lanes without a
// valid source lane read 0.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wavefront, returned to every lane (identical bits,
// so decisions taken on it are uniform). Inclusive scan inside each row of 16
// lanes (row_shr 1, 2, 4, 8), then row_bcast 15 and 31 carry the row totals
// into lane 63, which is read back as a scalar.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0x111>(v);
  v += dpp_move<0x112>(v);
  v += dpp_move<0x114>(v);
  v += dpp_move<0x118>(v);
  v += dpp_move<0x142>(v);
  v += dpp_move<0x143>(v);
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), 63);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// dst(e, src(e)) for e < count, the workgroup's loads issued eight per thread at a
// time before any is waited for (a loop with one load per iteration would pay a
// full memory round trip per element).
template <class Src, class Dst>
__device__ __forceinline__ void stage8(int count, Src src, Dst dst) {
  constexpr int B = 8;
  for (int base = 0; base < count; base += B * (int)blockDim.x) {
    double t[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int e = base + (int)threadIdx.x + q * (int)blockDim.x;
      t[q] = e < count ? src(e) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int e = base + (int)threadIdx.x + q * (int)blockDim.x;
      if (e < count) dst(e, t[q]);
    }
  }
}

// Value of v in lane l (l uniform over the wavefront).
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// N independent wave sums at once: every DPP step is applied to all N values
// before the next, so the N dependency chains interleave instead of running
// one after the other.
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_move<0x111>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_move<0x112>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_move<0x114>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_move<0x118>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_move<0x142>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_move<0x143>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v[q]);
    const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), 63);
    const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    v[q] = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
  }
}

// Maximum over the 64 lanes of a wavefront (same DPP pattern as wave_sum).
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move<0x111>(v));
  v = fmax(v, dpp_move<0x112>(v));
  v = fmax(v, dpp_move<0x114>(v));
  v = fmax(v, dpp_move<0x118>(v));
  v = fmax(v, dpp_move<0x142>(v));
  v = fmax(v, dpp_move<0x143>(v));
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), 63);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Columns whose largest entry is below this are treated as exactly zero by the
// Householder factorisations (no reflector): the frame directions a rank-deficient
// bond carries hold rounding noise that shrinks geometrically along a sweep, and
// 1/|v|^2 of such a column would overflow.
constexpr double HH_TINY = 1e-290;
// Columns whose largest entry lies outside (HH_SMALL, HH_BIG) are rescaled before
// |x|^2 is formed (its terms could underflow or overflow); others are used as they are.
constexpr double HH_SMALL = 1e-100, HH_BIG = 1e100;

// One round of the parallel cyclic ordering with the columns in registers: each
// wavefront takes P pairs at a time, loads their 2P columns (m <= 64 T) in one go,
// reduces the P inner products together and rotates. Per pair the arithmetic and
// the order of every sum are those of the one-pair loop in jacobi_cols.
template <int T, int P>
__device__ __forceinline__ void jacobi_round_regs(double* X, int m, int ldx, int n, double* V, int ldv, int ne, int r,
                                                  double* nrm, double tiny2, double tol, int* flag, int* nrot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int base = wave * P; base < ne / 2; base += nw * P) {
    int pp[P], qq[P];
    bool act[P];
    double a[P], b[P], c[P];
    double xp[P][T], xq[P][T];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int pi = base + u;
      int p = n, q = n;
      if (pi < ne / 2) {
        if (pi == 0) { p = ne - 1; q = r; }
        else { p = (r + pi) % (ne - 1); q = (r - pi + ne - 1) % (ne - 1); }
      }
      // p, q are uniform over the wavefront: scalar registers
      p = __builtin_amdgcn_readfirstlane(p);
      q = __builtin_amdgcn_readfirstlane(q);
      act[u] = p < n && q < n;
      a[u] = act[u] ? nrm[p] : 0.0;
      b[u] = act[u] ? nrm[q] : 0.0;
      act[u] = act[u] && (a[u] > tiny2) && (b[u] > tiny2);
      pp[u] = p; qq[u] = q;
    }
#pragma unroll
    for (int u = 0; u < P; ++u)
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int i = lane + 64 * t;
        const bool ok = act[u] && i < m;
        xp[u][t] = ok ? X[(long)pp[u] * ldx + i] : 0.0;
        xq[u][t] = ok ? X[(long)qq[u] * ldx + i] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < P; ++u) {
      c[u] = 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) c[u] += xp[u][t] * xq[u][t];
    }
    wave_sum_n<P>(c);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      if (!act[u] || fabs(c[u]) <= tol * sqrt(a[u]) * sqrt(b[u])) continue;
      const double zeta = (b[u] - a[u]) / (2.0 * c[u]);
      const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int i = lane + 64 * t;
        if (i < m) {
          X[(long)pp[u] * ldx + i] = cs * xp[u][t] - sn * xq[u][t];
          X[(long)qq[u] * ldx + i] = sn * xp[u][t] + cs * xq[u][t];
        }
      }
      if (V) {
        double* vp = V + (long)pp[u] * ldv;
        double* vq = V + (long)qq[u] * ldv;
        for (int i = lane; i < n; i += 64) {
          const double x = vp[i], w = vq[i];
          vp[i] = cs * x - sn * w;
          vq[i] = sn * x + cs * w;
        }
      }
      if (lane == 0) {
        nrm[pp[u]] = a[u] - tt * c[u];
        nrm[qq[u]] = b[u] + tt * c[u];
        *flag = 1;
        atomicAdd(nrot, 1);
      }
    }
  }
}

// One-sided Jacobi (Hestenes 1958) on the n columns of X (m rows; column j at
// X + j*ldx), n <= 512. Rotations are accumulated into V (n x n, column j at
// V + j*ldv) when V is not null. Parallel cyclic (round-robin) ordering: each round
// rotates n/2 disjoint column pairs. Column norms are kept in LDS and updated with
// the rotation (a' = a - t g, b' = b + t g), recomputed exactly at the start of
// every sweep, so a pair costs one wavefront reduction (its inner product g). For
// m <= 256 the pairs of a wavefront are taken four at a time with their columns in
// registers (jacobi_round_regs), which hides the load latency of a matrix that
// lives in global memory. Stops after a sweep without rotations
// (|x_p.x_q| <= tol |x_p| |x_q|).
__device__ __forceinline__ void jacobi_cols(double* X, int m, int ldx, int n, double* V, int ldv, int* flag,
                            double* cnt = nullptr) {
  __shared__ double nrm[512];
  __shared__ double fro2_s[16];
  __shared__ int nrot;
  if (threadIdx.x == 0) nrot = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int ne = n + (n & 1);
  const double tol = 4.0e-16 * sqrt((double)(m > 1 ? m : 1));
  if (n < 2) return;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // exact column norms; their sum (the Frobenius norm) is invariant under rotations
    double f = 0.0;
    for (int j = wave; j < n; j += nw) {
      double a = 0.0;
      for (int i = lane; i < m; i += 64) { const double u = X[(long)j * ldx + i]; a += u * u; }
      a = wave_sum(a);
      if (lane == 0) nrm[j] = a;
      f += a;
    }
    if (lane == 0) fro2_s[wave] = f;
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    double fro2 = 0.0;
    for (int w = 0; w < nw; ++w) fro2 += fro2_s[w];
    // columns below (1e-15)^2 of the Frobenius norm squared are at round-off level:
    // their inner products are noise, so they count as converged
    const double tiny2 = 1e-30 * fro2 + 1e-300;
    for (int r = 0; r < ne - 1; ++r) {
      if (m <= 128) {
        jacobi_round_regs<2, 4>(X, m, ldx, n, V, ldv, ne, r, nrm, tiny2, tol, flag, &nrot);
      } else if (m <= 256) {
        jacobi_round_regs<4, 2>(X, m, ldx, n, V, ldv, ne, r, nrm, tiny2, tol, flag, &nrot);
      } else {
        for (int pi = wave; pi < ne / 2; pi += nw) {
          int p, q;
          if (pi == 0) { p = ne - 1; q = r; }
          else { p = (r + pi) % (ne - 1); q = (r - pi + ne - 1) % (ne - 1); }
          if (p >= n || q >= n) continue;
          const double a = nrm[p], b = nrm[q];
          if (!(a > tiny2) || !(b > tiny2)) continue;
          double* xp = X + (long)p * ldx;
          double* xq = X + (long)q * ldx;
          double c = 0;
          for (int i = lane; i < m; i += 64) c += xp[i] * xq[i];
          c = wave_sum(c);
          if (fabs(c) <= tol * sqrt(a) * sqrt(b)) continue;
          const double zeta = (b - a) / (2.0 * c);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int i = lane; i < m; i += 64) {
            const double u = xp[i], w = xq[i];
            xp[i] = cs * u - sn * w;
            xq[i] = sn * u + cs * w;
          }
          if (V) {
            double* vp = V + (long)p * ldv;
            double* vq = V + (long)q * ldv;
            for (int i = lane; i < n; i += 64) {
              const double u = vp[i], w = vq[i];
              vp[i] = cs * u - sn * w;
              vq[i] = sn * u + cs * w;
            }
          }
          if (lane == 0) {
            nrm[p] = a - t * c;
            nrm[q] = b + t * c;
            *flag = 1;
            atomicAdd(&nrot, 1);
          }
        }
      }
      __syncthreads();
    }
    const int fl = *flag;
    __syncthreads();
    if (cnt && threadIdx.x == 0) {
      // algorithmic work of this sweep: norms (2mn), per rotation an inner product
      // (2m) and the rotation of two columns (6m) plus two columns of V (6n)
      atomicAdd(cnt, 2.0 * m * n + (double)nrot * (8.0 * m + (V ? 6.0 * n : 0.0)));
      atomicAdd(cnt + 1, 16.0 * ((double)m * n + (V ? (double)n * n : 0.0)));
      nrot = 0;
    }
    __syncthreads();
    if (fl == 0) break;
  }
}

// ---------------------------------------------------------------------------
// Symmetric eigen-decomposition for one workgroup (1024 threads): Householder
// reduction to tridiagonal form, explicit accumulation of its orthogonal factor,
// then the implicit QL iteration with Wilkinson shifts on the tridiagonal matrix
// (the textbook method, e.g. Golub & Van Loan, Matrix Computations, Sec. 8.3).
// G: m x m symmetric, both triangles stored, column j at G + j*ldg; overwritten.
// On exit lam[i] is an eigenvalue and column i of Z (Z + i*ldz) its unit
// eigenvector, unordered. lam and work (6 m doubles) should be in LDS; Z may be in
// global memory. m <= 960 (one thread of the last wavefront runs the scalar QL
// recurrence while the first ceil(m/64) wavefronts rotate the rows of Z).
// ---------------------------------------------------------------------------
__device__ void sym_eig(double* G, int m, int ldg, double* Z, int ldz, double* lam, double* work) {
  __shared__ int nrot[2], top[2];
  __shared__ double psum[1024];                   // partial sums of the tridiagonalisation matvec
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  double* e = work;             // sub-diagonal: e[i] couples i and i + 1
  double* tau = work + m;       // reflector factors
  double* v = work + 2 * m;     // current reflector
  double* pw = work + 3 * m;    // p = tau A v, then w = p - (tau/2)(p.v) v
  double* rc = work + 4 * m;    // cosines and sines of the Givens rotations of one QL
  double* rs = work + 5 * m;    // iteration; v and pw (free by then) hold the other buffer
  // --- 1. tridiagonalisation: H_j = I - tau_j v_j v_j^T acts on rows/columns j+1..m-1
  for (int j = 0; j + 2 < m; ++j) {
    const int n2 = m - j - 1;
    double* x = G + (long)j * ldg + j + 1;          // column j below the diagonal
    if (wave == 0) {
      double mx = 0.0, ss = 0.0;
      for (int i = lane; i < n2; i += 64) { const double t = x[i]; mx = fmax(mx, fabs(t)); ss += t * t; }
      mx = wave_max(mx);
      ss = wave_sum(ss);
      const bool live = mx > HH_TINY;
      const bool rescale = live && !(mx > HH_SMALL && mx < HH_BIG);
      const double sc = !live ? 0.0 : (rescale ? 1.0 / mx : 1.0);
      if (rescale) {
        ss = 0.0;
        for (int i = lane; i < n2; i += 64) { const double t = x[i] * sc; ss += t * t; }
        ss = wave_sum(ss);
      }
      const double x0 = x[0] * sc;
      double alpha = 0.0, tj = 0.0, v0 = 0.0;
      if (live) {
        alpha = x0 >= 0 ? -sqrt(ss) : sqrt(ss);
        v0 = x0 - alpha;
        const double vv = ss - x0 * x0 + v0 * v0;
        tj = vv > 0.0 ? 2.0 / vv : 0.0;
      }
      for (int i = lane; i < n2; i += 64) {
        const double vi = (i == 0) ? v0 : x[i] * sc;
        v[j + 1 + i] = vi;
        x[i] = vi;                                   // kept for the accumulation of Q
      }
      if (lane == 0) {
        tau[j] = tj;
        lam[j] = G[(long)j * ldg + j];
        e[j] = live ? (rescale ? alpha * mx : alpha) : x0;   // x0 = 0 when not live
      }
    }
    __syncthreads();
    const double tj = tau[j];
    if (tj != 0.0) {
      // p_i = tau sum_k A(i, k) v_k over the trailing block: thread (part, row) sums
      // its part of k for row i; consecutive threads read consecutive rows of each
      // column (coalesced), and the loads of a thread are independent of each other
      {
        const int RS = m <= 256 ? 256 : 512, parts = (int)blockDim.x / RS;
        const int r = tid % RS, part = tid / RS, i = j + 1 + r;
        const int kl = (n2 + parts - 1) / parts, k0 = j + 1 + part * kl, k1 = min(m, k0 + kl);
        double a = 0.0;
        if (i < m)
          for (int k = k0; k < k1; ++k) a += G[(long)k * ldg + i] * v[k];
        psum[part * RS + r] = a;
        __syncthreads();
        if (tid < n2) {
          double t = 0.0;
          for (int q = 0; q < parts; ++q) t += psum[q * RS + tid];
          pw[j + 1 + tid] = tj * t;
        }
      }
      __syncthreads();
      double pv = 0.0;
      if (wave == 0) {
        for (int i = j + 1 + lane; i < m; i += 64) pv += pw[i] * v[i];
        pv = wave_sum(pv);
      }
      __syncthreads();
      if (wave == 0) {
        const double K = 0.5 * tj * pv;
        for (int i = j + 1 + lane; i < m; i += 64) pw[i] -= K * v[i];
      }
      __syncthreads();
      // A -= v w^T + w v^T on the trailing block
      for (long q = tid; q < (long)n2 * n2; q += blockDim.x) {
        const int k = j + 1 + (int)(q / n2), i = j + 1 + (int)(q % n2);
        G[(long)k * ldg + i] -= v[i] * pw[k] + pw[i] * v[k];
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (m >= 2) {
      lam[m - 2] = G[(long)(m - 2) * ldg + m - 2];
      e[m - 2] = G[(long)(m - 2) * ldg + m - 1];
      tau[m - 2] = 0.0;
    }
    lam[m - 1] = G[(long)(m - 1) * ldg + m - 1];
    e[m - 1] = 0.0;
    tau[m - 1] = 0.0;
  }
  // --- 2. Q = H_0 H_1 ... H_{m-3}, accumulated backwards into Z (starting from I)
  for (long q = tid; q < (long)m * m; q += blockDim.x) Z[(q / m) * ldz + q % m] = (q / m == q % m) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = m - 3; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    const double* vj = G + (long)j * ldg;          // v_j in rows j+1..m-1 of column j
    // s_c = tau v^T Z(:, c): four columns per wavefront at a time, their loads issued
    // together and their sums reduced together
    for (int c0 = j + 1 + 4 * wave; c0 < m; c0 += 4 * nw) {
      double a[4] = {0.0, 0.0, 0.0, 0.0};
      for (int i = j + 1 + lane; i < m; i += 64) {
        const double vi = vj[i];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (c0 + u < m) a[u] += vi * Z[(long)(c0 + u) * ldz + i];
      }
      wave_sum_n<4>(a);
      if (lane < 4 && c0 + lane < m) pw[c0 + lane] = tj * (lane == 0 ? a[0] : lane == 1 ? a[1] : lane == 2 ? a[2] : a[3]);
    }
    __syncthreads();
    const int n2 = m - j - 1;
    for (long q = tid; q < (long)n2 * n2; q += blockDim.x) {
      const int c = j + 1 + (int)(q / n2), i = j + 1 + (int)(q % n2);
      Z[(long)c * ldz + i] -= vj[i] * pw[c];
    }
    __syncthreads();
  }
  // --- 3. implicit QL on (lam, e); the rotations of each iteration are applied to
  // the columns of Z by the row threads while the last wavefront computes the next
  // iteration (ping-pong buffers (rc, rs) and (v, pw), up to m - 1 rotations each).
  // The whole last wavefront runs the recurrence in lock-step (lane 0 stores), so the
  // search for a negligible sub-diagonal element is a 64-wide ballot. The matrix is
  // scaled to norm <= 1 first, which makes sqrt(f^2 + g^2) safe in place of hypot.
  const bool scalar = (wave == nw - 1);
  __shared__ double qscale;
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < m; ++i) mx = fmax(mx, fabs(lam[i]) + 2.0 * fabs(e[i]));
    qscale = mx > 0.0 ? mx : 1.0;
  }
  __syncthreads();
  {
    const double inv = 1.0 / qscale;
    for (int i = tid; i < m; i += blockDim.x) { lam[i] *= inv; e[i] *= inv; }
  }
  __syncthreads();
  int ql_l = 0, ql_it = 0;                        // state of the QL wavefront (uniform)
  auto produce = [&](int b) {
    // one QL iteration (or the end); rotations for columns (i, i+1), i = top, top-1, ...
    double* cb = b ? v : rc;
    double* sb = b ? pw : rs;
    int cnt = -1, tp = 0;
    const double eps = 2.220446049250313e-16;
    while (ql_l < m) {
      const int l = ql_l;
      int mm = m - 1;
      for (int q0 = l; q0 < m - 1; q0 += 64) {
        const int q = q0 + lane;
        const bool small = q < m - 1 && fabs(e[q]) <= eps * (fabs(lam[q]) + fabs(lam[q + 1]));
        const unsigned long long mask = __ballot(small);
        if (mask) { mm = q0 + __ffsll((long long)mask) - 1; break; }
      }
      if (mm == l || ql_it >= 60) { ql_l++; ql_it = 0; continue; }
      ++ql_it;
      double g = (lam[l + 1] - lam[l]) / (2.0 * e[l]);
      double r = sqrt(g * g + 1.0);
      g = lam[mm] - lam[l] + e[l] / (g + (g >= 0 ? r : -r));
      double sn = 1.0, cs = 1.0, p = 0.0;
      cnt = 0;
      tp = mm - 1;
      bool under = false;
      double lam_up = lam[mm];                    // lam[i + 1] of the current step (old value)
      double ei = e[mm - 1], li = lam[mm - 1];     // e[i], lam[i] of the current step
      // The steps i = mm-1 .. l run in chunks of 64. At the start of a chunk lane j
      // reads the operands e[i-1], lam[i-1] of its step i = i0 - j (a step writes
      // only entries i + 1, which no later step of the iteration reads, so these are
      // the values the step would read), each step takes them with a lane read, and
      // lane j keeps the outputs of step i0 - j until the chunk ends and they are
      // stored together: no LDS access waits inside the recurrence.
      for (int i0 = mm - 1; i0 >= l && !under; i0 -= 64) {
        const int cn = min(64, i0 - l + 1);
        const int ip = i0 - 1 - lane;
        const bool has = lane < cn && ip >= l;
        const double E = has ? e[ip] : 0.0, Lm = has ? lam[ip] : 0.0;
        double se = 0.0, sl = 0.0, sc = 0.0, ss = 0.0;
        const int c0 = cnt;
        int done = 0;
        for (int j = 0; j < cn; ++j) {
          const double en = lane_value(E, j), ln = lane_value(Lm, j);
          const double f = sn * ei, b2 = cs * ei;
          const double r2 = f * f + g * g;
          if (r2 == 0.0) {
            under = true;
            break;
          }
          // 1/sqrt(r2): hardware estimate, two Newton steps (quadratic convergence from
          // the estimate's ~2^-26 relative error to rounding level)
          double ir = __builtin_amdgcn_rsq(r2);
          ir = fma(ir, fma(-0.5 * r2 * ir, ir, 0.5), ir);
          ir = fma(ir, fma(-0.5 * r2 * ir, ir, 0.5), ir);
          const double rr = r2 * ir;
          sn = f * ir;
          cs = g * ir;
          g = lam_up - p;
          r = (li - g) * sn + 2.0 * cs * b2;
          p = sn * r;
          const bool mine = lane == j;
          se = mine ? rr : se;
          sl = mine ? g + p : sl;
          sc = mine ? cs : sc;
          ss = mine ? sn : ss;
          g = cs * r - b2;
          ++cnt;
          ++done;
          lam_up = li;
          ei = en;
          li = ln;
        }
        if (lane < done) {
          e[i0 - lane + 1] = se;
          lam[i0 - lane + 1] = sl;
          cb[c0 + lane] = sc;
          sb[c0 + lane] = ss;
        }
        if (under && lane == 0) {
          // r2 underflowed at step i0 - done: the iteration ends there
          const int i = i0 - done;
          e[i + 1] = 0.0;
          lam[i + 1] = lam_up - p;
          e[mm] = 0.0;
        }
      }
      if (!under && lane == 0) {
        lam[l] -= p;
        e[l] = g;
        e[mm] = 0.0;
      }
      break;
    }
    if (lane == 0) {
      nrot[b] = cnt;      // -1: converged
      top[b] = tp;
    }
  };
  if (scalar) produce(0);
  __syncthreads();
  for (int t = 0;; ++t) {
    const int b = t & 1;
    const int cnt = nrot[b];
    if (cnt < 0) break;
    if (scalar) {
      produce(b ^ 1);
    } else if (tid < m) {
      // rotate row tid of Z: columns (i, i+1) for i = top, top-1, ..., top-cnt+1
      const int k = tid, tp = top[b];
      const double* cb = b ? v : rc;
      const double* sb = b ? pw : rs;
      double zup = Z[(long)(tp + 1) * ldz + k];
      // the column entries are loaded eight at a time ahead of their rotations
      for (int q0 = 0; q0 < cnt; q0 += 8) {
        double zi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) zi[u] = (q0 + u < cnt) ? Z[(long)(tp - q0 - u) * ldz + k] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (q0 + u < cnt) {
            const int i = tp - q0 - u;
            const double c = cb[q0 + u], sn = sb[q0 + u];
            Z[(long)(i + 1) * ldz + k] = sn * zi[u] + c * zup;
            zup = c * zi[u] - sn * zup;
          }
        }
      }
      Z[(long)(tp - cnt + 1) * ldz + k] = zup;
    }
    __syncthreads();
  }
  for (int i = tid; i < m; i += blockDim.x) lam[i] *= qscale;
  __syncthreads();
}

// Column norms of X and the permutation sorting them in decreasing order
// (ties by index). sig[j] = |x_j|, ord[pos] = j.
__device__ void sorted_norms(const double* X, int m, int ldx, int n, double* sig, int* ord) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = wave; j < n; j += nw) {
    double a = 0;
    for (int i = lane; i < m; i += 64) { const double u = X[(long)j * ldx + i]; a += u * u; }
    a = wave_sum(a);
    if (lane == 0) sig[j] = sqrt(a);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    int pos = 0;
    const double s = sig[j];
    for (int i = 0; i < n; ++i) pos += (sig[i] > s) || (sig[i] == s && i < j);
    ord[pos] = j;
  }
  __syncthreads();
}

// Permutation sorting v[0..n) in decreasing order (ties by index): ord[pos] = j.
__device__ void rank_desc(const double* v, int n, int* ord) {
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    int pos = 0;
    const double s = v[j];
    for (int i = 0; i < n; ++i) pos += (v[i] > s) || (v[i] == s && i < j);
    ord[pos] = j;
  }
  __syncthreads();
}

// Truncation rank from sorted singular values s (via ord): smallest r whose
// discarded tail has norm <= delta, capped at cap, at least 1. Single thread.
__device__ int trunc_rank(const double* sig, const int* ord, int n, double delta, int cap) {
  double tail = 0.0;
  int r = n;
  for (int q = n - 1; q >= 0; --q) {
    const double s = sig[ord[q]];
    if (sqrt(tail + s * s) <= delta) { tail += s * s; r = q; }
    else break;
  }
  if (r > cap) r = cap;
  if (r < 1) r = 1;
  return r;
}

// Householder QR of X (m x n, column-major, ld m) in place: on exit the
// reflector vectors v_j occupy X[j.., j], R's strict upper part X[i, c] (i < c),
// R's diagonal in rdiag[j] and the reflector factors in tau[j]. r = min(m, n).
__device__ void householder(double* X, int m, int n, double* rdiag, double* tau) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int r = m < n ? m : n;
  for (int j = 0; j < r; ++j) {
    double* xj = X + (long)j * m;
    if (wave == 0) {
      // scale-invariant reflector (see qr_regs): v = x / mx with v_j = x_j / mx - alpha
      double mx = 0;
      for (int i = j + lane; i < m; i += 64) mx = fmax(mx, fabs(xj[i]));
      mx = wave_max(mx);
      const bool live = mx > HH_TINY;
      const double sc = live ? 1.0 / mx : 0.0;
      double s = 0;
      for (int i = j + lane; i < m; i += 64) s += (xj[i] * sc) * (xj[i] * sc);
      s = wave_sum(s);
      const double x0 = xj[j] * sc;
      for (int i = j + 1 + lane; i < m; i += 64) xj[i] *= sc;
      if (lane == 0) {
        if (!live) { rdiag[j] = 0.0; tau[j] = 0.0; xj[j] = 0.0; }
        else {
          const double nrm = sqrt(s);
          const double alpha = x0 >= 0 ? -nrm : nrm;
          const double v0 = x0 - alpha;
          rdiag[j] = alpha * mx;
          tau[j] = 2.0 / (s - x0 * x0 + v0 * v0);
          xj[j] = v0;
        }
      }
    }
    __syncthreads();
    const double tj = tau[j];
    if (tj != 0.0) {
      for (int c = j + 1 + wave; c < n; c += nw) {
        double* xc = X + (long)c * m;
        double w = 0;
        for (int i = j + lane; i < m; i += 64) w += xj[i] * xc[i];
        w = wave_sum(w) * tj;
        for (int i = j + lane; i < m; i += 64) xc[i] -= w * xj[i];
      }
    }
    __syncthreads();
  }
}

// Householder QR with register-resident columns (1024 threads = 16 waves).
// Column c lives in the registers of wave c % 16 (slot c / 16), rows spread over
// the lanes (row = lane + 64 i). Each reflector is formed by the wave owning its
// column and published through a double-buffered LDS vector, so a column costs a
// single workgroup barrier; the thin Q is then accumulated backwards with no
// barrier at all. Same contract as householder(): on exit X holds the reflectors
// (X[j.., j]) and R's strict upper part, rdiag / tau as there; in addition the
// thin Q (m x r) is handed element by element to qstore(row, col, value).
// Requires m <= 64 RPL, n <= 16 CPW; vbuf: 2m doubles of LDS.
template <int RPL, int CPW, class QStore>
__device__ void qr_regs(double* X, int m, int n, double* rdiag, double* tau, double* vbuf, QStore qstore) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = m < n ? m : n;
  double reg[CPW][RPL];
#pragma unroll
  for (int sl = 0; sl < CPW; ++sl) {
    const int c = sl * 16 + wave;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = lane + 64 * i;
      reg[sl][i] = (c < n && row < m) ? X[(long)c * m + row] : 0.0;
    }
  }
  __syncthreads();   // every wave has read X before owners overwrite columns
  for (int j = 0; j < r; ++j) {
    double* vb = vbuf + (j & 1) * m;
    if (wave == (j & 15)) {
      const int sj = j >> 4;
      double col[RPL];
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        col[i] = 0.0;
#pragma unroll
        for (int sl = 0; sl < CPW; ++sl)
          if (sl == sj) col[i] = reg[sl][i];
      }
      // reflector H = I - tau v v^T, v = x sc with v_j = x_j sc - alpha. The largest
      // entry mx and |x|^2 reduce together; sc = 1 unless mx is so small that |x|^2
      // could underflow, where the column is rescaled by 1 / mx (scale-invariant).
      double mx = 0.0, ss = 0.0, xs = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = lane + 64 * i;
        if (row >= j && row < m) { mx = fmax(mx, fabs(col[i])); ss += col[i] * col[i]; }
        if (i == (j >> 6)) xs = col[i];
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        double t0, t1;
        switch (q) {
          case 0: t0 = dpp_move<0x111>(mx); t1 = dpp_move<0x111>(ss); break;
          case 1: t0 = dpp_move<0x112>(mx); t1 = dpp_move<0x112>(ss); break;
          case 2: t0 = dpp_move<0x114>(mx); t1 = dpp_move<0x114>(ss); break;
          case 3: t0 = dpp_move<0x118>(mx); t1 = dpp_move<0x118>(ss); break;
          case 4: t0 = dpp_move<0x142>(mx); t1 = dpp_move<0x142>(ss); break;
          default: t0 = dpp_move<0x143>(mx); t1 = dpp_move<0x143>(ss); break;
        }
        mx = fmax(mx, t0);
        ss += t1;
      }
      mx = lane_value(mx, 63);
      ss = lane_value(ss, 63);
      const bool live = mx > HH_TINY;
      const bool rescale = live && !(mx > HH_SMALL && mx < HH_BIG);
      const double sc = !live ? 0.0 : (rescale ? 1.0 / mx : 1.0);
      if (rescale) {
        ss = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int row = lane + 64 * i;
          if (row >= j && row < m) ss += (col[i] * sc) * (col[i] * sc);
        }
        ss = wave_sum(ss);
      }
      const double x0 = lane_value(xs, j & 63) * sc;
      double alpha = 0.0, v0 = 0.0, tj = 0.0;
      if (live) {
        const double nrm = sqrt(ss);
        alpha = x0 >= 0 ? -nrm : nrm;
        v0 = x0 - alpha;
        tj = 2.0 / (ss - x0 * x0 + v0 * v0);
      }
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = lane + 64 * i;
        if (row < m) {
          const double v = (row < j || !live) ? 0.0 : (row == j ? v0 : col[i] * sc);
          vb[row] = v;
          // rows above j keep R's column j; rows from j on keep the reflector
          X[(long)j * m + row] = (row < j) ? col[i] : v;
        }
      }
      if (lane == 0) { tau[j] = tj; rdiag[j] = rescale ? alpha * mx : alpha; }
    }
    __syncthreads();
    const double tj = tau[j];
    if (tj != 0.0) {
      double vr[RPL];
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = lane + 64 * i;
        vr[i] = (row < m) ? vb[row] : 0.0;
      }
      // only the columns still to be reduced (c > j): the wave reductions are bound
      // by VALU issue, so skipping finished columns beats reducing all of them at once
#pragma unroll
      for (int sl = 0; sl < CPW; ++sl) {
        const int c = sl * 16 + wave;
        if (c > j && c < n) {
          double d = 0.0;
#pragma unroll
          for (int i = 0; i < RPL; ++i) d += vr[i] * reg[sl][i];
          d = wave_sum(d) * tj;
#pragma unroll
          for (int i = 0; i < RPL; ++i) reg[sl][i] -= d * vr[i];
        }
      }
    }
  }
  // columns never owned by a reflector (n > m) keep R's remaining rows
#pragma unroll
  for (int sl = 0; sl < CPW; ++sl) {
    const int c = sl * 16 + wave;
    if (c >= r && c < n) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = lane + 64 * i;
        if (row < m) X[(long)c * m + row] = reg[sl][i];
      }
    }
  }
  __syncthreads();
  // thin Q = H_0 ... H_{r-1} [I; 0], accumulated backwards in the same registers
#pragma unroll
  for (int sl = 0; sl < CPW; ++sl) {
    const int c = sl * 16 + wave;
#pragma unroll
    for (int i = 0; i < RPL; ++i) reg[sl][i] = (lane + 64 * i == c) ? 1.0 : 0.0;
  }
  for (int j = r - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    double vr[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int row = lane + 64 * i;
      vr[i] = (row >= j && row < m) ? X[(long)j * m + row] : 0.0;
    }
#pragma unroll
    for (int sl = 0; sl < CPW; ++sl) {
      const int c = sl * 16 + wave;
      if (c >= j && c < r) {
        double d = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) d += vr[i] * reg[sl][i];
        d = wave_sum(d) * tj;
#pragma unroll
        for (int i = 0; i < RPL; ++i) reg[sl][i] -= d * vr[i];
      }
    }
  }
#pragma unroll
  for (int sl = 0; sl < CPW; ++sl) {
    const int c = sl * 16 + wave;
    if (c < r) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int row = lane + 64 * i;
        if (row < m) qstore(row, c, reg[sl][i]);
      }
    }
  }
  __syncthreads();
}

// T[i * trs + j] = sum_t la(i, t) lb(t, j) for i < M, j < N on FP64 MFMA
// (16 x 16 tiles, one per wave at a time; each K-chunk of 64 is loaded into
// registers before its 16 MFMAs so the loads overlap). Any block size that is
// a multiple of 64.
template <class LA, class LB>
__device__ void wg_gemm_f64(int M, int N, int K, LA la, LB lb, double* T, long trs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tm = (M + 15) / 16, tn = (N + 15) / 16;
  for (int t = wave; t < tm * tn; t += nw) {
    const int m0 = (t / tn) * 16, n0 = (t % tn) * 16;
    v4d acc = v4d{0, 0, 0, 0};
    for (int kb = 0; kb < K; kb += 32) {
      double a[8], b[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = kb + 4 * q + lk;
        a[q] = (m0 + li < M && k < K) ? la(m0 + li, k) : 0.0;
        b[q] = (k < K && n0 + li < N) ? lb(k, n0 + li) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + lk + 4 * v, col = n0 + li;
      if (row < M && col < N) T[(long)row * trs + col] = acc[v];
    }
  }
}

// Thin Q (m x r, column-major ld m) from the reflectors left in X by householder().
__device__ void householder_q(const double* X, int m, int n, const double* tau, double* Q) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int r = m < n ? m : n;
  for (int e = threadIdx.x; e < m * r; e += blockDim.x) Q[e] = ((e % m) == (e / m)) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = r - 1; j >= 0; --j) {
    const double tj = tau[j];
    const double* v = X + (long)j * m;
    if (tj != 0.0) {
      for (int c = j + wave; c < r; c += nw) {
        double* qc = Q + (long)c * m;
        double w = 0;
        for (int i = j + lane; i < m; i += 64) w += v[i] * qc[i];
        w = wave_sum(w) * tj;
        for (int i = j + lane; i < m; i += 64) qc[i] -= w * v[i];
      }
    }
    __syncthreads();
  }
}

}  // namespace
