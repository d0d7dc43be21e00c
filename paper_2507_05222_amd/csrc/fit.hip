// Variational fit of a sum of MPO x MPS products at fixed bond dimension:
//   y ~ sum_t c_t M_t x_t          (M_t = identity for plain additions)
// Sec. 2.2 of arxiv 2507.05222: the expensive TT operations (elementwise
// products, mat-vecs) are done variationally, i.e. by optimising the cores of
// the result directly instead of forming the fused-bond product and rounding it
// (Table 1, "Variational" column). Single-site updates: with the other cores of y
// orthonormal, the optimal core k is the projection
//   Y_k = sum_t c_t  LA^t_k . M^t_k . X^t_k . RA^t_{k+1}
// (LA^t, RA^t: environments of <y| M_t |x_t>), so ||y - sum_t c_t M_t x_t||
// decreases monotonically over a sweep. The gauge is moved with Householder QR /
// LQ, no SVD is needed.
//
// Initialisation: either the current content of y (right-canonical, e.g. the
// result of the previous time step) or a random train on the capacity profile;
// with a random start the first left-to-right pass is a randomized sketch of the
// sum (the right environments of a random train compress the right part of the
// product, the QR of each projected core gives an orthonormal range).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/qtt.h"
#include "gemm_jobs.h"

namespace qtt_solver_detail {
double* solver_ws(qtt_ctx* ctx, size_t doubles, int* rc);
int* solver_iws(qtt_ctx* ctx, size_t ints, int* rc);
int set_error(qtt_ctx* ctx, int code, const char* msg);
int lds_of(qtt_ctx* ctx);
const double* identity_mpo(qtt_ctx* ctx, int L, const int** bond, int* rc);
}

namespace {

constexpr int MAXT = 4;        // terms per fit
constexpr int FB = 4;          // chains per fit launch group

struct FTerm {
  const double* A; const int* ab;     // MPO (slot wcap_t)
  const double* kx; const int* kxb;   // ket (slot ck_t)
  double coef;
};
struct FChain {
  double* y; int* yb;                 // the fitted train (cap cy)
  FTerm t[MAXT];
  double* ws;
};
struct FBatch {
  int n, nt;
  FChain c[FB];
};
struct FGeo {
  int L, k, cy, W, lds;
  int chi;          // bond cap of the random start
  int ck[MAXT], wcap[MAXT];
  unsigned long long seed;
};
// per-chain workspace: for each term its environments, transposes and scratch
struct FLay {
  size_t env[MAXT], LA[MAXT], RA[MAXT], Mt[MAXT], Mt2[MAXT], F1[MAXT], F2[MAXT];
  size_t tmpA, gp, slab, total;
  static FLay make(int L, int cy, const int* ck, int W, int nt) {
    FLay l;
    size_t o = 0;
    auto al = [](size_t v) { return (v + 63) & ~size_t(63); };
    for (int t = 0; t < nt; ++t) {
      const size_t C = std::max(cy, ck[t]);
      l.env[t] = (size_t)cy * W * ck[t];
      l.LA[t] = o; o += al((L + 1) * l.env[t]);
      l.RA[t] = o; o += al((L + 1) * l.env[t]);
      l.Mt[t] = o; o += al((size_t)L * 4 * W * W);
      l.Mt2[t] = o; o += al((size_t)L * 4 * W * W);
      l.F1[t] = o; o += al(C * W * 2 * C);
      l.F2[t] = o; o += al(C * 2 * W * C);
    }
    l.tmpA = o; o += al(4 * (size_t)cy * cy);
    l.gp = o; o += al(4 * 4 * (size_t)cy * cy);
    l.slab = o; o += al((size_t)nt * KSPLIT_MAX * 2 * cy * cy);   // split products of the projection
    l.total = o;
    return l;
  }
};

__device__ __forceinline__ size_t sl2(int cap) { return (size_t)cap * 2 * cap; }

// Mt[(s' w2 + b')][(b 2 + s)] = A[b][s'][s][b'];  Mt2[(b 2 + s)][(s' w2 + b')] = same
__global__ void k_fit_transposes(FBatch fb, FGeo g, FLay l) {
  const int k = blockIdx.x;
  const int ci = blockIdx.y / fb.nt, t = blockIdx.y % fb.nt;
  if (ci >= fb.n) return;
  const FTerm& tm = fb.c[ci].t[t];
  const int w = tm.ab[k], w2 = tm.ab[k + 1], wc = g.wcap[t];
  const double* Ak = tm.A + (long)k * wc * 4 * wc;
  double* T = fb.c[ci].ws + l.Mt[t] + (size_t)k * 4 * g.W * g.W;
  double* T2 = fb.c[ci].ws + l.Mt2[t] + (size_t)k * 4 * g.W * g.W;
  for (int e = threadIdx.x; e < 4 * w * w2; e += blockDim.x) {
    const int i = e / (2 * w), kk = e % (2 * w);
    const int sp = i / w2, bp = i % w2, b = kk / 2, s = kk % 2;
    const double v = Ak[(long)b * 4 * wc + sp * 2 * wc + s * wc + bp];
    T[e] = v;
    T2[(size_t)kk * (2 * w2) + i] = v;
  }
}

__global__ void k_fit_env_init(FBatch fb, FGeo g, FLay l) {
  if (blockIdx.x >= fb.n) return;
  if (threadIdx.x != 0) return;
  for (int t = 0; t < fb.nt; ++t) {
    fb.c[blockIdx.x].ws[l.LA[t]] = 1.0;
    fb.c[blockIdx.x].ws[l.RA[t] + (size_t)g.L * l.env[t]] = 1.0;
  }
}

// Random train on the capacity profile min(2^k, 2^(L-k), cy): entries +-1/sqrt(bond)
// from a counter-based hash (splitmix64 of seed, chain, site, index).
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_fit_random(FBatch fb, FGeo g) {
  const int k = blockIdx.x;
  if (blockIdx.y >= fb.n) return;
  const FChain& c = fb.c[blockIdx.y];
  auto prof = [&](int j) {
    const int a = j < 30 ? (1 << j) : (1 << 30), b = (g.L - j) < 30 ? (1 << (g.L - j)) : (1 << 30);
    int v = a < b ? a : b;
    return v < g.chi ? v : g.chi;
  };
  const int b0 = prof(k), b1 = prof(k + 1);
  const double sc = 1.0 / sqrt((double)b1);
  double* Y = c.y + (long)k * sl2(g.cy);
  const int S = g.cy * 2 * g.cy;
  for (int e = threadIdx.x; e < S; e += blockDim.x) {
    const int a = e / (2 * g.cy), bb = e % g.cy;
    double v = 0.0;
    if (a < b0 && bb < b1) {
      const unsigned long long h = mix64(g.seed ^ mix64(((unsigned long long)blockIdx.y << 40) ^
                                                        ((unsigned long long)k << 32) ^ (unsigned long long)e));
      v = (h >> 63) ? sc : -sc;
    }
    Y[e] = v;
  }
  if (threadIdx.x == 0) {
    c.yb[k + 1] = b1;
    if (k == 0) c.yb[0] = 1;
  }
}

// Householder QR (left-to-right move, bond kept) and LQ (right-to-left move) of core k of y
template <int RPL, int CPW>
__global__ void __launch_bounds__(1024) k_fit_lr_qr(FBatch fb, FGeo g, FLay l) {
  extern __shared__ double smem[];
  __shared__ double rdiag[512], tau[512], vbuf[1024];
  if (blockIdx.x >= fb.n) return;
  const FChain& c = fb.c[blockIdx.x];
  const int k = g.k, cap = g.cy;
  const int m = 2 * c.yb[k], n = c.yb[k + 1];
  const int r = m < n ? m : n;
  const bool fast = RPL > 0 && m <= 64 * RPL && n <= 16 * CPW;
  const size_t need = ((size_t)m * n + (fast ? 0 : (size_t)m * r)) * sizeof(double);
  double* X = (need <= (size_t)g.lds) ? smem : (c.ws + l.gp);
  double* Yk = c.y + (long)k * sl2(cap);
  const int S = cap * 2 * cap;
  stage8(m * n, [&](int e) { return Yk[(long)(e % m) * cap + e / m]; }, [&](int e, double v) { X[e] = v; });
  __syncthreads();
  if (fast) {
    for (int e = threadIdx.x; e < S; e += blockDim.x) Yk[e] = 0.0;
    auto qs = [&](int i, int j, double v) { Yk[(long)i * cap + j] = v; };
    if constexpr (RPL > 0) qr_regs<RPL, CPW>(X, m, n, rdiag, tau, vbuf, qs);
  } else {
    double* Q = X + (size_t)m * n;
    householder(X, m, n, rdiag, tau);
    householder_q(X, m, n, tau, Q);
    for (int e = threadIdx.x; e < S; e += blockDim.x) {
      const int i = e / cap, j = e % cap;
      Yk[e] = (i < m && j < r) ? Q[(long)j * m + i] : 0.0;
    }
  }
  if (threadIdx.x == 0) c.yb[k + 1] = r;
}

template <int RPL, int CPW>
__global__ void __launch_bounds__(1024) k_fit_rl_lq(FBatch fb, FGeo g, FLay l) {
  extern __shared__ double smem[];
  __shared__ double rdiag[512], tau[512], vbuf[1024];
  if (blockIdx.x >= fb.n) return;
  const FChain& c = fb.c[blockIdx.x];
  const int k = g.k, cap = g.cy;
  const int nb = c.yb[k], mb = c.yb[k + 1];
  const int m = 2 * mb, n = nb, r = m < n ? m : n;
  const bool fast = RPL > 0 && m <= 64 * RPL && n <= 16 * CPW;
  const size_t need = ((size_t)m * n + (fast ? 0 : (size_t)m * r)) * sizeof(double);
  double* X = (need <= (size_t)g.lds) ? smem : (c.ws + l.gp);
  double* Yk = c.y + (long)k * sl2(cap);
  const int S = cap * 2 * cap;
  stage8(m * n, [&](int e) {
    const int a = e / m, rho = e % m;
    return Yk[(long)a * 2 * cap + (rho / mb) * cap + rho % mb];
  }, [&](int e, double v) { X[e] = v; });
  __syncthreads();
  if (fast) {
    for (int e = threadIdx.x; e < S; e += blockDim.x) Yk[e] = 0.0;
    auto qs = [&](int rho, int j, double v) { Yk[(long)j * 2 * cap + (rho / mb) * cap + rho % mb] = v; };
    if constexpr (RPL > 0) qr_regs<RPL, CPW>(X, m, n, rdiag, tau, vbuf, qs);
  } else {
    double* Q = X + (size_t)m * n;
    householder(X, m, n, rdiag, tau);
    householder_q(X, m, n, tau, Q);
    for (int e = threadIdx.x; e < S; e += blockDim.x) {
      const int j = e / (2 * cap), s = (e / cap) % 2, bb = e % cap;
      Yk[e] = (j < r && bb < mb) ? Q[(long)j * m + s * mb + bb] : 0.0;
    }
  }
  if (threadIdx.x == 0) c.yb[k] = r;
}

struct Fitter {
  FBatch fb;
  FGeo g;
  FLay l;
  int mode;
  hipStream_t s;

  static void one(GemmJob& j) {
    std::memset(&j, 0, sizeof(j));
    j.nb = C_(1); j.sa = C_(0); j.sb = C_(0); j.sc = C_(0); j.skip = nullptr;
    j.alpha = 1.0; j.beta = 0.0;
  }
  // launch a list of jobs in groups of GB (one launch per group)
  void run(std::vector<GemmJob>& jobs, int maxb, int maxM, int maxN, int m, int ksplit = 1, long slab = 0) {
    for (size_t i0 = 0; i0 < jobs.size(); i0 += GB) {
      GemmBatch gb;
      std::memset(&gb, 0, sizeof(gb));
      gb.n = (int)std::min<size_t>(GB, jobs.size() - i0);
      gb.maxb = maxb;
      gb.ksplit = ksplit;
      gb.slab = slab;
      for (int i = 0; i < gb.n; ++i) gb.j[i] = jobs[i0 + i];
      run_jobs(gb, maxM, maxN, m, s);
    }
  }

  // T1 = LA_k K_k and G = Mt_k T1 for every (chain, term)
  void steps12(int k) {
    std::vector<GemmJob> a, b;
    int maxck = 1;
    for (int i = 0; i < fb.n; ++i)
      for (int t = 0; t < fb.nt; ++t) {
        const FChain& c = fb.c[i];
        const FTerm& tm = c.t[t];
        const int ck = g.ck[t];
        maxck = std::max(maxck, ck);
        GemmJob j1; one(j1);   // F1[(a,b)][(s,c')] = LA[(a,b)][a'] K[a'][(s,c')]
        j1.A = c.ws + l.LA[t] + (size_t)k * l.env[t]; j1.ars = C_(ck); j1.acs = C_(1);
        j1.B = tm.kx + (size_t)k * ck * 2 * ck; j1.brs = C_(2 * ck); j1.bcs = C_(1);
        j1.C = c.ws + l.F1[t]; j1.crs = C_(2 * ck); j1.ccs = C_(1);
        j1.M = B2(c.yb, k, tm.ab, k); j1.N = C_(2 * ck); j1.K = B1(tm.kxb, k);
        a.push_back(j1);
        GemmJob j2; one(j2);   // F2[a][(s',b')][c'] = Mt[(s',b')][(b,s)] F1[a][(b,s)][c']
        j2.A = c.ws + l.Mt[t] + (size_t)k * 4 * g.W * g.W; j2.ars = B1(tm.ab, k, 2); j2.acs = C_(1);
        j2.B = c.ws + l.F1[t]; j2.brs = C_(ck); j2.bcs = C_(1);
        j2.C = c.ws + l.F2[t]; j2.crs = C_(ck); j2.ccs = C_(1);
        j2.M = B1(tm.ab, k + 1, 2); j2.N = C_(ck); j2.K = B1(tm.ab, k, 2);
        j2.nb = B1(c.yb, k); j2.sb = B1(tm.ab, k, 2 * ck); j2.sc = B1(tm.ab, k + 1, 2 * ck);
        b.push_back(j2);
      }
    run(a, 1, g.cy * g.W, 2 * maxck, mode);
    run(b, g.cy, 2 * g.W, maxck, mode);
  }

  // Y_k = sum_t c_t F2_t . RA^t_{k+1}: every (chain, term) product, split over K, stores
  // its partial products in slabs of the chain's workspace, which are then summed
  // into Y_k in a fixed order (terms, then splits).
  void project(int k) {
    steps12(k);
    std::vector<GemmJob> d;
    int ks = 2;
    for (int t = 0; t < fb.nt; ++t) ks = std::max(ks, ksplit_for(2 * g.cy, g.cy, g.wcap[t] * g.ck[t]));
    const long sl = 2L * g.cy * g.cy;
    for (int t = 0; t < fb.nt; ++t) {
      for (int i = 0; i < fb.n; ++i) {
        const FChain& c = fb.c[i];
        const FTerm& tm = c.t[t];
        const int ck = g.ck[t];
        GemmJob j; one(j);     // Y[(a,s')][c] += coef F2[(a,s')][(b',c')] RA[c][(b',c')]
        j.A = c.ws + l.F2[t]; j.ars = B1(tm.ab, k + 1, ck); j.acs = C_(1);
        j.B = c.ws + l.RA[t] + (size_t)(k + 1) * l.env[t]; j.brs = C_(1); j.bcs = B1(tm.ab, k + 1, ck);
        j.C = c.ws + l.slab + (size_t)t * ks * sl; j.crs = C_(g.cy); j.ccs = C_(1);
        j.M = B1(c.yb, k, 2); j.N = B1(c.yb, k + 1); j.K = B1(tm.ab, k + 1, ck);
        j.alpha = tm.coef;
        d.push_back(j);
      }
    }
    run(d, 1, 2 * g.cy, g.cy, mode, ks, sl);
    SlabSum z;
    std::memset(&z, 0, sizeof(z));
    z.n = fb.n; z.nq = fb.nt * ks; z.k = k; z.cap = g.cy; z.slab = sl;
    for (int i = 0; i < fb.n; ++i) {
      z.dst[i] = fb.c[i].y + (size_t)k * g.cy * 2 * g.cy;
      z.src[i] = fb.c[i].ws + l.slab;
      z.bond[i] = fb.c[i].yb;
    }
    slab_sum(z, s);
  }

  // LA^t_{k+1}[p][(b', q)] = sum_{(a, s')} Y_k[(a, s')][p] F2_t[(a, s')][(b', q)]
  void la_step3(int k) {
    std::vector<GemmJob> d;
    int maxn = 1;
    for (int i = 0; i < fb.n; ++i)
      for (int t = 0; t < fb.nt; ++t) {
        const FChain& c = fb.c[i];
        const FTerm& tm = c.t[t];
        const int ck = g.ck[t];
        maxn = std::max(maxn, g.W * ck);
        GemmJob j; one(j);
        j.A = c.y + (size_t)k * g.cy * 2 * g.cy; j.ars = C_(1); j.acs = C_(g.cy);
        j.B = c.ws + l.F2[t]; j.brs = B1(tm.ab, k + 1, ck); j.bcs = C_(1);
        j.C = c.ws + l.LA[t] + (size_t)(k + 1) * l.env[t]; j.crs = B1(tm.ab, k + 1, ck); j.ccs = C_(1);
        j.M = B1(c.yb, k + 1); j.N = B1(tm.ab, k + 1, ck); j.K = B1(c.yb, k, 2);
        d.push_back(j);
      }
    run(d, 1, g.cy, maxn, mode);
  }

  // RA^t_k[(c, b)][c'] from RA^t_{k+1}
  void ra_update(int k) {
    std::vector<GemmJob> a, b, d;
    int maxck = 1;
    for (int i = 0; i < fb.n; ++i)
      for (int t = 0; t < fb.nt; ++t) {
        const FChain& c = fb.c[i];
        const FTerm& tm = c.t[t];
        const int ck = g.ck[t];
        maxck = std::max(maxck, ck);
        const double* RAn = c.ws + l.RA[t] + (size_t)(k + 1) * l.env[t];
        const double* Yk = c.y + (size_t)k * g.cy * 2 * g.cy;
        GemmJob j1; one(j1);   // F1[(c,s')][(b',d')] = Y[(c,s')][d] RA[d][(b',d')]
        j1.A = Yk; j1.ars = C_(g.cy); j1.acs = C_(1);
        j1.B = RAn; j1.brs = B1(tm.ab, k + 1, ck); j1.bcs = C_(1);
        j1.C = c.ws + l.F1[t]; j1.crs = B1(tm.ab, k + 1, ck); j1.ccs = C_(1);
        j1.M = B1(c.yb, k, 2); j1.N = B1(tm.ab, k + 1, ck); j1.K = B1(c.yb, k + 1);
        a.push_back(j1);
        GemmJob j2; one(j2);   // F2[c][(b,s)][d'] = Mt2[(b,s)][(s',b')] F1[c][(s',b')][d']
        j2.A = c.ws + l.Mt2[t] + (size_t)k * 4 * g.W * g.W; j2.ars = B1(tm.ab, k + 1, 2); j2.acs = C_(1);
        j2.B = c.ws + l.F1[t]; j2.brs = C_(ck); j2.bcs = C_(1);
        j2.C = c.ws + l.F2[t]; j2.crs = C_(ck); j2.ccs = C_(1);
        j2.M = B1(tm.ab, k, 2); j2.N = C_(ck); j2.K = B1(tm.ab, k + 1, 2);
        j2.nb = B1(c.yb, k); j2.sb = B1(tm.ab, k + 1, 2 * ck); j2.sc = B1(tm.ab, k, 2 * ck);
        b.push_back(j2);
        GemmJob j3; one(j3);   // RA_k[(c,b)][c'] = F2[(c,b)][(s,d')] K[c'][(s,d')]
        j3.A = c.ws + l.F2[t]; j3.ars = C_(2 * ck); j3.acs = C_(1);
        j3.B = tm.kx + (size_t)k * ck * 2 * ck; j3.brs = C_(1); j3.bcs = C_(2 * ck);
        j3.C = c.ws + l.RA[t] + (size_t)k * l.env[t]; j3.crs = C_(ck); j3.ccs = C_(1);
        j3.M = B2(c.yb, k, tm.ab, k); j3.N = B1(tm.kxb, k); j3.K = C_(2 * ck);
        d.push_back(j3);
      }
    run(a, 1, 2 * g.cy, g.W * maxck, mode);
    run(b, g.cy, 2 * g.W, maxck, mode);
    run(d, 1, g.cy * g.W, maxck, mode);
  }

  void qr(int k) {
    FGeo gg = g;
    gg.k = k;
    qttk::tmark(KC_LR_QR, s);
    if (g.cy <= 64) hipLaunchKernelGGL((k_fit_lr_qr<2, 4>), dim3(fb.n), dim3(1024), g.lds, s, fb, gg, l);
    else if (g.cy <= 128) hipLaunchKernelGGL((k_fit_lr_qr<4, 8>), dim3(fb.n), dim3(1024), g.lds, s, fb, gg, l);
    else hipLaunchKernelGGL((k_fit_lr_qr<0, 0>), dim3(fb.n), dim3(1024), g.lds, s, fb, gg, l);
    qttk::tmark(KC_LR_QR, s);
  }
  void lq(int k) {
    FGeo gg = g;
    gg.k = k;
    qttk::tmark(KC_LR_QR, s);
    if (g.cy <= 64) hipLaunchKernelGGL((k_fit_rl_lq<2, 4>), dim3(fb.n), dim3(1024), g.lds, s, fb, gg, l);
    else if (g.cy <= 128) hipLaunchKernelGGL((k_fit_rl_lq<4, 8>), dim3(fb.n), dim3(1024), g.lds, s, fb, gg, l);
    else hipLaunchKernelGGL((k_fit_rl_lq<0, 0>), dim3(fb.n), dim3(1024), g.lds, s, fb, gg, l);
    qttk::tmark(KC_LR_QR, s);
  }
};

}  // namespace

namespace qtt_solver_detail {
hipError_t fit_init(int lds) {
  const void* fns[] = {(const void*)k_fit_lr_qr<2, 4>, (const void*)k_fit_lr_qr<4, 8>, (const void*)k_fit_lr_qr<0, 0>,
                       (const void*)k_fit_rl_lq<2, 4>, (const void*)k_fit_rl_lq<4, 8>, (const void*)k_fit_rl_lq<0, 0>};
  hipError_t e = hipSuccess;
  for (const void* f : fns)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  return e;
}
}  // namespace qtt_solver_detail

extern "C" int qtt_fit(qtt_ctx* ctx, int n, int nterms, const qtt_term* terms, qtt_mps* y, int chi, int sweeps,
                       int init, int contract_dt, void* stream) {
  using namespace qtt_solver_detail;
  if (!ctx) return QTT_EINVAL;
  if (n < 1 || nterms < 1 || nterms > MAXT || !terms || !y || chi < 1 || sweeps < 0 || sweeps > 64 ||
      (init != 0 && init != 1) || contract_dt < QTT_F64 || contract_dt > QTT_BF16)
    return set_error(ctx, QTT_EINVAL, "fit: bad arguments");
  const int L = y[0].L, cy = y[0].cap;
  if (chi > cy) return set_error(ctx, QTT_ECAPACITY, "fit: chi exceeds the output capacity");
  int rc = 0;
  const int* idb = nullptr;
  const double* idm = identity_mpo(ctx, L, &idb, &rc);
  if (rc) return rc;
  std::vector<int32_t> id_host(L + 1, 1);
  int ck[MAXT], wcap[MAXT], W = 1;
  for (int t = 0; t < nterms; ++t) {
    const qtt_term& t0 = terms[t];
    if (!t0.x) return set_error(ctx, QTT_EINVAL, "fit: null ket");
    ck[t] = t0.x->cap;
    wcap[t] = t0.M ? t0.M->wcap : 1;
  }
  for (int i = 0; i < n; ++i) {
    if (!y[i].data || !y[i].bond || y[i].L != L || y[i].cap != cy || y[i].d != 2)
      return set_error(ctx, QTT_ESHAPE, "fit: outputs must share L and cap");
    for (int t = 0; t < nterms; ++t) {
      const qtt_term& tm = terms[(size_t)i * nterms + t];
      if (!tm.x || !tm.x->data || !tm.x->bond || tm.x->L != L || tm.x->cap != ck[t] || tm.x->d != 2)
        return set_error(ctx, QTT_ESHAPE, "fit: term kets must share L and, per term, the cap");
      if (tm.x->data == y[i].data) return set_error(ctx, QTT_EINVAL, "fit: output aliases an input");
      if (tm.M) {
        if (!tm.M->data || !tm.M->bond || !tm.M->bond_host || tm.M->L != L || tm.M->wcap != wcap[t])
          return set_error(ctx, QTT_ESHAPE, "fit: term MPOs must share L and, per term, wcap");
        for (int k = 0; k <= L; ++k) {
          if (tm.M->bond_host[k] < 1 || tm.M->bond_host[k] > tm.M->wcap) return set_error(ctx, QTT_ESHAPE, "fit: MPO bond");
          W = std::max(W, tm.M->bond_host[k]);
        }
      } else if (wcap[t] != 1) {
        return set_error(ctx, QTT_ESHAPE, "fit: identity terms must be identity for every problem");
      }
    }
  }
  hipStream_t s = (hipStream_t)stream;
  const FLay lay = FLay::make(L, cy, ck, W, nterms);
  double* ws = solver_ws(ctx, lay.total * std::min(n, FB), &rc);
  if (rc) return rc;
  for (int i0 = 0; i0 < n; i0 += FB) {
    Fitter F;
    F.fb.n = std::min(FB, n - i0);
    F.fb.nt = nterms;
    for (int i = 0; i < F.fb.n; ++i) {
      FChain& c = F.fb.c[i];
      std::memset(&c, 0, sizeof(c));
      c.y = y[i0 + i].data; c.yb = y[i0 + i].bond;
      c.ws = ws + lay.total * i;
      for (int t = 0; t < nterms; ++t) {
        const qtt_term& tm = terms[(size_t)(i0 + i) * nterms + t];
        c.t[t].coef = tm.coef;
        c.t[t].kx = tm.x->data; c.t[t].kxb = tm.x->bond;
        if (tm.M) { c.t[t].A = tm.M->data; c.t[t].ab = tm.M->bond; }
        else { c.t[t].A = idm; c.t[t].ab = idb; }
      }
    }
    F.g.L = L; F.g.k = 0; F.g.cy = cy; F.g.W = W; F.g.lds = lds_of(ctx); F.g.chi = chi;
    for (int t = 0; t < nterms; ++t) { F.g.ck[t] = ck[t]; F.g.wcap[t] = wcap[t]; }
    F.g.seed = 0x5EEDull + (unsigned long long)i0;
    F.l = lay;
    F.mode = contract_dt;
    F.s = s;
    // random start on the profile min(2^k, 2^(L-k), chi)
    if (init == 1) hipLaunchKernelGGL(k_fit_random, dim3(L, F.fb.n), dim3(256), 0, s, F.fb, F.g);
    hipLaunchKernelGGL(k_fit_transposes, dim3(L, F.fb.n * nterms), dim3(256), 0, s, F.fb, F.g, lay);
    hipLaunchKernelGGL(k_fit_env_init, dim3(F.fb.n), dim3(64), 0, s, F.fb, F.g, lay);
    for (int k = L - 1; k >= 1; --k) F.ra_update(k);
    const int passes = std::max(1, sweeps);
    for (int sw = 0; sw < passes; ++sw) {
      for (int k = 0; k <= L - 2; ++k) {
        F.project(k);
        F.qr(k);
        F.la_step3(k);
      }
      for (int k = L - 1; k >= 1; --k) {
        F.project(k);
        F.lq(k);
        F.ra_update(k);
      }
    }
    F.project(0);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ctx, QTT_EHIP, hipGetErrorString(e));
  return QTT_OK;
}
