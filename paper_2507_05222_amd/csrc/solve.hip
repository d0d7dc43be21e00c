// Single-site variational (ALS / one-site DMRG) solver of A x = b in TT format
// (Sec. 2.1.4 of arxiv 2507.05222: the cost C(x) = 1/2 x.Ax - x.b, local
// stationarity M_eff x_k = b_eff, DMRG-style sweeps; the local products use the
// "fast matvec" of App. G, i.e. successive contractions with the environment
// tensors instead of an assembled M_eff).
//
// Every contraction is a batched GEMM whose dimensions are products of bond
// dimensions read on the device (GemmJob with bond expressions), so a sweep is
// enqueued without host synchronisation; the host reads one FP64 number per
// chain and sweep to decide whether to continue.
//
// Convergence measure: before each local update the solver records the FP64
// residual of the local system, ||b_eff - M_eff x_k|| = ||P_k (b - A x)||, the
// global residual projected onto the frame of site k (P_k orthogonal). The
// largest of these over a sweep, divided by ||b||, is the reported residual.
// At a stationary point of the ALS iteration every projected residual is zero.
// The global form <x, A^T A x> - 2 <b, A x> + <b, b> is not used: for the
// pressure operator (condition number ~1e6 at 2^10 x 2^10) its cancellation
// error exceeds the tolerances of interest.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/qtt.h"
#include "gemm_jobs.h"

namespace {

// ---------------------------------------------------------------------------
// per-chain data of the solver
// ---------------------------------------------------------------------------
struct SChain {
  const double* A; const int* ab;   // MPO (wcap) and its device bonds
  const double* b; const int* bb;   // right-hand side (cap cb)
  double* x; int* xb;               // bra: unknown / fitted train (cap cx), updated in place
  const double* kx; const int* kxb; // ket: the train the environments contract with (cap ck)
  double* ws;                       // solver workspace
  double atol2;                     // absolute floor of the local residual (squared)
};
struct SBatch {
  int n;
  SChain c[GB];
};
struct SGeo {
  int L, k, cx, cb, wcap, W;
  int ck;           // slot capacity of the ket train
  double ltol;      // local CG: reduction of the initial local residual
  int maxit;        // CG iterations per local problem
  int lds;          // dynamic LDS budget (bytes) of the gauge-move kernels
  int mvs;          // local matvec: K-splits of its last product (slabs summed in order by the reader)
};

// workspace layout (doubles)
struct SLay {
  size_t LA, RA, Lb, Rb, F1, F2, F3, Mt, Mt2, beff, r, p, Ap, dinv, sc, tmpA, gp, LM, slab, total;
  size_t pcu, pcP, pcs, pcf, pce;   // the one-launch local CG: operand, slabs, partial sums, flags, epoch
  size_t env, envb;
  static SLay make(int L, int cx, int ck, int cb, int W) {
    SLay l;
    size_t o = 0;
    auto al = [](size_t v) { return (v + 63) & ~size_t(63); };
    l.env = (size_t)cx * W * ck;
    l.envb = (size_t)cx * cb;
    const size_t C = std::max(std::max(cx, ck), cb);
    l.LA = o; o += al((L + 1) * l.env);
    l.RA = o; o += al((L + 1) * l.env);
    l.Lb = o; o += al((L + 1) * l.envb);
    l.Rb = o; o += al((L + 1) * l.envb);
    l.F1 = o; o += al(C * W * 2 * C);
    l.F2 = o; o += al(C * 2 * W * C);   // also holds M_k T[a] of the last projection
    l.F3 = o; o += al(2 * C * C);
    l.Mt = o; o += al((size_t)L * 4 * W * W);
    l.Mt2 = o; o += al((size_t)L * 4 * W * W);
    l.beff = o; o += al(2 * (size_t)cx * cx);
    l.r = o; o += al(2 * (size_t)cx * cx);
    l.p = o; o += al(2 * (size_t)cx * cx);
    l.Ap = o; o += al((size_t)KSPLIT_MAX * 2 * cx * cx);   // split slabs of the local product
    l.dinv = o; o += al(2 * (size_t)cx * cx);
    l.sc = o; o += 64;
    l.tmpA = o; o += al(4 * (size_t)cx * cx);
    l.gp = o; o += al(4 * 4 * (size_t)cx * cx);
    l.LM = o; o += al((size_t)cx * 2 * W * 2 * cx);
    l.slab = o; o += al((size_t)KSPLIT_MAX * 2 * cx * cx);   // split products of the projection
    l.pcu = o; o += al(2 * (size_t)cx * cx);
    l.pcP = o; o += al((size_t)W * 2 * cx * cx);
    l.pcs = o; o += al(4 * 256);
    l.pcf = o; o += al(256 * 32 / 2);     // 256 flags of 128 bytes (unsigned)
    l.pce = o; o += 64;
    l.total = o;
    return l;
  }
};
// scalar slots
enum { S_RZ = 0, S_DONE, S_ITER, S_BN2, S_RN2, S_ITERS_TOTAL, S_RN0, S_PMAX, S_COUNT };

__device__ __forceinline__ size_t sl2(int cap) { return (size_t)cap * 2 * cap; }

// MPO transposes of site k: Mt[(s' w2 + b')][(b 2 + s)] = A[b][s'][s][b'];
// Mt2[(b 2 + s)][(s' w2 + b')] = A[b][s'][s][b'].
__global__ void k_transposes(SBatch sb, SGeo g, SLay l) {
  const int k = blockIdx.x;
  if (blockIdx.y >= sb.n) return;
  const SChain& c = sb.c[blockIdx.y];
  const int w = c.ab[k], w2 = c.ab[k + 1];
  const double* Ak = c.A + (long)k * g.wcap * 4 * g.wcap;
  double* T = c.ws + l.Mt + (size_t)k * 4 * g.W * g.W;
  double* T2 = c.ws + l.Mt2 + (size_t)k * 4 * g.W * g.W;
  for (int e = threadIdx.x; e < 4 * w * w2; e += blockDim.x) {
    const int i = e / (2 * w), kk = e % (2 * w);
    const int sp = i / w2, bp = i % w2, b = kk / 2, s = kk % 2;
    const double v = Ak[(long)b * 4 * g.wcap + sp * 2 * g.wcap + s * g.wcap + bp];
    T[e] = v;
    T2[(size_t)kk * (2 * w2) + i] = v;
  }
}

// environment initialisation: LA_0 = RA_L = Lb_0 = Rb_L = [1]; counters zero
__global__ void k_env_init(SBatch sb, SGeo g, SLay l) {
  if (blockIdx.x >= sb.n) return;
  const SChain& c = sb.c[blockIdx.x];
  if (threadIdx.x == 0) {
    c.ws[l.LA] = 1.0;
    c.ws[l.RA + (size_t)g.L * l.env] = 1.0;
    c.ws[l.Lb] = 1.0;
    c.ws[l.Rb + (size_t)g.L * l.envb] = 1.0;
  }
  if (threadIdx.x < S_COUNT) c.ws[l.sc + threadIdx.x] = 0.0;
  // barrier flags, epoch and failure flag of the one-launch local CG
  unsigned* f = reinterpret_cast<unsigned*>(c.ws + l.pcf);
  for (int e = threadIdx.x; e < 256 * 32; e += blockDim.x) f[e] = 0u;
  if (threadIdx.x < 2) reinterpret_cast<unsigned*>(c.ws + l.pce)[threadIdx.x] = 0u;
}

// start of a sweep: clear the maximum of the projected residuals
__global__ void k_sweep_reset(SBatch sb, SLay l) {
  if (blockIdx.x < sb.n && threadIdx.x == 0) sb.c[blockIdx.x].ws[l.sc + S_PMAX] = 0.0;
}

// Jacobi preconditioner of the local system: 1 / diag(M_eff)
__global__ void k_precond(SBatch sb, SGeo g, SLay l) {
  if (blockIdx.y >= sb.n) return;
  const SChain& c = sb.c[blockIdx.y];
  const int k = g.k, cx = g.cx;
  const int nl = c.xb[k], nr = c.xb[k + 1], w = c.ab[k], w2 = c.ab[k + 1];
  const double* LA = c.ws + l.LA + (size_t)k * l.env;
  const double* RA = c.ws + l.RA + (size_t)(k + 1) * l.env;
  const double* Ak = c.A + (long)k * g.wcap * 4 * g.wcap;
  double* dinv = c.ws + l.dinv;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 2 * cx * cx; e += gridDim.x * blockDim.x) {
    const int a = e / (2 * cx), s = (e / cx) % 2, cc = e % cx;
    double v = 0.0;
    if (a < nl && cc < nr) {
      for (int b = 0; b < w; ++b) {
        const double la = LA[((size_t)a * w + b) * cx + a];
        if (la == 0.0) continue;
        for (int b2 = 0; b2 < w2; ++b2)
          v += la * Ak[(long)b * 4 * g.wcap + s * 2 * g.wcap + s * g.wcap + b2] * RA[((size_t)cc * w2 + b2) * cx + cc];
      }
    }
    dinv[e] = v > 0.0 ? 1.0 / v : 1.0;
  }
}

// The same diagonal factored through the MPO bond b' (MPO bonds <= 32, capacity <= 64):
// T[(a, s)][b'] = sum_b LA[a][b][a] A[b][s][s][b'], then diag = sum_b' T[(a, s)][b'] RA[c][b'][c]
// (w w' + w' per element instead of w w'). Workgroup x takes the PD_RB rows (a, s) from
// x PD_RB on, all columns c; the diagonals of LA, A and RA it needs are staged into LDS
// with all loads in flight first.
constexpr int PD_W = 32, PD_C = 64, PD_RB = 16;
__global__ void __launch_bounds__(256) k_precond_fact(SBatch sb, SGeo g, SLay l) {
  __shared__ double Ad[PD_W][2][PD_W + 1];
  __shared__ double RAd[PD_C][PD_W + 1];
  __shared__ double LAd[PD_RB / 2][PD_W + 1];
  __shared__ double T[PD_RB][PD_W + 1];
  if (blockIdx.y >= sb.n) return;
  const SChain& c = sb.c[blockIdx.y];
  const int k = g.k, cx = g.cx;
  const int nl = c.xb[k], nr = c.xb[k + 1], w = c.ab[k], w2 = c.ab[k + 1];
  const double* LA = c.ws + l.LA + (size_t)k * l.env;
  const double* RA = c.ws + l.RA + (size_t)(k + 1) * l.env;
  const double* Ak = c.A + (long)k * g.wcap * 4 * g.wcap;
  double* dinv = c.ws + l.dinv;
  const int r0 = blockIdx.x * PD_RB, a0 = r0 / 2;
  stage8(w * 2 * w2, [&](int e) {
    const int b = e / (2 * w2), s = (e / w2) % 2, b2 = e % w2;
    return Ak[(long)b * 4 * g.wcap + s * 2 * g.wcap + s * g.wcap + b2];
  }, [&](int e, double v) { Ad[e / (2 * w2)][(e / w2) % 2][e % w2] = v; });
  stage8(nr * w2, [&](int e) {
    const int cc = e / w2, b2 = e % w2;
    return RA[((size_t)cc * w2 + b2) * cx + cc];
  }, [&](int e, double v) { RAd[e / w2][e % w2] = v; });
  stage8((PD_RB / 2) * w, [&](int e) {
    const int i = e / w, b = e % w, a = a0 + i;
    return a < nl ? LA[((size_t)a * w + b) * cx + a] : 0.0;
  }, [&](int e, double v) { LAd[e / w][e % w] = v; });
  __syncthreads();
  for (int e = threadIdx.x; e < PD_RB * w2; e += blockDim.x) {
    const int i = e / w2, b2 = e % w2, s = i & 1;
    double v = 0.0;
    for (int b = 0; b < w; ++b) v += LAd[i >> 1][b] * Ad[b][s][b2];
    T[i][b2] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < PD_RB * cx; e += blockDim.x) {
    const int i = e / cx, cc = e % cx, row = r0 + i;
    if (row >= 2 * cx) continue;
    double v = 0.0;
    if ((row >> 1) < nl && cc < nr)
      for (int b2 = 0; b2 < w2; ++b2) v += T[i][b2] * RAd[cc][b2];
    dinv[(size_t)row * cx + cc] = v > 0.0 ? 1.0 / v : 1.0;
  }
}

// Local CG (one workgroup per chain): vectors in [a][s][c] layout with row
// stride cx; the unknown is core k of x itself.
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

// Element e = (a 2 + s) cx + c of the local product M_eff v: the sum, in split
// order, of the g.mvs slabs of its split last product.
__device__ __forceinline__ double ap_take(const SChain& c, const SGeo& g, const SLay& l, int e) {
  const gcdp ap = as_global((const double*)(c.ws + l.Ap));
  const long n = 2L * g.cx * g.cx;
  double v = ap[e];
  for (int q = 1; q < g.mvs; ++q) v += ap[q * n + e];
  return v;
}

// first != 0: the residual belongs to the iterate before this local update; it is
// recorded as the reference of the relative stop and in the sweep maximum.
__global__ void __launch_bounds__(1024) k_cg_init(SBatch sb, SGeo g, SLay l, int first) {
  __shared__ double red[16];
  if (blockIdx.x >= sb.n) return;
  const SChain& c = sb.c[blockIdx.x];
  const int k = g.k, cx = g.cx;
  const int nl = c.xb[k], nr = c.xb[k + 1];
  double* sc = c.ws + l.sc;
  const double* beff = c.ws + l.beff;
  double* r = c.ws + l.r;
  double* p = c.ws + l.p;
  const double* dinv = c.ws + l.dinv;
  double rz = 0, bn = 0, rn = 0;
  for (int e = threadIdx.x; e < 2 * cx * cx; e += blockDim.x) {
    const int a = e / (2 * cx), cc = e % cx;
    double rv = 0, pv = 0;
    if (a < nl && cc < nr) {
      rv = beff[e] - ap_take(c, g, l, e);
      pv = dinv[e] * rv;
      rz += rv * pv; bn += beff[e] * beff[e]; rn += rv * rv;
    }
    r[e] = rv; p[e] = pv;
  }
  rz = block_sum(rz, red);
  bn = block_sum(bn, red);
  rn = block_sum(rn, red);
  if (threadIdx.x == 0) {
    if (first) {
      sc[S_RN0] = rn;
      sc[S_PMAX] = fmax(sc[S_PMAX], rn);
    }
    const double thr = fmax(g.ltol * g.ltol * (first ? rn : sc[S_RN0]), c.atol2);
    sc[S_RZ] = rz; sc[S_BN2] = bn; sc[S_RN2] = rn; sc[S_ITER] = 0;
    sc[S_DONE] = (bn == 0.0 || rn <= thr || g.maxit <= 0) ? 1.0 : 0.0;
  }
}

// Two sums over the workgroup with one pair of barriers.
__device__ void block_sum2(double& u, double& v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  u = wave_sum(u);
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) { red[wave] = u; red[16 + wave] = v; }
  __syncthreads();
  double tu = 0.0, tv = 0.0;
  for (int i = 0; i < nw; ++i) { tu += red[i]; tv += red[16 + i]; }
  u = tu; v = tv;
}

// One preconditioned CG iteration of every chain (one workgroup per chain).
// Up to 8 elements per thread (2 cx^2 <= 8192) all operands are loaded once, in
// one round trip, and kept in registers through the three phases.
__global__ void __launch_bounds__(1024) k_cg_step(SBatch sb, SGeo g, SLay l) {
  __shared__ double red[32];
  if (blockIdx.x >= sb.n) return;
  const SChain& c = sb.c[blockIdx.x];
  const gdp sc = as_global(c.ws + l.sc);
  const double done0 = sc[S_DONE], rz = sc[S_RZ], it0 = sc[S_ITER], rn0 = sc[S_RN0];
  if (done0 != 0.0) return;
  const int k = g.k, cx = g.cx, n = 2 * cx * cx;
  const int nl = c.xb[k], nr = c.xb[k + 1];
  const gdp x = as_global(c.x + (long)k * sl2(cx));
  const gdp r = as_global(c.ws + l.r);
  const gdp p = as_global(c.ws + l.p);
  const gcdp dinv = as_global((const double*)(c.ws + l.dinv));
  const int tid = threadIdx.x;
  double pAp = 0.0, rn = 0.0, rz2 = 0.0, alpha = 0.0;
  bool done;
  if (n <= 8 * 1024) {
    double pv[8], av[8], xv[8], rv[8], dv[8];
    bool ok[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 1024 * q;
      const bool in = e < n;
      ok[q] = in && (e / (2 * cx)) < nl && (e % cx) < nr;
      pv[q] = in ? p[e] : 0.0;
      av[q] = ok[q] ? ap_take(c, g, l, e) : 0.0;
      xv[q] = ok[q] ? x[e] : 0.0;
      rv[q] = ok[q] ? r[e] : 0.0;
      dv[q] = ok[q] ? dinv[e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) pAp += pv[q] * av[q];
    pAp = block_sum(pAp, red);
    alpha = pAp > 0.0 ? rz / pAp : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (ok[q]) {
        const int e = tid + 1024 * q;
        x[e] = xv[q] + alpha * pv[q];
        rv[q] -= alpha * av[q];
        r[e] = rv[q];
        rn += rv[q] * rv[q];
        rz2 += rv[q] * dv[q] * rv[q];
      }
    }
    block_sum2(rn, rz2, red);
    done = !(pAp > 0.0) || rn <= fmax(g.ltol * g.ltol * rn0, c.atol2) || it0 + 1.0 >= g.maxit;
    if (!done) {
      const double beta = rz > 0.0 ? rz2 / rz : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (ok[q]) p[tid + 1024 * q] = dv[q] * rv[q] + beta * pv[q];
    }
  } else {
    for (int e = tid; e < n; e += blockDim.x) {
      const int a = e / (2 * cx), cc = e % cx;
      if (a < nl && cc < nr) pAp += p[e] * ap_take(c, g, l, e);
    }
    pAp = block_sum(pAp, red);
    alpha = pAp > 0.0 ? rz / pAp : 0.0;
    for (int e = tid; e < n; e += blockDim.x) {
      const int a = e / (2 * cx), cc = e % cx;
      if (a < nl && cc < nr) {
        x[e] += alpha * p[e];
        const double v = r[e] - alpha * ap_take(c, g, l, e);   // second and last read
        r[e] = v;
        rn += v * v;
        rz2 += v * dinv[e] * v;
      }
    }
    block_sum2(rn, rz2, red);
    done = !(pAp > 0.0) || rn <= fmax(g.ltol * g.ltol * rn0, c.atol2) || it0 + 1.0 >= g.maxit;
    if (!done) {
      const double beta = rz > 0.0 ? rz2 / rz : 0.0;
      for (int e = tid; e < n; e += blockDim.x) p[e] = dinv[e] * r[e] + beta * p[e];
    }
  }
  __syncthreads();
  if (tid == 0) {
    sc[S_RZ] = rz2; sc[S_RN2] = rn; sc[S_ITER] = it0 + 1.0;
    sc[S_ITERS_TOTAL] += 1.0;
    sc[S_DONE] = done ? 1.0 : 0.0;
  }
}

// ---------------------------------------------------------------------------
// The whole local CG of a site in one cooperative launch (FP64, slot capacity <= 64)
// ---------------------------------------------------------------------------
// The local product is M_eff v = sum_{b'} LM_{b'} V RA_{b'}^T, with V the local
// vector as a (2 b_k) x b_{k+1} matrix, LM_{b'} the rows of LM = LA_k A_k with MPO
// index b' and RA_{b'}[c][c'] = RA_{k+1}[(c, b')][c']. The G = W * RB workgroups of a
// chain split it into units (b', block of 32 rows (a, s')): a unit computes its
// 32 x b_{k+1} block of LM_{b'} V RA_{b'}^T on FP64 MFMA, with its LM and RA tiles
// resident in LDS for the whole solve, and stores it as slab b'. Every workgroup
// also owns a contiguous slice of the local vector, holds the CG state of that
// slice in registers and sums the slabs of its elements in b' order.
// The iteration is Jacobi-preconditioned CG in the Chronopoulos-Gear arrangement
// (both inner products of an iteration reduced together), with (u, A u) summed
// from the units' shares as the slabs are formed: two device-wide barriers per
// iteration. Inner products are per-workgroup partial sums added in
// workgroup order by every workgroup, so all take the same decisions and the
// result does not depend on scheduling. Stop rule and counters are those of
// k_cg_init / k_cg_step.
constexpr int PC_THREADS = 256;
constexpr int PC_RB = 32;           // rows (a, s') of a unit
constexpr int PC_CAP = 64;          // largest slot capacity of the one-launch path
constexpr int PC_PER = 8;           // slice elements per thread: 2 cx^2 / G <= 32 cx <= 8 * 256
constexpr int PC_MAXG = 256;        // workgroups per chain (flags and partial sums)
constexpr int PC_LDL = 2 * PC_CAP + 1, PC_LDU = PC_CAP + 1, PC_LDR = PC_CAP + 1, PC_LDT = PC_CAP + 1;
constexpr size_t PC_LDS =
    (size_t)(PC_RB * PC_LDL + 2 * PC_CAP * PC_LDU + PC_CAP * PC_LDR + PC_RB * PC_LDT) * sizeof(double);
constexpr int PC_FLAG = 32;         // unsigned ints between two workgroups' flags (128 bytes)
constexpr int PC_SPIN = 1 << 22;    // polls before a barrier wait is abandoned

// Barrier of the G workgroups of one chain: each publishes its epoch in its own
// flag after an agent-scope release of its writes; wavefront 0 of each polls all
// G flags, then acquires. A wait that outlasts PC_SPIN polls (or sees the chain's
// failure flag) sets the failure flag and returns false in every thread.
__device__ bool pc_barrier(unsigned* flags, int G, int bid, unsigned epoch, int* fail, int* bad) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0) __hip_atomic_store(&flags[bid * PC_FLAG], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    bool ok = true;
    for (int spins = 0;; ++spins) {
      bool mine = true;
      for (int i = lane; i < G; i += 64)
        mine = mine && (int)(__hip_atomic_load(&flags[i * PC_FLAG], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                             epoch) >= 0;
      if (__all(mine)) break;
      if (spins > PC_SPIN || __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        if (lane == 0) __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (lane == 0) *bad = ok ? 0 : 1;
  }
  __syncthreads();
  return *bad == 0;
}

// Sum of the G per-workgroup partials in slots[0 .. G), in a fixed order; every
// wavefront computes it, with identical bits in every workgroup.
__device__ __forceinline__ double pc_gsum(const double* slots, int G) {
  double v = 0.0;
  for (int i = threadIdx.x & 63; i < G; i += 64) v += slots[i];
  return wave_sum(v);
}

// Workgroup sums of three values (fixed order), returned to every thread.
__device__ __forceinline__ void pc_bsum3(double& a, double& b, double& c, double (*red)[PC_THREADS / 64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v[3] = {a, b, c};
  wave_sum_n<3>(v);
  __syncthreads();
  if (lane == 0) { red[0][wave] = v[0]; red[1][wave] = v[1]; red[2][wave] = v[2]; }
  __syncthreads();
  a = b = c = 0.0;
  for (int w = 0; w < PC_THREADS / 64; ++w) { a += red[0][w]; b += red[1][w]; c += red[2][w]; }
}

// Two 16 x 16 FP64 MFMA tiles sharing their A operand: acc0 += A B0, acc1 += A B1 over
// K (a multiple of 4), A read at a[kk] (row of the lane's tile row, step `as` per k),
// B0 at b[kk * ldb] and B1 sixteen columns further. The K loop runs in blocks of 16:
// all twelve LDS reads of a block are issued before its MFMAs, and even and odd
// k-steps accumulate separately (two chains per tile), summed at the end.
__device__ __forceinline__ void mfma_pair(const double* a, int as, const double* b, int ldb, int K, v4d& acc0,
                                          v4d& acc1) {
  v4d e0 = {0, 0, 0, 0}, e1 = {0, 0, 0, 0}, o0 = {0, 0, 0, 0}, o1 = {0, 0, 0, 0};
  int kk = 0;
  for (; kk + 16 <= K; kk += 16) {
    double av[4], b0[4], b1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = a[(kk + 4 * u) * as];
      b0[u] = b[(kk + 4 * u) * ldb];
      b1[u] = b[(kk + 4 * u) * ldb + 16];
    }
#pragma unroll
    for (int u = 0; u < 4; u += 2) {
      e0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b0[u], e0, 0, 0, 0);
      e1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b1[u], e1, 0, 0, 0);
      o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u + 1], b0[u + 1], o0, 0, 0, 0);
      o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u + 1], b1[u + 1], o1, 0, 0, 0);
    }
  }
  for (; kk < K; kk += 4) {
    const double av = a[kk * as], b0 = b[kk * ldb], b1 = b[kk * ldb + 16];
    e0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, e0, 0, 0, 0);
    e1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, e1, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) { acc0[v] = e0[v] + o0[v]; acc1[v] = e1[v] + o1[v]; }
}
// The same with B stored transposed (consecutive k contiguous): B0 of the lane at
// b[kk], B1 at b[boff + kk].
__device__ __forceinline__ void mfma_pair_t(const double* a, const double* b, int boff, int K, v4d& acc0,
                                            v4d& acc1) {
  v4d e0 = {0, 0, 0, 0}, e1 = {0, 0, 0, 0}, o0 = {0, 0, 0, 0}, o1 = {0, 0, 0, 0};
  int kk = 0;
  for (; kk + 16 <= K; kk += 16) {
    double av[4], b0[4], b1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = a[kk + 4 * u];
      b0[u] = b[kk + 4 * u];
      b1[u] = b[boff + kk + 4 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; u += 2) {
      e0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b0[u], e0, 0, 0, 0);
      e1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], b1[u], e1, 0, 0, 0);
      o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u + 1], b0[u + 1], o0, 0, 0, 0);
      o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u + 1], b1[u + 1], o1, 0, 0, 0);
    }
  }
  for (; kk < K; kk += 4) {
    const double av = a[kk], b0 = b[kk], b1 = b[boff + kk];
    e0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, e0, 0, 0, 0);
    e1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, e1, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) { acc0[v] = e0[v] + o0[v]; acc1[v] = e1[v] + o1[v]; }
}

__global__ void __launch_bounds__(PC_THREADS) k_cg_coop(SBatch sb, SGeo g, SLay l, int G, int first, double* cnt) {
  extern __shared__ double smem[];
  double* LMs = smem;                               // [PC_RB][PC_LDL]   rows of LM_{b'} of this unit
  double* Us = LMs + PC_RB * PC_LDL;                // [2 PC_CAP][PC_LDU] the operand V
  double* RAs = Us + 2 * PC_CAP * PC_LDU;           // [PC_CAP][PC_LDR]   RA_{b'}[c][c']
  double* Ts = RAs + PC_CAP * PC_LDR;               // [PC_RB][PC_LDT]    LM_{b'} V rows of this unit
  __shared__ double red[3][PC_THREADS / 64];
  __shared__ int bad;
  if ((int)blockIdx.y >= sb.n) return;
  const SChain& c = sb.c[blockIdx.y];
  const int bid = blockIdx.x, tid = threadIdx.x;
  const int k = g.k, cx = g.cx, n = 2 * cx * cx;
  const int nl = c.xb[k], nr = c.xb[k + 1], w2 = c.ab[k + 1];
  const int RB = (2 * cx + PC_RB - 1) / PC_RB;
  const int bp = bid / RB, rb = bid % RB;
  const bool unit = bp < w2 && rb * PC_RB < 2 * nl;
  double* sc = c.ws + l.sc;
  double* u = c.ws + l.pcu;
  double* P = c.ws + l.pcP;
  double* slots = c.ws + l.pcs;                     // [4][PC_MAXG]: rho, gamma, |b|^2, delta
  unsigned* flags = reinterpret_cast<unsigned*>(c.ws + l.pcf);
  unsigned* ep = reinterpret_cast<unsigned*>(c.ws + l.pce);
  int* fail = reinterpret_cast<int*>(ep + 1);
  unsigned epoch = ep[0];                           // written back by workgroup 0 at the end
  const double rn0_prev = sc[S_RN0], pmax_prev = sc[S_PMAX], iters_prev = sc[S_ITERS_TOTAL];
  double* X = c.x + (long)k * sl2(cx);
  const double* LM = c.ws + l.LM;
  const double* RA = c.ws + l.RA + (size_t)(k + 1) * l.env;

  // resident tiles of the unit (zero outside the actual bonds); every load of a
  // thread is issued before the first is waited for
  if (unit) {
    constexpr int NT = PC_RB * 2 * PC_CAP / PC_THREADS, NR = PC_CAP * PC_CAP / PC_THREADS;
    double tl[NT], tr[NR];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int e = tid + PC_THREADS * q, i = e / (2 * PC_CAP), j = e % (2 * PC_CAP), row = rb * PC_RB + i;
      tl[q] = (row < 2 * nl && j < 2 * nl) ? LM[((long)row * w2 + bp) * 2 * cx + j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int e = tid + PC_THREADS * q, cc = e / PC_CAP, cp = e % PC_CAP;
      tr[q] = (cc < nr && cp < nr) ? RA[((long)cc * w2 + bp) * cx + cp] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int e = tid + PC_THREADS * q;
      LMs[(e / (2 * PC_CAP)) * PC_LDL + e % (2 * PC_CAP)] = tl[q];
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int e = tid + PC_THREADS * q;
      RAs[(e / PC_CAP) * PC_LDR + e % PC_CAP] = tr[q];
    }
  }
  // the CG state of this workgroup's slice, in registers
  const int SL = (n + G - 1) / G, e0 = bid * SL, e1 = min(n, e0 + SL);
  double xr[PC_PER], rr[PC_PER], pr[PC_PER], sr[PC_PER], ur[PC_PER], wr[PC_PER], dr[PC_PER], br[PC_PER];
  bool ok[PC_PER];
#pragma unroll
  for (int j = 0; j < PC_PER; ++j) {
    const int e = e0 + tid + PC_THREADS * j;
    ok[j] = e < e1 && (e / (2 * cx)) < nl && (e % cx) < nr;
    xr[j] = ok[j] ? X[e] : 0.0;
    dr[j] = ok[j] ? c.ws[l.dinv + e] : 0.0;
    br[j] = ok[j] ? c.ws[l.beff + e] : 0.0;
    rr[j] = pr[j] = sr[j] = ur[j] = wr[j] = 0.0;
  }
  const int lane = tid & 63, wv = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int r0 = (wv & 1) * 16, c0 = (wv >> 1) * 32;
  // slabs of the unit: P[b'][(a, s')][c] <- (LM_{b'} V RA_{b'}^T)[rows of the unit];
  // returns this thread's share of the unit's part of (V, M_eff V)
  auto product = [&](const double* V) {
    double vav = 0.0;
    {
      // the operand into LDS: all 32 loads of a thread in flight at once
      constexpr int NU = 2 * PC_CAP * PC_CAP / PC_THREADS;
      double tv[NU];
#pragma unroll
      for (int q = 0; q < NU; ++q) {
        const int e = tid + PC_THREADS * q, j = e / PC_CAP, cc = e % PC_CAP;
        tv[q] = (j < 2 * nl && cc < nr) ? V[j * cx + cc] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < NU; ++q) {
        const int e = tid + PC_THREADS * q;
        Us[(e / PC_CAP) * PC_LDU + e % PC_CAP] = tv[q];
      }
    }
    __syncthreads();
    if (unit) {
      v4d a0, a1;
      mfma_pair(LMs + (r0 + li) * PC_LDL + lk, 1, Us + lk * PC_LDU + c0 + li, PC_LDU, (2 * nl + 3) & ~3, a0, a1);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Ts[(r0 + lk + 4 * v) * PC_LDT + c0 + li] = a0[v];
        Ts[(r0 + lk + 4 * v) * PC_LDT + c0 + 16 + li] = a1[v];
      }
    }
    __syncthreads();
    if (unit) {
      v4d a0, a1;
      mfma_pair_t(Ts + (r0 + li) * PC_LDT + lk, RAs + (c0 + li) * PC_LDR + lk, 16 * PC_LDR, (nr + 3) & ~3, a0, a1);
      double* Pb = P + (long)bp * n;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q = rb * PC_RB + r0 + lk + 4 * v;
        if (q < 2 * nl) {
          if (c0 + li < nr) {
            Pb[q * cx + c0 + li] = a0[v];
            vav += Us[q * PC_LDU + c0 + li] * a0[v];
          }
          if (c0 + 16 + li < nr) {
            Pb[q * cx + c0 + 16 + li] = a1[v];
            vav += Us[q * PC_LDU + c0 + 16 + li] * a1[v];
          }
        }
      }
    }
    return vav;
  };
  // sum of the slabs at element e in b' order, eight loads in flight at a time
  auto slab_total = [&](int e) {
    double v = 0.0;
    for (int b0 = 0; b0 < w2; b0 += 8) {
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = (b0 + q < w2) ? P[(long)(b0 + q) * n + e] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) v += t[q];
    }
    return v;
  };

  // r = b - A x, u = D r
  product(X);
  if (!pc_barrier(flags, G, bid, ++epoch, fail, &bad)) return;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
  for (int j = 0; j < PC_PER; ++j) {
    const int e = e0 + tid + PC_THREADS * j;
    if (ok[j]) {
      rr[j] = br[j] - slab_total(e);
      ur[j] = dr[j] * rr[j];
      t0 += rr[j] * rr[j]; t1 += rr[j] * ur[j]; t2 += br[j] * br[j];
    }
    if (e < e1) u[e] = ur[j];
  }
  pc_bsum3(t0, t1, t2, red);
  if (tid == 0) { slots[bid] = t0; slots[PC_MAXG + bid] = t1; slots[2 * PC_MAXG + bid] = t2; }
  if (!pc_barrier(flags, G, bid, ++epoch, fail, &bad)) return;
  const double rho0 = pc_gsum(slots, G);
  double gam = pc_gsum(slots + PC_MAXG, G);
  const double bn = pc_gsum(slots + 2 * PC_MAXG, G);
  const double thr = fmax(g.ltol * g.ltol * (first ? rho0 : rn0_prev), c.atol2);
  double rho = rho0, gam_prev = 0.0, alpha_prev = 0.0;
  int its = 0;
  bool done = (bn == 0.0 || rho0 <= thr || g.maxit <= 0);
  while (!done) {
    // w = A u in slabs; delta = (u, w) from the units' shares, published with the slabs
    double d0 = product(u), z1 = 0.0, z2 = 0.0;
    pc_bsum3(d0, z1, z2, red);
    if (tid == 0) slots[3 * PC_MAXG + bid] = d0;
    if (!pc_barrier(flags, G, bid, ++epoch, fail, &bad)) return;
#pragma unroll
    for (int j = 0; j < PC_PER; ++j)
      if (ok[j]) wr[j] = slab_total(e0 + tid + PC_THREADS * j);
    const double delta = pc_gsum(slots + 3 * PC_MAXG, G);
    const double beta = its == 0 ? 0.0 : gam / gam_prev;
    const double den = its == 0 ? delta : delta - beta * gam / alpha_prev;
    if (!(den > 0.0) || !(gam > 0.0)) break;      // breakdown (exact solution or loss of definiteness)
    const double alpha = gam / den;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
#pragma unroll
    for (int j = 0; j < PC_PER; ++j) {
      const int e = e0 + tid + PC_THREADS * j;
      if (ok[j]) {
        pr[j] = ur[j] + beta * pr[j];
        sr[j] = wr[j] + beta * sr[j];
        xr[j] += alpha * pr[j];
        rr[j] -= alpha * sr[j];
        ur[j] = dr[j] * rr[j];
        q0 += rr[j] * rr[j]; q1 += rr[j] * ur[j];
      }
      if (e < e1) u[e] = ur[j];
    }
    pc_bsum3(q0, q1, q2, red);
    if (tid == 0) { slots[bid] = q0; slots[PC_MAXG + bid] = q1; }
    if (!pc_barrier(flags, G, bid, ++epoch, fail, &bad)) return;
    rho = pc_gsum(slots, G);
    gam_prev = gam;
    gam = pc_gsum(slots + PC_MAXG, G);
    alpha_prev = alpha;
    ++its;
    done = rho <= thr || its >= g.maxit;
  }
#pragma unroll
  for (int j = 0; j < PC_PER; ++j)
    if (ok[j]) X[e0 + tid + PC_THREADS * j] = xr[j];
  if (bid == 0 && tid == 0) {
    sc[S_ITER] = its;
    sc[S_ITERS_TOTAL] = iters_prev + its;
    sc[S_RN2] = rho;
    sc[S_DONE] = 1.0;
    if (first) { sc[S_RN0] = rho0; sc[S_PMAX] = fmax(pmax_prev, rho0); }
    ep[0] = epoch;
    if (cnt) {
      // algorithmic work of the (its + 1) local products: LM V then (.) RA^T, actual bonds
      const double m1 = 2.0 * nl * w2, k1 = 2.0 * nl;
      const double fl = 2.0 * m1 * k1 * nr + 2.0 * (2.0 * nl) * ((double)w2 * nr) * nr;
      const double by = 8.0 * (m1 * k1 + k1 * nr + (double)w2 * nr * nr + 2.0 * nl * nr);
      atomicAdd(cnt, (its + 1) * fl);
      atomicAdd(cnt + 1, (its + 1) * by);
    }
  }
}

// Right-to-left gauge move at site k by Householder LQ (bond kept):
// Y_k (b_k x 2 b_{k+1}): Y_k^T = Q R  ->  core k <- Q^T, Y_{k-1} <- Y_{k-1} R^T.
template <int RPL, int CPW>
__global__ void __launch_bounds__(1024) k_rl_qr(SBatch sb, SGeo g, SLay l) {
  extern __shared__ double smem[];
  __shared__ double rdiag[512], tau[512], vbuf[1024];
  if (blockIdx.x >= sb.n) return;
  const SChain& c = sb.c[blockIdx.x];
  const int k = g.k, cap = g.cx;
  const int nb = c.xb[k], mb = c.xb[k + 1];
  const int m = 2 * mb, n = nb, r = m < n ? m : n;
  const bool fast = RPL > 0 && m <= 64 * RPL && n <= 16 * CPW;
  const size_t need = ((size_t)m * n + (fast ? 0 : (size_t)m * r)) * sizeof(double);
  // The budget passed in smem size is checked by the host; fall back to global scratch otherwise.
  double* X = (need <= (size_t)g.lds) ? smem : (c.ws + l.gp);
  double* Yk = c.x + (long)k * sl2(cap);
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
  // Y_{k-1} <- Y_{k-1} R^T  (R: r x n upper trapezoidal; R^T: n x r); rows (a0, s)
  const int np = c.xb[k - 1];
  double* Yp = c.x + (long)(k - 1) * sl2(cap);
  double* T = c.ws + l.tmpA;
  __syncthreads();
  auto la = [&](int rho, int t) { return Yp[(long)rho * cap + t]; };
  auto lb = [&](int t, int j) { return t == j ? rdiag[j] : (t > j ? X[(long)t * m + j] : 0.0); };
  wg_gemm_f64(2 * np, r, n, la, lb, T, cap);
  __syncthreads();
  stage8(S, [&](int e) { return (e / (2 * cap) < np && e % cap < r) ? T[e] : 0.0; },
         [&](int e, double v) { Yp[e] = v; });
  if (threadIdx.x == 0) c.xb[k] = r;
}

// Left-to-right gauge move at site k by Householder QR (bond kept):
// core k (2 b_k x b_{k+1}) = Q R -> core k <- Q, core k+1 <- R core k+1.
template <int RPL, int CPW>
__global__ void __launch_bounds__(1024) k_lr_qr_keep(SBatch sb, SGeo g, SLay l) {
  extern __shared__ double smem[];
  __shared__ double rdiag[512], tau[512], vbuf[1024];
  if (blockIdx.x >= sb.n) return;
  const SChain& c = sb.c[blockIdx.x];
  const int k = g.k, cap = g.cx;
  const int m = 2 * c.xb[k], n = c.xb[k + 1];
  const int r = m < n ? m : n;
  const bool fast = RPL > 0 && m <= 64 * RPL && n <= 16 * CPW;
  const size_t need = ((size_t)m * n + (fast ? 0 : (size_t)m * r)) * sizeof(double);
  double* X = (need <= (size_t)g.lds) ? smem : (c.ws + l.gp);
  double* Yk = c.x + (long)k * sl2(cap);
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
  // core k+1 <- R core k+1: rows j < r, columns (s, bb) contiguous
  double* Yn = c.x + (long)(k + 1) * sl2(cap);
  double* T = c.ws + l.tmpA;
  __syncthreads();
  auto la = [&](int j, int t) { return t == j ? rdiag[j] : (t > j ? X[(long)t * m + j] : 0.0); };
  auto lb = [&](int t, int nu) { return Yn[(long)t * 2 * cap + nu]; };
  wg_gemm_f64(r, 2 * cap, n, la, lb, T, 2 * cap);
  __syncthreads();
  stage8(S, [&](int e) { return (e / (2 * cap) < r) ? T[e] : 0.0; }, [&](int e, double v) { Yn[e] = v; });
  if (threadIdx.x == 0) c.xb[k + 1] = r;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Solver {
  SBatch sb;
  SGeo g;
  SLay l;
  int mode;
  hipStream_t s;
  int lds;

  GemmBatch batch(int maxb) const {
    GemmBatch gb;
    std::memset(&gb, 0, sizeof(gb));
    gb.n = sb.n;
    gb.maxb = maxb;
    return gb;
  }
  static void one(GemmJob& j) {
    j.nb = C_(1); j.sa = C_(0); j.sb = C_(0); j.sc = C_(0); j.skip = nullptr;
    j.alpha = 1.0; j.beta = 0.0;
  }
  // A table of GEMM jobs and the largest output extents its launch has to cover.
  struct JobSet {
    GemmBatch g;
    int M, N;
  };
  void run(const JobSet& j, int mmode) { run_jobs(j.g, j.M, j.N, mmode, s); }
  // Two independent FP64 job tables of one step: one launch when the kernel-argument
  // table holds both (each job keeps its own shapes; workgroups beyond a job's tiles
  // or batch count exit at once), otherwise one launch each.
  void run_pair(const JobSet& a, const JobSet& b) {
    if (a.g.n + b.g.n > GB) {
      run(a, 0);
      run(b, 0);
      return;
    }
    GemmBatch m = a.g;
    for (int i = 0; i < b.g.n; ++i) m.j[m.n + i] = b.g.j[i];
    m.n += b.g.n;
    m.maxb = std::max(a.g.maxb, b.g.maxb);
    run_jobs(m, std::max(a.M, b.M), std::max(a.N, b.N), 0, s);
  }

  // LA_{k+1} from LA_k (contraction of site k): LA[(a, b)][a'] with bra index a
  // (cap cx) and ket index a' (cap ck). Steps 1-2 are shared with the projection.
  JobSet la1(int k) const {
    const int ck = g.ck, W = g.W;
    GemmBatch g1 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      const double* LAk = c.ws + l.LA + (size_t)k * l.env;
      const double* Kk = c.kx + (size_t)k * ck * 2 * ck;
      GemmJob& a = g1.j[i]; one(a);    // F[(a,b)][(s,c')] = LA[(a,b)][a'] K[a'][(s,c')]
      a.A = LAk; a.ars = C_(ck); a.acs = C_(1);
      a.B = Kk; a.brs = C_(2 * ck); a.bcs = C_(1);
      a.C = c.ws + l.F1; a.crs = C_(2 * ck); a.ccs = C_(1);
      a.M = B2(c.xb, k, c.ab, k); a.N = C_(2 * ck); a.K = B1(c.kxb, k);
    }
    return {g1, g.cx * W, 2 * ck};
  }
  JobSet la2(int k) const {
    const int ck = g.ck, W = g.W;
    GemmBatch g2 = batch(g.cx);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      GemmJob& b = g2.j[i]; one(b);    // G[a][(s',b')][c'] = Mt[(s',b')][(b,s)] F[a][(b,s)][c']
      b.A = c.ws + l.Mt + (size_t)k * 4 * W * W; b.ars = B1(c.ab, k, 2); b.acs = C_(1);
      b.B = c.ws + l.F1; b.brs = C_(ck); b.bcs = C_(1);
      b.C = c.ws + l.F2; b.crs = C_(ck); b.ccs = C_(1);
      b.M = B1(c.ab, k + 1, 2); b.N = C_(ck); b.K = B1(c.ab, k, 2);
      b.nb = B1(c.xb, k); b.sb = B1(c.ab, k, 2 * ck); b.sc = B1(c.ab, k + 1, 2 * ck);
    }
    return {g2, 2 * W, ck};
  }
  void la_steps12(int k, int mmode) {
    run(la1(k), mmode);
    run(la2(k), mmode);
  }
  // LA_{k+1}[p][(b', q)] = sum_{(a, s')} X_k[(a, s')][p] G[(a, s')][(b', q)]
  JobSet la3(int k) const {
    const int cx = g.cx, ck = g.ck, W = g.W;
    GemmBatch g3 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      GemmJob& d = g3.j[i]; one(d);
      d.A = c.x + (size_t)k * cx * 2 * cx; d.ars = C_(1); d.acs = C_(cx);
      d.B = c.ws + l.F2; d.brs = B1(c.ab, k + 1, ck); d.bcs = C_(1);
      d.C = c.ws + l.LA + (size_t)(k + 1) * l.env; d.crs = B1(c.ab, k + 1, ck); d.ccs = C_(1);
      d.M = B1(c.xb, k + 1); d.N = B1(c.ab, k + 1, ck); d.K = B1(c.xb, k, 2);
    }
    return {g3, cx, W * ck};
  }
  void la_step3(int k, int mmode) { run(la3(k), mmode); }

  // RA_k from RA_{k+1}: RA[(c, b)][c'] with bra index c (cap cx), ket index c' (cap ck)
  JobSet ra1(int k) const {
    const int cx = g.cx, ck = g.ck, W = g.W;
    GemmBatch g1 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      const double* RAn = c.ws + l.RA + (size_t)(k + 1) * l.env;
      const double* Xk = c.x + (size_t)k * cx * 2 * cx;
      GemmJob& a = g1.j[i]; one(a);    // F[(c,s')][(b',d')] = X[(c,s')][d] RA[d][(b',d')]
      a.A = Xk; a.ars = C_(cx); a.acs = C_(1);
      a.B = RAn; a.brs = B1(c.ab, k + 1, ck); a.bcs = C_(1);
      a.C = c.ws + l.F1; a.crs = B1(c.ab, k + 1, ck); a.ccs = C_(1);
      a.M = B1(c.xb, k, 2); a.N = B1(c.ab, k + 1, ck); a.K = B1(c.xb, k + 1);
    }
    return {g1, 2 * cx, W * ck};
  }
  JobSet ra2(int k) const {
    const int cx = g.cx, ck = g.ck, W = g.W;
    GemmBatch g2 = batch(cx);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      GemmJob& b = g2.j[i]; one(b);    // G[c][(b,s)][d'] = Mt2[(b,s)][(s',b')] F[c][(s',b')][d']
      b.A = c.ws + l.Mt2 + (size_t)k * 4 * W * W; b.ars = B1(c.ab, k + 1, 2); b.acs = C_(1);
      b.B = c.ws + l.F1; b.brs = C_(ck); b.bcs = C_(1);
      b.C = c.ws + l.F2; b.crs = C_(ck); b.ccs = C_(1);
      b.M = B1(c.ab, k, 2); b.N = C_(ck); b.K = B1(c.ab, k + 1, 2);
      b.nb = B1(c.xb, k); b.sb = B1(c.ab, k + 1, 2 * ck); b.sc = B1(c.ab, k, 2 * ck);
    }
    return {g2, 2 * W, ck};
  }
  JobSet ra3(int k) const {
    const int cx = g.cx, ck = g.ck, W = g.W;
    GemmBatch g3 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      double* RAk = c.ws + l.RA + (size_t)k * l.env;
      const double* Kk = c.kx + (size_t)k * ck * 2 * ck;
      GemmJob& d = g3.j[i]; one(d);    // RA_k[(c,b)][c'] = G[(c,b)][(s,d')] K[c'][(s,d')]
      d.A = c.ws + l.F2; d.ars = C_(2 * ck); d.acs = C_(1);
      d.B = Kk; d.brs = C_(1); d.bcs = C_(2 * ck);
      d.C = RAk; d.crs = C_(ck); d.ccs = C_(1);
      d.M = B2(c.xb, k, c.ab, k); d.N = B1(c.kxb, k); d.K = C_(2 * ck);
    }
    return {g3, cx * W, ck};
  }
  void ra_update(int k, int mmode = 0) {
    run(ra1(k), mmode);
    run(ra2(k), mmode);
    run(ra3(k), mmode);
  }

  // Variational projection of M x onto the frame of the bra at site k:
  // X_k <- LA_k M_k K_k RA_{k+1} (leaves G = M_k T[a] in F2 for la_step3). The last
  // product is split over K into slabs, summed into X_k in split order.
  void project(int k, int mmode) {
    const int cx = g.cx, ck = g.ck, W = g.W;
    la_steps12(k, mmode);
    const long sl = 2L * cx * cx;
    GemmBatch g3 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      GemmJob& d = g3.j[i]; one(d);    // X[(a,s')][c] = G[(a,s')][(b',c')] RA[c][(b',c')]
      d.A = c.ws + l.F2; d.ars = B1(c.ab, k + 1, ck); d.acs = C_(1);
      d.B = c.ws + l.RA + (size_t)(k + 1) * l.env; d.brs = C_(1); d.bcs = B1(c.ab, k + 1, ck);
      d.C = c.ws + l.slab; d.crs = C_(cx); d.ccs = C_(1);
      d.M = B1(c.xb, k, 2); d.N = B1(c.xb, k + 1); d.K = B1(c.ab, k + 1, ck);
    }
    g3.ksplit = ksplit_for(2 * cx, cx, W * ck);
    g3.slab = sl;
    run_jobs(g3, 2 * cx, cx, mmode, s);
    SlabSum z;
    std::memset(&z, 0, sizeof(z));
    z.n = sb.n; z.nq = g3.ksplit; z.k = k; z.cap = cx; z.slab = sl;
    for (int i = 0; i < sb.n; ++i) {
      z.dst[i] = sb.c[i].x + (size_t)k * cx * 2 * cx;
      z.src[i] = sb.c[i].ws + l.slab;
      z.bond[i] = sb.c[i].xb;
    }
    slab_sum(z, s);
  }

  JobSet lb1(int k) const {
    const int cx = g.cx, cb = g.cb;
    GemmBatch g1 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      const double* Bk = c.b + (size_t)k * cb * 2 * cb;
      GemmJob& a = g1.j[i]; one(a);    // F[a][(s,g)] = Lb[a][al] B[al][(s,g)]
      a.A = c.ws + l.Lb + (size_t)k * l.envb; a.ars = C_(cb); a.acs = C_(1);
      a.B = Bk; a.brs = C_(2 * cb); a.bcs = C_(1);
      a.C = c.ws + l.F3; a.crs = C_(2 * cb); a.ccs = C_(1);
      a.M = B1(c.xb, k); a.N = C_(2 * cb); a.K = B1(c.bb, k);
    }
    return {g1, cx, 2 * cb};
  }
  JobSet lb2(int k) const {
    const int cx = g.cx, cb = g.cb;
    GemmBatch g2 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      const double* Xk = c.x + (size_t)k * cx * 2 * cx;
      GemmJob& b = g2.j[i]; one(b);    // Lb'[p][g] = X[(a,s)][p] F[(a,s)][g]
      b.A = Xk; b.ars = C_(1); b.acs = C_(cx);
      b.B = c.ws + l.F3; b.brs = C_(cb); b.bcs = C_(1);
      b.C = c.ws + l.Lb + (size_t)(k + 1) * l.envb; b.crs = C_(cb); b.ccs = C_(1);
      b.M = B1(c.xb, k + 1); b.N = B1(c.bb, k + 1); b.K = B1(c.xb, k, 2);
    }
    return {g2, cx, cb};
  }

  JobSet rb1(int k) const {
    const int cx = g.cx, cb = g.cb;
    GemmBatch g1 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      const double* Bk = c.b + (size_t)k * cb * 2 * cb;
      GemmJob& a = g1.j[i]; one(a);    // F[(al,s)][d] = B[(al,s)][g] Rb[d][g]
      a.A = Bk; a.ars = C_(cb); a.acs = C_(1);
      a.B = c.ws + l.Rb + (size_t)(k + 1) * l.envb; a.brs = C_(1); a.bcs = C_(cb);
      a.C = c.ws + l.F3; a.crs = C_(cx); a.ccs = C_(1);
      a.M = B1(c.bb, k, 2); a.N = B1(c.xb, k + 1); a.K = B1(c.bb, k + 1);
    }
    return {g1, 2 * cb, cx};
  }
  JobSet rb2(int k) const {
    const int cx = g.cx, cb = g.cb;
    GemmBatch g2 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      const double* Xk = c.x + (size_t)k * cx * 2 * cx;
      GemmJob& b = g2.j[i]; one(b);    // Rb[c][al] = X[c][(s,d)] F[(al,s)][d]
      b.A = Xk; b.ars = C_(2 * cx); b.acs = C_(1);
      b.B = c.ws + l.F3; b.brs = C_(1); b.bcs = C_(2 * cx);
      b.C = c.ws + l.Rb + (size_t)k * l.envb; b.crs = C_(cb); b.ccs = C_(1);
      b.M = B1(c.xb, k); b.N = B1(c.bb, k); b.K = C_(2 * cx);
    }
    return {g2, cx, cb};
  }
  // The operator and right-hand-side environments of a site (FP64) do not depend on
  // each other (F1/F2 and F3 are separate buffers): their first and second steps
  // share launches, three launches instead of five.
  void left_envs(int k) {
    run_pair(la1(k), lb1(k));
    run_pair(la2(k), lb2(k));
    run(la3(k), 0);
  }
  void right_envs(int k) {
    run_pair(ra1(k), rb1(k));
    run_pair(ra2(k), rb2(k));
    run(ra3(k), 0);
  }

  void beff(int k) {
    const int cx = g.cx, cb = g.cb;
    GemmBatch g1 = batch(1), g2 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      const double* Bk = c.b + (size_t)k * cb * 2 * cb;
      GemmJob& a = g1.j[i]; one(a);
      a.A = c.ws + l.Lb + (size_t)k * l.envb; a.ars = C_(cb); a.acs = C_(1);
      a.B = Bk; a.brs = C_(2 * cb); a.bcs = C_(1);
      a.C = c.ws + l.F3; a.crs = C_(2 * cb); a.ccs = C_(1);
      a.M = B1(c.xb, k); a.N = C_(2 * cb); a.K = B1(c.bb, k);
      GemmJob& b = g2.j[i]; one(b);    // beff[(a,s)][c] = F[(a,s)][g] Rb[c][g]
      b.A = c.ws + l.F3; b.ars = C_(cb); b.acs = C_(1);
      b.B = c.ws + l.Rb + (size_t)(k + 1) * l.envb; b.brs = C_(1); b.bcs = C_(cb);
      b.C = c.ws + l.beff; b.crs = C_(cx); b.ccs = C_(1);
      b.M = B1(c.xb, k, 2); b.N = B1(c.xb, k + 1); b.K = B1(c.bb, k + 1);
    }
    run_jobs(g1, cx, 2 * cb, 0, s);
    run_jobs(g2, 2 * cx, cx, 0, s);
  }

  // LM[(a, s', b')][(a', s)] = sum_b LA_k[a][b][a'] A_k[b][s'][s][b'] (left environment
  // times the MPO core), once per local problem: the local product is then two GEMMs.
  void build_lm(int k) {
    const int cx = g.cx, W = g.W;
    for (int i = 0; i < 2; ++i) {
      GemmBatch gb = batch(cx);
      for (int q = 0; q < sb.n; ++q) {
        const SChain& c = sb.c[q];
        GemmJob& j = gb.j[q]; one(j);    // per a: LM_a[(s',b')][a'] (input index s = i) = Mt_i[(s',b')][b] LA_a[b][a']
        j.A = c.ws + l.Mt + (size_t)k * 4 * W * W + i; j.ars = B1(c.ab, k, 2); j.acs = C_(2);
        j.B = c.ws + l.LA + (size_t)k * l.env; j.brs = C_(cx); j.bcs = C_(1);
        j.C = c.ws + l.LM + i; j.crs = C_(2 * cx); j.ccs = C_(2);
        j.M = B1(c.ab, k + 1, 2); j.N = B1(c.xb, k); j.K = B1(c.ab, k);
        j.nb = B1(c.xb, k); j.sb = B1(c.ab, k, cx); j.sc = B1(c.ab, k + 1, 4 * cx);
      }
      run_jobs(gb, 2 * W, cx, 0, s);
    }
  }

  // out = M_eff v at site k (v, out: [a][s][c], row stride cx): T = LM v, then
  // out = T RA, the last product split over K (g.mvs > 1) into slabs that the CG
  // kernels sum in split order as they read them.
  void matvec(int k, bool v_is_x, int mmode) {
    const int cx = g.cx, W = g.W;
    GemmBatch g1 = batch(1), g3 = batch(1);
    for (int i = 0; i < sb.n; ++i) {
      const SChain& c = sb.c[i];
      const double* v = v_is_x ? (c.x + (size_t)k * cx * 2 * cx) : (c.ws + l.p);
      const double* skip = v_is_x ? nullptr : (c.ws + l.sc + S_DONE);
      GemmJob& a = g1.j[i]; one(a);    // T[(a,s',b')][c'] = LM[(a,s',b')][(a',s)] v[(a',s)][c']
      a.A = c.ws + l.LM; a.ars = C_(2 * cx); a.acs = C_(1);
      a.B = v; a.brs = C_(cx); a.bcs = C_(1);
      a.C = c.ws + l.F2; a.crs = C_(cx); a.ccs = C_(1);
      a.M = B2(c.xb, k, c.ab, k + 1, 2); a.N = C_(cx); a.K = B1(c.xb, k, 2);
      a.skip = skip;
      GemmJob& d = g3.j[i]; one(d);    // out[(a,s')][c] = T[(a,s')][(b',c')] RA[c][(b',c')]
      d.A = c.ws + l.F2; d.ars = B1(c.ab, k + 1, cx); d.acs = C_(1);
      d.B = c.ws + l.RA + (size_t)(k + 1) * l.env; d.brs = C_(1); d.bcs = B1(c.ab, k + 1, cx);
      d.C = c.ws + l.Ap; d.crs = C_(cx); d.ccs = C_(1);
      d.M = B1(c.xb, k, 2); d.N = B1(c.xb, k + 1); d.K = B1(c.ab, k + 1, cx);
      d.skip = skip;
    }
    g3.ksplit = g.mvs;
    g3.slab = 2L * cx * cx;
    run_jobs(g1, cx * 2 * W, cx, mmode, s);
    run_jobs(g3, 2 * cx, cx, mmode, s);
  }

  // Local CG at site k. Iterations are enqueued in chunks of growing length; after
  // each chunk the host reads the per-chain convergence flags (one small copy) and
  // stops enqueuing once every chain has converged. Kernels of converged chains
  // exit at once, so the chunking changes the launch count, not the arithmetic.
  // With a low-precision matvec (mmode != 0) the solve is restarted from the FP64
  // residual r = b_eff - M_eff x a few times (iterative refinement): the MFMA
  // products only have to reduce the error of each correction, while the residual
  // that decides convergence is always exact to FP64.
  double* flags = nullptr;   // host pinned, GB entries
  bool flag_copy_failed = false;   // a failed flag read stops the enqueuing; the sweep reports it
  int coopG = 0;             // workgroups per chain of the one-launch local CG (0: not used)
  bool coop_failed = false;  // a cooperative launch was refused; the sweep reports it
  void local_solve(int k, int mmode) {
    SGeo gg = g;
    gg.k = k;
    beff(k);
    build_lm(k);
    if (g.W <= PD_W && g.cx <= PD_C)
      hipLaunchKernelGGL(k_precond_fact, dim3((2 * g.cx + PD_RB - 1) / PD_RB, sb.n), dim3(256), 0, s, sb, gg, l);
    else hipLaunchKernelGGL(k_precond, dim3(8, sb.n), dim3(256), 0, s, sb, gg, l);
    if (mmode == 0 && coopG > 0) {
      int first = 1, G = coopG;
      double* cnt = nullptr;
      qttk::tmark(KC_CG_COOP, s);
      cnt = qttk::tcount(KC_CG_COOP);
      void* args[] = {(void*)&sb, (void*)&gg, (void*)&l, (void*)&G, (void*)&first, (void*)&cnt};
      if (hipLaunchCooperativeKernel((const void*)k_cg_coop, dim3(G, sb.n), dim3(PC_THREADS), args, PC_LDS, s) !=
          hipSuccess)
        coop_failed = true;
      qttk::tmark(KC_CG_COOP, s);
      return;
    }
    const int reps = (mmode == 0) ? 1 : 4;
    const int per = std::max(1, g.maxit / reps);
    gg.maxit = per;
    for (int rep = 0; rep < reps; ++rep) {
      matvec(k, true, 0);
      hipLaunchKernelGGL(k_cg_init, dim3(sb.n), dim3(1024), 0, s, sb, gg, l, rep == 0 ? 1 : 0);
      cg_iterations(gg, k, mmode, per);
    }
  }
  void cg_iterations(const SGeo& gg, int k, int mmode, int maxit) {
    int it = 0, chunk = 4;
    while (it < maxit) {
      const int m = std::min(chunk, maxit - it);
      for (int j = 0; j < m; ++j) {
        matvec(k, false, mmode);
        qttk::tmark(KC_CG, s);
        hipLaunchKernelGGL(k_cg_step, dim3(sb.n), dim3(1024), 0, s, sb, gg, l);
        qttk::tmark(KC_CG, s);
      }
      it += m;
      chunk = std::min(2 * chunk, 64);
      if (it >= maxit || !flags) break;
      bool ok = true;
      for (int i = 0; i < sb.n; ++i)
        ok = ok && hipMemcpyAsync(flags + i, sb.c[i].ws + l.sc + S_DONE, sizeof(double), hipMemcpyDeviceToHost,
                                  s) == hipSuccess;
      ok = ok && hipStreamSynchronize(s) == hipSuccess;
      if (!ok) {
        flag_copy_failed = true;
        break;
      }
      bool all = true;
      for (int i = 0; i < sb.n; ++i) all = all && flags[i] != 0.0;
      if (all) break;
    }
  }

  void lr_move(int k) {
    SGeo gg = g;
    gg.k = k;
    qttk::tmark(KC_LR_QR, s);
    if (g.cx <= 64) hipLaunchKernelGGL((k_lr_qr_keep<2, 4>), dim3(sb.n), dim3(1024), lds, s, sb, gg, l);
    else if (g.cx <= 128) hipLaunchKernelGGL((k_lr_qr_keep<4, 8>), dim3(sb.n), dim3(1024), lds, s, sb, gg, l);
    else hipLaunchKernelGGL((k_lr_qr_keep<0, 0>), dim3(sb.n), dim3(1024), lds, s, sb, gg, l);
    qttk::tmark(KC_LR_QR, s);
  }
  void rl_move(int k) {
    SGeo gg = g;
    gg.k = k;
    qttk::tmark(KC_LR_QR, s);
    if (g.cx <= 64) hipLaunchKernelGGL((k_rl_qr<2, 4>), dim3(sb.n), dim3(1024), lds, s, sb, gg, l);
    else if (g.cx <= 128) hipLaunchKernelGGL((k_rl_qr<4, 8>), dim3(sb.n), dim3(1024), lds, s, sb, gg, l);
    else hipLaunchKernelGGL((k_rl_qr<0, 0>), dim3(sb.n), dim3(1024), lds, s, sb, gg, l);
    qttk::tmark(KC_LR_QR, s);
  }
};

}  // namespace

// residual helpers implemented with the public dot entry points
extern "C" int qtt_poisson_solve(qtt_ctx* ctx, int n, const qtt_mpo* A, const qtt_mps* b, qtt_mps* x,
                                 const qtt_solve_opts* opts, qtt_solve_info* info, void* stream);

namespace qtt_solver_detail {
// Declared in api.hip: workspace access for the solver.
double* solver_ws(qtt_ctx* ctx, size_t doubles, int* rc);
int set_error(qtt_ctx* ctx, int code, const char* msg);
int lds_of(qtt_ctx* ctx);
int coop_of(qtt_ctx* ctx);
double* pinned(qtt_ctx* ctx, size_t doubles, int* rc);
}

namespace qtt_solver_detail {
hipError_t solver_init(int lds) {
  const void* fns[] = {(const void*)k_rl_qr<2, 4>, (const void*)k_rl_qr<4, 8>, (const void*)k_rl_qr<0, 0>,
                       (const void*)k_lr_qr_keep<2, 4>, (const void*)k_lr_qr_keep<4, 8>, (const void*)k_lr_qr_keep<0, 0>};
  hipError_t e = hipSuccess;
  for (const void* f : fns)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_cg_coop, hipFuncAttributeMaxDynamicSharedMemorySize, (int)PC_LDS);
  return e;
}

// Workgroups of the one-launch local CG that can be resident at once on `device`
// (0 if the device cannot launch it cooperatively).
int coop_capacity(int device) {
  int coop = 0, per_cu = 0, cus = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_cg_coop, PC_THREADS, PC_LDS) != hipSuccess)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return per_cu * cus;
}
}

extern "C" int qtt_poisson_solve(qtt_ctx* ctx, int n, const qtt_mpo* A, const qtt_mps* b, qtt_mps* x,
                                 const qtt_solve_opts* opts, qtt_solve_info* info, void* stream) {
  using namespace qtt_solver_detail;
  if (!ctx) return QTT_EINVAL;
  if (n < 1 || !A || !b || !x || !opts) return set_error(ctx, QTT_EINVAL, "solve: bad arguments");
  if (opts->contract_dt < QTT_F64 || opts->contract_dt > QTT_BF16 || opts->max_sweeps < 0 || opts->max_local_iters < 0)
    return set_error(ctx, QTT_EINVAL, "solve: bad options");
  const int L = x[0].L, cx = x[0].cap, cb = b[0].cap, wcap = A[0].wcap;
  int W = 1;
  for (int i = 0; i < n; ++i) {
    if (!x[i].data || !x[i].bond || !b[i].data || !b[i].bond || !A[i].data || !A[i].bond || !A[i].bond_host)
      return set_error(ctx, QTT_EINVAL, "solve: null pointer");
    if (x[i].L != L || b[i].L != L || A[i].L != L || x[i].cap != cx || b[i].cap != cb || A[i].wcap != wcap ||
        x[i].d != 2 || b[i].d != 2)
      return set_error(ctx, QTT_ESHAPE, "solve: problems must share L, d and capacities");
    for (int k = 0; k <= L; ++k) W = std::max(W, A[i].bond_host[k]);
  }
  if (L < 2 || cx > 256 || cb > 512 || W > wcap) return set_error(ctx, QTT_ESHAPE, "solve: unsupported sizes");
  hipStream_t s = (hipStream_t)stream;
  const SLay lay = SLay::make(L, cx, cx, cb, W);
  int rc = 0;
  double* ws = solver_ws(ctx, lay.total * std::min(n, GB), &rc);
  if (rc) return rc;
  const int lds = lds_of(ctx);
  int status = QTT_OK;
  for (int i0 = 0; i0 < n; i0 += GB) {
    Solver S;
    S.sb.n = std::min(GB, n - i0);
    for (int i = 0; i < S.sb.n; ++i) {
      SChain& c = S.sb.c[i];
      c.A = A[i0 + i].data; c.ab = A[i0 + i].bond;
      c.b = b[i0 + i].data; c.bb = b[i0 + i].bond;
      c.x = x[i0 + i].data; c.xb = x[i0 + i].bond;
      c.kx = c.x; c.kxb = c.xb;
      c.ws = ws + lay.total * i;
    }
    S.g = SGeo{L, 0, cx, cb, wcap, W, cx, opts->local_tol, opts->max_local_iters, lds};
    S.g.mvs = ksplit_for(2 * cx, cx, W * cx);
    S.l = lay;
    S.mode = opts->contract_dt;
    S.s = s;
    S.lds = lds;
    S.flags = nullptr;
    {
      // one-launch local CG: FP64 products, slot capacity <= 64, all workgroups resident
      const int G = W * ((2 * cx + PC_RB - 1) / PC_RB);
      if (opts->contract_dt == QTT_F64 && cx <= PC_CAP && G <= PC_MAXG && G * S.sb.n <= coop_of(ctx)) S.coopG = G;
    }
    hipLaunchKernelGGL(k_transposes, dim3(L, S.sb.n), dim3(256), 0, s, S.sb, S.g, lay);
    hipLaunchKernelGGL(k_env_init, dim3(S.sb.n), dim3(256), 0, s, S.sb, S.g, lay);
    // right-canonical start (bond structure kept), right environments
    for (int k = L - 1; k >= 1; --k) S.rl_move(k);
    for (int k = L - 1; k >= 1; --k) S.right_envs(k);

    // ||b||^2 once (FP64); the absolute floor of each local residual is a share of
    // the global target
    double bb[GB], res[GB], best[GB];
    {
      std::vector<qtt_mps> bs(S.sb.n);
      for (int i = 0; i < S.sb.n; ++i) bs[i] = b[i0 + i];
      if ((rc = qtt_dot(ctx, S.sb.n, bs.data(), bs.data(), bb, stream))) return rc;
    }
    for (int i = 0; i < S.sb.n; ++i) {
      S.sb.c[i].atol2 = opts->tol * opts->tol * bb[i] / (4.0 * L);
      res[i] = best[i] = INFINITY;
      if (info) { info[i0 + i].residual0 = NAN; info[i0 + i].residual = NAN; info[i0 + i].sweeps = 0; }
    }
    // b = 0: the solution is the zero train. Its local problems have b_eff = 0 and stop
    // at once, so x is zeroed here (a zero core keeps the train zero through the gauge
    // moves, which pass R = 0 on to the neighbour).
    {
      ZeroList z{0, (long)L * cx * 2 * cx, {}};
      for (int i = 0; i < S.sb.n; ++i)
        if (bb[i] == 0.0) z.p[z.n++] = S.sb.c[i].x;
      zero_list(z, s);
    }
    double* pmax = pinned(ctx, 3 * GB + 8 * (size_t)n, &rc);   // residuals, CG flags, local CG failure words
    if (rc) return rc;
    S.flags = pmax + GB;
    int sweeps = 0;
    bool all_done = false;
    while (!all_done && sweeps < opts->max_sweeps) {
      hipLaunchKernelGGL(k_sweep_reset, dim3(S.sb.n), dim3(64), 0, s, S.sb, lay);
      // left-to-right half sweep
      for (int k = 0; k < L; ++k) {
        S.local_solve(k, S.mode);
        if (k < L - 1) {
          S.lr_move(k);
          S.left_envs(k);
        }
      }
      // right-to-left half sweep
      for (int k = L - 1; k >= 1; --k) {
        S.rl_move(k);
        S.right_envs(k);
        S.local_solve(k - 1, S.mode);
      }
      ++sweeps;
      if (S.flag_copy_failed) return set_error(ctx, QTT_EHIP, "solve: copy of the CG flags failed");
      if (S.coop_failed) return set_error(ctx, QTT_EHIP, "solve: cooperative launch of the local CG refused");
      for (int i = 0; i < S.sb.n; ++i)
        if (hipMemcpyAsync(pmax + i, S.sb.c[i].ws + lay.sc + S_PMAX, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(pmax + 2 * GB + i, S.sb.c[i].ws + lay.pce, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
          return set_error(ctx, QTT_EHIP, "solve: copy of the residual failed");
      if (hipStreamSynchronize(s) != hipSuccess) return set_error(ctx, QTT_EHIP, "solve: stream sync failed");
      for (int i = 0; i < S.sb.n; ++i) {
        unsigned ef[2];
        std::memcpy(ef, pmax + 2 * GB + i, sizeof(ef));
        if (ef[1] != 0u) return set_error(ctx, QTT_EHIP, "solve: a barrier wait of the local CG timed out");
      }
      all_done = true;
      bool improving = false;
      for (int i = 0; i < S.sb.n; ++i) {
        res[i] = bb[i] > 0.0 ? std::sqrt(pmax[i] / bb[i]) : 0.0;
        all_done = all_done && res[i] <= opts->tol;
        if (res[i] < 0.9 * best[i]) improving = true;
        best[i] = std::min(best[i], res[i]);
        if (info) {
          if (sweeps == 1) info[i0 + i].residual0 = res[i];
          info[i0 + i].residual = res[i];
          info[i0 + i].sweeps = sweeps;
        }
      }
      if (sweeps >= 2 && !improving) break;   // stagnated at the bond-limited floor
    }
    // total local iterations
    double* pin = pinned(ctx, 8 * (size_t)n, &rc);
    if (rc) return rc;
    for (int i = 0; i < S.sb.n; ++i)
      if (hipMemcpyAsync(pin + i, S.sb.c[i].ws + lay.sc + S_ITERS_TOTAL, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
        return set_error(ctx, QTT_EHIP, "solve: copy of counters failed");
    if (hipStreamSynchronize(s) != hipSuccess) return set_error(ctx, QTT_EHIP, "solve: stream sync failed");
    for (int i = 0; i < S.sb.n; ++i) {
      if (info) info[i0 + i].local_iters = (int)pin[i];
      if (!std::isfinite(res[i]) || !std::isfinite(bb[i])) status = QTT_ENUMERIC;
      else if (res[i] > opts->tol && status == QTT_OK) status = QTT_ENOTCONVERGED;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ctx, QTT_EHIP, hipGetErrorString(e));
  if (status == QTT_ENOTCONVERGED) set_error(ctx, QTT_ENOTCONVERGED, "solve: tolerance not reached");
  return status;
}

// ---------------------------------------------------------------------------
// variational fitting of y ~ M x (single-site, fixed bonds): each site update is
// the exact projection of M x onto the orthonormal frame of the other cores of y,
// so ||y - M x|| decreases monotonically (the variational mat-vec of Sec. 2.2).
// y must be right-canonical on entry and is right-canonical on exit.
// ---------------------------------------------------------------------------
namespace qtt_solver_detail {
int fit_sweeps(qtt_ctx* ctx, int n, const qtt_mpo* M, const qtt_mps* x, qtt_mps* y, int sweeps, int mode,
               void* stream) {
  if (sweeps <= 0) return QTT_OK;
  const int L = x[0].L, cx = y[0].cap, ck = x[0].cap, wcap = M[0].wcap;
  int W = 1;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k <= L; ++k) W = std::max(W, M[i].bond_host[k]);
  hipStream_t s = (hipStream_t)stream;
  const SLay lay = SLay::make(L, cx, ck, 1, W);
  int rc = 0;
  double* ws = solver_ws(ctx, lay.total * std::min(n, GB), &rc);
  if (rc) return rc;
  for (int i0 = 0; i0 < n; i0 += GB) {
    Solver S;
    S.sb.n = std::min(GB, n - i0);
    for (int i = 0; i < S.sb.n; ++i) {
      SChain& c = S.sb.c[i];
      std::memset(&c, 0, sizeof(c));
      c.A = M[i0 + i].data; c.ab = M[i0 + i].bond;
      c.x = y[i0 + i].data; c.xb = y[i0 + i].bond;
      c.kx = x[i0 + i].data; c.kxb = x[i0 + i].bond;
      c.ws = ws + lay.total * i;
    }
    S.g = SGeo{L, 0, cx, 1, wcap, W, ck, 0.0, 0, lds_of(ctx)};
    S.g.mvs = 1;
    S.l = lay;
    S.mode = mode;
    S.s = s;
    S.lds = lds_of(ctx);
    S.flags = nullptr;
    hipLaunchKernelGGL(k_transposes, dim3(L, S.sb.n), dim3(256), 0, s, S.sb, S.g, lay);
    hipLaunchKernelGGL(k_env_init, dim3(S.sb.n), dim3(256), 0, s, S.sb, S.g, lay);
    for (int k = L - 1; k >= 1; --k) S.ra_update(k, mode);
    for (int sw = 0; sw < sweeps; ++sw) {
      for (int k = 0; k <= L - 2; ++k) {
        S.project(k, mode);
        S.lr_move(k);
        S.la_step3(k, mode);
      }
      for (int k = L - 1; k >= 1; --k) {
        S.project(k, mode);
        S.rl_move(k);
        S.ra_update(k, mode);
      }
    }
    S.project(0, mode);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(ctx, QTT_EHIP, hipGetErrorString(e));
  return QTT_OK;
}
}  // namespace qtt_solver_detail
