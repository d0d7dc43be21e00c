// C-ABI entry points (include/qtt.h): validation, workspace management and the
// site-by-site orchestration of the kernels in kernels.hip.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qtt.h"
#include "host_linalg.h"
#include "internal.h"

namespace qtt_solver_detail {
hipError_t solver_init(int lds);
int coop_capacity(int device);
hipError_t fit_init(int lds);
int fit_sweeps(qtt_ctx* ctx, int n, const qtt_mpo* M, const qtt_mps* x, qtt_mps* y, int sweeps, int mode,
               void* stream);
}

struct qtt_ctx {
  int device = 0;
  int lds = 64 * 1024;
  int coop = 0;                // workgroups of the one-launch local CG resident at once (0: unavailable)
  double* scratch = nullptr;   // this device's copy of the file-scope scratch array (qtt_dot_noalloc)
  std::string err;
  double* ws = nullptr;        // chain workspaces (device)
  size_t ws_cap = 0;           // doubles
  double* tmp = nullptr;       // temporary trains (device)
  size_t tmp_cap = 0;          // bytes
  double* pinned = nullptr;    // host pinned scalars
  size_t pinned_cap = 0;       // doubles
  double* sws = nullptr;       // solver workspace (device)
  size_t sws_cap = 0;          // doubles
  int* siws = nullptr;         // solver integer workspace (device)
  size_t siws_cap = 0;
  double* pool = nullptr;      // fractional-step temporaries (device)
  size_t pool_cap = 0;         // bytes
  // side streams and events: calls with more chains than one launch holds run up to
  // QTT_LANES launch batches at once, each on its own stream and workspace
  hipStream_t side[QTT_LANES] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[QTT_LANES] = {};
  double* idm = nullptr;       // identity MPO cores (bond 1), for plain terms of a fit
  int* idb = nullptr;          // its bonds (all ones)
  int id_L = 0;
  // the state (u, v, p storage and shape) of the last completed fractional step:
  // the step's temporaries hold its intermediate fields, the warm start of the
  // next step of the same state only
  const void* step_warm_id[3] = {nullptr, nullptr, nullptr};
  uint64_t step_warm_gen = 0;   // the caller's state id (0 = none)
  int step_warm_L = 0, step_warm_cap = 0;
};

// Scratch of qtt_dot_noalloc: every GPU the library runs on holds its own copy of
// this array until the process ends. Host code reaches it only through the device
// address qtt_create obtains (ctx->scratch); the array's name is not a device address.
constexpr size_t QTT_NOALLOC_DOUBLES = (size_t)1 << 20;   // 8 MiB
static __device__ __align__(256) double scratch[QTT_NOALLOC_DOUBLES];

namespace {

int fail(qtt_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

#define HIPCHK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(ctx, QTT_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int launch_status(qtt_ctx* ctx) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, QTT_EHIP, "kernel launch: %s", hipGetErrorString(e));
  return QTT_OK;
}

// Batches of a call with more than QTT_BMAX chains: batch i runs on lane i % lanes.
// With one lane everything stays on the caller's stream; otherwise the side streams
// first wait for the caller's stream (fork) and the caller's stream then waits for
// each of them (join), so the call keeps the stream semantics of a single launch
// sequence (also under graph capture).
int lanes_for(int n) { return std::min(QTT_LANES, (n + QTT_BMAX - 1) / QTT_BMAX); }

hipStream_t lane_stream(qtt_ctx* ctx, int lanes, int lane, hipStream_t s) {
  return lanes > 1 ? ctx->side[lane] : s;
}

int lanes_fork(qtt_ctx* ctx, int lanes, hipStream_t s) {
  if (lanes < 2) return QTT_OK;
  HIPCHK(ctx, hipEventRecord(ctx->fork, s));
  for (int j = 0; j < lanes; ++j) HIPCHK(ctx, hipStreamWaitEvent(ctx->side[j], ctx->fork, 0));
  return QTT_OK;
}

int lanes_join(qtt_ctx* ctx, int lanes, hipStream_t s) {
  if (lanes < 2) return QTT_OK;
  for (int j = 0; j < lanes; ++j) {
    HIPCHK(ctx, hipEventRecord(ctx->join[j], ctx->side[j]));
    HIPCHK(ctx, hipStreamWaitEvent(s, ctx->join[j], 0));
  }
  return QTT_OK;
}

int ensure_ws(qtt_ctx* ctx, size_t doubles) {
  if (doubles <= ctx->ws_cap) return QTT_OK;
  if (ctx->ws) {
    HIPCHK(ctx, hipDeviceSynchronize());
    HIPCHK(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
  }
  const size_t want = doubles + doubles / 4;
  HIPCHK(ctx, hipMalloc(&ctx->ws, want * sizeof(double)));
  HIPCHK(ctx, hipMemset(ctx->ws, 0, want * sizeof(double)));   // padding entries must be finite
  ctx->ws_cap = want;
  return QTT_OK;
}

int ensure_tmp(qtt_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->tmp_cap) return QTT_OK;
  if (ctx->tmp) {
    HIPCHK(ctx, hipDeviceSynchronize());
    HIPCHK(ctx, hipFree(ctx->tmp));
    ctx->tmp = nullptr;
  }
  const size_t want = bytes + bytes / 4;
  HIPCHK(ctx, hipMalloc(&ctx->tmp, want));
  HIPCHK(ctx, hipMemset(ctx->tmp, 0, want));
  ctx->tmp_cap = want;
  return QTT_OK;
}

int ensure_pinned(qtt_ctx* ctx, size_t doubles) {
  if (doubles <= ctx->pinned_cap) return QTT_OK;
  if (ctx->pinned) HIPCHK(ctx, hipHostFree(ctx->pinned));
  ctx->pinned = nullptr;
  HIPCHK(ctx, hipHostMalloc(&ctx->pinned, doubles * sizeof(double), hipHostMallocDefault));
  ctx->pinned_cap = doubles;
  return QTT_OK;
}

int check_mps(qtt_ctx* ctx, const qtt_mps& m, const char* what) {
  if (!m.data || !m.bond) return fail(ctx, QTT_EINVAL, "%s: null pointer", what);
  if (m.L < 2 || m.L > 64) return fail(ctx, QTT_ESHAPE, "%s: L = %d outside [2, 64]", what, m.L);
  if (m.d != 2) return fail(ctx, QTT_ESHAPE, "%s: physical dimension %d (only 2 supported)", what, m.d);
  if (m.cap < 1 || m.cap > 512) return fail(ctx, QTT_ESHAPE, "%s: cap = %d outside [1, 512]", what, m.cap);
  return QTT_OK;
}

int check_mpo(qtt_ctx* ctx, const qtt_mpo& m, int L, const char* what, int* wmax) {
  if (!m.data || !m.bond || !m.bond_host) return fail(ctx, QTT_EINVAL, "%s: null pointer", what);
  if (m.L != L) return fail(ctx, QTT_ESHAPE, "%s: L = %d, expected %d", what, m.L, L);
  if (m.wcap < 1 || m.wcap > 512) return fail(ctx, QTT_ESHAPE, "%s: wcap = %d", what, m.wcap);
  if (m.bond_host[0] != 1 || m.bond_host[L] != 1) return fail(ctx, QTT_ESHAPE, "%s: boundary bonds must be 1", what);
  for (int k = 0; k <= L; ++k) {
    if (m.bond_host[k] < 1 || m.bond_host[k] > m.wcap)
      return fail(ctx, QTT_ESHAPE, "%s: bond[%d] = %d outside [1, wcap]", what, k, m.bond_host[k]);
    *wmax = std::max(*wmax, m.bond_host[k]);
  }
  return QTT_OK;
}

int check_trunc(qtt_ctx* ctx, const qtt_trunc* tr) {
  if (!tr) return fail(ctx, QTT_EINVAL, "null truncation");
  if (!(tr->rel_tol >= 0.0) || tr->chi_max < 1 || tr->fit_sweeps < 0 || tr->fit_sweeps > 64)
    return fail(ctx, QTT_EINVAL, "bad truncation (tol %g, chi %d, fit %d)", tr->rel_tol, tr->chi_max, tr->fit_sweeps);
  return QTT_OK;
}

int split_for(int K) {
  int s = K / 512;
  return std::max(1, std::min(8, s));
}

Geo make_geo(int L, int capx, int capy, int wcap, int W, double tol, int chi, int mode, int cap2, int splits, int lds) {
  Geo g;
  g.L = L; g.k = 0; g.capx = capx; g.capy = capy; g.wcap = wcap; g.W = W; g.d = 2;
  g.tol = tol; g.chi_max = chi; g.mode = mode; g.cap2 = cap2; g.splits = splits; g.lds = lds;
  return g;
}

// Right-to-left truncated SVD sweep over the trains of b (their y), then core 0.
void rl_sweep(const Batch& b, Geo g, hipStream_t s) {
  for (int k = g.L - 1; k >= 1; --k) {
    g.k = k;
    qttk::rl_svd_site(b, g, k != g.L - 1, s);
  }
  qttk::rl_finish(b, g, s);
}

// Left-to-right Householder QR sweep over the trains of b (their y).
void lr_sweep(const Batch& b, Geo g, hipStream_t s) {
  for (int k = 0; k <= g.L - 2; ++k) {
    g.k = k;
    qttk::lr_qr_site(b, g, k != 0, s);
  }
  qttk::lr_finish(b, g, s);
}

// zip-up of the chains of b: y <- M x, left-orthogonal, truncated per site.
void zipup(const Batch& b, Geo g, const WsLayout& wl, hipStream_t s) {
  qttk::zip_init(b, wl, s);
  qttk::mpo_transpose(b, g, s);
  for (int k = 0; k < g.L; ++k) {
    g.k = k;
    qttk::zip_contract(b, g, s);
    if (k < g.L - 1) {
      qttk::zip_gram(b, g, s);
      qttk::zip_factor(b, g, s);
      qttk::zip_carry(b, g, s);
    } else {
      qttk::zip_last(b, g, s);
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

int qtt_create(int device, qtt_ctx** out) {
  if (!out) return QTT_EINVAL;
  *out = nullptr;
  qtt_ctx* ctx = new qtt_ctx();
  ctx->device = device;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) { delete ctx; return QTT_EHIP; }
  int lds = 0;
  e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  if (e != hipSuccess) { delete ctx; return QTT_EHIP; }
  // keep room for the static shared arrays of the factorisation kernels
  ctx->lds = std::max(16 * 1024, std::min(lds, 160 * 1024) - 16 * 1024);
  e = qttk::init(ctx->lds);
  if (e == hipSuccess) e = qtt_solver_detail::solver_init(ctx->lds);
  if (e == hipSuccess) e = qtt_solver_detail::fit_init(ctx->lds);
  if (e != hipSuccess) { delete ctx; return QTT_EHIP; }
  ctx->coop = qtt_solver_detail::coop_capacity(device);
  // device address of this device's scratch array (the device is current here)
  e = hipGetSymbolAddress((void**)&ctx->scratch, HIP_SYMBOL(scratch));
  for (int j = 0; j < QTT_LANES && e == hipSuccess; ++j) {
    e = hipStreamCreateWithFlags(&ctx->side[j], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->join[j], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming);
  if (e != hipSuccess) { qtt_destroy(ctx); return QTT_EHIP; }
  *out = ctx;
  return QTT_OK;
}

void qtt_destroy(qtt_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  if (ctx->ws) hipFree(ctx->ws);
  if (ctx->tmp) hipFree(ctx->tmp);
  if (ctx->pinned) hipHostFree(ctx->pinned);
  if (ctx->sws) hipFree(ctx->sws);
  if (ctx->siws) hipFree(ctx->siws);
  if (ctx->pool) hipFree(ctx->pool);
  if (ctx->idm) hipFree(ctx->idm);
  if (ctx->idb) hipFree(ctx->idb);
  for (int j = 0; j < QTT_LANES; ++j) {
    if (ctx->side[j]) hipStreamDestroy(ctx->side[j]);
    if (ctx->join[j]) hipEventDestroy(ctx->join[j]);
  }
  if (ctx->fork) hipEventDestroy(ctx->fork);
  delete ctx;
}

const char* qtt_last_error(const qtt_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int qtt_apply_mpo(qtt_ctx* ctx, int n, const qtt_mpo* M, const qtt_mps* x, qtt_mps* y, const qtt_trunc* tr,
                  int contract_dt, void* stream) {
  if (!ctx) return QTT_EINVAL;
  if (n < 1 || !M || !x || !y) return fail(ctx, QTT_EINVAL, "apply: bad arguments");
  if (contract_dt < QTT_F64 || contract_dt > QTT_BF16) return fail(ctx, QTT_EINVAL, "apply: bad dtype %d", contract_dt);
  int rc = check_trunc(ctx, tr);
  if (rc) return rc;
  const int L = x[0].L, capx = x[0].cap, capy = y[0].cap, wcap = M[0].wcap;
  int W = 1;
  for (int i = 0; i < n; ++i) {
    if ((rc = check_mps(ctx, x[i], "apply x")) || (rc = check_mps(ctx, y[i], "apply y"))) return rc;
    if ((rc = check_mpo(ctx, M[i], L, "apply M", &W))) return rc;
    if (x[i].L != L || y[i].L != L || x[i].cap != capx || y[i].cap != capy || M[i].wcap != wcap)
      return fail(ctx, QTT_ESHAPE, "apply: problems of one call must share L and capacities");
    if (x[i].data == y[i].data) return fail(ctx, QTT_EINVAL, "apply: x and y alias");
  }
  // the zip-up factorises Gram matrices of order 2 * bond in one workgroup (at most 512)
  if (std::min(tr->chi_max, capy) > 256)
    return fail(ctx, QTT_ESHAPE, "apply: min(chi_max, y.cap) = %d exceeds 256", std::min(tr->chi_max, capy));
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const int splits = split_for(W * capx);
  const WsLayout wl = WsLayout::make(L, std::max(capx, capy), W, splits);
  const int lanes = lanes_for(n);
  if ((rc = ensure_ws(ctx, wl.total * std::min(n, lanes * QTT_BMAX)))) return rc;
  const int chi = std::min(tr->chi_max, capy);
  if ((rc = lanes_fork(ctx, lanes, s))) return rc;
  for (int i0 = 0, bi = 0; i0 < n; i0 += QTT_BMAX, ++bi) {
    const int lane = bi % lanes;
    Batch b;
    b.n = std::min(QTT_BMAX, n - i0);
    for (int i = 0; i < b.n; ++i) {
      Chain& c = b.c[i];
      std::memset(&c, 0, sizeof(c));
      c.x = x[i0 + i].data; c.xb = x[i0 + i].bond;
      c.y = y[i0 + i].data; c.yb = y[i0 + i].bond;
      c.m = M[i0 + i].data; c.mb = M[i0 + i].bond;
      c.ws = ctx->ws + wl.total * ((size_t)lane * QTT_BMAX + i);
    }
    Geo g = make_geo(L, capx, capy, wcap, W, tr->rel_tol, chi, contract_dt, capx, splits, ctx->lds);
    const hipStream_t ls = lane_stream(ctx, lanes, lane, s);
    zipup(b, g, wl, ls);
    rl_sweep(b, g, ls);
  }
  // join first: on a launch error the caller's stream still orders after every batch
  if ((rc = lanes_join(ctx, lanes, s))) return rc;
  if ((rc = launch_status(ctx))) return rc;
  // variational refinement (Sec. 2.2): fitting sweeps at the bonds chosen above
  return qtt_solver_detail::fit_sweeps(ctx, n, M, x, y, tr->fit_sweeps, contract_dt, stream);
}

int qtt_from_dense(qtt_ctx* ctx, const double* dense, int32_t L, const qtt_trunc* tr, qtt_mps* out, void* stream) {
  if (!ctx) return QTT_EINVAL;
  if (!dense || !out || L < 1 || L > 26) return fail(ctx, QTT_EINVAL, "from_dense: bad arguments");
  int rc = check_trunc(ctx, tr);
  if (rc) return rc;
  if ((rc = check_mps(ctx, *out, "from_dense out"))) return rc;
  if (out->L != L) return fail(ctx, QTT_ESHAPE, "from_dense: out.L = %d, expected %d", out->L, L);
  const int cap = out->cap;
  std::vector<double> v(dense, dense + ((size_t)1 << L));
  for (double x : v)
    if (!std::isfinite(x)) return fail(ctx, QTT_ENUMERIC, "from_dense: non-finite input");
  const HostTT T = tt_svd_host(v, L, 2, tr->rel_tol, std::min(tr->chi_max, cap), 0.0);
  std::vector<double> slots((size_t)L * cap * 2 * cap, 0.0);
  std::vector<int32_t> bonds(L + 1);
  for (int k = 0; k <= L; ++k) bonds[k] = T.bl[k];
  for (int k = 0; k < L; ++k)
    for (int a = 0; a < T.bl[k]; ++a)
      for (int s2 = 0; s2 < 2; ++s2)
        for (int b = 0; b < T.bl[k + 1]; ++b)
          slots[(size_t)k * cap * 2 * cap + (size_t)a * 2 * cap + s2 * cap + b] =
              T.cores[k][((size_t)a * 2 + s2) * T.bl[k + 1] + b];
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(ctx, hipMemcpyAsync(out->data, slots.data(), slots.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipMemcpyAsync(out->bond, bonds.data(), bonds.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHK(ctx, hipStreamSynchronize(s));   // the host buffers are released on return
  return QTT_OK;
}

int qtt_round(qtt_ctx* ctx, int n, qtt_mps* x, const qtt_trunc* tr, void* stream) {
  if (!ctx) return QTT_EINVAL;
  if (n < 1 || !x) return fail(ctx, QTT_EINVAL, "round: bad arguments");
  int rc = check_trunc(ctx, tr);
  if (rc) return rc;
  const int L = x[0].L, cap = x[0].cap;
  for (int i = 0; i < n; ++i) {
    if ((rc = check_mps(ctx, x[i], "round x"))) return rc;
    if (x[i].L != L || x[i].cap != cap) return fail(ctx, QTT_ESHAPE, "round: problems must share L and cap");
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const WsLayout wl = WsLayout::make(L, cap, 1, 1);
  const int lanes = lanes_for(n);
  if ((rc = ensure_ws(ctx, wl.total * std::min(n, lanes * QTT_BMAX)))) return rc;
  if ((rc = lanes_fork(ctx, lanes, s))) return rc;
  for (int i0 = 0, bi = 0; i0 < n; i0 += QTT_BMAX, ++bi) {
    const int lane = bi % lanes;
    Batch b;
    b.n = std::min(QTT_BMAX, n - i0);
    for (int i = 0; i < b.n; ++i) {
      Chain& c = b.c[i];
      std::memset(&c, 0, sizeof(c));
      c.y = x[i0 + i].data; c.yb = x[i0 + i].bond;
      c.ws = ctx->ws + wl.total * ((size_t)lane * QTT_BMAX + i);
    }
    Geo g = make_geo(L, cap, cap, 1, 1, tr->rel_tol, std::min(tr->chi_max, cap), 0, cap, 1, ctx->lds);
    const hipStream_t ls = lane_stream(ctx, lanes, lane, s);
    qttk::ws_init(b, wl, ls);
    lr_sweep(b, g, ls);
    rl_sweep(b, g, ls);
  }
  if ((rc = lanes_join(ctx, lanes, s))) return rc;
  return launch_status(ctx);
}

int qtt_add(qtt_ctx* ctx, int n, const double* a, const qtt_mps* x, const double* bw, const qtt_mps* y,
            qtt_mps* z, const qtt_trunc* tr, void* stream) {
  if (!ctx) return QTT_EINVAL;
  if (n < 1 || !a || !x || !bw || !y || !z) return fail(ctx, QTT_EINVAL, "add: bad arguments");
  int rc = check_trunc(ctx, tr);
  if (rc) return rc;
  const int L = x[0].L, capx = x[0].cap, capy = y[0].cap, capz = z[0].cap;
  for (int i = 0; i < n; ++i) {
    if ((rc = check_mps(ctx, x[i], "add x")) || (rc = check_mps(ctx, y[i], "add y")) ||
        (rc = check_mps(ctx, z[i], "add z")))
      return rc;
    if (x[i].L != L || y[i].L != L || z[i].L != L || x[i].cap != capx || y[i].cap != capy || z[i].cap != capz)
      return fail(ctx, QTT_ESHAPE, "add: problems must share L and capacities");
    if (z[i].data == x[i].data || z[i].data == y[i].data) return fail(ctx, QTT_EINVAL, "add: z aliases an input");
  }
  const int caps = capx + capy;
  if (caps > 512) return fail(ctx, QTT_ESHAPE, "add: cap_x + cap_y = %d exceeds 512", caps);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const WsLayout wl = WsLayout::make(L, caps, 1, 1);
  const int chunk = std::min(n, QTT_BMAX);
  if ((rc = ensure_ws(ctx, wl.total * chunk))) return rc;
  const size_t tslot = (size_t)L * caps * 2 * caps;
  const size_t tbytes = chunk * (tslot * sizeof(double) + 128 * sizeof(int));
  if ((rc = ensure_tmp(ctx, tbytes))) return rc;
  for (int i0 = 0; i0 < n; i0 += QTT_BMAX) {
    Batch b;
    b.n = std::min(QTT_BMAX, n - i0);
    int* tb = reinterpret_cast<int*>(ctx->tmp + chunk * tslot);
    for (int i = 0; i < b.n; ++i) {
      Chain& c = b.c[i];
      std::memset(&c, 0, sizeof(c));
      c.x = x[i0 + i].data; c.xb = x[i0 + i].bond;
      c.x2 = y[i0 + i].data; c.x2b = y[i0 + i].bond;
      c.y = ctx->tmp + tslot * i; c.yb = tb + 128 * i;
      c.alpha = a[i0 + i]; c.beta = bw[i0 + i];
      c.ws = ctx->ws + wl.total * i;
    }
    Geo g = make_geo(L, capx, caps, 1, 1, tr->rel_tol, std::min(tr->chi_max, capz), 0, capy, 1, ctx->lds);
    qttk::direct_sum(b, g, s);
    qttk::ws_init(b, wl, s);
    Geo gs = make_geo(L, caps, caps, 1, 1, tr->rel_tol, std::min(tr->chi_max, capz), 0, caps, 1, ctx->lds);
    lr_sweep(b, gs, s);
    rl_sweep(b, gs, s);
    // copy the rounded sum into z
    Batch bc;
    bc.n = b.n;
    for (int i = 0; i < b.n; ++i) {
      Chain& c = bc.c[i];
      std::memset(&c, 0, sizeof(c));
      c.x = b.c[i].y; c.xb = b.c[i].yb;
      c.y = z[i0 + i].data; c.yb = z[i0 + i].bond;
      c.alpha = 1.0;
    }
    Geo gc = make_geo(L, caps, capz, 1, 1, 0.0, capz, 0, caps, 1, ctx->lds);
    qttk::copy_mps(bc, gc, s);
  }
  return launch_status(ctx);
}

static int dot_impl(qtt_ctx* ctx, int n, const qtt_mps* x, const qtt_mpo* A, const qtt_mps* y, double* out,
                    void* stream) {
  if (!ctx) return QTT_EINVAL;
  if (n < 1 || !x || !y || !out) return fail(ctx, QTT_EINVAL, "dot: bad arguments");
  int rc;
  const int L = x[0].L, capx = x[0].cap, capy = y[0].cap;
  int W = 1, wcap = 1;
  for (int i = 0; i < n; ++i) {
    if ((rc = check_mps(ctx, x[i], "dot x")) || (rc = check_mps(ctx, y[i], "dot y"))) return rc;
    if (x[i].L != L || y[i].L != L || x[i].cap != capx || y[i].cap != capy)
      return fail(ctx, QTT_ESHAPE, "dot: problems must share L and capacities");
    if (A) {
      if ((rc = check_mpo(ctx, A[i], L, "dot A", &W))) return rc;
      if (A[i].wcap != A[0].wcap) return fail(ctx, QTT_ESHAPE, "dot: MPOs must share wcap");
      wcap = A[0].wcap;
    }
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const WsLayout wl = WsLayout::make(L, std::max(capx, capy), W, 1);
  const int chunk = std::min(n, QTT_BMAX);
  if ((rc = ensure_ws(ctx, wl.total * chunk))) return rc;
  if ((rc = ensure_pinned(ctx, n))) return rc;
  for (int i0 = 0; i0 < n; i0 += QTT_BMAX) {
    Batch b;
    b.n = std::min(QTT_BMAX, n - i0);
    for (int i = 0; i < b.n; ++i) {
      Chain& c = b.c[i];
      std::memset(&c, 0, sizeof(c));
      c.x = x[i0 + i].data; c.xb = x[i0 + i].bond;
      c.x2 = y[i0 + i].data; c.x2b = y[i0 + i].bond;
      if (A) { c.m = A[i0 + i].data; c.mb = A[i0 + i].bond; }
      c.ws = ctx->ws + wl.total * i;
    }
    Geo g = make_geo(L, capx, capx, wcap, W, 0.0, 1, 0, capy, 1, ctx->lds);
    if (A) qttk::mpo_transpose(b, g, s);
    qttk::dot_init(b, g, s);
    for (int k = 0; k < L; ++k) {
      g.k = k;
      qttk::dot_step(b, g, A != nullptr, s);
    }
    qttk::dot_finish(b, g, s);
    for (int i = 0; i < b.n; ++i)
      HIPCHK(ctx, hipMemcpyAsync(ctx->pinned + i0 + i, b.c[i].ws + wl.scal + SC_DOT, sizeof(double),
                                 hipMemcpyDeviceToHost, s));
  }
  if ((rc = launch_status(ctx))) return rc;
  HIPCHK(ctx, hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i) out[i] = ctx->pinned[i];
  return QTT_OK;
}

int qtt_dot(qtt_ctx* ctx, int n, const qtt_mps* x, const qtt_mps* y, double* out, void* stream) {
  return dot_impl(ctx, n, x, nullptr, y, out, stream);
}

int qtt_dot_noalloc(qtt_ctx* ctx, int n, const qtt_mps* x, const qtt_mps* y, double* out, void* stream) {
  if (!ctx) return QTT_EINVAL;
  if (n < 1 || !x || !y || !out) return fail(ctx, QTT_EINVAL, "dot_noalloc: bad arguments");
  if (!ctx->scratch) return fail(ctx, QTT_EHIP, "dot_noalloc: no scratch address");
  int rc;
  const int L = x[0].L, capx = x[0].cap, capy = y[0].cap;
  for (int i = 0; i < n; ++i) {
    if ((rc = check_mps(ctx, x[i], "dot_noalloc x")) || (rc = check_mps(ctx, y[i], "dot_noalloc y"))) return rc;
    if (x[i].L != L || y[i].L != L || x[i].cap != capx || y[i].cap != capy)
      return fail(ctx, QTT_ESHAPE, "dot_noalloc: problems must share L and capacities");
  }
  const WsLayout wl = WsLayout::make(L, std::max(capx, capy), 1, 1);
  if (wl.total > QTT_NOALLOC_DOUBLES)
    return fail(ctx, QTT_ECAPACITY, "dot_noalloc: one problem needs %zu doubles of scratch, the limit is %zu",
                wl.total, QTT_NOALLOC_DOUBLES);
  const int per = (int)std::min<size_t>(QTT_BMAX, QTT_NOALLOC_DOUBLES / wl.total);
  hipStream_t s = (hipStream_t)stream;
  for (int i0 = 0; i0 < n; i0 += per) {
    Batch b;
    b.n = std::min(per, n - i0);
    for (int i = 0; i < b.n; ++i) {
      Chain& c = b.c[i];
      std::memset(&c, 0, sizeof(c));
      c.x = x[i0 + i].data; c.xb = x[i0 + i].bond;
      c.x2 = y[i0 + i].data; c.x2b = y[i0 + i].bond;
      c.ws = ctx->scratch + wl.total * i;
    }
    Geo g = make_geo(L, capx, capx, 1, 1, 0.0, 1, 0, capy, 1, ctx->lds);
    qttk::dot_init(b, g, s);
    for (int k = 0; k < L; ++k) {
      g.k = k;
      qttk::dot_step(b, g, 0, s);
    }
    qttk::dot_finish(b, g, s);
    qttk::dot_out(b, g, out + i0, s);
  }
  return launch_status(ctx);
}

int qtt_dot_mpo(qtt_ctx* ctx, int n, const qtt_mps* x, const qtt_mpo* A, const qtt_mps* y, double* out,
                void* stream) {
  if (!A) return fail(ctx, QTT_EINVAL, "dot_mpo: null MPO");
  return dot_impl(ctx, n, x, A, y, out, stream);
}

int qtt_apply_local(qtt_ctx* ctx, int n, const qtt_mpo* D, const qtt_mps* x, qtt_mps* y, void* stream) {
  if (!ctx) return QTT_EINVAL;
  if (n < 1 || !D || !x || !y) return fail(ctx, QTT_EINVAL, "apply_local: bad arguments");
  int rc;
  const int L = x[0].L, capx = x[0].cap, capy = y[0].cap, wcap = D[0].wcap;
  for (int i = 0; i < n; ++i) {
    int W = 1;
    if ((rc = check_mps(ctx, x[i], "apply_local x")) || (rc = check_mps(ctx, y[i], "apply_local y"))) return rc;
    if ((rc = check_mpo(ctx, D[i], L, "apply_local D", &W))) return rc;
    if (W != 1) return fail(ctx, QTT_ESHAPE, "apply_local: MPO bond %d (must be 1)", W);
    if (x[i].L != L || y[i].L != L || x[i].cap != capx || y[i].cap != capy || D[i].wcap != wcap)
      return fail(ctx, QTT_ESHAPE, "apply_local: problems must share L and capacities");
    if (capy < capx) return fail(ctx, QTT_ECAPACITY, "apply_local: y cap %d < x cap %d", capy, capx);
  }
  HIPCHK(ctx, hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  for (int i0 = 0; i0 < n; i0 += QTT_BMAX) {
    Batch b;
    b.n = std::min(QTT_BMAX, n - i0);
    for (int i = 0; i < b.n; ++i) {
      Chain& c = b.c[i];
      std::memset(&c, 0, sizeof(c));
      c.x = x[i0 + i].data; c.xb = x[i0 + i].bond;
      c.y = y[i0 + i].data; c.yb = y[i0 + i].bond;
      c.m = D[i0 + i].data; c.mb = D[i0 + i].bond;
    }
    Geo g = make_geo(L, capx, capy, wcap, 1, 0.0, capy, 0, capx, 1, ctx->lds);
    qttk::apply_local(b, g, s);
  }
  return launch_status(ctx);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// workspace access for solve.hip / step.hip
// ---------------------------------------------------------------------------
namespace qtt_solver_detail {

template <class T>
static T* grow(qtt_ctx* ctx, T*& buf, size_t& cap, size_t count, int* rc) {
  *rc = QTT_OK;
  if (count <= cap) return buf;
  if (buf) {
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipFree(buf);
    buf = nullptr;
    cap = 0;
    if (e != hipSuccess) { *rc = fail(ctx, QTT_EHIP, "free: %s", hipGetErrorString(e)); return nullptr; }
  }
  const size_t want = count + count / 4;
  hipError_t e = hipMalloc(&buf, want * sizeof(T));
  if (e == hipSuccess) e = hipMemset(buf, 0, want * sizeof(T));   // padding entries must be finite
  if (e != hipSuccess) { *rc = fail(ctx, QTT_EHIP, "hipMalloc(%zu): %s", want * sizeof(T), hipGetErrorString(e)); return nullptr; }
  cap = want;
  return buf;
}

double* solver_ws(qtt_ctx* ctx, size_t doubles, int* rc) { return grow(ctx, ctx->sws, ctx->sws_cap, doubles, rc); }
int* solver_iws(qtt_ctx* ctx, size_t ints, int* rc) { return grow(ctx, ctx->siws, ctx->siws_cap, ints, rc); }
double* step_pool(qtt_ctx* ctx, size_t doubles, int* rc) {
  size_t cap = ctx->pool_cap / sizeof(double);
  double* p = grow(ctx, ctx->pool, cap, doubles, rc);
  ctx->pool_cap = cap * sizeof(double);
  return p;
}
int set_error(qtt_ctx* ctx, int code, const char* msg) { return fail(ctx, code, "%s", msg); }
const double* identity_mpo(qtt_ctx* ctx, int L, const int** bond, int* rc) {
  *rc = QTT_OK;
  if (ctx->id_L < L) {
    if (ctx->idm) { (void)hipDeviceSynchronize(); (void)hipFree(ctx->idm); (void)hipFree(ctx->idb); }
    ctx->idm = nullptr; ctx->idb = nullptr; ctx->id_L = 0;
    std::vector<double> cores((size_t)L * 4, 0.0);
    for (int k = 0; k < L; ++k) { cores[4 * k + 0] = 1.0; cores[4 * k + 3] = 1.0; }   // [1][o][i][1] = delta(o, i)
    std::vector<int> ones(L + 1, 1);
    hipError_t e = hipMalloc(&ctx->idm, cores.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&ctx->idb, ones.size() * sizeof(int));
    if (e == hipSuccess) e = hipMemcpy(ctx->idm, cores.data(), cores.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->idb, ones.data(), ones.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) { *rc = fail(ctx, QTT_EHIP, "identity MPO: %s", hipGetErrorString(e)); return nullptr; }
    ctx->id_L = L;
  }
  *bond = ctx->idb;
  return ctx->idm;
}
bool step_warm(qtt_ctx* ctx, uint64_t gen, const void* const id[3], int L, int cap) {
  return gen != 0 && ctx->step_warm_gen == gen && ctx->step_warm_L == L && ctx->step_warm_cap == cap &&
         ctx->step_warm_id[0] == id[0] && ctx->step_warm_id[1] == id[1] && ctx->step_warm_id[2] == id[2];
}
void set_step_warm(qtt_ctx* ctx, uint64_t gen, const void* const id[3], int L, int cap) {
  ctx->step_warm_gen = gen; ctx->step_warm_L = L; ctx->step_warm_cap = cap;
  for (int i = 0; i < 3; ++i) ctx->step_warm_id[i] = id[i];
}
int lds_of(qtt_ctx* ctx) { return ctx->lds; }
int device_of(qtt_ctx* ctx) { return ctx->device; }
int coop_of(qtt_ctx* ctx) { return ctx->coop; }
double* pinned(qtt_ctx* ctx, size_t doubles, int* rc) {
  *rc = ensure_pinned(ctx, doubles);
  return *rc ? nullptr : ctx->pinned;
}

}  // namespace qtt_solver_detail

// ---------------------------------------------------------------------------
// measurement hook
// ---------------------------------------------------------------------------
extern "C" int qtt_timer_start(qtt_ctx* ctx, int kernel_class) {
  if (!ctx) return QTT_EINVAL;
  if (kernel_class < -1 || kernel_class >= KC_COUNT) return fail(ctx, QTT_EINVAL, "timer: bad kernel class");
  qttk::Timer& t = qttk::timer();
  if (!t.cnt) HIPCHK(ctx, hipMalloc(&t.cnt, 2 * sizeof(double)));
  HIPCHK(ctx, hipDeviceSynchronize());
  HIPCHK(ctx, hipMemset(t.cnt, 0, 2 * sizeof(double)));
  t.used = 0;
  t.kc = kernel_class;
  return QTT_OK;
}

extern "C" int qtt_timer_read(qtt_ctx* ctx, int64_t* launches, double* ms, double* flops, double* bytes,
                              double* overhead_ms) {
  if (!ctx || !launches || !ms || !flops || !bytes || !overhead_ms) return QTT_EINVAL;
  qttk::Timer& t = qttk::timer();
  HIPCHK(ctx, hipDeviceSynchronize());
  double total = 0.0;
  for (size_t i = 0; i + 1 < t.used; i += 2) {
    float e = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&e, t.ev[i], t.ev[i + 1]));
    total += e;
  }
  double c[2] = {0.0, 0.0};
  if (t.cnt) HIPCHK(ctx, hipMemcpy(c, t.cnt, sizeof(c), hipMemcpyDeviceToHost));
  *launches = (int64_t)(t.used / 2);
  *ms = total;
  *flops = c[0];
  *bytes = c[1];
  *overhead_ms = qttk::bracket_overhead_ms(nullptr);
  t.kc = -1;
  return QTT_OK;
}

extern "C" int qtt_timer_durations(qtt_ctx* ctx, double* ms, int64_t cap, int64_t* n) {
  if (!ctx || !n || cap < 0 || (cap > 0 && !ms)) return QTT_EINVAL;
  qttk::Timer& t = qttk::timer();
  HIPCHK(ctx, hipDeviceSynchronize());
  const int64_t have = (int64_t)(t.used / 2);
  *n = have < cap ? have : cap;
  for (int64_t i = 0; i < *n; ++i) {
    float e = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&e, t.ev[2 * i], t.ev[2 * i + 1]));
    ms[i] = e;
  }
  return QTT_OK;
}
