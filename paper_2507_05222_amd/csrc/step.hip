// One Chorin fractional step in TT format (Sec. 3.3 of arxiv 2507.05222).
//
//   gradients   g = D v + b_D(v_wall, v_inf)            (curvilinear derivatives with
//                                                         ghost-point corrections, Sec. 3.1)
//   convection  c = v_x (.) g_x + v_z (.) g_z             (elementwise products through the
//                                                         copy tensor, Sec. 2.1.3)
//   predictor   |J|^(1/2)(I - dt/Re Lap)|J|^(-1/2) w = |J|^(1/2)(v - dt c + dt/Re b_Lap),
//               v* = |J|^(-1/2) w                        (Eq. intermediate_vel_eq, SPD form)
//   pressure    (-|J| Lap_p) p = (1/dt)(-|J| div v* + b_W) (Eq. Poisson, J-weighted, Sec. 3.3)
//   projection  v = v* - dt grad_p p
//
// Every linear combination of products is one variational fit (Sec. 2.2,
// qtt_fit) at the state's bond dimension; the two solves are the variational
// ALS solver (qtt_poisson_solve). Independent chains run batched. When the
// previous step on this context advanced the same state (same id and storage),
// the fits start from that step's results, otherwise from a random sketch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/qtt.h"
#include "host_linalg.h"
#include "internal.h"

extern "C" size_t qtt_ws_act_floats(int batch);
extern "C" int qtt_ws_input_host(const double* coarse_b, double re, double alpha, float* in, double* rms);
extern "C" int qtt_ws_forward(qtt_ctx* ctx, const float* params, const float* in, int batch, float* acts, float* out,
                              int bf16, void* stream);

namespace qtt_solver_detail {
double* step_pool(qtt_ctx* ctx, size_t doubles, int* rc);
int set_error(qtt_ctx* ctx, int code, const char* msg);
bool step_warm(qtt_ctx* ctx, uint64_t gen, const void* const id[3], int L, int cap);
void set_step_warm(qtt_ctx* ctx, uint64_t gen, const void* const id[3], int L, int cap);
}

namespace {
enum { GXU = 0, GZU, GXV, GZV, CONVU, CONVV, RSU, RSV, WU, WV, US, VS, BT, PRED, X0, NTMP };
constexpr int CN = 6;                       // coarse grid of the warm start: 2^6 x 2^6
constexpr size_t WS_FLOATS = (size_t)(3 + 96 + 1) * 4096;   // network input, activations, output

// Coarse (2^6 x 2^6, block-averaged) field of a train in interleaved order: the
// cores past the first 2 CN are contracted with [1/2, 1/2]. Host, from host copies
// of the slots (cap) and bonds. grid[I * 64 + J].
void coarse_field(const std::vector<double>& slots, const std::vector<int>& bl, int L, int cap, std::vector<double>& grid) {
  const int Lc = 2 * CN;
  auto core = [&](int k, int a, int s, int b) { return slots[(size_t)k * cap * 2 * cap + (size_t)a * 2 * cap + s * cap + b]; };
  std::vector<double> r(1, 1.0);                  // bl[k] vector, from the right
  for (int k = L - 1; k >= Lc; --k) {
    std::vector<double> nr(bl[k], 0.0);
    for (int a = 0; a < bl[k]; ++a)
      for (int b = 0; b < bl[k + 1]; ++b) nr[a] += 0.5 * (core(k, a, 0, b) + core(k, a, 1, b)) * r[b];
    r.swap(nr);
  }
  // left-to-right contraction of the first Lc cores (the last one closed with r)
  std::vector<double> v(1, 1.0);
  int rows = 1;
  for (int k = 0; k < Lc; ++k) {
    const int a0 = bl[k], b0 = (k == Lc - 1) ? 1 : bl[k + 1];
    std::vector<double> nv((size_t)rows * 2 * b0, 0.0);
    for (int q = 0; q < rows; ++q)
      for (int a = 0; a < a0; ++a) {
        const double x = v[(size_t)q * a0 + a];
        if (x == 0.0) continue;
        for (int s2 = 0; s2 < 2; ++s2)
          for (int b = 0; b < b0; ++b) {
            const double c = (k == Lc - 1) ? [&] { double t = 0; for (int bb = 0; bb < bl[k + 1]; ++bb) t += core(k, a, s2, bb) * r[bb]; return t; }()
                                           : core(k, a, s2, b);
            nv[((size_t)q * 2 + s2) * b0 + b] += x * c;
          }
      }
    v.swap(nv);
    rows *= 2;
  }
  // interleaved index: digit 2m = bit m (MSB first) of the row I, digit 2m+1 of the column J
  grid.assign(4096, 0.0);
  for (int q = 0; q < 4096; ++q) {
    int I = 0, J = 0;
    for (int m = 0; m < CN; ++m) {
      I = 2 * I + ((q >> (Lc - 1 - 2 * m)) & 1);
      J = 2 * J + ((q >> (Lc - 2 - 2 * m)) & 1);
    }
    grid[(size_t)I * 64 + J] = v[q];
  }
}
}

// Learned initial guess of the pressure solve (the rule is stated with
// qtt_fractional_step in the header).
static int learned_guess(qtt_ctx* ctx, const qtt_flow_ops* ops, qtt_flow_state* st, const qtt_step_opts* o, qtt_mps* T,
                         int L, int cap, int chi, float* wsf, qtt_step_info* info, void* stream) {
  using namespace qtt_solver_detail;
  const qtt_ws_model& m = *o->warm;
  hipStream_t s = (hipStream_t)stream;
  const size_t slot = (size_t)L * cap * 2 * cap;
  std::vector<double> hs(slot);
  std::vector<int> hb(L + 1);
  if (hipMemcpyAsync(hs.data(), T[BT].data, slot * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(hb.data(), T[BT].bond, (L + 1) * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(ctx, QTT_EHIP, "step: copy of the pressure right-hand side failed");
  std::vector<double> cb;
  coarse_field(hs, hb, L, cap, cb);
  std::vector<float> in(3 * 4096);
  double rms = 0.0;
  if (qtt_ws_input_host(cb.data(), m.re, m.alpha, in.data(), &rms) != QTT_OK) return QTT_OK;   // b = 0: no guess
  float* din = wsf;
  float* acts = wsf + 3 * 4096;
  float* dout = acts + qtt_ws_act_floats(1);
  if (hipMemcpyAsync(din, in.data(), in.size() * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess)
    return set_error(ctx, QTT_EHIP, "step: copy of the network input failed");
  int rc = qtt_ws_forward(ctx, m.params, din, 1, acts, dout, m.bf16, stream);
  if (rc) return rc;
  std::vector<float> out(4096);
  if (hipMemcpyAsync(out.data(), dout, 4096 * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(ctx, QTT_EHIP, "step: copy of the network output failed");
  // coarse prediction in interleaved order, TT-SVD to bond m.chi, prolongation by
  // appended [1, 1] cores, then fitted at the state's bond
  const int Lc = 2 * CN;
  std::vector<double> pv(4096);
  for (int q = 0; q < 4096; ++q) {
    int I = 0, J = 0;
    for (int k = 0; k < CN; ++k) {
      I = 2 * I + ((q >> (Lc - 1 - 2 * k)) & 1);
      J = 2 * J + ((q >> (Lc - 2 - 2 * k)) & 1);
    }
    pv[q] = (double)out[(size_t)I * 64 + J] * m.out_scale * rms;
  }
  HostTT tt = tt_svd_host(pv, Lc, 2, 0.0, m.chi, 0.0);
  std::vector<double> ps(slot, 0.0);
  std::vector<int> pb(L + 1, 1);
  for (int k = 0; k < Lc; ++k) {
    pb[k + 1] = tt.bl[k + 1];
    for (int a = 0; a < tt.bl[k]; ++a)
      for (int s2 = 0; s2 < 2; ++s2)
        for (int b = 0; b < tt.bl[k + 1]; ++b)
          ps[(size_t)k * cap * 2 * cap + (size_t)a * 2 * cap + s2 * cap + b] = tt.cores[k][((size_t)a * 2 + s2) * tt.bl[k + 1] + b];
  }
  for (int k = Lc; k < L; ++k) {
    ps[(size_t)k * cap * 2 * cap + 0 * cap + 0] = 1.0;
    ps[(size_t)k * cap * 2 * cap + 1 * cap + 0] = 1.0;
  }
  if (hipMemcpyAsync(T[PRED].data, ps.data(), slot * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(T[PRED].bond, pb.data(), (L + 1) * sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(ctx, QTT_EHIP, "step: copy of the prolonged prediction failed");
  qtt_term t{1.0, nullptr, &T[PRED]};
  if ((rc = qtt_fit(ctx, 1, 1, &t, &T[X0], chi, 2, 1, QTT_F64, stream))) return rc;
  // energies J(x) = x.Px/2 - b.x of the candidate and of the previous pressure
  qtt_mps xs[2] = {T[X0], st->p};
  qtt_mps bs[2] = {T[BT], T[BT]};
  qtt_mpo Ps[2] = {ops->P, ops->P};
  double xax[2], bx[2];
  if ((rc = qtt_dot_mpo(ctx, 2, xs, Ps, xs, xax, stream))) return rc;
  if ((rc = qtt_dot(ctx, 2, bs, xs, bx, stream))) return rc;
  // each candidate at its optimal scale a* = b.x / x.Px, where J(a* x) = -(b.x)^2 / (2 x.Px):
  // the comparison then rates the direction of a candidate, not its amplitude
  auto best = [](double xpx, double b_x, double* a) {
    *a = (xpx > 0.0) ? b_x / xpx : 0.0;
    return (xpx > 0.0) ? -0.5 * b_x * b_x / xpx : 0.0;
  };
  double aw, ap;
  const double jw = best(xax[0], bx[0], &aw), jp = best(xax[1], bx[1], &ap);
  if (info) { info->warm_energy = jw; info->prev_energy = jp; }
  if (std::isfinite(jw) && jw < jp) {
    Batch b;
    b.n = 1;
    std::memset(&b.c[0], 0, sizeof(Chain));
    b.c[0].x = T[X0].data; b.c[0].xb = T[X0].bond; b.c[0].y = st->p.data; b.c[0].yb = st->p.bond;
    b.c[0].alpha = aw;
    Geo g;
    std::memset(&g, 0, sizeof(g));
    g.L = L; g.capx = cap; g.capy = st->p.cap; g.d = 2;
    qttk::copy_mps(b, g, s);
    if (info) info->warm_used = 1;
  }
  return QTT_OK;
}

extern "C" int qtt_ws_coarse(qtt_ctx* ctx, const qtt_mps* x, double* grid, void* stream) {
  using namespace qtt_solver_detail;
  if (!ctx) return QTT_EINVAL;
  if (!x || !x->data || !x->bond || !grid || x->d != 2 || x->L < 2 * CN)
    return set_error(ctx, QTT_EINVAL, "ws_coarse: needs a train of at least 12 binary cores");
  hipStream_t s = (hipStream_t)stream;
  const size_t slot = (size_t)x->L * x->cap * 2 * x->cap;
  std::vector<double> hs(slot);
  std::vector<int> hb(x->L + 1);
  if (hipMemcpyAsync(hs.data(), x->data, slot * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(hb.data(), x->bond, (x->L + 1) * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(ctx, QTT_EHIP, "ws_coarse: copy failed");
  std::vector<double> g;
  coarse_field(hs, hb, x->L, x->cap, g);
  std::memcpy(grid, g.data(), 4096 * sizeof(double));
  return QTT_OK;
}

extern "C" int qtt_fractional_step(qtt_ctx* ctx, const qtt_flow_ops* ops, qtt_flow_state* st, const qtt_step_opts* o,
                                   qtt_step_info* info, void* stream) {
  using namespace qtt_solver_detail;
  if (!ctx) return QTT_EINVAL;
  if (!ops || !st || !o || !(o->dt > 0.0)) return set_error(ctx, QTT_EINVAL, "step: bad arguments");
  if (o->contract_dt < QTT_F64 || o->contract_dt > QTT_BF16 || o->product_dt < QTT_F64 || o->product_dt > QTT_BF16)
    return set_error(ctx, QTT_EINVAL, "step: bad dtype");
  const int L = st->u.L, cap = st->u.cap;
  if (st->v.L != L || st->p.L != L || st->v.cap != cap || !st->u.data || !st->v.data || !st->p.data)
    return set_error(ctx, QTT_ESHAPE, "step: u, v must share L and cap; p must share L");
  if (o->warm && (L < 2 * CN || st->p.cap != cap || o->warm->chi < 1 || o->warm->chi > cap || !o->warm->params))
    return set_error(ctx, QTT_EINVAL, "step: the warm start needs n >= 6, p.cap == u.cap, 1 <= chi <= cap");
  if (o->rhs_out && (o->rhs_out->L != L || o->rhs_out->cap < std::min(o->trunc.chi_max, cap) || !o->rhs_out->data))
    return set_error(ctx, QTT_ESHAPE, "step: rhs_out needs the state's L and cap >= its bond");
  if (info) { info->warm_used = 0; info->warm_energy = 0.0; info->prev_energy = 0.0; }
  const qtt_mps* bcs[7] = {&ops->bx_u, &ops->bz_u, &ops->bx_v, &ops->bz_v, &ops->bL_u, &ops->bL_v, &ops->bW};
  for (auto* b : bcs)
    if (b->L != L || b->cap != ops->bx_u.cap) return set_error(ctx, QTT_ESHAPE, "step: boundary vectors must share L and cap");

  // temporaries: NTMP trains of cap `cap` and two diagonal MPOs (wcap = cap)
  const size_t slot = (size_t)L * cap * 2 * cap;
  const size_t mslot = (size_t)L * cap * 4 * cap;
  const size_t ints = (size_t)(NTMP + 2) * 64;
  int rc = 0;
  double* pool = step_pool(ctx, NTMP * slot + 2 * mslot + ints / 2 + 64 + WS_FLOATS / 2 + 64, &rc);
  if (rc) return rc;
  int* ib = reinterpret_cast<int*>(pool + NTMP * slot + 2 * mslot);
  float* wsf = reinterpret_cast<float*>(pool + NTMP * slot + 2 * mslot + ints / 2 + 64);
  qtt_mps T[NTMP];
  for (int i = 0; i < NTMP; ++i) T[i] = qtt_mps{L, 2, cap, ib + 64 * i, pool + slot * i};
  std::vector<int32_t> diag_bonds(L + 1, cap);
  diag_bonds[0] = diag_bonds[L] = 1;
  qtt_mpo DU{L, cap, diag_bonds.data(), ib + 64 * NTMP, pool + NTMP * slot};
  qtt_mpo DV{L, cap, diag_bonds.data(), ib + 64 * (NTMP + 1), pool + NTMP * slot + mslot};

  const int chi = std::min(o->trunc.chi_max, cap);
  // warm fits only when the temporaries come from the previous step of this state
  const void* const sid[3] = {st->u.data, st->v.data, st->p.data};
  const bool warm = step_warm(ctx, st->id, sid, L, cap);
  const int init = warm ? 0 : 1;
  const int sweeps = warm ? std::max(1, o->trunc.fit_sweeps) : std::max(2, o->trunc.fit_sweeps);
  const int mode = o->contract_dt;
  const double dt = o->dt;
  hipStream_t s = (hipStream_t)stream;
  auto term = [](double c, const qtt_mpo* M, const qtt_mps* x) { return qtt_term{c, M, x}; };

  // (1) curvilinear gradients with their boundary corrections
  {
    qtt_term t[8] = {term(1, &ops->Dx, &st->u), term(1, nullptr, &ops->bx_u),
                     term(1, &ops->Dz, &st->u), term(1, nullptr, &ops->bz_u),
                     term(1, &ops->Dx, &st->v), term(1, nullptr, &ops->bx_v),
                     term(1, &ops->Dz, &st->v), term(1, nullptr, &ops->bz_v)};
    qtt_mps y[4] = {T[GXU], T[GZU], T[GXV], T[GZV]};
    if ((rc = qtt_fit(ctx, 4, 2, t, y, chi, sweeps, init, mode, stream))) return rc;
  }
  // (2) convection (v.grad) v: diagonal MPOs of u, v (copy tensor) times the gradients
  {
    Batch b;
    b.n = 2;
    std::memset(&b.c[0], 0, sizeof(Chain) * 2);
    b.c[0].x = st->u.data; b.c[0].xb = st->u.bond; b.c[0].y = const_cast<double*>(DU.data); b.c[0].yb = const_cast<int*>(DU.bond);
    b.c[1].x = st->v.data; b.c[1].xb = st->v.bond; b.c[1].y = const_cast<double*>(DV.data); b.c[1].yb = const_cast<int*>(DV.bond);
    Geo g;
    std::memset(&g, 0, sizeof(g));
    g.L = L; g.capx = cap; g.capy = cap; g.wcap = cap; g.d = 2;
    qttk::diag_mpo(b, g, s);
    qtt_term t[4] = {term(1, &DU, &T[GXU]), term(1, &DV, &T[GZU]),
                     term(1, &DU, &T[GXV]), term(1, &DV, &T[GZV])};
    qtt_mps y[2] = {T[CONVU], T[CONVV]};
    if ((rc = qtt_fit(ctx, 2, 2, t, y, chi, sweeps, init, o->product_dt, stream))) return rc;
  }
  // (3) predictor right-hand side scaled by |J|^(1/2): Jh (v - dt c + b_Lap); solve
  {
    qtt_term t[6] = {term(1, &ops->Jh, &st->u), term(-dt, &ops->Jh, &T[CONVU]), term(1, &ops->Jh, &ops->bL_u),
                     term(1, &ops->Jh, &st->v), term(-dt, &ops->Jh, &T[CONVV]), term(1, &ops->Jh, &ops->bL_v)};
    qtt_mps y[2] = {T[RSU], T[RSV]};
    if ((rc = qtt_fit(ctx, 2, 3, t, y, chi, sweeps, init, mode, stream))) return rc;
    // initial guess of the solve: w0 = |J|^(1/2) rhs (H = I + O(dt/Re)); it carries the
    // bond structure of the right-hand side, which single-site updates cannot enlarge
    Batch b;
    b.n = 2;
    std::memset(&b.c[0], 0, sizeof(Chain) * 2);
    for (int i = 0; i < 2; ++i) {
      b.c[i].x = y[i].data; b.c[i].xb = y[i].bond; b.c[i].y = T[WU + i].data; b.c[i].yb = T[WU + i].bond;
      b.c[i].alpha = 1.0;
    }
    Geo g;
    std::memset(&g, 0, sizeof(g));
    g.L = L; g.capx = cap; g.capy = cap; g.d = 2;
    qttk::copy_mps(b, g, s);
    qtt_mpo hs[2] = {ops->Hs, ops->Hs};
    qtt_mps w[2] = {T[WU], T[WV]};
    qtt_solve_info hi[2];
    qtt_solve_opts ho = o->helmholtz;
    rc = qtt_poisson_solve(ctx, 2, hs, y, w, &ho, hi, stream);
    if (rc && rc != QTT_ENOTCONVERGED) return rc;
    if (info) { info->helm_u = hi[0]; info->helm_v = hi[1]; }
    qtt_mpo jmh[2] = {ops->Jmh, ops->Jmh};
    qtt_mps vs[2] = {T[US], T[VS]};
    if ((rc = qtt_apply_local(ctx, 2, jmh, w, vs, stream))) return rc;
  }
  // (4) J-weighted divergence and the pressure solve
  {
    const double idt = 1.0 / dt;
    qtt_term t[3] = {term(idt, &ops->Wx, &T[US]), term(idt, &ops->Wz, &T[VS]), term(idt, nullptr, &ops->bW)};
    if ((rc = qtt_fit(ctx, 1, 3, t, &T[BT], chi, sweeps, init, mode, stream))) return rc;
    if (o->rhs_out) {
      Batch b;
      b.n = 1;
      std::memset(&b.c[0], 0, sizeof(Chain));
      b.c[0].x = T[BT].data; b.c[0].xb = T[BT].bond; b.c[0].y = o->rhs_out->data; b.c[0].yb = o->rhs_out->bond;
      b.c[0].alpha = 1.0;
      Geo g;
      std::memset(&g, 0, sizeof(g));
      g.L = L; g.capx = cap; g.capy = o->rhs_out->cap; g.d = 2;
      qttk::copy_mps(b, g, s);
    }
    // the learned guess competes with state->p only when state->p is not this state's
    // previous pressure (its first step on the context, or another state ran since)
    if (o->warm && !warm && (rc = learned_guess(ctx, ops, st, o, T, L, cap, chi, wsf, info, stream))) return rc;
    qtt_solve_info pi;
    qtt_solve_opts po = o->poisson;
    rc = qtt_poisson_solve(ctx, 1, &ops->P, &T[BT], &st->p, &po, &pi, stream);
    if (rc && rc != QTT_ENOTCONVERGED) return rc;
    if (info) info->poisson = pi;
  }
  // (5) projection v = v* - dt grad p (the old velocity is the initial frame)
  {
    qtt_term t[4] = {term(1, nullptr, &T[US]), term(-dt, &ops->Dxp, &st->p),
                     term(1, nullptr, &T[VS]), term(-dt, &ops->Dzp, &st->p)};
    qtt_mps y[2] = {st->u, st->v};
    if ((rc = qtt_fit(ctx, 2, 2, t, y, chi, sweeps, init, mode, stream))) return rc;
  }
  set_step_warm(ctx, st->id, sid, L, cap);
  return QTT_OK;
}
