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
// previous step on this context advanced the same state (same u, v, p storage),
// the fits start from that step's results, otherwise from a random sketch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/qtt.h"
#include "internal.h"

namespace qtt_solver_detail {
double* step_pool(qtt_ctx* ctx, size_t doubles, int* rc);
int set_error(qtt_ctx* ctx, int code, const char* msg);
bool step_warm(qtt_ctx* ctx, const void* const id[3], int L, int cap);
void set_step_warm(qtt_ctx* ctx, const void* const id[3], int L, int cap);
}

namespace {
enum { GXU = 0, GZU, GXV, GZV, CONVU, CONVV, RSU, RSV, WU, WV, US, VS, BT, NTMP };
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
  const qtt_mps* bcs[7] = {&ops->bx_u, &ops->bz_u, &ops->bx_v, &ops->bz_v, &ops->bL_u, &ops->bL_v, &ops->bW};
  for (auto* b : bcs)
    if (b->L != L || b->cap != ops->bx_u.cap) return set_error(ctx, QTT_ESHAPE, "step: boundary vectors must share L and cap");

  // temporaries: NTMP trains of cap `cap` and two diagonal MPOs (wcap = cap)
  const size_t slot = (size_t)L * cap * 2 * cap;
  const size_t mslot = (size_t)L * cap * 4 * cap;
  const size_t ints = (size_t)(NTMP + 2) * 64;
  int rc = 0;
  double* pool = step_pool(ctx, NTMP * slot + 2 * mslot + ints / 2 + 64, &rc);
  if (rc) return rc;
  int* ib = reinterpret_cast<int*>(pool + NTMP * slot + 2 * mslot);
  qtt_mps T[NTMP];
  for (int i = 0; i < NTMP; ++i) T[i] = qtt_mps{L, 2, cap, ib + 64 * i, pool + slot * i};
  std::vector<int32_t> diag_bonds(L + 1, cap);
  diag_bonds[0] = diag_bonds[L] = 1;
  qtt_mpo DU{L, cap, diag_bonds.data(), ib + 64 * NTMP, pool + NTMP * slot};
  qtt_mpo DV{L, cap, diag_bonds.data(), ib + 64 * (NTMP + 1), pool + NTMP * slot + mslot};

  const int chi = std::min(o->trunc.chi_max, cap);
  // warm fits only when the temporaries come from the previous step of this state
  const void* const sid[3] = {st->u.data, st->v.data, st->p.data};
  const bool warm = step_warm(ctx, sid, L, cap);
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
  set_step_warm(ctx, sid, L, cap);
  return QTT_OK;
}
