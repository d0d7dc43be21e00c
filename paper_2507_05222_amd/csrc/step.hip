// One Chorin fractional step in TT format (Sec. 3.3 of arxiv 2507.05222),
// composed from the library's own entry points:
//   convection     (v.grad) v with v and its curvilinear gradients (Hadamard
//                  products through the copy tensor, Sec. 2.1.3),
//   predictor      (I - dt/Re Lap) v* = v - dt (v.grad) v (Eq. intermediate_vel_eq),
//                  solved variationally in the symmetric form
//                  |J|^(1/2)(I - dt/Re Lap)|J|^(-1/2) w = |J|^(1/2) rhs, v* = |J|^(-1/2) w,
//   pressure       (-|J| Lap) p = -|J| (1/dt) div v* (Eq. Poisson, J-weighted, Sec. 3.3),
//   projection     v = v* - dt grad p.
// Independent chains (u and v, the four gradients, the four products) run
// batched in one call each.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/qtt.h"
#include "internal.h"

namespace qtt_solver_detail {
double* step_pool(qtt_ctx* ctx, size_t doubles, int* rc);
int set_error(qtt_ctx* ctx, int code, const char* msg);
}

namespace {
enum {
  A_GXU = 0, A_GZU, A_GXV, A_GZV, GXU, GZU, GXV, GZV, H0, H1, H2, H3, CONVU, CONVV, R1U, R1V, RHSU, RHSV,
  RSU, RSV, WU, WV, US, VS, D0, D1, D01, BT, Q0, Q1, NTMP
};
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

  const qtt_trunc* tr = &o->trunc;
  const int mode = o->contract_dt;
  const double dt = o->dt;
  hipStream_t s = (hipStream_t)stream;

  // (1) curvilinear gradients of u and v: D x + boundary correction (Sec. 3.1)
  {
    qtt_mpo M[4] = {ops->Dx, ops->Dz, ops->Dx, ops->Dz};
    qtt_mps x[4] = {st->u, st->u, st->v, st->v};
    qtt_mps y[4] = {T[A_GXU], T[A_GZU], T[A_GXV], T[A_GZV]};
    if ((rc = qtt_apply_mpo(ctx, 4, M, x, y, tr, mode, stream))) return rc;
    double one[4] = {1, 1, 1, 1};
    qtt_mps b[4] = {ops->bx_u, ops->bz_u, ops->bx_v, ops->bz_v};
    qtt_mps z[4] = {T[GXU], T[GZU], T[GXV], T[GZV]};
    if ((rc = qtt_add(ctx, 4, one, y, one, b, z, tr, stream))) return rc;
  }
  // (2) convection: u d_x u + v d_z u, u d_x v + v d_z v (elementwise products)
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
    qtt_mpo M[4] = {DU, DV, DU, DV};
    qtt_mps x[4] = {T[GXU], T[GZU], T[GXV], T[GZV]};
    qtt_mps y[4] = {T[H0], T[H1], T[H2], T[H3]};
    if ((rc = qtt_apply_mpo(ctx, 4, M, x, y, tr, o->product_dt, stream))) return rc;
    double one[2] = {1, 1};
    qtt_mps a2[2] = {T[H0], T[H2]}, b2[2] = {T[H1], T[H3]}, c2[2] = {T[CONVU], T[CONVV]};
    if ((rc = qtt_add(ctx, 2, one, a2, one, b2, c2, tr, stream))) return rc;
  }
  // (3) predictor right-hand side, scaled by |J|^(1/2)
  {
    double one[2] = {1, 1}, mdt[2] = {-dt, -dt};
    qtt_mps uv[2] = {st->u, st->v}, cv[2] = {T[CONVU], T[CONVV]}, r1[2] = {T[R1U], T[R1V]};
    if ((rc = qtt_add(ctx, 2, one, uv, mdt, cv, r1, tr, stream))) return rc;
    qtt_mps bl[2] = {ops->bL_u, ops->bL_v}, rhs[2] = {T[RHSU], T[RHSV]};
    if ((rc = qtt_add(ctx, 2, one, r1, one, bl, rhs, tr, stream))) return rc;
    qtt_mpo jh[2] = {ops->Jh, ops->Jh};
    qtt_mps rs[2] = {T[RSU], T[RSV]}, w[2] = {T[WU], T[WV]};
    if ((rc = qtt_apply_local(ctx, 2, jh, rhs, rs, stream))) return rc;
    // initial guess w0 = |J|^(1/2) rhs (H = I + O(dt/Re)); it carries the bond
    // structure of the right-hand side, which single-site updates cannot enlarge
    {
      Batch b;
      b.n = 2;
      std::memset(&b.c[0], 0, sizeof(Chain) * 2);
      for (int i = 0; i < 2; ++i) {
        b.c[i].x = rs[i].data; b.c[i].xb = rs[i].bond; b.c[i].y = w[i].data; b.c[i].yb = w[i].bond;
        b.c[i].alpha = 1.0;
      }
      Geo g;
      std::memset(&g, 0, sizeof(g));
      g.L = L; g.capx = cap; g.capy = cap; g.d = 2;
      qttk::copy_mps(b, g, s);
    }
    qtt_mpo hs[2] = {ops->Hs, ops->Hs};
    qtt_solve_info hi[2];
    qtt_solve_opts ho = o->helmholtz;
    rc = qtt_poisson_solve(ctx, 2, hs, rs, w, &ho, hi, stream);
    if (rc && rc != QTT_ENOTCONVERGED) return rc;
    if (info) { info->helm_u = hi[0]; info->helm_v = hi[1]; }
    qtt_mpo jmh[2] = {ops->Jmh, ops->Jmh};
    qtt_mps vs[2] = {T[US], T[VS]};
    if ((rc = qtt_apply_local(ctx, 2, jmh, w, vs, stream))) return rc;
  }
  // (4) J-weighted divergence and pressure solve
  {
    qtt_mpo M[2] = {ops->Wx, ops->Wz};
    qtt_mps x[2] = {T[US], T[VS]}, y[2] = {T[D0], T[D1]};
    if ((rc = qtt_apply_mpo(ctx, 2, M, x, y, tr, mode, stream))) return rc;
    double one = 1.0, idt = 1.0 / dt;
    if ((rc = qtt_add(ctx, 1, &one, &T[D0], &one, &T[D1], &T[D01], tr, stream))) return rc;
    if ((rc = qtt_add(ctx, 1, &idt, &T[D01], &idt, &ops->bW, &T[BT], tr, stream))) return rc;
    qtt_solve_info pi;
    qtt_solve_opts po = o->poisson;
    rc = qtt_poisson_solve(ctx, 1, &ops->P, &T[BT], &st->p, &po, &pi, stream);
    if (rc && rc != QTT_ENOTCONVERGED) return rc;
    if (info) info->poisson = pi;
  }
  // (5) projection v = v* - dt grad p
  {
    qtt_mpo M[2] = {ops->Dxp, ops->Dzp};
    qtt_mps x[2] = {st->p, st->p}, y[2] = {T[Q0], T[Q1]};
    if ((rc = qtt_apply_mpo(ctx, 2, M, x, y, tr, mode, stream))) return rc;
    double one[2] = {1, 1}, mdt[2] = {-dt, -dt};
    qtt_mps vs[2] = {T[US], T[VS]}, out[2] = {st->u, st->v};
    if ((rc = qtt_add(ctx, 2, one, vs, mdt, y, out, tr, stream))) return rc;
  }
  return QTT_OK;
}
