// Host-side construction of the cylinder operators as TT-matrices (setup, FP64).
//
// Sec. 3.2.3 builds the curvilinear operators once per grid; the paper builds
// the grid and its metric terms classically and encodes them into TTs
// (Sec. 4, grid paragraph). This file does the same on the host:
//   * O-grid points of App. E and metric terms by central differences (App. A);
//   * every operator written as a 3x3 stencil sum_o c_o(i,j) u(i+di, j+dj),
//     from the computational stencils of App. A composed with the metric
//     coefficients (Eq. curviliner-deriavtive, the seven-term Laplacian);
//   * ghost-point boundaries (Sec. 3.1): neighbours on the wall row (i = -1) or
//     the far-field row (i = N) go into a boundary-correction vector (velocity)
//     or are folded into the stencil (pressure, p_{-1} = p_0; p_N = 0);
//   * each coefficient field c_o encoded by TT-SVD, the shift S_o written as a
//     carry automaton (bond 2 per axis), the product diag(c_o) S_o formed core
//     by core with the copy tensor (Sec. 2.1.3), the terms direct-summed
//     (Sec. 2.1.1) and the MPO rounded, dropping singular values below 1e-14
//     of the largest at each bond (Sec. 3.2.3).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/qtt.h"
#include "host_linalg.h"
#include "cylinder_parts.h"

namespace {

struct Grid {
  int n, N;
  double r_out, deta, dxi;
  std::vector<double> r;     // rows i = -2 .. N+1  -> index i + 2
  std::vector<double> th;    // j = 0 .. N-1
  // metric terms on rows i = -1 .. N (index i + 1), N columns
  std::vector<double> x_xi, x_eta, z_xi, z_eta, J, g11, g22, g12;

  explicit Grid(int n_, double r_out_) : n(n_), N(1 << n_), r_out(r_out_) {
    deta = 1.0 / (N + 1);
    dxi = 1.0 / N;
    const double ratio = 2.0 * r_out / 1.0;   // D_outer / D with D = 1 (App. E, Eq. mesh)
    r.resize(N + 4);
    for (int i = -2; i <= N + 1; ++i) r[i + 2] = 0.5 * std::pow(ratio, (i + 1) * deta);
    th.resize(N);
    for (int j = 0; j < N; ++j) th[j] = 2.0 * M_PI * j * dxi;
    const int R = N + 2;
    x_xi.assign(R * N, 0); x_eta = z_xi = z_eta = J = g11 = g22 = g12 = x_xi;
    for (int i = -1; i <= N; ++i) {
      for (int j = 0; j < N; ++j) {
        const int jp = (j + 1) % N, jm = (j + N - 1) % N;
        auto X = [&](int ii, int jj) { return r[ii + 2] * std::cos(th[jj]); };
        auto Z = [&](int ii, int jj) { return r[ii + 2] * std::sin(th[jj]); };
        const int q = (i + 1) * N + j;
        x_xi[q] = (X(i, jp) - X(i, jm)) / (2 * dxi);
        z_xi[q] = (Z(i, jp) - Z(i, jm)) / (2 * dxi);
        x_eta[q] = (X(i + 1, j) - X(i - 1, j)) / (2 * deta);
        z_eta[q] = (Z(i + 1, j) - Z(i - 1, j)) / (2 * deta);
        J[q] = x_xi[q] * z_eta[q] - x_eta[q] * z_xi[q];
        g11[q] = x_xi[q] * x_xi[q] + z_xi[q] * z_xi[q];
        g22[q] = x_eta[q] * x_eta[q] + z_eta[q] * z_eta[q];
        g12[q] = x_xi[q] * x_eta[q] + z_xi[q] * z_eta[q];
      }
    }
  }
  double at(const std::vector<double>& a, int i, int j) const {  // rows -1..N
    return a[(i + 1) * N + ((j % N) + N) % N];
  }
};

// A 3x3 stencil operator: c[o][i*N + j], o = (di+1)*3 + (dj+1), on interior points.
struct Stencil {
  int N;
  std::vector<double> c[9];
  explicit Stencil(int N_) : N(N_) { for (auto& v : c) v.assign((size_t)N_ * N_, 0.0); }
  double& at(int di, int dj, int i, int j) { return c[(di + 1) * 3 + (dj + 1)][(size_t)i * N + j]; }
};

// Adds coef(i,j) * (computational stencil `kind`) to S. kind: 0 d_xi, 1 d_eta,
// 2 d_xixi, 3 d_etaeta, 4 d_xieta (App. A, second-order central).
template <class F>
void add_term(Stencil& S, const Grid& g, int kind, F coef) {
  const int N = g.N;
  const double hx = g.dxi, he = g.deta;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double a = coef(i, j);
      if (a == 0.0) continue;
      switch (kind) {
        case 0: S.at(0, 1, i, j) += a / (2 * hx); S.at(0, -1, i, j) -= a / (2 * hx); break;
        case 1: S.at(1, 0, i, j) += a / (2 * he); S.at(-1, 0, i, j) -= a / (2 * he); break;
        case 2: S.at(0, 1, i, j) += a / (hx * hx); S.at(0, 0, i, j) -= 2 * a / (hx * hx);
                S.at(0, -1, i, j) += a / (hx * hx); break;
        case 3: S.at(1, 0, i, j) += a / (he * he); S.at(0, 0, i, j) -= 2 * a / (he * he);
                S.at(-1, 0, i, j) += a / (he * he); break;
        case 4: { const double w = a / (4 * hx * he);
                  S.at(1, 1, i, j) += w; S.at(1, -1, i, j) -= w; S.at(-1, 1, i, j) -= w; S.at(-1, -1, i, j) += w; }
                break;
      }
    }
}

Stencil make_dx(const Grid& g) {   // (1/J)(z_eta d_xi - z_xi d_eta)
  Stencil S(g.N);
  add_term(S, g, 0, [&](int i, int j) { return g.at(g.z_eta, i, j) / g.at(g.J, i, j); });
  add_term(S, g, 1, [&](int i, int j) { return -g.at(g.z_xi, i, j) / g.at(g.J, i, j); });
  return S;
}
Stencil make_dz(const Grid& g) {   // (1/J)(-x_eta d_xi + x_xi d_eta)
  Stencil S(g.N);
  add_term(S, g, 0, [&](int i, int j) { return -g.at(g.x_eta, i, j) / g.at(g.J, i, j); });
  add_term(S, g, 1, [&](int i, int j) { return g.at(g.x_xi, i, j) / g.at(g.J, i, j); });
  return S;
}
Stencil make_lap(const Grid& g) {  // seven-term Laplacian of App. A
  Stencil S(g.N);
  auto a22 = [&](int i, int j) { return g.at(g.g22, i, j) / g.at(g.J, i, j); };
  auto a11 = [&](int i, int j) { return g.at(g.g11, i, j) / g.at(g.J, i, j); };
  auto a12 = [&](int i, int j) { return g.at(g.g12, i, j) / g.at(g.J, i, j); };
  auto dxi = [&](auto f, int i, int j) { return (f(i, j + 1) - f(i, j - 1)) / (2 * g.dxi); };
  auto deta = [&](auto f, int i, int j) { return (f(i + 1, j) - f(i - 1, j)) / (2 * g.deta); };
  auto iJ = [&](int i, int j) { return 1.0 / g.at(g.J, i, j); };
  add_term(S, g, 0, [&](int i, int j) { return iJ(i, j) * (dxi(a22, i, j) - deta(a12, i, j)); });
  add_term(S, g, 2, [&](int i, int j) { return iJ(i, j) * a22(i, j); });
  add_term(S, g, 1, [&](int i, int j) { return iJ(i, j) * (deta(a11, i, j) - dxi(a12, i, j)); });
  add_term(S, g, 4, [&](int i, int j) { return -2.0 * iJ(i, j) * a12(i, j); });
  add_term(S, g, 3, [&](int i, int j) { return iJ(i, j) * a11(i, j); });
  return S;
}

// Boundary-correction vector of a Dirichlet field: sum over neighbours on row -1 / N.
std::vector<double> dirichlet_bc(const Stencil& S, const Grid& g, const std::vector<double>& wall,
                                 const std::vector<double>& outer) {
  const int N = g.N;
  std::vector<double> b((size_t)N * N, 0.0);
  for (int di = -1; di <= 1; ++di)
    for (int dj = -1; dj <= 1; ++dj) {
      const auto& c = S.c[(di + 1) * 3 + (dj + 1)];
      for (int i = 0; i < N; ++i) {
        const int ii = i + di;
        if (ii >= 0 && ii < N) continue;
        const auto& val = ii < 0 ? wall : outer;
        for (int j = 0; j < N; ++j) b[(size_t)i * N + j] += c[(size_t)i * N + j] * val[((j + dj) % N + N) % N];
      }
    }
  return b;
}

// Pressure boundaries: p_{-1,j} = p_{0,j} folded into the row-0 stencil; p_N = 0 (dropped).
void fold_pressure(Stencil& S) {
  const int N = S.N;
  for (int dj = -1; dj <= 1; ++dj)
    for (int j = 0; j < N; ++j) {
      S.at(0, dj, 0, j) += S.at(-1, dj, 0, j);
      S.at(-1, dj, 0, j) = 0.0;
    }
}

// Left-multiply by diag(f) (f on interior points).
void scale_rows(Stencil& S, const std::vector<double>& f) {
  for (auto& c : S.c)
    for (size_t q = 0; q < c.size(); ++q) c[q] *= f[q];
}

// ---------------------------------------------------------------------------
// TT encodings
// ---------------------------------------------------------------------------

// Bit order of the encodings of the current qtt_build_host call (QTT_ORDER_*),
// per thread: interleaved i_1 j_1 i_2 j_2 ... or concatenated i_1 .. i_n j_1 .. j_n
// (Sec. 3.2.1), MSB first in both.
thread_local int t_order = QTT_ORDER_INTERLEAVED;

// Position of grid point (i, j) in the dense vector of the current order.
size_t qidx(int i, int j, int n) {
  if (t_order == QTT_ORDER_CONCATENATED) return ((size_t)i << n) | (size_t)j;
  size_t q = 0;
  for (int m = 0; m < n; ++m) {
    q = (q << 2) | ((size_t)((i >> (n - 1 - m)) & 1) << 1) | (size_t)((j >> (n - 1 - m)) & 1);
  }
  return q;
}

// Is core k a digit of the eta (row) index in the current order?
bool eta_core(int k, int n) { return t_order == QTT_ORDER_CONCATENATED ? k < n : (k % 2 == 0); }

std::vector<double> to_qtt_order(const std::vector<double>& f, int n) {
  const int N = 1 << n;
  std::vector<double> v((size_t)N * N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) v[qidx(i, j, n)] = f[(size_t)i * N + j];
  return v;
}

// Shift automaton core for one digit (Sec. 2.1.2 via binary addition with carry):
// (S x)(out) = x(out + s) with s in {-1, 0, +1}; carry flows from the least
// significant digit (right) to the most significant (left).
// T[c_left][o][r][c_right] = 1 iff r == (o + s*c_right) mod 2 and c_left is the
// carry (s=+1) or borrow (s=-1) produced; for s = 0 only c = 0 is used.
double shift_digit(int s, int cl, int o, int r, int cr) {
  if (s == 0) return (cl == 0 && cr == 0 && o == r) ? 1.0 : 0.0;
  if (s > 0) {
    const int t = o + cr;
    return ((t & 1) == r && (t >> 1) == cl) ? 1.0 : 0.0;
  }
  const int t = o - cr;
  return (((t % 2) + 2) % 2 == r && (t < 0 ? 1 : 0) == cl) ? 1.0 : 0.0;
}

// MPO of the 2D shift u(i+di, j+dj), zero outside 0 <= i+di < N, periodic in j.
// Bond state (c_eta, c_xi), 4 states: each carry flows from its coordinate's least
// significant digit to its most significant one and passes unchanged through the
// cores of the other coordinate, so one automaton serves both bit orders.
HostTT shift_mpo(int n, int di, int dj) {
  const int L = 2 * n;
  HostTT T;
  T.L = L; T.d = 4;
  for (int k = 0; k < L; ++k) {
    const bool eta = eta_core(k, n);
    const int wl = (k == 0) ? 1 : 4, wr = (k == L - 1) ? 1 : 4;
    std::vector<double> core((size_t)wl * 4 * wr, 0.0);
    for (int a = 0; a < wl; ++a)
      for (int b = 0; b < wr; ++b)
        for (int o = 0; o < 2; ++o)
          for (int r = 0; r < 2; ++r) {
            double tot = 0.0;
            // enumerate full left states consistent with the boundary
            for (int ceL = 0; ceL < 2; ++ceL)
              for (int cxL = 0; cxL < 2; ++cxL) {
                if (k == 0) {                                   // MSB end
                  if (ceL != 0) continue;                       // zero fill in eta
                } else if (a != ceL * 2 + cxL) continue;
                int ceR, cxR;
                if (k == L - 1) { ceR = (di != 0); cxR = (dj != 0); }   // LSB end: initial carries
                else { ceR = b / 2; cxR = b % 2; }
                double v = 0.0;
                if (eta) v = shift_digit(di, ceL, o, r, ceR) * (cxL == cxR ? 1.0 : 0.0);
                else     v = shift_digit(dj, cxL, o, r, cxR) * (ceL == ceR ? 1.0 : 0.0);
                if (di == 0 && (ceL | ceR)) v = 0.0;
                if (dj == 0 && (cxL | cxR)) v = 0.0;
                tot += v;
              }
            core[((size_t)a * 4 + o * 2 + r) * wr + b] = tot;
          }
    T.cores.push_back(core);
    T.bl.push_back(wl);
  }
  T.bl.push_back(1);
  return T;
}

// diag(c) * S: core (a,p | o,r | b,q) = C[a][o][b] * S[p][o][r][q]  (copy tensor, Sec. 2.1.3)
HostTT diag_times(const HostTT& C, const HostTT& S) {
  HostTT P;
  P.L = C.L; P.d = 4;
  for (int k = 0; k < C.L; ++k) {
    const int ca = C.bl[k], cb = C.bl[k + 1], sa = S.bl[k], sb = S.bl[k + 1];
    std::vector<double> core((size_t)ca * sa * 4 * cb * sb, 0.0);
    for (int a = 0; a < ca; ++a)
      for (int p = 0; p < sa; ++p)
        for (int o = 0; o < 2; ++o)
          for (int r = 0; r < 2; ++r)
            for (int b = 0; b < cb; ++b)
              for (int q = 0; q < sb; ++q)
                core[(((size_t)(a * sa + p) * 4 + o * 2 + r) * cb + b) * sb + q] =
                    C.cores[k][((size_t)a * 2 + o) * cb + b] * S.cores[k][((size_t)p * 4 + o * 2 + r) * sb + q];
    P.cores.push_back(core);
    P.bl.push_back(ca * sa);
  }
  P.bl.push_back(C.bl[C.L] * S.bl[C.L]);
  return P;
}

// Operator stencil -> rounded MPO.
HostTT stencil_to_mpo(const Stencil& S, int n) {
  double cmax = 0.0;
  for (const auto& c : S.c) {
    double s2 = 0.0;
    for (double v : c) s2 += v * v;
    cmax = std::max(cmax, std::sqrt(s2));
  }
  HostTT acc;
  bool have = false;
  const int L = 2 * n;
  for (int di = -1; di <= 1; ++di)
    for (int dj = -1; dj <= 1; ++dj) {
      const auto& c = S.c[(di + 1) * 3 + (dj + 1)];
      double s2 = 0.0;
      for (double v : c) s2 += v * v;
      if (std::sqrt(s2) <= 1e-14 * cmax) continue;
      HostTT C = tt_svd_host(to_qtt_order(c, n), L, 2, 0.0, 1 << 30, 1e-14 * cmax);
      HostTT term = diag_times(C, shift_mpo(n, di, dj));
      if (!have) { acc = term; have = true; }
      else acc = tt_direct_sum(acc, term);
    }
  if (!have) {  // zero operator: bond-1 zero cores
    acc.L = L; acc.d = 4;
    for (int k = 0; k < L; ++k) { acc.cores.push_back(std::vector<double>(4, 0.0)); acc.bl.push_back(1); }
    acc.bl.push_back(1);
    return acc;
  }
  tt_round_host(acc, 1e-14);
  return acc;
}

// Dense interior field -> TT (bond-dimension set by relative tolerance 1e-14).
HostTT field_to_tt(const std::vector<double>& f, int n) {
  double s2 = 0.0;
  for (double v : f) s2 += v * v;
  const double nrm = std::sqrt(s2);
  return tt_svd_host(to_qtt_order(f, n), 2 * n, 2, 0.0, 1 << 30, 1e-14 * std::max(nrm, 1e-300));
}

// Diagonal bond-1 MPO of a field that must be rank one (e.g. |J|^(1/2)).
HostTT diag_mpo_of(const std::vector<double>& f, int n) {
  HostTT C = field_to_tt(f, n);
  HostTT D = diag_times(C, shift_mpo(n, 0, 0));
  tt_round_host(D, 1e-14);
  return D;
}

int write_mpo(const HostTT& T, int32_t wcap, double* out, int32_t* bond_out, int32_t* need) {
  int32_t w = 0;
  for (int b : T.bl) w = std::max(w, b);
  if (need) *need = w;
  if (!out) return QTT_OK;
  if (w > wcap) return QTT_ECAPACITY;
  const size_t slot = (size_t)wcap * 4 * wcap;
  std::memset(out, 0, sizeof(double) * slot * T.L);
  for (int k = 0; k < T.L; ++k) {
    const int a0 = T.bl[k], b0 = T.bl[k + 1];
    for (int a = 0; a < a0; ++a)
      for (int s = 0; s < 4; ++s)
        for (int b = 0; b < b0; ++b)
          out[k * slot + (size_t)a * 4 * wcap + s * wcap + b] = T.cores[k][((size_t)a * 4 + s) * b0 + b];
  }
  for (int k = 0; k <= T.L; ++k) bond_out[k] = T.bl[k];
  return QTT_OK;
}

int write_mps(const HostTT& T, int32_t cap, double* out, int32_t* bond_out, int32_t* need) {
  int32_t w = 0;
  for (int b : T.bl) w = std::max(w, b);
  if (need) *need = w;
  if (!out) return QTT_OK;
  if (w > cap) return QTT_ECAPACITY;
  const int d = T.d;
  const size_t slot = (size_t)cap * d * cap;
  std::memset(out, 0, sizeof(double) * slot * T.L);
  for (int k = 0; k < T.L; ++k) {
    const int a0 = T.bl[k], b0 = T.bl[k + 1];
    for (int a = 0; a < a0; ++a)
      for (int s = 0; s < d; ++s)
        for (int b = 0; b < b0; ++b)
          out[k * slot + (size_t)a * d * cap + s * cap + b] = T.cores[k][((size_t)a * d + s) * b0 + b];
  }
  for (int k = 0; k <= T.L; ++k) bond_out[k] = T.bl[k];
  return QTT_OK;
}

}  // namespace

// ---- pieces the TT-format construction (ttbuild.hip) shares ------------------
HostTT cyl_shift_mpo(int n, int di, int dj, int order) {
  const int saved = t_order;
  t_order = order;
  HostTT T = shift_mpo(n, di, dj);
  t_order = saved;
  return T;
}

double cyl_row_radius(int i, int n, double r_out) {
  const int N = 1 << n;
  return 0.5 * std::pow(2.0 * r_out, (i + 1) * (1.0 / (N + 1)));
}

extern "C" int qtt_build_host(const qtt_cylinder* cyl, int which, int32_t cap, double* out,
                              int32_t* bond_out, int32_t* need) {
  if (!cyl || cyl->n < 1 || cyl->n > 13 || !(cyl->r_out > 0.5)) return QTT_EINVAL;
  if (cyl->order != QTT_ORDER_INTERLEAVED && cyl->order != QTT_ORDER_CONCATENATED) return QTT_EINVAL;
  if (out && !bond_out) return QTT_EINVAL;
  struct OrderScope {      // the bit order of this call's encodings, restored on return
    int saved;
    explicit OrderScope(int o) : saved(t_order) { t_order = o; }
    ~OrderScope() { t_order = saved; }
  } order_scope(cyl->order);
  const int n = cyl->n;
  const Grid g(n, cyl->r_out);
  const int N = g.N;
  const size_t NN = (size_t)N * N;
  std::vector<double> absJ(NN), jh(NN), jmh(NN);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double a = std::fabs(g.at(g.J, i, j));
      absJ[(size_t)i * N + j] = a;
      jh[(size_t)i * N + j] = std::sqrt(a);
      jmh[(size_t)i * N + j] = 1.0 / std::sqrt(a);
    }
  std::vector<double> u_wall(N), v_wall(N), u_out(N, cyl->u_inf), v_out(N, 0.0);
  for (int j = 0; j < N; ++j) {           // Eq. (rot_bc); alpha = 0 is the resting wall
    u_wall[j] = cyl->alpha * std::sin(g.th[j]);
    v_wall[j] = -cyl->alpha * std::cos(g.th[j]);
  }
  auto mpo = [&](const HostTT& T) { return write_mpo(T, cap, out, bond_out, need); };
  auto vec = [&](const std::vector<double>& f) { return write_mps(field_to_tt(f, n), cap, out, bond_out, need); };
  const double c = (cyl->Re > 0) ? cyl->dt / cyl->Re : 0.0;

  switch (which) {
    case QTT_OP_DX: return mpo(stencil_to_mpo(make_dx(g), n));
    case QTT_OP_DZ: return mpo(stencil_to_mpo(make_dz(g), n));
    case QTT_OP_LAP: return mpo(stencil_to_mpo(make_lap(g), n));
    case QTT_OP_DXP: { Stencil S = make_dx(g); fold_pressure(S); return mpo(stencil_to_mpo(S, n)); }
    case QTT_OP_DZP: { Stencil S = make_dz(g); fold_pressure(S); return mpo(stencil_to_mpo(S, n)); }
    case QTT_OP_WX: case QTT_OP_WZ: {
      Stencil S = which == QTT_OP_WX ? make_dx(g) : make_dz(g);
      std::vector<double> m(NN);
      for (size_t q = 0; q < NN; ++q) m[q] = -absJ[q];
      scale_rows(S, m);
      return mpo(stencil_to_mpo(S, n));
    }
    case QTT_OP_P: {
      Stencil S = make_lap(g);
      fold_pressure(S);
      std::vector<double> m(NN);
      for (size_t q = 0; q < NN; ++q) m[q] = -absJ[q];
      scale_rows(S, m);
      return mpo(stencil_to_mpo(S, n));
    }
    case QTT_OP_HS: {
      // |J|^(1/2) (I - c Lap) |J|^(-1/2): coefficient of neighbour o at (i,j) times
      // |J|^(-1/2) of that neighbour; boundary neighbours vanish through the zero fill.
      Stencil L = make_lap(g);
      Stencil S(N);
      for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj)
          for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
              const int ii = i + di, jj = ((j + dj) % N + N) % N;
              if (ii < 0 || ii >= N) continue;
              double a = -c * L.at(di, dj, i, j);
              if (di == 0 && dj == 0) a += 1.0;
              S.at(di, dj, i, j) = jh[(size_t)i * N + j] * a * jmh[(size_t)ii * N + jj];
            }
      return mpo(stencil_to_mpo(S, n));
    }
    case QTT_OP_JH: return mpo(diag_mpo_of(jh, n));
    case QTT_OP_JMH: return mpo(diag_mpo_of(jmh, n));
    case QTT_VEC_BX_U: return vec(dirichlet_bc(make_dx(g), g, u_wall, u_out));
    case QTT_VEC_BZ_U: return vec(dirichlet_bc(make_dz(g), g, u_wall, u_out));
    case QTT_VEC_BX_V: return vec(dirichlet_bc(make_dx(g), g, v_wall, v_out));
    case QTT_VEC_BZ_V: return vec(dirichlet_bc(make_dz(g), g, v_wall, v_out));
    case QTT_VEC_BL_U: case QTT_VEC_BL_V: {
      auto b = dirichlet_bc(make_lap(g), g, which == QTT_VEC_BL_U ? u_wall : v_wall,
                            which == QTT_VEC_BL_U ? u_out : v_out);
      for (auto& x : b) x *= c;
      return vec(b);
    }
    case QTT_VEC_BW: {
      auto bx = dirichlet_bc(make_dx(g), g, u_wall, u_out);
      auto bz = dirichlet_bc(make_dz(g), g, v_wall, v_out);
      for (size_t q = 0; q < NN; ++q) bx[q] = -absJ[q] * (bx[q] + bz[q]);
      return vec(bx);
    }
    case QTT_VEC_ABSJ: return vec(absJ);
    default: return QTT_EINVAL;
  }
}

extern "C" int qtt_tt_svd_host(const double* dense, int32_t L, int32_t d, const qtt_trunc* tr,
                               int32_t cap, double* out, int32_t* bond_out) {
  if (!dense || !tr || !out || !bond_out || L < 1 || d < 2 || cap < 1) return QTT_EINVAL;
  size_t n = 1;
  for (int k = 0; k < L; ++k) n *= (size_t)d;
  std::vector<double> v(dense, dense + n);
  HostTT T = tt_svd_host(v, L, d, tr->rel_tol, std::min<int>(tr->chi_max, cap), 0.0);
  return write_mps(T, cap, out, bond_out, nullptr);
}

// Wall forces of App. F (drag and lift coefficients, rho = U = D = 1, Eq. liftdrag)
// from the first two interior rows of u and v, the first of p, and the prescribed
// wall velocity (Eq. rot_bc): tau = -(p + 2/(3Re) div v) I + (1/Re)(grad v + grad v^T),
// force = sum_j tau n_j (D/2) 2 pi d_xi with n = (cos, sin) into the fluid; wall
// derivatives one-sided second order in eta (rows -1, 0, 1), central in xi along
// the wall, mapped with the row -1 metric terms.
extern "C" int qtt_forces_host(const qtt_cylinder* cyl, const double* rows, double* cd, double* cl) {
  if (!cyl || !rows || !cd || !cl || cyl->n < 2 || cyl->n > 14 || !(cyl->Re > 0.0)) return QTT_EINVAL;
  const Grid g(cyl->n, cyl->r_out);
  const int N = g.N;
  const double* u0 = rows;
  const double* u1 = rows + N;
  const double* v0 = rows + 2 * N;
  const double* v1 = rows + 3 * N;
  const double* p0 = rows + 4 * N;
  std::vector<double> uw(N), vw(N);
  for (int j = 0; j < N; ++j) { uw[j] = cyl->alpha * std::sin(g.th[j]); vw[j] = -cyl->alpha * std::cos(g.th[j]); }
  auto grad = [&](const std::vector<double>& fw, const double* f0, const double* f1, int j, double* fx, double* fz) {
    const double fxi = (fw[(j + 1) % N] - fw[(j + N - 1) % N]) / (2.0 * g.dxi);
    const double feta = (-3.0 * fw[j] + 4.0 * f0[j] - f1[j]) / (2.0 * g.deta);
    const double J = g.at(g.J, -1, j);
    *fx = (g.at(g.z_eta, -1, j) * fxi - g.at(g.z_xi, -1, j) * feta) / J;
    *fz = (-g.at(g.x_eta, -1, j) * fxi + g.at(g.x_xi, -1, j) * feta) / J;
  };
  const double Re = cyl->Re, ds = g.r[1] * 2.0 * M_PI * g.dxi;    // r[1] is row -1: the wall, D/2
  double Fx = 0.0, Fz = 0.0;
  for (int j = 0; j < N; ++j) {
    double ux, uz, vx, vz;
    grad(uw, u0, u1, j, &ux, &uz);
    grad(vw, v0, v1, j, &vx, &vz);
    const double div = ux + vz, pres = p0[j] + 2.0 / (3.0 * Re) * div;
    const double t11 = -pres + 2.0 / Re * ux, t22 = -pres + 2.0 / Re * vz, t12 = (uz + vx) / Re;
    const double c = std::cos(g.th[j]), s = std::sin(g.th[j]);
    Fx += (t11 * c + t12 * s) * ds;
    Fz += (t12 * c + t22 * s) * ds;
  }
  *cd = 2.0 * Fx;
  *cl = 2.0 * Fz;
  return QTT_OK;
}

// Strouhal number and lift amplitude of a lift history (Sec. 4.1.2: interpolated
// zero crossings of C_L; Eq. st with D = U = 1): over the last `window` of the
// samples, y = C_L - mean; upward crossings (y_i < 0 <= y_{i+1}) are located by
// linear interpolation; St = 1 / (mean spacing of the crossings).
extern "C" int qtt_strouhal_host(const double* t, const double* cl, int64_t n, double window, int32_t min_crossings,
                                 double* st, double* amp) {
  if (!t || !cl || !st || !amp || n < 2 || !(window > 0.0 && window <= 1.0) || min_crossings < 2) return QTT_EINVAL;
  const int64_t n0 = (int64_t)((double)n * (1.0 - window));
  const int64_t m = n - n0;
  if (m < 2) return QTT_EINVAL;
  double mean = 0.0, lo = cl[n0], hi = cl[n0];
  for (int64_t i = n0; i < n; ++i) {
    mean += cl[i];
    lo = std::min(lo, cl[i]);
    hi = std::max(hi, cl[i]);
  }
  mean /= (double)m;
  *amp = 0.5 * (hi - lo);
  double first = 0.0, last = 0.0;
  int64_t count = 0;
  for (int64_t i = n0; i + 1 < n; ++i) {
    const double y0 = cl[i] - mean, y1 = cl[i + 1] - mean;
    if (y0 < 0.0 && y1 >= 0.0) {
      const double tc = t[i] - y0 * (t[i + 1] - t[i]) / (y1 - y0);
      if (count == 0) first = tc;
      last = tc;
      ++count;
    }
  }
  *st = (count >= min_crossings && last > first) ? (double)(count - 1) / (last - first) : NAN;
  return QTT_OK;
}

// Input of the learned warm start's network from the block-averaged right-hand
// side b (64 x 64, [eta][xi]): channels b / rms(b), Re / 200, alpha / 2 (FP32,
// NCHW); rms(b) is returned, being the scale of the network's output.
extern "C" int qtt_ws_input_host(const double* coarse_b, double re, double alpha, float* in, double* rms) {
  if (!coarse_b || !in || !rms) return QTT_EINVAL;
  double ms = 0.0;
  for (int e = 0; e < 4096; ++e) ms += coarse_b[e] * coarse_b[e];
  const double r = std::sqrt(ms / 4096.0);
  *rms = r;
  if (!(r > 0.0) || !std::isfinite(r)) return QTT_ENUMERIC;
  for (int e = 0; e < 4096; ++e) {
    in[e] = (float)(coarse_b[e] / r);
    in[4096 + e] = (float)(re / 200.0);
    in[8192 + e] = (float)(alpha / 2.0);
  }
  return QTT_OK;
}
