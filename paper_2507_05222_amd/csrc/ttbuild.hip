// The cylinder's curvilinear operators built in TT format on the device (Sec. 3.2.2
// mesh generation, Sec. 3.2.3 operator construction), as an alternative to the
// classical construction of builder.cpp. Nothing here forms a field of 2^n x 2^n
// values: the grid coordinates are direct sums of concatenated 1D trains, the metric
// terms come from derivative MPOs applied to them, the Jacobian from Hadamard
// products, its inverse from an ALS solve of diag(J) a = 1, and the operators from
// MPO products diag(c) D with the computational derivatives D. Every operation is
// followed by a truncation (Sec. 3.2.3: 1e-14 for the fields, 1e-13 for the
// operators); products are formed exactly and rounded by QR and Jacobi SVD sweeps.
//
// Host code only touches O(n 2^n) data: the 1D boundary curves (wall, far field,
// unit normals) and the small cores of the shift automata.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/qtt.h"
#include "cylinder_parts.h"
#include "host_linalg.h"
#include "internal.h"

namespace qtt_solver_detail {
// Declared in api.hip.
int set_error(qtt_ctx* ctx, int code, const char* msg);
int device_of(qtt_ctx* ctx);
}

namespace {
using qtt_solver_detail::set_error;

constexpr double TT_TOL = 1e-14;   // truncation after every TT operation (Sec. 3.2.3)
// The device rounding bounds the discarded Frobenius norm by rel_tol / sqrt(sites - 1)
// per bond; to drop, as the paper does, what lies below 1e-14 of the train's norm at
// each bond, rel_tol is scaled by sqrt(sites - 1).
inline double bond_tol(int sites, double tol = TT_TOL) { return tol * std::sqrt((double)std::max(sites - 1, 1)); }
// The operators themselves (MPO sums and products) are rounded at 1e-13 per bond: the
// chain of operations before them (metric terms, products, the inverse Jacobian) leaves
// singular values of some 1e-13 of the operator's norm that carry no structure, and
// rounding at 1e-14 would keep them (D_x at 2^7 x 2^7: bond 20 instead of 8).
constexpr double OP_TOL = 1e-13;
constexpr int FCAP = 32;           // slot capacity of the fields (coordinates, metric terms)
constexpr int MAXW = 128;          // largest MPO bond handled (before rounding)
// A field derived by a cancelling sum counts as zero below this fraction of its
// operands' scale: the operands carry the 1e-14 truncations of the operations
// before them, so the noise such a sum leaves is some 1e-14 of that scale.
constexpr double ZERO_TOL = 1e-12;

// ---- kernels (one workgroup per site, setup only) ------------------------------

// m <- scale diag(x): M[a][o][r][b] = x[a][o][b] if o == r (copy tensor, Sec. 2.1.3),
// the scale applied to the first core only
__global__ void __launch_bounds__(256) k_diag_of(const double* x, const int32_t* xb, int cap, double scale,
                                                 double* m, int32_t* mb, int L) {
  const int k = blockIdx.x;
  const int a0 = xb[k], b0 = xb[k + 1];
  if (k != 0) scale = 1.0;
  const size_t sx = (size_t)cap * 2 * cap, sm = (size_t)cap * 4 * cap;
  for (int e = threadIdx.x; e < cap * 4 * cap; e += blockDim.x) {
    const int a = e / (4 * cap), s = (e / cap) % 4, b = e % cap;
    const int o = s >> 1, r = s & 1;
    m[k * sm + e] = (a < a0 && b < b0 && o == r) ? scale * x[k * sx + (size_t)a * 2 * cap + o * cap + b] : 0.0;
  }
  if (threadIdx.x == 0) {
    mb[k] = a0;
    if (k == L - 1) mb[L] = b0;
  }
}

// out <- diag(c) D: core ((a, p), (o, r), (b, q)) = C[a][o][b] D[p][o][r][q]
__global__ void __launch_bounds__(256) k_diag_times(const double* c, const int32_t* cb, int ccap, const double* d,
                                                    const int32_t* db, int dcap, double* out, int32_t* ob, int ocap,
                                                    int L) {
  const int k = blockIdx.x;
  const int ca = cb[k], cbb = cb[k + 1], da = db[k], dbb = db[k + 1];
  const size_t sc = (size_t)ccap * 2 * ccap, sd = (size_t)dcap * 4 * dcap, so = (size_t)ocap * 4 * ocap;
  for (int e = threadIdx.x; e < ocap * 4 * ocap; e += blockDim.x) {
    const int A = e / (4 * ocap), s = (e / ocap) % 4, B = e % ocap;
    double v = 0.0;
    if (A < ca * da && B < cbb * dbb) {
      const int a = A / da, p = A % da, b = B / dbb, q = B % dbb, o = s >> 1;
      v = c[k * sc + (size_t)a * 2 * ccap + o * ccap + b] * d[k * sd + (size_t)p * 4 * dcap + s * dcap + q];
    }
    out[k * so + e] = v;
  }
  if (threadIdx.x == 0) {
    ob[k] = ca * da;
    if (k == L - 1) ob[L] = cbb * dbb;
  }
}

// y = M x exactly (bonds multiply): core ((w1, a1), o, (w2, a2)) = sum_r M[w1][o][r][w2] x[a1][r][a2]
__global__ void __launch_bounds__(256) k_mpo_mps_exact(const double* m, const int32_t* mb, int wcap, const double* x,
                                                       const int32_t* xb, int xcap, double* y, int32_t* yb, int ycap,
                                                       int L) {
  const int k = blockIdx.x;
  const int w1 = mb[k], w2 = mb[k + 1], a1 = xb[k], a2 = xb[k + 1];
  const size_t sm = (size_t)wcap * 4 * wcap, sx = (size_t)xcap * 2 * xcap, sy = (size_t)ycap * 2 * ycap;
  for (int e = threadIdx.x; e < ycap * 2 * ycap; e += blockDim.x) {
    const int A = e / (2 * ycap), o = (e / ycap) % 2, B = e % ycap;
    double v = 0.0;
    if (A < w1 * a1 && B < w2 * a2) {
      const int p = A / a1, a = A % a1, q = B / a2, b = B % a2;
      for (int r = 0; r < 2; ++r)
        v += m[k * sm + (size_t)p * 4 * wcap + (o * 2 + r) * wcap + q] * x[k * sx + (size_t)a * 2 * xcap + r * xcap + b];
    }
    y[k * sy + e] = v;
  }
  if (threadIdx.x == 0) {
    yb[k] = w1 * a1;
    if (k == L - 1) yb[L] = w2 * a2;
  }
}

// An MPO as a train of 2L cores of dimension 2 (the row index o, then the column
// index r of each site): core 2k [a][o][(a, o)] is a copy of the bond, core 2k+1
// [(a, o)][r][b] = M[a][o][r][b]. The split is exact, so rounding the train rounds
// the MPO's bonds (the intermediate bonds are merged back afterwards).
__global__ void __launch_bounds__(256) k_mpo_split(const double* m, const int32_t* mb, int wcap, double* y,
                                                   int32_t* yb, int cap, int L) {
  const int k = blockIdx.x;
  const int w = mb[k], w2 = mb[k + 1];
  const size_t sl = (size_t)cap * 2 * cap, sm = (size_t)wcap * 4 * wcap;
  double* y0 = y + (size_t)(2 * k) * sl;
  double* y1 = y0 + sl;
  for (int e = threadIdx.x; e < cap * 2 * cap; e += blockDim.x) {
    const int a = e / (2 * cap), s = (e / cap) % 2, b = e % cap;
    y0[e] = (a < w && b == a * 2 + s) ? 1.0 : 0.0;
    y1[e] = (a < 2 * w && b < w2) ? m[k * sm + (size_t)(a / 2) * 4 * wcap + ((a % 2) * 2 + s) * wcap + b] : 0.0;
  }
  if (threadIdx.x == 0) {
    yb[2 * k] = w;
    yb[2 * k + 1] = 2 * w;
    if (k == L - 1) yb[2 * L] = w2;
  }
}

// Inverse of the split: M[a][o][r][b] = sum_t Y_2k[a][o][t] Y_2k+1[t][r][b]
__global__ void __launch_bounds__(256) k_mpo_merge(const double* y, const int32_t* yb, int cap, double* m,
                                                   int32_t* mb, int wcap, int L) {
  const int k = blockIdx.x;
  const int w = yb[2 * k], mm = yb[2 * k + 1], w2 = yb[2 * k + 2];
  const size_t sl = (size_t)cap * 2 * cap, sm = (size_t)wcap * 4 * wcap;
  const double* y0 = y + (size_t)(2 * k) * sl;
  const double* y1 = y0 + sl;
  for (int e = threadIdx.x; e < wcap * 4 * wcap; e += blockDim.x) {
    const int a = e / (4 * wcap), s = (e / wcap) % 4, b = e % wcap;
    const int o = s >> 1, r = s & 1;
    double v = 0.0;
    if (a < w && b < w2)
      for (int t = 0; t < mm; ++t) v += y0[(size_t)a * 2 * cap + o * cap + t] * y1[(size_t)t * 2 * cap + r * cap + b];
    m[k * sm + e] = v;
  }
  if (threadIdx.x == 0) {
    mb[k] = w;
    if (k == L - 1) mb[L] = w2;
  }
}

// ---- device trains ------------------------------------------------------------

struct DTT {           // MPS (d = 2) in slot layout
  int L = 0, cap = 0;
  double* data = nullptr;
  int32_t* bond = nullptr;
  qtt_mps desc() const { return qtt_mps{L, 2, cap, bond, data}; }
};

struct DMPO {          // MPO in slot layout, bonds on the device and the host
  int L = 0, wcap = 0;
  double* data = nullptr;
  int32_t* bond = nullptr;
  std::vector<int32_t> hb;
  qtt_mpo desc() const { return qtt_mpo{L, wcap, hb.data(), bond, data}; }
  int wmax() const { return *std::max_element(hb.begin(), hb.end()); }
};

#define TRY(expr)              \
  do {                         \
    const int rc_ = (expr);    \
    if (rc_ != QTT_OK) return rc_; \
  } while (0)

class Builder {
 public:
  Builder(qtt_ctx* ctx, const qtt_cylinder& cyl, hipStream_t s)
      : ctx_(ctx), s_(s), n_(cyl.n), L_(2 * cyl.n), N_(1 << cyl.n), order_(cyl.order), r_out_(cyl.r_out) {
    deta_ = 1.0 / (N_ + 1);
    dxi_ = 1.0 / N_;
  }
  ~Builder() {
    (void)hipStreamSynchronize(s_);
    for (void* p : allocs_) (void)hipFree(p);
  }

  int fail(int code, const char* what) { return set_error(ctx_, code, what); }

  // ---- allocation and transfers
  template <class T>
  int alloc(T** p, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return fail(QTT_EHIP, "build_tt: hipMalloc");
    allocs_.push_back(q);
    *p = static_cast<T*>(q);
    return QTT_OK;
  }
  int make(int cap, DTT& t, int L = 0) {
    t.L = L ? L : L_;
    t.cap = cap;
    TRY(alloc(&t.data, (size_t)t.L * cap * 2 * cap));
    TRY(alloc(&t.bond, (size_t)t.L + 1));
    return QTT_OK;
  }
  int make_mpo(const std::vector<int32_t>& hb, DMPO& m) {
    m.L = L_;
    m.hb = hb;
    m.wcap = m.wmax();
    if (m.wcap > MAXW) return fail(QTT_ECAPACITY, "build_tt: an intermediate MPO bond exceeds 128");
    TRY(alloc(&m.data, (size_t)L_ * m.wcap * 4 * m.wcap));
    TRY(alloc(&m.bond, (size_t)L_ + 1));
    if (hipMemcpyAsync(m.bond, hb.data(), hb.size() * sizeof(int32_t), hipMemcpyHostToDevice, s_) != hipSuccess)
      return fail(QTT_EHIP, "build_tt: bond upload");
    return sync();
  }
  int sync() { return hipStreamSynchronize(s_) == hipSuccess ? QTT_OK : fail(QTT_EHIP, "build_tt: stream"); }
  int launched() { return hipGetLastError() == hipSuccess ? QTT_OK : fail(QTT_EHIP, "build_tt: kernel launch"); }
  int bonds(const DTT& t, std::vector<int32_t>& hb) {
    hb.assign(t.L + 1, 0);
    if (hipMemcpyAsync(hb.data(), t.bond, hb.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s_) != hipSuccess)
      return fail(QTT_EHIP, "build_tt: bond read");
    return sync();
  }
  int upload(const HostTT& T, int cap, DTT& t) {
    for (int b : T.bl)
      if (b > cap) return fail(QTT_ECAPACITY, "build_tt: a boundary train exceeds the field capacity");
    TRY(make(cap, t, T.L));
    std::vector<double> slots((size_t)T.L * cap * 2 * cap, 0.0);
    for (int k = 0; k < T.L; ++k)
      for (int a = 0; a < T.bl[k]; ++a)
        for (int q = 0; q < 2; ++q)
          for (int b = 0; b < T.bl[k + 1]; ++b)
            slots[(size_t)k * cap * 2 * cap + (size_t)a * 2 * cap + q * cap + b] =
                T.cores[k][((size_t)a * 2 + q) * T.bl[k + 1] + b];
    std::vector<int32_t> hb(T.bl.begin(), T.bl.end());
    if (hipMemcpyAsync(t.data, slots.data(), slots.size() * sizeof(double), hipMemcpyHostToDevice, s_) != hipSuccess ||
        hipMemcpyAsync(t.bond, hb.data(), hb.size() * sizeof(int32_t), hipMemcpyHostToDevice, s_) != hipSuccess)
      return fail(QTT_EHIP, "build_tt: upload");
    return sync();   // the host buffers are released on return
  }
  int upload_mpo(const HostTT& T, DMPO& m) {
    std::vector<int32_t> hb(T.bl.begin(), T.bl.end());
    TRY(make_mpo(hb, m));
    const int w = m.wcap;
    std::vector<double> slots((size_t)T.L * w * 4 * w, 0.0);
    for (int k = 0; k < T.L; ++k)
      for (int a = 0; a < T.bl[k]; ++a)
        for (int q = 0; q < 4; ++q)
          for (int b = 0; b < T.bl[k + 1]; ++b)
            slots[(size_t)k * w * 4 * w + (size_t)a * 4 * w + q * w + b] = T.cores[k][((size_t)a * 4 + q) * T.bl[k + 1] + b];
    if (hipMemcpyAsync(m.data, slots.data(), slots.size() * sizeof(double), hipMemcpyHostToDevice, s_) != hipSuccess)
      return fail(QTT_EHIP, "build_tt: upload");
    return sync();
  }

  // ---- TT operations on the device (the library's own entry points and kernels)
  int diag_of(const DTT& x, double scale, DMPO& m) {
    std::vector<int32_t> hb;
    TRY(bonds(x, hb));
    m.L = L_;
    m.hb = hb;
    m.wcap = x.cap;
    TRY(alloc(&m.data, (size_t)L_ * x.cap * 4 * x.cap));
    TRY(alloc(&m.bond, (size_t)L_ + 1));
    hipLaunchKernelGGL(k_diag_of, dim3(L_), dim3(256), 0, s_, x.data, x.bond, x.cap, scale, m.data, m.bond, L_);
    return launched();
  }
  // y = M x: the exact product (bonds multiply), rounded by QR and one-sided Jacobi SVD
  // sweeps (accurate down to the smallest singular values it keeps), into a field of
  // capacity FCAP; tol < 0 leaves the product unrounded but for the cap
  int apply_tol(const DMPO& M, const DTT& x, DTT& y, double tol) {
    std::vector<int32_t> xb;
    TRY(bonds(x, xb));
    int cap = 1;
    for (int k = 0; k <= L_; ++k) cap = std::max(cap, (int)(M.hb[k] * xb[k]));
    if (cap > 512) return fail(QTT_ECAPACITY, "build_tt: an exact product exceeds capacity 512");
    DTT big;
    TRY(make(cap, big));
    hipLaunchKernelGGL(k_mpo_mps_exact, dim3(L_), dim3(256), 0, s_, M.data, M.bond, M.wcap, x.data, x.bond, x.cap,
                       big.data, big.bond, cap, L_);
    TRY(launched());
    qtt_mps bd = big.desc();
    const qtt_trunc tr{std::max(tol, 0.0), FCAP, 0};
    TRY(qtt_round(ctx_, 1, &bd, &tr, s_));
    return copy_into(big, y);
  }
  int apply(const DMPO& M, const DTT& x, DTT& y) { return apply_tol(M, x, y, bond_tol(L_)); }
  // y (capacity FCAP) <- x (bonds <= FCAP)
  int copy_into(const DTT& x, DTT& y) {
    std::vector<int32_t> hb;
    TRY(bonds(x, hb));
    TRY(make(FCAP, y));
    if (hipMemsetAsync(y.data, 0, sizeof(double) * (size_t)L_ * FCAP * 2 * FCAP, s_) != hipSuccess)
      return fail(QTT_EHIP, "build_tt: clear");
    for (int k = 0; k < L_; ++k) {
      if (hb[k] > FCAP || hb[k + 1] > FCAP) return fail(QTT_ECAPACITY, "build_tt: a field exceeds capacity 32");
      for (int q = 0; q < 2; ++q)
        if (hipMemcpy2DAsync(y.data + (size_t)k * FCAP * 2 * FCAP + (size_t)q * FCAP, sizeof(double) * 2 * FCAP,
                             x.data + (size_t)k * x.cap * 2 * x.cap + (size_t)q * x.cap, sizeof(double) * 2 * x.cap,
                             sizeof(double) * hb[k + 1], hb[k], hipMemcpyDeviceToDevice, s_) != hipSuccess)
          return fail(QTT_EHIP, "build_tt: copy");
    }
    if (hipMemcpyAsync(y.bond, hb.data(), sizeof(int32_t) * (L_ + 1), hipMemcpyHostToDevice, s_) != hipSuccess)
      return fail(QTT_EHIP, "build_tt: bonds");
    return sync();
  }
  int hadamard(const DTT& a, const DTT& b, DTT& y) {   // Sec. 2.1.3: diag(a) applied to b
    DMPO A;
    TRY(diag_of(a, 1.0, A));
    return apply(A, b, y);
  }
  int lin(double a, const DTT& x, double b, const DTT& y, DTT& z) {   // Sec. 2.1.1 with rounding
    TRY(make(FCAP, z));
    const qtt_mps xd = x.desc(), yd = y.desc();
    qtt_mps zd = z.desc();
    const qtt_trunc tr{bond_tol(L_), FCAP, 0};
    return qtt_add(ctx_, 1, &a, &xd, &b, &yd, &zd, &tr, s_);
  }
  int diag_times(const DTT& c, const DMPO& D, DMPO& out) {
    std::vector<int32_t> cb, hb(L_ + 1);
    TRY(bonds(c, cb));
    for (int k = 0; k <= L_; ++k) hb[k] = cb[k] * D.hb[k];
    TRY(make_mpo(hb, out));
    hipLaunchKernelGGL(k_diag_times, dim3(L_), dim3(256), 0, s_, c.data, c.bond, c.cap, D.data, D.bond, D.wcap,
                       out.data, out.bond, out.wcap, L_);
    return launched();
  }
  int split(const DMPO& M, int cap, DTT& t) {
    TRY(make(cap, t, 2 * L_));
    hipLaunchKernelGGL(k_mpo_split, dim3(L_), dim3(256), 0, s_, M.data, M.bond, M.wcap, t.data, t.bond, cap, L_);
    return launched();
  }
  int merge(const DTT& t, DMPO& M) {
    std::vector<int32_t> tb, hb(L_ + 1);
    TRY(bonds(t, tb));
    for (int k = 0; k <= L_; ++k) hb[k] = tb[2 * k];
    TRY(make_mpo(hb, M));
    hipLaunchKernelGGL(k_mpo_merge, dim3(L_), dim3(256), 0, s_, t.data, t.bond, t.cap, M.data, M.bond, M.wcap, L_);
    return launched();
  }
  // a A + b B, rounded (the direct sum and rounding of the split trains)
  int mpo_lin(double a, const DMPO& A, double b, const DMPO& B, DMPO& out) {
    const int ca = 2 * A.wmax(), cb = 2 * B.wmax();
    DTT sa, sb, sz;
    TRY(split(A, ca, sa));
    TRY(split(B, cb, sb));
    TRY(make(ca + cb, sz, 2 * L_));
    const qtt_mps ad = sa.desc(), bd = sb.desc();
    qtt_mps zd = sz.desc();
    const qtt_trunc tr{bond_tol(2 * L_, OP_TOL), ca + cb, 0};
    TRY(qtt_add(ctx_, 1, &a, &ad, &b, &bd, &zd, &tr, s_));
    return merge(sz, out);
  }
  int mpo_round(const DMPO& A, DMPO& out) {
    DTT t;
    TRY(split(A, 2 * A.wmax(), t));
    qtt_mps td = t.desc();
    const qtt_trunc tr{bond_tol(2 * L_, OP_TOL), t.cap, 0};
    TRY(qtt_round(ctx_, 1, &td, &tr, s_));
    return merge(t, out);
  }
  // a = 1 / j for a field of one sign (Sec. 3.2.3: the LSE diag(j) a = 1, solved by
  // ALS); sgn = -1 when j < 0, so that the operator diag(sgn j) is positive definite.
  // The ALS solution is then polished by Newton steps a <- a + a (1 - j a) in TT
  // arithmetic (the error 1 - j a squares at each step): eight steps at most, fewer if
  // ||1 - j a|| / ||1|| reaches 2e-14; the floor of the truncated arithmetic is some
  // 1e-13 (accepted up to 1e-12).
  int inverse(const DTT& j, double sgn, DTT& a) {
    DMPO Jm;
    TRY(diag_of(j, sgn, Jm));
    DTT b, one, x;
    TRY(upload(outer(ones(), ones(), sgn), FCAP, b));
    TRY(upload(outer(ones(), ones()), FCAP, one));
    TRY(upload(seed_train(4), FCAP, x));
    const qtt_mpo md = Jm.desc();
    const qtt_mps bd = b.desc();
    qtt_mps xd = x.desc();
    qtt_solve_opts o{1e-11, 40, 400, 1e-14, QTT_F64};
    qtt_solve_info info{};
    const int rc = qtt_poisson_solve(ctx_, 1, &md, &bd, &xd, &o, &info, s_);
    if (rc != QTT_OK && rc != QTT_ENOTCONVERGED) return rc;
    double n1 = 0.0, res = INFINITY;
    TRY(norm(one, &n1));
    for (int it = 0;; ++it) {
      DTT p, r, c, x1;
      TRY(hadamard(j, x, p));
      TRY(lin(1.0, one, -1.0, p, r));
      TRY(norm(r, &res));
      res /= n1;
      if (res <= 2e-14 || it == 8) break;
      TRY(hadamard(x, r, c));
      TRY(lin(1.0, x, 1.0, c, x1));
      x = x1;
    }
    if (!(res <= 1e-12)) {
      char msg[160];
      snprintf(msg, sizeof(msg), "build_tt: the inverse Jacobian stalls at ||1 - J a|| / ||1|| = %.2e (ALS %.2e)", res,
               info.residual);
      return fail(QTT_ENOTCONVERGED, msg);
    }
    a = x;
    return QTT_OK;
  }

  // ---- host construction of the small 1D / boundary pieces
  HostTT ones() const {               // 1 on n cores
    HostTT T;
    T.L = n_; T.d = 2;
    for (int k = 0; k < n_; ++k) { T.cores.push_back({1.0, 1.0}); T.bl.push_back(1); }
    T.bl.push_back(1);
    return T;
  }
  HostTT unit(int i) const {          // e_i on n cores (MSB first)
    HostTT T;
    T.L = n_; T.d = 2;
    for (int k = 0; k < n_; ++k) {
      const int bit = (i >> (n_ - 1 - k)) & 1;
      T.cores.push_back({bit ? 0.0 : 1.0, bit ? 1.0 : 0.0});
      T.bl.push_back(1);
    }
    T.bl.push_back(1);
    return T;
  }
  HostTT encode(const std::vector<double>& v) const {   // a 1D vector of 2^n values by TT-SVD
    double s2 = 0.0;
    for (double x : v) s2 += x * x;
    return tt_svd_host(v, n_, 2, 0.0, 1 << 30, TT_TOL * std::max(std::sqrt(s2), 1e-300));
  }
  // exponential wall-normal spacing s_i = Q (e^{kappa (i+1) deta} - 1) / (e^kappa - 1)
  // (Sec. 3.2.2), with Q = r_out - 1/2 and e^kappa = 2 r_out (App. E): the
  // exponential is a product of one factor per bit (rank 1), minus a constant.
  HostTT spacing() const {
    const double Q = r_out_ - 0.5, ek = 2.0 * r_out_, kap = std::log(ek), A = Q / (ek - 1.0);
    HostTT E, C = ones();
    E.L = n_; E.d = 2;
    for (int k = 0; k < n_; ++k) {
      const double f = std::exp(kap * deta_ * std::ldexp(1.0, n_ - 1 - k));
      const double pre = (k == 0) ? A * std::exp(kap * deta_) : 1.0;
      E.cores.push_back({pre, pre * f});
      E.bl.push_back(1);
    }
    E.bl.push_back(1);
    C.cores[0][0] = C.cores[0][1] = -A;
    HostTT S = tt_direct_sum(E, C);
    tt_round_host(S, TT_TOL);
    return S;
  }
  // eta-train (x) xi-train in the grid's bit order: "concatenation" of Sec. 3.2.2,
  // with the cores interleaved for the interleaved order (exact, bonds multiply).
  HostTT outer(const HostTT& eta, const HostTT& xi, double scale = 1.0) const {
    HostTT T;
    T.L = L_; T.d = 2;
    if (order_ == QTT_ORDER_CONCATENATED) {
      for (int k = 0; k < n_; ++k) { T.cores.push_back(eta.cores[k]); T.bl.push_back(eta.bl[k]); }
      for (int k = 0; k < n_; ++k) { T.cores.push_back(xi.cores[k]); T.bl.push_back(xi.bl[k]); }
      T.bl.push_back(1);
    } else {
      for (int k = 0; k < n_; ++k) {
        const int ea = eta.bl[k], eb = eta.bl[k + 1], xa = xi.bl[k], xb = xi.bl[k + 1];
        std::vector<double> c1((size_t)ea * xa * 2 * eb * xa, 0.0), c2((size_t)eb * xa * 2 * eb * xb, 0.0);
        for (int a = 0; a < ea; ++a)          // eta digit: (a, p) -> (a', p)
          for (int p = 0; p < xa; ++p)
            for (int q = 0; q < 2; ++q)
              for (int b = 0; b < eb; ++b)
                c1[(((size_t)a * xa + p) * 2 + q) * eb * xa + (size_t)b * xa + p] = eta.cores[k][((size_t)a * 2 + q) * eb + b];
        for (int a = 0; a < eb; ++a)          // xi digit: (a, p) -> (a, p')
          for (int p = 0; p < xa; ++p)
            for (int q = 0; q < 2; ++q)
              for (int b = 0; b < xb; ++b)
                c2[(((size_t)a * xa + p) * 2 + q) * eb * xb + (size_t)a * xb + b] = xi.cores[k][((size_t)p * 2 + q) * xb + b];
        T.cores.push_back(c1); T.bl.push_back(ea * xa);
        T.cores.push_back(c2); T.bl.push_back(eb * xa);
      }
      T.bl.push_back(1);
    }
    for (double& v : T.cores[0]) v *= scale;
    return T;
  }
  HostTT sum(HostTT A, const HostTT& B) const {
    HostTT S = tt_direct_sum(A, B);
    tt_round_host(S, TT_TOL);
    return S;
  }
  HostTT seed_train(int chi) const {   // a fixed positive start of the ALS solve
    HostTT T;
    T.L = L_; T.d = 2;
    unsigned long long h = 0x9e3779b97f4a7c15ull;
    T.bl.push_back(1);
    for (int k = 0; k < L_; ++k) {
      const int a = T.bl[k];
      const int b = (k == L_ - 1) ? 1 : std::min({chi, 1 << std::min(k + 1, 30), 1 << std::min(L_ - k - 1, 30)});
      std::vector<double> c((size_t)a * 2 * b);
      for (auto& v : c) {
        h ^= h >> 33; h *= 0xff51afd7ed558ccdull; h ^= h >> 33;
        v = ((double)(h >> 11) / 9007199254740992.0) * 0.1 + (&v == &c[0] ? 1.0 : 0.0);
      }
      T.cores.push_back(c);
      T.bl.push_back(b);
    }
    return T;
  }
  // computational derivatives as TT-matrices: sums of scaled shift automata, rounded
  HostTT stencil(std::initializer_list<std::pair<std::pair<int, int>, double>> terms) const {
    HostTT acc;
    bool have = false;
    for (const auto& t : terms) {
      HostTT S = cyl_shift_mpo(n_, t.first.first, t.first.second, order_);
      for (double& v : S.cores[0]) v *= t.second;
      acc = have ? tt_direct_sum(acc, S) : S;
      have = true;
    }
    tt_round_host(acc, TT_TOL);
    return acc;
  }

  // ---- fields with a truncation threshold relative to their operands' scale: a sum
  // that cancels (g12 and the metric derivatives of an orthogonal grid) becomes an
  // exact zero instead of high-rank rounding noise
  struct Field {
    DTT t;
    bool zero = false;
  };
  int norm(const DTT& x, double* out) {
    const qtt_mps xd = x.desc();
    double d = 0.0;
    TRY(qtt_dot(ctx_, 1, &xd, &xd, &d, s_));
    *out = std::sqrt(std::max(d, 0.0));
    return QTT_OK;
  }
  // z <- z rounded with threshold TT_TOL * scale, or zero below it
  int settle(Field& z, double scale) {
    double nz = 0.0;
    TRY(norm(z.t, &nz));
    if (!(nz > ZERO_TOL * scale)) {
      z.zero = true;
      return QTT_OK;
    }
    qtt_mps zd = z.t.desc();
    const qtt_trunc tr{bond_tol(L_) * scale / nz, FCAP, 0};
    return qtt_round(ctx_, 1, &zd, &tr, s_);
  }
  // (the helpers below overwrite their output Field entirely, zero flag included)
  int lin_f(double a, const Field& x, double b, const Field& y, Field& z) {
    z = Field{};
    if (x.zero && y.zero) { z.zero = true; return QTT_OK; }
    double nx = 0.0, ny = 0.0;
    if (!x.zero) TRY(norm(x.t, &nx));
    if (!y.zero) TRY(norm(y.t, &ny));
    TRY(make(FCAP, z.t));
    const qtt_mps xd = (x.zero ? y : x).t.desc(), yd = (y.zero ? x : y).t.desc();
    const double aa = x.zero ? 0.0 : a, bb = y.zero ? 0.0 : b;
    qtt_mps zd = z.t.desc();
    const qtt_trunc tr{0.0, FCAP, 0};
    TRY(qtt_add(ctx_, 1, &aa, &xd, &bb, &yd, &zd, &tr, s_));
    return settle(z, std::max(std::fabs(a) * nx, std::fabs(b) * ny));
  }
  int had_f(const Field& a, const Field& b, Field& y) {
    y = Field{};
    if (a.zero || b.zero) { y.zero = true; return QTT_OK; }
    return hadamard(a.t, b.t, y.t);
  }
  // y = D x with D a computational derivative of norm <= dnorm
  int apply_f(const DMPO& D, double dnorm, const Field& x, Field& y) {
    y = Field{};
    if (x.zero) { y.zero = true; return QTT_OK; }
    double nx = 0.0;
    TRY(norm(x.t, &nx));
    TRY(apply_tol(D, x.t, y.t, 0.0));
    return settle(y, dnorm * nx);
  }
  // out += coef * diag(c) D (out empty: out = coef * diag(c) D)
  int accumulate(DMPO& out, bool& have, double coef, const Field& c, const DMPO& D) {
    if (c.zero) return QTT_OK;
    DMPO T;
    TRY(diag_times(c.t, D, T));
    if (!have) {
      have = true;
      DMPO U;
      TRY(mpo_lin(coef, T, 0.0, T, U));
      out = U;
      return QTT_OK;
    }
    DMPO U;
    TRY(mpo_lin(1.0, out, coef, T, U));
    out = U;
    return QTT_OK;
  }
  int accumulate_diag(DMPO& out, double coef, const Field& c) {
    if (c.zero) return QTT_OK;
    DMPO F, U;
    TRY(diag_of(c.t, 1.0, F));
    TRY(mpo_lin(1.0, out, coef, F, U));
    out = U;
    return QTT_OK;
  }

  // ---- the construction
  int run(int which, DMPO* mpo_out, DTT* vec_out) {
    const double he = deta_, hx = dxi_;
    // Sec. 3.2.2: 1D boundary curves and unit normals along xi, spacing and ones along eta
    std::vector<double> xg(N_), zg(N_), nx(N_), nz(N_), xf(N_), zf(N_);
    for (int j = 0; j < N_; ++j) {
      const double th = 2.0 * M_PI * j * hx;
      nx[j] = std::cos(th); nz[j] = std::sin(th);
      xg[j] = 0.5 * nx[j]; zg[j] = 0.5 * nz[j];   // the wall (unit cylinder)
      xf[j] = r_out_ * nx[j]; zf[j] = r_out_ * nz[j];   // the far-field row
    }
    const HostTT one = ones(), s = spacing();
    const HostTT Xg = encode(xg), Zg = encode(zg), Nx = encode(nx), Nz = encode(nz);
    DTT a1, a2, x, z;
    TRY(upload(outer(one, Xg), FCAP, a1));
    TRY(upload(outer(s, Nx), FCAP, a2));
    TRY(lin(1.0, a1, 1.0, a2, x));            // x = 1 u x_G + s u n_x
    TRY(upload(outer(one, Zg), FCAP, a1));
    TRY(upload(outer(s, Nz), FCAP, a2));
    TRY(lin(1.0, a1, 1.0, a2, z));            // z = 1 u z_G + s u n_z
    if (which == QTT_VEC_MESH_X || which == QTT_VEC_MESH_Z) {
      *vec_out = which == QTT_VEC_MESH_X ? x : z;
      return QTT_OK;
    }
    // computational derivatives (App. A, second-order central; zero outside the rows)
    DMPO Dxi, Deta;
    TRY(upload_mpo(stencil({{{0, 1}, 0.5 / hx}, {{0, -1}, -0.5 / hx}}), Dxi));
    TRY(upload_mpo(stencil({{{1, 0}, 0.5 / he}, {{-1, 0}, -0.5 / he}}), Deta));
    // ghost rows of the coordinates: the wall (row -1) and the far field (row N)
    const HostTT e0 = unit(0), eN = unit(N_ - 1);
    DTT gx, gz;
    TRY(upload(sum(outer(e0, Xg, -0.5 / he), outer(eN, encode(xf), 0.5 / he)), FCAP, gx));
    TRY(upload(sum(outer(e0, Zg, -0.5 / he), outer(eN, encode(zf), 0.5 / he)), FCAP, gz));
    // metric terms
    DTT x_xi, z_xi, x_eta, z_eta, t;
    TRY(apply(Dxi, x, x_xi));
    TRY(apply(Dxi, z, z_xi));
    TRY(apply(Deta, x, t));
    TRY(lin(1.0, t, 1.0, gx, x_eta));
    TRY(apply(Deta, z, t));
    TRY(lin(1.0, t, 1.0, gz, z_eta));
    // Jacobian determinant (Sec. 3.2.3) and its inverse by ALS
    DTT p1, p2, j;
    TRY(hadamard(x_xi, z_eta, p1));
    TRY(hadamard(x_eta, z_xi, p2));
    TRY(lin(1.0, p1, -1.0, p2, j));
    if (which == QTT_VEC_JAC) {
      *vec_out = j;
      return QTT_OK;
    }
    // the O-grid runs counter-clockwise in xi and outwards in eta, so J < 0 everywhere
    DTT ji;
    TRY(inverse(j, -1.0, ji));
    DTT row0;
    TRY(upload(outer(e0, one), FCAP, row0));
    if (which == QTT_OP_LAP || which == QTT_OP_P) {
      DMPO lap;
      TRY(laplacian(Dxi, Deta, x_xi, z_xi, x_eta, z_eta, ji, row0, which == QTT_OP_P, lap));
      if (which == QTT_OP_LAP) {
        *mpo_out = lap;
        return QTT_OK;
      }
      DMPO W;      // P = -|J| Lap_p = J Lap_p
      TRY(diag_times(j, lap, W));
      return mpo_round(W, *mpo_out);
    }
    DTT c1, c2;
    DMPO A, B, D;
    const bool dx = which == QTT_OP_DX || which == QTT_OP_DXP || which == QTT_OP_WX;
    const bool dz = which == QTT_OP_DZ || which == QTT_OP_DZP || which == QTT_OP_WZ;
    if (!dx && !dz) return fail(QTT_EINVAL, "build_tt: object not built in TT format");
    if (dx) {   // D_x = C1 D_xi - C2 D_eta, c1 = z_eta / J, c2 = z_xi / J
      TRY(hadamard(z_eta, ji, c1));
      TRY(hadamard(z_xi, ji, c2));
      TRY(diag_times(c1, Dxi, A));
      TRY(diag_times(c2, Deta, B));
      TRY(mpo_lin(1.0, A, -1.0, B, D));
    } else {    // D_z = -C1 D_xi + C2 D_eta, c1 = x_eta / J, c2 = x_xi / J
      TRY(hadamard(x_eta, ji, c1));
      TRY(hadamard(x_xi, ji, c2));
      TRY(diag_times(c1, Dxi, A));
      TRY(diag_times(c2, Deta, B));
      TRY(mpo_lin(-1.0, A, 1.0, B, D));
    }
    if (which == QTT_OP_DX || which == QTT_OP_DZ) {
      *mpo_out = D;
      return QTT_OK;
    }
    if (which == QTT_OP_WX || which == QTT_OP_WZ) {   // -|J| D = J D
      DMPO W;
      TRY(diag_times(j, D, W));
      return mpo_round(W, *mpo_out);
    }
    // pressure gradient: p_{-1} = p_0 folds the wall-row neighbour (coefficient of
    // u(i-1, j) on row 0: +c2 / (2 deta) for D_x, -c2 / (2 deta) for D_z) into the centre
    DTT f;
    TRY(hadamard(row0, c2, f));
    DMPO F;
    TRY(diag_of(f, 1.0, F));
    return mpo_lin(1.0, D, (dx ? 0.5 : -0.5) / he, F, *mpo_out);
  }

  // The seven-term Laplacian of App. A in TT format:
  //   Lap = A_xi D_xi + A_xixi D_xixi + A_eta D_eta + A_xieta D_xieta + A_etaeta D_etaeta,
  //   A_xi = (d_xi a22 - d_eta a12) / J, A_eta = (d_eta a11 - d_xi a12) / J,
  //   A_xixi = a22 / J, A_etaeta = a11 / J, A_xieta = -2 a12 / J,  a_kl = g_kl / J,
  // with the metric tensor g from Hadamard products of the metric terms. The eta
  // differences of a11, a12 reach the wall and far-field rows, whose values enter as
  // boundary vectors (from the 1D boundary curves, the rows next to them and the
  // spacing). fold: the pressure form (p_{-1} = p_0), whose row-0 stencil takes the
  // wall-row neighbours: + (A_etaeta / deta^2 - A_eta / (2 deta)) at the centre and
  // - A_xieta D_xi / (2 deta) from the mixed term.
  int laplacian(const DMPO& Dxi, const DMPO& Deta, const DTT& x_xi, const DTT& z_xi, const DTT& x_eta,
                const DTT& z_eta, const DTT& ji, const DTT& row0, bool fold, DMPO& out) {
    const double he = deta_, hx = dxi_;
    auto F = [](const DTT& t) { Field f; f.t = t; return f; };
    const Field Xx = F(x_xi), Zx = F(z_xi), Xe = F(x_eta), Ze = F(z_eta), Ji = F(ji);
    Field q1, q2, g11, g22, g12, a11, a22, a12;
    TRY(had_f(Xx, Xx, q1)); TRY(had_f(Zx, Zx, q2)); TRY(lin_f(1.0, q1, 1.0, q2, g11));
    TRY(had_f(Xe, Xe, q1)); TRY(had_f(Ze, Ze, q2)); TRY(lin_f(1.0, q1, 1.0, q2, g22));
    TRY(had_f(Xx, Xe, q1)); TRY(had_f(Zx, Ze, q2)); TRY(lin_f(1.0, q1, 1.0, q2, g12));
    TRY(had_f(g11, Ji, a11)); TRY(had_f(g22, Ji, a22)); TRY(had_f(g12, Ji, a12));
    // a11, a12 on the wall row (-1) and the far-field row (N), from the mesh formula
    // on rows -2 .. 0 and N-1 .. N+1
    const double Q = r_out_ - 0.5, ek = 2.0 * r_out_, kap = std::log(ek);
    auto sp = [&](int i) { return Q * (std::exp(kap * (i + 1) * he) - 1.0) / (ek - 1.0); };
    std::vector<double> w11(N_), w12(N_), f11(N_), f12(N_);
    for (int side = 0; side < 2; ++side) {
      const int i = side ? N_ : -1;
      for (int jj = 0; jj < N_; ++jj) {
        const double th = 2.0 * M_PI * jj * hx, thp = th + 2.0 * M_PI * hx, thm = th - 2.0 * M_PI * hx;
        const double r = 0.5 + sp(i), re = (sp(i + 1) - sp(i - 1)) / (2.0 * he);
        const double xx = r * (std::cos(thp) - std::cos(thm)) / (2.0 * hx), zx = r * (std::sin(thp) - std::sin(thm)) / (2.0 * hx);
        const double xe = re * std::cos(th), ze = re * std::sin(th);
        const double J = xx * ze - xe * zx;
        (side ? f11 : w11)[jj] = (xx * xx + zx * zx) / J;
        (side ? f12 : w12)[jj] = (xx * xe + zx * ze) / J;
      }
    }
    auto ghost = [&](const std::vector<double>& wall, const std::vector<double>& far, Field& g) -> int {
      g = Field{};
      double s2 = 0.0;
      for (int jj = 0; jj < N_; ++jj) s2 += wall[jj] * wall[jj] + far[jj] * far[jj];
      if (!(std::sqrt(s2) > 0.0)) { g.zero = true; return QTT_OK; }
      HostTT w = encode(wall), f = encode(far);
      return upload(sum(outer(unit(0), w, -0.5 / he), outer(unit(N_ - 1), f, 0.5 / he)), FCAP, g.t);
    };
    Field g_a11, g_a12;
    TRY(ghost(w11, f11, g_a11));
    // g12 of the boundary rows is a cancelling sum as well: drop it at the same threshold
    {
      double m12 = 0.0, m11 = 0.0;
      for (int jj = 0; jj < N_; ++jj) {
        m12 = std::max({m12, std::fabs(w12[jj]), std::fabs(f12[jj])});
        m11 = std::max({m11, std::fabs(w11[jj]), std::fabs(f11[jj])});
      }
      if (m12 <= ZERO_TOL * m11) g_a12.zero = true;
      else TRY(ghost(w12, f12, g_a12));
    }
    Field dxi_a22, deta_a12, deta_a11, dxi_a12, t1, t2, cxi, ceta, cxx, cee, cxe;
    TRY(apply_f(Dxi, 1.0 / hx, a22, dxi_a22));
    TRY(apply_f(Deta, 1.0 / he, a12, t1));
    TRY(lin_f(1.0, t1, 1.0, g_a12, deta_a12));
    TRY(apply_f(Deta, 1.0 / he, a11, t1));
    TRY(lin_f(1.0, t1, 1.0, g_a11, deta_a11));
    TRY(apply_f(Dxi, 1.0 / hx, a12, dxi_a12));
    TRY(lin_f(1.0, dxi_a22, -1.0, deta_a12, t1)); TRY(had_f(t1, Ji, cxi));
    TRY(lin_f(1.0, deta_a11, -1.0, dxi_a12, t2)); TRY(had_f(t2, Ji, ceta));
    TRY(had_f(a22, Ji, cxx));
    TRY(had_f(a11, Ji, cee));
    TRY(had_f(a12, Ji, cxe));
    DMPO Dxx, Dee, Dxe;
    TRY(upload_mpo(stencil({{{0, 1}, 1.0 / (hx * hx)}, {{0, 0}, -2.0 / (hx * hx)}, {{0, -1}, 1.0 / (hx * hx)}}), Dxx));
    TRY(upload_mpo(stencil({{{1, 0}, 1.0 / (he * he)}, {{0, 0}, -2.0 / (he * he)}, {{-1, 0}, 1.0 / (he * he)}}), Dee));
    const double w = 1.0 / (4.0 * hx * he);
    TRY(upload_mpo(stencil({{{1, 1}, w}, {{1, -1}, -w}, {{-1, 1}, -w}, {{-1, -1}, w}}), Dxe));
    bool have = false;
    TRY(accumulate(out, have, 1.0, cxx, Dxx));
    TRY(accumulate(out, have, 1.0, cee, Dee));
    TRY(accumulate(out, have, 1.0, cxi, Dxi));
    TRY(accumulate(out, have, 1.0, ceta, Deta));
    TRY(accumulate(out, have, -2.0, cxe, Dxe));
    if (!have) return fail(QTT_ENUMERIC, "build_tt: the Laplacian has no nonzero coefficient");
    if (!fold) return QTT_OK;
    const Field R0 = F(row0);
    Field c0, u1, u2;
    TRY(lin_f(1.0 / (he * he), cee, -0.5 / he, ceta, u1));
    TRY(had_f(R0, u1, c0));
    TRY(accumulate_diag(out, 1.0, c0));
    TRY(had_f(R0, cxe, u2));
    return accumulate(out, have, 2.0 * 0.5 / he, u2, Dxi);   // -(-2 a12 / J) D_xi / (2 deta)
  }

 private:
  qtt_ctx* ctx_;
  hipStream_t s_;
  int n_, L_, N_, order_;
  double r_out_, deta_, dxi_;
  std::vector<void*> allocs_;
};

}  // namespace

extern "C" int qtt_build_tt(qtt_ctx* ctx, const qtt_cylinder* cyl, int which, int32_t cap, double* out,
                            int32_t* bond_out, int32_t* bond_host, int32_t* need, void* stream) {
  if (!ctx) return QTT_EINVAL;
  if (!cyl || cyl->n < 2 || cyl->n > 13 || !(cyl->r_out > 0.5))
    return set_error(ctx, QTT_EINVAL, "build_tt: bad cylinder");
  if (cyl->order != QTT_ORDER_INTERLEAVED && cyl->order != QTT_ORDER_CONCATENATED)
    return set_error(ctx, QTT_EINVAL, "build_tt: bad bit order");
  if (out && (!bond_out || !bond_host)) return set_error(ctx, QTT_EINVAL, "build_tt: null bonds");
  const bool vec = which == QTT_VEC_MESH_X || which == QTT_VEC_MESH_Z || which == QTT_VEC_JAC;
  if (!vec && which != QTT_OP_DX && which != QTT_OP_DZ && which != QTT_OP_DXP && which != QTT_OP_DZP &&
      which != QTT_OP_WX && which != QTT_OP_WZ && which != QTT_OP_LAP && which != QTT_OP_P)
    return set_error(ctx, QTT_EINVAL, "build_tt: object not built in TT format");
  if (hipSetDevice(qtt_solver_detail::device_of(ctx)) != hipSuccess) return set_error(ctx, QTT_EHIP, "build_tt: hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  Builder B(ctx, *cyl, s);
  DMPO M;
  DTT V;
  int rc = B.run(which, &M, &V);
  if (rc) return rc;
  const int L = 2 * cyl->n;
  std::vector<int32_t> hb;
  if (vec) {
    if ((rc = B.bonds(V, hb))) return rc;
  } else {
    hb = M.hb;
  }
  const int32_t w = *std::max_element(hb.begin(), hb.end());
  if (need) *need = w;
  if (!out) return QTT_OK;
  if (w > cap) return set_error(ctx, QTT_ECAPACITY, "build_tt: the object needs a larger slot capacity");
  const int d = vec ? 2 : 4;
  const int src_cap = vec ? V.cap : M.wcap;
  const double* src = vec ? V.data : M.data;
  // copy the slots into the caller's capacity (2D copy: one row of d * cap' per bond index)
  if (hipMemsetAsync(out, 0, sizeof(double) * (size_t)L * cap * d * cap, s) != hipSuccess)
    return set_error(ctx, QTT_EHIP, "build_tt: clear");
  for (int k = 0; k < L; ++k)
    for (int q = 0; q < d; ++q)
      if (hipMemcpy2DAsync(out + (size_t)k * cap * d * cap + (size_t)q * cap, sizeof(double) * d * cap,
                           src + (size_t)k * src_cap * d * src_cap + (size_t)q * src_cap, sizeof(double) * d * src_cap,
                           sizeof(double) * hb[k + 1], hb[k], hipMemcpyDeviceToDevice, s) != hipSuccess)
        return set_error(ctx, QTT_EHIP, "build_tt: copy");
  if (hipMemcpyAsync(bond_out, hb.data(), sizeof(int32_t) * (L + 1), hipMemcpyHostToDevice, s) != hipSuccess)
    return set_error(ctx, QTT_EHIP, "build_tt: bonds");
  for (int k = 0; k <= L; ++k) bond_host[k] = hb[k];
  if (hipStreamSynchronize(s) != hipSuccess) return set_error(ctx, QTT_EHIP, "build_tt: stream");
  return QTT_OK;
}
