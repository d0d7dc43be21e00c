// Host FP64 tensor-train helpers (setup only). One-sided Jacobi SVD after
// Hestenes (1958); TT-SVD and rounding as successive SVDs (Sec. 2).
#include "host_linalg.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace {

// One-sided Jacobi on the columns of B (rows x cols, column-major in `b`),
// accumulating the rotations in V (cols x cols, column-major).
void jacobi_cols(int rows, int cols, std::vector<double>& b, std::vector<double>& V) {
  V.assign((size_t)cols * cols, 0.0);
  for (int i = 0; i < cols; ++i) V[(size_t)i * cols + i] = 1.0;
  const double eps = 2.2e-16 * std::max(1, rows);
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < cols - 1; ++p)
      for (int q = p + 1; q < cols; ++q) {
        double* bp = &b[(size_t)p * rows];
        double* bq = &b[(size_t)q * rows];
        double alpha = 0, beta = 0, gamma = 0;
        for (int i = 0; i < rows; ++i) { alpha += bp[i] * bp[i]; beta += bq[i] * bq[i]; gamma += bp[i] * bq[i]; }
        if (alpha == 0.0 || beta == 0.0) continue;
        if (std::fabs(gamma) <= eps * std::sqrt(alpha * beta)) continue;
        rotated = true;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < rows; ++i) {
          const double x = bp[i], y = bq[i];
          bp[i] = c * x - s * y;
          bq[i] = s * x + c * y;
        }
        double* vp = &V[(size_t)p * cols];
        double* vq = &V[(size_t)q * cols];
        for (int i = 0; i < cols; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
}

}  // namespace

void svd_host(int m, int n, const double* A, std::vector<double>& U, std::vector<double>& s,
              std::vector<double>& Vt) {
  const int r = std::min(m, n);
  std::vector<double> b, V;
  const bool tall = m >= n;
  // B = A (tall) or A^T (wide), stored column-major with `rows` rows
  const int rows = tall ? m : n, cols = tall ? n : m;
  b.resize((size_t)rows * cols);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      if (tall) b[(size_t)j * rows + i] = A[(size_t)i * n + j];
      else b[(size_t)i * rows + j] = A[(size_t)i * n + j];
    }
  jacobi_cols(rows, cols, b, V);
  std::vector<double> nrm(cols);
  for (int c = 0; c < cols; ++c) {
    double a = 0;
    for (int i = 0; i < rows; ++i) a += b[(size_t)c * rows + i] * b[(size_t)c * rows + i];
    nrm[c] = std::sqrt(a);
  }
  std::vector<int> ord(cols);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
  U.assign((size_t)m * r, 0.0);
  Vt.assign((size_t)r * n, 0.0);
  s.assign(r, 0.0);
  for (int k = 0; k < r; ++k) {
    const int c = ord[k];
    s[k] = nrm[c];
    const double inv = nrm[c] > 0 ? 1.0 / nrm[c] : 0.0;
    if (tall) {  // A V = W: U = W/s, Vt = V^T
      for (int i = 0; i < m; ++i) U[(size_t)i * r + k] = b[(size_t)c * rows + i] * inv;
      for (int j = 0; j < n; ++j) Vt[(size_t)k * n + j] = V[(size_t)c * cols + j];
    } else {     // A^T V = W: A = V W^T, U = V, Vt = (W/s)^T
      for (int i = 0; i < m; ++i) U[(size_t)i * r + k] = V[(size_t)c * cols + i];
      for (int j = 0; j < n; ++j) Vt[(size_t)k * n + j] = b[(size_t)c * rows + j] * inv;
    }
  }
}

HostTT tt_svd_host(const std::vector<double>& v, int L, int d, double rel_tol, int chi_max, double abs_thr) {
  HostTT T;
  T.L = L; T.d = d;
  double nrm = 0;
  for (double x : v) nrm += x * x;
  nrm = std::sqrt(nrm);
  const double delta = rel_tol / std::sqrt(std::max(L - 1, 1)) * nrm;
  std::vector<double> C = v;
  int r = 1;
  T.bl.push_back(1);
  for (int k = 0; k < L - 1; ++k) {
    const int m = r * d;
    const int n = (int)(C.size() / m);
    std::vector<double> U, s, Vt;
    svd_host(m, n, C.data(), U, s, Vt);
    const int full = (int)s.size();
    // smallest rank whose discarded tail is within delta
    int rk = full;
    double tail = 0.0;
    for (int q = full - 1; q >= 0; --q) {
      if (std::sqrt(tail + s[q] * s[q]) <= delta) { tail += s[q] * s[q]; rk = q; }
      else break;
    }
    while (rk > 0 && s[rk - 1] <= abs_thr) --rk;
    rk = std::max(1, std::min(rk, chi_max));
    std::vector<double> core((size_t)m * rk);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < rk; ++j) core[(size_t)i * rk + j] = U[(size_t)i * full + j];
    T.cores.push_back(core);
    T.bl.push_back(rk);
    std::vector<double> Cn((size_t)rk * n);
    for (int i = 0; i < rk; ++i)
      for (int j = 0; j < n; ++j) Cn[(size_t)i * n + j] = s[i] * Vt[(size_t)i * n + j];
    C.swap(Cn);
    r = rk;
  }
  T.cores.push_back(C);   // (r, d, 1)
  T.bl.push_back(1);
  return T;
}

HostTT tt_direct_sum(const HostTT& A, const HostTT& B) {
  HostTT C;
  C.L = A.L; C.d = A.d;
  const int L = A.L, d = A.d;
  C.bl.push_back(1);
  for (int k = 0; k < L; ++k) {
    const int a0 = A.bl[k], a1 = A.bl[k + 1], b0 = B.bl[k], b1 = B.bl[k + 1];
    const int c0 = (k == 0) ? 1 : a0 + b0;
    const int c1 = (k == L - 1) ? 1 : a1 + b1;
    std::vector<double> core((size_t)c0 * d * c1, 0.0);
    for (int s = 0; s < d; ++s) {
      for (int i = 0; i < a0; ++i)
        for (int j = 0; j < a1; ++j)
          core[((size_t)i * d + s) * c1 + j] += A.cores[k][((size_t)i * d + s) * a1 + j];
      const int oi = (k == 0) ? 0 : a0, oj = (k == L - 1) ? 0 : a1;
      for (int i = 0; i < b0; ++i)
        for (int j = 0; j < b1; ++j)
          core[((size_t)(i + oi) * d + s) * c1 + (j + oj)] += B.cores[k][((size_t)i * d + s) * b1 + j];
    }
    C.cores.push_back(core);
    C.bl.push_back(c1);
  }
  return C;
}

void tt_round_host(HostTT& T, double rel_thr) {
  const int L = T.L, d = T.d;
  // left-to-right orthogonalisation
  for (int k = 0; k < L - 1; ++k) {
    const int m = T.bl[k] * d, n = T.bl[k + 1];
    std::vector<double> U, s, Vt;
    svd_host(m, n, T.cores[k].data(), U, s, Vt);
    int r = (int)s.size();
    while (r > 1 && s[r - 1] == 0.0) --r;
    const int full = (int)s.size();
    std::vector<double> core((size_t)m * r);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < r; ++j) core[(size_t)i * r + j] = U[(size_t)i * full + j];
    // next core <- (s Vt)[:r] * next
    const int n1 = d * T.bl[k + 2];
    std::vector<double> nxt((size_t)r * n1, 0.0);
    for (int i = 0; i < r; ++i)
      for (int t = 0; t < n; ++t) {
        const double w = s[i] * Vt[(size_t)i * n + t];
        if (w == 0.0) continue;
        for (int j = 0; j < n1; ++j) nxt[(size_t)i * n1 + j] += w * T.cores[k + 1][(size_t)t * n1 + j];
      }
    T.cores[k] = core;
    T.cores[k + 1] = nxt;
    T.bl[k + 1] = r;
  }
  // right-to-left truncation
  for (int k = L - 1; k > 0; --k) {
    const int m = T.bl[k], n = d * T.bl[k + 1];
    std::vector<double> U, s, Vt;
    svd_host(m, n, T.cores[k].data(), U, s, Vt);
    const int full = (int)s.size();
    int r = 0;
    for (int q = 0; q < full; ++q) if (s[q] > rel_thr * s[0]) r = q + 1;
    r = std::max(r, 1);
    std::vector<double> core((size_t)r * n);
    for (int i = 0; i < r; ++i)
      for (int j = 0; j < n; ++j) core[(size_t)i * n + j] = Vt[(size_t)i * n + j];
    const int m0 = T.bl[k - 1] * d;
    std::vector<double> prv((size_t)m0 * r, 0.0);
    for (int i = 0; i < m0; ++i)
      for (int t = 0; t < m; ++t) {
        const double w = T.cores[k - 1][(size_t)i * m + t];
        if (w == 0.0) continue;
        for (int j = 0; j < r; ++j) prv[(size_t)i * r + j] += w * U[(size_t)t * full + j] * s[j];
      }
    T.cores[k] = core;
    T.cores[k - 1] = prv;
    T.bl[k] = r;
  }
}
