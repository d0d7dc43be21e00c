// Host FP64 tensor-train helpers used only at setup (operator construction and
// encoding of initial fields). The device path never calls these.
#pragma once
#include <vector>

struct HostTT {
  int L = 0, d = 2;
  std::vector<std::vector<double>> cores;   // core k: [bl[k]][d][bl[k+1]] row-major
  std::vector<int> bl;                      // L+1 bonds
};

// Thin SVD of a row-major m x n matrix by one-sided Jacobi (Hestenes). Returns
// r = min(m, n) singular triplets sorted by decreasing s: U (m x r, row-major),
// s (r), Vt (r x n, row-major).
void svd_host(int m, int n, const double* A, std::vector<double>& U, std::vector<double>& s,
              std::vector<double>& Vt);

// TT-SVD (successive SVDs, App. D / Sec. 2): per-bond discarded norm
// <= rel_tol/sqrt(L-1)*||v||, singular values <= abs_thr dropped, at most chi_max kept.
HostTT tt_svd_host(const std::vector<double>& v, int L, int d, double rel_tol, int chi_max, double abs_thr);

// Direct sum (Sec. 2.1.1): first cores side by side, last cores stacked, others block-diagonal.
HostTT tt_direct_sum(const HostTT& A, const HostTT& B);

// Rounding: left-to-right orthogonalisation, then right-to-left SVD dropping
// singular values below rel_thr times the largest at each bond (Sec. 3.2.3).
void tt_round_host(HostTT& T, double rel_thr);
