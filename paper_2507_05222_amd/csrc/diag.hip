// Read-out of grid rows from a QTT field (App. C: fixing the eta bits of the
// index leaves a train over the xi bits, contracted to 2^n values)
// for the diagnostics of Sec. 4 (wall forces, App. F). Host FP64 after one copy
// of the cores; the time step never calls it.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "../../include/qtt.h"

namespace qtt_solver_detail {
int set_error(qtt_ctx* ctx, int code, const char* msg);
}

extern "C" int qtt_read_rows(qtt_ctx* ctx, const qtt_mps* x, int nrows, const int32_t* rows, int32_t order,
                             double* out, void* stream) {
  using qtt_solver_detail::set_error;
  if (!ctx) return QTT_EINVAL;
  if (!x || !x->data || !x->bond || !rows || !out || nrows < 1 || x->d != 2 || x->L < 2 || (x->L & 1) ||
      (order != QTT_ORDER_INTERLEAVED && order != QTT_ORDER_CONCATENATED))
    return set_error(ctx, QTT_EINVAL, "read_rows: needs a binary train of 2n cores, a bit order and host buffers");
  const int L = x->L, n = L / 2, cap = x->cap, N = 1 << n;
  for (int r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= N) return set_error(ctx, QTT_EINVAL, "read_rows: row index out of range");
  hipStream_t s = (hipStream_t)stream;
  const size_t slot = (size_t)L * cap * 2 * cap;
  std::vector<double> hs(slot);
  std::vector<int> bl(L + 1);
  if (hipMemcpyAsync(hs.data(), x->data, slot * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(bl.data(), x->bond, (L + 1) * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(ctx, QTT_EHIP, "read_rows: copy failed");
  auto core = [&](int k, int a, int sb, int b) { return hs[(size_t)k * cap * 2 * cap + (size_t)a * 2 * cap + sb * cap + b]; };
  for (int r = 0; r < nrows; ++r) {
    const int I = rows[r];
    // v[q][a]: q over the xi bits met so far (MSB first), a the bond index
    std::vector<double> v(1, 1.0);
    int q = 1;
    for (int k = 0; k < L; ++k) {
      const int a0 = bl[k], b0 = bl[k + 1];
      const bool eta = order == QTT_ORDER_CONCATENATED ? k < n : (k & 1) == 0;
      if (eta) {                                // eta bit m of the row index, MSB first
        const int m = order == QTT_ORDER_CONCATENATED ? k : k / 2;
        const int bit = (I >> (n - 1 - m)) & 1;
        std::vector<double> nv((size_t)q * b0, 0.0);
        for (int t = 0; t < q; ++t)
          for (int a = 0; a < a0; ++a) {
            const double x0 = v[(size_t)t * a0 + a];
            if (x0 == 0.0) continue;
            for (int b = 0; b < b0; ++b) nv[(size_t)t * b0 + b] += x0 * core(k, a, bit, b);
          }
        v.swap(nv);
      } else {                                  // xi bit: both values kept
        std::vector<double> nv((size_t)q * 2 * b0, 0.0);
        for (int t = 0; t < q; ++t)
          for (int a = 0; a < a0; ++a) {
            const double x0 = v[(size_t)t * a0 + a];
            if (x0 == 0.0) continue;
            for (int sb = 0; sb < 2; ++sb)
              for (int b = 0; b < b0; ++b) nv[((size_t)t * 2 + sb) * b0 + b] += x0 * core(k, a, sb, b);
          }
        v.swap(nv);
        q *= 2;
      }
    }
    std::memcpy(out + (size_t)r * N, v.data(), (size_t)N * sizeof(double));
  }
  return QTT_OK;
}
