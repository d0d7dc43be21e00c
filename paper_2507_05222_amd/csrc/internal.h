// Internal declarations shared by the HIP kernels (kernels.hip) and the C-ABI
// orchestration (api.hip). Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#define QTT_BMAX 32      // chains per launch (kernel-argument job table)
#define QTT_LANES 4      // launch batches of one call that run at once (side streams)

// One chain of a batched operation: device pointers of its operands and its
// private workspace. Unused pointers are null.
struct Chain {
  const double* x;  const int* xb;   // input MPS cores / bonds
  double* y;        int* yb;         // output MPS cores / bonds
  const double* m;  const int* mb;   // MPO cores / bonds
  const double* x2; const int* x2b;  // second input MPS (direct sum, dots)
  double* ws;                        // workspace of this chain
  double alpha, beta;                // scalars (direct sum weights etc.)
};

struct Batch {
  int n;
  Chain c[QTT_BMAX];
};

// Shape parameters common to all chains of a launch.
struct Geo {
  int L;        // cores
  int k;        // current site
  int capx;     // slot capacity of x
  int capy;     // slot capacity of y
  int wcap;     // slot capacity of the MPO
  int W;        // max MPO bond over the batch (workspace sizing)
  int d;        // physical dimension of x / y (2)
  double tol;   // truncation rel_tol
  int chi_max;  // truncation cap
  int mode;     // contraction type: 0 f64, 1 f32, 2 bf16
  int cap2;     // slot capacity of the second input (x2)
  int splits;   // split-K factor of the Gram products
  int lds;      // dynamic LDS budget (bytes) of the one-workgroup kernels
  double* cnt;  // measurement counters (algorithmic flops, bytes) or null
};

// Kernel classes of the measurement hook (qtt_timer_start / qtt_timer_read).
enum KClass {
  KC_ZIP_CONTRACT = 0,  // zip-up site contractions (carry.X_k, and M_k.T1 when fused)
  KC_ZIP_GRAM = 1,      // Gram products of the zip-up
  KC_ZIP_FACTOR = 2,    // Jacobi eigen-decomposition of the Gram matrix
  KC_ZIP_CARRY = 3,     // carry projection U^T Theta
  KC_RL_SVD = 4,        // right-to-left Jacobi SVD sweep sites
  KC_LR_QR = 5,         // Householder QR / LQ gauge moves
  KC_JOBS = 6,          // environment / local-matvec / projection GEMMs, FP64 MFMA
  KC_CG = 7,            // local CG vector updates
  KC_JOBS_LP = 8,       // the same GEMMs on FP32 or BF16 MFMA
  KC_ZIP_MPO = 9,       // zip-up contraction with the MPO core (k_zip_t2)
  KC_CG_COOP = 10,      // local CG solves in one cooperative launch each (FP64 MFMA products)
  KC_COUNT = 11
};

namespace qttk {
struct Timer {
  int kc = -1;                   // active class, -1 = off
  double* cnt = nullptr;         // device counters [flops, bytes]
  std::vector<hipEvent_t> ev;    // begin/end pairs
  size_t used = 0;
};
Timer& timer();
// Records an event on s if class kc is being timed (call before and after a launch).
void tmark(int kc, hipStream_t s);
// Mean duration (ms) of an event bracket around an empty launch on s.
double bracket_overhead_ms(hipStream_t s);
// Device counter pointer for a launch of class kc (null unless kc is being timed).
inline double* tcount(int kc) { return timer().kc == kc ? timer().cnt : nullptr; }
}  // namespace qttk

// Workspace layout of one chain for the zip-up / sweeps (offsets in doubles).
struct WsLayout {
  size_t carry, t1, theta, gpart, tmpA, mt, scal, total;
  int splits;
  static WsLayout make(int L, int C, int W, int splits);
};

// Scalar slots inside the `scal` area of a chain workspace.
enum {
  SC_NORM2 = 0,     // squared norm of the train being rounded
  SC_TRUNC2 = 1,    // accumulated discarded squared singular values
  SC_BOND = 2,      // integer values stored as doubles (old bond etc.)
  SC_RANK = 3,
  SC_DOT = 4,
  SC_COUNT = 16
};

// ---- launchers (kernels.hip) ----------------------------------------------
namespace qttk {
// one-time setup: dynamic LDS limits of the one-workgroup kernels
hipError_t init(int lds_bytes);
void ws_init(const Batch& b, const WsLayout& wl, hipStream_t s);
void zip_init(const Batch& b, const WsLayout& wl, hipStream_t s);
void zip_t1(const Batch& b, const Geo& g, hipStream_t s);
void zip_t2(const Batch& b, const Geo& g, hipStream_t s);
// both zip-up contractions of a site: fused in one kernel (FP64, capx 64 or 128,
// MPO bond <= 32) or zip_t1 then zip_t2; zip_contract_fused returns false if it
// launched nothing
void zip_contract(const Batch& b, const Geo& g, hipStream_t s);
bool zip_contract_fused(const Batch& b, const Geo& g, hipStream_t s);
void zip_gram(const Batch& b, const Geo& g, hipStream_t s);
void zip_factor(const Batch& b, const Geo& g, hipStream_t s);
void mpo_transpose(const Batch& b, const Geo& g, hipStream_t s);
void zip_carry(const Batch& b, const Geo& g, hipStream_t s);
void zip_last(const Batch& b, const Geo& g, hipStream_t s);
// right-to-left truncated SVD sweep over y (in place), sites L-1 .. 1
void rl_svd_site(const Batch& b, const Geo& g, int from_tmp, hipStream_t s);
void rl_finish(const Batch& b, const Geo& g, hipStream_t s);
// left-to-right QR sweep over y (in place), sites 0 .. L-2
void lr_qr_site(const Batch& b, const Geo& g, int from_tmp, hipStream_t s);
void lr_finish(const Batch& b, const Geo& g, hipStream_t s);
// misc
void direct_sum(const Batch& b, const Geo& g, hipStream_t s);      // y <- alpha x (+) beta x2
void copy_mps(const Batch& b, const Geo& g, hipStream_t s);        // y <- alpha x (cap change allowed)
void diag_mpo(const Batch& b, const Geo& g, hipStream_t s);        // y (mpo slots, wcap=capx) <- diag(x)
void apply_local(const Batch& b, const Geo& g, hipStream_t s);     // y <- D x, D bond-1 MPO
// <x, y> (with_mpo = 0) or <x, M x2> (with_mpo = 1) by left environments; the
// result lands in the chain's scal[SC_DOT].
void dot_init(const Batch& b, const Geo& g, hipStream_t s);
void dot_step(const Batch& b, const Geo& g, int with_mpo, hipStream_t s);
void dot_finish(const Batch& b, const Geo& g, hipStream_t s);
void dot_out(const Batch& b, const Geo& g, double* out, hipStream_t s);   // device out[i] <- chain i's result
}  // namespace qttk
