/*
 * qtt.h -- C ABI of the MI355X (gfx950) library for the quantics-tensor-train
 * fractional-step method of arxiv 2507.05222 ("Quantum-Inspired Tensor-Network
 * Fractional-Step Method for Incompressible Flow in Curvilinear Coordinates").
 *
 * Every entry point takes plain pointers and sizes; no C++ or torch types cross
 * this boundary. Device pointers are HIP device allocations owned by the caller;
 * `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls are
 * stream-ordered; a call that returns a host scalar synchronises its stream first.
 *
 * Return value: QTT_OK (0) or a negative error code. No exception crosses the
 * ABI. On QTT_EINVAL / QTT_ESHAPE nothing has been launched and no output has
 * been written. qtt_last_error() gives the message of the last failure of a ctx.
 *
 * Data layout (Sec. 2, Eq. simpleMPS / simpleMatrix):
 *   A TT-vector (MPS) has L cores A[k] of shape (b_k, d, b_{k+1}), b_0 = b_L = 1.
 *   Core k is stored in slot k of `data`: slot size cap*d*cap doubles, element
 *   (a, s, c) at data[k*cap*d*cap + a*(d*cap) + s*cap + c]. Entries outside the
 *   actual bonds are zero (every library kernel that writes a core keeps this).
 *   `bond` is a DEVICE int32 array of length L+1 with the actual bond dims; the
 *   library updates it in place and never reallocates.
 *   The dense vector represented has its entry at index sum_k r_k d^(L-1-k)
 *   equal to A[0]^{r_0} ... A[L-1]^{r_{L-1}}: core 0 carries the most
 *   significant digit (App. D). A 2D field f(i, j) on a 2^n x 2^n grid uses the
 *   interleaved MSB-first bit order i_1 j_1 i_2 j_2 ... (core 2m <- bit m of i,
 *   core 2m+1 <- bit m of j).
 *   A TT-matrix (MPO) core has shape (w_k, 2 (out r'), 2 (in r), w_{k+1}) in slots
 *   of wcap*4*wcap doubles, element (b, r', r, c) at
 *   data[k*wcap*4*wcap + b*4*wcap + r'*2*wcap + r*wcap + c].
 */
#ifndef QTT_H
#define QTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  QTT_OK = 0,
  QTT_EINVAL = -1,       /* bad argument (null pointer, bad enum, bad count)      */
  QTT_ESHAPE = -2,       /* inconsistent L / d / capacities between operands     */
  QTT_ECAPACITY = -3,    /* a result needs more than the output capacity allows   */
  QTT_ENUMERIC = -4,     /* NaN or Inf detected in a result                       */
  QTT_ENOTCONVERGED = -5,/* solver stopped at max_sweeps above tol; x = best iterate */
  QTT_EHIP = -6          /* a HIP runtime call failed                              */
};

/* Arithmetic type of the site contractions (MFMA). Truncation (QR/SVD),
 * re-orthogonalisation, dot products and residuals are always FP64. */
typedef enum { QTT_F64 = 0, QTT_F32 = 1, QTT_BF16 = 2 } qtt_dtype;

/* MPS descriptor (host struct holding device pointers). */
typedef struct {
  int32_t L;        /* number of cores                                   */
  int32_t d;        /* physical dimension (2; 4 for an MPO seen as MPS)  */
  int32_t cap;      /* bond capacity (slot leading dimension)            */
  int32_t* bond;    /* DEVICE int32[L+1], actual bonds                   */
  double* data;     /* DEVICE double[L*cap*d*cap]                        */
} qtt_mps;

/* MPO descriptor. Bonds are fixed at construction and known on the host;
 * bond_host may hold upper bounds of the device values (it is used for
 * validation and workspace sizing only). */
typedef struct {
  int32_t L;
  int32_t wcap;             /* slot leading dimension                    */
  const int32_t* bond_host; /* HOST int32[L+1]                           */
  const int32_t* bond;      /* DEVICE int32[L+1] (same values)           */
  const double* data;       /* DEVICE double[L*wcap*4*wcap]              */
} qtt_mpo;

/* Truncation rule (Sec. 2: "neglecting singular values below a threshold or
 * selecting the first chi"): per bond, the discarded singular values s_i must
 * satisfy sqrt(sum s_i^2) <= rel_tol/sqrt(L-1) * ||x|| (so ||x - x~|| <= rel_tol ||x||),
 * and at most chi_max values are kept (chi_max <= cap of the output). */
typedef struct {
  double rel_tol;
  int32_t chi_max;
  int32_t fit_sweeps;   /* qtt_apply_mpo only: variational fitting sweeps after the
                           zip-up (Sec. 2.2), 0..64; other calls ignore it */
} qtt_trunc;

/* Options of the variational linear solve (Sec. 2.1.4, Eq. LSE).
 * Residual measure: before each local update the solver evaluates, in FP64,
 * r_k = ||P_k (b - A x)|| with P_k the orthogonal projection onto the frame of
 * site k (the residual of the local system). The "residual" of a sweep is the
 * largest r_k / ||b|| met in it; all r_k vanish at a stationary point of the
 * alternating iteration, and r_k <= ||b - A x|| always. */
typedef struct {
  double tol;               /* stop when the sweep residual is <= tol             */
  int32_t max_sweeps;       /* full sweeps (left-to-right + right-to-left), >= 1  */
  int32_t max_local_iters;  /* CG iterations per local problem                    */
  double local_tol;         /* local CG stops once its residual is below local_tol
                               times the local residual before the update, or below
                               tol * ||b|| / (2 sqrt(L))                          */
  int32_t contract_dt;      /* qtt_dtype of the local matrix-vector products      */
} qtt_solve_opts;

typedef struct {
  int32_t sweeps;           /* sweeps performed                                   */
  int32_t local_iters;      /* total CG iterations                                */
  double residual;          /* sweep residual of the last sweep (FP64)            */
  double residual0;         /* sweep residual of the first sweep                  */
} qtt_solve_info;

/* ---- context ------------------------------------------------------------ */

typedef struct qtt_ctx qtt_ctx;

/* Create a context on HIP device `device`. The context owns its scratch
 * workspace (grown on demand) and four streams of default priority with their
 * events (used only by calls of more than 32 problems), all freed by qtt_destroy.
 * Calls on one context share its workspace: issue them from one host thread, in
 * the order of one stream, or synchronise between them. QTT_EHIP if a HIP call
 * fails. */
int qtt_create(int device, qtt_ctx** out);
void qtt_destroy(qtt_ctx* ctx);
const char* qtt_last_error(const qtt_ctx* ctx);

/* ---- TT algebra (Sec. 2.1) -------------------------------------------------
 * Every operation takes `n` independent problems (arrays of n descriptors) and
 * runs them together, site by site. All problems of one call share L, d and the
 * capacities. One launch holds up to 32 problems; qtt_apply_mpo and qtt_round
 * with more run their launch batches up to four at a time on the context's own
 * streams, which wait for `stream` on entry and which `stream` waits for before
 * the call returns, so the call is ordered on `stream` like a single launch
 * sequence. */

/* y_i = round(M_i x_i): MPO times MPS (Sec. 2.1.2, mat-vec with fused bond) by a
 * left-to-right zip-up that truncates each site as it is formed, a right-to-left
 * truncated-SVD sweep (Sec. 2, TT-rounding) that fixes the bonds, and
 * tr->fit_sweeps single-site variational fitting sweeps at those bonds (Sec. 2.2,
 * the variational mat-vec of Table 1): each site becomes the projection of M x
 * onto the orthonormal frame of the other cores, so ||y - M x|| decreases.
 * y is left right-canonical (cores 1..L-1 right-orthonormal). x_i and y_i must
 * not alias. contract_dt selects the MFMA type of the site contractions. */
int qtt_apply_mpo(qtt_ctx* ctx, int n, const qtt_mpo* M, const qtt_mps* x, qtt_mps* y,
                  const qtt_trunc* tr, int contract_dt, void* stream);

/* TT-SVD of a dense vector into a device MPS (Sec. 2, Eq. simpleMPS; App. D for the
 * digit order): `dense` is a HOST array of 2^L doubles (1 <= L <= 26), entry
 * sum_k r_k 2^(L-1-k) at index r_0 .. r_{L-1} (core 0 the most significant digit).
 * Successive truncated SVDs from the left on the host (FP64, the qtt_trunc rule
 * with chi_max capped at out->cap), the cores are then copied into out's slots
 * (entries outside the bonds zero) and out->bond is set; the call synchronises
 * the stream. QTT_ENUMERIC if the input holds NaN or Inf. For encoding initial
 * fields and coarse predictions: the time step itself never decompresses. */
int qtt_from_dense(qtt_ctx* ctx, const double* dense, int32_t L, const qtt_trunc* tr, qtt_mps* out, void* stream);

/* In-place TT-rounding (Sec. 2: regular truncation): left-to-right Householder QR
 * sweep, then right-to-left truncated SVD (one-sided Jacobi) sweep, FP64.
 * The result is right-canonical. */
int qtt_round(qtt_ctx* ctx, int n, qtt_mps* x, const qtt_trunc* tr, void* stream);

/* z_i = round(a_i x_i + b_i y_i) (Sec. 2.1.1: direct sum, bond chi_a + chi_b, then
 * rounding). a, b are HOST arrays of n doubles. z may alias neither x nor y. */
int qtt_add(qtt_ctx* ctx, int n, const double* a, const qtt_mps* x, const double* b,
            const qtt_mps* y, qtt_mps* z, const qtt_trunc* tr, void* stream);

/* out[i] = <x_i, y_i> in FP64 (left environments). `out` is a HOST array of n
 * doubles; the stream is synchronised. */
int qtt_dot(qtt_ctx* ctx, int n, const qtt_mps* x, const qtt_mps* y, double* out, void* stream);

/* qtt_dot for callers that cannot allocate device or pinned memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * FP64 inner products, written to out (DEVICE, n doubles) in stream order; no
 * allocation and no synchronisation. Its workspace is a file-scope device array
 * of 2^20 doubles (8 MiB) that every GPU the library runs on holds until the
 * process ends: problems whose workspace (about 17 cap^2 doubles for cap =
 * max(x.cap, y.cap)) exceeds it are refused with QTT_ECAPACITY, larger batches run
 * in chunks. All calls on one GPU share that array: calls that overlap on one GPU
 * (other streams, other contexts, other threads) race and must be serialised by
 * the caller. */
int qtt_dot_noalloc(qtt_ctx* ctx, int n, const qtt_mps* x, const qtt_mps* y, double* out, void* stream);

/* out[i] = <x_i, A_i y_i> in FP64. HOST out; synchronises. */
int qtt_dot_mpo(qtt_ctx* ctx, int n, const qtt_mps* x, const qtt_mpo* A, const qtt_mps* y,
                double* out, void* stream);

/* Diagonal scaling by a bond-1 MPO: y_i = D_i x_i where every core of D_i is a
 * 2x2 matrix (w = 1). Exact (no truncation, bonds unchanged). */
int qtt_apply_local(qtt_ctx* ctx, int n, const qtt_mpo* D, const qtt_mps* x, qtt_mps* y, void* stream);

/* One term c M x of a variational fit; M == NULL means the identity. */
typedef struct {
  double coef;
  const qtt_mpo* M;
  const qtt_mps* x;
} qtt_term;

/* Variational fit y_i ~ sum_t c_it M_it x_it at fixed bonds (Sec. 2.2: the
 * variational mat-vec / addition / elementwise product of Table 1). Single-site
 * sweeps: each core of y becomes the projection of the sum onto the orthonormal
 * frame of the other cores (environments of <y|M_t|x_t>, contractions on MFMA in
 * contract_dt), the gauge moves by Householder QR/LQ; ||y - sum|| decreases
 * monotonically. terms: n*nterms entries, problem-major (nterms <= 4); term t of
 * every problem shares the ket capacity and the MPO wcap (or is the identity for
 * every problem). init = 1 starts from a random train on the profile
 * min(2^k, 2^(L-k), chi) (the first pass is then a randomized sketch of the sum);
 * init = 0 starts from the current content of y, which must be right-canonical
 * with bonds <= chi (e.g. the previous time step's result). sweeps (>= 1) full
 * left-right-left sweeps; y ends right-canonical. No input may alias y. */
int qtt_fit(qtt_ctx* ctx, int n, int nterms, const qtt_term* terms, qtt_mps* y, int chi, int sweeps,
            int init, int contract_dt, void* stream);

/* Single-site variational (ALS / one-site DMRG) solve of A x = b (Sec. 2.1.4,
 * Eq. LSE and its cost function; local problems by CG with the fast matvec of
 * App. G). A must be symmetric positive definite. On entry x holds the initial
 * guess (its bond structure is kept: single-site updates cannot grow bonds); on
 * exit the solution, right-canonical. At least one sweep is made. Sweeps stop
 * when every problem's sweep residual is <= tol, at max_sweeps, or when no
 * problem improved its best sweep residual by 10% (after two sweeps). info
 * (HOST, n entries, may be NULL) receives sweeps, CG iterations and the sweep
 * residuals. A problem with b = 0 gets x = 0 (residual 0). Returns
 * QTT_ENOTCONVERGED if some problem ended above tol (x then holds its last
 * iterate), QTT_ENUMERIC if b or a residual is not finite. */
int qtt_poisson_solve(qtt_ctx* ctx, int n, const qtt_mpo* A, const qtt_mps* b, qtt_mps* x,
                      const qtt_solve_opts* opts, qtt_solve_info* info, void* stream);

/* ---- fractional step (Sec. 3.3) ------------------------------------------- */

/* Operators of the cylinder problem, built once per grid (Sec. 3.2.3, App. A),
 * all in the interleaved order of a 2^n x 2^n O-grid (L = 2n cores).
 * Velocity operators carry Dirichlet rows (wall, far field) whose values enter
 * through the boundary-correction vectors (Sec. 3.1, ghost points); pressure
 * operators use p_{-1,j} = p_{0,j} at the wall and p = 0 at the far field. */
typedef struct {
  qtt_mpo Dx, Dz;           /* curvilinear first derivatives (velocity BCs)      */
  qtt_mpo Dxp, Dzp;         /* pressure gradient (pressure BCs)                  */
  qtt_mpo Wx, Wz;           /* -|J| d/dx, -|J| d/dz (J-weighted divergence)      */
  qtt_mpo Hs;               /* |J|^(1/2) (I - dt/Re Lap) |J|^(-1/2) on velocity (SPD) */
  qtt_mpo P;                /* -|J| Lap with pressure BCs (SPD)                  */
  qtt_mpo Jh, Jmh;          /* |J|^(1/2), |J|^(-1/2) as bond-1 diagonal MPOs     */
  qtt_mps bx_u, bz_u;       /* boundary corrections of Dx, Dz for u              */
  qtt_mps bx_v, bz_v;       /* ... for v                                         */
  qtt_mps bL_u, bL_v;       /* (dt/Re) x boundary corrections of Lap for u, v    */
  qtt_mps bW;               /* boundary correction of Wx u + Wz v                */
} qtt_flow_ops;

typedef struct {
  qtt_mps u, v, p;          /* current fields (right-canonical)                  */
  uint64_t id;              /* caller-chosen identity of this state, unique among the
                               states alive on a context; 0 = none (every step starts
                               its fits cold)                                       */
} qtt_flow_state;

/* Learned warm start of the pressure solve (see the qtt_ws_* calls below). */
typedef struct {
  const float* params;      /* DEVICE, QTT_WS_NPARAMS floats                       */
  double out_scale;         /* coarse pressure = output * out_scale * rms(coarse b) */
  double re, alpha;         /* conditioning inputs: Reynolds number, rotation rate */
  int32_t chi;              /* bond of the compressed coarse prediction, 1..cap    */
  int32_t bf16;             /* network forward with BF16 operands                 */
} qtt_ws_model;

typedef struct {
  double dt;                /* time step                                          */
  qtt_trunc trunc;          /* truncation of every TT operation of the step       */
  int32_t contract_dt;      /* qtt_dtype of the derivative, divergence and gradient
                               applies (differences of nearly equal terms: FP32 or FP64) */
  int32_t product_dt;       /* qtt_dtype of the convection (Hadamard) products    */
  qtt_solve_opts helmholtz; /* options of the two predictor solves                */
  qtt_solve_opts poisson;   /* options of the pressure solve                      */
  const qtt_ws_model* warm; /* NULL, or the learned warm start of the pressure solve */
  qtt_mps* rhs_out;         /* NULL, or receives the pressure right-hand side b   */
} qtt_step_opts;

typedef struct {
  qtt_solve_info helm_u, helm_v, poisson;
  int32_t warm_used;        /* 1 if the learned guess replaced the previous pressure */
  double warm_energy;       /* J at the optimal scale of the learned guess (0 if none) */
  double prev_energy;       /* the same for the previous pressure                  */
} qtt_step_info;

/* One Chorin fractional step (Sec. 3.3): explicit convection (Hadamard products of
 * v with its curvilinear gradients), implicit viscous predictor (Eq.
 * intermediate_vel_eq, solved variationally in the symmetric form
 * |J|^(1/2)(I - dt/Re Lap)|J|^(-1/2)), J-weighted pressure Poisson solve (Sec. 3.3),
 * projection v = v* - dt grad p. state->p is the initial guess of the pressure
 * solve and receives the new pressure. The solves read their FP64 residual on
 * the host once per sweep, so the call synchronises its stream. A solve that
 * stops at its bond-limited floor above tol is not an error here: info (HOST,
 * may be NULL) receives the sweeps, CG iterations and residuals of the three solves.
 * All seven boundary vectors must share one capacity. Every linear combination
 * (gradients, convection, right-hand sides, divergence, projection) is one
 * qtt_fit at bond min(trunc.chi_max, cap) with trunc.fit_sweeps sweeps; the
 * context keeps the step's intermediate trains, and when the previous step on
 * the context advanced the same state (same u, v, p storage) the fits start
 * from them, otherwise from a random sketch (one more sweep).
 * With opts->warm (n >= 6 cores per axis, state->p.cap == state->u.cap), on a step
 * whose state->p is not the previous pressure of this state on this context (the
 * state's first step, or another state stepped since; a running simulation keeps
 * its previous pressure, the better start, and pays nothing): b is
 * block-averaged to the 64 x 64 grid (its last 2(n-6) cores contracted with
 * [1/2, 1/2]), the network predicts the coarse pressure, which is compressed by
 * TT-SVD to bond warm->chi, prolonged piecewise constantly (2(n-6) appended
 * cores [1, 1]) and fitted at the state's bond. Both candidates, the prediction
 * and state->p, are rated at their optimal scale a* = b.x / x.Px by the solve's
 * cost function J(x) = x.Px/2 - b.x (Sec. 2.1.4), J(a* x) = -(b.x)^2 / (2 x.Px);
 * if the prediction rates lower, a* times it replaces state->p as the initial
 * guess. opts->rhs_out (cap >= the state's bond) receives b. */
int qtt_fractional_step(qtt_ctx* ctx, const qtt_flow_ops* ops, qtt_flow_state* state,
                        const qtt_step_opts* opts, qtt_step_info* info, void* stream);

/* ---- measurement hook (not part of the method) ----------------------------
 * While a kernel class is selected, every launch of that class is bracketed by
 * HIP events on its stream, and its GEMM-type kernels add their algorithmic work
 * (2 M N K flops and 8 (M K + K N + M N) bytes per product, with the actual bond
 * dimensions) to device counters. Classes: 0 zip-up site contractions (both
 * products of a site in one kernel in FP64 at slot capacity 64 or 128 with MPO
 * bond <= 32; otherwise the carry-times-core product alone), 1 zip-up Gram
 * products, 2 zip-up Jacobi factorisation, 3 zip-up carry projection, 4
 * right-to-left Jacobi SVD sites, 5 Householder QR/LQ moves, 6 environment /
 * local-matvec / projection GEMMs on FP64 MFMA, 7 local CG updates, 8 the GEMMs of
 * class 6 on FP32 or BF16 MFMA, 9 zip-up product with the MPO core when it is not
 * fused into class 0, 10 whole local CG solves of qtt_poisson_solve run as one
 * cooperative launch each (FP64 contractions at slot capacity <= 64: both products
 * of every iteration counted); -1 stops timing.
 * qtt_timer_read synchronises the device and returns the number of timed
 * launches, the summed duration of their event brackets (ms), the counted work,
 * and, for reference, the mean duration of the same bracket around an empty
 * launch on an idle stream (ms). A bracket holds the launch's dispatch besides
 * the kernel, so ms / launches bounds the kernel's own duration from above. */
int qtt_timer_start(qtt_ctx* ctx, int kernel_class);
int qtt_timer_read(qtt_ctx* ctx, int64_t* launches, double* ms, double* flops, double* bytes, double* overhead_ms);
/* Durations (ms) of the individual brackets of the last timed class, in launch
 * order: ms (host, cap entries) receives the first min(cap, launches) of them and
 * *n their number. Valid after qtt_timer_read until the next qtt_timer_start. */
int qtt_timer_durations(qtt_ctx* ctx, double* ms, int64_t cap, int64_t* n);

/* ---- host-side operator construction (setup, FP64, no GPU) ----------------
 * Builds, on the host, the TT cores of the operators and boundary vectors of a
 * 2^n x 2^n O-grid around a unit cylinder (App. E: r_i = 0.5 (2 r_out)^((i+1)/(N+1)),
 * metrics by central differences, App. A), encodes each coefficient field by
 * TT-SVD and assembles sum_o diag(c_o) Shift_o, then rounds the MPO, dropping
 * singular values below 1e-14 of the largest (Sec. 3.2.3).
 *
 * `which` selects the object (QTT_OP_* below). For an MPO, cores are written to
 * `out` (HOST, wcap*4*wcap*L doubles) and bonds to `bond_out` (HOST int32[L+1]);
 * for a vector (QTT_VEC_*), cores go to `out` with slot cap*2*cap and bonds to
 * bond_out. `wcap`/`cap` is the slot size the caller allocated;
 * QTT_ECAPACITY if the object needs more. Call with out == NULL to query the
 * needed capacity in *need. Parameters: n (cores per axis), r_out, Re, dt,
 * alpha (wall rotation rate, Eq. rot_bc), u_inf (far-field velocity). */
enum {
  QTT_OP_DX = 0, QTT_OP_DZ, QTT_OP_DXP, QTT_OP_DZP, QTT_OP_WX, QTT_OP_WZ,
  QTT_OP_HS, QTT_OP_P, QTT_OP_JH, QTT_OP_JMH, QTT_OP_LAP,
  QTT_VEC_BX_U = 100, QTT_VEC_BZ_U, QTT_VEC_BX_V, QTT_VEC_BZ_V, QTT_VEC_BL_U,
  QTT_VEC_BL_V, QTT_VEC_BW, QTT_VEC_ABSJ,
  QTT_VEC_MESH_X = 200, QTT_VEC_MESH_Z, QTT_VEC_JAC   /* qtt_build_tt only */
};
enum { QTT_ORDER_INTERLEAVED = 0, QTT_ORDER_CONCATENATED = 1 };
typedef struct {
  int32_t n;       /* cores per axis; L = 2n, grid 2^n x 2^n */
  double r_out;    /* outer radius (cylinder diameter 1)      */
  double Re, dt;   /* Reynolds number, time step              */
  double alpha;    /* wall rotation rate                       */
  double u_inf;    /* far-field velocity (x direction)         */
  int32_t order;   /* bit order of every encoding (Sec. 3.2.1): QTT_ORDER_INTERLEAVED,
                      core 2m <- bit m of i and core 2m+1 <- bit m of j, or
                      QTT_ORDER_CONCATENATED, cores 0..n-1 <- the bits of i and cores
                      n..2n-1 <- those of j; MSB first in both */
} qtt_cylinder;

int qtt_build_host(const qtt_cylinder* cyl, int which, int32_t cap, double* out,
                   int32_t* bond_out, int32_t* need);

/* The same operators built in TT format on the device (Sec. 3.2.2, Sec. 3.2.3),
 * without forming any 2^n x 2^n field: the grid coordinates x, z as direct sums of
 * an eta-train (ones, exponential wall-normal spacing) concatenated with a
 * xi-train (wall curve, unit normal; encoded from their 2^n values), in the
 * cylinder's bit order; metric terms by the computational central-difference
 * MPOs D_xi, D_eta applied to x, z (the wall and far-field rows enter as boundary
 * vectors); the Jacobian J = x_xi z_eta - x_eta z_xi by Hadamard products (each
 * product formed exactly, then rounded by QR and Jacobi SVD sweeps); 1/J
 * as the ALS solution of diag(-J) a = -1 (qtt_poisson_solve; J < 0 on this grid),
 * polished by Newton steps a <- a + a (1 - J a) (eight at most) down to
 * ||1 - J a|| / ||1|| of some 1e-13;
 * D_x = C1 D_xi - C2 D_eta with C1 = diag(z_eta / J), C2 = diag(z_xi / J) by
 * MPO products, D_z likewise; the seven-term Laplacian of App. A from the metric
 * tensor (Hadamard products) and the eta / xi differences of g_kl / J; the pressure
 * variants fold the wall-row neighbours into row 0 (p_{-1} = p_0), W = -|J| D and
 * P = -|J| Lap_p. Every field operation drops what lies below 1e-14 of its
 * result's norm at each bond, every operator sum or product below 1e-13; a sum
 * that cancels below 1e-12 of its operands' scale (g12 and the xi-derivatives of an
 * orthogonal grid) is taken as exactly zero.
 *
 * which: QTT_OP_DX, QTT_OP_DZ, QTT_OP_DXP, QTT_OP_DZP, QTT_OP_WX, QTT_OP_WZ,
 * QTT_OP_LAP, QTT_OP_P (an
 * MPO: `out` DEVICE double[L*cap*4*cap] in slot layout, `bond_out` DEVICE
 * int32[L+1], `bond_host` HOST int32[L+1]) or QTT_VEC_MESH_X, QTT_VEC_MESH_Z,
 * QTT_VEC_JAC (an MPS: `out` DEVICE double[L*cap*2*cap]). With out == NULL only
 * the needed capacity is returned in *need (HOST, may be NULL otherwise); the
 * object is built either way. QTT_ECAPACITY if cap is too small,
 * QTT_ENOTCONVERGED if the inverse Jacobian stalls above 1e-12.
 * Allocates its temporaries (setup only) and synchronises `stream`. Requires
 * 2 <= n <= 13. */
int qtt_build_tt(qtt_ctx* ctx, const qtt_cylinder* cyl, int which, int32_t cap, double* out,
                 int32_t* bond_out, int32_t* bond_host, int32_t* need, void* stream);

/* ---- diagnostics (Sec. 4, App. C, App. F) --------------------------------- */

/* Rows of a field in bit order `order` (QTT_ORDER_*; App. C: the eta bits of the
 * row index are fixed, the remaining train over the xi bits is contracted): out
 * (HOST, nrows * 2^(L/2) doubles) receives row rows[r] (0 <= rows[r] < 2^(L/2),
 * 0 = the first interior row next to the wall) at out + r * 2^(L/2). Synchronises
 * the stream. */
int qtt_read_rows(qtt_ctx* ctx, const qtt_mps* x, int nrows, const int32_t* rows, int32_t order, double* out,
                  void* stream);

/* Drag and lift coefficients (App. F, Eq. liftdrag; rho = U = D = 1) of the
 * cylinder cyl from rows (HOST, 5 * 2^n doubles): u on rows 0 and 1, v on rows 0
 * and 1, p on row 0 (row 0 next to the wall), with the wall velocity of Eq.
 * rot_bc. Stress tau = -(p + 2/(3Re) div v) I + (1/Re)(grad v + grad v^T), wall
 * derivatives one-sided second order in eta, central in xi; host FP64. */
int qtt_forces_host(const qtt_cylinder* cyl, const double* rows, double* cd, double* cl);

/* Strouhal number and lift amplitude of a sampled lift history (Sec. 4.1.2, Eq.
 * st with D = U = 1; host FP64): over the last `window` (0 < window <= 1) of the n
 * samples (t[i], cl[i]) (HOST arrays, t increasing), y = cl - mean(cl); upward
 * crossings y_i < 0 <= y_{i+1} are located by linear interpolation and
 * St = 1 / (mean spacing of the crossings); amp = (max cl - min cl) / 2 over the
 * window. St is NaN with fewer than min_crossings (>= 2) crossings. */
int qtt_strouhal_host(const double* t, const double* cl, int64_t n, double window, int32_t min_crossings,
                      double* st, double* amp);

/* Host TT-SVD of a dense vector of d^L doubles (App. D; same truncation rule as
 * qtt_trunc), used to encode initial fields. Writes cores into slots of
 * cap*d*cap doubles (HOST) and bonds to bond_out (HOST int32[L+1]). */
int qtt_tt_svd_host(const double* dense, int32_t L, int32_t d, const qtt_trunc* tr,
                    int32_t cap, double* out, int32_t* bond_out);

/* ---- learned warm start of the pressure solve ------------------------------
 * Not in the paper: its counterpart there is a TT preconditioner of the Poisson
 * solve (App. G, Sec. 4.3). A four-layer 3x3 convolutional network maps
 * (b, Re/200, alpha/2) on the 64 x 64 block-averaged grid (rows eta with zero
 * padding, columns xi with periodic padding) to a coarse pressure, which the
 * caller turns into an initial guess of qtt_poisson_solve. Channels 3 -> 32 ->
 * 32 -> 32 -> 1, the taps of layers 1-4 spaced 1, 2, 4, 8 apart (receptive field
 * 31 x 31), tanh after layers 1-3. All buffers are DEVICE float arrays,
 * NCHW with H = W = 64, owned by the caller; calls are stream-ordered.
 * Parameter layout: for layer l, w_l[co][ci][3][3] then b_l[co]. */
#define QTT_WS_NPARAMS 19681
#define QTT_WS_MSE_BLOCKS 64

/* Floats of the activation buffer of a batch (the outputs of layers 1-3). */
size_t qtt_ws_act_floats(int batch);
/* Forward pass: in [batch][3][64][64] -> out [batch][1][64][64]; acts receives
 * the layer outputs (qtt_ws_act_floats(batch) floats). bf16 != 0 rounds weights
 * and layer inputs to BF16 (FP32 accumulation). batch 1..4096. */
int qtt_ws_forward(qtt_ctx* ctx, const float* params, const float* in, int batch, float* acts, float* out,
                   int bf16, void* stream);
/* Backward pass of the FP32 forward with the same params/in/acts: gout is
 * dL/d(out) ([batch][64][64], overwritten as scratch), grads (QTT_WS_NPARAMS
 * floats) receives dL/d(params) (overwritten, not accumulated), scratch holds
 * 2 * batch * 32 * 64 * 64 floats. Reductions run in a fixed order. */
int qtt_ws_backward(qtt_ctx* ctx, const float* params, const float* in, int batch, float* acts, float* gout,
                    float* grads, float* scratch, void* stream);
/* Mean squared error over n values: gout = 2 (out - target) / n; partial
 * (QTT_WS_MSE_BLOCKS floats) receives per-block sums of squared errors. */
int qtt_ws_mse(qtt_ctx* ctx, const float* out, const float* target, int n, float* gout, float* partial,
               void* stream);
/* Block average of a train of L >= 12 binary cores in interleaved order onto
 * the 64 x 64 grid (its last L - 12 cores contracted with [1/2, 1/2]): grid
 * (HOST, 4096 doubles) receives [row eta][column xi]. Synchronises the stream. */
int qtt_ws_coarse(qtt_ctx* ctx, const qtt_mps* x, double* grid, void* stream);
/* Network input of one right-hand side (the rule used by qtt_fractional_step and by
 * the training pairs alike): coarse_b (HOST, 4096 doubles, [eta][xi]) ->
 * in (HOST, 3 x 4096 floats) = (b / rms(b), Re / 200, alpha / 2); *rms = rms(b), the
 * scale of the network's output. QTT_ENUMERIC (in unwritten) if rms(b) is 0 or
 * not finite. */
int qtt_ws_input_host(const double* coarse_b, double re, double alpha, float* in, double* rms);
/* One Adam step (Kingma & Ba, beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected,
 * step >= 1) on QTT_WS_NPARAMS parameters; m and v are the moment buffers. */
int qtt_ws_adam_step(qtt_ctx* ctx, float* params, const float* grads, float* m, float* v, int step, float lr,
                     void* stream);

#ifdef __cplusplus
}
#endif

#endif /* QTT_H */
