/*
 * fgfrft.h -- C ABI of the MI355X (gfx950) FGFRFT library.
 *
 * FGFRFT (arXiv 2602.20870) approximates the graph fractional Fourier
 * transform F^alpha of a unitary GFT matrix F by the L-order operator of
 * Definition 1,
 *
 *     Q_L^alpha = e^{j pi alpha} P + sum_{n=-L}^{L} c_n(alpha) F^n P_c,
 *     c_n(alpha) = sin(pi (alpha - n)) / (pi (alpha - n)),
 *
 * where P projects onto the eigenvalue -1 eigenspace of F and P_c = I - P
 * (Sec. III-B).  Algorithm 1 splits the work into an offline stage (the
 * projector and the powers M_n = F^n P_c) and an online stage (the linear
 * combination for each new order alpha); negative powers are conjugate
 * transposes, F^{-n} P_c = M_n^H (Proposition 2).
 *
 * Conventions for every call
 *   - Matrices are dense, row-major and contiguous.  Complex values are
 *     interleaved {re, im} pairs (the layout of complex64 / complex128).
 *   - Pointers named *_dev are HIP device memory owned by the caller; the
 *     library never allocates or frees device memory.  Pointers without the
 *     suffix are host memory.
 *   - Alignment: every device pointer is aligned to its element type (4 bytes
 *     for float32 and int32; 8 for float64, complex64 and complex128); every
 *     workspace (ws_dev) and the plan's persistent and scratch buffers are
 *     256-byte aligned.  Two calls need more: Q_dev of fgfrft_apply_operator
 *     16 bytes, and X_dev and Y_dev of fgfrft_apply and fgfrft_apply_operator
 *     8 bytes, also for float32 data.  hipMalloc and the torch caching
 *     allocator return blocks aligned to 256 bytes or more; a misaligned
 *     pointer is an argument error (FGFRFT_EINVAL).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Every call only enqueues work on it, except fgfrft_plan and
 *     fgfrft_grad, which synchronise it (they read results back to the host).
 *   - Argument errors are detected on the host before anything is enqueued
 *     and returned synchronously; nothing is written in that case.  A HIP
 *     launch failure returns FGFRFT_EHIP.  fgfrft_last_error() gives a
 *     thread-local description of the most recent failure.
 *   - A plan is read-only after fgfrft_plan returns: update, apply and grad
 *     may run concurrently on different streams provided each call has its
 *     own workspace.
 */
#ifndef FGFRFT_H
#define FGFRFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGFRFT_API __attribute__((visibility("default")))

typedef enum {
  FGFRFT_OK = 0,
  FGFRFT_EINVAL = -1,        /* bad size, pointer, type or workspace too small            */
  FGFRFT_ENOTUNITARY = -2,   /* max |F^H F - I| above 1e-10                                */
  FGFRFT_EALPHA = -3,        /* |alpha| >= L, or alpha not finite                          */
  FGFRFT_ENOMEM = -4,        /* caller-provided buffer smaller than the stated size        */
  FGFRFT_EHIP = -5,          /* a HIP runtime call or kernel launch failed                 */
  FGFRFT_EDRIFT = -6,        /* FP64 power recurrence lost orthogonality (||M_n^H M_n - P_c||_F / sqrt(N) > 1e-9) */
  FGFRFT_EUNSUPPORTED = -7   /* combination of sizes the library does not implement        */
} fgfrft_status;

/* Element type of F as handed to fgfrft_plan. */
typedef enum {
  FGFRFT_IN_C128 = 0,        /* complex128 F: complex power stack                          */
  FGFRFT_IN_F64 = 1          /* float64 F (real orthogonal): real power stack, Im Q = sin(pi alpha) P */
} fgfrft_intype;

/* Storage of the resident power stack (M_1..M_L and M_1^H..M_L^H). */
typedef enum {
  FGFRFT_STACK_FP32 = 0,     /* float32 (real F) or complex64 (complex F)                  */
  FGFRFT_STACK_BF16X2 = 1,   /* per real value a bf16 pair (hi, lo = bf16(x - hi)), 4 bytes */
  FGFRFT_STACK_FP16X2 = 2    /* per real value the fp16 pair of v = float(x) 2^12 (hi = fp16(v),
                                lo = fp16(v - hi)), 4 bytes: the operands the FP32 stack is
                                split into on the matrix cores, stored split, so every call
                                gives bitwise the FP32 stack's results without the split work */
} fgfrft_stacktype;

/* Which operator the plan's online stage produces. */
typedef enum {
  FGFRFT_FORM_SPLIT = 0,     /* Definition 1: the -1 eigenspace is split off (P), powers act on P_c */
  FGFRFT_FORM_STANDARD = 1   /* the plain truncated series sum_{n=-L}^{L} c_n(alpha) F^n without the
                                split (P = 0, M_0 = I): the ablation of Sec. IV-F / Table VI */
} fgfrft_form;

typedef struct fgfrft_plan_s* fgfrft_plan_t;

/* ---------------------------------------------------------------------------
 * Offline stage (Algorithm 1, offline part; Sec. III-G complexity)
 * ------------------------------------------------------------------------- */

/* Bytes of device memory a plan needs.  `persistent` must stay allocated for
 * the plan's lifetime (power stack, projector and, for real F, an N x 32
 * float32 slot for the -1 eigenspace basis); `scratch` is FP64
 * working memory used only during fgfrft_plan and free again when it returns.
 * Limits: 1 <= N <= 32768, 1 <= L <= 64. */
FGFRFT_API fgfrft_status fgfrft_plan_bytes(int N, int L, int intype, int stacktype,
                                           size_t* persistent, size_t* scratch);

/* Build a plan for the unitary F (N x N, row-major, device, float64 or
 * complex128 per `intype`) and the operator `form` (fgfrft_form).  On the GPU,
 * in FP64 (steps 2 and 3 only for FGFRFT_FORM_SPLIT; the standard form takes
 * P = 0, M_0 = I and reports r_minus1 = 0):
 *   1. unitarity check max|F^H F - I| <= 1e-10, else FGFRFT_ENOTUNITARY;
 *   2. the eigenvalue -1 eigenspace as the null space of F + I, found by
 *      Householder QR with column pivoting of F + I; the pivoted QR stops
 *      when every remaining column norm is <= tau (tau <= 0 selects 1e-6),
 *      and the trailing columns of the orthogonal factor give an orthonormal
 *      W with P = W W^H (F is normal, so null(F + I) is the complement of
 *      the range of F + I);
 *   3. M_0 = P_c = I - P, M_n = F M_{n-1} for n = 1..L, with the drift
 *      ||M_n^H M_n - P_c||_F / sqrt(N) checked at n = ceil(L/2) and n = L;
 *   4. M_1..M_L, their adjoints M_1^H..M_L^H (= F^{-n} P_c, Proposition 2)
 *      and P stored in `stacktype` format in `persistent_dev`; for real F
 *      with r_minus1 <= 32 also W as float32 (used by fgfrft_apply).
 * Synchronises `stream`.  F_dev is only read during the call.
 * On success *out receives a host-side handle (free with fgfrft_destroy);
 * persistent_dev must outlive it. */
FGFRFT_API fgfrft_status fgfrft_plan(const void* F_dev, int N, int L, int intype, int stacktype,
                                     int form, double tau, void* persistent_dev, size_t persistent_bytes,
                                     void* scratch_dev, size_t scratch_bytes, void* stream,
                                     fgfrft_plan_t* out);

/* Facts measured while planning: rank of the -1 eigenspace, max|F^H F - I|,
 * the larger of the two drift values, the largest remaining column norm of
 * F + I when the pivoted QR stopped (0 if r_minus1 = 0), the smallest
 * column norm it pivoted on (how close the nearest non-(-1) eigenvalue is)
 * and the threshold tau the QR stopped at (1e-6 when the plan was given
 * tau <= 0).  Any pointer may be NULL. */
FGFRFT_API fgfrft_status fgfrft_plan_info(fgfrft_plan_t plan, int* r_minus1, double* unitarity_defect,
                                          double* drift, double* stop_norm, double* last_pivot_norm,
                                          double* tau_used);

/* Device pointers to the resident data: stack (2L matrices of N*N elements of
 * the stack format: slot n-1 holds M_n, slot L+n-1 holds M_n^H, n = 1..L) and
 * P (N*N, float32 for real F, complex64 for complex F).  For inspection and tests. */
FGFRFT_API fgfrft_status fgfrft_plan_buffers(fgfrft_plan_t plan, void** stack_dev, void** P_dev);

FGFRFT_API void fgfrft_destroy(fgfrft_plan_t plan);  /* frees the host handle only */

/* ---------------------------------------------------------------------------
 * Online stage: operator update (Definition 1, Proposition 2, Algorithm 1
 * online part)
 * ------------------------------------------------------------------------- */

/* Workspace bytes for fgfrft_update with n_alpha orders. */
FGFRFT_API size_t fgfrft_update_workspace_bytes(fgfrft_plan_t plan, int n_alpha);

/* Q[a] = Q_L^{alphas[a]} for a = 0..n_alpha-1, written as complex64
 * [n_alpha][N][N] to Q_dev.  `alphas` is a host array (copied before the call
 * returns); each |alpha| < L, else FGFRFT_EALPHA.  Integer alpha goes through
 * the same formula, which then reduces to F^alpha (Remark on integer order).
 * The coefficients c_n(alpha), c_0, cos(pi alpha) and sin(pi alpha) are
 * evaluated on the GPU in FP64 (a-1), then every power-stack tile is read once
 * from HBM for all n_alpha orders and combined on the matrix cores with FP32
 * accumulation. */
FGFRFT_API fgfrft_status fgfrft_update(fgfrft_plan_t plan, const double* alphas, int n_alpha,
                                       void* Q_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* The same update with the orders already in device memory (float64 [n_alpha], e.g.
 * written by an earlier copy on the same stream).  Nothing is read back to the host,
 * so the call may be recorded by stream capture (hipGraph) and replayed with new order
 * values.  Orders cannot be range-checked on the host here: a plane whose order has
 * |alpha| >= L or is not finite is filled with NaN.  Workspace as for fgfrft_update. */
FGFRFT_API fgfrft_status fgfrft_update_dev(fgfrft_plan_t plan, const double* alphas_dev, int n_alpha,
                                           void* Q_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* The same update as fgfrft_update_dev for callers that cannot allocate (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): no workspace
 * argument, and the call allocates nothing.  Its coefficient and epilogue tables live in a
 * fixed 2.25 MiB device array inside the library, one copy per GPU, held until the process
 * ends; its device address is looked up once per device, on the first call made with that
 * device current.  1 <= n_alpha <= 4096, else FGFRFT_EINVAL.  Q_dev and alphas_dev as for
 * fgfrft_update_dev (8-byte aligned; out-of-range orders give NaN planes).  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (different streams or host
 * threads with work in flight at the same time) race on it and must be serialised by the
 * caller; calls in order on one stream are safe, since each call rewrites every table entry
 * it reads. */
FGFRFT_API fgfrft_status fgfrft_update_dev_static(fgfrft_plan_t plan, const double* alphas_dev, int n_alpha,
                                                  void* Q_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Apply to graph signals (Definition 2)
 * ------------------------------------------------------------------------- */

/* Workspace bytes for fgfrft_apply_operator: the per-signal scale table and its partial maxima and,
 * for real signals taken by the streaming kernel with pre-split signals, the signals split into
 * fp16 hi / lo parts (4 bytes per signal value). */
FGFRFT_API size_t fgfrft_apply_operator_workspace_bytes(int N, int n_alpha, int B, int x_shared);

/* Y[a] = op(Q[a]) X[a] for a = 0..n_alpha-1 with op = identity (adjoint = 0)
 * or the conjugate transpose (adjoint = 1; by Proposition 3 this is the
 * operator of order -alpha).  Q_dev: complex64 [n_alpha][N][N].
 * X_dev: [n_alpha][N][B] (x_shared = 0) or one [N][B] block for every order
 * (x_shared = 1), float32 (x_complex = 0) or complex64 (x_complex = 1).
 * Y_dev: complex64 [n_alpha][N][B], or float32 holding only the real part
 * when y_real = 1.  1 <= B <= 4096.  Q_dev 16-byte, X_dev and Y_dev 8-byte aligned. */
FGFRFT_API fgfrft_status fgfrft_apply_operator(const void* Q_dev, int N, int n_alpha, int adjoint,
                                               const void* X_dev, int x_complex, int x_shared, int B,
                                               void* Y_dev, int y_real, void* ws_dev, size_t ws_bytes,
                                               void* stream);

/* Workspace bytes for fgfrft_apply: operators for `chunk` orders at a time
 * plus the update and apply workspaces.  chunk <= 0 selects min(n_alpha, c) with c the number of
 * orders whose operators fit about 4 GiB (N^2 * 8 bytes each, N^2 * 4 on the real-F route),
 * clamped to [16, 256]: every update launch reads the whole stack, so fewer, larger launches.
 * Depends on x_complex: the real-F route below keeps 4 bytes per operator
 * entry instead of 8. */
FGFRFT_API size_t fgfrft_apply_workspace_bytes(fgfrft_plan_t plan, int n_alpha, int B, int x_complex,
                                               int x_shared, int chunk);

/* Y[a] = Q_L^{alphas[a]} X[a] (Definition 2): the operator update into the
 * workspace, `chunk` orders at a time, then the apply.  Same layouts as
 * fgfrft_apply_operator with y_real = 0.
 * Real-F route: for a real F (FGFRFT_IN_F64) the powers and P are real, so
 * Definition 1 splits as Q = R + j sin(pi alpha) P with R = Re Q real, and
 * P = W W^T with W an orthonormal basis of the -1 eigenspace.  When F is
 * real, X is real, N % 32 == 0, B % 64 == 0 and r_minus1 <= 32 (the plan
 * keeps W as float32 then), the update writes only R (float32, half the
 * bytes of Q) and the apply computes Y = R X + j sin(pi alpha) W (W^T X),
 * the rank-r term from the signals' projections.  Every other case forms the
 * complex64 Q and calls fgfrft_apply_operator's kernels. */
FGFRFT_API fgfrft_status fgfrft_apply(fgfrft_plan_t plan, const double* alphas, int n_alpha,
                                      const void* X_dev, int x_complex, int x_shared, int B,
                                      void* Y_dev, int chunk, void* ws_dev, size_t ws_bytes,
                                      void* stream);

/* Workspace bytes for fgfrft_apply_dev: the operators of all n_alpha orders (float32 R on the
 * real-F route, complex64 Q otherwise) plus the update and apply workspaces.  0 for a NULL plan
 * or n_alpha < 1 or B < 1. */
FGFRFT_API size_t fgfrft_apply_dev_workspace_bytes(fgfrft_plan_t plan, int n_alpha, int B, int x_complex,
                                                   int x_shared);

/* fgfrft_apply with the orders already on the device (alphas_dev: float64 [n_alpha], 8-byte
 * aligned) and all of them in one update launch: Y[a] = Q_L^{alphas_dev[a]} X[a] (Definition 2),
 * by the real-F route under the same conditions as fgfrft_apply, else through the complex64
 * operator.  Same layouts as fgfrft_apply.  The call only enqueues kernels on `stream` (no host
 * copy or synchronisation; capturable).  Orders are device data and are not range-checked: an
 * order with |alpha| >= L or a non-finite one gives NaN outputs for its signals. */
FGFRFT_API fgfrft_status fgfrft_apply_dev(fgfrft_plan_t plan, const double* alphas_dev, int n_alpha,
                                          const void* X_dev, int x_complex, int x_shared, int B, void* Y_dev,
                                          void* ws_dev, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Direct route: apply without forming any operator (Definition 2 with the
 * expansion of Definition 1 and Proposition 2)
 * ------------------------------------------------------------------------- */

/* Workspace bytes for fgfrft_apply_direct (column scales, coefficient table,
 * per-term-group partial sums). */
FGFRFT_API size_t fgfrft_apply_direct_workspace_bytes(fgfrft_plan_t plan, int ncols, int ldx);

/* Y[:, c] = Q_L^{alpha(c)} X[:, c] for c = 0..ncols-1, where column c has the order
 * alpha(c) = alphas_dev[col_order_dev[c]], computed from the resident stack as
 *   Y = c_0 X + (e^{j pi alpha} - c_0) P X + sum_{n=1}^{L} ( c_n M_n X + c_{-n} M_n^H X )
 * (P_c = I - P folded into the first two terms; the standard form has P = 0).  No N x N
 * operator is written or read: the stack is streamed once per 64 columns, so this route
 * wins when the signals of a batch are few compared with its orders (it moves
 * (2L+1) N^2 stack elements instead of 16 N^2 operator bytes per order).
 *   alphas_dev: float64 [n_alpha] device; col_order_dev: int32 [ncols] device, each in
 *   [0, n_alpha); X_dev: [N][ldx] row-major, float32 (x_complex = 0) or complex64
 *   (x_complex = 1); Y_dev: complex64 [N][ldy].  ncols <= ldx, ncols <= ldy.
 * Orders are device data and are not range-checked on the host: a column whose order
 * index is out of range, or whose order has |alpha| >= L or is not finite, is filled
 * with NaN.  Real F, real X and N % 32 == 0 take the matrix-core kernel (FP32 stack:
 * split fp16 operands; BF16X2 stack: its bf16 pairs with bf16-split signals; FP32
 * products of each term folded into FP64 sums); every other case takes a plain
 * FP64-accumulating kernel.  The call only enqueues work on `stream` (no host
 * synchronisation; capturable). */
FGFRFT_API fgfrft_status fgfrft_apply_direct(fgfrft_plan_t plan, const double* alphas_dev, int n_alpha,
                                             const int* col_order_dev, const void* X_dev, int x_complex,
                                             int ncols, int ldx, void* Y_dev, int ldy, void* ws_dev,
                                             size_t ws_bytes, void* stream);

/* Workspace bytes for fgfrft_apply_batched (per group of up to 64 requests: the gathered signals,
 * the results, the column map and the direct route's workspace; the largest group counts).
 * Returns 0 for a NULL plan or table, n_req < 1, or a signal count outside [0, 4096]. */
FGFRFT_API size_t fgfrft_apply_batched_workspace_bytes(fgfrft_plan_t plan, int n_req, const int* B_per_req,
                                                       int x_complex);

/* Grouped apply for serving (Definition 2, one order per request): request r gets
 *   Y_dev[r] = Q_L^{alphas[r]} X_dev[r]
 * for r = 0..n_req-1, each request with its own order and its own number of signals.
 *   alphas: host float64 [n_req], each finite with |alpha| < L (else FGFRFT_EALPHA, nothing
 *   enqueued); B_per_req: host int32 [n_req], each in [0, 4096] (0: the request is skipped);
 *   X_dev, Y_dev: host arrays of n_req device pointers; X_dev[r]: [N][B_per_req[r]] row-major,
 *   float32 (x_complex = 0) or complex64 (x_complex = 1), element-aligned; Y_dev[r]: complex64
 *   [N][B_per_req[r]], 8-byte aligned, not overlapping any X_dev.
 * The requests are taken in groups of 64: per group the signals are gathered into one column
 * block of the workspace, the direct route of fgfrft_apply_direct runs once over it (each column
 * with its request's order; the stack is streamed once per 64 columns), and the results are
 * scattered to Y_dev.  The request tables travel as kernel arguments, so nothing is copied from
 * the host: the call only enqueues work on `stream` and can be captured in a graph (the host
 * arrays are read during the call only).  Accuracy as fgfrft_apply_direct. */
FGFRFT_API fgfrft_status fgfrft_apply_batched(fgfrft_plan_t plan, const double* alphas, int n_req,
                                              const int* B_per_req, const void* const* X_dev, int x_complex,
                                              void* const* Y_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Gradients (Proposition 4)
 * ------------------------------------------------------------------------- */

/* Workspace bytes for fgfrft_grad. */
FGFRFT_API size_t fgfrft_grad_workspace_bytes(fgfrft_plan_t plan, int n_alpha, int B, int x_shared);

/* Gradients of a real loss l through Y[a] = Q_L^{alphas[a]} X[a].
 * GY_dev: complex64 [n_alpha][N][B] holding dl/dRe Y + j dl/dIm Y.
 *   dalpha[a] = Re sum_{n=-L}^{L} c_n'(alpha_a) <G_a, F^n P_c>
 *             + Re( j pi e^{j pi alpha_a} <G_a, P> ),
 *   with G_a = GY[a] X[a]^H and <A, B> = sum_ij conj(A_ij) B_ij;
 * dalpha is a host array of n_alpha doubles, written after the stream has
 * been synchronised.  G_a is formed on the GPU in FP32; the inner products
 * with the stack accumulate in FP64 per tile and are summed over tiles in a
 * fixed order (deterministic); the final combination with c_n'(alpha) is FP64.
 * dX_dev (may be NULL): Q(alpha_a)^H GY[a], float32 (real part) when
 * x_complex = 0, complex64 otherwise, shaped like X (summed over orders when
 * x_shared = 1). */
FGFRFT_API fgfrft_status fgfrft_grad(fgfrft_plan_t plan, const double* alphas, int n_alpha,
                                     const void* X_dev, int x_complex, int x_shared, int B,
                                     const void* GY_dev, double* dalpha, void* dX_dev,
                                     void* ws_dev, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Exact GFRFT online stage (the comparison method, Sec. II / Table IV)
 * ------------------------------------------------------------------------- */

/* Workspace bytes for fgfrft_gfrft_exact: one N x N complex128 matrix. */
FGFRFT_API size_t fgfrft_gfrft_exact_workspace_bytes(int N);

/* F^alpha = V diag(e^{j alpha theta}) V^H from a cached eigendecomposition of the unitary F
 * (the offline eigendecomposition is the caller's; the paper also excludes it from its online
 * timings).  V_dev and Vh_dev = V^H: complex128 N x N row-major; theta_dev: float64 [N] phases
 * in (-pi, pi]; out_dev: complex128 N x N.  FP64 throughout: the columns of V are scaled by
 * e^{j alpha theta_k} (FP64 sin/cos), then one complex FP64 GEMM on the matrix cores
 * (8 N^3 flops).  Any finite alpha.  1 <= N <= 32768. */
FGFRFT_API fgfrft_status fgfrft_gfrft_exact(const void* V_dev, const void* Vh_dev, const double* theta_dev, int N,
                                            double alpha, void* out_dev, void* ws_dev, size_t ws_bytes,
                                            void* stream);

/* ---------------------------------------------------------------------------
 * Measurement helper (not part of the method)
 * ------------------------------------------------------------------------- */

/* Writes `bytes` zero bytes to dst_dev with 16-byte nontemporal stores from a
 * grid-stride streaming kernel: the write bandwidth this device attains, the
 * ceiling for the store-dominated operator update.  dst_dev 16-byte aligned,
 * bytes a nonzero multiple of 16, else FGFRFT_EINVAL.  Enqueues on `stream`. */
FGFRFT_API fgfrft_status fgfrft_probe_write(void* dst_dev, size_t bytes, void* stream);

/* The operator update's HBM traffic with no arithmetic, for N % 64 == 0: per strip of 4 rows x
 * 64 positions (64 <= N <= 32704), stages the strip's tiles of n_tiles row-major N x N matrices of 4-byte values at
 * src_dev (n_tiles N^2 4 bytes, device, 16-byte aligned; the update stages its 2L stack matrices
 * and the projector) in LDS, then writes those positions of n_alpha complex64 N x N planes at
 * dst_dev (n_alpha N^2 8 bytes, device) in the update's store pattern (512-byte row runs, orders
 * in sequence).  The values written are meaningless.  1 <= n_tiles <= 65, n_alpha >= 1, else
 * FGFRFT_EINVAL.  Enqueues on `stream`. */
FGFRFT_API fgfrft_status fgfrft_probe_update_traffic(const void* src_dev, int N, int n_tiles, int n_alpha,
                                                     void* dst_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Errors
 * ------------------------------------------------------------------------- */
FGFRFT_API const char* fgfrft_strerror(int status);
FGFRFT_API const char* fgfrft_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FGFRFT_H */
