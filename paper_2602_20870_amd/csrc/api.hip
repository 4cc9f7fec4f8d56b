// C ABI of the FGFRFT library: argument validation, buffer carving and dispatch.
#include "internal.h"
#include "batch.h"
#include <cmath>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <map>
#include <mutex>
#include <new>
#include <utility>

namespace fgfrft {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

fgfrft_status hip_fail(hipError_t e, const char* what) {
  set_error("%s failed: %s", what, hipGetErrorString(e));
  return FGFRFT_EHIP;
}

// Dynamic-LDS limits set so far, per (kernel, device): the attribute belongs to the device the
// call is made on, and a later plan may need more LDS than an earlier one (the per-tile
// gradient kernel's LDS grows with L), so the largest value set is kept and only ever raised.
static std::mutex g_lds_mu;
static std::map<std::pair<const void*, int>, int> g_lds_set;

hipError_t raise_lds_limit(const void* kern, int bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  try {   // nothing may unwind through the C ABI
    std::lock_guard<std::mutex> lock(g_lds_mu);
    int& cur = g_lds_set[std::make_pair(kern, dev)];
    if (cur >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) cur = bytes;
    return e;
  } catch (...) {
    return hipErrorOutOfMemory;
  }
}

static bool valid_sizes(int N, int L, int intype, int stacktype) {
  if (N < 1 || N > 32768) { set_error("N=%d outside [1, 32768]", N); return false; }
  if (L < 1 || L > 64) { set_error("L=%d outside [1, 64]", L); return false; }
  if (intype != FGFRFT_IN_C128 && intype != FGFRFT_IN_F64) { set_error("bad intype %d", intype); return false; }
  if (stacktype != FGFRFT_STACK_FP32 && stacktype != FGFRFT_STACK_BF16X2 && stacktype != FGFRFT_STACK_FP16X2) {
    set_error("bad stacktype %d", stacktype);
    return false;
  }
  return true;
}

static bool aligned(const void* p, size_t a) { return (uintptr_t)p % a == 0; }

static size_t stack_elem_bytes(bool cplx) { return cplx ? 8 : 4; }

static fgfrft_status check_alphas(const Plan* p, const double* alphas, int n_alpha) {
  if (!alphas || n_alpha < 1) { set_error("alphas is NULL or n_alpha=%d < 1", n_alpha); return FGFRFT_EINVAL; }
  for (int a = 0; a < n_alpha; ++a) {
    if (!isfinite(alphas[a]) || fabs(alphas[a]) >= (double)p->L) {
      set_error("alphas[%d]=%g: need |alpha| < L=%d", a, alphas[a], p->L);
      return FGFRFT_EALPHA;
    }
  }
  return FGFRFT_OK;
}

}  // namespace fgfrft

using namespace fgfrft;

extern "C" {

fgfrft_status fgfrft_plan_bytes(int N, int L, int intype, int stacktype, size_t* persistent, size_t* scratch) {
  if (!valid_sizes(N, L, intype, stacktype)) return FGFRFT_EINVAL;
  const bool cplx = intype == FGFRFT_IN_C128;
  const size_t NN = (size_t)N * N;
  if (persistent)
    *persistent = align_up((size_t)2 * L * NN * stack_elem_bytes(cplx), 256) + align_up(NN * (cplx ? 8 : 4), 256) +
                  (cplx ? 0 : align_up((size_t)N * kWCols * sizeof(float), 256));
  if (scratch) *scratch = plan_scratch_bytes(N, L, cplx);
  return FGFRFT_OK;
}

fgfrft_status fgfrft_plan(const void* F_dev, int N, int L, int intype, int stacktype, int form, double tau,
                          void* persistent_dev,
                          size_t persistent_bytes, void* scratch_dev, size_t scratch_bytes, void* stream,
                          fgfrft_plan_t* out) {
  if (!out) { set_error("out is NULL"); return FGFRFT_EINVAL; }
  *out = nullptr;
  size_t need_p = 0, need_s = 0;
  fgfrft_status rc = fgfrft_plan_bytes(N, L, intype, stacktype, &need_p, &need_s);
  if (rc) return rc;
  if (form != FGFRFT_FORM_SPLIT && form != FGFRFT_FORM_STANDARD) { set_error("bad form %d", form); return FGFRFT_EINVAL; }
  if (!F_dev || !persistent_dev || !scratch_dev) { set_error("NULL device pointer"); return FGFRFT_EINVAL; }
  if (!aligned(F_dev, 8) || !aligned(persistent_dev, 256) || !aligned(scratch_dev, 256)) {
    set_error("F_dev must be 8-byte, persistent_dev and scratch_dev 256-byte aligned");
    return FGFRFT_EINVAL;
  }
  if (persistent_bytes < need_p) { set_error("persistent buffer %zu < %zu bytes", persistent_bytes, need_p); return FGFRFT_ENOMEM; }
  if (scratch_bytes < need_s) { set_error("scratch buffer %zu < %zu bytes", scratch_bytes, need_s); return FGFRFT_ENOMEM; }
  if (!(tau > 0.0)) tau = 1e-6;
  Plan* p = new (std::nothrow) Plan();
  if (!p) { set_error("host allocation failed"); return FGFRFT_ENOMEM; }
  p->N = N;
  p->L = L;
  p->LP = L <= 32 ? 32 : 64;
  p->cplx = intype == FGFRFT_IN_C128;
  p->stacktype = stacktype;
  p->form = form;
  p->tau = tau;
  p->stack_elem_bytes = stack_elem_bytes(p->cplx);
  p->stack = persistent_dev;
  p->P = (char*)persistent_dev + align_up((size_t)2 * L * N * N * p->stack_elem_bytes, 256);
  if (!p->cplx) p->W = (float*)((char*)p->P + align_up((size_t)N * N * sizeof(float), 256));
  rc = plan_build(p, F_dev, tau, scratch_dev, scratch_bytes, (hipStream_t)stream);
  if (rc) { delete p; return rc; }
  *out = (fgfrft_plan_t)p;
  return FGFRFT_OK;
}

fgfrft_status fgfrft_plan_info(fgfrft_plan_t plan, int* r_minus1, double* unitarity_defect, double* drift,
                               double* stop_norm, double* last_pivot_norm, double* tau_used) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  if (r_minus1) *r_minus1 = p->r_minus1;
  if (unitarity_defect) *unitarity_defect = p->unitarity_defect;
  if (drift) *drift = p->drift;
  if (stop_norm) *stop_norm = p->stop_norm;
  if (last_pivot_norm) *last_pivot_norm = p->last_pivot_norm;
  if (tau_used) *tau_used = p->tau;
  return FGFRFT_OK;
}

fgfrft_status fgfrft_plan_buffers(fgfrft_plan_t plan, void** stack_dev, void** P_dev) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  if (stack_dev) *stack_dev = p->stack;
  if (P_dev) *P_dev = p->P;
  return FGFRFT_OK;
}

void fgfrft_destroy(fgfrft_plan_t plan) { delete (Plan*)plan; }

size_t fgfrft_update_workspace_bytes(fgfrft_plan_t plan, int n_alpha) {
  if (!plan || n_alpha < 1) return 0;
  return update_ws_bytes((const Plan*)plan, n_alpha);
}

fgfrft_status fgfrft_update(fgfrft_plan_t plan, const double* alphas, int n_alpha, void* Q_dev, void* ws_dev,
                            size_t ws_bytes, void* stream) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  fgfrft_status rc = check_alphas(p, alphas, n_alpha);
  if (rc) return rc;
  if (!Q_dev || !ws_dev) { set_error("NULL device pointer"); return FGFRFT_EINVAL; }
  if (!aligned(Q_dev, 8) || !aligned(ws_dev, 256)) { set_error("Q_dev must be 8-byte and ws_dev 256-byte aligned"); return FGFRFT_EINVAL; }
  const size_t need = update_ws_bytes(p, n_alpha);
  if (ws_bytes < need) { set_error("update workspace %zu < %zu bytes", ws_bytes, need); return FGFRFT_ENOMEM; }
  hipStream_t s = (hipStream_t)stream;
  FG_HIP(hipMemcpyAsync(ws_dev, alphas, (size_t)n_alpha * sizeof(double), hipMemcpyHostToDevice, s));
  return update_launch(p, (const double*)ws_dev, n_alpha, Q_dev, ws_dev, s);
}

fgfrft_status fgfrft_update_dev(fgfrft_plan_t plan, const double* alphas_dev, int n_alpha, void* Q_dev, void* ws_dev,
                                size_t ws_bytes, void* stream) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  if (!alphas_dev || n_alpha < 1) { set_error("alphas_dev is NULL or n_alpha=%d < 1", n_alpha); return FGFRFT_EINVAL; }
  if (!Q_dev || !ws_dev) { set_error("NULL device pointer"); return FGFRFT_EINVAL; }
  if (!aligned(alphas_dev, 8) || !aligned(Q_dev, 8) || !aligned(ws_dev, 256)) {
    set_error("alphas_dev, Q_dev must be 8-byte and ws_dev 256-byte aligned");
    return FGFRFT_EINVAL;
  }
  const size_t need = update_ws_bytes(p, n_alpha);
  if (ws_bytes < need) { set_error("update workspace %zu < %zu bytes", ws_bytes, need); return FGFRFT_ENOMEM; }
  return update_launch(p, alphas_dev, n_alpha, Q_dev, ws_dev, (hipStream_t)stream);
}

size_t fgfrft_apply_operator_workspace_bytes(int N, int n_alpha, int B, int x_shared) {
  if (N < 1 || n_alpha < 1 || B < 1) return 0;
  return apply_ws_bytes(N, n_alpha, B, x_shared);
}

fgfrft_status fgfrft_apply_operator(const void* Q_dev, int N, int n_alpha, int adjoint, const void* X_dev, int x_complex,
                                    int x_shared, int B, void* Y_dev, int y_real, void* ws_dev, size_t ws_bytes,
                                    void* stream) {
  if (N < 1 || N > 32768 || n_alpha < 1 || B < 1 || B > 4096) {
    set_error("bad sizes N=%d n_alpha=%d B=%d", N, n_alpha, B);
    return FGFRFT_EINVAL;
  }
  if (!Q_dev || !X_dev || !Y_dev || !ws_dev) { set_error("NULL device pointer"); return FGFRFT_EINVAL; }
  if (!aligned(Q_dev, 16) || !aligned(X_dev, 8) || !aligned(Y_dev, 8) || !aligned(ws_dev, 256)) {
    set_error("Q_dev must be 16-byte, X_dev, Y_dev 8-byte and ws_dev 256-byte aligned");
    return FGFRFT_EINVAL;
  }
  const size_t need = apply_ws_bytes(N, n_alpha, B, x_shared);
  if (ws_bytes < need) { set_error("apply workspace %zu < %zu bytes", ws_bytes, need); return FGFRFT_ENOMEM; }
  return apply_launch(Q_dev, N, n_alpha, adjoint ? 1 : 0, X_dev, x_complex ? 1 : 0, x_shared ? 1 : 0, B, Y_dev,
                      y_real ? 1 : 0, ws_dev, (hipStream_t)stream);
}

// Orders per update launch of fgfrft_apply.  Every launch reads the whole stack, so the default takes as
// many orders as fit about 4 GiB of operators (at least 16, at most 256).
static int apply_chunk(const Plan* p, bool realF, int n_alpha, int chunk) {
  if (chunk <= 0) {
    const size_t per = (size_t)p->N * p->N * (realF ? 4 : 8);
    const size_t fit = ((size_t)4 << 30) / per;
    chunk = fit < 16 ? 16 : (fit > 256 ? 256 : (int)fit);
  }
  return chunk < n_alpha ? chunk : n_alpha;
}

size_t fgfrft_apply_workspace_bytes(fgfrft_plan_t plan, int n_alpha, int B, int x_complex, int x_shared, int chunk) {
  if (!plan || n_alpha < 1 || B < 1) return 0;
  const Plan* p = (const Plan*)plan;
  const int ch = apply_chunk(p, apply_real_supported(p, x_complex, B), n_alpha, chunk);
  if (apply_real_supported(p, x_complex, B))   // real F, real X: R = Re Q (4 bytes per entry)
    return align_up((size_t)n_alpha * 8, 256) + align_up((size_t)ch * p->N * p->N * 4, 256) + update_ws_bytes(p, ch) +
           apply_real_ws_bytes(p->N, ch, B, x_shared, p->r_minus1);
  return align_up((size_t)n_alpha * 8, 256) + align_up((size_t)ch * p->N * p->N * 8, 256) + update_ws_bytes(p, ch) +
         apply_ws_bytes(p->N, ch, B, x_shared);
}

fgfrft_status fgfrft_apply(fgfrft_plan_t plan, const double* alphas, int n_alpha, const void* X_dev, int x_complex,
                           int x_shared, int B, void* Y_dev, int chunk, void* ws_dev, size_t ws_bytes, void* stream) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  fgfrft_status rc = check_alphas(p, alphas, n_alpha);
  if (rc) return rc;
  if (B < 1 || B > 4096) { set_error("B=%d outside [1, 4096]", B); return FGFRFT_EINVAL; }
  if (!X_dev || !Y_dev || !ws_dev) { set_error("NULL device pointer"); return FGFRFT_EINVAL; }
  if ((uintptr_t)X_dev % 8 || (uintptr_t)Y_dev % 8 || (uintptr_t)ws_dev % 256) {
    set_error("X_dev, Y_dev must be 8-byte and ws_dev 256-byte aligned");
    return FGFRFT_EINVAL;
  }
  const int ch = apply_chunk(p, apply_real_supported(p, x_complex, B), n_alpha, chunk);
  const size_t need = fgfrft_apply_workspace_bytes(plan, n_alpha, B, x_complex, x_shared, chunk);
  if (ws_bytes < need) { set_error("apply workspace %zu < %zu bytes", ws_bytes, need); return FGFRFT_ENOMEM; }
  // real F and real signals: the update writes R = Re Q only and the apply adds the imaginary part
  // sin(pi alpha) P X from P's rank-r factor (same operator, half the operator bytes)
  const bool realF = apply_real_supported(p, x_complex, B);
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws_dev;
  double* al = (double*)base; base += align_up((size_t)n_alpha * 8, 256);
  void* Qc = base; base += align_up((size_t)ch * p->N * p->N * (realF ? 4 : 8), 256);
  void* uws = base; base += update_ws_bytes(p, ch);
  void* aws = base;
  FG_HIP(hipMemcpyAsync(al, alphas, (size_t)n_alpha * 8, hipMemcpyHostToDevice, s));
  const size_t NB = (size_t)p->N * B;
  for (int a0 = 0; a0 < n_alpha; a0 += ch) {
    const int nc = n_alpha - a0 < ch ? n_alpha - a0 : ch;
    if ((rc = update_launch(p, al + a0, nc, Qc, uws, s, realF))) return rc;
    const void* xa = x_shared ? X_dev : (const void*)((const char*)X_dev + a0 * NB * (x_complex ? 8 : 4));
    void* ya = (char*)Y_dev + a0 * NB * 8;
    if (realF) rc = apply_real_launch(p, (const float*)Qc, nc, al + a0, (const float*)xa, x_shared ? 1 : 0, B,
                                      (cplx64*)ya, aws, s);
    else rc = apply_launch(Qc, p->N, nc, 0, xa, x_complex ? 1 : 0, x_shared ? 1 : 0, B, ya, 0, aws, s);
    if (rc) return rc;
  }
  return FGFRFT_OK;
}

size_t fgfrft_apply_dev_workspace_bytes(fgfrft_plan_t plan, int n_alpha, int B, int x_complex, int x_shared) {
  if (!plan || n_alpha < 1 || B < 1) return 0;
  const Plan* p = (const Plan*)plan;
  const bool realF = apply_real_supported(p, x_complex, B);
  return align_up((size_t)n_alpha * p->N * p->N * (realF ? 4 : 8), 256) + update_ws_bytes(p, n_alpha) +
         (realF ? apply_real_ws_bytes(p->N, n_alpha, B, x_shared, p->r_minus1) : apply_ws_bytes(p->N, n_alpha, B, x_shared));
}

fgfrft_status fgfrft_apply_dev(fgfrft_plan_t plan, const double* alphas_dev, int n_alpha, const void* X_dev,
                               int x_complex, int x_shared, int B, void* Y_dev, void* ws_dev, size_t ws_bytes,
                               void* stream) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  if (!alphas_dev || n_alpha < 1) { set_error("alphas_dev is NULL or n_alpha=%d < 1", n_alpha); return FGFRFT_EINVAL; }
  if (B < 1 || B > 4096) { set_error("B=%d outside [1, 4096]", B); return FGFRFT_EINVAL; }
  if (!X_dev || !Y_dev || !ws_dev) { set_error("NULL device pointer"); return FGFRFT_EINVAL; }
  if (!aligned(alphas_dev, 8) || !aligned(X_dev, 8) || !aligned(Y_dev, 8) || !aligned(ws_dev, 256)) {
    set_error("alphas_dev, X_dev, Y_dev must be 8-byte and ws_dev 256-byte aligned");
    return FGFRFT_EINVAL;
  }
  const size_t need = fgfrft_apply_dev_workspace_bytes(plan, n_alpha, B, x_complex, x_shared);
  if (ws_bytes < need) { set_error("apply workspace %zu < %zu bytes", ws_bytes, need); return FGFRFT_ENOMEM; }
  const bool realF = apply_real_supported(p, x_complex, B);
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws_dev;
  void* Qc = base; base += align_up((size_t)n_alpha * p->N * p->N * (realF ? 4 : 8), 256);
  void* uws = base; base += update_ws_bytes(p, n_alpha);
  void* aws = base;
  fgfrft_status rc = update_launch(p, alphas_dev, n_alpha, Qc, uws, s, realF);
  if (rc) return rc;
  if (realF)
    return apply_real_launch(p, (const float*)Qc, n_alpha, alphas_dev, (const float*)X_dev, x_shared ? 1 : 0, B,
                             (cplx64*)Y_dev, aws, s);
  return apply_launch(Qc, p->N, n_alpha, 0, X_dev, x_complex ? 1 : 0, x_shared ? 1 : 0, B, Y_dev, 0, aws, s);
}

size_t fgfrft_apply_direct_workspace_bytes(fgfrft_plan_t plan, int ncols, int ldx) {
  if (!plan || ncols < 0 || ldx < 1 || ldx > (1 << 20)) return 0;
  return direct_ws_bytes((const Plan*)plan, ncols, ldx);
}

fgfrft_status fgfrft_apply_direct(fgfrft_plan_t plan, const double* alphas_dev, int n_alpha, const int* col_order_dev,
                                  const void* X_dev, int x_complex, int ncols, int ldx, void* Y_dev, int ldy,
                                  void* ws_dev, size_t ws_bytes, void* stream) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  if (n_alpha < 1 || ncols < 0 || ldx < 1 || ldy < 1 || ncols > ldx || ncols > ldy || ldx > (1 << 20) ||
      ldy > (1 << 20)) {
    set_error("bad sizes n_alpha=%d ncols=%d ldx=%d ldy=%d", n_alpha, ncols, ldx, ldy);
    return FGFRFT_EINVAL;
  }
  if (ncols == 0) return FGFRFT_OK;
  if (!alphas_dev || !col_order_dev || !X_dev || !Y_dev || !ws_dev) { set_error("NULL device pointer"); return FGFRFT_EINVAL; }
  if ((uintptr_t)X_dev % (x_complex ? 8 : 4) || (uintptr_t)Y_dev % 8 || (uintptr_t)ws_dev % 256 ||
      (uintptr_t)alphas_dev % 8 || (uintptr_t)col_order_dev % 4) {
    set_error("misaligned device pointer (X: element, Y: 8 bytes, ws: 256 bytes)");
    return FGFRFT_EINVAL;
  }
  const size_t need = direct_ws_bytes(p, ncols, ldx);
  if (ws_bytes < need) { set_error("direct workspace %zu < %zu bytes", ws_bytes, need); return FGFRFT_ENOMEM; }
  return direct_launch(p, alphas_dev, n_alpha, col_order_dev, X_dev, x_complex ? 1 : 0, ncols, ldx, Y_dev, ldy, ws_dev,
                       (hipStream_t)stream);
}

size_t fgfrft_apply_batched_workspace_bytes(fgfrft_plan_t plan, int n_req, const int* B_per_req, int x_complex) {
  if (!plan || n_req < 1 || !B_per_req) return 0;
  for (int r = 0; r < n_req; ++r)
    if (B_per_req[r] < 0 || B_per_req[r] > 4096) return 0;
  return batched_ws_bytes((const Plan*)plan, n_req, B_per_req, x_complex ? 1 : 0);
}

fgfrft_status fgfrft_apply_batched(fgfrft_plan_t plan, const double* alphas, int n_req, const int* B_per_req,
                                   const void* const* X_dev, int x_complex, void* const* Y_dev, void* ws_dev,
                                   size_t ws_bytes, void* stream) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  fgfrft_status rc = check_alphas(p, alphas, n_req);
  if (rc) return rc;
  if (!B_per_req || !X_dev || !Y_dev || !ws_dev) { set_error("NULL pointer"); return FGFRFT_EINVAL; }
  if (!aligned(ws_dev, 256)) { set_error("ws_dev must be 256-byte aligned"); return FGFRFT_EINVAL; }
  const size_t xe = x_complex ? 8 : 4;
  for (int r = 0; r < n_req; ++r) {
    if (B_per_req[r] < 0 || B_per_req[r] > 4096) {
      set_error("B_per_req[%d]=%d outside [0, 4096]", r, B_per_req[r]);
      return FGFRFT_EINVAL;
    }
    if (B_per_req[r] == 0) continue;
    if (!X_dev[r] || !Y_dev[r]) { set_error("request %d: NULL signal or output pointer", r); return FGFRFT_EINVAL; }
    if (!aligned(X_dev[r], xe) || !aligned(Y_dev[r], 8)) {
      set_error("request %d: signals must be element-aligned and outputs 8-byte aligned", r);
      return FGFRFT_EINVAL;
    }
  }
  const size_t need = batched_ws_bytes(p, n_req, B_per_req, x_complex ? 1 : 0);
  if (ws_bytes < need) { set_error("batched workspace %zu < %zu bytes", ws_bytes, need); return FGFRFT_ENOMEM; }
  return batched_launch(p, alphas, n_req, B_per_req, X_dev, x_complex ? 1 : 0, Y_dev, ws_dev, (hipStream_t)stream);
}

size_t fgfrft_grad_workspace_bytes(fgfrft_plan_t plan, int n_alpha, int B, int x_shared) {
  if (!plan || n_alpha < 1 || B < 1) return 0;
  return grad_ws_bytes((const Plan*)plan, n_alpha, B, x_shared);
}

fgfrft_status fgfrft_grad(fgfrft_plan_t plan, const double* alphas, int n_alpha, const void* X_dev, int x_complex,
                          int x_shared, int B, const void* GY_dev, double* dalpha, void* dX_dev, void* ws_dev,
                          size_t ws_bytes, void* stream) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  fgfrft_status rc = check_alphas(p, alphas, n_alpha);
  if (rc) return rc;
  if (B < 1 || B > 4096) { set_error("B=%d outside [1, 4096]", B); return FGFRFT_EINVAL; }
  if (!X_dev || !GY_dev || !dalpha || !ws_dev) { set_error("NULL pointer"); return FGFRFT_EINVAL; }
  const size_t xe = x_complex ? 8 : 4;
  if (!aligned(X_dev, xe) || !aligned(GY_dev, 8) || !aligned(dX_dev, xe) || !aligned(ws_dev, 256)) {
    set_error("X_dev, dX_dev must be element-aligned, GY_dev 8-byte and ws_dev 256-byte aligned");
    return FGFRFT_EINVAL;
  }
  if (p->stacktype == FGFRFT_STACK_BF16X2) { set_error("grad needs an FP32 or FP16X2 power stack"); return FGFRFT_EUNSUPPORTED; }
  try {   // host tables of the order loop: an allocation failure must not unwind through the C ABI
    return grad_run(p, alphas, n_alpha, X_dev, x_complex ? 1 : 0, x_shared ? 1 : 0, B, GY_dev, dalpha, dX_dev,
                    ws_dev, ws_bytes, (hipStream_t)stream);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return FGFRFT_ENOMEM;
  }
}

const char* fgfrft_strerror(int status) {
  switch (status) {
    case FGFRFT_OK: return "ok";
    case FGFRFT_EINVAL: return "invalid argument";
    case FGFRFT_ENOTUNITARY: return "F is not unitary";
    case FGFRFT_EALPHA: return "order out of range (need |alpha| < L)";
    case FGFRFT_ENOMEM: return "buffer too small";
    case FGFRFT_EHIP: return "HIP runtime error";
    case FGFRFT_EDRIFT: return "power recurrence drift";
    case FGFRFT_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

const char* fgfrft_last_error(void) { return g_err; }

size_t fgfrft_gfrft_exact_workspace_bytes(int N) {
  if (N < 1 || N > 32768) return 0;
  return align_up((size_t)N * N * 16, 256);
}

fgfrft_status fgfrft_gfrft_exact(const void* V_dev, const void* Vh_dev, const double* theta_dev, int N, double alpha,
                                 void* out_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  if (N < 1 || N > 32768) { set_error("N=%d outside [1, 32768]", N); return FGFRFT_EINVAL; }
  if (!std::isfinite(alpha)) { set_error("alpha is not finite"); return FGFRFT_EALPHA; }
  if (!V_dev || !Vh_dev || !theta_dev || !out_dev || !ws_dev) { set_error("NULL pointer"); return FGFRFT_EINVAL; }
  if (!aligned(V_dev, 8) || !aligned(Vh_dev, 8) || !aligned(theta_dev, 8) || !aligned(out_dev, 8) ||
      !aligned(ws_dev, 256)) {
    set_error("V_dev, Vh_dev, theta_dev, out_dev must be 8-byte and ws_dev 256-byte aligned");
    return FGFRFT_EINVAL;
  }
  if (ws_bytes < fgfrft_gfrft_exact_workspace_bytes(N)) {
    set_error("workspace %zu < %zu bytes", ws_bytes, fgfrft_gfrft_exact_workspace_bytes(N));
    return FGFRFT_ENOMEM;
  }
  return gfrft_exact_run(V_dev, Vh_dev, theta_dev, N, alpha, out_dev, ws_dev, (hipStream_t)stream);
}

}  // extern "C"
