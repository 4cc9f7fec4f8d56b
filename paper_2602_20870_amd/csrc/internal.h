// Internal declarations shared by the FGFRFT HIP sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include "../../include/fgfrft.h"

namespace fgfrft {

// ---------------------------------------------------------------- vector types
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef short shortx8 __attribute__((ext_vector_type(8)));

struct cplx64 { float re, im; };
struct cplx128 { double re, im; };

// Fixed power-of-two scales for the split 16-bit operands.  Power-stack and
// projector entries, coefficients and operator entries are bounded by ~1.1 in
// magnitude (entries of contractions of unitary matrices, |c_n| <= 1), so a
// factor 2^12 keeps every fp16 value normal and far from overflow.
constexpr float kStackScale = 4096.0f;
constexpr float kCoefScale = 4096.0f;
constexpr float kUnscale = 1.0f / (4096.0f * 4096.0f);

// ---------------------------------------------------------------- device helpers
// Fourier coefficient of Sec. III-A: c_n(alpha) = sinc(alpha - n) = sin(pi x) / (pi x), limit 1 at x = 0
// (FP64, sinpi is exact at integers so integer orders give Kronecker deltas).
__device__ __forceinline__ double sinc_pi(double x) { return x == 0.0 ? 1.0 : sinpi(x) / (M_PI * x); }

typedef __attribute__((address_space(3))) char lds_char;
__device__ __forceinline__ uint32_t lds_addr(const char* p) { return (uint32_t)(size_t)(const lds_char*)p; }

// s_waitcnt immediate (gfx9 encoding): vmcnt <= v and lgkmcnt == 0, expcnt not waited on
__host__ __device__ constexpr int wait_vm_lgkm0(int v) { return (v & 15) | ((v >> 4) << 14) | (7 << 4); }

// One 16-byte direct HBM-to-LDS load per lane (LDS destination: lds_base + 16 * lane).  Written
// out here rather than through the builtin so the compiler does not add its own "wait for every
// direct load" before each LDS read: a multi-stage ring waits explicitly for exactly the stage
// it reads.  The instruction has no register result; hardware reads the address at issue.  Callers
// wait for these loads with explicit s_waitcnt (vmcnt) before reading the LDS they fill.
__device__ __forceinline__ void lds_dma16(const void* g, uint32_t lds_base) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(lds_base), "v"(g)
               : "memory", "m0");
}

// Workgroup barrier without a memory fence: the waits it needs are explicit at the call site
// (a fence here would also wait for every direct LDS load still in flight, i.e. for the whole
// ring).  The signal fences keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void barrier_nofence() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// ---------------------------------------------------------------- plan object
struct Plan {
  int N = 0, L = 0, LP = 0;        // LP: L padded to a multiple of 32 (MFMA k extent)
  int cplx = 0;                    // 1: complex F, complex power stack
  int stacktype = 0;               // fgfrft_stacktype
  int form = 0;                    // fgfrft_form
  int r_minus1 = 0;
  double unitarity_defect = 0, drift = 0, stop_norm = 0, last_pivot_norm = 0, tau = 1e-6;
  void* stack = nullptr;           // [L][N][N] elements (4 B real / 8 B complex)
  void* P = nullptr;               // [N][N] float (real) or cplx64 (complex)
  float* W = nullptr;              // real F: [N][kWCols] float, P = W W^T (columns >= r_minus1 zero)
  int w_ok = 0;                    // 1: W holds the -1 eigenspace basis (real F, r_minus1 <= kWCols)
  size_t stack_elem_bytes = 0;
};

// Real F keeps an orthonormal basis W of the -1 eigenspace (P = W W^T) as float32, row-major
// [N][kWCols], when r_minus1 <= kWCols: the real-F apply forms P X = W (W^T X) from it.
constexpr int kWCols = 32;

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
fgfrft_status hip_fail(hipError_t e, const char* what);
// Raises a kernel's dynamic-LDS limit to at least `bytes` on the current device (a no-op when an
// earlier call on that device already set as much).  Safe to call from several host threads.
hipError_t raise_lds_limit(const void* kern, int bytes);
#define FG_HIP(call)                                              \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) return ::fgfrft::hip_fail(e_, #call);   \
  } while (0)
#define FG_LAUNCHED(what)                                         \
  do {                                                            \
    hipError_t e_ = hipGetLastError();                            \
    if (e_ != hipSuccess) return ::fgfrft::hip_fail(e_, what);    \
  } while (0)

static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- kernel entry points
// FP64 plan side (plan_f64.hip)
fgfrft_status gemm_f64(bool cplx, bool conj_a, int M, int Ncols, int K, const void* A, int lda,
                       const void* B, int ldb, void* C, int ldc, hipStream_t s);
fgfrft_status plan_build(Plan* p, const void* F, double tau, void* scratch, size_t scratch_bytes,
                         hipStream_t s);
size_t plan_scratch_bytes(int N, int L, bool cplx);
fgfrft_status gfrft_exact_run(const void* V, const void* Vh, const double* theta, int N, double alpha, void* out,
                              void* ws, hipStream_t s);

// Online side (update.hip)
size_t update_ws_bytes(const Plan* p, int n_alpha);
// real_plane (real F only): write R = Re Q as float32 [n_alpha][N][N] instead of complex64 Q.
fgfrft_status update_launch(const Plan* p, const double* alphas_dev, int n_alpha, void* Q,
                            void* ws, hipStream_t s, bool real_plane = false);
fgfrft_status coef_launch(const Plan* p, const double* alphas_dev, int n_alpha, int n_alpha_pad,
                          void* table, float4* epi, int deriv, hipStream_t s);

// Apply (apply.hip)
size_t apply_ws_bytes(int N, int n_alpha, int B, int x_shared);
// per-column power-of-two scales of X [nx][N][B] (max |x| s in [2^13, 2^14)), scale[(a, b)] = (s, 1/s);
// partial: nx * ceil(N / 64) * B floats of scratch
size_t colscale_partial_bytes(int N, int nx, int B);
fgfrft_status colscale_launch(const void* X, int x_complex, int N, int B, int nx, float2* scale, float* partial,
                              hipStream_t s);
// its first pass alone: partial[a][chunk][b] = max |X[a][i][b]| over the chunk's 64 rows
fgfrft_status colmax_launch(const void* X, int x_complex, int N, int B, int nx, float* partial, hipStream_t s);

// Signals split once for the matrix cores (apply.hip): real X [nx][N][ldx] (order stride xstride
// floats, 0 = one block for all), columns scaled by xs[a * xs_stride + col].x, written as
// Xs[a][cb][chunk][ks][c][part][lane][8] fp16 (64-column blocks, 32-wide k chunks, N % 32 == 0;
// columns >= ncols are zero; bf16 = true: bf16 hi / lo parts): xsplit_bytes(N, nx, ncols) bytes.
size_t xsplit_bytes(int N, int nx, int ncols);
fgfrft_status xsplit_launch(const float* X, int ldx, int ncols, int N, int nx, size_t xstride, const float2* xs,
                            int xs_stride, short* Xs, hipStream_t s, bool bf16 = false);

// Direct route (direct.hip)
size_t direct_ws_bytes(const Plan* p, int ncols, int ldx);
fgfrft_status direct_launch(const Plan* p, const double* alphas_dev, int n_alpha, const int* col_order_dev,
                            const void* X, int x_complex, int ncols, int ldx, void* Y, int ldy, void* ws,
                            hipStream_t s);
fgfrft_status apply_launch(const void* Q, int N, int n_alpha, int adjoint, const void* X, int x_complex,
                           int x_shared, int B, void* Y, int y_real, void* ws, hipStream_t s);

// Real-F apply (apply.hip): Y[a] = R[a] X[a] + j sin(pi alpha_a) W (W^T X[a]) with R = Re Q float32
// [n_alpha][N][N] from update_launch(..., real_plane = true); real X, N % 32 == 0, B % 64 == 0.
size_t apply_real_ws_bytes(int N, int n_alpha, int B, int x_shared, int r);
bool apply_real_supported(const Plan* p, int x_complex, int B);
fgfrft_status apply_real_launch(const Plan* p, const float* R, int n_alpha, const double* alphas_dev, const float* X,
                                int x_shared, int B, cplx64* Y, void* ws, hipStream_t s);
// Signal gradient through the real-F form (apply.hip): dX[a] = Re(Q(alphas[a]) GY[a]) = R[a] Re GY[a] -
// sin(pi alphas[a]) W (W^T Im GY[a]) as float32 [n_alpha][N][B], with R = Re Q(alphas[a]) from
// update_launch(..., real_plane = true); the same shape conditions as apply_real_supported.
size_t apply_real_dx_ws_bytes(int N, int n_alpha, int B, int r);
fgfrft_status apply_real_dx_launch(const Plan* p, const float* R, int n_alpha, const double* alphas_dev,
                                   const cplx64* GY, int B, float* dX, void* ws, hipStream_t s);

// Gradient (grad.hip)
size_t grad_ws_bytes(const Plan* p, int n_alpha, int B, int x_shared);
fgfrft_status grad_run(const Plan* p, const double* alphas_host, int n_alpha, const void* X, int x_complex,
                       int x_shared, int B, const void* GY, double* dalpha, void* dX, void* ws,
                       size_t ws_bytes, hipStream_t s);

}  // namespace fgfrft
