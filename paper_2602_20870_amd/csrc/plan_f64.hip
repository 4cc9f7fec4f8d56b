// Offline stage of Algorithm 1 on the GPU, in FP64:
//   unitarity check, eigenvalue -1 eigenspace of F (pivoted Householder QR of F + I),
//   projector P = W W^H, power recurrence M_n = F M_{n-1} with drift checks,
//   and conversion of M_1..M_L, their adjoints M_1^H..M_L^H and P to the resident format.
#include "internal.h"
#include <math.h>
#include <stdio.h>
#include <vector>

namespace fgfrft {

// ============================================================================
// complex helpers (real instantiation ignores the imaginary part)
// ============================================================================
struct cd { double re, im; };
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.re, -a.im}; }
__device__ __forceinline__ double cabs2(cd a) { return a.re * a.re + a.im * a.im; }

template <bool C> __device__ __forceinline__ cd ldz(const double* p, size_t i) {
  if (C) return {p[2 * i], p[2 * i + 1]};
  return {p[i], 0.0};
}
template <bool C> __device__ __forceinline__ void stz(double* p, size_t i, cd v) {
  if (C) { p[2 * i] = v.re; p[2 * i + 1] = v.im; }
  else p[i] = v.re;
}

// ============================================================================
// FP64 GEMM on the matrix cores: C = op(A) B, row-major, op = identity or ^H.
// 64x64 output tile per workgroup (4 waves, 32x32 each = 2x2 MFMA 16x16x4 tiles),
// k-chunks of 16 staged through LDS.
//   MFMA f64 16x16x4 operand layout: A lane l -> A[l%16][l/16], B lane l -> B[l/16][l%16],
//   result register r of lane l -> C[4r + l/16][l%16].
// ============================================================================
constexpr int GB = 64, GK = 16;

template <bool CPLX, bool CONJ_A>
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, int K, const double* __restrict__ A, int lda,
                                                  const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                  int ldc) {
  __shared__ double As_re[GK][GB + 1], Bs_re[GK][GB + 1];
  __shared__ double As_im[CPLX ? GK : 1][GB + 1], Bs_im[CPLX ? GK : 1][GB + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * GB, n0 = blockIdx.x * GB;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  doublex4 acc_re[2][2], acc_im[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      acc_re[i][j] = doublex4{0, 0, 0, 0};
      acc_im[i][j] = doublex4{0, 0, 0, 0};
    }

  for (int k0 = 0; k0 < K; k0 += GK) {
    // ---- stage op(A)[m0:m0+64, k0:k0+16] as As[k][m]
    if (!CONJ_A) {
      const int m = t >> 2, kq = (t & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + m, gk = k0 + kq + q;
        cd v = {0.0, 0.0};
        if (gm < M && gk < K) v = ldz<CPLX>(A, (size_t)gm * lda + gk);
        As_re[kq + q][m] = v.re;
        if (CPLX) As_im[kq + q][m] = v.im;
      }
    } else {
      const int k = t >> 4, mq = (t & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + mq + q, gk = k0 + k;
        cd v = {0.0, 0.0};
        if (gm < M && gk < K) v = cconj(ldz<CPLX>(A, (size_t)gk * lda + gm));
        As_re[k][mq + q] = v.re;
        if (CPLX) As_im[k][mq + q] = v.im;
      }
    }
    // ---- stage B[k0:k0+16, n0:n0+64] as Bs[k][n]
    {
      const int k = t >> 4, nq = (t & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gn = n0 + nq + q, gk = k0 + k;
        cd v = {0.0, 0.0};
        if (gn < N && gk < K) v = ldz<CPLX>(B, (size_t)gk * ldb + gn);
        Bs_re[k][nq + q] = v.re;
        if (CPLX) Bs_im[k][nq + q] = v.im;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int kr = kk + (lane >> 4), c16 = lane & 15;
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = As_re[kr][wm + i * 16 + c16];
        br[i] = Bs_re[kr][wn + i * 16 + c16];
        if (CPLX) {
          ai[i] = As_im[kr][wm + i * 16 + c16];
          bi[i] = Bs_im[kr][wn + i * 16 + c16];
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], acc_re[i][j], 0, 0, 0);
          if (CPLX) {
            acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi[j], acc_re[i][j], 0, 0, 0);
            acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], acc_im[i][j], 0, 0, 0);
            acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], acc_im[i][j], 0, 0, 0);
          }
        }
    }
    __syncthreads();
  }
  // ---- write back
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + 4 * r + (lane >> 4);
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) stz<CPLX>(C, (size_t)gm * ldc + gn, cd{acc_re[i][j][r], CPLX ? acc_im[i][j][r] : 0.0});
      }
}

fgfrft_status gemm_f64(bool cplx, bool conj_a, int M, int Nc, int K, const void* A, int lda, const void* B, int ldb,
                       void* C, int ldc, hipStream_t s) {
  dim3 grid(ceil_div(Nc, GB), ceil_div(M, GB)), block(256);
  const double* a = (const double*)A;
  const double* b = (const double*)B;
  double* c = (double*)C;
  if (cplx) {
    if (conj_a) k_gemm_f64<true, true><<<grid, block, 0, s>>>(M, Nc, K, a, lda, b, ldb, c, ldc);
    else k_gemm_f64<true, false><<<grid, block, 0, s>>>(M, Nc, K, a, lda, b, ldb, c, ldc);
  } else {
    if (conj_a) k_gemm_f64<false, true><<<grid, block, 0, s>>>(M, Nc, K, a, lda, b, ldb, c, ldc);
    else k_gemm_f64<false, false><<<grid, block, 0, s>>>(M, Nc, K, a, lda, b, ldb, c, ldc);
  }
  FG_LAUNCHED("gemm_f64");
  return FGFRFT_OK;
}

// ============================================================================
// Deterministic two-pass reductions over an N x N row-major matrix G:
//   mode 0: max_ij |G_ij - delta_ij|                         (unitarity defect)
//   mode 1: sum_ij |G_ij - (delta_ij - P_ij)|^2              (drift against P_c)
// ============================================================================
template <bool C>
__global__ __launch_bounds__(256) void k_reduce_partial(const double* __restrict__ G, const double* __restrict__ P,
                                                        int N, int mode, double* __restrict__ partial) {
  __shared__ double sh[256];
  const size_t total = (size_t)N * N;
  double acc = 0.0;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const size_t i = idx / N, j = idx % N;
    cd g = ldz<C>(G, idx);
    if (mode == 0) {
      if (i == j) g.re -= 1.0;
      acc = fmax(acc, sqrt(cabs2(g)));
    } else {
      cd p = ldz<C>(P, idx);
      const double d = (i == j) ? 1.0 : 0.0;
      cd e = {g.re - (d - p.re), g.im + p.im};
      acc += cabs2(e);
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] = mode == 0 ? fmax(sh[threadIdx.x], sh[threadIdx.x + st]) : sh[threadIdx.x] + sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ partial, int n, int mode,
                                                      double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc = mode == 0 ? fmax(acc, partial[i]) : acc + partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] = mode == 0 ? fmax(sh[threadIdx.x], sh[threadIdx.x + st]) : sh[threadIdx.x] + sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// ============================================================================
// Householder QR with column pivoting of A = F + I (column-major), stopped when
// every remaining column norm is <= tol.  Each step: one single-workgroup
// kernel picks the pivot, swaps it in and forms the reflector; a second kernel
// applies the reflector to the trailing columns and recomputes their norms.
// Steps after the stop see state->done and return at once, so the host loop
// needs no synchronisation.
// ============================================================================
struct QRState {
  int done;          // 1 once the stop test passed
  int k;             // number of reflectors (rank of F + I)
  double stop_norm;  // max remaining column norm at the stop
  double last_pivot; // norm of the last pivot column accepted
};

template <bool C>
__global__ __launch_bounds__(256) void k_plus_identity_colmajor(const double* __restrict__ F, int N, double* __restrict__ A) {
  const size_t total = (size_t)N * N;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const size_t i = idx / N, j = idx % N;  // F row-major (i, j)
    cd v = ldz<C>(F, idx);
    if (i == j) v.re += 1.0;
    stz<C>(A, j * (size_t)N + i, v);
  }
}

template <bool C>
__global__ __launch_bounds__(256) void k_colnorms(const double* __restrict__ A, int N, double* __restrict__ cn2) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= N) return;
  double s = 0.0;
  for (int i = lane; i < N; i += 64) s += cabs2(ldz<C>(A, (size_t)c * N + i));
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) cn2[c] = s;
}

template <bool C>
__global__ __launch_bounds__(1024) void k_qr_pivot_house(double* __restrict__ A, int N, int j, double* __restrict__ cn2,
                                                         double* __restrict__ tau, QRState* __restrict__ st,
                                                         double tol2) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  __shared__ int s_piv, s_stop;
  __shared__ double s_red[1024];
  const int t = threadIdx.x;
  if (st->done) return;
  // ---- pivot: largest remaining column norm (first index on ties)
  double best = -1.0;
  int bi = N;
  for (int c = j + t; c < N; c += 1024) {
    const double v = cn2[c];
    if (v > best) { best = v; bi = c; }
  }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s) {
      const double a = sv[t], b = sv[t + s];
      if (b > a || (b == a && si[t + s] < si[t])) { sv[t] = b; si[t] = si[t + s]; }
    }
    __syncthreads();
  }
  if (t == 0) {
    s_piv = si[0];
    s_stop = sv[0] <= tol2;
    if (s_stop) {
      st->done = 1;
      st->k = j;
      st->stop_norm = sqrt(fmax(sv[0], 0.0));
    } else {
      st->last_pivot = sqrt(sv[0]);
    }
  }
  __syncthreads();
  if (s_stop) return;
  const int p = s_piv;
  // ---- swap columns j and p; each thread owns rows i = t (mod 1024) throughout
  if (p != j) {
    for (int i = t; i < N; i += 1024) {
      cd a = ldz<C>(A, (size_t)j * N + i), b = ldz<C>(A, (size_t)p * N + i);
      stz<C>(A, (size_t)j * N + i, b);
      stz<C>(A, (size_t)p * N + i, a);
    }
    if (t == 0) { const double x = cn2[j]; cn2[j] = cn2[p]; cn2[p] = x; }
  }
  // ---- reflector for x = A[j:, j]: H^H x = beta e_1 with H = I - tau v v^H, v_0 = 1
  double part = 0.0;
  for (int i = t; i < N; i += 1024)
    if (i > j) part += cabs2(ldz<C>(A, (size_t)j * N + i));
  s_red[t] = part;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s) s_red[t] += s_red[t + s];
    __syncthreads();
  }
  const double xnorm2 = s_red[0];
  // the row-j element is owned by thread (j % 1024)
  __shared__ cd s_x0;
  if (t == (j & 1023)) s_x0 = ldz<C>(A, (size_t)j * N + j);
  __syncthreads();
  const cd x0 = s_x0;
  if (xnorm2 == 0.0 && x0.im == 0.0) {
    if (t == 0) { tau[2 * j] = 0.0; tau[2 * j + 1] = 0.0; }
    return;
  }
  const double beta = -copysign(sqrt(cabs2(x0) + xnorm2), x0.re);
  const cd tv = {(beta - x0.re) / beta, -x0.im / beta};
  const cd d = {x0.re - beta, x0.im};
  const double dd = cabs2(d);
  const cd scale = {d.re / dd, -d.im / dd};
  for (int i = t; i < N; i += 1024) {
    if (i <= j) continue;
    const size_t idx = (size_t)j * N + i;
    stz<C>(A, idx, cmul(ldz<C>(A, idx), scale));
  }
  if (t == (j & 1023)) stz<C>(A, (size_t)j * N + j, cd{beta, 0.0});
  if (t == 0) { tau[2 * j] = tv.re; tau[2 * j + 1] = tv.im; }
}

// Apply H_j^H = I - conj(tau_j) v v^H to columns c > j (one wave per column) and
// recompute their norms over rows j+1..N-1.
template <bool C>
__global__ __launch_bounds__(256) void k_qr_update(double* __restrict__ A, int N, int j, double* __restrict__ cn2,
                                                   const double* __restrict__ tau, const QRState* __restrict__ st) {
  if (st->done) return;
  const int lane = threadIdx.x & 63;
  const int c = j + 1 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= N) return;
  const cd tj = {tau[2 * j], tau[2 * j + 1]};
  if (tj.re == 0.0 && tj.im == 0.0) {
    double s = 0.0;
    for (int i = j + 1 + lane; i < N; i += 64) s += cabs2(ldz<C>(A, (size_t)c * N + i));
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) cn2[c] = s;
    return;
  }
  cd w = {0.0, 0.0};
  for (int i = j + lane; i < N; i += 64) {
    const cd v = (i == j) ? cd{1.0, 0.0} : ldz<C>(A, (size_t)j * N + i);
    const cd a = ldz<C>(A, (size_t)c * N + i);
    const cd pr = cmul(cconj(v), a);
    w.re += pr.re;
    w.im += pr.im;
  }
  for (int off = 32; off > 0; off >>= 1) {
    w.re += __shfl_xor(w.re, off);
    w.im += __shfl_xor(w.im, off);
  }
  const cd f = cmul(cconj(tj), w);
  double s = 0.0;
  for (int i = j + lane; i < N; i += 64) {
    const cd v = (i == j) ? cd{1.0, 0.0} : ldz<C>(A, (size_t)j * N + i);
    const size_t idx = (size_t)c * N + i;
    cd a = ldz<C>(A, idx);
    const cd u = cmul(f, v);
    a.re -= u.re;
    a.im -= u.im;
    stz<C>(A, idx, a);
    if (i > j) s += cabs2(a);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) cn2[c] = s;
}

// W[:, t] = H_0 H_1 ... H_{k-1} e_{k+t}: the last r columns of the orthogonal factor,
// an orthonormal basis of range(F + I)^perp = null(F + I) (F normal).  W column-major N x r.
template <bool C>
__global__ __launch_bounds__(256) void k_form_W(const double* __restrict__ A, int N, int k,
                                                const double* __restrict__ tau, double* __restrict__ W) {
  __shared__ double red_re[256], red_im[256];
  const int t = threadIdx.x, col = blockIdx.x;
  double* w = W + (C ? 2 : 1) * (size_t)col * N;
  for (int i = t; i < N; i += 256) stz<C>(w, i, cd{i == k + col ? 1.0 : 0.0, 0.0});
  for (int j = k - 1; j >= 0; --j) {
    const cd tj = {tau[2 * j], tau[2 * j + 1]};
    cd part = {0.0, 0.0};
    for (int i = t; i < N; i += 256) {  // rows stay owned by one thread across steps
      if (i < j) continue;
      const cd v = (i == j) ? cd{1.0, 0.0} : ldz<C>(A, (size_t)j * N + i);
      const cd pr = cmul(cconj(v), ldz<C>(w, i));
      part.re += pr.re;
      part.im += pr.im;
    }
    red_re[t] = part.re;
    red_im[t] = part.im;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) { red_re[t] += red_re[t + s]; red_im[t] += red_im[t + s]; }
      __syncthreads();
    }
    const cd f = cmul(tj, cd{red_re[0], red_im[0]});
    __syncthreads();
    for (int i = t; i < N; i += 256) {
      if (i < j) continue;
      const cd v = (i == j) ? cd{1.0, 0.0} : ldz<C>(A, (size_t)j * N + i);
      cd x = ldz<C>(w, i);
      const cd u = cmul(f, v);
      x.re -= u.re;
      x.im -= u.im;
      stz<C>(w, i, x);
    }
  }
}

// P = W W^H (row-major N x N) and Mprev = P_c = I - P.
template <bool C>
__global__ __launch_bounds__(256) void k_projector(const double* __restrict__ W, int N, int r, double* __restrict__ P,
                                                   double* __restrict__ Pc) {
  const size_t total = (size_t)N * N;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const size_t i = idx / N, j = idx % N;
    cd s = {0.0, 0.0};
    for (int q = 0; q < r; ++q) {
      const cd a = ldz<C>(W, (size_t)q * N + i), b = ldz<C>(W, (size_t)q * N + j);
      const cd pr = cmul(a, cconj(b));
      s.re += pr.re;
      s.im += pr.im;
    }
    stz<C>(P, idx, s);
    stz<C>(Pc, idx, cd{(i == j ? 1.0 : 0.0) - s.re, -s.im});
  }
}

// FP64 (row-major) -> resident format.  kind 0: float (real) / cplx64 (complex);
// kind 1: bf16 pair per real value (hi = bf16(x), lo = bf16(x - hi)), packed hi | lo << 16;
// kind 2: fp16 pair per real value of v = float(x) 2^12 (hi = fp16(v), lo = fp16(v - hi)), packed
// hi | lo << 16 -- exactly the operands the FP32 stack is split into when it is read.
__device__ __forceinline__ uint32_t bf16_pair(double x) {
  const float xf = (float)x;
  const __bf16 hi = (__bf16)xf;
  const __bf16 lo = (__bf16)(xf - (float)hi);
  return (uint32_t)__builtin_bit_cast(uint16_t, hi) | ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
}
__device__ __forceinline__ uint32_t fp16_pair(double x) {
  const float v = (float)x * kStackScale;
  const _Float16 hi = (_Float16)v;
  const _Float16 lo = (_Float16)(v - (float)hi);
  return (uint32_t)__builtin_bit_cast(uint16_t, hi) | ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
}
__device__ __forceinline__ uint32_t pair_of(double x, int kind) { return kind == 1 ? bf16_pair(x) : fp16_pair(x); }

template <bool C>
__global__ __launch_bounds__(256) void k_store(const double* __restrict__ M, size_t total, int kind, void* __restrict__ out) {
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const cd v = ldz<C>(M, idx);
    if (kind == 0) {
      if (C) ((cplx64*)out)[idx] = cplx64{(float)v.re, (float)v.im};
      else ((float*)out)[idx] = (float)v.re;
    } else {
      if (C) ((uint2*)out)[idx] = make_uint2(pair_of(v.re, kind), pair_of(v.im, kind));
      else ((uint32_t*)out)[idx] = pair_of(v.re, kind);
    }
  }
}

// Real F: the -1 eigenspace basis (column-major FP64 N x r) as float32 row-major [N][kWCols],
// columns r..kWCols-1 zero.
__global__ __launch_bounds__(256) void k_store_W(const double* __restrict__ W, int N, int r, float* __restrict__ out) {
  const size_t total = (size_t)N * kWCols;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const int i = (int)(idx / kWCols), q = (int)(idx % kWCols);
    out[idx] = q < r ? (float)W[(size_t)q * N + i] : 0.f;
  }
}

// out = conj(M)^T in the resident format (the negative powers F^{-n} P_c = M_n^H of
// Proposition 2), through 32x32 LDS tiles so both the FP64 read and the store are coalesced.
template <bool C>
__global__ __launch_bounds__(256) void k_store_adjoint(const double* __restrict__ M, int N, int kind, void* __restrict__ out) {
  __shared__ double tr[32][33], ti[32][33];
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = bi + r, j = bj + tx;
    cd v = {0.0, 0.0};
    if (i < N && j < N) v = ldz<C>(M, (size_t)i * N + j);
    tr[r][tx] = v.re;
    ti[r][tx] = v.im;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bj + r, j = bi + tx;   // out[i][j] = conj(M[j][i])
    if (i >= N || j >= N) continue;
    const size_t idx = (size_t)i * N + j;
    const double re = tr[tx][r], im = -ti[tx][r];
    if (kind == 0) {
      if (C) ((cplx64*)out)[idx] = cplx64{(float)re, (float)im};
      else ((float*)out)[idx] = (float)re;
    } else {
      if (C) ((uint2*)out)[idx] = make_uint2(pair_of(re, kind), pair_of(im, kind));
      else ((uint32_t*)out)[idx] = pair_of(re, kind);
    }
  }
}

// ============================================================================
// host orchestration
// ============================================================================
size_t plan_scratch_bytes(int N, int L, bool cplx) {
  (void)L;
  const size_t es = cplx ? 16 : 8;
  const size_t mat = align_up((size_t)N * N * es, 256);
  return 4 * mat + align_up((size_t)N * 8, 256) /*cn2*/ + align_up((size_t)N * 16, 256) /*tau*/ +
         align_up(sizeof(QRState), 256) + align_up(4096 * 8, 256) /*partials*/ + 256;
}

static fgfrft_status reduce(bool C, const double* G, const double* P, int N, int mode, double* partial,
                            double* out_dev, double* out_host, hipStream_t s) {
  const int nb = 4096;
  if (C) k_reduce_partial<true><<<nb, 256, 0, s>>>(G, P, N, mode, partial);
  else k_reduce_partial<false><<<nb, 256, 0, s>>>(G, P, N, mode, partial);
  FG_LAUNCHED("reduce_partial");
  k_reduce_final<<<1, 256, 0, s>>>(partial, nb, mode, out_dev);
  FG_LAUNCHED("reduce_final");
  FG_HIP(hipMemcpyAsync(out_host, out_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  FG_HIP(hipStreamSynchronize(s));
  return FGFRFT_OK;
}

static int grid_for(size_t total) {
  size_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

// ---- exact GFRFT online stage: W = V diag(e^{j alpha theta}), F^alpha = W V^H
__global__ __launch_bounds__(256) void k_phase_columns(const double* __restrict__ V, const double* __restrict__ theta,
                                                       int N, double alpha, double* __restrict__ W) {
  const size_t total = (size_t)N * N;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const int k = (int)(e % N);
    double sn, cs;
    sincos(alpha * theta[k], &sn, &cs);
    const double vr = V[2 * e], vi = V[2 * e + 1];
    W[2 * e] = vr * cs - vi * sn;
    W[2 * e + 1] = vr * sn + vi * cs;
  }
}

fgfrft_status gfrft_exact_run(const void* V, const void* Vh, const double* theta, int N, double alpha, void* out,
                              void* ws, hipStream_t s) {
  const size_t total = (size_t)N * N;
  k_phase_columns<<<grid_for(total), 256, 0, s>>>((const double*)V, theta, N, alpha, (double*)ws);
  FG_LAUNCHED("phase_columns");
  return gemm_f64(true, false, N, N, N, ws, N, Vh, N, out, N, s);
}

fgfrft_status plan_build(Plan* p, const void* F, double tau, void* scratch, size_t scratch_bytes, hipStream_t s) {
  const int N = p->N, L = p->L;
  const bool C = p->cplx != 0;
  const size_t es = C ? 16 : 8;
  const size_t mat = align_up((size_t)N * N * es, 256);
  if (scratch_bytes < plan_scratch_bytes(N, L, C)) {
    set_error("scratch buffer too small: %zu < %zu", scratch_bytes, plan_scratch_bytes(N, L, C));
    return FGFRFT_ENOMEM;
  }
  char* base = (char*)scratch;
  double* Abuf = (double*)base; base += mat;   // QR workspace, also G for the checks
  double* P64 = (double*)base; base += mat;
  double* Mprev = (double*)base; base += mat;
  double* Mcur = (double*)base; base += mat;   // also W before the recurrence
  double* cn2 = (double*)base; base += align_up((size_t)N * 8, 256);
  double* taub = (double*)base; base += align_up((size_t)N * 16, 256);
  QRState* st = (QRState*)base; base += align_up(sizeof(QRState), 256);
  double* partial = (double*)base; base += align_up(4096 * 8, 256);
  double* scal = (double*)base;
  const double* Fd = (const double*)F;
  const size_t total = (size_t)N * N;

  // ---- 1. unitarity: max |F^H F - I|
  fgfrft_status rc = gemm_f64(C, true, N, N, N, Fd, N, Fd, N, Abuf, N, s);
  if (rc) return rc;
  double h = 0.0;
  if ((rc = reduce(C, Abuf, nullptr, N, 0, partial, scal, &h, s))) return rc;
  p->unitarity_defect = h;
  if (!(h <= 1e-10)) {
    set_error("F is not unitary: max|F^H F - I| = %.3e > 1e-10", h);
    return FGFRFT_ENOTUNITARY;
  }

  // ---- 2. pivoted Householder QR of F + I (column-major); the standard form has no split
  const bool split = p->form == FGFRFT_FORM_SPLIT;
  int k = N;
  p->r_minus1 = 0;
  p->stop_norm = 0.0;
  p->last_pivot_norm = 0.0;
  if (split) {
    if (C) k_plus_identity_colmajor<true><<<grid_for(total), 256, 0, s>>>(Fd, N, Abuf);
    else k_plus_identity_colmajor<false><<<grid_for(total), 256, 0, s>>>(Fd, N, Abuf);
    FG_LAUNCHED("plus_identity");
    if (C) k_colnorms<true><<<ceil_div(N, 4), 256, 0, s>>>(Abuf, N, cn2);
    else k_colnorms<false><<<ceil_div(N, 4), 256, 0, s>>>(Abuf, N, cn2);
    FG_LAUNCHED("colnorms");
    FG_HIP(hipMemsetAsync(st, 0, sizeof(QRState), s));
    const double tol2 = tau * tau;
    for (int j = 0; j < N; ++j) {
      if (C) k_qr_pivot_house<true><<<1, 1024, 0, s>>>(Abuf, N, j, cn2, taub, st, tol2);
      else k_qr_pivot_house<false><<<1, 1024, 0, s>>>(Abuf, N, j, cn2, taub, st, tol2);
      const int ncols = N - j - 1;
      if (ncols > 0) {
        if (C) k_qr_update<true><<<ceil_div(ncols, 4), 256, 0, s>>>(Abuf, N, j, cn2, taub, st);
        else k_qr_update<false><<<ceil_div(ncols, 4), 256, 0, s>>>(Abuf, N, j, cn2, taub, st);
      }
    }
    FG_LAUNCHED("qr steps");
    QRState hs;
    FG_HIP(hipMemcpyAsync(&hs, st, sizeof(QRState), hipMemcpyDeviceToHost, s));
    FG_HIP(hipStreamSynchronize(s));
    k = hs.done ? hs.k : N;
    p->r_minus1 = N - k;
    p->stop_norm = hs.done ? hs.stop_norm : 0.0;
    p->last_pivot_norm = hs.last_pivot;
  }

  // ---- 3. W, P = W W^H, P_c = I - P
  const int r = p->r_minus1;
  if (r > 0) {
    if (C) k_form_W<true><<<r, 256, 0, s>>>(Abuf, N, k, taub, Mcur);
    else k_form_W<false><<<r, 256, 0, s>>>(Abuf, N, k, taub, Mcur);
    FG_LAUNCHED("form_W");
  }
  p->w_ok = 0;
  if (!C && p->W && r <= kWCols) {
    k_store_W<<<grid_for((size_t)N * kWCols), 256, 0, s>>>(Mcur, N, r, p->W);
    FG_LAUNCHED("store W");
    p->w_ok = 1;
  }
  if (C) k_projector<true><<<grid_for(total), 256, 0, s>>>(Mcur, N, r, P64, Mprev);
  else k_projector<false><<<grid_for(total), 256, 0, s>>>(Mcur, N, r, P64, Mprev);
  FG_LAUNCHED("projector");
  if (C) k_store<true><<<grid_for(total), 256, 0, s>>>(P64, total, 0, p->P);
  else k_store<false><<<grid_for(total), 256, 0, s>>>(P64, total, 0, p->P);
  FG_LAUNCHED("store P");

  // ---- 4. M_n = F M_{n-1}, stored as the resident stack; drift at ceil(L/2) and L
  const int kind = p->stacktype == FGFRFT_STACK_BF16X2 ? 1 : p->stacktype == FGFRFT_STACK_FP16X2 ? 2 : 0;
  double drift = 0.0;
  for (int n = 1; n <= L; ++n) {
    if ((rc = gemm_f64(C, false, N, N, N, Fd, N, Mprev, N, Mcur, N, s))) return rc;
    // slots 0..L-1 hold F^n P_c = M_n, slots L..2L-1 hold F^{-n} P_c = M_n^H (Proposition 2)
    void* dst = (char*)p->stack + (size_t)(n - 1) * total * p->stack_elem_bytes;
    void* dsth = (char*)p->stack + (size_t)(L + n - 1) * total * p->stack_elem_bytes;
    const dim3 tg(ceil_div(N, 32), ceil_div(N, 32));
    if (C) {
      k_store<true><<<grid_for(total), 256, 0, s>>>(Mcur, total, kind, dst);
      k_store_adjoint<true><<<tg, 256, 0, s>>>(Mcur, N, kind, dsth);
    } else {
      k_store<false><<<grid_for(total), 256, 0, s>>>(Mcur, total, kind, dst);
      k_store_adjoint<false><<<tg, 256, 0, s>>>(Mcur, N, kind, dsth);
    }
    FG_LAUNCHED("store stack");
    if (n == (L + 1) / 2 || n == L) {
      if ((rc = gemm_f64(C, true, N, N, N, Mcur, N, Mcur, N, Abuf, N, s))) return rc;
      double ss = 0.0;
      if ((rc = reduce(C, Abuf, P64, N, 1, partial, scal, &ss, s))) return rc;
      drift = fmax(drift, sqrt(ss) / sqrt((double)N));
    }
    double* tmp = Mprev; Mprev = Mcur; Mcur = tmp;
  }
  FG_HIP(hipStreamSynchronize(s));
  p->drift = drift;
  if (!(drift <= 1e-9)) {
    set_error("power recurrence drift %.3e > 1e-9", drift);
    return FGFRFT_EDRIFT;
  }
  return FGFRFT_OK;
}

}  // namespace fgfrft
