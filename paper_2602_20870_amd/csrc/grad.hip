// Gradients through Y[a] = Q_L^{alpha_a} X[a] (Proposition 4).
//
// For a real loss with GY = dl/dRe Y + j dl/dIm Y and G_a = GY[a] X[a]^H:
//   dl/dalpha_a = Re[ sum_{n=-L}^{L} c_n'(alpha_a) <G_a, F^n P_c> + j pi e^{j pi alpha_a} <G_a, P> ],
//   <A, B> = sum_ij conj(A_ij) B_ij, F^{-n} P_c = M_n^H, M_0 = P_c = I - P,
//   dl/dX[a] = Q(alpha_a)^H GY[a] = Q(-alpha_a) GY[a]                          (Proposition 3).
// The GPU forms the inner products T[a][k] = <G_a, B_k> for B_k in
// {M_1..M_L, M_1^H..M_L^H, P, I}; the host combines them with c_n'(alpha) in FP64.
//
// Steps per chunk of orders:
//   k_outer      G_a = GY[a] X[a]^H                     (FP32, LDS-tiled)
//   k_inner      per 16x16 tile: the tile's 2L stack matrices staged in LDS once,
//                partial sums of T over the tile's positions for every order of the chunk
//   k_inner_sum  fixed-order sum of the partials over all tiles in FP64 (deterministic)
#include "internal.h"
#include <math.h>
#include <vector>

namespace fgfrft {

constexpr int GT = 16, GPOS = 256;

// ---------------------------------------------------------------- G = GY X^H
// 64x64 output tile, 256 threads with 4x4 outputs each, k (signals) in chunks of 16.
template <bool XC>
__global__ __launch_bounds__(256) void k_outer(const cplx64* __restrict__ GY, const void* __restrict__ X, int x_shared,
                                               int N, int B, int a_first, cplx64* __restrict__ G) {
  __shared__ float Ar[16][65], Ai[16][65], Br[16][65], Bi[16][65];
  const int tid = threadIdx.x, a = a_first + blockIdx.z;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int ti = (tid / 16) * 4, tj = (tid % 16) * 4;
  const cplx64* gy = GY + (size_t)a * N * B;
  const size_t xoff = x_shared ? 0 : (size_t)a * N * B;
  float accr[4][4] = {}, acci[4][4] = {};
  for (int b0 = 0; b0 < B; b0 += 16) {
    for (int e = tid; e < 64 * 16; e += 256) {
      const int r = e / 16, c = e % 16;
      const int gi = i0 + r, gj = j0 + r, gb = b0 + c;
      cplx64 g = {0.f, 0.f};
      if (gi < N && gb < B) g = gy[(size_t)gi * B + gb];
      Ar[c][r] = g.re;
      Ai[c][r] = g.im;
      float xr = 0.f, xi = 0.f;
      if (gj < N && gb < B) {
        if (XC) { const float2 v = ((const float2*)X)[xoff + (size_t)gj * B + gb]; xr = v.x; xi = v.y; }
        else xr = ((const float*)X)[xoff + (size_t)gj * B + gb];
      }
      Br[c][r] = xr;
      Bi[c][r] = xi;
    }
    __syncthreads();
#pragma unroll 4
    for (int c = 0; c < 16; ++c) {
      float ar[4], ai[4], br[4], bi[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ar[q] = Ar[c][ti + q]; ai[q] = Ai[c][ti + q];
        br[q] = Br[c][tj + q]; bi[q] = Bi[c][tj + q];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {  // g * conj(x)
          accr[x][y] += ar[x] * br[y] + ai[x] * bi[y];
          acci[x][y] += ai[x] * br[y] - ar[x] * bi[y];
        }
    }
    __syncthreads();
  }
  cplx64* g = G + (size_t)blockIdx.z * N * N;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int gi = i0 + ti + x, gj = j0 + tj + y;
      if (gi < N && gj < N) g[(size_t)gi * N + gj] = cplx64{accr[x][y], acci[x][y]};
    }
}

// ---------------------------------------------------------------- T partials per tile
// One workgroup per 16x16 tile of positions.  LDS: S[pos][k][plane] for the 2L resident
// matrices (k < L: M_{k+1}, k >= L: M_{k-L+1}^H), Pt[pos][plane], Gs[a][pos][2] for up to AC
// orders at a time.  Thread (k, half) accumulates conj(G) * B_k over half of the tile's
// positions for every order of the sub-chunk; B_{2L} = P, B_{2L+1} = I.
constexpr int AC = 4;

template <bool CPLX>
__global__ __launch_bounds__(256) void k_inner(const void* __restrict__ stack, const void* __restrict__ Pm, int N, int L,
                                               int nb, const cplx64* __restrict__ G, int n_chunk,
                                               double* __restrict__ partial) {
  constexpr int NPL = CPLX ? 2 : 1;
  extern __shared__ __align__(16) float sm[];
  const int L2 = 2 * L;
  float* S = sm;                                         // [GPOS][L2][NPL]
  float* Pt = S + (size_t)GPOS * L2 * NPL;               // [GPOS][NPL]
  float* Gs = Pt + GPOS * NPL;                           // [AC][GPOS][2]
  const int tid = threadIdx.x;
  const int q = blockIdx.x;
  const int I = q / nb, J = q % nb;
  const size_t NN = (size_t)N * N;
  for (int it = tid; it < GPOS * L2; it += 256) {
    const int p = it % GPOS, k = it / GPOS;
    const int row = I * GT + p / GT, col = J * GT + p % GT;
    const bool inb = row < N && col < N;
    float* dst = S + ((size_t)p * L2 + k) * NPL;
    const size_t off = (size_t)k * NN + (size_t)row * N + col;
    if (CPLX) {
      const float2 v = inb ? ((const float2*)stack)[off] : make_float2(0.f, 0.f);
      dst[0] = v.x;
      dst[NPL - 1] = v.y;
    } else {
      dst[0] = inb ? ((const float*)stack)[off] : 0.f;
    }
  }
  for (int p = tid; p < GPOS; p += 256) {
    const int row = I * GT + p / GT, col = J * GT + p % GT;
    const bool inb = row < N && col < N;
    if (CPLX) {
      const float2 v = inb ? ((const float2*)Pm)[(size_t)row * N + col] : make_float2(0.f, 0.f);
      Pt[p * 2] = v.x;
      Pt[p * 2 + 1] = v.y;
    } else {
      Pt[p] = inb ? ((const float*)Pm)[(size_t)row * N + col] : 0.f;
    }
  }
  const int K = L2 + 2;
  for (int a0 = 0; a0 < n_chunk; a0 += AC) {
    const int na = min(AC, n_chunk - a0);
    __syncthreads();
    for (int it = tid; it < na * GPOS; it += 256) {
      const int p = it % GPOS, a = it / GPOS;
      const int row = I * GT + p / GT, col = J * GT + p % GT;
      cplx64 g = {0.f, 0.f};
      if (row < N && col < N) g = G[(size_t)(a0 + a) * NN + (size_t)row * N + col];
      Gs[(a * GPOS + p) * 2] = g.re;
      Gs[(a * GPOS + p) * 2 + 1] = g.im;
    }
    __syncthreads();
    for (int w = tid; w < 2 * K; w += 256) {
      const int k = w % K, half = w / K;
      double sr[AC], si[AC];   // FP64 accumulation (same FMA rate as FP32 here)
#pragma unroll
      for (int a = 0; a < AC; ++a) { sr[a] = 0.0; si[a] = 0.0; }
      for (int p = half * (GPOS / 2); p < (half + 1) * (GPOS / 2); ++p) {
        float br, bi = 0.f;
        if (k < L2) {
          const float* sp = S + ((size_t)p * L2 + k) * NPL;
          br = sp[0];
          if (CPLX) bi = sp[NPL - 1];
        } else if (k == L2) {
          br = Pt[p * NPL];
          if (CPLX) bi = Pt[p * NPL + NPL - 1];
        } else {
          br = (I * GT + p / GT == J * GT + p % GT) ? 1.f : 0.f;
        }
#pragma unroll
        for (int a = 0; a < AC; ++a) {  // conj(g) * b
          if (a < na) {
            const double gr = Gs[(a * GPOS + p) * 2], gi = Gs[(a * GPOS + p) * 2 + 1];
            sr[a] += gr * (double)br + gi * (double)bi;
            si[a] += gr * (double)bi - gi * (double)br;
          }
        }
      }
      for (int a = 0; a < na; ++a) {
        const size_t o = (((size_t)q * n_chunk + a0 + a) * 2 + half) * K + k;
        partial[2 * o] = sr[a];
        partial[2 * o + 1] = si[a];
      }
    }
  }
}

// T[a][k] = sum over tiles and both halves, in a fixed order, in FP64.
__global__ __launch_bounds__(256) void k_inner_sum(const double* __restrict__ partial, int ntiles, int n_chunk, int K,
                                                   int a_first, double* __restrict__ T) {
  __shared__ double rr[256], ri[256];
  const int a = blockIdx.y, k = blockIdx.x;
  double sr = 0.0, si = 0.0;
  for (int q = threadIdx.x; q < ntiles; q += 256)
    for (int t = 0; t < 2; ++t) {
      const size_t o = (((size_t)q * n_chunk + a) * 2 + t) * K + k;
      sr += partial[2 * o];
      si += partial[2 * o + 1];
    }
  rr[threadIdx.x] = sr;
  ri[threadIdx.x] = si;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) { rr[threadIdx.x] += rr[threadIdx.x + s]; ri[threadIdx.x] += ri[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    T[((size_t)(a_first + a) * K + k) * 2] = rr[0];
    T[((size_t)(a_first + a) * K + k) * 2 + 1] = ri[0];
  }
}

// dX (shared X): out += sum over the chunk's orders of Y[a]
template <bool REAL>
__global__ __launch_bounds__(256) void k_sum_orders(const void* __restrict__ Y, int n_chunk, size_t per, int first,
                                                    void* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < per; i += (size_t)gridDim.x * 256) {
    if (REAL) {
      float s = first ? 0.f : ((float*)out)[i];
      for (int a = 0; a < n_chunk; ++a) s += ((const float*)Y)[(size_t)a * per + i];
      ((float*)out)[i] = s;
    } else {
      float2 s = first ? make_float2(0.f, 0.f) : ((float2*)out)[i];
      for (int a = 0; a < n_chunk; ++a) {
        const float2 v = ((const float2*)Y)[(size_t)a * per + i];
        s.x += v.x;
        s.y += v.y;
      }
      ((float2*)out)[i] = s;
    }
  }
}

// ---------------------------------------------------------------- host
static int grad_chunk(const Plan* p, int n_alpha) {
  (void)p;
  return n_alpha < 8 ? n_alpha : 8;
}

static size_t inner_lds(const Plan* p) {
  const int NPL = p->cplx ? 2 : 1;
  return ((size_t)GPOS * 2 * p->L * NPL + GPOS * NPL + (size_t)AC * GPOS * 2) * sizeof(float);
}

size_t grad_ws_bytes(const Plan* p, int n_alpha, int B, int x_shared) {
  const int ch = grad_chunk(p, n_alpha);
  const int N = p->N, nb = ceil_div(N, GT), npairs = nb * nb, K = 2 * p->L + 2;
  size_t s = 0;
  s += align_up((size_t)ch * N * N * 8, 256);                       // G chunk / Q(-alpha) chunk
  s += align_up((size_t)npairs * ch * 2 * K * 16, 256);             // partials (complex FP64)
  s += align_up((size_t)n_alpha * K * 16, 256);                     // T
  s += align_up((size_t)ch * N * B * 8, 256);                       // dX chunk (shared X)
  s += update_ws_bytes(p, ch);
  s += apply_ws_bytes(N, ch, B, 0);
  s += align_up((size_t)n_alpha * 8, 256);
  (void)x_shared;
  return s;
}

static void coefficient_derivatives(double alpha, int L, std::vector<double>& d) {
  d.assign(2 * L + 1, 0.0);
  for (int n = -L; n <= L; ++n) {
    const double x = alpha - n;
    double v;
    if (fabs(x) < 1e-4) v = -M_PI * M_PI * x / 3.0 + pow(M_PI, 4) * x * x * x / 30.0;
    else v = (cos(M_PI * x) - sin(M_PI * x) / (M_PI * x)) / x;
    d[n + L] = v;
  }
}

fgfrft_status grad_run(const Plan* p, const double* alphas, int n_alpha, const void* X, int x_complex, int x_shared,
                       int B, const void* GY, double* dalpha, void* dX, void* ws, size_t ws_bytes, hipStream_t s) {
  const int N = p->N, L = p->L, K = 2 * L + 2;
  const int ch = grad_chunk(p, n_alpha);
  const int nb = ceil_div(N, GT), npairs = nb * nb;  // 16x16 tiles
  if (ws_bytes < grad_ws_bytes(p, n_alpha, B, x_shared)) {
    set_error("grad workspace too small: %zu < %zu", ws_bytes, grad_ws_bytes(p, n_alpha, B, x_shared));
    return FGFRFT_ENOMEM;
  }
  char* base = (char*)ws;
  cplx64* Gbuf = (cplx64*)base; base += align_up((size_t)ch * N * N * 8, 256);
  double* partial = (double*)base; base += align_up((size_t)npairs * ch * 2 * K * 16, 256);
  double* T = (double*)base; base += align_up((size_t)n_alpha * K * 16, 256);
  void* dXc = base; base += align_up((size_t)ch * N * B * 8, 256);
  void* uws = base; base += update_ws_bytes(p, ch);
  void* aws = base; base += apply_ws_bytes(N, ch, B, 0);
  double* neg_dev = (double*)base;

  const size_t lds = inner_lds(p);
  static bool attr[2] = {false, false};
  if (!attr[p->cplx]) {
    if (p->cplx) FG_HIP(hipFuncSetAttribute((const void*)k_inner<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    else FG_HIP(hipFuncSetAttribute((const void*)k_inner<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr[p->cplx] = true;
  }
  std::vector<double> neg(n_alpha);
  for (int a = 0; a < n_alpha; ++a) neg[a] = -alphas[a];
  FG_HIP(hipMemcpyAsync(neg_dev, neg.data(), (size_t)n_alpha * 8, hipMemcpyHostToDevice, s));
  const cplx64* gy = (const cplx64*)GY;
  const size_t NB = (size_t)N * B;
  for (int a0 = 0; a0 < n_alpha; a0 += ch) {
    const int nc = n_alpha - a0 < ch ? n_alpha - a0 : ch;
    // ---- dX = Q(-alpha) GY
    if (dX) {
      fgfrft_status rc = update_launch(p, neg_dev + a0, nc, Gbuf, uws, s);
      if (rc) return rc;
      void* dst = x_shared ? dXc : (void*)((char*)dX + (size_t)a0 * NB * (x_complex ? 8 : 4));
      rc = apply_launch(Gbuf, N, nc, 0, gy + (size_t)a0 * NB, 1, 0, B, dst, x_complex ? 0 : 1, aws, s);
      if (rc) return rc;
      if (x_shared) {
        const int g = (int)((NB + 255) / 256 < 4096 ? (NB + 255) / 256 : 4096);
        if (x_complex) k_sum_orders<false><<<g, 256, 0, s>>>(dXc, nc, NB, a0 == 0, dX);
        else k_sum_orders<true><<<g, 256, 0, s>>>(dXc, nc, NB, a0 == 0, dX);
        FG_LAUNCHED("sum_orders");
      }
    }
    // ---- G = GY X^H for the chunk
    {
      dim3 g(ceil_div(N, 64), ceil_div(N, 64), nc);
      const void* xa = x_shared ? X : (const void*)((const char*)X + (size_t)a0 * NB * (x_complex ? 8 : 4));
      if (x_complex) k_outer<true><<<g, 256, 0, s>>>(gy + (size_t)a0 * NB, xa, x_shared, N, B, 0, Gbuf);
      else k_outer<false><<<g, 256, 0, s>>>(gy + (size_t)a0 * NB, xa, x_shared, N, B, 0, Gbuf);
      FG_LAUNCHED("outer");
    }
    if (p->cplx) k_inner<true><<<npairs, 256, lds, s>>>(p->stack, p->P, N, L, nb, Gbuf, nc, partial);
    else k_inner<false><<<npairs, 256, lds, s>>>(p->stack, p->P, N, L, nb, Gbuf, nc, partial);
    FG_LAUNCHED("inner");
    k_inner_sum<<<dim3(K, nc), 256, 0, s>>>(partial, npairs, nc, K, a0, T);
    FG_LAUNCHED("inner_sum");
  }
  std::vector<double> Th((size_t)n_alpha * K * 2);
  FG_HIP(hipMemcpyAsync(Th.data(), T, Th.size() * 8, hipMemcpyDeviceToHost, s));
  FG_HIP(hipStreamSynchronize(s));
  std::vector<double> d;
  for (int a = 0; a < n_alpha; ++a) {
    const double al = alphas[a];
    coefficient_derivatives(al, L, d);
    const double* t = &Th[(size_t)a * K * 2];
    auto re = [&](int k) { return t[2 * k]; };
    auto im = [&](int k) { return t[2 * k + 1]; };
    double acc = 0.0;
    for (int n = 1; n <= L; ++n) acc += d[L + n] * re(n - 1) + d[L - n] * re(L + n - 1);
    // M_0 = I - P: <G, M_0> = <G, I> - <G, P>
    acc += d[L] * (re(2 * L + 1) - re(2 * L));
    // Re(j pi e^{j pi alpha} <G, P>) = -pi (sin(pi a) Re T_P + cos(pi a) Im T_P)
    acc += -M_PI * (sin(M_PI * al) * re(2 * L) + cos(M_PI * al) * im(2 * L));
    dalpha[a] = acc;
  }
  return FGFRFT_OK;
}

}  // namespace fgfrft
