// Apply the operator to graph signals (Definition 2): Y[a] = op(Q[a]) X[a],
// op = identity or conjugate transpose (Proposition 3: Q^{-alpha} = (Q^alpha)^H).
//
// Batched complex GEMM on the matrix cores.  Operands are split into fp16
// hi/lo parts (hi*hi + hi*lo + lo*hi, FP32 accumulation).  Q entries are
// bounded by ~1.1 and use the fixed 2^12 scale; each signal column of X gets
// its own power-of-two scale (from a max-abs pre-pass) so any FP32 input
// range keeps ~22 significant bits.
//
// Tiles: 64 output rows x 64 signals per workgroup, k-chunks of 32 through
// LDS.  Workgroups of one order are placed on one XCD (the hardware deals
// workgroup ids round-robin over the 8 XCDs), so X[a] is shared in that XCD's L2.
#include "internal.h"
#include <math.h>

namespace fgfrft {

constexpr int AM = 64, AN = 64, AK = 32;
constexpr int RS = 40;   // LDS row stride in 16-bit values (32 + 8 pad)

// ---------------------------------------------------------------- per-signal scales
// scale[(a, b)] = 2^e with max_i |X[a][i][b]| * 2^e in [2^13, 2^14); stored (s, 1/s).
__global__ __launch_bounds__(256) void k_colscale(const void* __restrict__ X, int x_complex, int N, int B, int nx,
                                                  float2* __restrict__ scale) {
  const int a = blockIdx.y;
  const int b = blockIdx.x * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  __shared__ float red[4][64];
  float m = 0.f;
  if (b < B && a < nx) {
    for (int i = rg; i < N; i += 4) {
      const size_t off = ((size_t)a * N + i) * B + b;
      if (x_complex) {
        const float2 v = ((const float2*)X)[off];
        m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
      } else {
        m = fmaxf(m, fabsf(((const float*)X)[off]));
      }
    }
  }
  red[rg][threadIdx.x & 63] = m;
  __syncthreads();
  if (rg == 0 && b < B && a < nx) {
    m = fmaxf(fmaxf(red[0][threadIdx.x], red[1][threadIdx.x]), fmaxf(red[2][threadIdx.x], red[3][threadIdx.x]));
    int e = 0;
    if (m > 0.f && isfinite(m)) {
      int E;
      frexpf(m, &E);
      e = 14 - E;
      if (e > 100) e = 100;
      if (e < -100) e = -100;
    }
    scale[(size_t)a * B + b] = make_float2(ldexpf(1.f, e), ldexpf(1.f, -e));
  }
}

__device__ __forceinline__ void split_h(float v, short& hi, short& lo) {
  const _Float16 h = (_Float16)v;
  const _Float16 l = (_Float16)(v - (float)h);
  hi = __builtin_bit_cast(short, h);
  lo = __builtin_bit_cast(short, l);
}
__device__ __forceinline__ floatx16 mma(shortx8 a, shortx8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0, 0, 0);
}

// LDS planes: Qs[plane re/im][part hi/lo][row][k], Xs[plane][part][col][k]; rows padded to RS.
template <bool ADJ, bool XC, bool YREAL>
__global__ __launch_bounds__(256) void k_apply(const cplx64* __restrict__ Q, int N, int n_alpha, const void* __restrict__ X,
                                               int x_shared, int B, const float2* __restrict__ xscale,
                                               void* __restrict__ Y, int nrb, int ncb) {
  constexpr int XPL = XC ? 2 : 1;
  __shared__ __align__(16) short Qs[2][2][AM][RS];
  __shared__ __align__(16) short Xs[XPL][2][AN][RS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // ---- XCD-aware decode: orders a = xcd (mod 8) live on XCD `xcd`
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int per_a = nrb * ncb;
  const int a = xcd + 8 * (slot / per_a);
  if (a >= n_alpha) return;
  const int rem = slot % per_a, rb = rem / ncb, cb = rem % ncb;
  const int i0 = rb * AM, b0 = cb * AN;
  const size_t NN = (size_t)N * N;
  const cplx64* Qa = Q + (size_t)a * NN;
  const size_t xoff = x_shared ? 0 : (size_t)a * N * B;
  const float2* xs = xscale + (x_shared ? 0 : (size_t)a * B);

  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int l32 = lane & 31, lh = lane >> 5;
  floatx16 acc_re = {}, acc_im = {};

  // staging coordinates.  Q (no adjoint): row qr = tid/4, 8 consecutive k from (tid%4)*8, so four
  // neighbouring threads read one 256-byte row segment.  Q (adjoint) and X: index xc = tid%64 along
  // the contiguous memory dimension, 8 consecutive k from (tid/64)*8.
  const int qr = ADJ ? (tid & 63) : (tid >> 2), qk = ADJ ? (tid >> 6) * 8 : (tid & 3) * 8;
  const int xc = tid & 63, xk = (tid >> 6) * 8;
  float xsc = 1.f;
  if (b0 + xc < B) xsc = xs[b0 + xc].x;

  // register staging of one k-chunk: op(Q)[i0 + qr][k0 + qk .. +7] and X[k0 + xk .. +7][b0 + xc].
  // The next chunk's global loads are issued before the current chunk's MFMAs, so they are in
  // flight while the matrix cores work (nothing in this loop stores to global memory).
  cplx64 qv[8];
  float xv[8], xw[8];
  auto fetch = [&](int k0) {
    const int gi = i0 + qr, gk0 = k0 + qk;
    if (!ADJ && (N & 1) == 0 && gi < N && gk0 + 7 < N) {  // 16-byte aligned when N is even
      const float4* src = (const float4*)(Qa + (size_t)gi * N + gk0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float4 f = src[e];
        qv[2 * e] = cplx64{f.x, f.y};
        qv[2 * e + 1] = cplx64{f.z, f.w};
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gk = gk0 + e;
        qv[e] = cplx64{0.f, 0.f};
        if (gi < N && gk < N) {
          if (!ADJ) qv[e] = Qa[(size_t)gi * N + gk];
          else { qv[e] = Qa[(size_t)gk * N + gi]; qv[e].im = -qv[e].im; }
        }
      }
    }
    const int gb = b0 + xc;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int gk = k0 + xk + e;
      xv[e] = 0.f;
      xw[e] = 0.f;
      if (gb < B && gk < N) {
        const size_t off = xoff + (size_t)gk * B + gb;
        if (XC) { const float2 v = ((const float2*)X)[off]; xv[e] = v.x; xw[e] = v.y; }
        else xv[e] = ((const float*)X)[off];
      }
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < N; k0 += AK) {
    // ---- split the fetched chunk into fp16 hi/lo parts in LDS (X scaled per column, transposed)
    {
      shortx8 vrh, vrl, vih, vil;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        short a_, b_, c_, d_;
        split_h(qv[e].re * kStackScale, a_, b_);
        split_h(qv[e].im * kStackScale, c_, d_);
        vrh[e] = a_; vrl[e] = b_; vih[e] = c_; vil[e] = d_;
      }
      *(shortx8*)&Qs[0][0][qr][qk] = vrh;
      *(shortx8*)&Qs[0][1][qr][qk] = vrl;
      *(shortx8*)&Qs[1][0][qr][qk] = vih;
      *(shortx8*)&Qs[1][1][qr][qk] = vil;
      shortx8 v0, v1;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        short h, l;
        split_h(xv[e] * xsc, h, l);
        v0[e] = h; v1[e] = l;
      }
      *(shortx8*)&Xs[0][0][xc][xk] = v0;
      *(shortx8*)&Xs[0][1][xc][xk] = v1;
      if (XC) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          short h, l;
          split_h(xw[e] * xsc, h, l);
          v0[e] = h; v1[e] = l;
        }
        *(shortx8*)&Xs[XPL - 1][0][xc][xk] = v0;
        *(shortx8*)&Xs[XPL - 1][1][xc][xk] = v1;
      }
    }
    __syncthreads();
    if (k0 + AK < N) fetch(k0 + AK);
#pragma unroll
    for (int ks = 0; ks < AK; ks += 16) {
      const int kk = ks + 8 * lh;
      const shortx8 qrh = *(const shortx8*)&Qs[0][0][wr + l32][kk];
      const shortx8 qrl = *(const shortx8*)&Qs[0][1][wr + l32][kk];
      const shortx8 qih = *(const shortx8*)&Qs[1][0][wr + l32][kk];
      const shortx8 qil = *(const shortx8*)&Qs[1][1][wr + l32][kk];
      const shortx8 xrh = *(const shortx8*)&Xs[0][0][wc + l32][kk];
      const shortx8 xrl = *(const shortx8*)&Xs[0][1][wc + l32][kk];
      acc_re = mma(qrh, xrh, acc_re);
      acc_re = mma(qrh, xrl, acc_re);
      acc_re = mma(qrl, xrh, acc_re);
      acc_im = mma(qih, xrh, acc_im);
      acc_im = mma(qih, xrl, acc_im);
      acc_im = mma(qil, xrh, acc_im);
      if (XC) {
        const shortx8 xih = *(const shortx8*)&Xs[XPL - 1][0][wc + l32][kk];
        const shortx8 xil = *(const shortx8*)&Xs[XPL - 1][1][wc + l32][kk];
        const shortx8 nqih = qih ^ (short)0x8000, nqil = qil ^ (short)0x8000;
        acc_re = mma(nqih, xih, acc_re);
        acc_re = mma(nqih, xil, acc_re);
        acc_re = mma(nqil, xih, acc_re);
        acc_im = mma(qrh, xih, acc_im);
        acc_im = mma(qrh, xil, acc_im);
        acc_im = mma(qrl, xih, acc_im);
      }
    }
    __syncthreads();
  }
  // ---- write back: lane holds column b = b0 + wc + l32, rows wr + 8(r/4) + 4 lh + r%4
  const int gb = b0 + wc + l32;
  if (gb >= B) return;
  const float u = xs[gb].y * (1.0f / kStackScale);
  const size_t yoff = (size_t)a * N * B;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int gi = i0 + wr + 8 * (r >> 2) + 4 * lh + (r & 3);
    if (gi < N) {
      const size_t off = yoff + (size_t)gi * B + gb;
      if (YREAL) ((float*)Y)[off] = acc_re[r] * u;
      else ((cplx64*)Y)[off] = cplx64{acc_re[r] * u, acc_im[r] * u};
    }
  }
}

size_t apply_ws_bytes(int N, int n_alpha, int B, int x_shared) {
  (void)N;
  return align_up((size_t)(x_shared ? 1 : n_alpha) * B * sizeof(float2), 256);
}

template <bool ADJ, bool XC, bool YR>
static void launch_apply_t(dim3 g, hipStream_t s, const cplx64* Q, int N, int n_alpha, const void* X, int x_shared,
                           int B, const float2* sc, void* Y, int nrb, int ncb) {
  k_apply<ADJ, XC, YR><<<g, 256, 0, s>>>(Q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb);
}

fgfrft_status apply_launch(const void* Q, int N, int n_alpha, int adjoint, const void* X, int x_complex, int x_shared,
                           int B, void* Y, int y_real, void* ws, hipStream_t s) {
  float2* sc = (float2*)ws;
  const int nx = x_shared ? 1 : n_alpha;
  k_colscale<<<dim3(ceil_div(B, 64), nx), 256, 0, s>>>(X, x_complex, N, B, nx, sc);
  FG_LAUNCHED("colscale");
  const int nrb = ceil_div(N, AM), ncb = ceil_div(B, AN);
  const size_t nblocks = (size_t)8 * ceil_div(n_alpha, 8) * nrb * ncb;
  if (nblocks > 0x7fffffff) {
    set_error("apply grid too large");
    return FGFRFT_EUNSUPPORTED;
  }
  dim3 g((unsigned)nblocks);
  const cplx64* q = (const cplx64*)Q;
  const int key = (adjoint ? 4 : 0) | (x_complex ? 2 : 0) | (y_real ? 1 : 0);
  switch (key) {
    case 0: launch_apply_t<false, false, false>(g, s, q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb); break;
    case 1: launch_apply_t<false, false, true>(g, s, q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb); break;
    case 2: launch_apply_t<false, true, false>(g, s, q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb); break;
    case 3: launch_apply_t<false, true, true>(g, s, q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb); break;
    case 4: launch_apply_t<true, false, false>(g, s, q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb); break;
    case 5: launch_apply_t<true, false, true>(g, s, q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb); break;
    case 6: launch_apply_t<true, true, false>(g, s, q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb); break;
    case 7: launch_apply_t<true, true, true>(g, s, q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb); break;
  }
  FG_LAUNCHED("apply");
  return FGFRFT_OK;
}

}  // namespace fgfrft
