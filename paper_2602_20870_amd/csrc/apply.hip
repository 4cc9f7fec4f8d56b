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
// Two passes: column maxima over chunks of CR rows (grid: (order, column block) x chunks),
// then the maximum over chunks and the power of two (fixed order, no atomics).
constexpr int CR = 64;

__global__ __launch_bounds__(256) void k_colmax(const void* __restrict__ X, int x_complex, int N, int B,
                                                float* __restrict__ partial) {
  const int ncb = (B + 63) / 64;
  const int a = blockIdx.x / ncb, ch = blockIdx.y, nch = gridDim.y;
  const int b = (blockIdx.x % ncb) * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  __shared__ float red[4][64];
  float m = 0.f;
  if (b < B) {
    const int i1 = (ch + 1) * CR < N ? (ch + 1) * CR : N;
    for (int i = ch * CR + rg; i < i1; i += 4) {
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
  if (rg == 0 && b < B)
    partial[((size_t)a * nch + ch) * B + b] =
        fmaxf(fmaxf(red[0][threadIdx.x], red[1][threadIdx.x]), fmaxf(red[2][threadIdx.x], red[3][threadIdx.x]));
}

__global__ __launch_bounds__(256) void k_colscale(const float* __restrict__ partial, int nch, int B, int nx,
                                                  float2* __restrict__ scale) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nx * B) return;
  const int a = idx / B, b = idx % B;
  float m = 0.f;
  for (int c = 0; c < nch; ++c) m = fmaxf(m, partial[((size_t)a * nch + c) * B + b]);
  int e = 0;
  if (m > 0.f && isfinite(m)) {
    int E;
    frexpf(m, &E);
    e = 14 - E;
    if (e > 100) e = 100;
    if (e < -100) e = -100;
  }
  scale[idx] = make_float2(ldexpf(1.f, e), ldexpf(1.f, -e));
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

// ---------------------------------------------------------------- streaming apply
// Y[a] = Q[a] X[a] for N % K2 == 0 and B % 64 == 0: 32 RG output rows x 64 signals per
// workgroup, k in stages of K2.  Each stage (32 RG rows x K2 of Q, K2 rows of X) moves from
// HBM/L2 straight into LDS with direct loads into a ring of NS stages, so NS - 1 stages are in
// flight while the matrix cores work on the current one; operands are split into fp16 hi/lo
// when a wave reads its fragments.  RG x KSPL waves: wave (g, p) computes rows 32g .. 32g + 31
// for both 32-signal blocks over part p of each stage's 16-wide k steps; with KSPL > 1 the
// parts' sums are added once at the end through LDS, in the fixed order p = 0, 1, ...
//   RG = 4, KSPL = 1, K2 = 32 or 16: two workgroups per CU, 256- or 128-byte Q row runs per stage;
//   RG = 4, KSPL = 2, K2 = 64: one workgroup per CU, two stages of 80 KB; every Q row is read as a
//   512-byte run per stage, which the memory system streams measurably faster than 256-byte runs.
// Q rows sit in LDS with their 16-byte chunks swizzled by row (chunk c of row r at
// c ^ (r mod SW)) so the fragment reads of 32 rows spread over the banks.
constexpr int M2 = 128;

template <bool XC, int K2, int RG = 4>
struct Apply2Layout {
  static constexpr int QB = 32 * RG * K2 * 8;         // Q stage bytes
  static constexpr int XB = K2 * 64 * (XC ? 8 : 4);   // X stage bytes
  static constexpr int SB = QB + XB;
  static constexpr int QROW = K2 * 8, CPR = K2 / 2, RPI = 1024 / QROW;   // row bytes, chunks, rows per load
  static constexpr int SW = CPR < 16 ? CPR : 16;      // swizzle period (rows)
};

// PRE (real signals, K2 = 32 or 64): X is the pre-split signal block of xsplit_launch, so a
// stage's B fragments are plain 16-byte LDS reads (no per-wave split of the same signals).
// ADJ (RG = 4, KSPL = 1): Y[a] = Q[a]^H X[a].  The 128 output rows i0.. of Q^H are the columns i0.. of
// Q, so a stage holds the k rows k0 .. k0 + K2 - 1 of Q restricted to those columns (one contiguous
// 1 KB run per row, one load instruction each) and a wave reads its operand fragments down the
// stage's columns, with the imaginary parts negated (Proposition 3: Q^{-alpha} = (Q^alpha)^H).
template <bool XC, bool YREAL, int NS, int K2, bool PRE = false, int RG = 4, int KSPL = 1, bool ADJ = false>
__global__ __launch_bounds__(64 * RG * KSPL, RG * KSPL == 4 ? 2 : 1) void k_apply2(
    const cplx64* __restrict__ Q, int N, int n_alpha, const void* __restrict__ X, int x_shared, int B,
    const float2* __restrict__ xscale, void* __restrict__ Y, int nrb, int ncb) {
  static_assert(!PRE || (!XC && K2 % 32 == 0), "pre-split signals: real, k stages of whole 32-row chunks");
  static_assert((K2 / 16) % KSPL == 0, "whole 16-wide k steps per part");
  static_assert(!ADJ || (RG == 4 && KSPL == 1 && !PRE), "adjoint: 128 rows, one k part, signals split per wave");
  using LY = Apply2Layout<XC, K2, RG>;
  constexpr int XE = XC ? 8 : 4, CPR = LY::CPR, RPI = LY::RPI, SW = LY::SW, NW = RG * KSPL;
  constexpr int QLW = LY::QB / (1024 * NW), XLW = LY::XB / (1024 * NW), LW = QLW + XLW;   // loads per wave
  static_assert(QLW * 1024 * NW == LY::QB && XLW * 1024 * NW == LY::XB, "whole loads per wave");
  static_assert(ADJ || (RPI * NW) % SW == 0, "row swizzle constant per wave");
  constexpr int KSW = K2 / 16 / KSPL;                 // 16-wide k steps per wave and stage
  extern __shared__ __align__(16) char sm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  const int rg = wave % RG, kp = wave / RG;           // row group, k part
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int per_a = nrb * ncb;
  const int a = xcd + 8 * (slot / per_a);
  if (a >= n_alpha) return;
  const int rem = slot % per_a, rb = rem / ncb, cb = rem % ncb;
  const int i0 = rb * 32 * RG, b0 = cb * 64;
  const size_t NN = (size_t)N * N;
  const char* Qa = (const char*)(Q + (size_t)a * NN);
  const char* Xa = (const char*)X + (x_shared ? 0 : (size_t)a * N * B * XE);
  const float2* xs = xscale + (x_shared ? 0 : (size_t)a * B);
  const int nch = N / K2;

  // Each direct load is a wave-uniform base plus a fixed per-lane 32-bit offset, so the offsets
  // stay in the same registers for the whole loop.  Q instruction i (i = wave + NW q) moves rows
  // i0 + RPI i .. + RPI - 1 (a row group past N: any valid rows, never written back; N % 8 == 0
  // so groups are whole); lane: row + lane / CPR, stored chunk lane % CPR holds chunk
  // (lane % CPR) ^ (row mod SW), which is the same for every q of a wave.  X instruction i moves
  // the next rows of k of the 64 signals.
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int qrow = lane / CPR;
  // ADJ: lane's 16 bytes are columns i0 + 2 lane, + 1 of a k row; past N (the last row block when
  // N % 128 != 0; N % 16 == 0 keeps pairs whole) any valid pair, never written back
  const uint32_t qoff =
      ADJ ? (uint32_t)((i0 + 2 * lane < N ? 2 * lane : N - 2 - i0) * 8)
          : (uint32_t)(((size_t)qrow * N + 2 * ((lane % CPR) ^ ((RPI * wv + qrow) % SW))) * 8);
  const uint32_t xoff_l = XC ? (uint32_t)(((size_t)(lane >> 5) * B + 2 * (lane & 31)) * 8)
                             : (uint32_t)(((size_t)(lane >> 4) * B + 4 * (lane & 15)) * 4);
  auto issue = [&](int it) {
    char* st = sm + (it % NS) * LY::SB;
    const int k0 = it * K2;
#pragma unroll
    for (int q = 0; q < QLW; ++q) {
      const int i = wv + NW * q;
      if (ADJ) {   // k row k0 + i, columns i0 ..
        lds_dma16(Qa + ((size_t)(k0 + i) * N + i0) * 8 + qoff, __builtin_amdgcn_readfirstlane(lds_addr(st + i * 1024)));
      } else {
        const int row0 = i0 + RPI * i < N ? i0 + RPI * i : N - RPI;
        const char* gb = Qa + ((size_t)row0 * N + k0) * 8;
        lds_dma16(gb + qoff, __builtin_amdgcn_readfirstlane(lds_addr(st + i * 1024)));
      }
    }
#pragma unroll
    for (int q = 0; q < XLW; ++q) {
      const int i = wv + NW * q;
      if (PRE) {
        const char* gb = (const char*)X + (((size_t)(x_shared ? 0 : a) * ncb + cb) * nch + it) * LY::XB + i * 1024;
        lds_dma16(gb + 16 * lane, __builtin_amdgcn_readfirstlane(lds_addr(st + LY::QB + i * 1024)));
      } else {
        const char* gb = Xa + ((size_t)(k0 + (XC ? 2 * i : 4 * i)) * B + b0) * XE;
        lds_dma16(gb + xoff_l, __builtin_amdgcn_readfirstlane(lds_addr(st + LY::QB + i * 1024)));
      }
    }
  };

  float xsc[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) xsc[c] = xs[b0 + 32 * c + l32].x;
  // settle these loads before the ring starts: a wait for them inside the loop would also wait
  // for every direct load issued after them
  asm volatile("" ::"v"(xsc[0]), "v"(xsc[1]));
  floatx16 acc_re[2] = {}, acc_im[2] = {};
  const int r = 32 * rg + l32;

  for (int it = 0; it < NS - 1 && it < nch; ++it) issue(it);
  for (int it = 0; it < nch; ++it) {
    // this wave's loads of stage it have landed (only the NS - 2 younger stages may still be in
    // flight) and its reads of stage it - 1 are done; after the barrier that holds for every wave
    if (it + NS - 1 <= nch) __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0((NS - 2) * LW));
    else __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
    barrier_nofence();
    if (it + NS - 1 < nch) issue(it + NS - 1);   // refills the slot of stage it - 1
    const char* st = sm + (it % NS) * LY::SB;
#pragma unroll
    for (int kk = 0; kk < KSW; ++kk) {
    const int ks = kp * KSW + kk;
    // A: Q[r][16 ks + 8 lh .. + 7] (4 chunks of two complex values)
    shortx8 arh, arl, aih, ail;
    if (ADJ) {
      // A[r][k] = conj(Q[k][i0 + r]): down column r of the stage, k = 16 ks + 8 lh + q
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float2 v = *(const float2*)(st + (16 * ks + 8 * lh + q) * 1024 + r * 8);
        short h, l;
        split_h(v.x * kStackScale, h, l); arh[q] = h; arl[q] = l;
        split_h(-v.y * kStackScale, h, l); aih[q] = h; ail[q] = l;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = (8 * ks + 4 * lh + q) ^ (r % SW);
        const float4 v = *(const float4*)(st + r * LY::QROW + c * 16);
        short h, l;
        split_h(v.x * kStackScale, h, l); arh[2 * q] = h; arl[2 * q] = l;
        split_h(v.y * kStackScale, h, l); aih[2 * q] = h; ail[2 * q] = l;
        split_h(v.z * kStackScale, h, l); arh[2 * q + 1] = h; arl[2 * q + 1] = l;
        split_h(v.w * kStackScale, h, l); aih[2 * q + 1] = h; ail[2 * q + 1] = l;
      }
    }
    shortx8 bxrh[2], bxrl[2], bxih[2], bxil[2];
    if (PRE) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const char* xb = st + LY::QB + ((ks * 2 + c) * 2) * 1024 + 16 * lane;
        bxrh[c] = *(const shortx8*)xb;
        bxrl[c] = *(const shortx8*)(xb + 1024);
      }
    } else
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = 32 * c + l32;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 16 * ks + 8 * lh + j;
        short h, l;
        if (XC) {
          const float2 v = *(const float2*)(st + LY::QB + (k * 64 + col) * 8);
          split_h(v.x * xsc[c], h, l); bxrh[c][j] = h; bxrl[c][j] = l;
          split_h(v.y * xsc[c], h, l); bxih[c][j] = h; bxil[c][j] = l;
        } else {
          const float v = *(const float*)(st + LY::QB + (k * 64 + col) * 4);
          split_h(v * xsc[c], h, l); bxrh[c][j] = h; bxrl[c][j] = l;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const shortx8 xrh = bxrh[c], xrl = bxrl[c], xih = bxih[c], xil = bxil[c];
      acc_re[c] = mma(arh, xrh, acc_re[c]);
      acc_re[c] = mma(arh, xrl, acc_re[c]);
      acc_re[c] = mma(arl, xrh, acc_re[c]);
      acc_im[c] = mma(aih, xrh, acc_im[c]);
      acc_im[c] = mma(aih, xrl, acc_im[c]);
      acc_im[c] = mma(ail, xrh, acc_im[c]);
      if (XC) {
        const shortx8 naih = aih ^ (short)0x8000, nail = ail ^ (short)0x8000;
        acc_re[c] = mma(naih, xih, acc_re[c]);
        acc_re[c] = mma(naih, xil, acc_re[c]);
        acc_re[c] = mma(nail, xih, acc_re[c]);
        acc_im[c] = mma(arh, xih, acc_im[c]);
        acc_im[c] = mma(arh, xil, acc_im[c]);
        acc_im[c] = mma(arl, xih, acc_im[c]);
      }
    }
    }
  }
  // write back: lane holds signal b0 + 32c + l32, rows 32 rg + 8(e/4) + 4 lh + e%4.  With KSPL
  // parts, every wave leaves its sums in LDS and wave (rg, p) adds up the elements e of its
  // share, over the parts in order, for both signal blocks.
  constexpr int NV = YREAL ? 32 : 64;                 // values per lane: 2 blocks x 16 (re [, im])
  constexpr int EP = 16 / KSPL;                       // elements per wave in the share
  const size_t yoff = (size_t)a * N * B;
  if (KSPL > 1) {
    __syncthreads();   // every wave is done with the ring
    float* mine = (float*)sm + (size_t)wave * NV * 64;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        mine[(c * 16 + e) * 64 + lane] = acc_re[c][e];
        if (!YREAL) mine[(32 + c * 16 + e) * 64 + lane] = acc_im[c][e];
      }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int gb = b0 + 32 * c + l32;
    const float u = xs[gb].y * (1.0f / kStackScale);
#pragma unroll
    for (int j = 0; j < EP; ++j) {
      const int e = KSPL == 1 ? j : kp * EP + j;
      float vr, vi = 0.f;
      if (KSPL == 1) {
        vr = acc_re[c][j];
        if (!YREAL) vi = acc_im[c][j];
      } else {
        const float* part0 = (const float*)sm + (size_t)rg * NV * 64;
        vr = part0[(c * 16 + e) * 64 + lane];
        if (!YREAL) vi = part0[(32 + c * 16 + e) * 64 + lane];
#pragma unroll
        for (int p = 1; p < KSPL; ++p) {
          const float* pp = (const float*)sm + (size_t)(p * RG + rg) * NV * 64;
          vr = vr + pp[(c * 16 + e) * 64 + lane];
          if (!YREAL) vi = vi + pp[(32 + c * 16 + e) * 64 + lane];
        }
      }
      const int gi = i0 + 32 * rg + 8 * (e >> 2) + 4 * lh + (e & 3);
      if (gi < N) {
        const size_t off = yoff + (size_t)gi * B + gb;
        if (YREAL) ((float*)Y)[off] = vr * u;
        else ((cplx64*)Y)[off] = cplx64{vr * u, vi * u};
      }
    }
  }
}

// ---------------------------------------------------------------- signals split once
// One thread per (order, column block, k chunk, ks, c, lane): 8 values of column
// 64 cb + 32 c + l32 at k = 32 chunk + 16 ks + 8 lh .. + 7, scaled by the column's power of two
// (exact) and split into fp16 hi / lo (or bf16 hi / lo); 2 KB per (ks, c) pair of one k chunk
// (hi then lo).
template <bool BF>
__global__ __launch_bounds__(256) void k_xsplit(const float* __restrict__ X, int ldx, int ncols, int N, int ncb,
                                                size_t xstride, const float2* __restrict__ xs, int xs_stride,
                                                short* __restrict__ Xs) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int nch = N / 32, a = blockIdx.y;
  if (idx >= (size_t)ncb * nch * 256) return;
  const int lane = (int)(idx & 63), c = (int)((idx >> 6) & 1), ks = (int)((idx >> 7) & 1);
  const size_t bc = idx >> 8;                        // cb * nch + chunk
  const int chunk = (int)(bc % nch), cb = (int)(bc / nch);
  const int col = cb * 64 + 32 * c + (lane & 31);
  const int k0 = chunk * 32 + 16 * ks + 8 * (lane >> 5);
  const float* Xa = X + (size_t)a * xstride;
  const float sc = col < ncols ? xs[(size_t)a * xs_stride + col].x : 0.f;
  shortx8 h, l;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float v = col < ncols ? Xa[(size_t)(k0 + j) * ldx + col] * sc : 0.f;
    short hh, ll;
    if (BF) {
      const __bf16 bh = (__bf16)v;
      const __bf16 bl = (__bf16)(v - (float)bh);
      hh = __builtin_bit_cast(short, bh);
      ll = __builtin_bit_cast(short, bl);
    } else {
      split_h(v, hh, ll);
    }
    h[j] = hh;
    l[j] = ll;
  }
  shortx8* dst = (shortx8*)(Xs + ((((size_t)a * ncb * nch + bc) * 2 + ks) * 2 + c) * 2 * 64 * 8);
  dst[lane] = h;
  dst[64 + lane] = l;
}

size_t xsplit_bytes(int N, int nx, int ncols) {
  return align_up((size_t)nx * ceil_div(ncols, 64) * (N / 32) * 8192, 256);
}

fgfrft_status xsplit_launch(const float* X, int ldx, int ncols, int N, int nx, size_t xstride, const float2* xs,
                            int xs_stride, short* Xs, hipStream_t s, bool bf16) {
  const size_t n = (size_t)ceil_div(ncols, 64) * (N / 32) * 256;
  const dim3 g((unsigned)((n + 255) / 256), nx);
  if (bf16) k_xsplit<true><<<g, 256, 0, s>>>(X, ldx, ncols, N, ceil_div(ncols, 64), xstride, xs, xs_stride, Xs);
  else k_xsplit<false><<<g, 256, 0, s>>>(X, ldx, ncols, N, ceil_div(ncols, 64), xstride, xs, xs_stride, Xs);
  FG_LAUNCHED("signal split");
  return FGFRFT_OK;
}

size_t colscale_partial_bytes(int N, int nx, int B) { return align_up((size_t)nx * ceil_div(N, CR) * B * sizeof(float), 256); }

fgfrft_status colmax_launch(const void* X, int x_complex, int N, int B, int nx, float* partial, hipStream_t s) {
  k_colmax<<<dim3(ceil_div(B, 64) * nx, ceil_div(N, CR)), 256, 0, s>>>(X, x_complex, N, B, partial);
  FG_LAUNCHED("column maxima");
  return FGFRFT_OK;
}

fgfrft_status colscale_launch(const void* X, int x_complex, int N, int B, int nx, float2* scale, float* partial,
                              hipStream_t s) {
  const int nch = ceil_div(N, CR);
  k_colmax<<<dim3(ceil_div(B, 64) * nx, nch), 256, 0, s>>>(X, x_complex, N, B, partial);
  k_colscale<<<ceil_div(nx * B, 256), 256, 0, s>>>(partial, nch, B, nx, scale);
  FG_LAUNCHED("colscale");
  return FGFRFT_OK;
}

// Pre-split signals pay when the same signals are split by many workgroups: a block shared by
// every order, or many signals per order (each Q row block re-splits them once per 64 columns).
// Real signals are split into fp16 hi/lo once (k_xsplit) for the 64-wide streaming kernel and,
// with 32-wide stages, when a block is shared or wide; otherwise each wave splits its fragments.
static bool apply_presplit(int N, int B, int x_complex, int x_shared) {
  return !x_complex && N % 32 == 0 && B % 64 == 0 && (N % 64 == 0 || x_shared || B >= 256);
}

size_t apply_ws_bytes(int N, int n_alpha, int B, int x_shared) {
  const size_t nx = x_shared ? 1 : n_alpha;
  size_t b = align_up(nx * B * sizeof(float2), 256) + colscale_partial_bytes(N, (int)nx, B);
  if (apply_presplit(N, B, 0, x_shared)) b += xsplit_bytes(N, (int)nx, B);   // real signals only
  return b;
}

template <bool ADJ, bool XC, bool YR>
static void launch_apply_t(dim3 g, hipStream_t s, const cplx64* Q, int N, int n_alpha, const void* X, int x_shared,
                           int B, const float2* sc, void* Y, int nrb, int ncb) {
  k_apply<ADJ, XC, YR><<<g, 256, 0, s>>>(Q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb);
}

template <bool XC, bool YR, int NS, int K2, bool PRE = false, int RG = 4, int KSPL = 1, bool ADJ = false>
static void launch_apply2_t(hipStream_t s, const cplx64* Q, int N, int n_alpha, const void* X, int x_shared, int B,
                            const float2* sc, void* Y, int ncb) {
  constexpr int lds = NS * Apply2Layout<XC, K2, RG>::SB;
  static_assert(lds <= (RG * KSPL == 4 ? 80 : 160) * 1024, "two workgroups per CU (4 waves), else one");
  static_assert(KSPL == 1 || RG * KSPL * (YR ? 32 : 64) * 64 * 4 <= lds, "the parts' sums fit the ring");
  const int nrb = ceil_div(N, 32 * RG);
  const unsigned g = (unsigned)(8 * ceil_div(n_alpha, 8) * nrb * ncb);   // bounded by the caller
  (void)raise_lds_limit((const void*)k_apply2<XC, YR, NS, K2, PRE, RG, KSPL, ADJ>, lds);   // a failure surfaces at the launch
  k_apply2<XC, YR, NS, K2, PRE, RG, KSPL, ADJ><<<g, 64 * RG * KSPL, lds, s>>>(Q, N, n_alpha, X, x_shared, B, sc, Y, nrb, ncb);
}


// ---------------------------------------------------------------- real-F apply
// For real F the operator splits as Q = R + j sin(pi alpha) P with R = Re Q real and P = W W^T of
// rank r_minus1 (Definition 1 with real powers), so Y = R X + j sin(pi alpha) W (W^T X): the
// update writes R only (4 N^2 bytes per order instead of 8 N^2) and this apply streams it once.
//
// One pass over the real signals X [nx][N][B] for both things the real-F apply needs from them:
// the column maxima of a CR-row chunk (as k_colmax) and, for q < r, the chunk's part of
// Z[a][q][b] = (W^T X[a])[q][b] (W row-major [N][kWCols]).  Grid (column blocks x orders, row
// chunks); 4 row groups x 64 columns per workgroup, fixed-order sums over the row groups.
__global__ __launch_bounds__(256) void k_colmax_wtx(const float* __restrict__ X, int N, int B,
                                                    const float* __restrict__ W, int r, float* __restrict__ pmax,
                                                    float* __restrict__ pz) {
  __shared__ float red[4][kWCols + 1][64];
  const int ncb = (B + 63) / 64;
  const int a = blockIdx.x / ncb, ch = blockIdx.y, nch = gridDim.y;
  const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int b = (blockIdx.x % ncb) * 64 + c;
  float m = 0.f, acc[kWCols];
#pragma unroll
  for (int q = 0; q < kWCols; ++q) acc[q] = 0.f;
  if (b < B) {
    const int i1 = (ch + 1) * CR < N ? (ch + 1) * CR : N;
    for (int i = ch * CR + rg; i < i1; i += 4) {
      const float x = X[((size_t)a * N + i) * B + b];
      m = fmaxf(m, fabsf(x));
      const float4* w = (const float4*)(W + (size_t)i * kWCols);
#pragma unroll
      for (int q4 = 0; q4 < kWCols / 4; ++q4) {
        if (4 * q4 >= r) break;
        const float4 v = w[q4];
        acc[4 * q4] = fmaf(v.x, x, acc[4 * q4]);
        acc[4 * q4 + 1] = fmaf(v.y, x, acc[4 * q4 + 1]);
        acc[4 * q4 + 2] = fmaf(v.z, x, acc[4 * q4 + 2]);
        acc[4 * q4 + 3] = fmaf(v.w, x, acc[4 * q4 + 3]);
      }
    }
  }
  red[rg][kWCols][c] = m;
#pragma unroll
  for (int q = 0; q < kWCols; ++q) red[rg][q][c] = acc[q];
  __syncthreads();
  const size_t part = (size_t)a * nch + ch;
  if (rg == 0 && b < B)
    pmax[part * B + b] = fmaxf(fmaxf(red[0][kWCols][c], red[1][kWCols][c]), fmaxf(red[2][kWCols][c], red[3][kWCols][c]));
  for (int e = threadIdx.x; e < r * 64; e += 256) {
    const int q = e / 64, cc = e % 64, bb = (blockIdx.x % ncb) * 64 + cc;
    if (bb < B) pz[(part * r + q) * B + bb] = (red[0][q][cc] + red[1][q][cc]) + (red[2][q][cc] + red[3][q][cc]);
  }
}

// Z[a][q][b] = sum over the row chunks of the partials, in chunk order.
__global__ __launch_bounds__(256) void k_zsum(const float* __restrict__ pz, int nch, int r, int B, int nx,
                                              float* __restrict__ Z) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)nx * r * B) return;
  const int b = (int)(idx % B), q = (int)((idx / B) % r), a = (int)(idx / ((size_t)r * B));
  float s = 0.f;
  for (int c = 0; c < nch; ++c) s += pz[(((size_t)a * nch + c) * r + q) * B + b];
  Z[((size_t)a * kWCols + q) * B + b] = s;
}

// Y[a] = R[a] X[a] + j sin(pi alpha_a) W Z[a] for N % K2 == 0 and B % 64 == 0: the streaming
// kernel's structure (32 RG output rows x 64 signals per workgroup, RG x KSPL waves, direct-load
// LDS ring of NS stages of K2 k) with a real operator: a stage holds 32 RG rows x K2 of R (4 K2-byte
// row runs, 16-byte chunks swizzled by row) and the K2 rows of pre-split signals; per 16-wide k step
// a wave splits its R fragment once (2 parts) and issues 3 products per 32-signal block; with
// KSPL > 1 the k parts' sums are added once at the end through LDS in a fixed order.
template <int K2, int RG>
struct ApplyRealLayout {
  static constexpr int QB = 32 * RG * K2 * 4, XB = K2 * 64 * 4, SB = QB + XB;
  static constexpr int QROW = K2 * 4, CPR = QROW / 16, RPI = 1024 / QROW;
  static constexpr int SW = CPR < 16 ? CPR : 16;      // swizzle period (rows)
};

// X is the pre-split signal block of xsplit_launch (fp16 hi / lo parts in fragment order), so the
// waves read their signal fragments with plain 16-byte LDS loads.
// DXO: float32 output Y[a] = R[a] X[a] - sin(pi alpha_a) W Z[a] (the real part of Q[a] (X + j X'[a])
// when Z[a] = W^T X'[a]: the signal gradient for real signals, with the orders negated).
template <bool DXO, int K2, int NS, int RG, int KSPL>
__global__ __launch_bounds__(64 * RG * KSPL, RG * KSPL == 4 ? 2 : 1) void k_apply_real(
    const float* __restrict__ R, int N, int n_alpha, const void* __restrict__ X, int x_shared, int B,
    const float2* __restrict__ xscale, const double* __restrict__ alphas, const float* __restrict__ W, int r,
    const float* __restrict__ Z, void* __restrict__ Y, int nrb, int ncb) {
  using LY = ApplyRealLayout<K2, RG>;
  constexpr int CPR = LY::CPR, RPI = LY::RPI, SW = LY::SW, NW = RG * KSPL;
  constexpr int QLW = LY::QB / (1024 * NW), XLW = LY::XB / (1024 * NW), LW = QLW + XLW;   // loads per wave
  static_assert(QLW * 1024 * NW == LY::QB && XLW * 1024 * NW == LY::XB, "whole loads per wave");
  static_assert((RPI * NW) % SW == 0, "row swizzle constant per wave");
  static_assert(K2 % 32 == 0 && (K2 / 16) % KSPL == 0, "whole pre-split chunks, whole k steps per part");
  constexpr int KSW = K2 / 16 / KSPL;
  extern __shared__ __align__(16) char sm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  const int rg = wave % RG, kp = wave / RG;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int per_a = nrb * ncb;
  const int a = xcd + 8 * (slot / per_a);
  if (a >= n_alpha) return;
  const int rem = slot % per_a, rb = rem / ncb, cb = rem % ncb;
  const int i0 = rb * 32 * RG, b0 = cb * 64;
  const size_t NN = (size_t)N * N;
  const char* Ra = (const char*)(R + (size_t)a * NN);
  const float2* xs = xscale + (x_shared ? 0 : (size_t)a * B);
  const int nch = N / K2;

  // R instruction i (i = wave + NW q) moves rows i0 + RPI i .. + RPI - 1 (a row group past N: rows
  // N - RPI.., never written back); lane: row + lane / CPR, LDS chunk lane % CPR holds source chunk
  // (lane % CPR) ^ (row mod SW), the same for every q of a wave.
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int qrow = lane / CPR;
  const uint32_t qoff = (uint32_t)(((size_t)qrow * N + 4 * ((lane % CPR) ^ ((RPI * wv + qrow) % SW))) * 4);
  auto issue = [&](int it) {
    char* st = sm + (it % NS) * LY::SB;
    const int k0 = it * K2;
#pragma unroll
    for (int q = 0; q < QLW; ++q) {
      const int i = wv + NW * q;
      const int row0 = i0 + RPI * i < N ? i0 + RPI * i : N - RPI;
      lds_dma16(Ra + ((size_t)row0 * N + k0) * 4 + qoff, __builtin_amdgcn_readfirstlane(lds_addr(st + i * 1024)));
    }
#pragma unroll
    for (int q = 0; q < XLW; ++q) {
      const int i = wv + NW * q;
      const char* gb = (const char*)X + (((size_t)(x_shared ? 0 : a) * ncb + cb) * nch + it) * LY::XB + i * 1024;
      lds_dma16(gb + 16 * lane, __builtin_amdgcn_readfirstlane(lds_addr(st + LY::QB + i * 1024)));
    }
  };

  floatx16 acc[2] = {};
  const int rr = 32 * rg + l32;

  for (int it = 0; it < NS - 1 && it < nch; ++it) issue(it);
  for (int it = 0; it < nch; ++it) {
    if (it + NS - 1 <= nch) __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0((NS - 2) * LW));
    else __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
    barrier_nofence();
    if (it + NS - 1 < nch) issue(it + NS - 1);
    const char* st = sm + (it % NS) * LY::SB;
#pragma unroll
    for (int kk = 0; kk < KSW; ++kk) {
      const int ks = kp * KSW + kk;
      shortx8 arh, arl;
#pragma unroll
      for (int q = 0; q < 2; ++q) {   // R[rr][16 ks + 8 lh .. + 7]: two chunks of four reals
        const int c = (4 * ks + 2 * lh + q) ^ (rr % SW);
        const float4 v = *(const float4*)(st + rr * LY::QROW + c * 16);
        short h, l;
        split_h(v.x * kStackScale, h, l); arh[4 * q] = h; arl[4 * q] = l;
        split_h(v.y * kStackScale, h, l); arh[4 * q + 1] = h; arl[4 * q + 1] = l;
        split_h(v.z * kStackScale, h, l); arh[4 * q + 2] = h; arl[4 * q + 2] = l;
        split_h(v.w * kStackScale, h, l); arh[4 * q + 3] = h; arl[4 * q + 3] = l;
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const char* xb = st + LY::QB + ((ks * 2 + c) * 2) * 1024 + 16 * lane;
        const shortx8 xh = *(const shortx8*)xb;
        const shortx8 xl = *(const shortx8*)(xb + 1024);
        acc[c] = mma(arh, xh, acc[c]);
        acc[c] = mma(arh, xl, acc[c]);
        acc[c] = mma(arl, xh, acc[c]);
      }
    }
  }
  // write back: lane holds signal b0 + 32c + l32, rows 32 rg + 8(e/4) + 4 lh + e%4; the imaginary
  // part is sin(pi alpha) (W Z[a]) with the rank-r factor (zero when r = 0).  With KSPL parts every
  // wave leaves its sums in LDS and wave (rg, p) adds up the elements of its share in part order.
  constexpr int EP = 16 / KSPL;
  if (KSPL > 1) {
    __syncthreads();   // every wave is done with the ring
    float* mine = (float*)sm + (size_t)wave * 32 * 64;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 16; ++e) mine[(c * 16 + e) * 64 + lane] = acc[c][e];
    __syncthreads();
  }
  const float sn = r > 0 ? (float)sinpi(alphas[a]) : 0.f;
  const float* Za = Z + (size_t)(x_shared ? 0 : a) * kWCols * B;
  const size_t yoff = (size_t)a * N * B;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int gb = b0 + 32 * c + l32;
    const float u = xs[gb].y * (1.0f / kStackScale);
#pragma unroll
    for (int j = 0; j < EP; ++j) {
      const int e = KSPL == 1 ? j : kp * EP + j;
      float v;
      if (KSPL == 1) {
        v = acc[c][j];
      } else {
        v = ((const float*)sm)[((size_t)rg * 32 + c * 16 + e) * 64 + lane];
#pragma unroll
        for (int p = 1; p < KSPL; ++p) v = v + ((const float*)sm)[((size_t)(p * RG + rg) * 32 + c * 16 + e) * 64 + lane];
      }
      const int gi = i0 + 32 * rg + 8 * (e >> 2) + 4 * lh + (e & 3);
      if (gi < N) {
        float im = 0.f;
        for (int q = 0; q < r; ++q) im = fmaf(W[(size_t)gi * kWCols + q], Za[(size_t)q * B + gb], im);
        if (DXO) ((float*)Y)[yoff + (size_t)gi * B + gb] = v * u - sn * im;
        else ((cplx64*)Y)[yoff + (size_t)gi * B + gb] = cplx64{v * u, sn * im};
      }
    }
  }
}

// Launch of the real-operator apply.  N % 64 == 0 and B <= 128: 64-wide stages (256-byte R row runs),
// eight waves over two k parts, three stages of 48 KB, one workgroup per CU; else 32-wide stages,
// four waves, three stages of 24 KB, two workgroups per CU.  Measured on knn4096 (real-F call, 256 orders x 64
// signals): 8.10 against 8.21 ms; 64 rows x 128-wide stages (512-byte runs, two stages of 64 KB)
// 8.42 ms, 128 rows x 64-wide with two stages 8.42 ms.
template <bool DXO>
static fgfrft_status launch_apply_real(hipStream_t s, const float* R, int N, int n_alpha, const short* Xs,
                                       int x_shared, int B, const float2* sc, const double* alphas_dev,
                                       const float* W, int r, const float* Z, void* Y) {
  const int ncb = B / 64;
  auto go = [&](auto kern, int NS, int RG, int KSPL, int sb) -> fgfrft_status {
    const int nrb = ceil_div(N, 32 * RG), lds = NS * sb;
    const size_t nblocks = (size_t)8 * ceil_div(n_alpha, 8) * nrb * ncb;
    if (nblocks > 0x7fffffff) {
      set_error("apply grid too large");
      return FGFRFT_EUNSUPPORTED;
    }
    FG_HIP(raise_lds_limit((const void*)kern, lds));
    kern<<<(unsigned)nblocks, 64 * RG * KSPL, lds, s>>>(R, N, n_alpha, Xs, x_shared, B, sc, alphas_dev, W, r, Z, Y,
                                                        nrb, ncb);
    return FGFRFT_OK;
  };
  static_assert(3 * ApplyRealLayout<64, 4>::SB <= 160 * 1024 && 3 * ApplyRealLayout<32, 4>::SB <= 80 * 1024,
                "rings fit the LDS");
  static_assert(8 * 32 * 64 * 4 <= 3 * ApplyRealLayout<64, 4>::SB, "the parts' sums fit the ring");
  // as the complex-operator apply: the wide stages while the call is bound by the operators' bytes
  if (N % 64 == 0 && B <= 128) return go(k_apply_real<DXO, 64, 3, 4, 2>, 3, 4, 2, ApplyRealLayout<64, 4>::SB);
  return go(k_apply_real<DXO, 32, 3, 4, 1>, 3, 4, 1, ApplyRealLayout<32, 4>::SB);
}

size_t apply_real_ws_bytes(int N, int n_alpha, int B, int x_shared, int r) {
  const size_t nx = x_shared ? 1 : n_alpha;
  const size_t nch = ceil_div(N, CR);
  return align_up(nx * B * sizeof(float2), 256) + colscale_partial_bytes(N, (int)nx, B) +
         align_up(nx * kWCols * B * sizeof(float), 256) + align_up(nx * nch * (size_t)r * B * sizeof(float), 256) +
         xsplit_bytes(N, (int)nx, B);
}

bool apply_real_supported(const Plan* p, int x_complex, int B) {
  return !p->cplx && !x_complex && p->w_ok && p->N % 32 == 0 && B % 64 == 0;
}

fgfrft_status apply_real_launch(const Plan* p, const float* R, int n_alpha, const double* alphas_dev, const float* X,
                                int x_shared, int B, cplx64* Y, void* ws, hipStream_t s) {
  const int N = p->N, r = p->form == FGFRFT_FORM_SPLIT ? p->r_minus1 : 0;
  const int nx = x_shared ? 1 : n_alpha;
  const int nch = ceil_div(N, CR);
  float2* sc = (float2*)ws;
  float* partial = (float*)((char*)ws + align_up((size_t)nx * B * sizeof(float2), 256));
  float* Z = (float*)((char*)partial + colscale_partial_bytes(N, nx, B));
  float* pz = (float*)((char*)Z + align_up((size_t)nx * kWCols * B * sizeof(float), 256));
  short* Xs = (short*)((char*)pz + align_up((size_t)nx * nch * r * B * sizeof(float), 256));
  k_colmax_wtx<<<dim3(ceil_div(B, 64) * nx, nch), 256, 0, s>>>(X, N, B, p->W, r, partial, pz);
  k_colscale<<<ceil_div(nx * B, 256), 256, 0, s>>>(partial, nch, B, nx, sc);
  if (r > 0) k_zsum<<<(unsigned)(((size_t)nx * r * B + 255) / 256), 256, 0, s>>>(pz, nch, r, B, nx, Z);
  FG_LAUNCHED("signal scales and W^T X");
  // the signals are split into fp16 hi / lo once (one extra pass over X) rather than by each of the
  // four waves of every workgroup that reads them: 3.57 against 3.80 ms per knn4096 launch
  fgfrft_status rc = xsplit_launch(X, B, B, N, nx, x_shared ? 0 : (size_t)N * B, sc, B, Xs, s);
  if (rc) return rc;
  rc = launch_apply_real<false>(s, R, N, n_alpha, Xs, x_shared, B, sc, alphas_dev, p->W, r, Z, Y);
  if (rc) return rc;
  FG_LAUNCHED("apply (real operator)");
  return FGFRFT_OK;
}

// GY [n][N][B] complex64 -> its real and imaginary planes, float32 [n][N][B] each.
__global__ __launch_bounds__(256) void k_deinterleave(const float2* __restrict__ GY, size_t n, float* __restrict__ re,
                                                      float* __restrict__ im) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float2 v = GY[i];
    re[i] = v.x;
    im[i] = v.y;
  }
}

size_t apply_real_dx_ws_bytes(int N, int n_alpha, int B, int r) {
  const size_t nch = ceil_div(N, CR), plane = (size_t)n_alpha * N * B * sizeof(float);
  return 2 * align_up(plane, 256) + apply_real_ws_bytes(N, n_alpha, B, 0, r) + colscale_partial_bytes(N, n_alpha, B) +
         align_up((size_t)n_alpha * nch * B * sizeof(float), 256);
}

fgfrft_status apply_real_dx_launch(const Plan* p, const float* R, int n_alpha, const double* alphas_dev,
                                   const cplx64* GY, int B, float* dX, void* ws, hipStream_t s) {
  const int N = p->N, r = p->form == FGFRFT_FORM_SPLIT ? p->r_minus1 : 0;
  const int nch = ceil_div(N, CR);
  const size_t n = (size_t)n_alpha * N * B, plane = align_up(n * sizeof(float), 256);
  char* w = (char*)ws;
  float* gr = (float*)w;
  float* gi = (float*)(w + plane);
  char* aw = w + 2 * plane;                                  // the real-F apply's own workspace layout
  float2* sc = (float2*)aw;
  float* partial = (float*)(aw + align_up((size_t)n_alpha * B * sizeof(float2), 256));
  float* Z = (float*)((char*)partial + colscale_partial_bytes(N, n_alpha, B));
  float* pz = (float*)((char*)Z + align_up((size_t)n_alpha * kWCols * B * sizeof(float), 256));
  short* Xs = (short*)((char*)pz + align_up((size_t)n_alpha * nch * r * B * sizeof(float), 256));
  char* extra = aw + apply_real_ws_bytes(N, n_alpha, B, 0, r);
  float* partial_im = (float*)extra;                         // column maxima of the imaginary plane (unused)
  const unsigned g = (unsigned)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
  k_deinterleave<<<g, 256, 0, s>>>((const float2*)GY, n, gr, gi);
  // scales of the real plane (the apply's signals), then W^T of the imaginary plane
  k_colmax_wtx<<<dim3(ceil_div(B, 64) * n_alpha, nch), 256, 0, s>>>(gr, N, B, p->W, 0, partial, pz);
  k_colscale<<<ceil_div(n_alpha * B, 256), 256, 0, s>>>(partial, nch, B, n_alpha, sc);
  if (r > 0) {
    k_colmax_wtx<<<dim3(ceil_div(B, 64) * n_alpha, nch), 256, 0, s>>>(gi, N, B, p->W, r, partial_im, pz);
    k_zsum<<<(unsigned)(((size_t)n_alpha * r * B + 255) / 256), 256, 0, s>>>(pz, nch, r, B, n_alpha, Z);
  }
  FG_LAUNCHED("gradient planes, scales and W^T");
  fgfrft_status rc = xsplit_launch(gr, B, B, N, n_alpha, (size_t)N * B, sc, B, Xs, s);
  if (rc) return rc;
  rc = launch_apply_real<true>(s, R, N, n_alpha, Xs, 0, B, sc, alphas_dev, p->W, r, Z, dX);
  if (rc) return rc;
  FG_LAUNCHED("signal gradient (real operator)");
  return FGFRFT_OK;
}

fgfrft_status apply_launch(const void* Q, int N, int n_alpha, int adjoint, const void* X, int x_complex, int x_shared,
                           int B, void* Y, int y_real, void* ws, hipStream_t s) {
  float2* sc = (float2*)ws;
  const int nx = x_shared ? 1 : n_alpha;
  float* partial = (float*)((char*)ws + align_up((size_t)nx * B * sizeof(float2), 256));
  fgfrft_status rc = colscale_launch(X, x_complex, N, B, nx, sc, partial, s);
  if (rc) return rc;
  const bool pre = !adjoint && apply_presplit(N, B, x_complex, x_shared);
  short* Xs = (short*)((char*)partial + colscale_partial_bytes(N, nx, B));
  if (pre) {
    rc = xsplit_launch((const float*)X, B, B, N, nx, x_shared ? 0 : (size_t)N * B, sc, B, Xs, s);
    if (rc) return rc;
  }
  // streaming kernel: k stages of 32 (real signals, 2-stage ring) or 16 (complex, 3-stage ring)
  if (adjoint && N % (x_complex ? 16 : 32) == 0 && B % 64 == 0) {
    const int ncb = B / 64;
    if ((size_t)8 * ceil_div(n_alpha, 8) * ceil_div(N, 128) * ncb > 0x7fffffff) {
      set_error("apply grid too large");
      return FGFRFT_EUNSUPPORTED;
    }
    const cplx64* q = (const cplx64*)Q;
    switch ((x_complex ? 2 : 0) | (y_real ? 1 : 0)) {
      case 0: launch_apply2_t<false, false, 2, 32, false, 4, 1, true>(s, q, N, n_alpha, X, x_shared, B, sc, Y, ncb); break;
      case 1: launch_apply2_t<false, true, 2, 32, false, 4, 1, true>(s, q, N, n_alpha, X, x_shared, B, sc, Y, ncb); break;
      case 2: launch_apply2_t<true, false, 3, 16, false, 4, 1, true>(s, q, N, n_alpha, X, x_shared, B, sc, Y, ncb); break;
      case 3: launch_apply2_t<true, true, 3, 16, false, 4, 1, true>(s, q, N, n_alpha, X, x_shared, B, sc, Y, ncb); break;
    }
    FG_LAUNCHED("apply (adjoint)");
    return FGFRFT_OK;
  }
  if (!adjoint && N % (x_complex ? 16 : 32) == 0 && B % 64 == 0) {
    const int ncb = B / 64;
    const size_t nblocks = (size_t)8 * ceil_div(n_alpha, 8) * ceil_div(N, 64) * ncb;   // the largest grid below
    if (nblocks > 0x7fffffff) {
      set_error("apply grid too large");
      return FGFRFT_EUNSUPPORTED;
    }
    const cplx64* q = (const cplx64*)Q;
    // 64-wide k stages (512-byte Q row runs, one workgroup per CU) while the call is bound by the
    // operators' bytes (up to two 64-signal blocks); wider signal blocks re-read each operator from
    // the caches and are bound by the matrix cores, where two workgroups per CU with 32-wide stages
    // do better (32 operators x 1024 shared signals at N = 8192: 27.9 against 29.6 ms)
    const bool wide = N % 64 == 0 && B <= 128;
    if (pre) {
      if (wide && y_real) launch_apply2_t<false, true, 2, 64, true, 4, 2>(s, q, N, n_alpha, Xs, x_shared, B, sc, Y, ncb);
      else if (wide) launch_apply2_t<false, false, 2, 64, true, 4, 2>(s, q, N, n_alpha, Xs, x_shared, B, sc, Y, ncb);
      else if (y_real) launch_apply2_t<false, true, 2, 32, true>(s, q, N, n_alpha, Xs, x_shared, B, sc, Y, ncb);
      else launch_apply2_t<false, false, 2, 32, true>(s, q, N, n_alpha, Xs, x_shared, B, sc, Y, ncb);
      FG_LAUNCHED("apply");
      return FGFRFT_OK;
    }
    switch ((x_complex ? 2 : 0) | (y_real ? 1 : 0)) {
      case 0: launch_apply2_t<false, false, 2, 32>(s, q, N, n_alpha, X, x_shared, B, sc, Y, ncb); break;
      case 1: launch_apply2_t<false, true, 2, 32>(s, q, N, n_alpha, X, x_shared, B, sc, Y, ncb); break;
      case 2: launch_apply2_t<true, false, 3, 16>(s, q, N, n_alpha, X, x_shared, B, sc, Y, ncb); break;
      case 3: launch_apply2_t<true, true, 3, 16>(s, q, N, n_alpha, X, x_shared, B, sc, Y, ncb); break;
    }
    FG_LAUNCHED("apply");
    return FGFRFT_OK;
  }
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
