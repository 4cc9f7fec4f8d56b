// Online stage of Algorithm 1: coefficients (Sec. III-A) and the operator update (Prop. 2)
//   Q[a] = e^{j pi alpha_a} P + c_0 P_c + sum_{n=1}^{L} ( c_n F^n P_c + c_{-n} F^{-n} P_c ),
// rewritten with P_c = I - P as
//   Q[a] = sum_{k} A[a][k] S_k + (e^{j pi alpha} - c_0) P + c_0 I,
// where S_k runs over the 2L resident matrices M_1..M_L, M_1^H..M_L^H.
//
// This is a contraction [n_alpha x 2L] . [2L x N^2] on the matrix cores.  A workgroup
// owns a strip of TR rows x 64 columns of positions: it stages the 2L stack tiles of the
// strip in LDS once (direct HBM-to-LDS loads), then its 4 waves produce those positions of
// Q for every order of the call (all waves on the same group of 32 orders at a time), so
// each stack element is read from HBM once per call.  With paired blocks each store instruction
// writes a 512-byte run of one row of one operator plane.  The P and identity
// terms ride in one extra MFMA k-step whose B operand is built in registers, so the
// epilogue is only the power-of-two unscale.
//
// Precision: each FP32 operand x is split into 16-bit parts hi = h(x), lo = h(x - hi);
// the products hi*hi + hi*lo + lo*hi accumulate in FP32.  With fp16 parts (after a 2^12
// scale) this keeps ~22 significant bits; with bf16 parts (BF16X2 stack) ~16 bits.
#include "internal.h"
#include <math.h>
#include <type_traits>

namespace fgfrft {


// ------------------------------------------------------------ coefficients (a-1)
template <bool BF>
__device__ __forceinline__ void split16(double v, uint16_t& hi, uint16_t& lo) {
  if (BF) {
    const float f = (float)v;
    const __bf16 h = (__bf16)f;
    const __bf16 l = (__bf16)(f - (float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  } else {
    const float f = (float)(v * (double)kCoefScale);
    const _Float16 h = (_Float16)f;
    const _Float16 l = (_Float16)(f - (float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  }
}

// Table row a (2 KP halves): [main hi (KP) | main lo (KP)] with main k < L: c_{k+1}(alpha),
// L <= k < 2L: c_{-(k-L+1)}(alpha), else 0.  epi[a] = (cos(pi a) - c_0, sin(pi a), c_0, 0):
// the coefficients of P and I (Re Q gains (cos - c_0) P_re - sin P_im + c_0 I, Im Q gains
// sin P_re + (cos - c_0) P_im).  Rows a >= n_alpha are zero.
template <bool BF>
__global__ __launch_bounds__(256) void k_coef(const double* __restrict__ alphas, int n_alpha, int n_pad, int L, int KP,
                                              uint16_t* __restrict__ table, float4* __restrict__ epi) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int a = idx / KP, k = idx % KP;
  if (a >= n_pad) return;
  const bool va = a < n_alpha;
  const double al = va ? alphas[a] : 0.0;
  const bool bad = va && !(fabs(al) < (double)L);   // only reachable through the device-order entry
  double c = 0.0;
  if (va && k < L) c = sinc_pi(al - (double)(k + 1));
  else if (va && k < 2 * L) c = sinc_pi(al + (double)(k - L + 1));
  if (bad) c = __builtin_nan("");
  uint16_t h, l;
  split16<BF>(c, h, l);
  uint16_t* row = table + (size_t)a * 2 * KP;
  row[k] = h;
  row[KP + k] = l;
  if (k == 0) {
    if (bad) {
      const float nan = __builtin_nanf("");
      epi[a] = make_float4(nan, nan, nan, 0.f);
    } else if (va) {
      const double c0 = sinc_pi(al);
      epi[a] = make_float4((float)(cospi(al) - c0), (float)sinpi(al), (float)c0, 0.f);
    } else {
      epi[a] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

// ------------------------------------------------------------ update kernel (a-2)
// s_waitcnt immediate (gfx9 encoding) that waits for vmcnt = 0 only (expcnt 7, lgkmcnt 15: no wait)
constexpr int kWaitVmcnt0 = 0x0F70;

__device__ __forceinline__ int swz(int p, int c) { return (c & ~7) | ((c ^ p) & 7); }

template <bool BF>
__device__ __forceinline__ floatx16 mfma16(shortx8 a, shortx8 b, floatx16 c) {
  if (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0, 0, 0);
}

// split one FP32 value into 16-bit hi/lo bit patterns (fp16 after the 2^12 scale, or bf16)
template <bool BF>
__device__ __forceinline__ void split_f32(float x, short& hi, short& lo) {
  if (BF) {
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    hi = __builtin_bit_cast(short, h);
    lo = __builtin_bit_cast(short, l);
  } else {
    const float v = x * kStackScale;
    const _Float16 h = (_Float16)v;
    const _Float16 l = (_Float16)(v - (float)h);
    hi = __builtin_bit_cast(short, h);
    lo = __builtin_bit_cast(short, l);
  }
}

// One group of 32 orders (a0 .. a0+31, local table index g0 ..) for one 32-position block:
// KS x 3 split products over the stack, 6 over the P/identity step, then 16 stores per lane
// (lane: position p = blk*32 + l32; orders a0 + 8(r/4) + 4 lh + r%4).
//
// OFF32: the per-lane part of the store address, (4 lh N^2 + row N + col) * 8 bytes, fits 32 bits
// (N <= 10240); the plane part is uniform, so every store is one scalar base plus one fixed 32-bit
// vector offset and no per-store 64-bit vector addresses are kept in registers.
//
// ROUT (real F only): the real plane alone, R = Re Q, is written as float32 [n_alpha][N][N]; for real
// F the imaginary plane is sin(pi alpha) P, which the real-F apply adds from the projector's factor.
template <bool CPLX, int KP, bool BF, bool OFF32, bool ROUT = false>
__device__ __forceinline__ void order_group(const shortx8* T, const float4* E, int g0, int a0, int n_alpha,
                                            bool fast, int row, int col, int N, size_t NN, int l32, int lh,
                                            const shortx8 (&bh)[CPLX ? 2 : 1][KP / 16],
                                            const shortx8 (&bl)[CPLX ? 2 : 1][KP / 16], shortx8 bxh, shortx8 bxl,
                                            void* __restrict__ Qv) {
  static_assert(!(ROUT && CPLX), "real-plane output needs a real F");
  constexpr int NPL = CPLX ? 2 : 1;
  constexpr int CH = KP / 4, G8 = KP / 8, KS = KP / 16;
  const float unscale = BF ? 1.0f : kUnscale;
  const int al = g0 + l32;   // this lane's order (A row), local index
  floatx16 acc_re = {}, acc_im = {};
#pragma unroll
  for (int pl = 0; pl < NPL; ++pl) {
    floatx16 acc = {};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const shortx8 aH = T[al * CH + swz(al, 2 * ks + lh)];
      const shortx8 aL = T[al * CH + swz(al, G8 + 2 * ks + lh)];
      acc = mfma16<BF>(aH, bh[pl][ks], acc);
      acc = mfma16<BF>(aH, bl[pl][ks], acc);
      acc = mfma16<BF>(aL, bh[pl][ks], acc);
    }
    if (pl == 0) acc_re = acc; else acc_im = acc;
  }
  // extra-step A rows: Re (cos - c_0, -sin, c_0), Im (sin, cos - c_0, 0) on k = 0..2
  shortx8 xrH = {}, xrL = {}, xiH = {}, xiL = {};
  if (lh == 0) {
    const float4 e = E[al];
    short h, l;
    split_f32<BF>(e.x, h, l); xrH[0] = h; xrL[0] = l; xiH[1] = h; xiL[1] = l;
    split_f32<BF>(-e.y, h, l); xrH[1] = h; xrL[1] = l;
    split_f32<BF>(e.y, h, l); xiH[0] = h; xiL[0] = l;
    split_f32<BF>(e.z, h, l); xrH[2] = h; xrL[2] = l;
  }
  acc_re = mfma16<BF>(xrH, bxh, acc_re);
  acc_re = mfma16<BF>(xrH, bxl, acc_re);
  acc_re = mfma16<BF>(xrL, bxh, acc_re);
  if constexpr (ROUT) {
    // lanes of a half-wave: 32 consecutive positions of one order's row (128-byte runs); the plane
    // offset walks in scalar registers, each store adds one fixed per-lane offset
    float* ql = (float*)Qv + (size_t)(a0 + 4 * lh) * NN + (size_t)row * N + col;
    if (fast) {
      const size_t plane = NN * sizeof(float);
      size_t po = (size_t)a0 * plane;
      const size_t vo = ((size_t)4 * lh * NN + (size_t)row * N + col) * sizeof(float);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float* dst = OFF32 ? (float*)((char*)Qv + po + (uint32_t)vo) : (float*)((char*)Qv + po + vo);
          __builtin_nontemporal_store(acc_re[4 * m + i] * unscale, dst);
          po += plane;
          asm volatile("" : "+s"(po));
        }
        po += 4 * plane;
        asm volatile("" : "+s"(po));
      }
    } else if (row < N && col < N) {
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (a0 + 8 * (r >> 2) + 4 * lh + (r & 3) < n_alpha) ql[(size_t)(8 * (r >> 2) + (r & 3)) * NN] = acc_re[r] * unscale;
    }
    return;
  }
  cplx64* __restrict__ Q = (cplx64*)Qv;
  acc_im = mfma16<BF>(xiH, bxh, acc_im);
  acc_im = mfma16<BF>(xiH, bxl, acc_im);
  acc_im = mfma16<BF>(xiL, bxh, acc_im);
  if (OFF32) {
    const uint32_t voff = (uint32_t)(((size_t)4 * lh * NN + (size_t)row * N + col) * sizeof(cplx64));
    char* qa = (char*)(Q + (size_t)a0 * NN);
    if (fast) {
#pragma unroll
      for (int r = 0; r < 16; ++r)
        *(cplx64*)(qa + (size_t)(8 * (r >> 2) + (r & 3)) * NN * sizeof(cplx64) + voff) =
            cplx64{acc_re[r] * unscale, acc_im[r] * unscale};
    } else if (row < N && col < N) {
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (a0 + 8 * (r >> 2) + 4 * lh + (r & 3) < n_alpha)
          *(cplx64*)(qa + (size_t)(8 * (r >> 2) + (r & 3)) * NN * sizeof(cplx64) + voff) =
              cplx64{acc_re[r] * unscale, acc_im[r] * unscale};
    }
  } else {
    cplx64* ql = Q + (size_t)(a0 + 4 * lh) * NN + (size_t)row * N + col;
    if (fast) {
#pragma unroll
      for (int r = 0; r < 16; ++r)
        ql[(size_t)(8 * (r >> 2) + (r & 3)) * NN] = cplx64{acc_re[r] * unscale, acc_im[r] * unscale};
    } else if (row < N && col < N) {
#pragma unroll
      for (int r = 0; r < 16; ++r)
        if (a0 + 8 * (r >> 2) + 4 * lh + (r & 3) < n_alpha)
          ql[(size_t)(8 * (r >> 2) + (r & 3)) * NN] = cplx64{acc_re[r] * unscale, acc_im[r] * unscale};
    }
  }
}

// ---- staging layout
// R[k][pos][plane] holds the strip's stack values exactly as stored in HBM (fp32, or one bf16
// hi/lo pair per real value), k < KP (rows 2L..KP-1 stay zero), followed by Pt[pos][plane] (fp32).
// The 16-bit split happens when a consumer moves its fragments into registers.
typedef __attribute__((address_space(3))) void lds_void;

// Interior strip whose rows start 16-byte aligned: every instruction moves 1 KB of R (64 lanes
// x 16 bytes) from HBM straight into LDS; producer wave pw of NPW issues instructions pw, pw+NPW, ..
template <bool CPLX, int TR, int TC, int NPW>
__device__ __forceinline__ void stage_direct(const void* __restrict__ stack, int N, int L, int row0, int col0, char* R,
                                             int pw, int lane) {
  constexpr int EB = CPLX ? 8 : 4, PT = TR * TC;
  const int ninst = 2 * L * PT * EB / 1024;      // 2L * PT * EB is a multiple of 1 KB (PT * EB >= 512)
  const size_t NN = (size_t)N * N;
  for (int i = pw; i < ninst; i += NPW) {
    const int e0 = (i * 1024 + 16 * lane) / EB;  // first element of this lane's 16 bytes in R
    const int k = e0 / PT, pos = e0 % PT;
    const char* g = (const char*)stack + ((size_t)k * NN + (size_t)(row0 + pos / TC) * N + col0 + pos % TC) * EB;
    __builtin_amdgcn_global_load_lds(g, (lds_void*)(R + i * 1024), 16, 0, 0);
  }
}

// Any strip (edges, unaligned N): element by element through registers, zero outside the matrix.
template <bool CPLX, int TR, int TC, int NTH>
__device__ __forceinline__ void stage_generic(const void* __restrict__ stack, int N, int L, int row0, int col0,
                                              char* R, int t) {
  constexpr int NPL = CPLX ? 2 : 1, PT = TR * TC;
  const size_t NN = (size_t)N * N;
  uint32_t* dst = (uint32_t*)R;
  const uint32_t* src = (const uint32_t*)stack;
  for (int e = t; e < 2 * L * PT; e += NTH) {
    const int k = e / PT, pos = e % PT;
    const int row = row0 + pos / TC, col = col0 + pos % TC;
    const bool inb = row < N && col < N;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl)
      dst[e * NPL + pl] = inb ? src[((size_t)k * NN + (size_t)row * N + col) * NPL + pl] : 0u;
  }
}

template <bool CPLX, int TR, int TC, int NTH>
__device__ __forceinline__ void stage_p(const void* __restrict__ Pm, int N, int row0, int col0, float* Pt, int t) {
  constexpr int NPL = CPLX ? 2 : 1, PT = TR * TC;
  for (int p = t; p < PT; p += NTH) {
    const int row = row0 + p / TC, col = col0 + p % TC;
    const bool inb = row < N && col < N;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) Pt[p * NPL + pl] = inb ? ((const float*)Pm)[((size_t)row * N + col) * NPL + pl] : 0.f;
  }
}

// B fragments for this lane's position p of the strip (all k, split into 16-bit parts) and the
// extra k-step operand (P_re, P_im, identity at k = 0..2 for lanes lh == 0, zero elsewhere).
// SM: stack storage (0 FP32, split here; 1 bf16 pairs; 2 fp16 pairs of the 2^12-scaled value, both
// used as stored).  The P tile is FP32 in every format.
template <bool CPLX, int KP, int TR, int TC, int SM>
__device__ __forceinline__ void load_fragments_raw(const uint32_t* R, const float* Pt, int N, int row0, int col0,
                                                   int p, int lh, shortx8 (&bh)[CPLX ? 2 : 1][KP / 16],
                                                   shortx8 (&bl)[CPLX ? 2 : 1][KP / 16], shortx8& bxh, shortx8& bxl) {
  constexpr int NPL = CPLX ? 2 : 1;
  constexpr int KS = KP / 16, PT = TR * TC;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 16 * ks + 8 * lh + j;
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl) {
        const uint32_t bits = R[((size_t)k * PT + p) * NPL + pl];
        short h, l;
        if (SM != 0) { h = (short)(bits & 0xffff); l = (short)(bits >> 16); }
        else split_f32<false>(__builtin_bit_cast(float, bits), h, l);
        bh[pl][ks][j] = h;
        bl[pl][ks][j] = l;
      }
    }
  bxh = shortx8{};
  bxl = shortx8{};
  if (lh == 0) {
    const int row = row0 + p / TC, col = col0 + p % TC;
    const float pr = CPLX ? Pt[2 * p] : Pt[p];
    const float pi = CPLX ? Pt[2 * p + 1] : 0.f;
    short h, l;
    split_f32<SM == 1>(pr, h, l);
    bxh[0] = h; bxl[0] = l;
    split_f32<SM == 1>(pi, h, l);
    bxh[1] = h; bxl[1] = l;
    split_f32<SM == 1>((row == col && row < N) ? 1.f : 0.f, h, l);
    bxh[2] = h; bxl[2] = l;
  }
}

template <bool CPLX, int KP, int TR, int TC, int CAP_ = (KP <= 64 ? 256 : 128)>
struct StripLayout {
  static constexpr int NPL = CPLX ? 2 : 1, PT = TR * TC, CH = KP / 4;
  static constexpr int CAP = CAP_;                                     // orders per LDS table chunk
  static constexpr size_t RB = (size_t)KP * PT * NPL * 4;              // raw stack tiles
  static constexpr size_t PB = ((size_t)PT * NPL * 4 + 15) / 16 * 16;  // P tile
  static constexpr size_t TB = (size_t)CAP * CH * 16;                  // coefficient table
  static constexpr size_t bytes = RB + PB + TB + (size_t)CAP * 16;      // + epilogue table
};

typedef float f32x2 __attribute__((ext_vector_type(2)));

// v_permlane32_swap: x's lanes 32..63 trade places with y's lanes 0..31.  The two results are
// copied out of the returned vector before the bit casts: this compiler lowers a bit cast of a
// vector element as a load from the vector's first element (both casts would read x's result).
__device__ __forceinline__ void swap_halves(float& x, float& y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                                  false, false);
  const unsigned rx = r[0], ry = r[1];
  x = __builtin_bit_cast(float, rx);
  y = __builtin_bit_cast(float, ry);
}

// Epilogue of one group of 32 orders for a lane's two neighbouring positions (col, col + 1 of
// row; lane half lh holds orders a0 + 8(r/4) + 4 lh + r%4 of accumulator element r).
template <bool OFF32>
__device__ __forceinline__ void store_pair(const floatx16& re0, const floatx16& im0, const floatx16& re1,
                                           const floatx16& im1, int a0, int n_alpha, bool fast, int row, int col,
                                           int N, size_t NN, int lh, float unscale, cplx64* __restrict__ Q) {
  if (fast) {   // interior, full group of orders, N even
    // Exchange half-waves so that each store instruction writes one order's whole 64-position row
    // run (512 contiguous bytes of one plane): after the swap, lane (l32, lh) holds position
    // col + lh of order 8m + i in (a, c) and of order 8m + 4 + i in (b, d), r = 4m + i.  The plane
    // offset advances by one plane per store and is pinned to scalar registers, so each store is
    // a uniform base plus one per-lane offset (no per-store 64-bit addresses held in vector
    // registers, which would leave too few for the fragments).
    const size_t plane = NN * sizeof(cplx64);
    size_t po = (size_t)a0 * plane;
    const size_t vo = ((size_t)row * N + col + lh) * sizeof(cplx64);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      float a[4], b[4], c[4], d[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = re0[4 * m + i] * unscale; b[i] = re1[4 * m + i] * unscale;
        c[i] = im0[4 * m + i] * unscale; d[i] = im1[4 * m + i] * unscale;
        swap_halves(a[i], b[i]);
        swap_halves(c[i], d[i]);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const f32x2 v = h == 0 ? f32x2{a[i], c[i]} : f32x2{b[i], d[i]};
          if (OFF32) __builtin_nontemporal_store(v, (f32x2*)((char*)Q + po + (uint32_t)vo));
          else __builtin_nontemporal_store(v, (f32x2*)((char*)Q + po + vo));
          po += plane;
          asm volatile("" : "+s"(po));
        }
    }
  } else if (row < N) {
    cplx64* ql = Q + (size_t)(a0 + 4 * lh) * NN + (size_t)row * N + col;
#pragma unroll
    for (int r = 0; r < 16; ++r)
      if (a0 + 8 * (r >> 2) + 4 * lh + (r & 3) < n_alpha) {
        cplx64* q = ql + (size_t)(8 * (r >> 2) + (r & 3)) * NN;
        if (col < N) q[0] = cplx64{re0[r] * unscale, im0[r] * unscale};
        if (col + 1 < N) q[1] = cplx64{re1[r] * unscale, im1[r] * unscale};
      }
  }
}

// Real-plane epilogue (ROUT): lane l32 holds positions col, col + 1 of orders a0 + 8(r/4) + 4 lh + r%4
// in (re0[r], re1[r]); each store instruction writes one 256-byte row run in each of two planes.
template <bool OFF32>
__device__ __forceinline__ void store_pair_real(const floatx16& re0, const floatx16& re1, int a0, int n_alpha,
                                                bool fast, int row, int col, int N, size_t NN, int lh, float unscale,
                                                float* __restrict__ R) {
  if (fast) {
    const size_t plane = NN * sizeof(float);
    size_t po = (size_t)a0 * plane;
    const size_t vo = ((size_t)4 * lh * NN + (size_t)row * N + col) * sizeof(float);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const f32x2 v = f32x2{re0[4 * m + i] * unscale, re1[4 * m + i] * unscale};
        if (OFF32) __builtin_nontemporal_store(v, (f32x2*)((char*)R + po + (uint32_t)vo));
        else __builtin_nontemporal_store(v, (f32x2*)((char*)R + po + vo));
        po += plane;
        asm volatile("" : "+s"(po));
      }
      po += 4 * plane;
      asm volatile("" : "+s"(po));
    }
  } else if (row < N) {
    float* ql = R + (size_t)(a0 + 4 * lh) * NN + (size_t)row * N + col;
#pragma unroll
    for (int r = 0; r < 16; ++r)
      if (a0 + 8 * (r >> 2) + 4 * lh + (r & 3) < n_alpha) {
        float* q = ql + (size_t)(8 * (r >> 2) + (r & 3)) * NN;
        if (col < N) q[0] = re0[r] * unscale;
        if (col + 1 < N) q[1] = re1[r] * unscale;
      }
  }
}

// Two 32-position blocks whose lanes hold the even (block 0) and odd (block 1) position of one
// column pair: the same MFMA sequence per block as order_group; a half-wave exchange then gives each
// lane one position of two orders, so every store instruction writes one order's 64-position row
// run (512 contiguous bytes of a single plane; against two 512-byte runs in planes four orders apart
// the stores alone stream 7% faster and the whole kernel runs 2% faster).  The operator planes are
// streamed out with nontemporal stores (they are far larger than the caches).
template <bool CPLX, int KP, bool BF, bool OFF32, bool ROUT = false>
__device__ __forceinline__ void order_pair(const shortx8* T, const float4* E, int g0, int a0, int n_alpha, bool fast,
                                           int row, int col, int N, size_t NN, int l32, int lh,
                                           const shortx8 (&bh0)[CPLX ? 2 : 1][KP / 16],
                                           const shortx8 (&bl0)[CPLX ? 2 : 1][KP / 16], shortx8 bxh0, shortx8 bxl0,
                                           const shortx8 (&bh1)[CPLX ? 2 : 1][KP / 16],
                                           const shortx8 (&bl1)[CPLX ? 2 : 1][KP / 16], shortx8 bxh1, shortx8 bxl1,
                                           void* __restrict__ Q) {
  static_assert(!(ROUT && CPLX), "real-plane output needs a real F");
  constexpr int NPL = CPLX ? 2 : 1;
  constexpr int CH = KP / 4, G8 = KP / 8, KS = KP / 16;
  const float unscale = BF ? 1.0f : kUnscale;
  const int al = g0 + l32;
  floatx16 re0 = {}, im0 = {}, re1 = {}, im1 = {};
#pragma unroll
  for (int pl = 0; pl < NPL; ++pl) {
    floatx16 c0 = {}, c1 = {};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const shortx8 aH = T[al * CH + swz(al, 2 * ks + lh)];
      const shortx8 aL = T[al * CH + swz(al, G8 + 2 * ks + lh)];
      c0 = mfma16<BF>(aH, bh0[pl][ks], c0);
      c1 = mfma16<BF>(aH, bh1[pl][ks], c1);
      c0 = mfma16<BF>(aH, bl0[pl][ks], c0);
      c1 = mfma16<BF>(aH, bl1[pl][ks], c1);
      c0 = mfma16<BF>(aL, bh0[pl][ks], c0);
      c1 = mfma16<BF>(aL, bh1[pl][ks], c1);
    }
    if (pl == 0) { re0 = c0; re1 = c1; } else { im0 = c0; im1 = c1; }
  }
  shortx8 xrH = {}, xrL = {}, xiH = {}, xiL = {};
  if (lh == 0) {
    const float4 e = E[al];
    short h, l;
    split_f32<BF>(e.x, h, l); xrH[0] = h; xrL[0] = l; xiH[1] = h; xiL[1] = l;
    split_f32<BF>(-e.y, h, l); xrH[1] = h; xrL[1] = l;
    split_f32<BF>(e.y, h, l); xiH[0] = h; xiL[0] = l;
    split_f32<BF>(e.z, h, l); xrH[2] = h; xrL[2] = l;
  }
  re0 = mfma16<BF>(xrH, bxh0, re0); re1 = mfma16<BF>(xrH, bxh1, re1);
  re0 = mfma16<BF>(xrH, bxl0, re0); re1 = mfma16<BF>(xrH, bxl1, re1);
  re0 = mfma16<BF>(xrL, bxh0, re0); re1 = mfma16<BF>(xrL, bxh1, re1);
  if constexpr (ROUT) {
    store_pair_real<OFF32>(re0, re1, a0, n_alpha, fast, row, col, N, NN, lh, unscale, (float*)Q);
    return;
  }
  im0 = mfma16<BF>(xiH, bxh0, im0); im1 = mfma16<BF>(xiH, bxh1, im1);
  im0 = mfma16<BF>(xiH, bxl0, im0); im1 = mfma16<BF>(xiH, bxl1, im1);
  im0 = mfma16<BF>(xiL, bxh0, im0); im1 = mfma16<BF>(xiL, bxh1, im1);
  store_pair<OFF32>(re0, im0, re1, im1, a0, n_alpha, fast, row, col, N, NN, lh, unscale, (cplx64*)Q);
}

// Table chunk of ncap orders into LDS with direct HBM/L2-to-LDS loads: LDS 16-byte chunk m =
// a * CH + c' receives table chunk a * CH + swz(a, c') (the swizzle is its own inverse), so a
// lane's destination is contiguous per instruction as the direct loads require.  Rows past ncap
// are not loaded (never read).  Wave w of NW.
template <int KP, int NW>
__device__ __forceinline__ void load_table_direct(const uint16_t* __restrict__ table, int c0, int ncap, shortx8* T,
                                                  int w, int lane) {
  constexpr int CH = KP / 4;
  const shortx8* tsrc = (const shortx8*)(table + (size_t)c0 * 2 * KP);
  const int nchunk = ncap * CH;                 // multiple of 64 (ncap is a multiple of 32, CH of 8)
  for (int i = w; i * 64 < nchunk; i += NW) {
    const int m = i * 64 + lane, a = m / CH, c = m % CH;
    __builtin_amdgcn_global_load_lds((const void*)(tsrc + a * CH + swz(a, c)), (lds_void*)(T + i * 64), 16, 0, 0);
  }
}

// Operator update kernel: one workgroup per strip of TR x 64 positions (two per CU).  It stages the
// strip's 2L stack tiles in LDS with direct loads, moves each wave's B fragments into registers,
// then reuses the LDS for the coefficient table, CAP orders at a time, and runs the order loop,
// which touches only LDS, the matrix cores and stores: nothing in it waits on the memory counter
// the stores also use, so the stores stream without drains.
template <bool CPLX, int KP, int TR, int TC, int SM, int NT, int MINW, bool OFF32, int CAPV, bool PAIR, bool ROUT>
__global__ __launch_bounds__(NT, MINW) void k_update_strip(const void* __restrict__ stack, const void* __restrict__ Pm,
                                                           int N, int L, int nJ, const uint16_t* __restrict__ table,
                                                           const float4* __restrict__ epi, int n_alpha, int n_pad,
                                                           void* __restrict__ Q) {
  using LY = StripLayout<CPLX, KP, TR, TC, CAPV>;
  constexpr int NPL = LY::NPL, CH = LY::CH, KS = KP / 16, PT = LY::PT, CAP = LY::CAP;
  constexpr int NW = NT / 64, NBLK = PT / 32, BPW = NBLK >= NW ? NBLK / NW : 1;
  constexpr bool BF = SM == 1;   // bf16 matrix cores for a BF16X2 stack, fp16 otherwise
  extern __shared__ __align__(16) shortx8 smem[];
  char* R = (char*)smem;
  float* Pt = (float*)(R + LY::RB);
  shortx8* T = smem;
  float4* E = (float4*)(T + CAP * CH);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  const int I = blockIdx.x / nJ, J = blockIdx.x % nJ;
  const int row0 = I * TR, col0 = J * TC;
  const size_t NN = (size_t)N * N;
  const bool interior = row0 + TR <= N && col0 + TC <= N;

  for (int e = tid; e < (KP - 2 * L) * PT * NPL; e += NT) ((uint32_t*)R)[2 * L * PT * NPL + e] = 0u;
  if (((size_t)N * (CPLX ? 8 : 4)) % 16 == 0 && interior) stage_direct<CPLX, TR, TC, NW>(stack, N, L, row0, col0, R, wave, lane);
  else stage_generic<CPLX, TR, TC, NT>(stack, N, L, row0, col0, R, tid);
  stage_p<CPLX, TR, TC, NT>(Pm, N, row0, col0, Pt, tid);
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __syncthreads();
  // PAIR: the strip is cut into 64-column row segments (TC / 64 per row); wave w owns segments
  // w * BPW/2 .. (BPW/2 per wave), and block j holds the positions of segment w * BPW/2 + j/2 with
  // column parity j & 1.  Otherwise block j is positions (wave + NW j) * 32 + 0..31.
  static_assert(!PAIR || (BPW % 2 == 0 && NW * BPW / 2 * 64 == TR * TC && TC % 64 == 0),
                "paired blocks cover the strip in 64-column row segments");
  auto pos_of = [&](int j) {
    if (PAIR) return (wave * (BPW / 2) + j / 2) * 64 + 2 * l32 + (j & 1);
    const int blk = wave + NW * j < NBLK ? wave + NW * j : NBLK - 1;
    return blk * 32 + l32;
  };
  shortx8 bh[BPW][NPL][KS], bl[BPW][NPL][KS], bxh[BPW], bxl[BPW];
#pragma unroll
  for (int j = 0; j < BPW; ++j)
    load_fragments_raw<CPLX, KP, TR, TC, SM>((const uint32_t*)R, Pt, N, row0, col0, pos_of(j), lh, bh[j], bl[j], bxh[j],
                                         bxl[j]);
  for (int c0 = 0; c0 < n_pad; c0 += CAP) {
    const int ncap = n_pad - c0 < CAP ? n_pad - c0 : CAP;
    __syncthreads();   // previous users of the LDS are done
    load_table_direct<KP, NW>(table, c0, ncap, T, wave, lane);
    for (int a = tid; a < ncap; a += NT) E[a] = epi[c0 + a];
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (wave >= NBLK) continue;
    for (int g0 = 0; g0 < ncap; g0 += 32) {
      const int a0 = c0 + g0;
      const bool fast = interior && a0 + 32 <= n_alpha;
      if constexpr (PAIR) {
#pragma unroll
        for (int j = 0; j < BPW; j += 2) {
          const int p = pos_of(j);
          order_pair<CPLX, KP, BF, OFF32, ROUT>(T, E, g0, a0, n_alpha, fast && (N % 2) == 0, row0 + p / TC,
                                          col0 + p % TC, N, NN, l32, lh, bh[j], bl[j], bxh[j], bxl[j], bh[j + 1],
                                          bl[j + 1], bxh[j + 1], bxl[j + 1], Q);
        }
      } else {
#pragma unroll
        for (int j = 0; j < BPW; ++j) {
          const int blk = wave + NW * j;
          if (blk >= NBLK) break;
          const int p = blk * 32 + l32;
          order_group<CPLX, KP, BF, OFF32, ROUT>(T, E, g0, a0, n_alpha, fast, row0 + p / TC, col0 + p % TC, N, NN,
                                           l32, lh, bh[j], bl[j], bxh[j], bxl[j], Q);
        }
      }
    }
  }
}

// ------------------------------------------------------------ host side
static int n_pad_of(int n_alpha) { return ceil_div(n_alpha, 32) * 32; }
static int kp_of(int L) { return ceil_div(2 * L, 32) * 32; }

size_t update_ws_bytes(const Plan* p, int n_alpha) {
  const int np = n_pad_of(n_alpha), KP = kp_of(p->L);
  return align_up((size_t)n_alpha * 8, 256) + align_up((size_t)np * 2 * KP * 2, 256) + align_up((size_t)np * 16, 256);
}

fgfrft_status coef_launch(const Plan* p, const double* alphas_dev, int n_alpha, int n_pad, void* table, float4* epi,
                          int, hipStream_t s) {
  const int KP = kp_of(p->L);
  const int total = n_pad * KP;
  const bool bf = p->stacktype == FGFRFT_STACK_BF16X2;
  if (bf) k_coef<true><<<ceil_div(total, 256), 256, 0, s>>>(alphas_dev, n_alpha, n_pad, p->L, KP, (uint16_t*)table, epi);
  else k_coef<false><<<ceil_div(total, 256), 256, 0, s>>>(alphas_dev, n_alpha, n_pad, p->L, KP, (uint16_t*)table, epi);
  FG_LAUNCHED("coef");
  return FGFRFT_OK;
}

template <bool CPLX, int KP, int TR, int TC, int SM, int NT, int MINW, int CAPV = (KP <= 64 ? 256 : 128), bool PAIR = false,
          bool ROUT = false>
static fgfrft_status launch_update_strip(const Plan* p, const uint16_t* table, const float4* epi, int n_alpha,
                                         int n_pad, void* Q, hipStream_t s) {
  using LY = StripLayout<CPLX, KP, TR, TC, CAPV>;
  constexpr size_t lds = LY::RB + LY::PB > LY::TB + (size_t)LY::CAP * 16 ? LY::RB + LY::PB : LY::TB + (size_t)LY::CAP * 16;
  static_assert(lds <= 160 * 1024, "LDS budget");
  const bool off32 = (size_t)5 * p->N * p->N * sizeof(cplx64) < ((size_t)1 << 32);
  auto kern = off32 ? k_update_strip<CPLX, KP, TR, TC, SM, NT, MINW, true, CAPV, PAIR, ROUT>
                    : k_update_strip<CPLX, KP, TR, TC, SM, NT, MINW, false, CAPV, PAIR, ROUT>;
  FG_HIP(raise_lds_limit((const void*)kern, (int)lds));
  const int nI = ceil_div(p->N, TR), nJ = ceil_div(p->N, TC);
  kern<<<nI * nJ, NT, lds, s>>>(p->stack, p->P, p->N, p->L, nJ, table, epi, n_alpha, n_pad, Q);
  FG_LAUNCHED("update");
  return FGFRFT_OK;
}

// (KP, TR, pairing): strips of TR rows x 64 columns; the staged tiles, and then the order table
// (up to 256 orders for KP <= 64, 128 beyond), fit 64-68 KB of LDS, two workgroups of 4 waves per CU.
template <int SM, bool ROUT = false>
static fgfrft_status dispatch(const Plan* p, const uint16_t* table, const float4* epi, int n_alpha, int np, void* Q,
                              hipStream_t s) {
  const int KP = kp_of(p->L);
  if (!p->cplx) {
    switch (KP) {
      case 32: return launch_update_strip<false, 32, 8, 64, SM, 256, 2, 256, false, ROUT>(p, table, epi, n_alpha, np, Q, s);
      case 64: return launch_update_strip<false, 64, 4, 64, SM, 256, 2, 256, true, ROUT>(p, table, epi, n_alpha, np, Q, s);
      case 96: return launch_update_strip<false, 96, 2, 64, SM, 256, 2, 128, false, ROUT>(p, table, epi, n_alpha, np, Q, s);
      case 128: return launch_update_strip<false, 128, 2, 64, SM, 256, 2, 128, false, ROUT>(p, table, epi, n_alpha, np, Q, s);
    }
  } else if constexpr (!ROUT) {
    switch (KP) {
      case 32: return launch_update_strip<true, 32, 4, 64, SM, 256, 2, 256, true>(p, table, epi, n_alpha, np, Q, s);
      case 64: return launch_update_strip<true, 64, 2, 64, SM, 256, 2, 256, false>(p, table, epi, n_alpha, np, Q, s);
      // 32 < L <= 64: one-row strips (two of the four waves run the order loop)
      case 96: return launch_update_strip<true, 96, 1, 64, SM, 256, 2, 128, false>(p, table, epi, n_alpha, np, Q, s);
      case 128: return launch_update_strip<true, 128, 1, 64, SM, 256, 2, 128, false>(p, table, epi, n_alpha, np, Q, s);
    }
  }
  set_error("unsupported L=%d for %s F", p->L, p->cplx ? "complex" : "real");
  return FGFRFT_EUNSUPPORTED;
}

fgfrft_status update_launch(const Plan* p, const double* alphas_dev, int n_alpha, void* Q, void* ws, hipStream_t s,
                            bool real_plane) {
  if (real_plane && p->cplx) {
    set_error("the real-plane update needs a real F");
    return FGFRFT_EUNSUPPORTED;
  }
  const int np = n_pad_of(n_alpha), KP = kp_of(p->L);
  char* base = (char*)ws + align_up((size_t)n_alpha * 8, 256);
  uint16_t* table = (uint16_t*)base;
  float4* epi = (float4*)(base + align_up((size_t)np * 2 * KP * 2, 256));
  fgfrft_status rc = coef_launch(p, alphas_dev, n_alpha, np, table, epi, 0, s);
  if (rc) return rc;
  switch (p->stacktype) {
    case FGFRFT_STACK_BF16X2:
      return real_plane ? dispatch<1, true>(p, table, epi, n_alpha, np, Q, s) : dispatch<1>(p, table, epi, n_alpha, np, Q, s);
    case FGFRFT_STACK_FP16X2:
      return real_plane ? dispatch<2, true>(p, table, epi, n_alpha, np, Q, s) : dispatch<2>(p, table, epi, n_alpha, np, Q, s);
    default:
      return real_plane ? dispatch<0, true>(p, table, epi, n_alpha, np, Q, s) : dispatch<0>(p, table, epi, n_alpha, np, Q, s);
  }
}

}  // namespace fgfrft
