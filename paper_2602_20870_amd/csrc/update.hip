// Online stage of Algorithm 1: coefficients (Sec. III-A) and the operator update (Prop. 2)
//   Q[a] = e^{j pi alpha_a} P + c_0 P_c + sum_{n=1}^{L} ( c_n F^n P_c + c_{-n} F^{-n} P_c ),
// rewritten with P_c = I - P as
//   Q[a] = sum_{k} A[a][k] S_k + (e^{j pi alpha} - c_0) P + c_0 I,
// where S_k runs over the 2L resident matrices M_1..M_L, M_1^H..M_L^H.
//
// This is a contraction [n_alpha x 2L] . [2L x N^2] on the matrix cores.  A workgroup
// owns a strip of TR rows x 64 columns of positions: it stages the 2L stack tiles of the
// strip in LDS once, then its 4 waves produce those positions of Q for every order of the
// call (all waves on the same group of 32 orders at a time), so
// each stack element is read from HBM once per call and each store writes 256-byte runs
// of a row.  The P and identity terms ride in one extra MFMA k-step whose B operand is
// built in registers, so the epilogue is only the power-of-two unscale.
//
// Precision: each FP32 operand x is split into 16-bit parts hi = h(x), lo = h(x - hi);
// the products hi*hi + hi*lo + lo*hi accumulate in FP32.  With fp16 parts (after a 2^12
// scale) this keeps ~22 significant bits; with bf16 parts (BF16X2 stack) ~16 bits.
#include "internal.h"
#include <math.h>
#include <type_traits>

namespace fgfrft {

constexpr int TCOLS = 64;  // columns per strip

// ------------------------------------------------------------ coefficients (a-1)
__device__ __forceinline__ double sinc_pi(double x) { return x == 0.0 ? 1.0 : sinpi(x) / (M_PI * x); }

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

// Phase 1 stages the strip's 2L stack tiles in LDS as S[plane][pos][chunk] (chunk = 8 x 16-bit
// values; chunks 0..KP/8-1 hold the hi parts of S_0..S_{KP-1}, KP/8..KP/4-1 the lo parts; chunk
// index swizzled by position).  Phase 2 moves each wave's B fragments (its position block(s), all
// k) into registers.  Phase 3 reuses the LDS for the coefficient table of up to CAP orders,
// T[order][chunk] (same hi/lo chunking, swizzled by order) and E[order] = epi.  The order loop
// then reads only LDS, so nothing in it waits on the memory counter that the stores also use.
template <bool CPLX, int KP, int TR, bool BF, int NT, int MINW>
__global__ __launch_bounds__(NT, MINW) void k_update(const void* __restrict__ stack, const void* __restrict__ Pm, int N,
                                                   int L, int nJ, const uint16_t* __restrict__ table,
                                                   const float4* __restrict__ epi, int n_alpha, int n_pad,
                                                   cplx64* __restrict__ Q) {
  constexpr int NPL = CPLX ? 2 : 1;
  constexpr int CH = KP / 4, G8 = KP / 8, KS = KP / 16;
  constexpr int PT = TR * TCOLS;          // positions per strip
  constexpr int NBLK = PT / 32;           // 32-position MFMA column blocks
  constexpr int NW = NT / 64;             // waves
  constexpr int BPW = NBLK >= NW ? NBLK / NW : 1;   // blocks per wave
  constexpr int CAP = KP <= 64 ? 256 : 128;         // orders per LDS table chunk
  extern __shared__ __align__(16) shortx8 smem[];
  shortx8* S = smem;                                          // phase 1: [NPL][PT][CH]
  float* Pt = (float*)(smem + (size_t)NPL * PT * CH);         // phase 1: [PT][NPL]
  shortx8* T = smem;                                          // phase 3: [CAP][CH]
  float4* E = (float4*)(smem + (size_t)CAP * CH);             // phase 3: [CAP]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  const int I = blockIdx.x / nJ, J = blockIdx.x % nJ;
  const int row0 = I * TR, col0 = J * TCOLS;
  const size_t NN = (size_t)N * N;

  // ---- phase 1: stage the strip (unit = 8 consecutive stack matrices x V positions of one row,
  // V elements per 16-byte load; all loads of a thread are issued before any is used)
  constexpr int EB = CPLX ? 8 : 4;
  constexpr int V = 16 / EB;
  constexpr int NUNIT = (PT / V) * G8;
  constexpr int UPT = (NUNIT + NT - 1) / NT;
  {
    const bool vec_ok = (N % V) == 0;
    uint4 raw[UPT][8];
#pragma unroll
    for (int m = 0; m < UPT; ++m) {
      const int u = tid + NT * m;
      const int vq = u % (PT / V), g = u / (PT / V);
      const int p0 = vq * V;
      const int row = row0 + p0 / TCOLS, col = col0 + p0 % TCOLS;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = g * 8 + e;
        raw[m][e] = make_uint4(0, 0, 0, 0);
        if (u >= NUNIT || k >= 2 * L || row >= N) continue;
        const char* base = (const char*)stack + ((size_t)k * NN + (size_t)row * N + col) * EB;
        if (vec_ok && col + V <= N) {
          raw[m][e] = *(const uint4*)base;
        } else {
          uint32_t w[4] = {0, 0, 0, 0};
          for (int q = 0; q < V; ++q)
            if (col + q < N) {
              if (EB == 4) w[q] = ((const uint32_t*)base)[q];
              else { w[2 * q] = ((const uint32_t*)base)[2 * q]; w[2 * q + 1] = ((const uint32_t*)base)[2 * q + 1]; }
            }
          raw[m][e] = make_uint4(w[0], w[1], w[2], w[3]);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < UPT; ++m) {
      const int u = tid + NT * m;
      if (u >= NUNIT) continue;
      const int vq = u % (PT / V), g = u / (PT / V);
#pragma unroll
      for (int q = 0; q < V; ++q) {
        const int p = vq * V + q;
        shortx8 vh[NPL], vl[NPL];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t w[4] = {raw[m][e].x, raw[m][e].y, raw[m][e].z, raw[m][e].w};
#pragma unroll
          for (int pl = 0; pl < NPL; ++pl) {
            const uint32_t bits = w[q * NPL + pl];
            short h, l;
            if (BF) { h = (short)(bits & 0xffff); l = (short)(bits >> 16); }
            else split_f32<false>(__builtin_bit_cast(float, bits), h, l);
            vh[pl][e] = h;
            vl[pl][e] = l;
          }
        }
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) {
          shortx8* base = S + ((size_t)pl * PT + p) * CH;
          base[swz(p, g)] = vh[pl];
          base[swz(p, G8 + g)] = vl[pl];
        }
      }
    }
  }
  for (int p = tid; p < PT; p += NT) {
    const int row = row0 + p / TCOLS, col = col0 + p % TCOLS;
    const bool inb = row < N && col < N;
    if (CPLX) {
      const float2 v = inb ? ((const float2*)Pm)[(size_t)row * N + col] : make_float2(0.f, 0.f);
      Pt[p * 2] = v.x;
      Pt[p * 2 + 1] = v.y;
    } else {
      Pt[p] = inb ? ((const float*)Pm)[(size_t)row * N + col] : 0.f;
    }
  }
  __syncthreads();

  // ---- phase 2: this wave's B fragments (blocks wave + NW j) into registers
  shortx8 bh[BPW][NPL][KS], bl[BPW][NPL][KS], bxh[BPW], bxl[BPW];
#pragma unroll
  for (int j = 0; j < BPW; ++j) {
    const int blk = wave + NW * j < NBLK ? wave + NW * j : NBLK - 1;
    const int p = blk * 32 + l32;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const shortx8* rowS = S + ((size_t)pl * PT + p) * CH;
        bh[j][pl][ks] = rowS[swz(p, 2 * ks + lh)];
        bl[j][pl][ks] = rowS[swz(p, G8 + 2 * ks + lh)];
      }
    // extra k-step: (P_re, P_im, identity) at k = 0..2 for lanes lh == 0, zero elsewhere
    bxh[j] = shortx8{};
    bxl[j] = shortx8{};
    if (lh == 0) {
      const int row = row0 + p / TCOLS, col = col0 + p % TCOLS;
      const float pr = CPLX ? Pt[2 * p] : Pt[p];
      const float pi = CPLX ? Pt[2 * p + 1] : 0.f;
      short h, l;
      split_f32<BF>(pr, h, l);
      bxh[j][0] = h; bxl[j][0] = l;
      split_f32<BF>(pi, h, l);
      bxh[j][1] = h; bxl[j][1] = l;
      split_f32<BF>((row == col && row < N) ? 1.f : 0.f, h, l);
      bxh[j][2] = h; bxl[j][2] = l;
    }
  }
  const float unscale = BF ? 1.0f : kUnscale;
  const bool interior = row0 + TR <= N && col0 + TCOLS <= N;

  // ---- phase 3: orders in chunks of CAP through LDS
  for (int c0 = 0; c0 < n_pad; c0 += CAP) {
    const int ncap = n_pad - c0 < CAP ? n_pad - c0 : CAP;
    __syncthreads();   // previous users of the LDS are done
    // copy the table chunk in batches of 4 loads per thread, all in flight before any is used
    constexpr int TPT = CAP * CH / NT;
    static_assert(TPT % 4 == 0, "table copy batches");
    const shortx8* tsrc = (const shortx8*)(table + (size_t)c0 * 2 * KP);
#pragma unroll
    for (int b = 0; b < TPT; b += 4) {
      shortx8 v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int it = tid + NT * (b + q);
        v[q] = it / CH < ncap ? tsrc[it] : shortx8{};
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int it = tid + NT * (b + q), a = it / CH, c = it % CH;
        T[a * CH + swz(a, c)] = v[q];
      }
    }
    for (int a = tid; a < ncap; a += NT) E[a] = epi[c0 + a];
    __syncthreads();
    if (wave >= NBLK) continue;
    for (int g0 = 0; g0 < ncap; g0 += 32) {
      const int a0 = c0 + g0;
      const int al = g0 + l32;                 // this lane's order (A row), local index
      const bool fast = interior && a0 + 32 <= n_alpha;
#pragma unroll
      for (int j = 0; j < BPW; ++j) {
        const int blk = wave + NW * j;
        if (blk >= NBLK) break;
        const int p = blk * 32 + l32;
        floatx16 acc_re = {}, acc_im = {};
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) {
          floatx16 acc = {};
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            const shortx8 aH = T[al * CH + swz(al, 2 * ks + lh)];
            const shortx8 aL = T[al * CH + swz(al, G8 + 2 * ks + lh)];
            acc = mfma16<BF>(aH, bh[j][pl][ks], acc);
            acc = mfma16<BF>(aH, bl[j][pl][ks], acc);
            acc = mfma16<BF>(aL, bh[j][pl][ks], acc);
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
        acc_re = mfma16<BF>(xrH, bxh[j], acc_re);
        acc_re = mfma16<BF>(xrH, bxl[j], acc_re);
        acc_re = mfma16<BF>(xrL, bxh[j], acc_re);
        acc_im = mfma16<BF>(xiH, bxh[j], acc_im);
        acc_im = mfma16<BF>(xiH, bxl[j], acc_im);
        acc_im = mfma16<BF>(xiL, bxh[j], acc_im);
        // store: lane holds position p (column), orders a0 + 8(r/4) + 4 lh + r%4
        const int row = row0 + p / TCOLS, col = col0 + p % TCOLS;
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

template <bool CPLX, int KP, int TR, bool BF, int NT, int MINW>
static fgfrft_status launch_update_t(const Plan* p, const uint16_t* table, const float4* epi, int n_alpha, int n_pad,
                                     void* Q, hipStream_t s) {
  constexpr int NPL = CPLX ? 2 : 1;
  constexpr int CAP = KP <= 64 ? 256 : 128;
  const size_t lds_stage = (size_t)NPL * TR * TCOLS * (KP / 4) * 16 + (size_t)TR * TCOLS * NPL * 4;
  const size_t lds_table = (size_t)CAP * (KP / 4) * 16 + (size_t)CAP * 16;
  const size_t lds = lds_stage > lds_table ? lds_stage : lds_table;
  auto kern = k_update<CPLX, KP, TR, BF, NT, MINW>;
  static bool attr_set = false;
  if (!attr_set) {
    FG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_set = true;
  }
  const int nI = ceil_div(p->N, TR), nJ = ceil_div(p->N, TCOLS);
  kern<<<nI * nJ, NT, lds, s>>>(p->stack, p->P, p->N, p->L, nJ, table, epi, n_alpha, n_pad, (cplx64*)Q);
  FG_LAUNCHED("update");
  return FGFRFT_OK;
}

// (KP, TR): strips of TR rows x 64 columns sized so the staged tiles (and the order table)
// fit 64-68 KB of LDS, two workgroups of 4 waves per CU.
template <bool BF>
static fgfrft_status dispatch(const Plan* p, const uint16_t* table, const float4* epi, int n_alpha, int np, void* Q,
                              hipStream_t s) {
  const int KP = kp_of(p->L);
  if (!p->cplx) {
    switch (KP) {
      case 32: return launch_update_t<false, 32, 8, BF, 256, 2>(p, table, epi, n_alpha, np, Q, s);
      case 64: return launch_update_t<false, 64, 4, BF, 256, 2>(p, table, epi, n_alpha, np, Q, s);
      case 96: return launch_update_t<false, 96, 2, BF, 256, 2>(p, table, epi, n_alpha, np, Q, s);
      case 128: return launch_update_t<false, 128, 2, BF, 256, 2>(p, table, epi, n_alpha, np, Q, s);
    }
  } else {
    switch (KP) {
      case 32: return launch_update_t<true, 32, 4, BF, 256, 2>(p, table, epi, n_alpha, np, Q, s);
      case 64: return launch_update_t<true, 64, 2, BF, 256, 2>(p, table, epi, n_alpha, np, Q, s);
    }
  }
  set_error("unsupported L=%d for %s F", p->L, p->cplx ? "complex" : "real");
  return FGFRFT_EUNSUPPORTED;
}

fgfrft_status update_launch(const Plan* p, const double* alphas_dev, int n_alpha, void* Q, void* ws, hipStream_t s) {
  const int np = n_pad_of(n_alpha), KP = kp_of(p->L);
  char* base = (char*)ws + align_up((size_t)n_alpha * 8, 256);
  uint16_t* table = (uint16_t*)base;
  float4* epi = (float4*)(base + align_up((size_t)np * 2 * KP * 2, 256));
  fgfrft_status rc = coef_launch(p, alphas_dev, n_alpha, np, table, epi, 0, s);
  if (rc) return rc;
  return p->stacktype == FGFRFT_STACK_BF16X2 ? dispatch<true>(p, table, epi, n_alpha, np, Q, s)
                                             : dispatch<false>(p, table, epi, n_alpha, np, Q, s);
}

}  // namespace fgfrft
