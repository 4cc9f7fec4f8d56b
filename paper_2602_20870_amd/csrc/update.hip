// Online stage of Algorithm 1: coefficients (Sec. III-A) and the operator update
//   Q[a] = e^{j pi alpha_a} P + c_0 P_c + sum_{n=1}^{L} ( c_n M_n + c_{-n} M_n^H )     (Prop. 2)
// computed as  c_0 I + (e^{j pi alpha} - c_0) P + sum_n c_n M_n + sum_n c_{-n} M_n^H  (P_c = I - P).
//
// The two sums form a contraction [n_alpha x 2L] . [2L x N^2] that runs on the
// matrix cores.  A workgroup owns a tile pair {(I,J), (J,I)} of 16x16 positions:
// it stages the L power-stack tiles of both blocks in LDS once (so M_n^H never
// needs its own copy: the transposed partner tile supplies it) and then produces
// those positions of Q for every order of the call, so each stack tile is read
// from HBM exactly once per call.
//
// Precision: each FP32 operand x is split into 16-bit parts hi = h(x),
// lo = h(x - hi); the products hi*hi + hi*lo + lo*hi accumulate in FP32.  With
// fp16 parts (after a 2^12 scale) this keeps ~22 significant bits, with bf16
// parts (the pre-split BF16X2 stack) ~16 bits.
#include "internal.h"
#include <math.h>

namespace fgfrft {

constexpr int TT = 16;           // tile edge
constexpr int TPOS = TT * TT;    // positions per tile

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

// table row a (4*LP halves): [c_n hi | c_n lo | c_{-n} hi | c_{-n} lo], n = 1..L at k = n-1,
// zero for k >= L and for padded rows a >= n_alpha.
// epi[a] = (c_0, cos(pi alpha) - c_0, sin(pi alpha), 0).
template <bool BF>
__global__ __launch_bounds__(256) void k_coef(const double* __restrict__ alphas, int n_alpha, int n_pad, int L, int LP,
                                              uint16_t* __restrict__ table, float4* __restrict__ epi) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int a = idx / LP, k = idx % LP;
  if (a >= n_pad) return;
  const bool va = a < n_alpha;
  const double al = va ? alphas[a] : 0.0;
  const bool vk = va && k < L;
  const double cp = vk ? sinc_pi(al - (double)(k + 1)) : 0.0;
  const double cn = vk ? sinc_pi(al + (double)(k + 1)) : 0.0;
  uint16_t h, l;
  uint16_t* row = table + (size_t)a * 4 * LP;
  split16<BF>(cp, h, l);
  row[k] = h;
  row[LP + k] = l;
  split16<BF>(cn, h, l);
  row[2 * LP + k] = h;
  row[3 * LP + k] = l;
  if (k == 0) {
    if (va) {
      const double c0 = sinc_pi(al);
      epi[a] = make_float4((float)c0, (float)(cospi(al) - c0), (float)sinpi(al), 0.0f);
    } else {
      epi[a] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

// ------------------------------------------------------------ update kernel (a-2)
__device__ __forceinline__ int swz(int p, int c) { return (c & ~7) | ((c ^ (p ^ (p >> 4))) & 7); }

template <bool BF>
__device__ __forceinline__ floatx16 mfma16(shortx8 a, shortx8 b, floatx16 c) {
  if (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0, 0, 0);
}

// split one FP32 value (scaled for fp16) into 16-bit hi/lo bit patterns
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

// LDS: S[tile][plane][pos][chunk] with chunk = 8 x 16-bit values; chunks 0..LP/8-1 hold hi parts of
// n = 1..LP, chunks LP/8..LP/4-1 the lo parts.  Chunk index swizzled per position (bank spread for
// both the natural and the transposed read order).
template <bool CPLX, int LP, bool BF>
__global__ __launch_bounds__(256) void k_update(const void* __restrict__ stack, const void* __restrict__ Pm, int N, int L,
                                                int nb, const uint16_t* __restrict__ table,
                                                const float4* __restrict__ epi, int n_alpha, int n_pad,
                                                cplx64* __restrict__ Q) {
  constexpr int NPL = CPLX ? 2 : 1;
  constexpr int CH = LP / 4;         // chunks per position row
  constexpr int G8 = LP / 8;         // groups of 8 powers
  extern __shared__ __align__(16) shortx8 smem[];
  shortx8* S = smem;                                                     // [2][NPL][TPOS][CH]
  float* Pt = (float*)(smem + 2 * NPL * TPOS * CH);                      // [2][TPOS][NPL]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // ---- tile pair (I, J), I <= J, from the linear block index
  const int q = blockIdx.x;
  int I = (int)((2.0 * nb + 1.0 - sqrt((2.0 * nb + 1.0) * (2.0 * nb + 1.0) - 8.0 * q)) * 0.5);
  if (I < 0) I = 0;
  while (I > 0 && I * nb - I * (I - 1) / 2 > q) --I;
  while ((I + 1) * nb - (I + 1) * I / 2 <= q) ++I;
  const int J = I + (q - (I * nb - I * (I - 1) / 2));
  const bool diag = (I == J);
  const int ntiles = diag ? 1 : 2;
  const size_t NN = (size_t)N * N;

  // ---- stage the power-stack tiles (and P) of the pair
  for (int it = tid; it < ntiles * TPOS * G8; it += 256) {
    const int p = it % TPOS, g = (it / TPOS) % G8, t = it / (TPOS * G8);
    const int row = (t == 0 ? I : J) * TT + p / TT, col = (t == 0 ? J : I) * TT + p % TT;
    const bool inb = row < N && col < N;
    short hi[NPL][8], lo[NPL][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int n = g * 8 + e + 1;
      const size_t off = (size_t)(n - 1) * NN + (size_t)row * N + col;
      if (!inb || n > L) {
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) { hi[pl][e] = 0; lo[pl][e] = 0; }
        continue;
      }
      if (!BF) {
        if (CPLX) {
          const float2 v = ((const float2*)stack)[off];
          split_f32<false>(v.x, hi[0][e], lo[0][e]);
          split_f32<false>(v.y, hi[NPL - 1][e], lo[NPL - 1][e]);
        } else {
          split_f32<false>(((const float*)stack)[off], hi[0][e], lo[0][e]);
        }
      } else {
        if (CPLX) {
          const uint2 v = ((const uint2*)stack)[off];
          hi[0][e] = (short)(v.x & 0xffff); lo[0][e] = (short)(v.x >> 16);
          hi[NPL - 1][e] = (short)(v.y & 0xffff); lo[NPL - 1][e] = (short)(v.y >> 16);
        } else {
          const uint32_t v = ((const uint32_t*)stack)[off];
          hi[0][e] = (short)(v & 0xffff); lo[0][e] = (short)(v >> 16);
        }
      }
    }
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) {
      shortx8 vh, vl;
#pragma unroll
      for (int e = 0; e < 8; ++e) { vh[e] = hi[pl][e]; vl[e] = lo[pl][e]; }
      shortx8* base = S + ((size_t)(t * NPL + pl) * TPOS + p) * CH;
      base[swz(p, g)] = vh;
      base[swz(p, G8 + g)] = vl;
    }
  }
  for (int it = tid; it < ntiles * TPOS; it += 256) {
    const int p = it % TPOS, t = it / TPOS;
    const int row = (t == 0 ? I : J) * TT + p / TT, col = (t == 0 ? J : I) * TT + p % TT;
    const bool inb = row < N && col < N;
    if (CPLX) {
      const float2 v = inb ? ((const float2*)Pm)[(size_t)row * N + col] : make_float2(0.f, 0.f);
      Pt[(t * TPOS + p) * 2] = v.x;
      Pt[(t * TPOS + p) * 2 + 1] = v.y;
    } else {
      Pt[t * TPOS + p] = inb ? ((const float*)Pm)[(size_t)row * N + col] : 0.f;
    }
  }
  __syncthreads();

  const int nblk = ntiles * (TPOS / 32);
  const int l32 = lane & 31, lh = lane >> 5;
  const float unscale = BF ? 1.0f : kUnscale;
  for (int a0 = 0; a0 < n_pad; a0 += 32) {
    // coefficient fragments (A operand: row = order a0 + l32, k = 16 ks + 8 lh .. +7)
    shortx8 aPh[LP / 16], aPl[LP / 16], aNh[LP / 16], aNl[LP / 16];
    const shortx8* trow = (const shortx8*)(table + (size_t)(a0 + l32) * 4 * LP);
#pragma unroll
    for (int ks = 0; ks < LP / 16; ++ks) {
      aPh[ks] = trow[(0 * LP + 16 * ks) / 8 + lh];
      aPl[ks] = trow[(1 * LP + 16 * ks) / 8 + lh];
      aNh[ks] = trow[(2 * LP + 16 * ks) / 8 + lh];
      aNl[ks] = trow[(3 * LP + 16 * ks) / 8 + lh];
    }
    for (int ob = wave; ob < nblk; ob += 4) {
      const int t = ob / (TPOS / 32);
      const int to = diag ? 0 : 1 - t;                 // tile holding the transposed partner
      const int p = (ob % (TPOS / 32)) * 32 + l32;     // this lane's output position (B column)
      const int pT = (p % TT) * TT + p / TT;
      floatx16 acc[NPL];
#pragma unroll
      for (int pl = 0; pl < NPL; ++pl) {
        acc[pl] = floatx16{};
        const shortx8* rowP = S + ((size_t)(t * NPL + pl) * TPOS + p) * CH;
        const shortx8* rowN = S + ((size_t)(to * NPL + pl) * TPOS + pT) * CH;
#pragma unroll
        for (int ks = 0; ks < LP / 16; ++ks) {
          const int ch = 2 * ks + lh;
          const shortx8 bh = rowP[swz(p, ch)], bl = rowP[swz(p, G8 + ch)];
          acc[pl] = mfma16<BF>(aPh[ks], bh, acc[pl]);
          acc[pl] = mfma16<BF>(aPh[ks], bl, acc[pl]);
          acc[pl] = mfma16<BF>(aPl[ks], bh, acc[pl]);
          const shortx8 nh = rowN[swz(pT, ch)], nl = rowN[swz(pT, G8 + ch)];
          shortx8 ch_ = aNh[ks], cl_ = aNl[ks];
          if (CPLX && pl == 1) {  // Im (M_n^H)_{ij} = -Im (M_n)_{ji}
            ch_ ^= (short)0x8000;
            cl_ ^= (short)0x8000;
          }
          acc[pl] = mfma16<BF>(ch_, nh, acc[pl]);
          acc[pl] = mfma16<BF>(ch_, nl, acc[pl]);
          acc[pl] = mfma16<BF>(cl_, nh, acc[pl]);
        }
      }
      // ---- epilogue: + c_0 delta_ij + (e^{j pi alpha} - c_0) P_ij, store complex64
      const int row = (t == 0 ? I : J) * TT + p / TT, col = (t == 0 ? J : I) * TT + p % TT;
      if (row < N && col < N) {
        float pr, pi;
        if (CPLX) { pr = Pt[(t * TPOS + p) * 2]; pi = Pt[(t * TPOS + p) * 2 + 1]; }
        else { pr = Pt[t * TPOS + p]; pi = 0.f; }
        const float dg = (row == col) ? 1.f : 0.f;
        cplx64* qbase = Q + (size_t)row * N + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int a = a0 + 8 * (r >> 2) + 4 * lh + (r & 3);
          if (a < n_alpha) {
            const float4 e = epi[a];
            float re = acc[0][r] * unscale + e.x * dg + e.y * pr - e.z * pi;
            float im = e.z * pr + e.y * pi;
            if (CPLX) im += acc[NPL - 1][r] * unscale;
            qbase[(size_t)a * NN] = cplx64{re, im};
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------ host side
static int n_pad_of(int n_alpha) { return ceil_div(n_alpha, 32) * 32; }

size_t update_ws_bytes(const Plan* p, int n_alpha) {
  const int np = n_pad_of(n_alpha);
  return align_up((size_t)n_alpha * 8, 256) + align_up((size_t)np * 4 * p->LP * 2, 256) +
         align_up((size_t)np * 16, 256);
}

fgfrft_status coef_launch(const Plan* p, const double* alphas_dev, int n_alpha, int n_pad, void* table, float4* epi,
                          int /*unused*/, hipStream_t s) {
  const int total = n_pad * p->LP;
  const bool bf = p->stacktype == FGFRFT_STACK_BF16X2;
  if (bf) k_coef<true><<<ceil_div(total, 256), 256, 0, s>>>(alphas_dev, n_alpha, n_pad, p->L, p->LP, (uint16_t*)table, epi);
  else k_coef<false><<<ceil_div(total, 256), 256, 0, s>>>(alphas_dev, n_alpha, n_pad, p->L, p->LP, (uint16_t*)table, epi);
  FG_LAUNCHED("coef");
  return FGFRFT_OK;
}

template <bool CPLX, int LP, bool BF>
static fgfrft_status launch_update_t(const Plan* p, const uint16_t* table, const float4* epi, int n_alpha, int n_pad,
                                     void* Q, hipStream_t s) {
  constexpr int NPL = CPLX ? 2 : 1;
  const size_t lds = (size_t)2 * NPL * TPOS * (LP / 4) * 16 + (size_t)2 * TPOS * NPL * 4;
  auto kern = k_update<CPLX, LP, BF>;
  static bool attr_set = false;
  if (!attr_set) {
    FG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr_set = true;
  }
  const int nb = ceil_div(p->N, TT);
  const int npairs = nb * (nb + 1) / 2;
  kern<<<npairs, 256, lds, s>>>(p->stack, p->P, p->N, p->L, nb, table, epi, n_alpha, n_pad, (cplx64*)Q);
  FG_LAUNCHED("update");
  return FGFRFT_OK;
}

fgfrft_status update_launch(const Plan* p, const double* alphas_dev, int n_alpha, void* Q, void* ws, hipStream_t s) {
  const int np = n_pad_of(n_alpha);
  char* base = (char*)ws + align_up((size_t)n_alpha * 8, 256);
  uint16_t* table = (uint16_t*)base;
  base += align_up((size_t)np * 4 * p->LP * 2, 256);
  float4* epi = (float4*)base;
  fgfrft_status rc = coef_launch(p, alphas_dev, n_alpha, np, table, epi, 0, s);
  if (rc) return rc;
  const bool bf = p->stacktype == FGFRFT_STACK_BF16X2;
  if (!p->cplx) {
    if (p->LP == 32) return bf ? launch_update_t<false, 32, true>(p, table, epi, n_alpha, np, Q, s)
                               : launch_update_t<false, 32, false>(p, table, epi, n_alpha, np, Q, s);
    if (p->LP == 64) return bf ? launch_update_t<false, 64, true>(p, table, epi, n_alpha, np, Q, s)
                               : launch_update_t<false, 64, false>(p, table, epi, n_alpha, np, Q, s);
  } else {
    if (p->LP == 32) return bf ? launch_update_t<true, 32, true>(p, table, epi, n_alpha, np, Q, s)
                               : launch_update_t<true, 32, false>(p, table, epi, n_alpha, np, Q, s);
  }
  set_error("unsupported L=%d for %s F", p->L, p->cplx ? "complex" : "real");
  return FGFRFT_EUNSUPPORTED;
}

}  // namespace fgfrft
