// Direct route of the transform: Y[:, c] = Q_L^{alpha(c)} X[:, c] without forming any operator.
// With P_c = I - P (Sec. III-B), Definition 1 and Proposition 2 give
//   Q X = c_0 X + (e^{j pi alpha} - c_0) P X + sum_{t < 2L} gamma_t S_t X,
// where S_t runs over the resident M_1..M_L, M_1^H..M_L^H and gamma_t = c_{t+1} (t < L) or
// c_{-(t-L+1)} (t >= L).  Every signal column carries its own order, so the coefficient of a
// term is a per-column scalar.
//
// Matrix-core kernel (real F, real X, N % 32 == 0; `k_direct_pair` below): the signals are split
// once into fp16 hi/lo (after a power-of-two scale per column) in the order the matrix cores read
// them (`k_direct_prep`, in the apply's split layout); every resident tile M_n[I, J] feeds both M_n X
// (rows I) and M_n^T X (rows J), so the stored adjoints are not read; partial sums of row blocks,
// runs and waves are added in a fixed order by a second kernel, with the identity term c_0 X.
//
// A BF16X2 stack (a packed bf16 hi / lo pair per entry) feeds the bf16 matrix cores directly with
// bf16-split signals; an FP16X2 stack (the fp16 pair the FP32 stack would be split into) feeds the
// fp16 matrix cores directly, with the FP32 stack's results bit for bit.  Every other configuration (complex F, complex X, N % 32 != 0) takes a plain
// kernel with one thread per output and FP64 accumulation.
#include "internal.h"
#include <math.h>
#include <type_traits>

namespace fgfrft {

constexpr int DM = 128;                          // output rows per workgroup (4 waves x 32)
constexpr int DK = 32;                           // k per ring stage
constexpr int DAB = DM * DK * 4;                 // stack tile bytes per stage (16 KB)
constexpr int DXB = DK * 64 * 4;                 // signal tile bytes per stage (8 KB: fp16 hi + lo)
constexpr int DSB = DAB + DXB;

// ---------------------------------------------------------------- coefficient table
// Rows of ncp floats; for column c with order alpha and signal scale s (1 on the plain path):
//   t < 2L : gamma_t;   2L : cos(pi alpha) - c_0;   2L + 1 : sin(pi alpha);
//   2L + 2 : c_0;       2L + 3 : 1 / (unscale s).
// Padding columns (c >= ncols) are 0; an order index outside [0, n_alpha) or an order with
// |alpha| >= L (or not finite) makes the whole column NaN.
__global__ __launch_bounds__(256) void k_dcoef(const double* __restrict__ alphas, int n_alpha,
                                               const int* __restrict__ col_order, int ncols, int ncp, int L,
                                               const float2* __restrict__ xs, float unscale, float* __restrict__ gam) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= (2 * L + 4) * ncp) return;
  const int t = idx / ncp, c = idx % ncp;
  float v = 0.f;
  if (c < ncols) {
    const int a = col_order[c];
    const double al = (a >= 0 && a < n_alpha) ? alphas[a] : __builtin_nan("");
    if (!(fabs(al) < (double)L)) {
      v = __builtin_nanf("");
    } else {
      double g;
      if (t < L) g = sinc_pi(al - (double)(t + 1));
      else if (t < 2 * L) g = sinc_pi(al + (double)(t - L + 1));
      else if (t == 2 * L) g = cospi(al) - sinc_pi(al);
      else if (t == 2 * L + 1) g = sinpi(al);
      else if (t == 2 * L + 2) g = sinc_pi(al);
      else g = 1.0 / ((double)unscale * (xs ? (double)xs[c].x : 1.0));
      v = (float)g;
    }
  }
  gam[idx] = v;
}

// ---------------------------------------------------------------- matrix-core kernel
__device__ __forceinline__ void dsplit(float v, short& hi, short& lo) {
  const _Float16 h = (_Float16)v;
  const _Float16 l = (_Float16)(v - (float)h);
  hi = __builtin_bit_cast(short, h);
  lo = __builtin_bit_cast(short, l);
}
// The matrix-core route's set-up in one launch, one workgroup per (64-column block, 32-row chunk):
// the block's column scales from the column maxima of chunks of 64 rows (as k_colscale: 2^e with
// max |x| 2^e in [2^13, 2^14)), the chunk's signals scaled and split into hi / lo parts in the
// layout of xsplit_launch, and, in the chunk-0 workgroup, the block's coefficient rows (as k_dcoef).
// The results are bitwise those of the three separate kernels; a call launches two kernels fewer.
template <bool BF>
__global__ __launch_bounds__(256) void k_direct_prep(const float* __restrict__ X, int ldx, int ncols, int N,
                                                     const float* __restrict__ colpart, int nchm,
                                                     const double* __restrict__ alphas, int n_alpha,
                                                     const int* __restrict__ col_order, int L, int ncp,
                                                     float unscale, float* __restrict__ gam,
                                                     short* __restrict__ Xs) {
  __shared__ float s_sc[64];
  const int nch = N / 32, bc = blockIdx.x, chunk = bc % nch, cb = bc / nch;
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int col = cb * 64 + tid;
    float sc = 0.f;
    if (col < ncols) {
      float m = 0.f;
      for (int c = 0; c < nchm; ++c) m = fmaxf(m, colpart[(size_t)c * ldx + col]);
      int e = 0;
      if (m > 0.f && isfinite(m)) {
        int E;
        frexpf(m, &E);
        e = 14 - E;
        if (e > 100) e = 100;
        if (e < -100) e = -100;
      }
      sc = ldexpf(1.f, e);
    }
    s_sc[tid] = sc;
  }
  __syncthreads();
  // 8 values of column 64 cb + 32 c + l32 at k = 32 chunk + 16 ks + 8 lh .. + 7
  const int lane = tid & 63, c = (tid >> 6) & 1, ks = (tid >> 7) & 1;
  const int col = cb * 64 + 32 * c + (lane & 31);
  const int k0 = chunk * 32 + 16 * ks + 8 * (lane >> 5);
  const float sc = s_sc[32 * c + (lane & 31)];
  shortx8 h, l;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float v = col < ncols ? X[(size_t)(k0 + j) * ldx + col] * sc : 0.f;
    short hh, ll;
    if (BF) {
      const __bf16 bh = (__bf16)v;
      const __bf16 bl = (__bf16)(v - (float)bh);
      hh = __builtin_bit_cast(short, bh);
      ll = __builtin_bit_cast(short, bl);
    } else {
      dsplit(v, hh, ll);
    }
    h[j] = hh;
    l[j] = ll;
  }
  shortx8* dst = (shortx8*)(Xs + (((size_t)bc * 2 + ks) * 2 + c) * 2 * 64 * 8);
  dst[lane] = h;
  dst[64 + lane] = l;
  if (chunk == 0) {
    for (int idx = tid; idx < (2 * L + 4) * 64; idx += 256) {
      const int t = idx >> 6, cc = cb * 64 + (idx & 63);
      float v = 0.f;
      if (cc < ncols) {
        const int a = col_order[cc];
        const double al = (a >= 0 && a < n_alpha) ? alphas[a] : __builtin_nan("");
        if (!(fabs(al) < (double)L)) {
          v = __builtin_nanf("");
        } else {
          double g;
          if (t < L) g = sinc_pi(al - (double)(t + 1));
          else if (t < 2 * L) g = sinc_pi(al + (double)(t - L + 1));
          else if (t == 2 * L) g = cospi(al) - sinc_pi(al);
          else if (t == 2 * L + 1) g = sinpi(al);
          else if (t == 2 * L + 2) g = sinc_pi(al);
          else g = 1.0 / ((double)unscale * (double)s_sc[idx & 63]);
          v = (float)g;
        }
      }
      gam[(size_t)t * ncp + cc] = v;
    }
  }
}

template <bool BF>
__device__ __forceinline__ floatx16 dmma(shortx8 a, shortx8 b, floatx16 c) {
  if (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0, 0, 0);
}

// bf16 hi / lo of an FP32 value (the projector of a BF16X2 plan is kept in FP32)
__device__ __forceinline__ void bsplit(float v, short& hi, short& lo) {
  const __bf16 h = (__bf16)v;
  const __bf16 l = (__bf16)(v - (float)h);
  hi = __builtin_bit_cast(short, h);
  lo = __builtin_bit_cast(short, l);
}

// ---------------------------------------------------------------- paired matrix-core kernel
// Each resident tile M_n[I, J] serves both products that need it: M_n X for the output rows I and
// M_n^T X (= M_n^H X, real F) for the output rows J, so the stored adjoint copies are never read
// and the call streams L + 1 matrices (M_1..M_L, P) instead of 2L + 1.  A workgroup owns 128
// output rows I (4 waves x 32), 64 columns and a run of CPR 32-wide chunks J; per chunk it walks
// the L + 1 terms (stage = (chunk, term)).  Wave w's negative products sum over its own 32 rows
// of I, with the signals of those rows held in registers (pre-split, loaded once).  Per stage:
//   positive: acc = S_t[I, J] X[J]   -> FP32 sum over the run, coefficient c_{t+1} (P: cos - c_0,
//             and sin for the imaginary part);
//   negative: acc = S_t[I_w, J]^T X[I_w] -> FP32 sum over the chunk's terms, coefficient
//             c_{-(t+1)}; written as a partial of rows J when the chunk's terms are done.
// Partials: pos / im [G][N][ncp] (runs), neg [nIB][N][ncp] (row blocks; the waves' parts are
// added in LDS first).
// SM: stack storage, 0 FP32 (split here), 1 bf16 pairs, 2 fp16 pairs (used as stored).
template <int SM>
__global__ __launch_bounds__(256, 2) void k_direct_pair(const float* __restrict__ stack, const float* __restrict__ P,
                                                        int N, int L, const short* __restrict__ Xs, int ncp,
                                                        const float* __restrict__ gam, int CPR, int G, int nIB,
                                                        int ncb, float* __restrict__ part_pos,
                                                        float* __restrict__ part_im, float* __restrict__ part_neg) {
  constexpr int NS = 2;
  constexpr bool BF = SM == 1;
  extern __shared__ __align__(16) char sm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int cb = slot % ncb, w = (slot / ncb) * 8 + xcd;
  if (w >= nIB * G) return;
  const int ib = w % nIB, g = w / nIB;
  const int i0 = ib * DM, b0 = cb * 64;
  const int nch = N / DK, T1 = L + 1;
  const int cfirst = g * CPR, clast = cfirst + CPR < nch ? cfirst + CPR : nch;
  const int nst = (clast - cfirst) * T1;

  // all coefficient rows (2L + 2) for the 64 columns
  float* gl = (float*)(sm + NS * DSB);
  for (int e = tid; e < (2 * L + 2) * 64; e += 256) gl[e] = gam[(size_t)(e >> 6) * ncp + b0 + (e & 63)];

  // signals of this wave's 32 rows of I (the k range of its negative products), pre-split: chunk
  // i0 / 32 + wave of the column block; zero past N
  const char* xsb = (const char*)Xs + (size_t)cb * nch * DXB;
  const int ich = i0 / DK + wave;
  shortx8 xih[2][2], xil[2][2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (ich < nch) {
        const shortx8* src = (const shortx8*)(xsb + (size_t)ich * DXB + ((ks * 2 + c) * 2) * 1024);
        xih[ks][c] = src[lane];
        xil[ks][c] = src[64 + lane];
      } else {
        xih[ks][c] = shortx8{};
        xil[ks][c] = shortx8{};
      }
    }
  // settle these loads before the ring starts: a wait for them inside the loop would also wait for
  // every direct load issued after them
  asm volatile("" ::"v"(xih[0][0]), "v"(xih[0][1]), "v"(xih[1][0]), "v"(xih[1][1]));
  asm volatile("" ::"v"(xil[0][0]), "v"(xil[0][1]), "v"(xil[1][0]), "v"(xil[1][1]));
  __syncthreads();

  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const uint32_t aoff = (uint32_t)((((size_t)(lane >> 3)) * N + 4 * ((lane & 7) ^ (lane >> 3))) * 4);
  auto issue = [&](int it, int jc, int t) {   // stage it = (chunk jc, term t)
    char* st = sm + (it % NS) * DSB;
    const float* A = t < L ? stack + (size_t)t * N * N : P;
#pragma unroll
    for (int q = 0; q < DAB / 4096; ++q) {
      const int i = wv + 4 * q;
      const int row0 = i0 + 8 * i <= N - 8 ? i0 + 8 * i : N - 8;
      const char* gb = (const char*)(A + (size_t)row0 * N + jc * DK);
      lds_dma16(gb + aoff, __builtin_amdgcn_readfirstlane(lds_addr(st + i * 1024)));
    }
#pragma unroll
    for (int q = 0; q < DXB / 4096; ++q) {
      const int i = wv + 4 * q;
      const char* gb = xsb + (size_t)jc * DXB + i * 1024;
      lds_dma16(gb + 16 * lane, __builtin_amdgcn_readfirstlane(lds_addr(st + DAB + i * 1024)));
    }
  };

  float sum_pos[2][16] = {}, sum_im[2][16] = {}, sum_neg[2][16] = {};
  const int r = 32 * wave + l32;
  // stage counters advance incrementally: (jc, t) of the stage consumed, (jn, tn) of the one issued next
  int jc = cfirst, t = 0, jn = cfirst, tn = 0;
  auto advance = [&](int& j, int& k) { if (++k == T1) { k = 0; ++j; } };
  issue(0, jn, tn);
  advance(jn, tn);
  for (int it = 0; it < nst; ++it) {
    // this wave's loads of stage it have landed and its LDS reads of stage it - 1 are done; after the
    // barrier that holds for every wave, so stage it + 1 may refill the other slot
    __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
    barrier_nofence();
    if (it + 1 < nst) {
      issue(it + 1, jn, tn);
      advance(jn, tn);
    }
    const char* st = sm + (it % NS) * DSB;
    // the stage's work; for the pair-stored stacks compiled separately for the projector stage and the
    // stack terms (no per-chunk branches in the fragment assembly), for the FP32 stack one body with a
    // run-time test (a second copy would not fit the register budget)
    auto stage = [&](auto isp_tag, bool isp_rt) {
    const bool isP = decltype(isp_tag)::value || isp_rt;
    // ---- positive: S_t[I, J] X[J]
    floatx16 acc[2] = {};
#pragma unroll
    for (int ks = 0; ks < DK / 16; ++ks) {
      shortx8 ah, al;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ch = (4 * ks + 2 * lh + q) ^ (r & 7);
        const float4 v = *(const float4*)(st + r * (DK * 4) + ch * 16);
        short h, l;
        if (SM != 0 && !isP) {
          const uint4 u4 = __builtin_bit_cast(uint4, v);
          ah[4 * q + 0] = (short)(u4.x & 0xffff); al[4 * q + 0] = (short)(u4.x >> 16);
          ah[4 * q + 1] = (short)(u4.y & 0xffff); al[4 * q + 1] = (short)(u4.y >> 16);
          ah[4 * q + 2] = (short)(u4.z & 0xffff); al[4 * q + 2] = (short)(u4.z >> 16);
          ah[4 * q + 3] = (short)(u4.w & 0xffff); al[4 * q + 3] = (short)(u4.w >> 16);
        } else if (BF) {
          bsplit(v.x, h, l); ah[4 * q + 0] = h; al[4 * q + 0] = l;
          bsplit(v.y, h, l); ah[4 * q + 1] = h; al[4 * q + 1] = l;
          bsplit(v.z, h, l); ah[4 * q + 2] = h; al[4 * q + 2] = l;
          bsplit(v.w, h, l); ah[4 * q + 3] = h; al[4 * q + 3] = l;
        } else {
          dsplit(v.x * kStackScale, h, l); ah[4 * q + 0] = h; al[4 * q + 0] = l;
          dsplit(v.y * kStackScale, h, l); ah[4 * q + 1] = h; al[4 * q + 1] = l;
          dsplit(v.z * kStackScale, h, l); ah[4 * q + 2] = h; al[4 * q + 2] = l;
          dsplit(v.w * kStackScale, h, l); ah[4 * q + 3] = h; al[4 * q + 3] = l;
        }
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const char* xb = st + DAB + ((ks * 2 + c) * 2) * 1024 + 16 * lane;
        const shortx8 bh = *(const shortx8*)xb, bl = *(const shortx8*)(xb + 1024);
        acc[c] = dmma<BF>(ah, bh, acc[c]);
        acc[c] = dmma<BF>(ah, bl, acc[c]);
        acc[c] = dmma<BF>(al, bh, acc[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float gp = gl[(isP ? 2 * L : t) * 64 + 32 * c + l32];
#pragma unroll
      for (int e = 0; e < 16; ++e) sum_pos[c][e] = fmaf(gp, acc[c][e], sum_pos[c][e]);
      if (isP) {
        const float gi = gl[(2 * L + 1) * 64 + 32 * c + l32];
#pragma unroll
        for (int e = 0; e < 16; ++e) sum_im[c][e] = fmaf(gi, acc[c][e], sum_im[c][e]);
      }
    }
    if (!isP) {
      // ---- negative: S_t[I_w, J]^T X[I_w]; lane (j = l32, lh) holds tile rows 32 w + 16 ks + 8 lh + e
      // of column j (chunk j / 4 of those rows, swizzled by row)
      floatx16 an[2] = {};
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        shortx8 th, tl;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int rr = 32 * wave + 16 * ks + 8 * lh + e;
          const float v = *(const float*)(st + rr * (DK * 4) + (((l32 >> 2) ^ (rr & 7)) * 16) + (l32 & 3) * 4);
          short h, l;
          if (SM != 0) {
            const uint32_t u = __builtin_bit_cast(uint32_t, v);
            h = (short)(u & 0xffff);
            l = (short)(u >> 16);
          } else {
            dsplit(v * kStackScale, h, l);
          }
          th[e] = h;
          tl[e] = l;
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          an[c] = dmma<BF>(th, xih[ks][c], an[c]);
          an[c] = dmma<BF>(th, xil[ks][c], an[c]);
          an[c] = dmma<BF>(tl, xih[ks][c], an[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float gn = gl[(L + t) * 64 + 32 * c + l32];
#pragma unroll
        for (int e = 0; e < 16; ++e) sum_neg[c][e] = fmaf(gn, an[c][e], sum_neg[c][e]);
      }
    } else {
      // the chunk's terms are done: the four waves' negative partials (rows J of this chunk) are
      // added through the stage's LDS slot (free once every wave has passed this barrier; the next
      // refill of it comes after the next iteration's barrier) and wave 0 writes the sum
      barrier_nofence();
      float* red = (float*)(sm + (it % NS) * DSB);             // [wave 1..3][c][e][lane]: 24 KB
      if (wave > 0) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int e = 0; e < 16; ++e) red[(((wave - 1) * 2 + c) * 16 + e) * 64 + lane] = sum_neg[c][e];
      }
      __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(63));              // LDS writes done (lgkmcnt 0)
      barrier_nofence();
      if (wave == 0) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int col = b0 + 32 * c + l32;
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            float v = sum_neg[c][e];
#pragma unroll
            for (int q = 0; q < 3; ++q) v += red[((q * 2 + c) * 16 + e) * 64 + lane];
            const int gj = jc * DK + 8 * (e >> 2) + 4 * lh + (e & 3);
            part_neg[((size_t)ib * N + gj) * ncp + col] = v;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) sum_neg[c][e] = 0.f;
    }
    };
    if (SM == 0) stage(std::false_type{}, t == L);
    else if (t == L) stage(std::true_type{}, true);
    else stage(std::false_type{}, false);
    advance(jc, t);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = b0 + 32 * c + l32;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int gi = i0 + 32 * wave + 8 * (e >> 2) + 4 * lh + (e & 3);
      if (gi < N) {
        const size_t o = ((size_t)g * N + gi) * ncp + col;
        part_pos[o] = sum_pos[c][e];
        part_im[o] = sum_im[c][e];
      }
    }
  }
}

// Y[i][c] = u (sum_g pos[g][i][c] + sum_q neg[q][i][c]) + c_0 X[i][c] + j u sum_g im[g][i][c],
// partials in a fixed order.
__global__ __launch_bounds__(256) void k_direct_pair_reduce(const float* __restrict__ part_pos,
                                                            const float* __restrict__ part_im,
                                                            const float* __restrict__ part_neg, int G, int NQ, int N,
                                                            int ncp, int ncols, int L, const float* __restrict__ gam,
                                                            const float* __restrict__ X, int ldx,
                                                            cplx64* __restrict__ Y, int ldy) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)N * ncols) return;
  const int i = (int)(idx / ncols), c = (int)(idx % ncols);
  float re = 0.f, im = 0.f;
  for (int g = 0; g < G; ++g) {
    re += part_pos[((size_t)g * N + i) * ncp + c];
    im += part_im[((size_t)g * N + i) * ncp + c];
  }
  for (int q = 0; q < NQ; ++q) re += part_neg[((size_t)q * N + i) * ncp + c];
  const float c0 = gam[(size_t)(2 * L + 2) * ncp + c], u = gam[(size_t)(2 * L + 3) * ncp + c];
  Y[(size_t)i * ldy + c] = cplx64{re * u + c0 * X[(size_t)i * ldx + c], im * u};
}

// ---------------------------------------------------------------- plain kernel (any configuration)
struct dc { double re, im; };

template <bool C, int SM>
__device__ __forceinline__ dc stack_elem(const void* S, size_t idx) {
  if (SM != 0) {
    auto dec = [](uint32_t w) {
      if (SM == 1) return (double)__uint_as_float(w << 16) + (double)__uint_as_float(w & 0xffff0000u);
      const _Float16 h = __builtin_bit_cast(_Float16, (uint16_t)(w & 0xffff));
      const _Float16 l = __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
      return ((double)h + (double)l) * (1.0 / kStackScale);
    };
    if (C) {
      const uint2 w = ((const uint2*)S)[idx];
      return dc{dec(w.x), dec(w.y)};
    }
    return dc{dec(((const uint32_t*)S)[idx]), 0.0};
  }
  if (C) {
    const cplx64 v = ((const cplx64*)S)[idx];
    return dc{(double)v.re, (double)v.im};
  }
  return dc{(double)((const float*)S)[idx], 0.0};
}

template <bool XC>
__device__ __forceinline__ dc sig_elem(const void* X, size_t idx) {
  if (XC) {
    const cplx64 v = ((const cplx64*)X)[idx];
    return dc{(double)v.re, (double)v.im};
  }
  return dc{(double)((const float*)X)[idx], 0.0};
}

// One thread per output (i, c), columns fastest so a wave reads one stack row (broadcast) and
// consecutive signal entries.  The P matrix is always FP32 / complex64.
template <bool C, int SM, bool XC>
__global__ __launch_bounds__(256) void k_direct_plain(const void* __restrict__ stack, const void* __restrict__ P, int N,
                                                      int L, const void* __restrict__ X, int ldx, int ncols, int ncp,
                                                      const float* __restrict__ gam, cplx64* __restrict__ Y,
                                                      int ldy) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)N * ncols) return;
  const int i = (int)(idx / ncols), c = (int)(idx % ncols);
  const size_t NN = (size_t)N * N;
  const size_t sb = C ? 8 : 4;   // one resident element: float / bf16 pair, or two of them
  double yr = 0.0, yi = 0.0;
  for (int t = 0; t <= 2 * L; ++t) {
    double zr = 0.0, zi = 0.0;
    for (int j = 0; j < N; ++j) {
      const dc s = t < 2 * L ? stack_elem<C, SM>((const char*)stack + (size_t)t * NN * sb, (size_t)i * N + j)
                             : stack_elem<C, 0>(P, (size_t)i * N + j);
      const dc x = sig_elem<XC>(X, (size_t)j * ldx + c);
      zr += s.re * x.re - s.im * x.im;
      zi += s.re * x.im + s.im * x.re;
    }
    if (t < 2 * L) {
      const double gm = (double)gam[(size_t)t * ncp + c];
      yr += gm * zr;
      yi += gm * zi;
    } else {
      const double pr = (double)gam[(size_t)(2 * L) * ncp + c], pi = (double)gam[(size_t)(2 * L + 1) * ncp + c];
      yr += pr * zr - pi * zi;
      yi += pr * zi + pi * zr;
    }
  }
  const double c0 = (double)gam[(size_t)(2 * L + 2) * ncp + c];
  const dc x = sig_elem<XC>(X, (size_t)i * ldx + c);
  Y[(size_t)i * ldy + c] = cplx64{(float)(yr + c0 * x.re), (float)(yi + c0 * x.im)};
}

// ---------------------------------------------------------------- host side
// Paired kernel grid: runs of CPR chunks J per row block, enough runs for one round of resident
// workgroups; runs depend on N and L only.
struct PairGrid {
  int nIB, ncb, ncp, nch, G, CPR, lds;
};

static PairGrid pair_grid(int N, int L, int ncols) {
  PairGrid d;
  d.nIB = ceil_div(N, DM);
  d.ncb = ceil_div(ncols, 64);
  d.ncp = d.ncb * 64;
  d.nch = N / DK > 0 ? N / DK : 1;
  d.lds = 2 * DSB + (2 * L + 2) * 64 * 4;
  const int wpc = d.lds <= 80 * 1024 ? 2 : 1;
  int G = 256 * wpc / d.nIB;
  if (G < 1) G = 1;
  if (G > d.nch) G = d.nch;
  d.CPR = ceil_div(d.nch, G);
  d.G = ceil_div(d.nch, d.CPR);
  return d;
}

struct DirectWs {
  float2* xs;
  float* colpart;
  float* gam;
  short* Xs;
  float* part_re;
  float* part_im;
  float* part_neg;
  size_t bytes;
};

static DirectWs direct_ws(const Plan* p, int ncols, int ldx, void* base) {
  const int N = p->N, L = p->L;
  const PairGrid d = pair_grid(N, L, ncols);
  const int G = d.G;
  DirectWs w;
  char* b = (char*)base;
  size_t off = 0;
  w.xs = (float2*)(b + off); off += align_up((size_t)ldx * sizeof(float2), 256);
  w.colpart = (float*)(b + off); off += colscale_partial_bytes(N, 1, ldx);
  w.gam = (float*)(b + off); off += align_up((size_t)(2 * L + 4) * d.ncp * sizeof(float), 256);
  w.Xs = (short*)(b + off); off += align_up((size_t)d.ncb * d.nch * DXB, 256);
  w.part_re = (float*)(b + off); off += align_up((size_t)G * N * d.ncp * sizeof(float), 256);
  w.part_im = (float*)(b + off); off += align_up((size_t)G * N * d.ncp * sizeof(float), 256);
  w.part_neg = (float*)(b + off); off += align_up((size_t)d.nIB * N * d.ncp * sizeof(float), 256);
  w.bytes = off;
  return w;
}


size_t direct_ws_bytes(const Plan* p, int ncols, int ldx) {
  if (ncols < 1) return 256;
  return direct_ws(p, ncols, ldx, nullptr).bytes;
}

template <bool C, int SM, bool XC>
static void launch_plain(const Plan* p, const void* X, int ldx, int ncols, int ncp, const float* gam, void* Y, int ldy,
                         hipStream_t s) {
  const size_t n = (size_t)p->N * ncols;
  k_direct_plain<C, SM, XC><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p->stack, p->P, p->N, p->L, X, ldx, ncols, ncp,
                                                                        gam, (cplx64*)Y, ldy);
}

fgfrft_status direct_launch(const Plan* p, const double* alphas_dev, int n_alpha, const int* col_order_dev,
                            const void* X, int x_complex, int ncols, int ldx, void* Y, int ldy, void* ws,
                            hipStream_t s) {
  if (ncols == 0) return FGFRFT_OK;
  const int N = p->N, L = p->L;
  const PairGrid d = pair_grid(N, L, ncols);
  const DirectWs w = direct_ws(p, ncols, ldx, ws);
  const bool bf = p->stacktype == FGFRFT_STACK_BF16X2;
  const bool fast = !p->cplx && !x_complex && N % DK == 0;
  const int nrow = 2 * L + 4;
  if (!fast) {
    k_dcoef<<<ceil_div(nrow * d.ncp, 256), 256, 0, s>>>(alphas_dev, n_alpha, col_order_dev, ncols, d.ncp, L, nullptr,
                                                          1.0f, w.gam);
    FG_LAUNCHED("direct coefficients");
    const int sm = p->stacktype;   // 0 FP32, 1 BF16X2, 2 FP16X2
    const int key = (p->cplx ? 6 : 0) + 2 * sm + (x_complex ? 1 : 0);
    switch (key) {
      case 0: launch_plain<false, 0, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 1: launch_plain<false, 0, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 2: launch_plain<false, 1, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 3: launch_plain<false, 1, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 4: launch_plain<false, 2, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 5: launch_plain<false, 2, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 6: launch_plain<true, 0, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 7: launch_plain<true, 0, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 8: launch_plain<true, 1, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 9: launch_plain<true, 1, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 10: launch_plain<true, 2, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 11: launch_plain<true, 2, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
    }
    FG_LAUNCHED("direct (plain)");
    return FGFRFT_OK;
  }
  fgfrft_status rc = colmax_launch(X, 0, N, ldx, 1, w.colpart, s);
  if (rc) return rc;
  // scales, split signals and coefficient rows in one launch
  const unsigned npre = (unsigned)(d.ncb * (N / 32));
  if (bf)
    k_direct_prep<true><<<npre, 256, 0, s>>>((const float*)X, ldx, ncols, N, w.colpart, ceil_div(N, 64), alphas_dev,
                                             n_alpha, col_order_dev, L, d.ncp, 1.0f, w.gam, w.Xs);
  else
    k_direct_prep<false><<<npre, 256, 0, s>>>((const float*)X, ldx, ncols, N, w.colpart, ceil_div(N, 64), alphas_dev,
                                              n_alpha, col_order_dev, L, d.ncp, kStackScale, w.gam, w.Xs);
  FG_LAUNCHED("direct set-up");
  const size_t nb = (size_t)8 * ceil_div(d.nIB * d.G, 8) * d.ncb;
  if (nb > 0x7fffffff) {
    set_error("direct grid too large");
    return FGFRFT_EUNSUPPORTED;
  }
  auto kp = bf ? k_direct_pair<1> : p->stacktype == FGFRFT_STACK_FP16X2 ? k_direct_pair<2> : k_direct_pair<0>;
  FG_HIP(raise_lds_limit((const void*)kp, d.lds));
  kp<<<(unsigned)nb, 256, d.lds, s>>>((const float*)p->stack, (const float*)p->P, N, L, w.Xs, d.ncp, w.gam, d.CPR,
                                      d.G, d.nIB, d.ncb, w.part_re, w.part_im, w.part_neg);
  FG_LAUNCHED("direct");
  const size_t n = (size_t)N * ncols;
  k_direct_pair_reduce<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(w.part_re, w.part_im, w.part_neg, d.G, d.nIB, N,
                                                                   d.ncp, ncols, L, w.gam, (const float*)X, ldx,
                                                                   (cplx64*)Y, ldy);
  FG_LAUNCHED("direct reduce");
  return FGFRFT_OK;
}

}  // namespace fgfrft
