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
//   k_rownorm2_max, k_gbound_scale   per-order power-of-two scales of G and of the outer product's operands
//   k_outer_split  G_a = GY[a] X[a]^H on split-fp16 matrix cores, written split (and, for real F with
//                  N % 32 == 0, in the paired layout); k_outer for the other shapes
//   k_inner_pair   T partials, each stack matrix read on half of its positions (paired layout);
//                  k_inner_mfma over all positions otherwise; k_inner per 16x16 tile for N % 8 != 0
//   k_inner_sum_wg / k_inner_sum   fixed-order sum of the partials in FP64 (deterministic)
#include "internal.h"
#include <math.h>
#include <type_traits>
#include <vector>

namespace fgfrft {

constexpr int GT = 16, GPOS = 256;

// ---------------------------------------------------------------- G = GY X^H
// 64x64 output tile per workgroup, one 32x32 block per wave, on the matrix cores in FP32
// (v_mfma_f32_32x32x2_f32: FP32 products and sums, the accuracy of the plain FMA form); the
// signals advance in chunks of 32 staged through LDS as separate real / imaginary planes
// (zero outside N x B).  G = GY conj(X): Re = gr xr + gi xi, Im = gi xr - gr xi.
constexpr int OKC = 32, OPITCH = OKC + 1;

__device__ __forceinline__ floatx16 mfma_f32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// fp16 hi / lo split of an FP32 value (already scaled into the fp16 range) and the split-fp16 product
__device__ __forceinline__ void split16h(float v, short& hi, short& lo) {
  const _Float16 h = (_Float16)v;
  const _Float16 l = (_Float16)(v - (float)h);
  hi = __builtin_bit_cast(short, h);
  lo = __builtin_bit_cast(short, l);
}
__device__ __forceinline__ floatx16 mma16(shortx8 a, shortx8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0, 0, 0);
}

// Split layout of G for the matrix-core inner products (PRE): per order, positions in blocks of 8
// consecutive ones, 64 bytes per block: fp16 parts [Re hi x 8][Re lo x 8][Im hi x 8][Im lo x 8] of
// G * s_a (s_a the order's power-of-two scale), the same 8 bytes per position as complex64.

// VEC: B % 4 == 0 and 16-byte aligned GY and X, so the staging moves 16 bytes per load.
// PRE: G is written in the split layout above, scaled by gsc[blockIdx.z].x (N % 8 == 0); otherwise
// as complex64 FP32.
template <bool XC, bool VEC, bool PRE>
__global__ __launch_bounds__(256) void k_outer(const cplx64* __restrict__ GY, const void* __restrict__ X, int x_shared,
                                               int N, int B, int a_first, cplx64* __restrict__ G,
                                               const float2* __restrict__ gsc) {
  constexpr int SM_IN = (XC ? 4 : 3) * 64 * OPITCH;
  constexpr int SM_FLOATS = PRE && SM_IN < 8192 ? 8192 : SM_IN;
  static_assert(!PRE || SM_FLOATS * 4 >= 64 * 512, "LDS staging of one split 64 x 64 tile");
  __shared__ __align__(16) float smf[SM_FLOATS];
  float (*Ar)[OPITCH] = (float (*)[OPITCH])smf;
  float (*Ai)[OPITCH] = (float (*)[OPITCH])(smf + 64 * OPITCH);
  float (*Br)[OPITCH] = (float (*)[OPITCH])(smf + 2 * 64 * OPITCH);
  float (*Bi)[OPITCH] = (float (*)[OPITCH])(smf + 3 * 64 * OPITCH);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lk = lane >> 5;
  const int a = a_first + blockIdx.z;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const cplx64* gy = GY + (size_t)a * N * B;
  const size_t xoff = x_shared ? 0 : (size_t)a * N * B;
  floatx16 accr = {}, acci = {};
  for (int b0 = 0; b0 < B; b0 += OKC) {
    if (VEC) {
      for (int e = tid; e < 64 * (OKC / 2); e += 256) {       // GY: two complex values per load
        const int r = e / (OKC / 2), q = e % (OKC / 2);
        const int gi = i0 + r, gb = b0 + 2 * q;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gi < N && gb < B) v = *(const float4*)(gy + (size_t)gi * B + gb);
        Ar[r][2 * q] = v.x; Ai[r][2 * q] = v.y; Ar[r][2 * q + 1] = v.z; Ai[r][2 * q + 1] = v.w;
      }
      if (XC) {
        for (int e = tid; e < 64 * (OKC / 2); e += 256) {
          const int r = e / (OKC / 2), q = e % (OKC / 2);
          const int gj = j0 + r, gb = b0 + 2 * q;
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (gj < N && gb < B) v = *(const float4*)((const float2*)X + xoff + (size_t)gj * B + gb);
          Br[r][2 * q] = v.x; Bi[r][2 * q] = v.y; Br[r][2 * q + 1] = v.z; Bi[r][2 * q + 1] = v.w;
        }
      } else {
        for (int e = tid; e < 64 * (OKC / 4); e += 256) {      // X: four real values per load
          const int r = e / (OKC / 4), q = e % (OKC / 4);
          const int gj = j0 + r, gb = b0 + 4 * q;
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (gj < N && gb < B) v = *(const float4*)((const float*)X + xoff + (size_t)gj * B + gb);
          Br[r][4 * q] = v.x; Br[r][4 * q + 1] = v.y; Br[r][4 * q + 2] = v.z; Br[r][4 * q + 3] = v.w;
        }
      }
    } else
    for (int e = tid; e < 64 * OKC; e += 256) {
      const int r = e / OKC, c = e % OKC;
      const int gi = i0 + r, gj = j0 + r, gb = b0 + c;
      cplx64 g = {0.f, 0.f};
      if (gi < N && gb < B) g = gy[(size_t)gi * B + gb];
      Ar[r][c] = g.re;
      Ai[r][c] = g.im;
      float xr = 0.f, xi = 0.f;
      if (gj < N && gb < B) {
        if (XC) { const float2 v = ((const float2*)X)[xoff + (size_t)gj * B + gb]; xr = v.x; xi = v.y; }
        else xr = ((const float*)X)[xoff + (size_t)gj * B + gb];
      }
      Br[r][c] = xr;
      if (XC) Bi[r][c] = xi;
    }
    __syncthreads();
    // A: lane holds row wi + l32 at k = 2 ks + lk; B: column wj + l32 at the same k
#pragma unroll 4
    for (int ks = 0; ks < OKC / 2; ++ks) {
      const int k = 2 * ks + lk;
      const float ar = Ar[wi + l32][k], ai = Ai[wi + l32][k], br = Br[wj + l32][k];
      accr = mfma_f32(ar, br, accr);
      acci = mfma_f32(ai, br, acci);
      if (XC) {
        const float bi = Bi[wj + l32][k];
        accr = mfma_f32(ai, bi, accr);
        acci = mfma_f32(-ar, bi, acci);
      }
    }
    __syncthreads();
  }
  // lane holds column j0 + wj + l32, rows i0 + wi + 8 (e / 4) + 4 lk + e % 4
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef int i4v __attribute__((ext_vector_type(4)));
  const int gj = j0 + wj + l32;
  if constexpr (PRE) {
    // split into fp16 parts, staged in LDS as 64 rows x 512 bytes in the split layout, then written
    // out as 16-byte pieces (each tile row is 512 contiguous bytes of G), nontemporal
    const float sc = gsc[blockIdx.z].x;
    uint16_t* st = (uint16_t*)smf;
    const int c = wj + l32;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int rr = wi + 8 * (e >> 2) + 4 * lk + (e & 3);
      const float vr = accr[e] * sc, vi = acci[e] * sc;
      const _Float16 rh = (_Float16)vr, ih = (_Float16)vi;
      const _Float16 rl = (_Float16)(vr - (float)rh), il = (_Float16)(vi - (float)ih);
      uint16_t* blk = st + rr * 256 + (c >> 3) * 32 + (c & 7);
      blk[0] = __builtin_bit_cast(uint16_t, rh);
      blk[8] = __builtin_bit_cast(uint16_t, rl);
      blk[16] = __builtin_bit_cast(uint16_t, ih);
      blk[24] = __builtin_bit_cast(uint16_t, il);
    }
    __syncthreads();
    char* g = (char*)(G + (size_t)blockIdx.z * N * N);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int idx = k * 256 + tid;            // 16-byte piece: row idx / 32, piece idx % 32 of the row
      const int rr = idx >> 5, pc = idx & 31;
      const int gi = i0 + rr, gpos = j0 + 2 * pc;   // first of the piece's positions (4 B per position per part)
      if (gi < N && j0 + (pc >> 2) * 8 < N) {
        const i4v v = *(const i4v*)((const char*)st + rr * 512 + pc * 16);
        __builtin_nontemporal_store(v, (i4v*)(g + ((size_t)gi * N + j0) * 8 + pc * 16));
      }
      (void)gpos;
    }
    return;
  }
  // complex64 G streamed out with nontemporal stores (the chunk's G is far larger than the caches;
  // 4% faster than plain stores)
  cplx64* g = G + (size_t)blockIdx.z * N * N;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int gi = i0 + wi + 8 * (e >> 2) + 4 * lk + (e & 3);
    if (gi < N && gj < N) __builtin_nontemporal_store(f2v{accr[e], acci[e]}, (f2v*)(g + (size_t)gi * N + gj));
  }
}

// Largest row norm^2 sum_b |V[a][i][b]|^2 over the 64 rows of a chunk (grid: orders x chunks; V
// complex64 or float32 [n][N][B], order stride `stride` elements, 0 for one block shared by all).
template <bool CPX>
__global__ __launch_bounds__(256) void k_rownorm2_max(const void* __restrict__ V, int N, int B, size_t stride,
                                                      float* __restrict__ out) {
  __shared__ float red[4];
  const int a = blockIdx.x, ch = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i1 = (ch + 1) * 64 < N ? (ch + 1) * 64 : N;
  float m = 0.f;
  for (int i = ch * 64 + w; i < i1; i += 4) {
    float t = 0.f;
    for (int b = lane; b < B; b += 64) {
      const size_t o = (size_t)a * stride + (size_t)i * B + b;
      if (CPX) {
        const float2 v = ((const float2*)V)[o];
        t += v.x * v.x + v.y * v.y;
      } else {
        const float v = ((const float*)V)[o];
        t += v * v;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    m = fmaxf(m, t);
  }
  if (lane == 0) red[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[(size_t)a * gridDim.y + ch] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Order scale from an a-priori bound: |G_a[i][j]| <= ||GY_a[i,:]|| ||X_a[j,:]|| (Cauchy-Schwarz), so
// with m = max_i ||GY_a[i,:]|| max_j ||X_a[j,:]|| (1 + 2^-10 for the rounding of the norms) the scale
// 2^e puts m 2^e in [2^13, 2^14): every scaled entry of G is below 2^14, its fp16 parts stay finite.
// Also the operand scales of the split-fp16 outer product: s_gy, s_x with (largest row norm) s in
// [2^13, 2^14) (every entry is at most its row's norm), and s_a / (s_gy s_x), all powers of two.
__device__ __forceinline__ int pow2_exp_for(float m) {
  int e = 0;
  if (m > 0.f && isfinite(m)) {
    int E;
    frexpf(m, &E);
    e = 14 - E;
    if (e > 100) e = 100;
    if (e < -100) e = -100;
  }
  return e;
}

__global__ __launch_bounds__(256) void k_gbound_scale(const float* __restrict__ gy2, const float* __restrict__ x2,
                                                      int nch, int x_shared, float2* __restrict__ gsc,
                                                      float4* __restrict__ osc) {
  __shared__ float r1[256], r2[256];
  const int a = blockIdx.x;
  float m1 = 0.f, m2 = 0.f;
  for (int c = threadIdx.x; c < nch; c += 256) {
    m1 = fmaxf(m1, gy2[(size_t)a * nch + c]);
    m2 = fmaxf(m2, x2[(size_t)(x_shared ? 0 : a) * nch + c]);
  }
  r1[threadIdx.x] = m1;
  r2[threadIdx.x] = m2;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      r1[threadIdx.x] = fmaxf(r1[threadIdx.x], r1[threadIdx.x + st]);
      r2[threadIdx.x] = fmaxf(r2[threadIdx.x], r2[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float n1 = sqrtf(r1[0]) * (1.f + 1.f / 1024.f), n2 = sqrtf(r2[0]) * (1.f + 1.f / 1024.f);
    const int e = pow2_exp_for(n1 * n2), e1 = pow2_exp_for(n1), e2 = pow2_exp_for(n2);
    gsc[a] = make_float2(ldexpf(1.f, e), ldexpf(1.f, -e));
    osc[a] = make_float4(ldexpf(1.f, e1), ldexpf(1.f, e2), ldexpf(1.f, e - e1 - e2), 0.f);
  }
}

// ---------------------------------------------------------------- operands of the outer product, split once
// GY (complex64) and X (float32 or complex64) [n][N][B] scaled by the order's power of two (osc[v].x for
// GY, osc[v].y for X; one block shared by all orders takes osc[0], the same for every order since it
// depends on X alone) and split into fp16 hi / lo per 8 consecutive signals: complex [Re hi x 8]
// [Re lo x 8][Im hi x 8][Im lo x 8] (64 bytes), real [hi x 8][lo x 8] (32 bytes), so a block keeps the
// bytes and offsets of its 8 source elements.  These are the values k_outer_split would otherwise
// split per wave and per tile (each GY row is used by N / 64 tiles and two waves).
template <bool CPX>
__global__ __launch_bounds__(256) void k_presplit(const void* __restrict__ V, size_t nblk, int N, int B,
                                                  const float4* __restrict__ osc, int comp, int shared,
                                                  char* __restrict__ out) {
  const int bpr = B >> 3;   // 8-signal blocks per row
  for (size_t t = (size_t)blockIdx.x * 256 + threadIdx.x; t < nblk; t += (size_t)gridDim.x * 256) {
    const size_t row = t / bpr;                           // v * N + i
    const int v = shared ? 0 : (int)(row / (size_t)N);
    const float4 o = osc[v];
    const float s = comp ? o.y : o.x;
    const size_t e0 = t * 8;                              // first element of the block
    if (CPX) {
      const float4* src = (const float4*)((const cplx64*)V + e0);
      shortx8 rh, rl, ih, il;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 w = src[q];
        short h, l;
        split16h(w.x * s, h, l); rh[2 * q] = h; rl[2 * q] = l;
        split16h(w.y * s, h, l); ih[2 * q] = h; il[2 * q] = l;
        split16h(w.z * s, h, l); rh[2 * q + 1] = h; rl[2 * q + 1] = l;
        split16h(w.w * s, h, l); ih[2 * q + 1] = h; il[2 * q + 1] = l;
      }
      shortx8* dst = (shortx8*)(out + e0 * 8);
      dst[0] = rh; dst[1] = rl; dst[2] = ih; dst[3] = il;
    } else {
      const float4* src = (const float4*)((const float*)V + e0);
      shortx8 hi, lo;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const float4 w = src[q];
        short h, l;
        split16h(w.x * s, h, l); hi[4 * q] = h; lo[4 * q] = l;
        split16h(w.y * s, h, l); hi[4 * q + 1] = h; lo[4 * q + 1] = l;
        split16h(w.z * s, h, l); hi[4 * q + 2] = h; lo[4 * q + 2] = l;
        split16h(w.w * s, h, l); hi[4 * q + 3] = h; lo[4 * q + 3] = l;
      }
      shortx8* dst = (shortx8*)(out + e0 * 4);
      dst[0] = hi; dst[1] = lo;
    }
  }
}

// ---------------------------------------------------------------- paired layout of G (real F)
// For real F the stack holds M_n^H = M_n^T, so the inner products with M_n and with M_n^H can share one
// read of the stack: beside G on a position (i, j) the kernel needs G on the mirrored position (j, i).
// Positions are grouped in 32-wide row segments (i, jb) = row i, columns 32 jb .. 32 jb + 31 with
// jb >= i / 32 (on or above the diagonal 32 x 32 blocks), numbered band by band (band b: rows
// 32 b .. 32 b + 31), row by row within a band, jb ascending within a row (N % 32 == 0).  Per order two
// planes of 256 bytes per segment in the split layout (the plane Lt follows the plane U):
//   U  [segment][t]:  G[i][32 jb + t], zero where 32 jb + t < i,
//   Lt [segment][t]:  G[32 jb + t][i], zero where 32 jb + t <= i,
// so every position of G appears exactly once, and for the segment's stack rows
//   <G, M_n> = sum U . M_n + Lt . M_n^H,   <G, M_n^H> = sum U . M_n^H + Lt . M_n,
//   <G, P> = sum (U + Lt) . P (P symmetric),   <G, I> = sum U . I (Lt is zero on the diagonal).
__host__ __device__ inline int pair_nseg(int N) { const int nb = N >> 5; return 16 * nb * (nb + 1); }
__host__ __device__ inline int pair_band_base(int b, int nb) { return 32 * (b * nb - b * (b - 1) / 2); }
__host__ __device__ inline int pair_seg(int i, int jb, int nb) {
  const int b = i >> 5;
  return pair_band_base(b, nb) + (i & 31) * (nb - b) + (jb - b);
}
constexpr int PAIR_SEG_BYTES = 512;

// ---------------------------------------------------------------- G = GY X^H, split-fp16 products
// The same 64 x 64 output tile per workgroup (one 32 x 32 block per wave) as k_outer, on
// v_mfma_f32_32x32x16_f16 with the operands split by k_presplit.  Per chunk of 64 signals the tile's
// 64 GY rows (32 KB) and 64 X rows (16 or 32 KB) move into LDS once with direct loads (16-byte chunks
// swizzled by row so the fragment reads of 32 rows spread over the banks), and the four waves read
// their fragments from there as stored: per 16 signals 6 products (real X) or 12 (complex X) instead
// of 16 or 32 FP32 ones.  Output: G s_a in the split layout (as k_outer with PRE).
// B % 64 == 0; rows past N read row N - 1 and are not stored.
// PAIR: output in the paired layout (N % 32 == 0).  A tile below the diagonal (blockIdx.y > blockIdx.x)
// goes only into Lt parts, i.e. transposed: there the MFMA operands trade places, so each lane holds a
// GY row and the staging writes stay along the segments.
constexpr int OS_GROW = 64 * 8;                 // bytes of one GY row chunk (64 complex)

template <bool XC, bool PAIR>
__global__ __launch_bounds__(256) void k_outer_split(const cplx64* __restrict__ GY, const void* __restrict__ X,
                                                     int x_shared, int N, int B, cplx64* __restrict__ G,
                                                     const float4* __restrict__ osc) {
  constexpr int XROW = 64 * (XC ? 8 : 4), XCPR = XROW / 16;
  constexpr int GB = 64 * OS_GROW, XB = 64 * XROW;
  static_assert(GB + XB >= 64 * 512, "the output staging reuses the input LDS");
  static_assert(!PAIR || GB + XB >= 192 * 256, "a diagonal tile stages 192 half segments");
  extern __shared__ __align__(16) char osm[];
  char* gs = osm;
  char* xs = osm + GB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  const int a = blockIdx.z;
  const int by = blockIdx.y, bx = blockIdx.x;   // tile
  const int i0 = by * 64, j0 = bx * 64;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  // PAIR: the operands trade places in a tile below the diagonal and, in a diagonal tile, in the wave of
  // the 32 x 32 block below the diagonal
  const bool lower = by > bx, diag = by == bx;
  const bool swp = PAIR && (lower || (diag && wi > wj));
  const float4 sc = osc[a];
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  // GY: instruction k (wave + 4q) moves rows 2k, 2k + 1: lane -> row 2k + lane / 32, LDS chunk lane % 32
  // holding source chunk (lane % 32) ^ (row % 32).  X: rows of XROW bytes, 1024 / XROW rows per instruction.
  const int grr = lane >> 5, gsl = lane & 31;
  constexpr int XRPI = 1024 / XROW;
  const int xrr = lane / XCPR, xsl = lane % XCPR;
  floatx16 accr = {}, acci = {};
  // the whole signal loop once per operand order (SW: operands traded), chosen per wave
  auto signal_loop = [&](auto sw_tag) {
  constexpr bool SW = decltype(sw_tag)::value;
  for (int b0 = 0; b0 < B; b0 += 64) {
    if (b0 > 0) __syncthreads();   // every wave has read the previous chunk
#pragma unroll
    for (int q = 0; q < GB / 4096; ++q) {
      const int k = wv + 4 * q, row = 2 * k + grr;
      const int gi = min(i0 + row, N - 1);
      const char* src = (const char*)(GY + ((size_t)a * N + gi) * B + b0) + 16 * (gsl ^ (row & 31));
      lds_dma16(src, __builtin_amdgcn_readfirstlane(lds_addr(gs + k * 1024)));
    }
#pragma unroll
    for (int q = 0; q < XB / 4096; ++q) {
      const int k = wv + 4 * q, row = XRPI * k + xrr;
      const int gj = min(j0 + row, N - 1);
      const size_t xr = ((size_t)(x_shared ? 0 : a) * N + gj) * B + b0;
      const char* src = (XC ? (const char*)((const cplx64*)X + xr) : (const char*)((const float*)X + xr)) +
                        16 * (xsl ^ (row % XCPR));
      lds_dma16(src, __builtin_amdgcn_readfirstlane(lds_addr(xs + k * 1024)));
    }
    __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
    barrier_nofence();
    const int ra = wi + l32, rb = wj + l32;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      // fragments read as split (k_presplit): block 2 ks + lh of the row, chunks [Re hi][Re lo][Im hi][Im lo]
      // (complex) or [hi][lo] (real X)
      auto frag = [](const char* row, int c) { return *(const shortx8*)(row + c * 16); };
      const char* ga = gs + ra * OS_GROW;
      const shortx8 arh = frag(ga, (8 * ks + 4 * lh + 0) ^ (ra & 31)), arl = frag(ga, (8 * ks + 4 * lh + 1) ^ (ra & 31));
      const shortx8 aih = frag(ga, (8 * ks + 4 * lh + 2) ^ (ra & 31)), ail = frag(ga, (8 * ks + 4 * lh + 3) ^ (ra & 31));
      const char* xa = xs + rb * XROW;
      shortx8 xrh, xrl, xih = {}, xil = {};
      if (XC) {
        xrh = frag(xa, (8 * ks + 4 * lh + 0) ^ (rb % XCPR));
        xrl = frag(xa, (8 * ks + 4 * lh + 1) ^ (rb % XCPR));
        xih = frag(xa, (8 * ks + 4 * lh + 2) ^ (rb % XCPR));
        xil = frag(xa, (8 * ks + 4 * lh + 3) ^ (rb % XCPR));
      } else {
        xrh = frag(xa, (4 * ks + 2 * lh + 0) ^ (rb % XCPR));
        xrl = frag(xa, (4 * ks + 2 * lh + 1) ^ (rb % XCPR));
      }
      // G = GY conj(X)^T: Re = gr xr + gi xi, Im = gi xr - gr xi (real X: xi = 0); every product is
      // symmetric in its operands, so trading them (SW) only transposes the wave's 32 x 32 block
      auto mm = [](shortx8 u, shortx8 v, floatx16 c) { return SW ? mma16(v, u, c) : mma16(u, v, c); };
      accr = mm(arh, xrh, accr); accr = mm(arh, xrl, accr); accr = mm(arl, xrh, accr);
      acci = mm(aih, xrh, acci); acci = mm(aih, xrl, acci); acci = mm(ail, xrh, acci);
      if (XC) {
        accr = mm(aih, xih, accr); accr = mm(aih, xil, accr); accr = mm(ail, xih, accr);
        const shortx8 narh = arh ^ (short)0x8000, narl = arl ^ (short)0x8000;
        acci = mm(narh, xih, acci); acci = mm(narh, xil, acci); acci = mm(narl, xih, acci);
      }
    }
  }
  };
  if (swp) signal_loop(std::true_type{});
  else signal_loop(std::false_type{});
  typedef int i4v __attribute__((ext_vector_type(4)));
  if constexpr (PAIR) {
    // stage the tile's 256-byte half segments (U or Lt of one segment) in LDS, then 16-byte pieces out.
    // Upper tile: U of segments (i0 + r, 2 bx + s), half segment 2 r + s.  Lower tile: Lt of segments
    // (j0 + c, 2 by + s), half segment 2 c + s.  Diagonal tile: whole segments g = 0 (rows i0 .., column
    // block 2 by), 1 (rows i0 .., 2 by + 1), 2 (rows i0 + 32 .., 2 by + 1), half segment 2 (32 g + r) + part.
    const int nb = N >> 5;
    __syncthreads();   // every wave is done with the input LDS
    // The lane's element u of the wave's block lands in half segment hb + 2 u at position l32.  In the
    // two diagonal 32 x 32 blocks of a diagonal tile (row u, column l32 of the block) it goes to U of row u
    // on and above the diagonal; below it U of row u gets zero and the value goes to Lt of row l32 (half
    // segment hb + 2 l32 + 1, position u); Lt of row u gets zero on and left of the diagonal.
    int hb;
    if (!diag) hb = lower ? 2 * wj + (wi >> 5) : 2 * wi + (wj >> 5);
    else hb = wi != wj ? 64 + (wi > wj ? 1 : 0) : 4 * wi;
    const bool dblk = diag && wi == wj;
    uint16_t* st = (uint16_t*)osm;
    auto put = [&](int h, int t, _Float16 rh, _Float16 rl, _Float16 ih, _Float16 il) {
      uint16_t* blk = st + h * 128 + (t >> 3) * 32 + (t & 7);
      blk[0] = __builtin_bit_cast(uint16_t, rh);
      blk[8] = __builtin_bit_cast(uint16_t, rl);
      blk[16] = __builtin_bit_cast(uint16_t, ih);
      blk[24] = __builtin_bit_cast(uint16_t, il);
    };
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int u = 8 * (e >> 2) + 4 * lh + (e & 3);
      const float vr = accr[e] * sc.z, vi = acci[e] * sc.z;
      const _Float16 rh = (_Float16)vr, ih = (_Float16)vi;
      const _Float16 rl = (_Float16)(vr - (float)rh), il = (_Float16)(vi - (float)ih);
      if (!dblk) {
        put(hb + 2 * u, l32, rh, rl, ih, il);
      } else {
        const _Float16 z = (_Float16)0.0f;
        const bool below = l32 < u;
        if (below) {
          put(hb + 2 * u, l32, z, z, z, z);
          put(hb + 2 * l32 + 1, u, rh, rl, ih, il);
        } else {
          put(hb + 2 * u, l32, rh, rl, ih, il);
        }
        if (l32 <= u) put(hb + 2 * u + 1, l32, z, z, z, z);
      }
    }
    __syncthreads();
    const size_t plane = (size_t)pair_nseg(N) * (PAIR_SEG_BYTES / 2);
    char* g = (char*)G + (size_t)a * 2 * plane;
    // piece k of this thread: half segment h = 16 k + tid / 16, 16-byte piece tid % 16 of it; all LDS
    // reads first, then the stores
    auto target = [&](int h, int& i, int& jb) -> int {   // segment row, column block; returns the part
      if (!diag) {
        i = (lower ? j0 : i0) + (h >> 1);
        jb = 2 * (lower ? by : bx) + (h & 1);
        return lower ? 1 : 0;
      }
      const int q = h >> 1, gg = q >> 5;
      i = i0 + (gg == 2 ? 32 : 0) + (q & 31);
      jb = 2 * by + (gg == 0 ? 0 : 1);
      return h & 1;
    };
    const int pc = tid & 15;
    auto copy_out = [&](auto npieces) {
      constexpr int NP = decltype(npieces)::value;
      i4v v[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) v[k] = *(const i4v*)((const char*)st + (16 * k + (tid >> 4)) * 256 + pc * 16);
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        int i, jb;
        const int part = target(16 * k + (tid >> 4), i, jb);
        if (i < N && jb < nb)
          __builtin_nontemporal_store(
              v[k], (i4v*)(g + part * plane + (size_t)pair_seg(i, jb, nb) * (PAIR_SEG_BYTES / 2) + pc * 16));
      }
    };
    if (diag) copy_out(std::integral_constant<int, 12>{});
    else copy_out(std::integral_constant<int, 8>{});
    return;
  }
  // lane holds column wj + l32, rows wi + 8 (e / 4) + 4 lh + e % 4: split G s_a into LDS in the split
  // layout (reusing the input LDS), then 16-byte pieces out (each tile row is 512 contiguous bytes of
  // G), nontemporal
  __syncthreads();
  uint16_t* st = (uint16_t*)osm;
  const int c = wj + l32;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int rr = wi + 8 * (e >> 2) + 4 * lh + (e & 3);
    const float vr = accr[e] * sc.z, vi = acci[e] * sc.z;
    const _Float16 rh = (_Float16)vr, ih = (_Float16)vi;
    const _Float16 rl = (_Float16)(vr - (float)rh), il = (_Float16)(vi - (float)ih);
    uint16_t* blk = st + rr * 256 + (c >> 3) * 32 + (c & 7);
    blk[0] = __builtin_bit_cast(uint16_t, rh);
    blk[8] = __builtin_bit_cast(uint16_t, rl);
    blk[16] = __builtin_bit_cast(uint16_t, ih);
    blk[24] = __builtin_bit_cast(uint16_t, il);
  }
  __syncthreads();
  char* g = (char*)(G + (size_t)a * N * N);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int idx = k * 256 + tid;             // 16-byte piece: row idx / 32, piece idx % 32 of the row
    const int rr = idx >> 5, pc = idx & 31;
    const int grow = i0 + rr;
    if (grow < N && j0 + (pc >> 2) * 8 < N) {
      const i4v v = *(const i4v*)((const char*)st + rr * 512 + pc * 16);
      __builtin_nontemporal_store(v, (i4v*)(g + ((size_t)grow * N + j0) * 8 + pc * 16));
    }
  }
}

template <bool XC, bool PAIR>
static fgfrft_status outer_split_launch(dim3 g, hipStream_t s, const cplx64* GY, const void* X, int x_shared, int N,
                                        int B, cplx64* G, const float4* osc) {
  constexpr int lds = 64 * OS_GROW + 64 * 64 * (XC ? 8 : 4);
  FG_HIP(raise_lds_limit((const void*)k_outer_split<XC, PAIR>, lds));
  k_outer_split<XC, PAIR><<<g, 256, lds, s>>>(GY, X, x_shared, N, B, G, osc);
  return FGFRFT_OK;
}

// ---------------------------------------------------------------- T partials per tile
// One workgroup per 16x16 tile of positions.  LDS: S[pos][k][plane] for the 2L resident
// matrices (k < L: M_{k+1}, k >= L: M_{k-L+1}^H), Pt[pos][plane], Gs[a][pos][2] for up to AC
// orders at a time.  Thread (k, half) accumulates conj(G) * B_k over half of the tile's
// positions for every order of the sub-chunk; B_{2L} = P, B_{2L+1} = I.
constexpr int AC = 4;

// value of one FP16X2 stack entry (fp16 pair of the 2^12-scaled value)
__device__ __forceinline__ float fp16_pair_value(uint32_t w) {
  const _Float16 h = __builtin_bit_cast(_Float16, (uint16_t)(w & 0xffff));
  const _Float16 l = __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
  return ((float)h + (float)l) * (1.0f / kStackScale);
}

// SM 2: FP16X2 stack entries, decoded on staging.
template <bool CPLX, int SM>
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
    if (SM == 2) {
      if (CPLX) {
        const uint2 w = inb ? ((const uint2*)stack)[off] : make_uint2(0u, 0u);
        dst[0] = fp16_pair_value(w.x);
        dst[NPL - 1] = fp16_pair_value(w.y);
      } else {
        dst[0] = inb ? fp16_pair_value(((const uint32_t*)stack)[off]) : 0.f;
      }
    } else if (CPLX) {
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

// ---------------------------------------------------------------- T partials on the matrix cores
// T[a][k] = sum_p conj(G_a[p]) B_k[p] is a contraction over the N^2 positions p of
// [orders x positions] . [positions x k].  One workgroup per CU streams a contiguous range of
// positions in stages of PC: the stage's G values (64 orders) and its 2L + 1 stack/P rows move
// into LDS with direct loads (a ring of NS stages, NS - 1 of them in flight while one is
// consumed), the identity row is written in place, and 8 waves (a-block = w & 1, k-block
// kb0 + (w >> 1)) run v_mfma_f32_32x32x16_f16 on operands split into fp16 hi/lo (scaled by 2^12
// each).  FP32 accumulators are flushed into FP64 every 256 positions; per-workgroup FP64
// partials are summed over workgroups in a fixed order.
// Rows of B in LDS: 0..2L-1 stack, 2L P, 2L+1..RD-1 copies (ignored columns), RD identity,
// then zero rows up to KP2 = 32 KB.  G rows and B rows keep their 16-byte chunks swizzled by
// row so fragment reads of 32 rows spread over the banks.
constexpr int IM_NA = 64, IM_NW = 8, IM_FLPOS = 256;   // FP32 -> FP64 flush every IM_FLPOS positions


template <bool CPLX, int PC>
struct InnerLayout {
  static constexpr int EB = CPLX ? 8 : 4;
  static constexpr int GROW = PC * 8, GCPR = GROW / 16, GB = IM_NA * GROW;
  static constexpr int SROW = PC * EB, SCPR = SROW / 16, SRPI = 1024 / SROW;
  __host__ __device__ static int rd(int L) { return (2 * L + 1 + SRPI - 1) / SRPI * SRPI; }   // rows moved by direct loads
  __host__ __device__ static int kp2(int L) { return (rd(L) + 1 + 31) / 32 * 32; }
  __host__ __device__ static size_t stage_bytes(int L) { return (size_t)GB + (size_t)kp2(L) * SROW; }
};

// s_waitcnt vmcnt <= n (n < 64, lgkmcnt 0) for a value known only at run time (the direct loads a wave
// issues per stage depend on L and on the wave)
__device__ __forceinline__ void wait_vm_upto(int n) {
  switch (n) {
#define FG_W(k) case k: __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(k)); break;
    FG_W(0) FG_W(1) FG_W(2) FG_W(3) FG_W(4) FG_W(5) FG_W(6) FG_W(7) FG_W(8) FG_W(9) FG_W(10) FG_W(11)
    FG_W(12) FG_W(13) FG_W(14) FG_W(15) FG_W(16) FG_W(17) FG_W(18) FG_W(19) FG_W(20) FG_W(21) FG_W(22)
    FG_W(23) FG_W(24) FG_W(25) FG_W(26) FG_W(27) FG_W(28) FG_W(29) FG_W(30) FG_W(31)
#undef FG_W
    default: __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0)); break;
  }
}

// SM 2: the stack rows (k < 2L) are FP16X2 pairs, used as stored; P, its copies and the identity row
// are FP32 and split here, as every row is for SM 0.
template <bool CPLX, int PC, int KBW, int NS, int SM>
__global__ __launch_bounds__(64 * IM_NW, 1) void k_inner_mfma(const void* __restrict__ stack, const void* __restrict__ Pm,
                                                             int N, int L, const cplx64* __restrict__ G, int n_c,
                                                             const float2* __restrict__ gsc, int spw, int nstage,
                                                             int kb0, double* __restrict__ partial) {
  using LY = InnerLayout<CPLX, PC>;
  constexpr int EB = LY::EB;
  extern __shared__ __align__(16) char smc[];
  char* sm = smc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  const int ab = wave & 1, kg = wave >> 1;
  const int RD = LY::rd(L), KP2 = LY::kp2(L), KB = KP2 / 32;
  const size_t SB = LY::stage_bytes(L);
  const size_t NN = (size_t)N * N;
  const int st0 = blockIdx.x * spw, st1 = st0 + spw < nstage ? st0 + spw : nstage;
  const int wv = __builtin_amdgcn_readfirstlane(wave);

  // direct loads this wave issues per stage (G rows, then stack/P rows), for the ring's waits
  const int nbi = RD / LY::SRPI;
  const int lw = (LY::GB / 1024 - wv + IM_NW - 1) / IM_NW + (nbi - wv + IM_NW - 1) / IM_NW;
  constexpr int FL = IM_FLPOS / PC;
  // zero rows past the identity row (every ring slot); never written afterwards
  for (int s = 0; s < NS; ++s) {
    uint32_t* z = (uint32_t*)(sm + s * SB + LY::GB + (size_t)(RD + 1) * LY::SROW);
    for (int e = tid; e < (KP2 - RD - 1) * LY::SROW / 4; e += 64 * IM_NW) z[e] = 0u;
  }

  auto issue = [&](int st) {
    char* buf = sm + (st % NS) * SB;
    const size_t p0 = (size_t)st * PC;
    // G: instruction i moves order rows 1024/GROW * i .. (orders past n_c read order 0)
    for (int i = wv; i < LY::GB / 1024; i += IM_NW) {
      const int r = i * (1024 / LY::GROW) + lane / LY::GCPR, sl = lane % LY::GCPR;
      const int c = sl ^ (r % LY::GCPR);
      const int a = r < n_c ? r : 0;
      lds_dma16((const char*)(G + (size_t)a * NN + p0 + 2 * c), __builtin_amdgcn_readfirstlane(lds_addr(buf + i * 1024)));
    }
    // B rows 0..RD-1: stack matrices, P, then copies of P
    for (int i = wv; i < RD / LY::SRPI; i += IM_NW) {
      const int k = i * LY::SRPI + lane / LY::SCPR, sl = lane % LY::SCPR;
      const int c = sl ^ (k % LY::SCPR);
      const char* src = k < 2 * L ? (const char*)stack + (size_t)k * NN * EB : (const char*)Pm;
      lds_dma16(src + (p0 + (size_t)c * (16 / EB)) * EB,
                __builtin_amdgcn_readfirstlane(lds_addr(buf + LY::GB + i * 1024)));
    }
    // identity row RD
    for (int e = tid; e < PC; e += 64 * IM_NW) {
      const size_t p = p0 + e;
      const int c = (e * EB / 16) ^ (RD % LY::SCPR);
      float* dst = (float*)(buf + LY::GB + (size_t)RD * LY::SROW + c * 16 + (e * EB) % 16);
      dst[0] = (p % (size_t)(N + 1)) == 0 ? 1.f : 0.f;
      if (CPLX) dst[1] = 0.f;
    }
  };

  floatx16 fre[KBW], fim[KBW];
  double dre[KBW][16], dim[KBW][16];
#pragma unroll
  for (int m = 0; m < KBW; ++m) {
    fre[m] = floatx16{}; fim[m] = floatx16{};
#pragma unroll
    for (int e = 0; e < 16; ++e) { dre[m][e] = 0.0; dim[m][e] = 0.0; }
  }
  const int r = 32 * ab + l32;   // this lane's order row (G is split and scaled per order by k_outer)
  for (int q = 0; q < NS - 1 && st0 + q < st1; ++q) issue(st0 + q);
  int since = 0;
  for (int st = st0; st < st1; ++st) {
    // this wave's loads of stage st have landed (only the NS - 2 younger stages may still be in
    // flight) and its LDS reads of stage st - 1 are done; after the barrier that holds for every wave
    if (st + NS - 1 <= st1) wait_vm_upto((NS - 2) * lw);
    else __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
    barrier_nofence();
    if (st + NS - 1 < st1) issue(st + NS - 1);   // refills the slot read in stage st - 1
    const char* buf = sm + (st % NS) * SB;
#pragma unroll
    for (int ks = 0; ks < PC / 16; ++ks) {
      // G[r][16 ks + 8 lh .. + 7], already split and scaled: block 2 ks + lh, parts Re hi / lo, Im hi / lo
      const char* grow = buf + (size_t)r * LY::GROW;
      const int sw = r % LY::GCPR;
      const shortx8 arh = *(const shortx8*)(grow + ((8 * ks + 4 * lh + 0) ^ sw) * 16);
      const shortx8 arl = *(const shortx8*)(grow + ((8 * ks + 4 * lh + 1) ^ sw) * 16);
      const shortx8 aih = *(const shortx8*)(grow + ((8 * ks + 4 * lh + 2) ^ sw) * 16);
      const shortx8 ail = *(const shortx8*)(grow + ((8 * ks + 4 * lh + 3) ^ sw) * 16);
#pragma unroll
      for (int m = 0; m < KBW; ++m) {
        const int kb = kb0 + kg + 4 * m;
        if (kb >= KB) break;
        const int k = 32 * kb + l32;
        shortx8 brh, brl, bih, bil;
        const char* row = buf + LY::GB + (size_t)k * LY::SROW;
        const bool pairs = SM == 2 && k < 2 * L;
        if (CPLX) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {   // two complex per chunk
            const int c = (8 * ks + 4 * lh + q) ^ (k % LY::SCPR);
            const float4 v = *(const float4*)(row + c * 16);
            if (pairs) {
              const uint4 u = __builtin_bit_cast(uint4, v);
              brh[2 * q] = (short)(u.x & 0xffff); brl[2 * q] = (short)(u.x >> 16);
              bih[2 * q] = (short)(u.y & 0xffff); bil[2 * q] = (short)(u.y >> 16);
              brh[2 * q + 1] = (short)(u.z & 0xffff); brl[2 * q + 1] = (short)(u.z >> 16);
              bih[2 * q + 1] = (short)(u.w & 0xffff); bil[2 * q + 1] = (short)(u.w >> 16);
            } else {
              short h, l;
              split16h(v.x * kStackScale, h, l); brh[2 * q] = h; brl[2 * q] = l;
              split16h(v.y * kStackScale, h, l); bih[2 * q] = h; bil[2 * q] = l;
              split16h(v.z * kStackScale, h, l); brh[2 * q + 1] = h; brl[2 * q + 1] = l;
              split16h(v.w * kStackScale, h, l); bih[2 * q + 1] = h; bil[2 * q + 1] = l;
            }
          }
        } else {
#pragma unroll
          for (int q = 0; q < 2; ++q) {   // four reals per chunk
            const int c = (4 * ks + 2 * lh + q) ^ (k % LY::SCPR);
            const float4 v = *(const float4*)(row + c * 16);
            if (pairs) {
              const uint4 u = __builtin_bit_cast(uint4, v);
              brh[4 * q] = (short)(u.x & 0xffff); brl[4 * q] = (short)(u.x >> 16);
              brh[4 * q + 1] = (short)(u.y & 0xffff); brl[4 * q + 1] = (short)(u.y >> 16);
              brh[4 * q + 2] = (short)(u.z & 0xffff); brl[4 * q + 2] = (short)(u.z >> 16);
              brh[4 * q + 3] = (short)(u.w & 0xffff); brl[4 * q + 3] = (short)(u.w >> 16);
            } else {
              short h, l;
              split16h(v.x * kStackScale, h, l); brh[4 * q] = h; brl[4 * q] = l;
              split16h(v.y * kStackScale, h, l); brh[4 * q + 1] = h; brl[4 * q + 1] = l;
              split16h(v.z * kStackScale, h, l); brh[4 * q + 2] = h; brl[4 * q + 2] = l;
              split16h(v.w * kStackScale, h, l); brh[4 * q + 3] = h; brl[4 * q + 3] = l;
            }
          }
        }
        // conj(g) b: Re = gr br + gi bi, Im = gr bi - gi br (real b: Re = gr b, Im = -gi b)
        fre[m] = mma16(arh, brh, fre[m]);
        fre[m] = mma16(arh, brl, fre[m]);
        fre[m] = mma16(arl, brh, fre[m]);
        fim[m] = mma16(aih, brh, fim[m]);
        fim[m] = mma16(aih, brl, fim[m]);
        fim[m] = mma16(ail, brh, fim[m]);
        if (CPLX) {
          fre[m] = mma16(aih, bih, fre[m]);
          fre[m] = mma16(aih, bil, fre[m]);
          fre[m] = mma16(ail, bih, fre[m]);
          // Im accumulates gi br (subtracted at the end) minus gr bi: add (-gr) bi here
          const shortx8 narh = arh ^ (short)0x8000, narl = arl ^ (short)0x8000;
          fim[m] = mma16(narh, bih, fim[m]);
          fim[m] = mma16(narh, bil, fim[m]);
          fim[m] = mma16(narl, bih, fim[m]);
        }
      }
    }
    if (++since == FL || st + 1 == st1) {   // flush into FP64
      since = 0;
#pragma unroll
      for (int m = 0; m < KBW; ++m)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          dre[m][e] += (double)fre[m][e];
          dim[m][e] += (double)fim[m][e];
          fre[m][e] = 0.f;
          fim[m][e] = 0.f;
        }
    }
  }
  // partial[blockIdx][a][kk][re, im]: lane holds k column 32 kb + l32, orders
  // 32 ab + 8 (e / 4) + 4 lh + e % 4; column RD is the identity (kk = 2L + 1)
  const int K = 2 * L + 2;
#pragma unroll
  for (int m = 0; m < KBW; ++m) {
    const int kb = kb0 + kg + 4 * m;
    if (kb >= KB) break;
    const int k = 32 * kb + l32;
    const int kk = k <= 2 * L ? k : (k == RD ? 2 * L + 1 : -1);
    if (kk < 0) continue;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int a = 32 * ab + 8 * (e >> 2) + 4 * lh + (e & 3);
      if (a < n_c) {
        const double unscale = (double)gsc[a].y / (double)kStackScale;
        const size_t o = (((size_t)blockIdx.x * n_c + a) * K + kk) * 2;
        partial[o] = dre[m][e] * unscale;
        partial[o + 1] = -dim[m][e] * unscale;
      }
    }
  }
}

// G in the paired layout: stage s is segment s (its U and Lt, 2 x 256 bytes per order) and the
// segment's 32 positions of the 2L stack matrices, P and the identity, so each stack matrix is read on
// the segments only (about half of its positions).  The contraction per stage runs over 64 positions:
// U against the column's own row, then Lt against its partner row (M_n <-> M_n^H; P, the identity,
// the copies and the zero rows pair with themselves).  For complex F the partner entries enter
// conjugated (M_n(j, i) = conj(M_n^H(i, j)), P Hermitian), so the Lt half accumulates conj(g) conj(b):
// its products with the imaginary parts of b change sign.  Ring, waves, splitting and FP64 flushes
// (every 256 contracted positions) as in k_inner_mfma; the workgroups take contiguous ranges of segments.
constexpr int IP_GB = IM_NA * PAIR_SEG_BYTES;   // G bytes of one stage
constexpr int IP_FL = IM_FLPOS / 64;            // stages per FP32 accumulation

template <bool CPLX, int NS, int SM>
__global__ __launch_bounds__(64 * IM_NW, 1) void k_inner_pair(const void* __restrict__ stack, const void* __restrict__ Pm,
                                                             int N, int L, const char* __restrict__ G, int n_c,
                                                             const float2* __restrict__ gsc, int spw, int kb0,
                                                             double* __restrict__ partial) {
  using LY = InnerLayout<CPLX, 32>;
  constexpr int EB = LY::EB;
  extern __shared__ __align__(16) char smc[];
  char* sm = smc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  const int ab = wave & 1, kg = wave >> 1;
  const int RD = LY::rd(L), KP2 = LY::kp2(L), KB = KP2 / 32;
  const size_t SB = IP_GB + (size_t)KP2 * LY::SROW;
  const size_t NN = (size_t)N * N;
  const int nb = N >> 5, nseg = pair_nseg(N);
  const size_t plane = (size_t)nseg * (PAIR_SEG_BYTES / 2), ostride = 2 * plane;
  const int st0 = blockIdx.x * spw, st1 = st0 + spw < nseg ? st0 + spw : nseg;
  const int wv = __builtin_amdgcn_readfirstlane(wave);

  const int nbi = RD / LY::SRPI;
  const int lw = (IP_GB / 1024 - wv + IM_NW - 1) / IM_NW + (nbi - wv + IM_NW - 1) / IM_NW;
  for (int s = 0; s < NS; ++s) {
    uint32_t* z = (uint32_t*)(sm + s * SB + IP_GB + (size_t)(RD + 1) * LY::SROW);
    for (int e = tid; e < (KP2 - RD - 1) * LY::SROW / 4; e += 64 * IM_NW) z[e] = 0u;
  }
  // segment of the next stage to issue: row ci, column block cjb
  int ci = 0, cjb = 0;
  if (st0 < st1) {
    int b = 0;
    while (b + 1 < nb && pair_band_base(b + 1, nb) <= st0) ++b;
    const int rem = st0 - pair_band_base(b, nb), w = nb - b;
    ci = 32 * b + rem / w;
    cjb = b + rem % w;
  }

  auto issue = [&](int st) {
    char* buf = sm + (st % NS) * SB;
    const size_t p0 = (size_t)ci * N + 32 * cjb;
    const char* gs = G + (size_t)st * (PAIR_SEG_BYTES / 2);
    // G: instruction i moves orders 2 i, 2 i + 1 (orders past n_c read order 0); LDS row of an order:
    // U chunks 0..15, Lt chunks 16..31
    for (int i = wv; i < IP_GB / 1024; i += IM_NW) {
      const int r = 2 * i + lh;
      const int c = l32 ^ (r & 31);
      const int a = r < n_c ? r : 0;
      lds_dma16(gs + (size_t)a * ostride + (c >> 4) * plane + (c & 15) * 16,
                __builtin_amdgcn_readfirstlane(lds_addr(buf + i * 1024)));
    }
    // B rows 0..RD-1: stack matrices, P, then copies of P
    for (int i = wv; i < nbi; i += IM_NW) {
      const int k = i * LY::SRPI + lane / LY::SCPR, sl = lane % LY::SCPR;
      const int c = sl ^ (k % LY::SCPR);
      const char* src = k < 2 * L ? (const char*)stack + (size_t)k * NN * EB : (const char*)Pm;
      lds_dma16(src + (p0 + (size_t)c * (16 / EB)) * EB,
                __builtin_amdgcn_readfirstlane(lds_addr(buf + IP_GB + i * 1024)));
    }
    // identity row RD
    for (int e = tid; e < 32; e += 64 * IM_NW) {
      const size_t p = p0 + e;
      const int c = (e * EB / 16) ^ (RD % LY::SCPR);
      float* dst = (float*)(buf + IP_GB + (size_t)RD * LY::SROW + c * 16 + (e * EB) % 16);
      dst[0] = (p % (size_t)(N + 1)) == 0 ? 1.f : 0.f;
      if (CPLX) dst[1] = 0.f;
    }
    if (++cjb == nb) { ++ci; cjb = ci >> 5; }
  };

  floatx16 fre = {}, fim = {};
  double dre[16], dim[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) { dre[e] = 0.0; dim[e] = 0.0; }
  const int r = 32 * ab + l32;
  const int kb = kb0 + kg;
  const bool kact = kb < KB;
  const int k = 32 * kb + l32;
  const int kpart = k < L ? k + L : (k < 2 * L ? k - L : k);
  const bool pairs = SM == 2 && k < 2 * L;   // the partner row is a stack row too
  for (int q = 0; q < NS - 1 && st0 + q < st1; ++q) issue(st0 + q);
  int since = 0;
  for (int st = st0; st < st1; ++st) {
    if (st + NS - 1 <= st1) wait_vm_upto((NS - 2) * lw);
    else __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
    barrier_nofence();
    if (st + NS - 1 < st1) issue(st + NS - 1);
    const char* buf = sm + (st % NS) * SB;
    if (kact) {
#pragma unroll
      for (int vk = 0; vk < 4; ++vk) {
        const bool lt = vk >= 2;   // the Lt half, against the partner rows
        const char* grow = buf + (size_t)r * PAIR_SEG_BYTES;
        const int sw = r & 31;
        const shortx8 arh = *(const shortx8*)(grow + ((8 * vk + 4 * lh + 0) ^ sw) * 16);
        const shortx8 arl = *(const shortx8*)(grow + ((8 * vk + 4 * lh + 1) ^ sw) * 16);
        const shortx8 aih = *(const shortx8*)(grow + ((8 * vk + 4 * lh + 2) ^ sw) * 16);
        const shortx8 ail = *(const shortx8*)(grow + ((8 * vk + 4 * lh + 3) ^ sw) * 16);
        const int row = lt ? kpart : k, kk = vk & 1;
        const char* brow = buf + IP_GB + (size_t)row * LY::SROW;
        shortx8 brh, brl, bih = {}, bil = {};
        if (CPLX) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {   // two complex per chunk
            const int c = (8 * kk + 4 * lh + q) ^ (row % LY::SCPR);
            const float4 v = *(const float4*)(brow + c * 16);
            if (pairs) {
              const uint4 u = __builtin_bit_cast(uint4, v);
              brh[2 * q] = (short)(u.x & 0xffff); brl[2 * q] = (short)(u.x >> 16);
              bih[2 * q] = (short)(u.y & 0xffff); bil[2 * q] = (short)(u.y >> 16);
              brh[2 * q + 1] = (short)(u.z & 0xffff); brl[2 * q + 1] = (short)(u.z >> 16);
              bih[2 * q + 1] = (short)(u.w & 0xffff); bil[2 * q + 1] = (short)(u.w >> 16);
            } else {
              short h, l;
              split16h(v.x * kStackScale, h, l); brh[2 * q] = h; brl[2 * q] = l;
              split16h(v.y * kStackScale, h, l); bih[2 * q] = h; bil[2 * q] = l;
              split16h(v.z * kStackScale, h, l); brh[2 * q + 1] = h; brl[2 * q + 1] = l;
              split16h(v.w * kStackScale, h, l); bih[2 * q + 1] = h; bil[2 * q + 1] = l;
            }
          }
        } else {
#pragma unroll
          for (int q = 0; q < 2; ++q) {   // four reals per chunk
            const int c = (4 * kk + 2 * lh + q) ^ (row % LY::SCPR);
            const float4 v = *(const float4*)(brow + c * 16);
            if (pairs) {
              const uint4 u = __builtin_bit_cast(uint4, v);
              brh[4 * q] = (short)(u.x & 0xffff); brl[4 * q] = (short)(u.x >> 16);
              brh[4 * q + 1] = (short)(u.y & 0xffff); brl[4 * q + 1] = (short)(u.y >> 16);
              brh[4 * q + 2] = (short)(u.z & 0xffff); brl[4 * q + 2] = (short)(u.z >> 16);
              brh[4 * q + 3] = (short)(u.w & 0xffff); brl[4 * q + 3] = (short)(u.w >> 16);
            } else {
              short h, l;
              split16h(v.x * kStackScale, h, l); brh[4 * q] = h; brl[4 * q] = l;
              split16h(v.y * kStackScale, h, l); brh[4 * q + 1] = h; brl[4 * q + 1] = l;
              split16h(v.z * kStackScale, h, l); brh[4 * q + 2] = h; brl[4 * q + 2] = l;
              split16h(v.w * kStackScale, h, l); brh[4 * q + 3] = h; brl[4 * q + 3] = l;
            }
          }
        }
        // conj(g) b: Re = gr br + gi bi, Im = gr bi - gi br; conj(g) conj(b) (Lt half, complex F):
        // Re = gr br - gi bi, Im = -(gr bi + gi br).  fim accumulates the negated imaginary part.
        fre = mma16(arh, brh, fre);
        fre = mma16(arh, brl, fre);
        fre = mma16(arl, brh, fre);
        fim = mma16(aih, brh, fim);
        fim = mma16(aih, brl, fim);
        fim = mma16(ail, brh, fim);
        if (CPLX) {
          const shortx8 sih = lt ? aih ^ (short)0x8000 : aih, sil = lt ? ail ^ (short)0x8000 : ail;
          const shortx8 srh = lt ? arh : arh ^ (short)0x8000, srl = lt ? arl : arl ^ (short)0x8000;
          fre = mma16(sih, bih, fre);
          fre = mma16(sih, bil, fre);
          fre = mma16(sil, bih, fre);
          fim = mma16(srh, bih, fim);
          fim = mma16(srh, bil, fim);
          fim = mma16(srl, bih, fim);
        }
      }
    }
    if (++since == IP_FL || st + 1 == st1) {
      since = 0;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        dre[e] += (double)fre[e];
        dim[e] += (double)fim[e];
        fre[e] = 0.f;
        fim[e] = 0.f;
      }
    }
  }
  if (!kact) return;
  const int K = 2 * L + 2;
  const int kk = k <= 2 * L ? k : (k == RD ? 2 * L + 1 : -1);
  if (kk < 0) return;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int a = 32 * ab + 8 * (e >> 2) + 4 * lh + (e & 3);
    if (a < n_c) {
      const double unscale = (double)gsc[a].y / (double)kStackScale;
      const size_t o = (((size_t)blockIdx.x * n_c + a) * K + kk) * 2;
      partial[o] = dre[e] * unscale;
      partial[o + 1] = -dim[e] * unscale;
    }
  }
}

// T[a][k] = sum over workgroups in a fixed order (FP64).
__global__ __launch_bounds__(256) void k_inner_sum_wg(const double* __restrict__ partial, int nwg, int n_c, int K,
                                                      int a_first, double* __restrict__ T) {
  __shared__ double rr[256], ri[256];
  const int a = blockIdx.y, k = blockIdx.x;
  double sr = 0.0, si = 0.0;
  for (int g = threadIdx.x; g < nwg; g += 256) {
    const size_t o = (((size_t)g * n_c + a) * K + k) * 2;
    sr += partial[o];
    si += partial[o + 1];
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
// Orders per pass: the G (and Q(-alpha)) chunk buffer holds ch N x N complex64 matrices; up to 64
// orders (two MFMA row blocks) within about 4 GB, at least 8.
static int grad_chunk(const Plan* p, int n_alpha) {
  const size_t per = (size_t)p->N * p->N * 8;
  size_t ch = ((size_t)4 << 30) / per;
  if (ch > 64) ch = 64;
  if (ch < 8) ch = 8;
  return n_alpha < (int)ch ? n_alpha : (int)ch;
}

static size_t inner_lds(const Plan* p) {
  const int NPL = p->cplx ? 2 : 1;
  return ((size_t)GPOS * 2 * p->L * NPL + GPOS * NPL + (size_t)AC * GPOS * 2) * sizeof(float);
}

// matrix-core inner products: stages of 32 positions (real stack) or 16 (complex), N % 8 == 0, as
// many ring stages as fit the LDS (at most 4, at least 2)
constexpr int IM_PC_REAL = 32, IM_PC_CPLX = 16;
static int inner_stages(const Plan* p) {
  const size_t sb = p->cplx ? InnerLayout<true, IM_PC_CPLX>::stage_bytes(p->L)
                            : InnerLayout<false, IM_PC_REAL>::stage_bytes(p->L);
  const int ns = (int)((160 * 1024) / sb);
  return ns > 4 ? 4 : ns;
}
static bool inner_mfma_ok(const Plan* p) {
  if (p->N % 8) return false;
  const int kp2 = p->cplx ? InnerLayout<true, IM_PC_CPLX>::kp2(p->L) : InnerLayout<false, IM_PC_REAL>::kp2(p->L);
  return inner_stages(p) >= 2 && kp2 <= 256;
}
static int inner_mfma_wgs() { return 256; }

// paired inner products (N % 32 == 0): stage bytes 32 KB of G + the stack rows, ring of up to 3
static size_t pair_stage_bytes(const Plan* p) {
  return p->cplx ? IP_GB + (size_t)InnerLayout<true, 32>::kp2(p->L) * InnerLayout<true, 32>::SROW
                 : IP_GB + (size_t)InnerLayout<false, 32>::kp2(p->L) * InnerLayout<false, 32>::SROW;
}
static int pair_stages_fit(const Plan* p) {
  const int ns = (int)((160 * 1024) / pair_stage_bytes(p));
  return ns > 3 ? 3 : ns;
}
static bool inner_pair_ok(const Plan* p) {
  return p->N % 32 == 0 && inner_mfma_ok(p) && pair_stages_fit(p) >= 2 &&
         (p->stacktype == FGFRFT_STACK_FP32 || p->stacktype == FGFRFT_STACK_FP16X2);
}
static int inner_pair_grid(const Plan* p) {
  const int nseg = pair_nseg(p->N);
  return nseg < inner_mfma_wgs() ? nseg : inner_mfma_wgs();
}
// bytes of one order's G: N x N complex64 or split, or the paired layout (1 + 32 / N times that)
static size_t g_order_bytes(const Plan* p) {
  const size_t plain = (size_t)p->N * p->N * 8;
  if (!inner_pair_ok(p)) return plain;
  const size_t pair = (size_t)pair_nseg(p->N) * PAIR_SEG_BYTES;
  return pair > plain ? pair : plain;
}

template <bool CPLX, int NS, int SM>
static fgfrft_status inner_pair_launch_ns(const Plan* p, const char* G, int nc, const float2* gsc, double* partial,
                                          hipStream_t s) {
  using LY = InnerLayout<CPLX, 32>;
  const int nseg = pair_nseg(p->N);
  const int nwg = inner_pair_grid(p), spw = ceil_div(nseg, nwg);
  const int lds = (int)(NS * pair_stage_bytes(p));
  const int KB = LY::kp2(p->L) / 32;
  auto kern = k_inner_pair<CPLX, NS, SM>;
  FG_HIP(raise_lds_limit((const void*)kern, lds));
  for (int kb0 = 0; kb0 < KB; kb0 += 4)
    kern<<<nwg, 64 * IM_NW, lds, s>>>(p->stack, p->P, p->N, p->L, G, nc, gsc, spw, kb0, partial);
  FG_LAUNCHED("inner_pair");
  return FGFRFT_OK;
}
template <bool CPLX>
static fgfrft_status inner_pair_launch_c(const Plan* p, const char* G, int nc, const float2* gsc, double* partial,
                                         hipStream_t s) {
  const bool f16 = p->stacktype == FGFRFT_STACK_FP16X2;
  if (pair_stages_fit(p) >= 3)
    return f16 ? inner_pair_launch_ns<CPLX, 3, 2>(p, G, nc, gsc, partial, s)
               : inner_pair_launch_ns<CPLX, 3, 0>(p, G, nc, gsc, partial, s);
  return f16 ? inner_pair_launch_ns<CPLX, 2, 2>(p, G, nc, gsc, partial, s)
             : inner_pair_launch_ns<CPLX, 2, 0>(p, G, nc, gsc, partial, s);
}
static fgfrft_status inner_pair_launch(const Plan* p, const char* G, int nc, const float2* gsc, double* partial,
                                       hipStream_t s) {
  return p->cplx ? inner_pair_launch_c<true>(p, G, nc, gsc, partial, s)
                 : inner_pair_launch_c<false>(p, G, nc, gsc, partial, s);
}

size_t grad_ws_bytes(const Plan* p, int n_alpha, int B, int x_shared) {
  const int ch = grad_chunk(p, n_alpha);
  const int N = p->N, nb = ceil_div(N, GT), npairs = nb * nb, K = 2 * p->L + 2;
  size_t part = (size_t)npairs * ch * 2 * K * 16;                   // partials (complex FP64)
  const size_t part2 = (size_t)inner_mfma_wgs() * ch * K * 16;
  if (part2 > part) part = part2;
  size_t s = 0;
  s += align_up((size_t)ch * g_order_bytes(p), 256);                // G chunk / Q(-alpha) chunk
  s += align_up(part, 256);
  s += align_up((size_t)n_alpha * K * 16, 256);                     // T
  s += align_up((size_t)ch * N * B * 8, 256);                       // dX chunk (shared X)
  s += update_ws_bytes(p, ch);
  s += apply_ws_bytes(N, ch, B, 0);
  s += align_up((size_t)n_alpha * 8, 256);
  s += align_up((size_t)2 * ch * ceil_div(N, 64) * 4, 256);         // row-norm maxima of GY and X
  s += align_up((size_t)ch * 16, 256);                              // operand scales of the split outer product
  s += align_up((size_t)ch * 8, 256);                               // G scales
  s += align_up((size_t)ch * N * B * 8, 256);                       // GY split (k_presplit)
  s += align_up((size_t)(x_shared ? 1 : ch) * N * B * 8, 256);      // X split
  if (apply_real_supported(p, 0, B)) s += apply_real_dx_ws_bytes(N, ch, B, p->r_minus1);   // real-F dX
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

static const void* inner_tile_kernel(const Plan* p) {
  const bool f16 = p->stacktype == FGFRFT_STACK_FP16X2;
  if (p->cplx) return f16 ? (const void*)k_inner<true, 2> : (const void*)k_inner<true, 0>;
  return f16 ? (const void*)k_inner<false, 2> : (const void*)k_inner<false, 0>;
}

static int inner_mfma_grid(const Plan* p) {
  const int pc = p->cplx ? IM_PC_CPLX : IM_PC_REAL;
  const int nstage = (int)(((size_t)p->N * p->N) / pc);
  return nstage < inner_mfma_wgs() ? nstage : inner_mfma_wgs();
}

template <bool CPLX, int PC, int NS, int SM>
static fgfrft_status inner_mfma_launch_ns(const Plan* p, const cplx64* G, int nc, const float2* gsc, double* partial,
                                          hipStream_t s) {
  using LY = InnerLayout<CPLX, PC>;
  static_assert(IM_FLPOS % PC == 0, "flush interval in whole stages");
  const int nstage = (int)(((size_t)p->N * p->N) / PC);
  const int nwg = inner_mfma_grid(p), spw = ceil_div(nstage, nwg);
  const int lds = (int)(NS * LY::stage_bytes(p->L));
  const int KB = LY::kp2(p->L) / 32;
  auto kern = k_inner_mfma<CPLX, PC, 1, NS, SM>;
  FG_HIP(raise_lds_limit((const void*)kern, lds));
  // four k-blocks (one per wave pair) per pass over the positions
  for (int kb0 = 0; kb0 < KB; kb0 += 4)
    kern<<<nwg, 64 * IM_NW, lds, s>>>(p->stack, p->P, p->N, p->L, G, nc, gsc, spw, nstage, kb0, partial);
  FG_LAUNCHED("inner_mfma");
  return FGFRFT_OK;
}

template <bool CPLX, int PC, int SM>
static fgfrft_status inner_mfma_launch_sm(const Plan* p, const cplx64* G, int nc, const float2* gsc, double* partial,
                                          hipStream_t s) {
  switch (inner_stages(p)) {
    case 2: return inner_mfma_launch_ns<CPLX, PC, 2, SM>(p, G, nc, gsc, partial, s);
    case 3: return inner_mfma_launch_ns<CPLX, PC, 3, SM>(p, G, nc, gsc, partial, s);
    default: return inner_mfma_launch_ns<CPLX, PC, 4, SM>(p, G, nc, gsc, partial, s);
  }
}

template <bool CPLX, int PC>
static fgfrft_status inner_mfma_launch(const Plan* p, const cplx64* G, int nc, const float2* gsc, double* partial,
                                       hipStream_t s) {
  if (p->stacktype == FGFRFT_STACK_FP16X2) return inner_mfma_launch_sm<CPLX, PC, 2>(p, G, nc, gsc, partial, s);
  return inner_mfma_launch_sm<CPLX, PC, 0>(p, G, nc, gsc, partial, s);
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
  const int nrch = ceil_div(N, 64);
  size_t part = (size_t)npairs * ch * 2 * K * 16;
  const size_t part2 = (size_t)inner_mfma_wgs() * ch * K * 16;
  if (part2 > part) part = part2;
  char* base = (char*)ws;
  cplx64* Gbuf = (cplx64*)base; base += align_up((size_t)ch * g_order_bytes(p), 256);
  double* partial = (double*)base; base += align_up(part, 256);
  double* T = (double*)base; base += align_up((size_t)n_alpha * K * 16, 256);
  void* dXc = base; base += align_up((size_t)ch * N * B * 8, 256);
  void* uws = base; base += update_ws_bytes(p, ch);
  void* aws = base; base += apply_ws_bytes(N, ch, B, 0);
  double* neg_dev = (double*)base; base += align_up((size_t)n_alpha * 8, 256);
  float* gy2 = (float*)base;
  float* x2 = gy2 + (size_t)ch * nrch;
  base += align_up((size_t)2 * ch * nrch * 4, 256);
  float4* osc = (float4*)base;
  base += align_up((size_t)ch * 16, 256);
  float2* gsc = (float2*)base;
  base += align_up((size_t)ch * 8, 256);
  char* gys = base;                                   // GY split for the outer product
  base += align_up((size_t)ch * N * B * 8, 256);
  char* xsp = base;                                   // X split
  base += align_up((size_t)(x_shared ? 1 : ch) * N * B * 8, 256);
  void* rdxws = base;                                 // real-F dX (apply_real_dx_launch)
  const bool realdx = !x_complex && apply_real_supported(p, 0, B);
  const bool use_mfma = inner_mfma_ok(p);
  const bool use_pair = inner_pair_ok(p);   // N % 32 == 0: paired layout when G is split on MFMA
  bool split_outer = false;

  const size_t lds = inner_lds(p);
  if (!use_mfma)
    FG_HIP(raise_lds_limit(inner_tile_kernel(p), (int)lds));
  std::vector<double> neg(n_alpha);
  for (int a = 0; a < n_alpha; ++a) neg[a] = -alphas[a];
  FG_HIP(hipMemcpyAsync(neg_dev, neg.data(), (size_t)n_alpha * 8, hipMemcpyHostToDevice, s));
  const cplx64* gy = (const cplx64*)GY;
  const size_t NB = (size_t)N * B;
  for (int a0 = 0; a0 < n_alpha; a0 += ch) {
    const int nc = n_alpha - a0 < ch ? n_alpha - a0 : ch;
    // ---- dX = Q(-alpha) GY
    if (dX) {
      void* dst = x_shared ? dXc : (void*)((char*)dX + (size_t)a0 * NB * (x_complex ? 8 : 4));
      fgfrft_status rc;
      if (realdx) {   // real F, real X: R = Re Q(-alpha) only, the rank-r imaginary part from W
        rc = update_launch(p, neg_dev + a0, nc, Gbuf, uws, s, true);
        if (rc) return rc;
        rc = apply_real_dx_launch(p, (const float*)Gbuf, nc, neg_dev + a0, gy + (size_t)a0 * NB, B, (float*)dst, rdxws,
                                  s);
      } else {
        rc = update_launch(p, neg_dev + a0, nc, Gbuf, uws, s);
        if (rc) return rc;
        rc = apply_launch(Gbuf, N, nc, 0, gy + (size_t)a0 * NB, 1, 0, B, dst, x_complex ? 0 : 1, aws, s);
      }
      if (rc) return rc;
      if (x_shared) {
        const int g = (int)((NB + 255) / 256 < 4096 ? (NB + 255) / 256 : 4096);
        if (x_complex) k_sum_orders<false><<<g, 256, 0, s>>>(dXc, nc, NB, a0 == 0, dX);
        else k_sum_orders<true><<<g, 256, 0, s>>>(dXc, nc, NB, a0 == 0, dX);
        FG_LAUNCHED("sum_orders");
      }
    }
    // ---- G = GY X^H for the chunk (split and scaled per order for the matrix-core inner products)
    {
      dim3 g(ceil_div(N, 64), ceil_div(N, 64), nc);
      const void* xa = x_shared ? X : (const void*)((const char*)X + (size_t)a0 * NB * (x_complex ? 8 : 4));
      const cplx64* gya = gy + (size_t)a0 * NB;
      if (use_mfma) {   // per-order scales from the row norms of GY and X
        k_rownorm2_max<true><<<dim3(nc, nrch), 256, 0, s>>>(gya, N, B, NB, gy2);
        const int nx = x_shared ? 1 : nc;
        if (x_complex) k_rownorm2_max<true><<<dim3(nx, nrch), 256, 0, s>>>(xa, N, B, NB, x2);
        else k_rownorm2_max<false><<<dim3(nx, nrch), 256, 0, s>>>(xa, N, B, NB, x2);
        k_gbound_scale<<<nc, 256, 0, s>>>(gy2, x2, nrch, x_shared, gsc, osc);
        FG_LAUNCHED("gradient scales");
      }
      const bool vec = B % 4 == 0 && (uintptr_t)gya % 16 == 0 && (uintptr_t)xa % 16 == 0;
      const int key = (x_complex ? 4 : 0) | (vec ? 2 : 0) | (use_mfma ? 1 : 0);
      split_outer = use_mfma && vec && B % 64 == 0;
      if (split_outer) {   // split-fp16 products on LDS-staged operands, split once beforehand
        const int nx = x_shared ? 1 : nc;
        const size_t gblk = (size_t)nc * N * (B / 8), xblk = (size_t)nx * N * (B / 8);
        const unsigned gg = (unsigned)((gblk + 255) / 256 < 8192 ? (gblk + 255) / 256 : 8192);
        const unsigned gx = (unsigned)((xblk + 255) / 256 < 8192 ? (xblk + 255) / 256 : 8192);
        k_presplit<true><<<gg, 256, 0, s>>>(gya, gblk, N, B, osc, 0, 0, gys);
        if (x_complex) k_presplit<true><<<gx, 256, 0, s>>>(xa, xblk, N, B, osc, 1, x_shared, xsp);
        else k_presplit<false><<<gx, 256, 0, s>>>(xa, xblk, N, B, osc, 1, x_shared, xsp);
        FG_LAUNCHED("presplit");
        const cplx64* gyv = (const cplx64*)gys;
        fgfrft_status rc;
        if (use_pair) rc = x_complex ? outer_split_launch<true, true>(g, s, gyv, xsp, x_shared, N, B, Gbuf, osc)
                                     : outer_split_launch<false, true>(g, s, gyv, xsp, x_shared, N, B, Gbuf, osc);
        else rc = x_complex ? outer_split_launch<true, false>(g, s, gyv, xsp, x_shared, N, B, Gbuf, osc)
                            : outer_split_launch<false, false>(g, s, gyv, xsp, x_shared, N, B, Gbuf, osc);
        if (rc) return rc;
      } else
      switch (key) {
        case 0: k_outer<false, false, false><<<g, 256, 0, s>>>(gya, xa, x_shared, N, B, 0, Gbuf, gsc); break;
        case 1: k_outer<false, false, true><<<g, 256, 0, s>>>(gya, xa, x_shared, N, B, 0, Gbuf, gsc); break;
        case 2: k_outer<false, true, false><<<g, 256, 0, s>>>(gya, xa, x_shared, N, B, 0, Gbuf, gsc); break;
        case 3: k_outer<false, true, true><<<g, 256, 0, s>>>(gya, xa, x_shared, N, B, 0, Gbuf, gsc); break;
        case 4: k_outer<true, false, false><<<g, 256, 0, s>>>(gya, xa, x_shared, N, B, 0, Gbuf, gsc); break;
        case 5: k_outer<true, false, true><<<g, 256, 0, s>>>(gya, xa, x_shared, N, B, 0, Gbuf, gsc); break;
        case 6: k_outer<true, true, false><<<g, 256, 0, s>>>(gya, xa, x_shared, N, B, 0, Gbuf, gsc); break;
        case 7: k_outer<true, true, true><<<g, 256, 0, s>>>(gya, xa, x_shared, N, B, 0, Gbuf, gsc); break;
      }
      FG_LAUNCHED("outer");
    }
    if (use_mfma && use_pair && split_outer) {   // G in the paired layout
      fgfrft_status rc = inner_pair_launch(p, (const char*)Gbuf, nc, gsc, partial, s);
      if (rc) return rc;
      k_inner_sum_wg<<<dim3(K, nc), 256, 0, s>>>(partial, inner_pair_grid(p), nc, K, a0, T);
      FG_LAUNCHED("inner_sum");
    } else if (use_mfma) {
      fgfrft_status rc = p->cplx ? inner_mfma_launch<true, IM_PC_CPLX>(p, Gbuf, nc, gsc, partial, s)
                                 : inner_mfma_launch<false, IM_PC_REAL>(p, Gbuf, nc, gsc, partial, s);
      if (rc) return rc;
      k_inner_sum_wg<<<dim3(K, nc), 256, 0, s>>>(partial, inner_mfma_grid(p), nc, K, a0, T);
      FG_LAUNCHED("inner_sum");
    } else {
      auto kt = (void (*)(const void*, const void*, int, int, int, const cplx64*, int, double*))inner_tile_kernel(p);
      kt<<<npairs, 256, lds, s>>>(p->stack, p->P, N, L, nb, Gbuf, nc, partial);
      FG_LAUNCHED("inner");
      k_inner_sum<<<dim3(K, nc), 256, 0, s>>>(partial, npairs, nc, K, a0, T);
      FG_LAUNCHED("inner_sum");
    }
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
