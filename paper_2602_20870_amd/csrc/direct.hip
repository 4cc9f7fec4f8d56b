// Direct route of the transform: Y[:, c] = Q_L^{alpha(c)} X[:, c] without forming any operator.
// With P_c = I - P (Sec. III-B), Definition 1 and Proposition 2 give
//   Q X = c_0 X + (e^{j pi alpha} - c_0) P X + sum_{t < 2L} gamma_t S_t X,
// where S_t runs over the resident M_1..M_L, M_1^H..M_L^H and gamma_t = c_{t+1} (t < L) or
// c_{-(t-L+1)} (t >= L).  Every signal column carries its own order, so the coefficient of a
// term is a per-column scalar.
//
// Matrix-core kernel (real F, FP32 stack, real X, N % 32 == 0): the signals are split once into
// fp16 hi/lo (after a power-of-two scale per column) in the order the matrix cores read them
// (xsplit_launch, shared with the apply).  A
// workgroup owns 128 output rows x 64 columns and a contiguous run of the (2L + 1) x N/32 stages
// (term, 32-wide k chunk) of that tile; the runs are balanced so the whole grid is one round of
// resident workgroups (three per CU) when the tile count allows.  Stack and signal tiles stream from HBM into
// an LDS ring with direct loads; the products of one term (stack split into fp16 hi/lo when a
// wave reads its fragments, hi*hi + hi*lo + lo*hi) accumulate in FP32 and are folded into an FP64
// sum with the column's coefficient when the term ends, so no FP32 chain runs over more than the
// N products of one term.  The P term's products fold twice: into the real part with
// cos(pi alpha) - c_0 and into the imaginary part with sin(pi alpha).  Runs write partial sums
// that a second kernel adds in a fixed order (deterministic), with the identity term c_0 X.
//
// A BF16X2 stack (a packed bf16 hi / lo pair per entry) feeds the bf16 matrix cores directly with
// bf16-split signals.  Every other configuration (complex F, complex X, N % 32 != 0) takes a plain
// kernel with one thread per output and FP64 accumulation.
#include "internal.h"
#include <math.h>

namespace fgfrft {

constexpr int DM = 128;                          // output rows per workgroup (4 waves x 32)
constexpr int DK = 32;                           // k per ring stage
constexpr int DAB = DM * DK * 4;                 // stack tile bytes per stage (16 KB)
constexpr int DXB = DK * 64 * 4;                 // signal tile bytes per stage (8 KB: fp16 hi + lo)
constexpr int DSB = DAB + DXB;
constexpr int DLW = DAB / 4096 + DXB / 4096;     // direct loads per wave per stage
// Ring of NS stages.  NS = 3: 80 KB of LDS, two workgroups per CU, runs touch up to 24 terms;
// NS = 2: 53 KB, three workgroups per CU, up to 16 terms.
template <int NS> struct DirectCfg {
  static constexpr int TG = NS == 3 ? 24 : 16;              // terms one run may touch
  static constexpr int LDS = NS * DSB + (TG + 1) * 64 * 4;
  static constexpr int WPC = NS == 3 ? 2 : 3;               // workgroups per CU
  static_assert(LDS * WPC <= 160 * 1024, "LDS budget");
};

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

// Grid: 8 * ceil(nIB * G / 8) * ncb workgroups; workgroup (row block ib, run g, column block cb)
// takes stages [g SPW, min((g + 1) SPW, T nch)) of its tile, stage st = (term st / nch, k chunk
// st % nch).  Ids are dealt round-robin over the 8 XCDs; the column blocks of one (row block,
// run) get consecutive ids on one XCD, so a stack tile read for one column block is an L2 hit for
// the others.  part_re, part_im: [G][N][ncp]; part_im is written only by runs that reach P.
// BF: BF16X2 stack (each real entry a packed bf16 pair, hi in the low half), bf16 matrix cores,
// unscaled operands; the P stages split their FP32 tiles into bf16 hi / lo.
template <int DNS, bool BF>
__global__ __launch_bounds__(256, DirectCfg<DNS>::WPC) void k_direct(const float* __restrict__ stack, const float* __restrict__ P, int N,
                                                   int L, const short* __restrict__ Xs, int ncp,
                                                   const float* __restrict__ gam, int SPW, int G, int nIB, int ncb,
                                                   float* __restrict__ part_re, float* __restrict__ part_im) {
  extern __shared__ __align__(16) char sm[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, lh = lane >> 5;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int cb = slot % ncb, w = (slot / ncb) * 8 + xcd;
  if (w >= nIB * G) return;
  const int ib = w % nIB, g = w / nIB;
  const int i0 = ib * DM, b0 = cb * 64;
  const int T = 2 * L + 1, nch = N / DK;
  const int s0 = g * SPW;
  const int s1 = s0 + SPW < T * nch ? s0 + SPW : T * nch;
  const int nst = s1 - s0;
  const int tfirst = s0 / nch, nterm = (s1 - 1) / nch - tfirst + 1;
  const bool hasP = s1 > 2 * L * nch;

  // coefficients of the terms this run touches for the 64 columns (row nterm: the sin row of P)
  float* gl = (float*)(sm + DNS * DSB);
  for (int e = tid; e < (nterm + 1) * 64; e += 256) {
    const int tl = e >> 6, col = e & 63;
    const int row = tl < nterm ? tfirst + tl : (hasP ? T : -1);
    gl[e] = row >= 0 ? gam[(size_t)row * ncp + b0 + col] : 0.f;
  }
  __syncthreads();

  // Direct loads: a wave-uniform base plus a fixed per-lane 32-bit offset.  Stack instruction
  // i (i = wave + 4q) moves tile rows 8i .. 8i + 7 (a row group past N: the last valid group,
  // never written back); lane: row 8i + lane / 8, stored chunk lane % 8 holds the row's 16-byte
  // chunk (lane % 8) ^ (lane / 8), so chunk c of tile row r sits at c ^ (r % 8).  Signal
  // instruction i moves the i-th kilobyte of the stage's pre-split signal block.
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const uint32_t aoff = (uint32_t)((((size_t)(lane >> 3)) * N + 4 * ((lane & 7) ^ (lane >> 3))) * 4);
  const char* xsb = (const char*)Xs + (size_t)cb * nch * DXB;
  auto issue = [&](int it) {
    char* st = sm + (it % DNS) * DSB;
    const int gs = s0 + it, t = gs / nch, chunk = gs - t * nch;
    const int k0 = chunk * DK;
    const float* A = t < 2 * L ? stack + (size_t)t * N * N : P;
#pragma unroll
    for (int q = 0; q < DAB / 4096; ++q) {
      const int i = wv + 4 * q;
      const int row0 = i0 + 8 * i <= N - 8 ? i0 + 8 * i : N - 8;
      const char* gb = (const char*)(A + (size_t)row0 * N + k0);
      lds_dma16(gb + aoff, __builtin_amdgcn_readfirstlane(lds_addr(st + i * 1024)));
    }
#pragma unroll
    for (int q = 0; q < DXB / 4096; ++q) {
      const int i = wv + 4 * q;
      const char* gb = xsb + (size_t)chunk * DXB + i * 1024;
      lds_dma16(gb + 16 * lane, __builtin_amdgcn_readfirstlane(lds_addr(st + DAB + i * 1024)));
    }
  };

  // acc: FP32 products of the current term; at the end of each term (or of the run) they are
  // folded with the column's coefficient into FP64 sums of the real part, so an output sees one
  // FP32 chain of at most N products per term.  The imaginary part is the P term alone.
  double sum_re[2][16] = {};
  float sum_im[2][16] = {};
  floatx16 acc[2] = {};
  const int r = 32 * wave + l32;
  for (int it = 0; it < DNS - 1 && it < nst; ++it) issue(it);
  for (int it = 0; it < nst; ++it) {
    // this wave's loads of stage it have landed (only the DNS - 2 younger stages may still be in
    // flight) and its LDS reads of stage it - 1 are done; after the barrier that holds for all waves
    if (it + DNS - 1 <= nst) __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0((DNS - 2) * DLW));
    else __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
    barrier_nofence();
    if (it + DNS - 1 < nst) issue(it + DNS - 1);   // refills the slot of stage it - 1
    const char* st = sm + (it % DNS) * DSB;
#pragma unroll
    for (int ks = 0; ks < DK / 16; ++ks) {
      // A: S_t[i0 + r][k0 + 16 ks + 8 lh .. + 7], two 16-byte chunks, split after the 2^12 scale
      shortx8 ah, al;
      const bool pstage = BF && (s0 + it) / nch == 2 * L;      // wave-uniform
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int ch = (4 * ks + 2 * lh + q) ^ (r & 7);
        const float4 v = *(const float4*)(st + r * (DK * 4) + ch * 16);
        short h, l;
        if (BF && !pstage) {
          const uint4 w = __builtin_bit_cast(uint4, v);
          ah[4 * q + 0] = (short)(w.x & 0xffff); al[4 * q + 0] = (short)(w.x >> 16);
          ah[4 * q + 1] = (short)(w.y & 0xffff); al[4 * q + 1] = (short)(w.y >> 16);
          ah[4 * q + 2] = (short)(w.z & 0xffff); al[4 * q + 2] = (short)(w.z >> 16);
          ah[4 * q + 3] = (short)(w.w & 0xffff); al[4 * q + 3] = (short)(w.w >> 16);
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
    const int gs = s0 + it;
    if ((gs + 1) % nch == 0 || it == nst - 1) {     // the term ends here (or the run does)
      const int tl = gs / nch - tfirst;
      const bool isP = tfirst + tl == 2 * L;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double gr = (double)gl[tl * 64 + 32 * c + l32];
#pragma unroll
        for (int e = 0; e < 16; ++e) sum_re[c][e] = fma(gr, (double)acc[c][e], sum_re[c][e]);
        if (isP) {
          const float gi = gl[nterm * 64 + 32 * c + l32];
#pragma unroll
          for (int e = 0; e < 16; ++e) sum_im[c][e] = fmaf(gi, acc[c][e], sum_im[c][e]);
        }
        acc[c] = floatx16{};
      }
    }
  }
  // lane holds column b0 + 32 c + l32, rows 32 wave + 8 (e / 4) + 4 lh + e % 4
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = b0 + 32 * c + l32;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int gi = i0 + 32 * wave + 8 * (e >> 2) + 4 * lh + (e & 3);
      if (gi < N) {
        const size_t o = ((size_t)g * N + gi) * ncp + col;
        part_re[o] = (float)sum_re[c][e];
        if (hasP) part_im[o] = sum_im[c][e];
      }
    }
  }
}

// Y[i][c] = (sum_g part_re[g][i][c]) u + c_0 X[i][c] + j (sum_{g >= gP} part_im[g][i][c]) u,
// runs in a fixed order.
__global__ __launch_bounds__(256) void k_direct_reduce(const float* __restrict__ part_re,
                                                       const float* __restrict__ part_im, int G, int gP, int N,
                                                       int ncp, int ncols, int L, const float* __restrict__ gam,
                                                       const float* __restrict__ X, int ldx,
                                                       cplx64* __restrict__ Y, int ldy) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)N * ncols) return;
  const int i = (int)(idx / ncols), c = (int)(idx % ncols);
  float re = 0.f, im = 0.f;
  for (int g = 0; g < G; ++g) re += part_re[((size_t)g * N + i) * ncp + c];
  for (int g = gP; g < G; ++g) im += part_im[((size_t)g * N + i) * ncp + c];
  const float c0 = gam[(size_t)(2 * L + 2) * ncp + c], u = gam[(size_t)(2 * L + 3) * ncp + c];
  Y[(size_t)i * ldy + c] = cplx64{re * u + c0 * X[(size_t)i * ldx + c], im * u};
}

// ---------------------------------------------------------------- plain kernel (any configuration)
struct dc { double re, im; };

template <bool C, bool BF>
__device__ __forceinline__ dc stack_elem(const void* S, size_t idx) {
  if (BF) {
    auto dec = [](uint32_t w) {
      return (double)__uint_as_float(w << 16) + (double)__uint_as_float(w & 0xffff0000u);
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
template <bool C, bool BF, bool XC>
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
      const dc s = t < 2 * L ? stack_elem<C, BF>((const char*)stack + (size_t)t * NN * sb, (size_t)i * N + j)
                             : stack_elem<C, false>(P, (size_t)i * N + j);
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
// Runs per tile: enough for one round of the resident workgroups per CU when the tiles allow,
// and at most TG - 1 terms of stages per run (the coefficient rows a run keeps in LDS).
struct DirectGrid {
  int nIB, ncb, ncp, nch, G, SPW, gP;
};

// Two ring stages with three workgroups per CU measured a few percent faster than three stages
// with two workgroups per CU at N = 4096, L = 32 (64 and 256 columns).
constexpr int kDirectNS = 2;
using DCfg = DirectCfg<kDirectNS>;

static DirectGrid direct_grid(int N, int L, int ncols) {
  const int TG = DCfg::TG, WPC = DCfg::WPC;
  DirectGrid d;
  d.nIB = ceil_div(N, DM);
  d.ncb = ceil_div(ncols, 64);
  d.ncp = d.ncb * 64;
  d.nch = N / DK > 0 ? N / DK : 1;
  const int T = 2 * L + 1, total = T * d.nch;
  // the runs depend on N and L only, so a column's result (its FP64 fold and reduction order)
  // does not depend on how many other columns share the call
  const long units = d.nIB;
  int G = (int)(256 * WPC / units);
  const int gmin = ceil_div(T, TG - 1);
  if (G < gmin) G = gmin;
  if (G > total) G = total;
  d.SPW = ceil_div(total, G);
  d.G = ceil_div(total, d.SPW);
  d.gP = (2 * L * d.nch) / d.SPW;
  return d;
}

struct DirectWs {
  float2* xs;
  float* colpart;
  float* gam;
  short* Xs;
  float* part_re;
  float* part_im;
  size_t bytes;
};

static DirectWs direct_ws(const Plan* p, int ncols, int ldx, void* base) {
  const int N = p->N, L = p->L;
  const DirectGrid d = direct_grid(N, L, ncols);
  DirectWs w;
  char* b = (char*)base;
  size_t off = 0;
  w.xs = (float2*)(b + off); off += align_up((size_t)ldx * sizeof(float2), 256);
  w.colpart = (float*)(b + off); off += colscale_partial_bytes(N, 1, ldx);
  w.gam = (float*)(b + off); off += align_up((size_t)(2 * L + 4) * d.ncp * sizeof(float), 256);
  w.Xs = (short*)(b + off); off += align_up((size_t)d.ncb * d.nch * DXB, 256);
  w.part_re = (float*)(b + off); off += align_up((size_t)d.G * N * d.ncp * sizeof(float), 256);
  w.part_im = (float*)(b + off); off += align_up((size_t)d.G * N * d.ncp * sizeof(float), 256);
  w.bytes = off;
  return w;
}

size_t direct_ws_bytes(const Plan* p, int ncols, int ldx) {
  if (ncols < 1) return 256;
  return direct_ws(p, ncols, ldx, nullptr).bytes;
}

template <bool C, bool BF, bool XC>
static void launch_plain(const Plan* p, const void* X, int ldx, int ncols, int ncp, const float* gam, void* Y, int ldy,
                         hipStream_t s) {
  const size_t n = (size_t)p->N * ncols;
  k_direct_plain<C, BF, XC><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p->stack, p->P, p->N, p->L, X, ldx, ncols, ncp,
                                                                        gam, (cplx64*)Y, ldy);
}

fgfrft_status direct_launch(const Plan* p, const double* alphas_dev, int n_alpha, const int* col_order_dev,
                            const void* X, int x_complex, int ncols, int ldx, void* Y, int ldy, void* ws,
                            hipStream_t s) {
  if (ncols == 0) return FGFRFT_OK;
  const int N = p->N, L = p->L;
  const DirectGrid d = direct_grid(N, L, ncols);
  const DirectWs w = direct_ws(p, ncols, ldx, ws);
  const bool bf = p->stacktype == FGFRFT_STACK_BF16X2;
  const bool fast = !p->cplx && !x_complex && N % DK == 0;
  const int nrow = 2 * L + 4;
  if (!fast) {
    k_dcoef<<<ceil_div(nrow * d.ncp, 256), 256, 0, s>>>(alphas_dev, n_alpha, col_order_dev, ncols, d.ncp, L, nullptr,
                                                          1.0f, w.gam);
    FG_LAUNCHED("direct coefficients");
    const int key = (p->cplx ? 4 : 0) | (p->stacktype == FGFRFT_STACK_BF16X2 ? 2 : 0) | (x_complex ? 1 : 0);
    switch (key) {
      case 0: launch_plain<false, false, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 1: launch_plain<false, false, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 2: launch_plain<false, true, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 3: launch_plain<false, true, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 4: launch_plain<true, false, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 5: launch_plain<true, false, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 6: launch_plain<true, true, false>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
      case 7: launch_plain<true, true, true>(p, X, ldx, ncols, d.ncp, w.gam, Y, ldy, s); break;
    }
    FG_LAUNCHED("direct (plain)");
    return FGFRFT_OK;
  }
  fgfrft_status rc = colscale_launch(X, 0, N, ldx, 1, w.xs, w.colpart, s);
  if (rc) return rc;
  k_dcoef<<<ceil_div(nrow * d.ncp, 256), 256, 0, s>>>(alphas_dev, n_alpha, col_order_dev, ncols, d.ncp, L, w.xs,
                                                        bf ? 1.0f : kStackScale, w.gam);
  FG_LAUNCHED("direct coefficients");
  rc = xsplit_launch((const float*)X, ldx, ncols, N, 1, 0, w.xs, 0, w.Xs, s, bf);
  if (rc) return rc;
  const size_t nblocks = (size_t)8 * ceil_div(d.nIB * d.G, 8) * d.ncb;
  if (nblocks > 0x7fffffff) {
    set_error("direct grid too large");
    return FGFRFT_EUNSUPPORTED;
  }
  static bool attr_set = false;
  if (!attr_set) {
    FG_HIP(hipFuncSetAttribute((const void*)k_direct<kDirectNS, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               DCfg::LDS));
    FG_HIP(hipFuncSetAttribute((const void*)k_direct<kDirectNS, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               DCfg::LDS));
    attr_set = true;
  }
  auto kern = bf ? k_direct<kDirectNS, true> : k_direct<kDirectNS, false>;
  kern<<<(unsigned)nblocks, 256, DCfg::LDS, s>>>((const float*)p->stack, (const float*)p->P, N, L, w.Xs, d.ncp, w.gam,
                                                 d.SPW, d.G, d.nIB, d.ncb, w.part_re, w.part_im);
  FG_LAUNCHED("direct");
  const size_t n = (size_t)N * ncols;
  k_direct_reduce<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(w.part_re, w.part_im, d.G, d.gP, N, d.ncp, ncols, L,
                                                              w.gam, (const float*)X, ldx, (cplx64*)Y, ldy);
  FG_LAUNCHED("direct reduce");
  return FGFRFT_OK;
}

}  // namespace fgfrft
