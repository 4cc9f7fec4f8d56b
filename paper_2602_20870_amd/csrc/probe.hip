// Measurement helpers, not part of the method: the write bandwidth a plain streaming kernel attains
// on this device, and the time the operator update's own traffic takes with no arithmetic (the
// update writes 8 N^2 bytes per order and reads its stack tiles once per call).
#include "internal.h"

namespace fgfrft {

// Every lane writes 16-byte nontemporal stores, consecutive lanes to consecutive addresses, in a
// grid-stride loop over n16 chunks of 16 bytes.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_stream_write(f32x4* __restrict__ dst, size_t n16, float v) {
  const f32x4 x = {v, v, v, v};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256)
    __builtin_nontemporal_store(x, dst + i);
}

// The operator update's traffic without its arithmetic: one workgroup per strip of 4 rows x 64
// positions (two per CU, as the update), which stages its tiles of nt row-major N x N matrices of
// 4-byte values (4 rows x 256 bytes each) in LDS with direct loads, waits for them, then writes the
// strip's positions of every order as complex64 with nontemporal stores: wave w writes row w,
// orders in sequence, one 512-byte run per store, as the update's paired epilogue does.
__global__ __launch_bounds__(256, 2) void k_update_traffic(const char* __restrict__ src, int N, int nt, int n_alpha,
                                                          f32x2* __restrict__ dst) {
  extern __shared__ __align__(16) float lds_f[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int spr = N / 64, r0 = (blockIdx.x / spr) * 4, c0 = (blockIdx.x % spr) * 64;
  const size_t NN = (size_t)N * N;
  const uint32_t off = (uint32_t)(((size_t)(r0 + (lane >> 4)) * N + c0) * 4 + (lane & 15) * 16);
  for (int t = w; t < nt; t += 4)
    lds_dma16(src + (size_t)t * NN * 4 + off, __builtin_amdgcn_readfirstlane(lds_addr((const char*)lds_f + t * 1024)));
  __builtin_amdgcn_s_waitcnt(wait_vm_lgkm0(0));
  __syncthreads();
  float x = 0.f;
  for (int t = 0; t < nt; ++t) x += lds_f[t * 256 + w * 64 + lane];   // keeps the loads live
  const f32x2 v = {x, -x};
  f32x2* q = dst + (size_t)(r0 + w) * N + c0 + lane;
  for (int a = 0; a < n_alpha; ++a) __builtin_nontemporal_store(v, q + (size_t)a * NN);
}

}  // namespace fgfrft

using namespace fgfrft;

extern "C" fgfrft_status fgfrft_probe_update_traffic(const void* src_dev, int N, int n_tiles, int n_alpha,
                                                     void* dst_dev, void* stream) {
  if (!src_dev || !dst_dev || N < 64 || N % 64 || N > 32704 || n_tiles < 1 || n_tiles > 65 || n_alpha < 1 ||
      (uintptr_t)src_dev % 16 || (uintptr_t)dst_dev % 8) {
    set_error("fgfrft_probe_update_traffic: non-NULL aligned buffers, N a multiple of 64 in [64, 32704], "
              "1 <= n_tiles <= 65, n_alpha >= 1");
    return FGFRFT_EINVAL;
  }
  const size_t strips = (size_t)N * N / 256;
  if (strips > 0x7fffffff) {
    set_error("fgfrft_probe_update_traffic: grid too large");
    return FGFRFT_EINVAL;
  }
  const int lds = n_tiles * 1024;
  (void)raise_lds_limit((const void*)k_update_traffic, lds);   // a failure surfaces at the launch
  k_update_traffic<<<(unsigned)strips, 256, lds, (hipStream_t)stream>>>((const char*)src_dev, N, n_tiles, n_alpha,
                                                                         (f32x2*)dst_dev);
  FG_LAUNCHED("update traffic");
  return FGFRFT_OK;
}

extern "C" fgfrft_status fgfrft_probe_write(void* dst_dev, size_t bytes, void* stream) {
  if (!dst_dev || bytes == 0 || bytes % 16 || (uintptr_t)dst_dev % 16) {
    set_error("fgfrft_probe_write: dst_dev must be non-NULL and 16-byte aligned, bytes a nonzero multiple of 16");
    return FGFRFT_EINVAL;
  }
  const size_t n16 = bytes / 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;     // 64 workgroups per compute unit, grid-stride beyond
  k_stream_write<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>((f32x4*)dst_dev, n16, 0.f);
  FG_LAUNCHED("stream write");
  return FGFRFT_OK;
}
