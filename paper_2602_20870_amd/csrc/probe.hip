// Measurement helper: the write bandwidth a plain streaming kernel attains on this device, the
// ceiling for kernels whose traffic is mostly stores (the operator update writes 8 N^2 bytes per
// order and reads the stack once per call).  Not part of the method.
#include "internal.h"

namespace fgfrft {

// Every lane writes 16-byte nontemporal stores, consecutive lanes to consecutive addresses, in a
// grid-stride loop over n16 chunks of 16 bytes.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_write(f32x4* __restrict__ dst, size_t n16, float v) {
  const f32x4 x = {v, v, v, v};
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256)
    __builtin_nontemporal_store(x, dst + i);
}

}  // namespace fgfrft

using namespace fgfrft;

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
