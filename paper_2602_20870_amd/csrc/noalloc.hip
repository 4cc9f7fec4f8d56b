// Operator update without any allocation or caller workspace: the coefficient table and the
// epilogue table that fgfrft_update_dev keeps in the caller's workspace live here in one fixed
// device array per GPU instead (for callers that cannot allocate: stream capture, tight serving
// loops).  Same kernels, same results as fgfrft_update_dev.
#include "internal.h"
#include <mutex>

namespace fgfrft {

// Largest order batch of the allocation-free update: its tables need update_ws_bytes(plan, 4096)
// <= 2.1 MiB for every supported L (coefficient table 4096 x 2 x 128 x 2 bytes, epilogue table
// 4096 x 16 bytes, plus the unused 32 KiB order slot at the front of the workspace layout).
constexpr int kStaticMaxOrders = 4096;
constexpr size_t kStaticScratchBytes = (size_t)9 << 18;   // 2.25 MiB

// Device-side storage, one copy per GPU.  Host code never uses this name as an address: it is a
// host-side stand-in there.  Kernels get the device address from hipGetSymbolAddress below.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each GPU, set once

// The device address of this GPU's copy of `scratch`, looked up on the first call made with that
// device current and kept for later calls.
static fgfrft_status scratch_on_current_device(void** out) {
  int dev = 0;
  FG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the static scratch table covers", dev, kMaxDevices);
    return FGFRFT_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    FG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      set_error("hipGetSymbolAddress returned NULL for the static scratch array");
      return FGFRFT_EHIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FGFRFT_OK;
}

}  // namespace fgfrft

using namespace fgfrft;

extern "C" fgfrft_status fgfrft_update_dev_static(fgfrft_plan_t plan, const double* alphas_dev, int n_alpha,
                                                  void* Q_dev, void* stream) {
  if (!plan) { set_error("NULL plan"); return FGFRFT_EINVAL; }
  const Plan* p = (const Plan*)plan;
  if (!alphas_dev || n_alpha < 1) { set_error("alphas_dev is NULL or n_alpha=%d < 1", n_alpha); return FGFRFT_EINVAL; }
  if (n_alpha > kStaticMaxOrders) {
    set_error("n_alpha=%d above the allocation-free update's limit of %d orders per call", n_alpha, kStaticMaxOrders);
    return FGFRFT_EINVAL;
  }
  if (!Q_dev) { set_error("NULL device pointer"); return FGFRFT_EINVAL; }
  if ((uintptr_t)alphas_dev % 8 || (uintptr_t)Q_dev % 8) {
    set_error("alphas_dev and Q_dev must be 8-byte aligned");
    return FGFRFT_EINVAL;
  }
  const size_t need = update_ws_bytes(p, n_alpha);
  if (need > kStaticScratchBytes) {
    set_error("update tables need %zu bytes, above the static scratch of %zu bytes", need, kStaticScratchBytes);
    return FGFRFT_EINVAL;
  }
  void* ws = nullptr;
  fgfrft_status rc = scratch_on_current_device(&ws);
  if (rc) return rc;
  // k_coef writes every entry of the table and epilogue rows the update kernel reads (padding
  // orders included), so nothing left by an earlier call is ever read.
  return update_launch(p, alphas_dev, n_alpha, Q_dev, ws, (hipStream_t)stream);
}
