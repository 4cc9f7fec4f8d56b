// Grouped apply for serving (batch.hip; not part of the ABI).
#pragma once
#include "internal.h"

namespace fgfrft {

// Request r has order alphas[r] and signals X[r] ([N][B_per_req[r]], float32 or complex64) and gets
// complex64 Y[r] ([N][B_per_req[r]]).  Requests are taken in groups of kBatchReq whose table travels
// as a kernel argument; per group one gather, one direct-route pass and one scatter.
constexpr int kBatchReq = 64, kBatchRows = 32;
struct BatchTable {
  const void* x[kBatchReq];
  void* y[kBatchReq];
  int off[kBatchReq];     // first column of the request in the gathered block
  int b[kBatchReq];       // its signal count
  double alpha[kBatchReq];
};
size_t batched_ws_bytes(const Plan* p, int n_req, const int* B_per_req, int x_complex);
fgfrft_status batched_launch(const Plan* p, const double* alphas, int n_req, const int* B_per_req,
                             const void* const* X, int x_complex, void* const* Y, void* ws, hipStream_t s);

}  // namespace fgfrft
