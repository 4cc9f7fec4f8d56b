// Grouped apply (Definition 2 for many requests at once): requests with their own orders and
// signal counts go through one pass of the direct route.  The request table travels as a kernel
// argument (nothing is copied from the host, so the call can be captured), the requests' signals are
// gathered into one column block, the direct route runs once over it, and the results are
// scattered back to the requests' outputs.
#include "batch.h"

namespace fgfrft {

template <typename T>
__global__ __launch_bounds__(256) void k_batch_gather(BatchTable tab, int N, int ldc, T* __restrict__ Xc,
                                                      int* __restrict__ col_order, double* __restrict__ alphas) {
  const int r = blockIdx.y, B = tab.b[r], off = tab.off[r];
  if (B == 0) return;
  const T* x = (const T*)tab.x[r];
  if (blockIdx.x == 0) {
    for (int c = threadIdx.x; c < B; c += 256) col_order[off + c] = r;
    if (threadIdx.x == 0) alphas[r] = tab.alpha[r];
  }
  const int n0 = blockIdx.x * kBatchRows, nr = N - n0 < kBatchRows ? N - n0 : kBatchRows;
  for (int e = threadIdx.x; e < nr * B; e += 256) {
    const int n = n0 + e / B, c = e % B;
    Xc[(size_t)n * ldc + off + c] = x[(size_t)n * B + c];
  }
}

__global__ __launch_bounds__(256) void k_batch_scatter(BatchTable tab, int N, int ldc, const cplx64* __restrict__ Yc) {
  const int r = blockIdx.y, B = tab.b[r], off = tab.off[r];
  if (B == 0) return;
  cplx64* y = (cplx64*)tab.y[r];
  const int n0 = blockIdx.x * kBatchRows, nr = N - n0 < kBatchRows ? N - n0 : kBatchRows;
  for (int e = threadIdx.x; e < nr * B; e += 256) {
    const int n = n0 + e / B, c = e % B;
    y[(size_t)n * B + c] = Yc[(size_t)n * ldc + off + c];
  }
}

// workspace of one group of requests with ncols columns in all, and the offsets of its parts
static size_t batch_group_ws(const Plan* p, int ncols, int x_complex, size_t* o_col, size_t* o_x, size_t* o_y,
                             size_t* o_d) {
  const size_t N = p->N, xe = x_complex ? 8 : 4;
  size_t s = align_up((size_t)kBatchReq * 8, 256);   // orders of the group
  if (o_col) *o_col = s;
  s += align_up((size_t)ncols * 4, 256);               // column -> request
  if (o_x) *o_x = s;
  s += align_up(N * ncols * xe, 256);                  // gathered signals [N][ncols]
  if (o_y) *o_y = s;
  s += align_up(N * ncols * 8, 256);                   // results [N][ncols]
  if (o_d) *o_d = s;
  s += direct_ws_bytes(p, ncols, ncols);
  return s;
}

size_t batched_ws_bytes(const Plan* p, int n_req, const int* B_per_req, int x_complex) {
  size_t best = 0;
  for (int g0 = 0; g0 < n_req; g0 += kBatchReq) {
    int cols = 0;
    for (int r = g0; r < n_req && r < g0 + kBatchReq; ++r) cols += B_per_req[r];
    const size_t s = batch_group_ws(p, cols > 0 ? cols : 1, x_complex, nullptr, nullptr, nullptr, nullptr);
    if (s > best) best = s;
  }
  return best;
}

fgfrft_status batched_launch(const Plan* p, const double* alphas, int n_req, const int* B_per_req,
                             const void* const* X, int x_complex, void* const* Y, void* ws, hipStream_t s) {
  const int N = p->N;
  for (int g0 = 0; g0 < n_req; g0 += kBatchReq) {
    const int ng = n_req - g0 < kBatchReq ? n_req - g0 : kBatchReq;
    BatchTable tab = {};
    int cols = 0;
    for (int r = 0; r < ng; ++r) {
      tab.x[r] = X[g0 + r];
      tab.y[r] = Y[g0 + r];
      tab.b[r] = B_per_req[g0 + r];
      tab.off[r] = cols;
      tab.alpha[r] = alphas[g0 + r];
      cols += tab.b[r];
    }
    if (cols == 0) continue;
    size_t oc, ox, oy, od;
    batch_group_ws(p, cols, x_complex, &oc, &ox, &oy, &od);
    char* w = (char*)ws;
    double* al = (double*)w;
    int* col = (int*)(w + oc);
    void* Xc = w + ox;
    cplx64* Yc = (cplx64*)(w + oy);
    const dim3 grid(ceil_div(N, kBatchRows), ng);
    if (x_complex) k_batch_gather<cplx64><<<grid, 256, 0, s>>>(tab, N, cols, (cplx64*)Xc, col, al);
    else k_batch_gather<float><<<grid, 256, 0, s>>>(tab, N, cols, (float*)Xc, col, al);
    FG_LAUNCHED("batch gather");
    fgfrft_status rc = direct_launch(p, al, ng, col, Xc, x_complex, cols, cols, Yc, cols, w + od, s);
    if (rc) return rc;
    k_batch_scatter<<<grid, 256, 0, s>>>(tab, N, cols, Yc);
    FG_LAUNCHED("batch scatter");
  }
  return FGFRFT_OK;
}

}  // namespace fgfrft
