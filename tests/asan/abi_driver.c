/* Drives the library's host-side argument checks under AddressSanitizer and UndefinedBehaviorSanitizer
 * (host code instrumented, no GPU needed): every call below must be refused before anything is
 * enqueued, with the status the header documents, and the error text must be well formed.
 * Exit status 0 iff every expectation holds. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/fgfrft.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
  const char* detail = fgfrft_last_error();
  if (got != want) {
    fprintf(stderr, "FAIL %s: status %d, expected %d (%s)\n", what, got, want, detail);
    ++failures;
  }
  if (strlen(detail) >= 512) {
    fprintf(stderr, "FAIL %s: error text not terminated within its buffer\n", what);
    ++failures;
  }
}

int main(void) {
  size_t pb = 0, sb = 0;
  /* sizes */
  expect(fgfrft_plan_bytes(0, 10, 1, 0, &pb, &sb), FGFRFT_EINVAL, "plan_bytes N=0");
  expect(fgfrft_plan_bytes(32769, 10, 1, 0, &pb, &sb), FGFRFT_EINVAL, "plan_bytes N too large");
  expect(fgfrft_plan_bytes(64, 0, 1, 0, &pb, &sb), FGFRFT_EINVAL, "plan_bytes L=0");
  expect(fgfrft_plan_bytes(64, 65, 0, 0, &pb, &sb), FGFRFT_EINVAL, "plan_bytes L=65");
  expect(fgfrft_plan_bytes(64, 10, 7, 0, &pb, &sb), FGFRFT_EINVAL, "plan_bytes intype");
  expect(fgfrft_plan_bytes(64, 10, 1, 9, &pb, &sb), FGFRFT_EINVAL, "plan_bytes stacktype");
  expect(fgfrft_plan_bytes(32768, 64, 0, 2, &pb, &sb), FGFRFT_OK, "plan_bytes largest");
  if (pb < (size_t)2 * 64 * 32768 * 32768 * 8) { fprintf(stderr, "FAIL plan_bytes overflow\n"); ++failures; }
  expect(fgfrft_plan_bytes(100, 7, 1, 1, NULL, NULL), FGFRFT_OK, "plan_bytes NULL outputs");
  /* plan: bad arguments, nothing allocated or launched */
  fgfrft_plan_t plan = (fgfrft_plan_t)(uintptr_t)1;
  static char buf[4096] __attribute__((aligned(256)));
  expect(fgfrft_plan(NULL, 64, 10, 1, 0, 0, 0.0, buf, 1, buf, 1, NULL, NULL), FGFRFT_EINVAL, "plan out NULL");
  expect(fgfrft_plan(NULL, 64, 10, 1, 0, 0, 0.0, buf, 1, buf, 1, NULL, &plan), FGFRFT_EINVAL, "plan F NULL");
  if (plan != NULL) { fprintf(stderr, "FAIL plan: *out not cleared\n"); ++failures; }
  expect(fgfrft_plan(buf, 64, 10, 1, 0, 5, 0.0, buf, 1, buf, 1, NULL, &plan), FGFRFT_EINVAL, "plan form");
  expect(fgfrft_plan(buf + 1, 64, 10, 1, 0, 0, 0.0, buf, 1 << 30, buf, 1 << 30, NULL, &plan), FGFRFT_EINVAL,
         "plan misaligned F");
  expect(fgfrft_plan(buf, 64, 10, 1, 0, 0, 0.0, buf, 16, buf, 16, NULL, &plan), FGFRFT_ENOMEM,
         "plan persistent too small");
  /* calls on a NULL plan */
  double al[2] = {0.5, -0.5};
  double dal[2];
  expect(fgfrft_plan_info(NULL, NULL, NULL, NULL, NULL, NULL, NULL), FGFRFT_EINVAL, "plan_info NULL");
  expect(fgfrft_plan_buffers(NULL, NULL, NULL), FGFRFT_EINVAL, "plan_buffers NULL");
  expect(fgfrft_update(NULL, al, 2, buf, buf, 256, NULL), FGFRFT_EINVAL, "update NULL plan");
  expect(fgfrft_update_dev(NULL, al, 2, buf, buf, 256, NULL), FGFRFT_EINVAL, "update_dev NULL plan");
  expect(fgfrft_update_dev_static(NULL, al, 2, buf, NULL), FGFRFT_EINVAL, "update_dev_static NULL plan");
  expect(fgfrft_apply(NULL, al, 2, buf, 0, 0, 4, buf, 0, buf, 256, NULL), FGFRFT_EINVAL, "apply NULL plan");
  expect(fgfrft_apply_direct(NULL, al, 2, NULL, buf, 0, 4, 4, buf, 4, buf, 256, NULL), FGFRFT_EINVAL,
         "apply_direct NULL plan");
  expect(fgfrft_grad(NULL, al, 2, buf, 0, 0, 4, buf, dal, NULL, buf, 256, NULL), FGFRFT_EINVAL, "grad NULL plan");
  {
    int bq[2] = {4, 3};
    const void* xs[2] = {buf, buf};
    void* ys[2] = {buf, buf};
    expect(fgfrft_apply_batched(NULL, al, 2, bq, xs, 0, ys, buf, 256, NULL), FGFRFT_EINVAL, "apply_batched NULL plan");
    if (fgfrft_apply_batched_workspace_bytes(NULL, 2, bq, 0) != 0) {
      fprintf(stderr, "FAIL apply_batched workspace query on a NULL plan\n");
      ++failures;
    }
  }
  if (fgfrft_update_workspace_bytes(NULL, 4) != 0 || fgfrft_apply_workspace_bytes(NULL, 4, 4, 0, 0, 0) != 0 ||
      fgfrft_apply_direct_workspace_bytes(NULL, 4, 4) != 0 || fgfrft_grad_workspace_bytes(NULL, 4, 4, 0) != 0) {
    fprintf(stderr, "FAIL workspace queries on a NULL plan\n");
    ++failures;
  }
  fgfrft_destroy(NULL);
  /* plan-free calls */
  expect(fgfrft_apply_operator(buf, 0, 1, 0, buf, 0, 0, 4, buf, 0, buf, 256, NULL), FGFRFT_EINVAL, "apply_operator N=0");
  expect(fgfrft_apply_operator(buf, 64, 1, 0, buf, 0, 0, 4097, buf, 0, buf, 256, NULL), FGFRFT_EINVAL,
         "apply_operator B too large");
  expect(fgfrft_apply_operator(buf + 8, 64, 1, 0, buf, 0, 0, 4, buf, 0, buf, 1 << 20, NULL), FGFRFT_EINVAL,
         "apply_operator misaligned Q");
  expect(fgfrft_apply_operator(buf, 64, 1, 0, buf, 0, 0, 4, buf, 0, buf, 8, NULL), FGFRFT_ENOMEM,
         "apply_operator workspace too small");
  if (fgfrft_apply_operator_workspace_bytes(0, 1, 1, 0) != 0) { fprintf(stderr, "FAIL ws bytes N=0\n"); ++failures; }
  expect(fgfrft_gfrft_exact(buf, buf, (const double*)buf, 0, 0.5, buf, buf, 256, NULL), FGFRFT_EINVAL, "exact N=0");
  expect(fgfrft_gfrft_exact(buf, buf, (const double*)buf, 8, 1.0 / 0.0, buf, buf, 256, NULL), FGFRFT_EALPHA,
         "exact alpha inf");
  expect(fgfrft_gfrft_exact(buf, buf, (const double*)buf, 8, 0.5, buf, buf, 16, NULL), FGFRFT_ENOMEM,
         "exact workspace too small");
  expect(fgfrft_probe_write(NULL, 64, NULL), FGFRFT_EINVAL, "probe_write NULL");
  expect(fgfrft_probe_write(buf, 17, NULL), FGFRFT_EINVAL, "probe_write size");
  expect(fgfrft_apply_dev(NULL, (const double*)buf, 1, buf, 0, 0, 64, buf, buf, 1 << 20, NULL), FGFRFT_EINVAL,
         "apply_dev NULL plan");
  if (fgfrft_apply_dev_workspace_bytes(NULL, 4, 64, 0, 0) != 0) { fprintf(stderr, "FAIL apply_dev ws\n"); ++failures; }
  expect(fgfrft_probe_update_traffic(NULL, 64, 4, 1, buf, NULL), FGFRFT_EINVAL, "probe_update_traffic NULL");
  expect(fgfrft_probe_update_traffic(buf, 96, 4, 1, buf, NULL), FGFRFT_EINVAL, "probe_update_traffic N");
  expect(fgfrft_probe_update_traffic(buf, 64, 0, 1, buf, NULL), FGFRFT_EINVAL, "probe_update_traffic tiles");
  /* error strings */
  for (int c = 1; c >= -9; --c) {
    const char* t = fgfrft_strerror(c);
    if (!t || !*t) { fprintf(stderr, "FAIL strerror(%d)\n", c); ++failures; }
  }
  if (failures == 0) printf("abi driver: all checks passed\n");
  return failures == 0 ? 0 : 1;
}
