/*
 * abi_driver.c -- calls every entry point of librid with a null handle and
 * with invalid sizes, pointers and leading dimensions, checking that each
 * returns its argument error before touching a device.  Built against a
 * copy of the library whose host code is instrumented with AddressSanitizer
 * and UndefinedBehaviorSanitizer, it checks the host-side argument
 * arithmetic for undefined behaviour (overflow in size products, bad
 * shifts) and bad memory accesses.  CPU only: no call reaches the GPU.
 */
#include <stdint.h>
#include <stdio.h>

#include "rid.h"

static int fails = 0;
#define EXPECT(cond)                                                       \
  do {                                                                     \
    if (!(cond)) {                                                         \
      fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                             \
    }                                                                      \
  } while (0)

int main(void) {
  char buf[4096] __attribute__((aligned(64)));
  void *p = buf, *odd = buf + 8;
  int64_t J[4] = {0, 1, 2, 3};
  double sig;
  uint64_t used;
  const int64_t huge = INT64_C(1) << 62;
  const rid_status INV = RID_ERR_INVALID_ARG;
  EXPECT(rid_create(NULL, 0) == INV);
  EXPECT(rid_destroy(NULL) == RID_OK);
  EXPECT(rid_last_hip_error(NULL) == 0);
  EXPECT(rid_reserve(NULL, 1, 1, 1, 1) == INV);
  EXPECT(rid_reserve(NULL, -1, 1, 1, 1) == INV);
  EXPECT(rid_set_qr(NULL, 0) == INV);
  EXPECT(rid_set_sketch(NULL, 0) == INV);
  EXPECT(rid_gaussian(NULL, NULL, huge, huge, 0, 0, p, huge) == INV);
  EXPECT(rid_gaussian(NULL, NULL, -1, 4, 0, 0, p, 4) == INV);
  EXPECT(rid_srft_operator(NULL, NULL, 4, huge, 0, p, huge) == INV);
  EXPECT(rid_sketch(NULL, NULL, RID_C128, RID_FP64, huge, huge, huge, p, huge, 0, p, huge) ==
         INV);
  EXPECT(rid_sketch(NULL, NULL, RID_C128, RID_FP64, 8, 4, 2, odd, 8, 0, p, 2) == INV);
  EXPECT(rid_sketch_explicit(NULL, NULL, RID_C64, RID_BF16X2, 8, 4, 2, p, 8, p, 8, p, 2) ==
         INV);
  EXPECT(rid_pivqr(NULL, NULL, huge, huge, huge, p, huge, J, NULL, 1e-12) == INV);
  EXPECT(rid_pivqr(NULL, NULL, 4, 8, 2, odd, 4, J, NULL, -1.0) == INV);
  EXPECT(rid_interp(NULL, NULL, huge, huge, p, huge, J, p, huge) == INV);
  EXPECT(rid_residual(NULL, NULL, RID_C128, RID_FP64, huge, huge, huge, p, huge, J, p, huge,
                      1, 0, &sig, NULL) == INV);
  EXPECT(rid_decompose(NULL, NULL, RID_C128, RID_FP64, huge, huge, huge, huge, p, huge, 0, 1,
                       0, 1e-12, J, p, huge, &sig, &used) == INV);
  EXPECT(rid_decompose_explicit(NULL, NULL, RID_C128, RID_FP64, 8, 4, 2, 2, p, 8, NULL, 8, 0,
                                1, 0, 1e-12, J, p, 2, &sig, &used) == INV);
  EXPECT(rid_svd(NULL, NULL, RID_C128, huge, huge, huge, p, huge, J, p, huge, p, huge, &sig, p,
                 huge, NULL) == INV);
  EXPECT(rid_query_status(NULL, NULL) == INV);
  EXPECT(rid_profile(NULL, 1) == INV);
  EXPECT(rid_profile_read(NULL, 0, NULL, NULL) == INV);
  {
    rid_job job = {8, 4, 2, 2, p, 8, 0, J, p, 2, &sig};
    int st;
    EXPECT(rid_decompose_batched(NULL, NULL, RID_C128, RID_FP64, &job, 1, 1, 0, 1e-12, &st,
                                 &used) == INV);
    EXPECT(rid_tune_batched(NULL, NULL, RID_C128, RID_FP64, &job, 1, 1, NULL, NULL, NULL) ==
           INV);
  }
  EXPECT(rid_set_batch_plan(NULL, 1024, 1 << 18, 8) == INV);
  EXPECT(rid_get_batch_plan(NULL, NULL, NULL, NULL) == INV);
  {
    rid_server s = NULL;
    rid_server_config bad = {0, 1, 1, 1, 8};
    EXPECT(rid_server_create(&s, 0, &bad, NULL, NULL, NULL) == INV);
    EXPECT(rid_server_submit(NULL, NULL, NULL) == INV);
    EXPECT(rid_server_drain(NULL) == INV);
    EXPECT(rid_server_stats(NULL, NULL, NULL, NULL) == INV);
    EXPECT(rid_server_destroy(NULL) == INV);
  }
  EXPECT(rid_status_string(12345) != NULL);
  if (fails) {
    fprintf(stderr, "%d check(s) failed\n", fails);
    return 1;
  }
  printf("argument checks under sanitizers: all checks passed\n");
  return 0;
}
