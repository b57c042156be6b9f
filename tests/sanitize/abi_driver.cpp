// Host sanitizer driver for the library's host-side validation (test
// infrastructure): calls the C ABI with NULL handles, bad dtypes, shapes past
// the limits and sizes large enough to overflow careless arithmetic, all of
// which must be rejected before any device call (no GPU is touched).  Built
// from the library sources, host side only, with the sanitizers, by
// tests/test_sanitizers.py, which fails on any report or a non-zero exit.
#include <stdint.h>
#include <stdio.h>

#include "rsvd.h"

static int fails = 0;
#define EXPECT(cond)                                                               \
  do {                                                                             \
    if (!(cond)) { fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #cond); ++fails; } \
  } while (0)

int main() {
  for (int32_t c = -10; c <= 5; ++c) EXPECT(rsvd_status_string(c) != nullptr);
  rsvd_plan_t h = nullptr;
  EXPECT(rsvd_plan_create(nullptr, 100, 10, 8, RSVD_F32, 0, 0, nullptr) == RSVD_ERR_ARG);
  EXPECT(rsvd_plan_create(&h, 100, 10, 8, 9, 0, 0, nullptr) == RSVD_ERR_ARG);
  EXPECT(rsvd_plan_create(&h, 100, 10, 0, RSVD_F32, 0, 0, nullptr) == RSVD_ERR_ARG);
  EXPECT(rsvd_plan_create(&h, 5, 10, 8, RSVD_F32, 0, 0, nullptr) == RSVD_ERR_SHAPE);
  EXPECT(rsvd_plan_create(&h, 1000, 200, 193, RSVD_F32, 0, 0, nullptr) == RSVD_ERR_SHAPE);
  EXPECT(rsvd_plan_create(&h, 5000, 2000, 32, RSVD_F32, 1, 0, nullptr) == RSVD_ERR_SHAPE);
  EXPECT(rsvd_plan_create(&h, 5000, 200, 32, RSVD_BF16, 1, 0, nullptr) == RSVD_ERR_ARG);
  EXPECT(h == nullptr);
  char buf[256];
  void* a = buf;
  double* d = reinterpret_cast<double*>(buf);
  int32_t* k32 = reinterpret_cast<int32_t*>(buf);
  EXPECT(rsvd_solve(nullptr, a, 100, 10, 10, nullptr, 2, 2, 1, 0.9, a, 2, d, a, 2, k32) ==
         RSVD_ERR_ARG);
  EXPECT(rsvd_solve_krylov(nullptr, a, 100, 10, 10, 2, 2, 1, 0.9, nullptr, a, 2, d, a, 2, k32) ==
         RSVD_ERR_ARG);
  EXPECT(gram_eig_solve(nullptr, a, 100, 10, 10, 0.9, 0, nullptr, 0, d, a, 10, k32) ==
         RSVD_ERR_ARG);
  // allocation-free entry point: every rejection happens on the host
  const int64_t big = (int64_t)1 << 55;
  EXPECT(rsvd_solve_noalloc(a, 1000, 64, 64, RSVD_BF16, 8, 4, 1, 0.9, 1, a, 8, d, a, 8, k32, k32,
                            nullptr) == RSVD_ERR_ARG);
  EXPECT(rsvd_solve_noalloc(a, 10, 64, 64, RSVD_F32, 8, 4, 1, 0.9, 1, a, 8, d, a, 8, k32, k32,
                            nullptr) == RSVD_ERR_SHAPE);
  EXPECT(rsvd_solve_noalloc(a, 2000000, 512, 512, RSVD_F32, 64, 16, 2, 0.9, 1, a, 64, d, a, 64,
                            k32, k32, nullptr) == RSVD_ERR_SHAPE);
  EXPECT(rsvd_solve_noalloc(a, big, 1 << 20, 1 << 20, RSVD_F64, 100, 92, 2, 0.9, 1, a, 100, d, a,
                            100, k32, k32, nullptr) == RSVD_ERR_SHAPE);
  EXPECT(rsvd_solve_noalloc(a, big, big / 2, big / 2, RSVD_F64, 1, 0, 0, 0.9, 1, a, 1, d, a, 1,
                            k32, k32, nullptr) == RSVD_ERR_SHAPE);
  EXPECT(rsvd_solve_noalloc(a, 5000, 512, 512, RSVD_F32, 190, 16, 2, 0.9, 1, a, 190, d, a, 190,
                            k32, k32, nullptr) == RSVD_ERR_SHAPE);
  EXPECT(rsvd_solve_noalloc(a, 1000, 64, 64, RSVD_F32, 8, 4, -1, 0.9, 1, a, 8, d, a, 8, k32, k32,
                            nullptr) == RSVD_ERR_ARG);
  // batches and servers
  rsvd_batch_t b = nullptr;
  EXPECT(rsvd_batch_create(nullptr, 2, 1000, 100, 16, RSVD_F32, 0) == RSVD_ERR_ARG);
  EXPECT(rsvd_batch_create(&b, 0, 1000, 100, 16, RSVD_F32, 0) == RSVD_ERR_ARG);
  EXPECT(rsvd_batch_create(&b, 65, 1000, 100, 16, RSVD_F32, 0) == RSVD_ERR_ARG);
  EXPECT(rsvd_batch_solve(nullptr, nullptr, 0, nullptr) == RSVD_ERR_ARG);
  rsvd_server_t sv = nullptr;
  EXPECT(rsvd_server_create(nullptr, 2, 1000, 100, 16, RSVD_F32, 0, 1 << 30, 0) == RSVD_ERR_ARG);
  EXPECT(rsvd_server_create(&sv, 2, 1000, 100, 16, RSVD_F32, 0, 0, 0) == RSVD_ERR_ARG);
  EXPECT(rsvd_server_create(&sv, 2, 1000, 100, 16, RSVD_F32, 0, 1 << 30, 6) == RSVD_ERR_ARG);
  EXPECT(rsvd_server_create(&sv, 2, 5000, 2000, 16, RSVD_F32, 0, 1 << 30,
                            RSVD_SERVER_GRAM_FALLBACK) == RSVD_ERR_SHAPE);
  EXPECT(rsvd_solve_adaptive(nullptr, a, 100, 10, 10, nullptr, 2, 2, 1, 0.9, 4, a, 4, d, a, 4,
                             k32) == RSVD_ERR_ARG);
  EXPECT(rsvd_server_submit(nullptr, nullptr, nullptr) == RSVD_ERR_ARG);
  EXPECT(rsvd_server_destroy(nullptr) == RSVD_OK);
  EXPECT(rsvd_batch_destroy(nullptr) == RSVD_OK);
  EXPECT(rsvd_plan_destroy(nullptr) == RSVD_OK);
  if (fails) fprintf(stderr, "%d checks failed\n", fails);
  else printf("abi driver ok\n");
  return fails ? 1 : 0;
}
