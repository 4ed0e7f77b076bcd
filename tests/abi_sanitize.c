/*
 * Host-side checks of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Built by tests/test_sanitize.py against a host-only build of the library (no device code; the
 * kernels are never launched).  Every call here either fails its argument checks before any GPU work
 * or computes a size or plan on the host: status codes, workspace sizes, plan queries, backward
 * layouts (tile choice, stored-output blocks), batch-plan validation and the split-step length
 * checks.  Calls that need the GPU return LDBP_EHIP on a machine without one and are accepted
 * either way.  Exits non-zero on the first unexpected status; the sanitizers abort on their own
 * findings.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/ldbp.h"

static int failures = 0;

#define EXPECT(call, want)                                                                       \
  do {                                                                                           \
    const int got_ = (call);                                                                     \
    if (got_ != (want)) {                                                                        \
      fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, #call, got_,      \
              (int)(want), ldbp_last_error());                                                   \
      ++failures;                                                                                \
    }                                                                                            \
  } while (0)

/* status OK, or LDBP_EHIP where the call needs a GPU that is not there */
#define EXPECT_OK_OR_HIP(call)                                                                   \
  do {                                                                                           \
    const int got_ = (call);                                                                     \
    if (got_ != LDBP_OK && got_ != LDBP_EHIP) {                                                  \
      fprintf(stderr, "line %d: %s returned %d (%s)\n", __LINE__, #call, got_, ldbp_last_error()); \
      ++failures;                                                                                \
    }                                                                                            \
  } while (0)

/* fake device addresses: never dereferenced, only checked for NULL, alignment and overlap */
#define FAKE(a) ((void*)(uintptr_t)(a))

static void status_strings(void) {
  const int codes[] = {LDBP_OK, LDBP_EINVAL, LDBP_EWORKSPACE, LDBP_EUNSUPPORTED, LDBP_EHIP, LDBP_ENONFINITE, -99, 7};
  for (size_t i = 0; i < sizeof(codes) / sizeof(codes[0]); ++i) {
    const char* s = ldbp_status_string(codes[i]);
    if (!s || !*s) {
      fprintf(stderr, "empty status string for %d\n", codes[i]);
      ++failures;
    }
  }
  if (!ldbp_version() || !ldbp_last_error()) ++failures;
}

static void forward_sizes(void) {
  const int32_t nt15[50] = {15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15,
                            15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15,
                            15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15, 15};
  const int32_t mixed[7] = {15, 3, 5, 25, 1, 9, 27};
  const int32_t even[3] = {15, 4, 3};
  const int32_t big[2] = {LDBP_MAX_TAPS + 2, 3};
  size_t b = 0;
  for (int dt = 0; dt < 2; ++dt)
    for (int np = 1; np <= 2; ++np) {
      EXPECT(ldbp_forward_workspace_size(dt, np, 64, 65536, 50, nt15, NULL, 0, NULL, &b), LDBP_OK);
      EXPECT(ldbp_forward_workspace_size(dt, np, 3, 3001, 7, mixed, NULL, 0, NULL, &b), LDBP_OK);
      EXPECT(ldbp_forward_workspace_size(dt, np, 2, 1, 7, mixed, NULL, 0, NULL, &b), LDBP_OK);
      for (int32_t s = 1; s <= LDBP_MAX_STEPS_PER_PASS; s += 7) {
        const ldbp_plan p = {s, 0, 0, LDBP_PLAN_SYMMETRIC};
        const int st = ldbp_forward_workspace_size(dt, np, 64, 65536, 50, nt15, NULL, 0, &p, &b);
        if (st != LDBP_OK && st != LDBP_EUNSUPPORTED) ++failures;
      }
      const ldbp_plan guard = {10, 1, 0, LDBP_PLAN_GUARD};
      EXPECT(ldbp_forward_workspace_size(dt, np, 64, 65536, 50, nt15, NULL, 0, &guard, &b), LDBP_OK);
    }
  EXPECT(ldbp_forward_workspace_size(0, 1, 4, 1000, 3, even, NULL, 0, NULL, &b), LDBP_EINVAL);
  EXPECT(ldbp_forward_workspace_size(0, 1, 4, 1000, 2, big, NULL, 0, NULL, &b), LDBP_EINVAL);
  EXPECT(ldbp_forward_workspace_size(0, 3, 4, 1000, 7, mixed, NULL, 0, NULL, &b), LDBP_EUNSUPPORTED);
  EXPECT(ldbp_forward_workspace_size(5, 1, 4, 1000, 7, mixed, NULL, 0, NULL, &b), LDBP_EINVAL);
  EXPECT(ldbp_forward_workspace_size(0, 1, 0, 1000, 7, mixed, NULL, 0, NULL, &b), LDBP_EINVAL);
  EXPECT(ldbp_forward_workspace_size(0, 1, 4, 0, 7, mixed, NULL, 0, NULL, &b), LDBP_EINVAL);
  EXPECT(ldbp_forward_workspace_size(0, 1, 4, 1000, 7, NULL, NULL, 0, NULL, &b), LDBP_EINVAL);
  EXPECT(ldbp_forward_workspace_size(0, 1, 4, 1000, 7, mixed, NULL, 0, NULL, NULL), LDBP_EINVAL);

  int32_t npasses = 0, tile = 0, smax = 0;
  for (int32_t opt = 0; opt <= 9; ++opt) {
    const ldbp_plan p = {10, 1, opt, LDBP_PLAN_SYMMETRIC};
    const int st = ldbp_forward_plan_query(0, 1, 64, 65536, 50, nt15, 0, &p, &npasses, &tile, &smax);
    if (st != LDBP_OK && st != LDBP_EINVAL && st != LDBP_EUNSUPPORTED) ++failures;
  }
  EXPECT(ldbp_forward_plan_query(0, 1, 64, 65536, 50, nt15, 2, NULL, &npasses, &tile, &smax), LDBP_OK);

  const int32_t nl[7] = {41, 41, 41, 41, 41, 41, 41};
  EXPECT(essm_forward_workspace_size(0, 1, 3, 3001, 7, mixed, nl, NULL, 0, NULL, &b), LDBP_OK);
  EXPECT(essm_forward_workspace_size(0, 1, 3, 3001, 7, mixed, NULL, NULL, 0, NULL, &b), LDBP_EINVAL);
  for (int edge = 0; edge <= 3; ++edge) {
    const int st = ldbp_forward_aperiodic_workspace_size(0, 1, 2, 5000, 7, mixed, NULL, edge, NULL, &b);
    if ((edge == LDBP_EDGE_ZERO || edge == LDBP_EDGE_VALID) ? st != LDBP_OK : st != LDBP_EINVAL) {
      fprintf(stderr, "aperiodic edge %d: status %d\n", edge, st);
      ++failures;
    }
  }
}

static void forward_argument_checks(void) {
  const int32_t nt[3] = {15, 3, 5};
  const size_t wave = (size_t)2 * 1000 * 8;
  /* NULL, misaligned and overlapping buffers are rejected before any GPU work */
  EXPECT(ldbp_forward(0, 1, 2, 1000, 3, nt, NULL, FAKE(0x100000), FAKE(0x200000), FAKE(0x300000), NULL, 0, NULL,
                      NULL, 0, NULL),
         LDBP_EINVAL);
  EXPECT(ldbp_forward(0, 1, 2, 1000, 3, nt, FAKE(0x10008), FAKE(0x100000), FAKE(0x200000), FAKE(0x300000), NULL, 0,
                      NULL, NULL, 0, NULL),
         LDBP_EINVAL);
  EXPECT(ldbp_forward(0, 1, 2, 1000, 3, nt, FAKE(0x10000), FAKE(0x100000), FAKE(0x200000),
                      FAKE(0x200000 + wave / 2), NULL, 0, NULL, NULL, 0, NULL),
         LDBP_EINVAL);
  /* the allocation-free forward: beyond its static scratch, refused before any HIP call */
  const ldbp_plan p = {1, 0, 0, 0};
  EXPECT(ldbp_forward_noalloc(0, 1, 1024, 1 << 20, 3, nt, FAKE(0x10000), FAKE(0x100000), FAKE(0x100000000ull),
                              FAKE(0x1000000000ull), NULL, 0, &p, NULL),
         LDBP_EWORKSPACE);
}

static void backward_layouts(void) {
  int32_t nt15[50];
  for (int i = 0; i < 50; ++i) nt15[i] = 15;
  const int32_t nt5[64] = {5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5,
                           5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5,
                           5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5, 5};
  size_t b = 0;
  for (int32_t every = 0; every <= 8; ++every) {
    const void* ck = every > 0 ? FAKE(0x100000) : NULL;
    EXPECT(ldbp_backward_workspace_size(0, 1, 64, 65536, 50, nt15, ck, every, &b), LDBP_OK);
    EXPECT(ldbp_backward_workspace_size(1, 1, 3, 3001, 50, nt15, ck, every, &b), LDBP_OK);
    EXPECT(ldbp_backward_workspace_size(0, 2, 8, 1 << 20, 64, nt5, ck, every, &b), LDBP_OK);
    EXPECT(ldbp_backward_workspace_size(0, 1, 2, 17, 50, nt15, ck, every, &b), LDBP_OK);
  }
  const int32_t nl[50] = {0};
  int32_t nlk[50];
  for (int i = 0; i < 50; ++i) nlk[i] = 41;
  (void)nl;
  EXPECT(essm_backward_workspace_size(0, 1, 64, 65536, 50, nt15, nlk, NULL, 0, &b), LDBP_OK);
  EXPECT(essm_backward_workspace_size(0, 1, 64, 65536, 50, nt15, nlk, FAKE(0x100000), 1, &b), LDBP_OK);
  EXPECT(ldbp_backward_workspace_size(0, 1, 64, 65536, 50, nt15, FAKE(0x100000), 0, &b), LDBP_EINVAL);
  EXPECT(ldbp_backward_workspace_size(0, 1, 64, 65536, 50, nt15, NULL, LDBP_MAX_STEPS_PER_PASS + 1, &b),
         LDBP_EINVAL);
  int32_t even[50];
  memcpy(even, nt15, sizeof(even));
  even[10] = 6;
  EXPECT(ldbp_backward_workspace_size(0, 1, 64, 65536, 50, even, NULL, 0, &b), LDBP_EINVAL);
}

static void batch_plans(void) {
  int64_t len[5] = {4096, 65536, 262144, 100, 1};
  int32_t nstep[5] = {2, 50, 10, 3, 1};
  int32_t taps[66];
  for (int i = 0; i < 66; ++i) taps[i] = 3 + 2 * (i % 4);
  ldbp_batch_plan* plan = NULL;
  EXPECT(ldbp_batch_plan_create(0, 1, 0, len, nstep, taps, NULL, &plan), LDBP_EINVAL);
  EXPECT(ldbp_batch_plan_create(0, 1, 5, NULL, nstep, taps, NULL, &plan), LDBP_EINVAL);
  EXPECT(ldbp_batch_plan_create(0, 1, 5, len, nstep, taps, NULL, NULL), LDBP_EINVAL);
  taps[7] = 4;
  EXPECT(ldbp_batch_plan_create(0, 1, 5, len, nstep, taps, NULL, &plan), LDBP_EINVAL);
  taps[7] = 5;
  plan = NULL;
  EXPECT_OK_OR_HIP(ldbp_batch_plan_create(0, 1, 5, len, nstep, taps, NULL, &plan));
  if (plan) EXPECT(ldbp_batch_plan_destroy(plan), LDBP_OK);

  ssm_link link;
  memset(&link, 0, sizeof(link));
  link.fs = 64e9;
  link.alpha = 4.6e-5;
  link.beta2 = -2.17e-26;
  link.gamma = 1.3e-3;
  link.span_len = 80e3;
  link.kerr_scale = 1.0;
  link.nspan = 3;
  link.nstep = 4;
  link.edfa_gain = 1;
  const int64_t lens_ok[4] = {4096, 4500, 162000, 1 << 16};
  const int32_t nspan[4] = {1, 2, 3, 2};
  size_t b = 0;
  for (int i = 0; i < 4; ++i) EXPECT(ssm_workspace_size(0, 1, 2, lens_ok[i], &link, &b), LDBP_OK);
  EXPECT(ssm_workspace_size(0, 1, 2, 4097, &link, &b), LDBP_EUNSUPPORTED);
  EXPECT(ssm_workspace_size(0, 3, 2, 4096, &link, &b), LDBP_EUNSUPPORTED);
  ssm_batch_plan* sp = NULL;
  EXPECT(ssm_batch_plan_create(0, 1, 4, lens_ok, nspan, &link, 2, &sp), LDBP_EINVAL);
  const int64_t lens_bad[2] = {4096, 4097 * 7};
  EXPECT(ssm_batch_plan_create(0, 1, 2, lens_bad, nspan, &link, 1, &sp), LDBP_EUNSUPPORTED);
  sp = NULL;
  EXPECT_OK_OR_HIP(ssm_batch_plan_create(0, 1, 4, lens_ok, nspan, &link, 1, &sp));
  if (sp) EXPECT(ssm_batch_plan_destroy(sp), LDBP_OK);

  EXPECT(ldbp_fft_workspace_size(0, 1, 4, 4500, &b), LDBP_OK);
  EXPECT(ldbp_fft_workspace_size(0, 1, 4, 4097, &b), LDBP_EUNSUPPORTED);
  EXPECT(tx_shape_workspace_size(0, 1, 4, 8192, 2, &b), LDBP_OK);
  EXPECT(rx_lpf_decimate_workspace_size(0, 1, 4, 16384, 8192, &b), LDBP_OK);
  EXPECT(rx_mse_workspace_size(0, 1, 4, 4096, 2, &b), LDBP_OK);
}

int main(void) {
  status_strings();
  forward_sizes();
  forward_argument_checks();
  backward_layouts();
  batch_plans();
  if (failures) {
    fprintf(stderr, "%d unexpected statuses\n", failures);
    return 1;
  }
  printf("abi_sanitize: ok\n");
  return 0;
}
