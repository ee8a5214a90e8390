/* Host-side driver for a build of the library with AddressSanitizer and
 * UndefinedBehaviorSanitizer on its host code (no GPU needed).  It calls
 * every entry point with arguments the host checks refuse, feeds the tuning
 * table reader malformed files, queries the configuration logic over the
 * whole supported size range, and builds ragged multiply and division plans
 * (their host-side scheduling runs in full; the device allocation at the end
 * then fails without a GPU).  A sanitizer report aborts the run; the last
 * line printed on success is "host checks passed". */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "bigint_rocm.h"

static int failures = 0;

static void expect(int cond, const char* what) {
  if (!cond) {
    fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

static void write_file(const char* path, const char* text) {
  FILE* f = fopen(path, "w");
  if (!f) {
    perror(path);
    exit(2);
  }
  fputs(text, f);
  fclose(f);
}

/* deterministic lengths, log-uniform over [lo, hi] (xorshift64) */
static uint64_t rng = 88172645463325252ull;
static uint64_t next_u64(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return rng;
}
static int64_t next_len(int64_t lo, int64_t hi) {
  const double u = (double)(next_u64() >> 11) / 9007199254740992.0;
  int64_t n = (int64_t)llround(exp(log((double)lo) + u * (log((double)hi) - log((double)lo))));
  if (n > hi) n = hi;
  if (n < lo) n = lo;
  return n;
}

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : ".";
  char path[4096];
  uint32_t* p = (uint32_t*)(uintptr_t)0x10000; /* never dereferenced: checks fail first */
  uint32_t* q = (uint32_t*)(uintptr_t)0x20000;

  expect(bigint_version() > 0, "version");
  for (int c = -6; c <= 3; ++c) expect(bigint_strerror(c) != NULL, "strerror");

  /* argument checks */
  expect(bigint_add(NULL, NULL, p, q, 8, 1, NULL) == BIGINT_EINVAL, "add null out");
  expect(bigint_add(p, NULL, p, q, 0, 1, NULL) == BIGINT_EINVAL, "add n = 0");
  expect(bigint_add(p + 1, NULL, p, q, 8, 1, NULL) == BIGINT_EINVAL, "add partial overlap");
  expect(bigint_sub(q, NULL, p, q, -3, 1, NULL) == BIGINT_EINVAL, "sub n < 0");
  expect(bigint_mul(p, p, 8, q, 8, 1, BIGINT_MUL_MFMA, NULL) == BIGINT_EINVAL, "mul overlap");
  expect(bigint_mul(p, q, 8, q, 8, -1, BIGINT_MUL_MFMA, NULL) == BIGINT_EINVAL, "mul batch < 0");
  expect(bigint_mul((uint32_t*)(uintptr_t)0x900000, p, 8, q, 8, 1, 77, NULL) == BIGINT_EINVAL, "mul algo");
  expect(bigint_mul((uint32_t*)(uintptr_t)0x900000, p, 3, q, 4, 1, BIGINT_MUL_KARATSUBA, NULL) ==
             BIGINT_EUNSUPPORTED, "karatsuba unequal");
  expect(bigint_mullo(NULL, p, q, 8, 1, NULL) == BIGINT_EINVAL, "mullo null");
  expect(bigint_add6(NULL, NULL, p, q, 8, 1, NULL) == BIGINT_EINVAL, "add6 null");
  expect(bigint_poly(NULL, p, q, 8, 1, NULL) == BIGINT_EINVAL, "poly null");
  expect(bigint_divmod(NULL, q, NULL, p, 8, q, 4, 1, NULL) == BIGINT_EINVAL, "divmod null");
  expect(bigint_divmod((uint32_t*)(uintptr_t)0x900000, (uint32_t*)(uintptr_t)0xa00000, NULL, p, 20000, q,
                       4, 1, NULL) == BIGINT_EUNSUPPORTED, "divmod too large");
  expect(bigint_divmod_noalloc(NULL, q, NULL, p, 8, q, 4, 1, NULL) == BIGINT_EINVAL, "noalloc null");
  expect(bigint_shinv(NULL, q, 4, 8, 1, NULL) == BIGINT_EINVAL, "shinv null");
  expect(bigint_digits7(NULL, p, 8, 4, 1, NULL) == BIGINT_EINVAL, "digits7 null");
  expect(bigint_conv7(NULL, p, 8, q, 8, 1, NULL) == BIGINT_EINVAL, "conv7 null");
  expect(bigint_plan_create(NULL, BIGINT_OP_MUL, NULL, NULL, 0, 0) == BIGINT_EINVAL, "plan null");
  {
    bigint_plan_t pl = NULL;
    const int64_t la[2] = {4, 0}, lb[2] = {4, 4};
    expect(bigint_plan_create(&pl, BIGINT_OP_MUL, la, lb, 2, 0) == BIGINT_EINVAL && pl == NULL,
           "plan zero length");
    expect(bigint_plan_create(&pl, 9, la, lb, 1, 0) == BIGINT_EINVAL, "plan op");
    expect(bigint_plan_create(&pl, BIGINT_OP_MUL, la, lb, 1, 64) == BIGINT_EINVAL, "plan flags");
    expect(bigint_plan_workspace_size(NULL, NULL) == BIGINT_EINVAL, "workspace null");
    (void)bigint_plan_destroy(NULL);
  }
  expect(bigint_set_mfma_config(5, 0, 0) == BIGINT_EINVAL, "config P");
  expect(bigint_set_mfma_config(0, 3, 0) == BIGINT_EINVAL, "config waves");
  expect(bigint_set_mfma_config(0, 0, 6) == BIGINT_EINVAL, "config digits");
  expect(bigint_set_mfma_tile(24) == BIGINT_EINVAL, "tile");

  /* the configuration logic over every size class (host arithmetic only) */
  for (int64_t n = 1; n <= BIGINT_MFMA_MAX_LIMBS + 8; n += (n < 4096 ? 1 : 7)) {
    int P = 0, w = 0, d = 0, parts = 0;
    const int rc = bigint_mfma_config(n, n, &P, &w, &d);
    expect(rc == BIGINT_OK || n > BIGINT_MFMA_MAX_LIMBS, "config query");
    if (rc == BIGINT_OK) expect((P == 4 || P == 8 || P == 16) && (d == 7 || d == 8), "config values");
    (void)bigint_mfma_tile(n, (n % 5) + 1);
    (void)bigint_mfma_split_parts(n, n, 1 + (n % 300), &parts);
    (void)bigint_mfma_split_parts(n, 1 + n / 3, 1, &parts);
  }

  /* the tuning table reader: malformed, truncated and oversized files */
  {
    static const char* bad[] = {
        "",
        "{}",
        "{\"bins\": []}",
        "{\"bins\": [{\"max_limbs\": 100, \"strips_per_band\": ",
        "{\"bins\": [{\"max_limbs\": 100, \"strips_per_band\": 8, \"waves\": 4}]}",
        "{\"bins\": [{\"max_limbs\": -5, \"strips_per_band\": 8, \"waves\": 4, \"digit_bits\": 8}]}",
        "{\"bins\": [{\"max_limbs\": 99999999999999999999, \"strips_per_band\": 8, \"waves\": 4, "
        "\"digit_bits\": 8}]}",
        "{\"bins\": [{\"max_limbs\": 100, \"strips_per_band\": 32, \"waves\": 8, \"digit_bits\": 8, \"tile\": 16}]}",
        "\"max_limbs\":",
        "\"max_limbs\": 7 \"strips_per_band\": 8 \"waves\": 1 \"digit_bits\": 7 \"tile\":",
    };
    for (size_t i = 0; i < sizeof(bad) / sizeof(bad[0]); ++i) {
      snprintf(path, sizeof(path), "%s/bad%zu.json", dir, i);
      write_file(path, bad[i]);
      expect(bigint_autotune_load(path) == BIGINT_EINVAL, "malformed table refused");
    }
    snprintf(path, sizeof(path), "%s/missing/none.json", dir);
    expect(bigint_autotune_load(path) == BIGINT_EINVAL, "missing file");
    /* a valid table behind a megabyte of padding */
    const size_t pad = 1 << 20;
    char* big = (char*)malloc(pad + 512);
    memset(big, ' ', pad);
    strcpy(big + pad,
           "{\"bins\": [{\"max_limbs\": 2000, \"strips_per_band\": 8, \"waves\": 4, \"digit_bits\": 8}, "
           "{\"max_limbs\": 18432, \"strips_per_band\": 16, \"waves\": 8, \"digit_bits\": 8, \"tile\": 32}]}");
    snprintf(path, sizeof(path), "%s/good.json", dir);
    write_file(path, big);
    free(big);
    expect(bigint_autotune_load(path) == BIGINT_OK, "valid table");
    int P = 0, w = 0, d = 0;
    expect(bigint_mfma_config(1000, 1000, &P, &w, &d) == BIGINT_OK && P == 8 && w == 4 && d == 8,
           "loaded entry");
    expect(bigint_mfma_tile(16384, 16384) == 32, "loaded tile");
    expect(bigint_autotune_load(NULL) == BIGINT_OK, "restore");
    expect(bigint_mfma_config(16384, 16384, &P, &w, &d) == BIGINT_OK && P == 16 && w == 8 && d == 8,
           "built-in entry");
  }

  /* plans: the host-side scheduling runs in full (ragged segments, fillers,
   * splits, the division queue); without a GPU the device allocation that
   * follows fails and the plan is freed */
  int plans_at_alloc = 0, plans_refused = 0, plans_built = 0;
  for (int t = 0; t < 24; ++t) {
    const int64_t batch = 1 + (int64_t)(next_u64() % 5000);
    int64_t* la = (int64_t*)malloc(sizeof(int64_t) * batch);
    int64_t* lb = (int64_t*)malloc(sizeof(int64_t) * batch);
    for (int64_t i = 0; i < batch; ++i) {
      la[i] = next_len(1, t % 3 == 0 ? 18432 : 16384);
      lb[i] = t % 2 ? la[i] : next_len(1, la[i]);
    }
    bigint_plan_t pl = NULL;
    const int op = t % 4 == 3 ? BIGINT_OP_DIVMOD : BIGINT_OP_MUL;
    const int flags = (t % 5 == 1) ? BIGINT_PLAN_PLAIN : ((t % 5 == 2) ? BIGINT_PLAN_NO_GRAPH : 0);
    const int rc = bigint_plan_create(&pl, op, la, lb, batch, flags);
    expect(rc == BIGINT_OK || rc == BIGINT_EHIP || rc == BIGINT_ENOMEM || rc == BIGINT_EUNSUPPORTED,
           "plan status");
    plans_at_alloc += rc == BIGINT_EHIP || rc == BIGINT_ENOMEM;
    plans_refused += rc == BIGINT_EUNSUPPORTED;
    plans_built += rc == BIGINT_OK;
    if (rc == BIGINT_OK) {
      int64_t seg[9 * 16];
      int n = 0;
      (void)bigint_plan_segments(pl, seg, 16, &n);
      size_t ws = 0;
      (void)bigint_plan_workspace_size(pl, &ws);
      bigint_plan_destroy(pl);
    } else {
      expect(pl == NULL, "failed plan not returned");
    }
    free(la);
    free(lb);
  }

  printf("plans: %d built, %d scheduled and stopped at the device allocation, %d refused as too large\n",
         plans_built, plans_at_alloc, plans_refused);
  if (failures) {
    fprintf(stderr, "%d host checks failed\n", failures);
    return 1;
  }
  printf("host checks passed\n");
  return 0;
}
