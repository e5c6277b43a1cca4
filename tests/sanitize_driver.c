/* Host-only driver of the C-ABI's validation and workspace-size paths, built
 * with AddressSanitizer and UndefinedBehaviorSanitizer on the host side of
 * the library (tests/test_sanitize.py).  No device is touched: every call is
 * a size query or an argument the library must refuse before launching.
 * Device pointers are a fake non-NULL address that validation never reads.
 * Exits non-zero on the first unexpected status; the sanitizers abort on any
 * invalid host access or undefined operation. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "tkmi.h"

#define FAKE ((void*)0x10000)

static int failures = 0;

static void expect(const char* what, tk_status got, tk_status want) {
  if (got != want) {
    fprintf(stderr, "FAIL %s: status %d, expected %d (%s)\n", what, (int)got, (int)want, tk_last_error());
    ++failures;
  }
}

static tk_tensor tensor(int order, const int64_t* dims, int dtype) {
  tk_tensor t;
  memset(&t, 0, sizeof(t));
  t.order = order;
  t.dtype = dtype;
  for (int k = 0; k < order; ++k) t.dims[k] = dims[k];
  t.data = FAKE;
  return t;
}

static tk_sketch sketch(int64_t s, int32_t ell) {
  tk_sketch k;
  k.s = s;
  k.ell = ell;
  k.reserved = 0;
  k.idx = (const int64_t*)FAKE;
  k.omega = FAKE;
  return k;
}

static void sketch_paths(void) {
  const int64_t dims[3] = {8, 9, 10};
  tk_tensor X = tensor(3, dims, TK_F32);
  tk_sketch sk[3] = {sketch(20, 5), sketch(30, 5), sketch(40, 5)};
  double* Z[3] = {(double*)FAKE, (double*)FAKE, (double*)FAKE};
  size_t n = 0;
  expect("sketch query", tucker_sketch_all_modes(&X, sk, Z, NULL, NULL, &n, NULL), TK_OK);
  sk[0].s = 4;   /* ell > s */
  expect("sketch ell > s", tucker_sketch_all_modes(&X, sk, Z, NULL, NULL, &n, NULL), TK_EINVAL);
  sk[0].s = 91;  /* more than the 90 columns */
  expect("sketch s > ncols", tucker_sketch_all_modes(&X, sk, Z, NULL, NULL, &n, NULL), TK_EINVAL);
  sk[0].s = 20;
  expect("sketch NULL X", tucker_sketch_all_modes(NULL, sk, Z, NULL, NULL, &n, NULL), TK_EINVAL);
  expect("sketch NULL size", tucker_sketch_all_modes(&X, sk, Z, NULL, NULL, NULL, NULL), TK_EINVAL);
  /* dimensions whose product overflows 64 bits */
  const int64_t huge[4] = {INT64_C(1) << 31, INT64_C(1) << 31, INT64_C(1) << 31, 3};
  tk_tensor H = tensor(4, huge, TK_F32);
  tk_sketch hs[4] = {sketch(20, 5), sketch(30, 5), sketch(40, 5), sketch(40, 2)};
  double* HZ[4] = {(double*)FAKE, (double*)FAKE, (double*)FAKE, (double*)FAKE};
  expect("sketch overflowing dims", tucker_sketch_all_modes(&H, hs, HZ, NULL, NULL, &n, NULL), TK_EINVAL);
  const int64_t zero[3] = {8, 0, 10};
  tk_tensor Z0 = tensor(3, zero, TK_F32);
  expect("sketch zero dim", tucker_sketch_all_modes(&Z0, sk, Z, NULL, NULL, &n, NULL), TK_EINVAL);
  tk_tensor O = tensor(3, dims, TK_F32);
  O.order = TK_MAX_ORDER + 1;
  expect("sketch order too large", tucker_sketch_all_modes(&O, sk, Z, NULL, NULL, &n, NULL), TK_EINVAL);
  O.order = 3;
  O.dtype = 7;
  expect("sketch bad dtype", tucker_sketch_all_modes(&O, sk, Z, NULL, NULL, &n, NULL), TK_EINVAL);
}

static void qr_paths(void) {
  const int64_t m[2] = {256, 100};
  const int32_t ell[2] = {42, 30};
  const int64_t s[2] = {2560, 900};
  const int32_t r[2] = {32, 20};
  double* Z[2] = {(double*)FAKE, (double*)FAKE};
  const void* Y[2] = {FAKE, FAKE};
  void* U[2] = {FAKE, FAKE};
  size_t n = 0;
  expect("qr query", tucker_qr(2, m, ell, Z, Y, TK_F32, s, r, U, TK_F32, NULL, NULL, &n, NULL), TK_OK);
  const int32_t rbad[2] = {43, 20};
  expect("qr rank > ell", tucker_qr(2, m, ell, Z, Y, TK_F32, s, rbad, U, TK_F32, NULL, NULL, &n, NULL), TK_EINVAL);
  expect("qr no matrices", tucker_qr(0, m, ell, Z, Y, TK_F32, s, r, U, TK_F32, NULL, NULL, &n, NULL), TK_OK);
  expect("qr negative count", tucker_qr(-1, m, ell, Z, Y, TK_F32, s, r, U, TK_F32, NULL, NULL, &n, NULL), TK_EINVAL);
}

static void core_paths(void) {
  const int64_t dims[4] = {64, 48, 40, 132};
  tk_tensor X = tensor(4, dims, TK_F32);
  const void* F[4] = {FAKE, FAKE, FAKE, FAKE};
  const int32_t cols[4] = {8, 6, 31, 32};
  size_t n = 0;
  expect("core query", tucker_core(&X, F, cols, FAKE, NULL, &n, NULL), TK_OK);
  const int32_t wide[4] = {8, 6, 31, 193};
  expect("core c > 192", tucker_core(&X, F, wide, FAKE, NULL, &n, NULL), TK_EINVAL);
  expect("reconstruct query",
         tucker_reconstruct(4, dims, TK_F32, FAKE, F, cols, &X, NULL, (double*)FAKE, NULL, &n, NULL), TK_OK);
  expect("reconstruct no output",
         tucker_reconstruct(4, dims, TK_F32, FAKE, F, cols, &X, NULL, NULL, NULL, &n, NULL), TK_EINVAL);
}

static void ht_paths(void) {
  /* balanced heap tree of order 4: root {0..3}, {0,1}, {2,3}, leaves */
  const int32_t left[7] = {1, 3, 5, -1, -1, -1, -1};
  const int32_t right[7] = {2, 4, 6, -1, -1, -1, -1};
  const int32_t first[7] = {0, 0, 2, 0, 1, 2, 3};
  const int32_t num[7] = {4, 2, 2, 1, 1, 1, 1};
  tk_tree tr = {7, left, right, first, num};
  const int64_t dims[4] = {18, 18, 18, 18};
  tk_tensor X = tensor(4, dims, TK_F32);
  const int32_t rank[7] = {0, 12, 12, 6, 6, 6, 6};
  tk_sketch sk[7];
  for (int t = 0; t < 7; ++t) sk[t] = sketch(200, 11);
  void* U[7] = {FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE};
  void* Bt[7] = {FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE};
  size_t n = 0;
  tk_status st = htucker_decompose(&X, &tr, rank, sk, U, Bt, NULL, NULL, &n, NULL);
  /* whatever the sketch sizes require, the call answers without touching memory */
  if (st != TK_OK && st != TK_EINVAL) expect("htucker query", st, TK_OK);
  const int32_t bad_left[7] = {1, 3, 5, -1, -1, -1, 9};
  tk_tree bad = {7, bad_left, right, first, num};
  expect("htucker bad tree", htucker_decompose(&X, &bad, rank, sk, U, Bt, NULL, NULL, &n, NULL), TK_EINVAL);
}

static void batch_paths(void) {
  const int64_t dims[3] = {20, 30, 40};
  tk_tensor X[1] = {tensor(3, dims, TK_F32)};
  const int32_t ranks[3] = {3, 4, 5};
  tk_sketch sk[3] = {sketch(200, 8), sketch(300, 9), sketch(400, 10)};
  void* U[3] = {FAKE, FAKE, FAKE};
  void* G[1] = {FAKE};
  size_t n = 0, nr = 0;
  expect("batch query", tucker_batch_plan_create(1, X, ranks, sk, U, G, NULL, NULL, NULL, &n, NULL, NULL), TK_OK);
  expect("batch query with residual",
         tucker_batch_plan_create(1, X, ranks, sk, U, G, NULL, (double*)FAKE, NULL, &nr, NULL, NULL), TK_OK);
  if (!(nr > n)) {
    fprintf(stderr, "FAIL batch residual workspace %zu <= %zu\n", nr, n);
    ++failures;
  }
  expect("batch count 0", tucker_batch_plan_create(0, X, ranks, sk, U, G, NULL, NULL, NULL, &n, NULL, NULL),
         TK_EINVAL);
  const int64_t wide[3] = {20, 300, 40};
  tk_tensor W[1] = {tensor(3, wide, TK_F32)};
  expect("batch wide trailing mode",
         tucker_batch_plan_create(1, W, ranks, sk, U, G, NULL, NULL, NULL, &n, NULL, NULL), TK_EUNSUPPORTED);
  expect("batch run NULL plan", tucker_batch_run(NULL, NULL), TK_EINVAL);
  tucker_batch_plan_destroy(NULL);
}

static void draw_paths(void) {
  const int64_t ncols[2] = {90, 80};
  const int32_t s[2] = {20, 81};    /* s > ncols for the second unit */
  const int32_t ell[2] = {5, 4};
  int64_t* idx[2] = {(int64_t*)FAKE, (int64_t*)FAKE};
  void* om[2] = {FAKE, FAKE};
  expect("draw s > ncols", tucker_draw_sketches(2, ncols, s, ell, 7, idx, om, TK_F32, NULL), TK_EINVAL);
  expect("draw bad dtype", tucker_draw_sketches(1, ncols, s, ell, 7, idx, om, TK_BF16, NULL), TK_EINVAL);
  expect("draw no units", tucker_draw_sketches(0, ncols, s, ell, 7, idx, om, TK_F32, NULL), TK_EINVAL);
}

int main(void) {
  if (strncmp(tk_version(), "tkmi", 4) != 0) {
    fprintf(stderr, "FAIL version %s\n", tk_version());
    return 1;
  }
  sketch_paths();
  qr_paths();
  core_paths();
  ht_paths();
  batch_paths();
  draw_paths();
  if (failures) return 1;
  printf("sanitized validation paths: ok\n");
  return 0;
}
