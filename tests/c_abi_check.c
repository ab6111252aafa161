/* A plain C99 caller of libsvd2: include/svd2.h must compile as C and every
 * call below must link and return the documented status without a GPU (each
 * is refused by the host-side argument checks before any HIP call, or is a
 * pure host query).  Exit status 0 when all hold; otherwise the number of
 * failed checks. */
#include <stdio.h>
#include <stdint.h>
#include "svd2.h"

static int failures = 0;
#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      fprintf(stderr, "c_abi_check: failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

int main(void) {
  hipStream_t st = (hipStream_t)0;
  dsvd2_args d = {0};
  zsvd2_args z = {0};
  ssvd2_args s = {0};
  csvd2_args c = {0};
  /* batched SVD: missing arrays, then contradictory flags */
  CHECK(dsvd2_batch(16, &d, SVD2_BACKSCALE_NONE, st) == SVD2_ERR_NULL);
  CHECK(zsvd2_batch(16, &z, SVD2_BACKSCALE_SAFE, st) == SVD2_ERR_NULL);
  CHECK(ssvd2_batch(16, &s, SVD2_RESCUE_FP64, NULL, 0, st) == SVD2_ERR_NULL);
  CHECK(csvd2_batch(16, &c, SVD2_RESCUE_FP64 | SVD2_RESCUE_SIGMA, NULL, 0, st) == SVD2_ERR_NULL);
  CHECK(dsvd2_batch(16, NULL, 0, st) == SVD2_ERR_NULL);
  CHECK(dsvd2_batch(16, &d, SVD2_BACKSCALE_SAFE | SVD2_BACKSCALE_ALL, st) == SVD2_ERR_FLAGS);
  CHECK(dsvd2_batch(16, &d, SVD2_RESCUE_FP64, st) == SVD2_ERR_FLAGS);
  CHECK(ssvd2_batch(16, &s, SVD2_RESCUE_SIGMA, NULL, 0, st) == SVD2_ERR_FLAGS);
  CHECK(ssvd2_batch(16, &s, SVD2_RESCUE_FP64 | SVD2_RESCUE_SIGMA | SVD2_RESCUE_TRI, NULL, 0, st) ==
        SVD2_ERR_FLAGS);
  /* phase outputs: missing structs or arrays, backscale refused */
  {
    dsvd2_urv df = {0};
    zsvd2_urv zf = {0};
    ssvd2_urv sf = {0};
    csvd2_urv cf = {0};
    CHECK(dsvd2_batch_urv(16, &d, NULL, 0, st) == SVD2_ERR_NULL);
    CHECK(dsvd2_batch_urv(16, &d, &df, 0, st) == SVD2_ERR_NULL);
    CHECK(zsvd2_batch_urv(16, &z, &zf, SVD2_BACKSCALE_SAFE, st) == SVD2_ERR_FLAGS);
    CHECK(ssvd2_batch_urv(16, &s, &sf, SVD2_RESCUE_FP64, NULL, 0, st) == SVD2_ERR_NULL);
    CHECK(csvd2_batch_urv(16, &c, &cf, SVD2_RESCUE_FP64 | SVD2_BACKSCALE_ALL, NULL, 0, st) == SVD2_ERR_FLAGS);
    CHECK(csvd2_batch_urv(0, &c, &cf, SVD2_RESCUE_SIGMA, NULL, 0, st) == SVD2_ERR_FLAGS);
  }
  /* workspace queries and launch shapes */
  CHECK(svd2_workspace_bytes(1000, SVD2_RESCUE_FP64) == 0);
  CHECK(svd2_workspace_bytes(1000, SVD2_RESCUE_FP64 | SVD2_RESCUE_QUEUE) >= 1000 * sizeof(uint32_t));
  CHECK(svd2_set_launch_kind(1, 96, 1) == SVD2_ERR_SIZE);
  CHECK(svd2_set_launch_kind(9, 128, 1) == SVD2_ERR_FLAGS);
  {
    int b0 = 0, p0 = 0, b = 0, p = 0;
    svd2_get_launch_kind(2, &b0, &p0);
    CHECK(svd2_set_launch_kind(2, 128, 2) == SVD2_OK);
    svd2_get_launch_kind(2, &b, &p);
    CHECK(b == 128 && p == 2);
    CHECK(svd2_set_launch_kind(2, b0, p0) == SVD2_OK);
  }
  CHECK(svd2_status_string(SVD2_ERR_ALIAS) != NULL);
  /* Kogbetliantz: sizes, missing buffers, flags */
  CHECK(kog_workspace_bytes(7, SVD2_KOG_F64) == 0);
  CHECK(kog_workspace_bytes(64, 9) == 0);
  CHECK(kog_workspace_bytes_flags(64, SVD2_KOG_F64, SVD2_KOG_TWO_STEP) >
        kog_workspace_bytes(64, SVD2_KOG_F64));
  CHECK(kog_svd_workspace_bytes(64, SVD2_KOG_C128, 0) > kog_workspace_bytes(64, SVD2_KOG_C128));
  CHECK(kog_sigma_workspace_bytes(64, SVD2_KOG_F32) > 0);
  CHECK(dkog_solve(64, NULL, 64, 1e-14, 40, NULL, NULL, NULL, 0, 0, st) == SVD2_ERR_NULL);
  CHECK(dkog_solve_noalloc(64, NULL, 64, 1e-14, 40, NULL, NULL, 0, st) == SVD2_ERR_NULL);
  CHECK(dkog_solve_noalloc(30274, (double *)(uintptr_t)4096, 30274, 1e-14, 40, NULL, NULL, 0, st) ==
        SVD2_ERR_SIZE);
  CHECK(dkog_solve_noalloc(64, (double *)(uintptr_t)4096, 64, 1e-14, 40, NULL, NULL, SVD2_KOG_GRAPH | 1, st) ==
        SVD2_ERR_FLAGS);
  CHECK(zkog_step(64, NULL, 64, 0, NULL, 0, SVD2_KOG_UNFUSED, st) == SVD2_ERR_NULL);
  CHECK(zkog_step(64, NULL, 64, 0, NULL, 0, SVD2_KOG_TWO_STEP, st) == SVD2_ERR_NULL);
  CHECK(zkog_step(64, NULL, 64, 0, NULL, 0, SVD2_KOG_TWO_STEP | SVD2_KOG_GRAPH, st) == SVD2_ERR_FLAGS);
  CHECK(skog_sweep(64, NULL, 64, NULL, 0, SVD2_KOG_GRAPH, st) == SVD2_ERR_FLAGS);
  CHECK(ckog_svd(64, NULL, 64, NULL, 64, NULL, 64, NULL, 1e-7, 40, NULL, NULL, NULL, 0, 0, st) ==
        SVD2_ERR_NULL);
  CHECK(kog_batch_workspace_bytes(1, NULL) == 0);
  CHECK(kog_batch_solve(1, NULL, NULL, 0, 0, st) == SVD2_ERR_NULL);
  CHECK(kog_batch_solve(1, NULL, NULL, 0, 64, st) == SVD2_ERR_FLAGS);
  CHECK(kog_set_fused_blocks_per_cu(0) == SVD2_ERR_SIZE);
  CHECK(kog_set_tile_rules(0, NULL, NULL, NULL) == SVD2_OK);
  CHECK(kog_set_two_step_tiles(0, NULL, NULL, NULL) == SVD2_OK);
  if (failures == 0) printf("c_abi_check: all checks passed\n");
  return failures;
}
