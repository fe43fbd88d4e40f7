/* Calls of the C boundary that need no GPU, compiled as C99 against the
 * public header only: sizes, argument errors, status strings. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "lbm.h"

static int fails = 0;
#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                       \
    }                                                                \
  } while (0)

int main(void) {
  size_t pop = 0, aux = 0;
  /* D3Q19 256^3 in FP32: 19 populations of 4 bytes per cell, whole chunks */
  CHECK(lbm_required_bytes(LBM_D3Q19, 256, 256, 256, LBM_STORE_F32, &pop, &aux) == LBM_OK);
  CHECK(pop >= (size_t)19 * 4 * 256 * 256 * 256);
  CHECK(aux >= (size_t)8 * 256 * 256 * 256); /* link and moving-link words */
  /* D2Q9 needs nz == 1 */
  CHECK(lbm_required_bytes(LBM_D2Q9, 64, 64, 2, LBM_STORE_F64, &pop, &aux) == LBM_ERR_ARG);
  CHECK(strlen(lbm_last_error(NULL)) > 0);
  /* tau <= 1/2 is rejected before any device call */
  lbm_lattice* h = NULL;
  CHECK(lbm_lattice_create(&h, LBM_D3Q19, 8, 8, 8, 0.5, LBM_STORE_F32, 0, NULL, 0, NULL, 0, NULL) ==
        LBM_ERR_ARG);
  CHECK(h == NULL);
  CHECK(lbm_step(NULL, 1) == LBM_ERR_ARG);
  /* the geometry rule: a fluid box streams out of itself unless every axis wraps */
  {
    uint8_t mat[27];
    memset(mat, 1, sizeof mat);
    CHECK(lbm_validate_geometry(LBM_D3Q19, 3, 3, 3, mat, 7u) == LBM_OK);
    CHECK(lbm_validate_geometry(LBM_D3Q19, 3, 3, 3, mat, 3u) == LBM_ERR_GEOMETRY);
    mat[13] = 4; /* no such material */
    CHECK(lbm_validate_geometry(LBM_D3Q19, 3, 3, 3, mat, 7u) == LBM_ERR_UNSUPPORTED);
  }
  CHECK(strcmp(lbm_status_string(LBM_OK), lbm_status_string(LBM_ERR_HIP)) != 0);
  if (fails == 0) printf("c abi ok\n");
  return fails == 0 ? 0 : 1;
}
