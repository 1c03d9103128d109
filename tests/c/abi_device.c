/* Plain C use of the library's device entry points (include/ftlm.h): the
 * 6-site s = 1/2 Heisenberg ring under its dihedral group, every M = 0 irrep
 * block built, H applied on device buffers to the identity (the block's
 * trace), and a Lanczos run of as many steps as the block has rows (exact
 * Ritz values).  Prints "key value"
 * lines that tests/test_c_abi.py checks against exact diagonalization. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "ftlm.h"

#define CHECK(x)                                          \
  do {                                                    \
    if ((x) != 0) {                                       \
      printf("error %s at line %d\n", ftlm_last_error(), __LINE__); \
      return 1;                                           \
    }                                                     \
  } while (0)

int main(void) {
  const int32_t bonds[12] = {0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 0};
  const ftlm_cluster cl = {6, 1, 6, bonds, NULL};
  const int32_t gens[12] = {1, 2, 3, 4, 5, 0, 0, 5, 4, 3, 2, 1};
  double e0 = 1e300, trace = 0.0;
  uint64_t rows = 0;
  for (int irrep = 0; irrep < 6; ++irrep) {
    ftlm_block* b = NULL;
    CHECK(ftlm_build_block(&cl, gens, 2, 0, irrep, 0, NULL, &b));
    ftlm_block_info info;
    CHECK(ftlm_block_info_get(b, &info));
    rows += info.D * (uint64_t)info.d_gamma;
    if (info.D == 0) {
      ftlm_block_free(b);
      continue;
    }
    /* H.V on the device with X = the identity (D vectors): the block's trace */
    const uint64_t D = info.D;
    const size_t bytes = D * D * sizeof(double);
    double *X = NULL, *Y = NULL;
    double* h = (double*)calloc(D * D, sizeof(double));
    for (uint64_t i = 0; i < D; ++i) h[i * D + i] = 1.0;
    if (hipMalloc((void**)&X, bytes) != hipSuccess || hipMalloc((void**)&Y, bytes) != hipSuccess) return 1;
    if (hipMemcpy(X, h, bytes, hipMemcpyHostToDevice) != hipSuccess) return 1;
    CHECK(ftlm_apply_H(b, X, Y, (int32_t)D, (int64_t)D, FTLM_F64, NULL));
    if (hipMemcpy(h, Y, bytes, hipMemcpyDeviceToHost) != hipSuccess) return 1;
    double tr = 0.0;
    for (uint64_t i = 0; i < D; ++i) tr += h[i * D + i];
    trace += info.d_gamma * tr;
    hipFree(X);
    hipFree(Y);
    free(h);
    /* Lanczos with as many steps as rows: its Ritz values are the block's eigenvalues */
    const int steps = (int)info.D;
    double* alpha = (double*)calloc((size_t)steps, sizeof(double));
    double* beta = (double*)calloc((size_t)steps, sizeof(double));
    double* theta = (double*)calloc((size_t)steps, sizeof(double));
    double* weight = (double*)calloc((size_t)steps, sizeof(double));
    int32_t n = 0;
    CHECK(ftlm_run(b, 1, steps, 7, FTLM_F64, FTLM_GAUSSIAN, alpha, beta, &n, NULL));
    CHECK(ftlm_tridiag_ritz(alpha, beta, n, theta, weight));
    double lo = theta[0];
    for (int i = 1; i < n; ++i)
      if (theta[i] < lo) lo = theta[i];
    if (lo < e0) e0 = lo;
    free(alpha);
    free(beta);
    free(theta);
    free(weight);
    ftlm_block_free(b);
  }
  printf("rows %llu\nE0 %.15f\ntrace %.15f\n", (unsigned long long)rows, e0, trace);
  return 0;
}
