/* Plain C use of the library's host-side entry points (include/ftlm.h): no
 * Python, no GPU.  Prints "key value" lines that tests/test_c_abi.py checks
 * against closed forms. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ftlm.h"

int main(void) {
  /* dihedral group of the 6-site ring: rotation and reflection */
  const int32_t gens[12] = {1, 2, 3, 4, 5, 0, 0, 5, 4, 3, 2, 1};
  ftlm_group* g = NULL;
  if (ftlm_group_create(6, gens, 2, &g) != 0) {
    printf("error %s\n", ftlm_last_error());
    return 1;
  }
  int32_t order = 0, nirr = 0, ncls = 0, n = 0;
  ftlm_group_info(g, &order, &nirr, &ncls, &n);
  printf("order %d\nirreps %d\nclasses %d\n", order, nirr, ncls);
  int32_t dims[64], ind[64], wts[64], class_of[64];
  double chars[64 * 64], resid = -1.0;
  if (ftlm_group_irreps(g, dims, ind, wts, chars, class_of, &resid) != 0) {
    printf("error %s\n", ftlm_last_error());
    return 1;
  }
  int sumsq = 0;
  for (int i = 0; i < nirr; ++i) sumsq += dims[i] * dims[i];
  printf("sum_dim_sq %d\nresidual_small %d\n", sumsq, resid < 1e-10);
  ftlm_group_free(g);

  /* a 2x2 Jacobi matrix [[1, 1], [1, 2]]: Ritz values (3 -+ sqrt 5) / 2 */
  const double alpha[2] = {1.0, 2.0}, beta[1] = {1.0};
  double theta[2], weight[2];
  if (ftlm_tridiag_ritz(alpha, beta, 2, theta, weight) != 0) return 1;
  printf("theta0 %.15f\ntheta1 %.15f\nweight_sum %.15f\n", theta[0], theta[1], weight[0] + weight[1]);

  /* one block of dimension 2, one chain with Ritz values 0 and 1 of weight
   * 1/2: Z = 1 + e^{-1/T}, E = e^{-1/T} / Z */
  const int32_t nsteps[1] = {2};
  const double th[2] = {0.0, 1.0}, w[2] = {0.5, 0.5};
  ftlm_ritz blk = {0, 1, 2, 1, 2, nsteps, th, w};
  const double T[1] = {1.0};
  double E, C, chi, logZ;
  if (ftlm_observables(&blk, 1, T, 1, 1.0, &E, &C, &chi, &logZ) != 0) return 1;
  printf("E %.15f\nC %.15f\nlogZ %.15f\n", E, C, logZ);

  /* an invalid generator is refused with a message */
  const int32_t bad[6] = {0, 0, 1, 2, 3, 4};
  ftlm_group* g2 = NULL;
  const int rc = ftlm_group_create(6, bad, 1, &g2);
  printf("bad_rc_nonzero %d\nbad_msg_nonempty %d\n", rc != 0, ftlm_last_error()[0] != 0);
  return 0;
}
