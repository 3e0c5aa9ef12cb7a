/* A plain C client of the C ABI (include/lb.h): device memory from the HIP
 * runtime, no Python. Creates a 3D plan, evaluates the energy and gradient of
 * a single-mode field, applies the Hessian, runs a short IMEX-TR solve and
 * prints the results as JSON for the calling test. */
#define _USE_MATH_DEFINES
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "lb.h"

/* the HIP runtime calls used here (declared to keep the client free of HIP headers) */
typedef int hipError_t;
extern hipError_t hipMalloc(void **ptr, size_t size);
extern hipError_t hipFree(void *ptr);
extern hipError_t hipMemcpy(void *dst, const void *src, size_t size, int kind);
#define H2D 1
#define D2H 2

#define CHECK(x)                                                         \
  do {                                                                   \
    int rc_ = (x);                                                       \
    if (rc_ < 0) {                                                       \
      fprintf(stderr, "%s failed: %d %s\n", #x, rc_, lb_last_error());   \
      return 1;                                                          \
    }                                                                    \
  } while (0)

int main(void) {
  const int n = 32;
  const double L = 4.0 * sqrt(2.0) * M_PI; /* |Bk| = 1 at index (2, 2, 0) */
  const size_t N = (size_t)n * n * n;
  lb_grid g = {3, {n, n, n}, {L, L, L}};
  lb_params prm = {-0.2, 0.3, 1.0, 1.0};
  lb_plan *plan = NULL;
  CHECK(lb_plan_create(&plan, &g, 1, LB_FP64, NULL));
  double *h = (double *)malloc(N * sizeof(double));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k)
        h[((size_t)i * n + j) * n + k] = 0.3 * cos(2.0 * M_PI * (2.0 * i + 2.0 * j) / n) + 0.01 * sin(2.0 * M_PI * k / n);
  double *psi, *grad, *hv, *E;
  if (hipMalloc((void **)&psi, N * 8) || hipMalloc((void **)&grad, N * 8) || hipMalloc((void **)&hv, N * 8) ||
      hipMalloc((void **)&E, 8)) {
    fprintf(stderr, "hipMalloc failed\n");
    return 1;
  }
  if (hipMemcpy(psi, h, N * 8, H2D)) return 1;
  CHECK(lb_energy_grad(plan, &prm, psi, E, grad));
  CHECK(lb_hessvec(plan, &prm, psi, grad, hv, 1));
  double e0, g0[2], hv0[2];
  if (hipMemcpy(&e0, E, 8, D2H) || hipMemcpy(g0, grad, 16, D2H) || hipMemcpy(hv0, hv, 16, D2H)) return 1;
  lb_tr_opts o;
  lb_tr_opts_default(&o);
  o.grad_norm_inf = 0;
  o.eps = 1e-8;
  o.sub.max_inner = 5000;
  lb_tr_info info;
  const int rc = lb_imex_tr_solve(plan, &prm, psi, &o, &info);
  CHECK(rc);
  printf("{\"energy0\": %.17g, \"grad0\": [%.17g, %.17g], \"hv0\": [%.17g, %.17g], \"status\": %d, "
         "\"energy\": %.17g, \"gnorm\": %.17g, \"outer\": %d, \"inner\": %d, \"sub_capped\": %d}\n",
         e0, g0[0], g0[1], hv0[0], hv0[1], rc, info.energy, info.gnorm, info.outer, info.inner_total, info.sub_capped);
  hipFree(psi);
  hipFree(grad);
  hipFree(hv);
  hipFree(E);
  free(h);
  CHECK(lb_plan_destroy(plan));
  return 0;
}
