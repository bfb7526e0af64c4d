/* Plain C99 run of the WU-VKLB step through the C ABI alone (no Python, no
 * torch in the process): a Sod shock tube of N cells to t = T in FP64 or
 * FP32, the library allocating its own workspace on the default stream.
 * Usage: abi_run N T fp64|fp32. Prints "t steps" and then U, one value per
 * line, variable after variable ([p][cells], FP64). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vklb.h"

static int check(vklb_status r, const vklb_solver* s, const char* what) {
  if (r != VKLB_OK) {
    fprintf(stderr, "%s: %s (%s)\n", what, vklb_status_str(r), vklb_last_error(s));
    return 1;
  }
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  const long n = atol(argv[1]);
  const double T = atof(argv[2]);
  const vklb_precision prec = strcmp(argv[3], "fp32") == 0 ? VKLB_FP32 : VKLB_FP64;
  if (n < 2 || n > (1L << 24) || !(T > 0.0)) return 2;
  vklb_system sys;
  vklb_grid grid;
  vklb_speed speed;
  vklb_equilibrium eq;
  vklb_bc bc[2] = {VKLB_BC_ZERO_GRADIENT, VKLB_BC_ZERO_GRADIENT};
  memset(&sys, 0, sizeof sys);
  memset(&grid, 0, sizeof grid);
  memset(&speed, 0, sizeof speed);
  memset(&eq, 0, sizeof eq);
  sys.kind = VKLB_EULER;
  sys.gamma = 1.4;
  grid.dim = 1;
  grid.n[0] = n;
  grid.n[1] = 1;
  grid.hi[0] = 1.0;
  grid.hi[1] = 1.0;
  speed.mode = VKLB_XI_CFL;
  speed.nu = 0.9;
  eq.c = 0.05;
  eq.k = 2.0;
  eq.set = VKLB_EQ_WEIGHTED;
  double* U = malloc(sizeof(double) * 3 * (size_t)n);
  if (!U) return 3;
  for (long i = 0; i < n; ++i) {  /* (rho, u, p) = (1, 0, 1) | (0.125, 0, 0.1) at x = 0.5 */
    const double x = (i + 0.5) / (double)n;
    const double rho = x < 0.5 ? 1.0 : 0.125, p = x < 0.5 ? 1.0 : 0.1;
    U[i] = rho;
    U[n + i] = 0.0;
    U[2 * n + i] = p / (sys.gamma - 1.0);
  }
  vklb_solver* s = NULL;
  if (check(vklb_create(&sys, VKLB_D1Q3, &grid, &speed, 1.0, bc, &eq, prec, NULL, NULL, 0, NULL, &s), NULL, "create"))
    return 4;
  int rc = check(vklb_set_end(s, T, -1), s, "set_end") || check(vklb_init(s, U), s, "init");
  double t = 0.0;
  int64_t steps = 0;
  int done = 0;
  while (!rc && !done) {
    rc = check(vklb_step(s, 256), s, "step") || check(vklb_progress(s, &t, &steps, &done), s, "progress");
  }
  if (!rc) rc = check(vklb_moments(s, U, &t, &steps), s, "moments");
  vklb_destroy(s);
  if (rc) {
    free(U);
    return 5;
  }
  printf("%.17g %lld\n", t, (long long)steps);
  for (long i = 0; i < 3 * n; ++i) printf("%.17g\n", U[i]);
  free(U);
  return 0;
}
