/* Plain C99 user of the C ABI (no GPU needed): status strings, workspace
 * sizing and argument validation, which come before any device call. Prints
 * one line per check; the test compares them. */
#include <stdio.h>
#include <string.h>

#include "vklb.h"

int main(void) {
  vklb_system sys;
  vklb_grid grid;
  vklb_speed speed;
  vklb_equilibrium eq;
  vklb_bc bc[2] = {VKLB_BC_ZERO_GRADIENT, VKLB_BC_ZERO_GRADIENT};
  vklb_solver* s = NULL;
  memset(&sys, 0, sizeof sys);
  memset(&grid, 0, sizeof grid);
  memset(&speed, 0, sizeof speed);
  memset(&eq, 0, sizeof eq);
  sys.kind = VKLB_EULER;
  sys.gamma = 1.4;
  grid.dim = 1;
  grid.n[0] = 65536;
  grid.n[1] = 1;
  grid.lo[0] = 0.0;
  grid.hi[0] = 1.0;
  grid.hi[1] = 1.0;
  speed.mode = VKLB_XI_CFL;
  speed.nu = 0.9;
  eq.c = 0.05;
  eq.k = 2.0;
  eq.set = VKLB_EQ_WEIGHTED;
  printf("status %s\n", vklb_status_str(VKLB_ERR_NONPHYSICAL));
  printf("workspace_fp64 %zu\n", vklb_workspace_bytes(&sys, VKLB_D1Q3, &grid, VKLB_FP64));
  /* omega outside (0, 2]: rejected before the GPU is touched */
  vklb_status r = vklb_create(&sys, VKLB_D1Q3, &grid, &speed, 2.5, bc, &eq, VKLB_FP64, NULL, NULL, 0, NULL, &s);
  printf("create_bad_omega %d %s\n", (int)r, vklb_last_error(NULL));
  printf("solver_null %d\n", s == NULL);
  return 0;
}
