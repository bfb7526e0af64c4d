// Kernel launchers per (system, dimension, precision, basis, strip width).
#pragma once

#include <hip/hip_runtime.h>

#include "vklb_kernels.hpp"

namespace vklb {

typedef hipError_t (*launch_fn)(const SolveDesc&, int grid, hipStream_t);
typedef hipError_t (*wg_fn)(const SolveDesc&, int count, int cells_per_lane, int lanes, hipStream_t);
typedef hipError_t (*batched_fn)(const SolveDesc* descs, const WorkItem* work, const int* nwork, int par, int grid,
                                 hipStream_t);

struct Launchers {
  launch_fn init_reduce = nullptr;
  launch_fn init_feq = nullptr;
  launch_fn step = nullptr;
  launch_fn moments = nullptr;
  batched_fn batched = nullptr;  // serving: tiles of many solves in one launch
  wg_fn run_wg = nullptr;        // 1D grids of up to wg_max_cells: many steps in one workgroup
  int wg_max_cells = 0;
  int block = 256;  // threads per step workgroup
};

// prec: 0 FP64, 1 FP32; basis: 0 populations, 1 delta, 2 compensated delta
// (FP32 only); width: 1D workgroup size (256/512), 2D strip width (64/128/256).
Launchers launchers_sw(int dim, int prec, int basis, int width);
Launchers launchers_euler(int dim, int prec, int basis, int width);
Launchers launchers_mhd(int dim, int prec, int basis, int width);
Launchers launchers_linear(int dim, int prec, int basis, int width);

}  // namespace vklb
