// Host-side helpers shared by the single-solve runtime and the serving pool:
// workspace layout, argument checks, kernel descriptors, launcher choice.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include "../../include/vklb.h"
#include "vklb_launch.hpp"

namespace vklb {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

inline int nvars(int kind, int dim) {
  switch (kind) {
    case VKLB_SHALLOW_WATER: return dim + 1;
    case VKLB_EULER: return dim + 2;
    case VKLB_MHD_GLM: return 9;
    case VKLB_LINEAR: return 1;
  }
  return 0;
}

struct Layout {
  size_t state_off, stage_off, fa_off, fb_off, part_off, diag_off, total;
  long long stride;
  int p, Q;
  int slots;  // stored slots of p planes per buffer: Q, or Q + 1 with the low part of U
  size_t elem;
};

// Stored basis (the kernels' BASIS) from vklb_options::basis: 0 all Q
// populations, 1 moving populations + U, 2 as 1 with U compensated (FP32).
// Default: FP64 populations; FP32 compensated in 1D (runs there take tens of
// thousands of steps and the launch, not HBM, bounds the step) and delta in 2D.
// -1: not a valid choice.
inline int resolve_basis(int opt, vklb_precision prec, int dim) {
  switch (opt) {
    case 0: return prec == VKLB_FP32 ? (dim == 1 ? 2 : 1) : 0;
    case 1: return 0;
    case 2: return 1;
    case 3: return prec == VKLB_FP32 ? 2 : -1;
  }
  return -1;
}

constexpr int kDiagBlocks = 512;
// Step grids of more workgroups than this fold each launch's partials into
// one entry (vklb_options.fold_partials = 0).
constexpr int kFoldAbove = 2048;

// Upper bound of the step grid over every strip width / band height choice.
inline long long max_step_blocks(const vklb_grid* g) {
  if (g->dim == 1) return (g->n[0] + 253) / 254;
  return ((g->n[0] + 63) / 64) * g->n[1];
}

// Cells from one row to the next in the population buffers: nx in 1D; in 2D
// nx rounded up to a multiple of 64, so that the 64 cells of a row a
// wavefront loads or stores start at a multiple of 64 whatever nx is, and
// each of its plane accesses is one aligned run of the blocked layout. The
// padding cells are never read or written by a step.
inline long long row_stride(const vklb_grid* g) {
  return g->dim == 2 ? (g->n[0] + 63) / 64 * 64 : g->n[0];
}

// basis: as resolve_basis returns it (sizes the population buffers).
inline bool layout_of(const vklb_system* sys, vklb_lattice lat, const vklb_grid* g, vklb_precision prec, int basis,
                      Layout* L) {
  if (!sys || !g) return false;
  if (g->dim != 1 && g->dim != 2) return false;
  if ((lat == VKLB_D1Q3) != (g->dim == 1)) return false;
  const int p = nvars(sys->kind, g->dim);
  if (p == 0) return false;
  const long long nx = g->n[0], ny = g->dim == 2 ? g->n[1] : 1;
  if (nx < 1 || ny < 1 || nx > (1ll << 30) || ny > (1ll << 30)) return false;
  const long long cells = nx * ny;
  if (cells > (1ll << 31) - 1) return false;
  // population buffers: padded rows in 2D (64-bit indices on the device; the
  // 2^31 limit is on natural cell indices, which non-physical reports carry)
  const long long pcells = row_stride(g) * ny;
  L->p = p;
  L->Q = g->dim == 1 ? 3 : 5;
  L->slots = L->Q + (basis == 2 ? 1 : 0);
  L->elem = prec == VKLB_FP32 ? 4 : 8;
  L->stride = (pcells + kBlock - 1) / kBlock * kBlock;  // whole storage blocks
  const size_t plane = size_t(L->stride) * L->elem;
  L->state_off = 0;
  L->stage_off = align_up(sizeof(DevState));
  L->fa_off = align_up(L->stage_off + size_t(p) * cells * 8);
  L->fb_off = align_up(L->fa_off + size_t(L->slots) * p * plane);
  L->part_off = align_up(L->fb_off + size_t(L->slots) * p * plane);
  L->diag_off = align_up(L->part_off + size_t(2) * 2 * max_step_blocks(g) * 8);
  L->total = align_up(L->diag_off + size_t(kDiagBlocks) * 9 * 2 * 8 + 256);
  return true;
}


// 2D: strip width; 1D: workgroup size (256 lanes measured faster than 512 at
// every 1D benchmark size: more, smaller workgroups start sooner).
inline int default_width(int dim, long long nx) {
  if (dim == 1) return 256;
  return nx <= 64 ? 64 : (nx <= 128 ? 128 : 256);
}
// Rows per 2D band for strips of `width` columns (width / 64 wavefronts per
// workgroup): the tallest power of two from 512 down to 4 that still gives the
// step at least 2048 wavefronts (two per SIMD, the most the MHD march's
// registers allow). A mid-size grid then does not leave SIMDs idle, and a
// large one runs its workgroups in one wave with few halo and edge-row reads
// per cell. Measured on MI355X (FP32, 256-column strips, us per step): 2D
// Euler 1024^2 33.2 with 8 rows against 56.4 with 32, 512^2 12.5 (4 rows)
// against 55.2; shallow water 1024^2 26.0 (8) against 45.9; MHD 512^2 37.6
// (4) against 59.2 (8), 2048^2 309 (32) against 321 (8); Euler 2048^2 and MHD
// 1024^2 keep 32 and 8. With the rows of whole bands interleaved: Euler
// 4096^2 472 (128 rows) against 529 (32), 8192^2 2017 (512) against 2082
// (32); shallow water 4096^2 354 (128) against 389 (32). MHD 1024^2 in
// 128-column strips: 16-row bands (one wave per SIMD) 126.9 us, 8-row 88.
inline int default_band(const vklb_grid* g, int width) {
  const long long strips = (g->n[0] + width - 1) / width, ny = g->dim == 2 ? g->n[1] : 1;
  const long long waves_per_group = (width + 63) / 64;
  int band = 512;
  while (band > 4 && strips * ((ny + band - 1) / band) * waves_per_group < 2048) band /= 2;
  return band;
}
// Largest band: the MHD march of the delta bases collides a band's halo cells
// into LDS for up to 64 rows; the others take any height.
inline int max_band(int kind, int dim, int basis) { return kind == VKLB_MHD_GLM && dim == 2 && basis >= 1 ? 64 : 4096; }
// Rows of halo columns per batch (1..32): measured fastest on MI355X with the
// default bands, one batch per band (MHD 8 rows; the others 32, 3% over 2).
inline int default_halo(int kind) { return kind == VKLB_MHD_GLM ? 8 : 32; }

inline int step_grid_of(const vklb_grid* g, int width, int band) {
  if (g->dim == 1) return int((g->n[0] + width - 3) / (width - 2));
  return int(((g->n[0] + width - 1) / width) * ((g->n[1] + band - 1) / band));
}

// Argument checks of vklb_create (Sec. 2.3 omega range, Sec. 3.2 CFL number,
// Sec. 3.4 dx == dy). Returns VKLB_OK or an error with a message.
inline vklb_status validate(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid, const vklb_speed* lambda,
                            double omega, const vklb_bc bc[2], const vklb_equilibrium* eq, vklb_precision prec,
                            const char** msg) {
  auto bad = [&](vklb_status st, const char* m) { *msg = m; return st; };
  if (!sys || !grid || !lambda || !bc || !eq) return bad(VKLB_ERR_ARG, "NULL argument");
  if (sys->kind < VKLB_SHALLOW_WATER || sys->kind > VKLB_LINEAR) return bad(VKLB_ERR_ARG, "unknown system");
  if (lat != VKLB_D1Q3 && lat != VKLB_D2Q5) return bad(VKLB_ERR_ARG, "unknown lattice");
  if (grid->dim != 1 && grid->dim != 2) return bad(VKLB_ERR_ARG, "grid dim must be 1 or 2");
  if ((lat == VKLB_D1Q3) != (grid->dim == 1)) return bad(VKLB_ERR_ARG, "lattice dimension does not match the grid");
  if (prec != VKLB_FP64 && prec != VKLB_FP32) return bad(VKLB_ERR_ARG, "unknown precision");
  if (!(omega > 0.0 && omega <= 2.0)) return bad(VKLB_ERR_ARG, "omega must be in (0, 2]");
  if (lambda->mode == VKLB_XI_CFL) {
    if (!(lambda->nu > 0.0 && lambda->nu <= 1.0)) return bad(VKLB_ERR_ARG, "nu must be in (0, 1]");
  } else if (lambda->mode == VKLB_XI_FIXED) {
    if (!(lambda->xi > 0.0) || !isfinite(lambda->xi)) return bad(VKLB_ERR_ARG, "xi must be > 0");
  } else {
    return bad(VKLB_ERR_ARG, "unknown speed mode");
  }
  if (eq->set < VKLB_EQ_WEIGHTED || eq->set > VKLB_EQ_DISCONTINUOUS) return bad(VKLB_ERR_ARG, "unknown equilibrium set");
  if (eq->set == VKLB_EQ_WEIGHTED) {
    if (!(eq->c >= 0.0) || !isfinite(eq->c)) return bad(VKLB_ERR_ARG, "c must be >= 0");
    if (!(eq->k >= 0.0)) return bad(VKLB_ERR_ARG, "k must be >= 0");
  }
  if (grid->n[0] < 1 || (grid->dim == 2 && grid->n[1] < 1)) return bad(VKLB_ERR_ARG, "empty grid");
  const double dx = (grid->hi[0] - grid->lo[0]) / double(grid->n[0]);
  if (!(dx > 0.0)) return bad(VKLB_ERR_ARG, "hi must exceed lo");
  if (grid->dim == 2) {
    const double dy = (grid->hi[1] - grid->lo[1]) / double(grid->n[1]);
    if (!(fabs(dx - dy) <= 1e-12 * dx)) return bad(VKLB_ERR_ARG, "the D2Q5 lattice needs dx == dy");
  }
  for (int a = 0; a < grid->dim; ++a) {
    if (bc[a] != VKLB_BC_PERIODIC && bc[a] != VKLB_BC_ZERO_GRADIENT && bc[a] != VKLB_BC_CHARACTERISTIC)
      return bad(VKLB_ERR_ARG, "unknown bc");
    if (bc[a] == VKLB_BC_CHARACTERISTIC && grid->dim != 1)
      return bad(VKLB_ERR_UNSUPPORTED, "characteristic boundaries: 1D only");
    if (bc[a] == VKLB_BC_CHARACTERISTIC && grid->n[0] < 2) return bad(VKLB_ERR_ARG, "characteristic boundaries need 2 cells");
  }
  if (sys->kind == VKLB_SHALLOW_WATER && !(sys->g > 0.0)) return bad(VKLB_ERR_ARG, "g must be > 0");
  if ((sys->kind == VKLB_EULER || sys->kind == VKLB_MHD_GLM) && !(sys->gamma > 1.0))
    return bad(VKLB_ERR_ARG, "gamma must be > 1");
  if (sys->kind == VKLB_MHD_GLM && !(sys->ch_factor > 0.0)) return bad(VKLB_ERR_ARG, "ch_factor must be > 0");
  Layout L;
  if (!layout_of(sys, lat, grid, prec, 0, &L)) return bad(VKLB_ERR_UNSUPPORTED, "grid too large or invalid");
  return VKLB_OK;
}

// After a step launch (or the initial reduction) that left the partials of
// parity `par`: fold them into entry 0 when the solve's launches read that
// entry alone (nred = 1).
inline hipError_t launch_fold(const SolveDesc& d, int par, hipStream_t s) {
  if (d.nred == d.nblocks) return hipSuccess;
  hipLaunchKernelGGL(k_fold_partials<1024>, dim3(1), dim3(1024), 0, s, d, par);
  return hipGetLastError();
}

// Checkpoint blobs hold the populations with their rows in grid order, so a
// blob does not depend on the band height of the solver that wrote it. Copy a
// population buffer between that order and the device's (mem_row; to_grid:
// device to grid order), in runs of 64 cells, which never cross a 256-cell
// block since rows are padded to a multiple of 64 cells.
inline void reorder_rows(const char* from, char* to, const SolveDesc& d, const Layout& L, bool down_odd, bool to_grid) {
  const size_t planes = size_t(L.slots) * L.p, run = size_t(64) * L.elem;
  auto off = [&](long long cell, size_t plane) {
    return ((size_t(cell) >> kBlockLog2) * planes + plane) * kBlock * L.elem + size_t(cell & (kBlock - 1)) * L.elem;
  };
  for (int r = 0; r < d.ny; ++r) {
    const long long m = mem_row(r, d.band, d.nfull, down_odd);
    for (long long x = 0; x < d.sx; x += 64) {
      const long long gc = (long long)r * d.sx + x, mc = m * d.sx + x;
      for (size_t pl = 0; pl < planes; ++pl)
        memcpy(to + off(to_grid ? gc : mc, pl), from + off(to_grid ? mc : gc, pl), run);
    }
  }
}

// Kernel descriptor of a solve whose workspace starts at `base`.
inline SolveDesc make_desc(char* base, const Layout& L, const vklb_system* sys, const vklb_grid* grid,
                           const vklb_speed* lambda, double omega, const vklb_bc bc[2], const vklb_equilibrium* eq,
                           int width, int band, int halo) {
  SolveDesc d;
  memset(&d, 0, sizeof d);
  d.fa = base + L.fa_off;
  d.fb = base + L.fb_off;
  d.st = reinterpret_cast<DevState*>(base + L.state_off);
  d.stage = reinterpret_cast<const double*>(base + L.stage_off);
  d.part = reinterpret_cast<double*>(base + L.part_off);
  d.ph.g = sys->g;
  d.ph.gamma = sys->gamma;
  d.ph.ch_factor = sys->kind == VKLB_MHD_GLM ? sys->ch_factor : 0.0;
  d.ph.adv[0] = sys->adv[0];
  d.ph.adv[1] = sys->adv[1];
  d.ph.omega = omega;
  // the centered and discontinuous sets are weighted sets with fixed (c, k)
  double c = eq->c, k = eq->k;
  if (eq->set == VKLB_EQ_CENTERED) {
    c = grid->dim == 1 ? 1.0 / 3.0 : 1.0 / 5.0;
    k = 0.0;
  } else if (eq->set == VKLB_EQ_DISCONTINUOUS) {
    c = 0.0;
    k = INFINITY;
  }
  d.ph.c = c;
  d.ph.kinf = isinf(k) ? 1 : 0;
  d.ph.k = d.ph.kinf ? 0.0 : k;
  d.ph.alpha_local = eq->alpha_local ? 1 : 0;
  d.dx = (grid->hi[0] - grid->lo[0]) / double(grid->n[0]);
  // centered set: xi = sqrt(3/2 | 5/2) max|lambda| / eta (subcharacteristic rule)
  d.nu = eq->set == VKLB_EQ_CENTERED ? lambda->nu / sqrt(grid->dim == 1 ? 1.5 : 2.5) : lambda->nu;
  d.xi_fixed = lambda->xi;
  d.xi_mode = lambda->mode == VKLB_XI_CFL ? 0 : 1;
  d.nx = int(grid->n[0]);
  d.ny = grid->dim == 2 ? int(grid->n[1]) : 1;
  d.sx = int(row_stride(grid));
  d.stride = L.stride;
  d.bcx = bc[0] == VKLB_BC_PERIODIC ? 0 : (bc[0] == VKLB_BC_CHARACTERISTIC ? 2 : 1);
  d.bcy = (grid->dim == 2 ? bc[1] : bc[0]) == VKLB_BC_PERIODIC ? 0 : 1;
  d.band = band;
  d.nfull = grid->dim == 2 && band > 0 ? int(d.ny / band) : 0;
  d.halo = halo;
  d.nblocks = step_grid_of(grid, width, band);
  d.nred = d.nblocks;
  return d;
}

inline Launchers pick_launchers(int kind, int dim, int prec, int basis, int width) {
  switch (kind) {
    case VKLB_SHALLOW_WATER: return launchers_sw(dim, prec, basis, width);
    case VKLB_EULER: return launchers_euler(dim, prec, basis, width);
    case VKLB_MHD_GLM: return launchers_mhd(dim, prec, basis, width);
    default: return launchers_linear(dim, prec, basis, width);
  }
}

// Fastest band and halo heights of the serving pool's batched 2D kernel for
// the solve of request r (vklb_tune over 128-column strips); defined with
// vklb_tune.
vklb_status tune_pool_shape(const vklb_request* r, vklb_precision prec, int steps, void* hip_stream, int* band,
                            int* halo, double* step_us);

inline int grid_for_cells(long long cells) {
  long long g = (cells + 255) / 256;
  return int(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace vklb
