/*
 * vklb.h -- C ABI of the MI355X (gfx950) weighted-upwind vector kinetic
 * lattice Boltzmann (WU-VKLB) solver.
 *
 * The method (Brown, Chaudhry, Shadid): vector populations f_q(x) in R^p
 * stream along lattice velocities v_q and relax to a weighted-upwind
 * equilibrium built from the conserved moments U = sum_q f_q and a
 * sigmoid-weighted eigen-split of the physical flux.
 *
 * Conventions used by every entry point
 *   - Every call returns vklb_status (VKLB_OK = 0). No exception or abort
 *     crosses the ABI; a failing call leaves a message for vklb_last_error().
 *   - Host arrays of conserved variables are FP64, structure of arrays:
 *     U[var * cells + cell], cell = j * n[0] + i (x fastest).
 *   - Variable order: shallow water (h, h u, [h v]); Euler (rho, rho u,
 *     [rho v], E); MHD-GLM (rho, rho u, rho v, rho w, E, B_x, B_y, B_z, psi)
 *     with three-component u and B in 1D and 2D; linear test system (u).
 *   - Population order: D1Q3 (+xi, 0, -xi); D2Q5 (+x, -x, 0, +y, -y).
 *   - Ownership: the caller owns host arrays, the device buffer passed to
 *     vklb_create (or the library allocates one when none is passed) and the
 *     HIP stream. The library owns the solver handle only.
 *   - Asynchrony: vklb_init, vklb_step and vklb_set_state enqueue work on
 *     the solver's stream and return; vklb_moments, vklb_diagnostics and
 *     vklb_get_state synchronize the stream and report device-side errors
 *     (non-physical states) detected since the last synchronizing call.
 */
#ifndef VKLB_H
#define VKLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VKLB_OK = 0,
  VKLB_ERR_ARG = -1,          /* invalid argument (see vklb_last_error) */
  VKLB_ERR_UNSUPPORTED = -2,  /* combination not built (e.g. lattice/grid mismatch) */
  VKLB_ERR_OOM = -3,          /* device buffer too small or allocation failed */
  VKLB_ERR_DEVICE = -4,       /* a HIP runtime call failed */
  VKLB_ERR_NONPHYSICAL = -5,  /* h, rho or p <= 0, or a non-finite value, was produced */
  VKLB_ERR_STATE = -6         /* call out of order (e.g. vklb_step before vklb_init) */
} vklb_status;

/* Hyperbolic systems (Sec. 5.1 shallow water, 5.2 Euler, 5.3 ideal MHD with
 * hyperbolic divergence cleaning; the linear system F^(d) = adv[d] u is a
 * test system with an exact Fourier solution). */
typedef enum { VKLB_SHALLOW_WATER = 0, VKLB_EULER = 1, VKLB_MHD_GLM = 2, VKLB_LINEAR = 3 } vklb_system_kind;

typedef struct {
  vklb_system_kind kind;
  double g;          /* gravity (shallow water) */
  double gamma;      /* adiabatic index (Euler, MHD) */
  double ch_factor;  /* MHD cleaning speed c_h = ch_factor * max c_f over the grid (6 in Sec. 5.3) */
  double adv[2];     /* advection speeds of the linear test system */
} vklb_system;

/* Lattices of Sec. 2.2 (D1Q3) and Sec. 3.4 (D2Q5); both include the rest velocity. */
typedef enum { VKLB_D1Q3 = 0, VKLB_D2Q5 = 1 } vklb_lattice;

/* Uniform cell-centred grid (Sec. 3.3: nodes dx/2 from the boundary). In 2D
 * the lattice needs dx == dy (Sec. 3.4). */
typedef struct {
  int dim;          /* 1 or 2; must match the lattice */
  int64_t n[2];     /* cells per axis; n[1] ignored in 1D */
  double lo[2], hi[2];
} vklb_grid;

/* Streaming speed xi = dx/dt (the "lambda" of the interface). CFL mode
 * updates it every step as max|lambda(U^n)| / nu (Sec. 3.2, 0 < nu <= 1);
 * FIXED keeps xi constant. With an end time, the step that reaches it uses
 * xi = dx / (T - t) so that t lands on T. */
typedef enum { VKLB_XI_CFL = 0, VKLB_XI_FIXED = 1 } vklb_xi_mode;
typedef struct {
  vklb_xi_mode mode;
  double nu;  /* CFL number (CFL mode) */
  double xi;  /* streaming speed (FIXED mode) */
} vklb_speed;

/* Boundary per axis:
 *  periodic (Sec. 3.3);
 *  zero gradient (the ghost beyond a boundary carries the post-collision
 *    populations of the boundary cell);
 *  characteristic, non-reflecting (Sec. 3.3; 1D only, every system, also
 *    in the serving pool; VKLB_ERR_UNSUPPORTED in 2D): at a boundary cell
 *    the characteristic variables W = P^{-1} U advance with the outgoing
 *    waves only, dW/dx taken as the first-order one-sided difference towards
 *    the interior, U_b^{n+1} = U_b - P (Lambda dW)' / xi, and the cell's
 *    populations become f^eq(U_b^{n+1}) with the step's xi. For MHD the nine
 *    waves include the cleaning pair +-c_h at the step's c_h. Both ends of
 *    the axis use it (bc[0] in 1D). */
typedef enum { VKLB_BC_PERIODIC = 0, VKLB_BC_ZERO_GRADIENT = 1, VKLB_BC_CHARACTERISTIC = 2 } vklb_bc;

/* Equilibrium distribution set.
 *  VKLB_EQ_WEIGHTED: the weighted-upwind set (Sec. 3.1 1D, Sec. 3.4 2D) with
 *    diffusive weight c and sigmoid sharpness k; k = INFINITY gives the step
 *    weights of the discontinuous split (Sec. 2.2; lambda >= 0 goes to +).
 *    The sigmoid normalizer max_j|lambda_j| is the global max over the grid
 *    (alpha_local = 0) or the cell's own max for that direction (1).
 *  VKLB_EQ_CENTERED: the centered flux set (Sec. 2.2): U/3 +- F/(2 xi) and
 *    U/3 in 1D, U/5 +- F^(d)/(2 xi) and U/5 in 2D (= weighted with c = 1/3 or
 *    1/5, k = 0; c and k are ignored). In VKLB_XI_CFL mode nu is read as the
 *    number eta of the subcharacteristic condition (Sec. 2.3):
 *    xi = sqrt(3/2) max|lambda| / eta in 1D, sqrt(5/2) max|lambda| / eta in 2D
 *    (the second moment of the D2Q5 centered set is 2 xi^2/5 per axis).
 *  VKLB_EQ_DISCONTINUOUS: the discontinuous upwind set (Sec. 2.2):
 *    F+/xi, U - (F+ - F-)/xi, -F-/xi (= weighted with c = 0, k = INFINITY;
 *    c and k are ignored); xi by the CFL rule of Sec. 3.2. */
typedef enum { VKLB_EQ_WEIGHTED = 0, VKLB_EQ_CENTERED = 1, VKLB_EQ_DISCONTINUOUS = 2 } vklb_equilibrium_set;

typedef struct {
  double c;
  double k;
  int alpha_local;
  int set;           /* vklb_equilibrium_set */
} vklb_equilibrium;

/* Storage/arithmetic precision of the populations. FP32 keeps FP64 for the
 * MHD eigenstructure of directions near the triple point (fast and slow
 * speeds nearly equal), for the time t, the streaming speed and the
 * diagnostics. */
typedef enum { VKLB_FP64 = 0, VKLB_FP32 = 1 } vklb_precision;

typedef struct {
  int basis;        /* stored basis of a cell:
                       1: all Q populations;
                       2: the moving populations and U in the rest slot (U^{n+1} = U^n plus the
                          streamed differences of the moving populations);
                       3: as 2 with U held as an FP32 pair hi + lo in one more slot and updated by
                          an error-free sum, so U's rounding does not build up over many steps
                          (FP32 only; VKLB_ERR_ARG with FP64);
                       0: default: FP64 -> 1; FP32 -> 3 in 1D, 2 in 2D.
                       Other values: VKLB_ERR_ARG. */
  int band_rows;    /* 2D: rows per workgroup band (MHD in the delta bases: at most 64, larger values
                       are taken as 64); 0 = the default: the tallest power of two from 512 down to
                       4 rows that gives a step at least 2048 wavefronts (two per SIMD) */
  int graph_chunk;  /* steps captured per HIP graph (0 = 512; < 0: plain launches) */
  int strip_width;  /* 2D: columns per workgroup (64, 128 or 256); 1D: lanes per workgroup
                       (256 or 512, each finishing W - 2 cells); 0 = tuned default */
  int halo_rows;    /* 2D: rows of the two halo columns collided per batch (1..32); 0 = tuned default */
  int small_grid;   /* 1D grids of up to 1024 cells (256 for MHD), any boundary condition,
                       run up to 1024 steps per launch in one workgroup, with bitwise the same
                       results as one launch per step: 0 = on, 512 lanes (256 for MHD), the fastest
                       measured; 256, 512 or 1024 = on with that many lanes; -1 = off */
  int fold_partials; /* the per-workgroup maxima a step leaves for the next (max |lambda|, max
                       c_f) are read by every workgroup of the next launch; for a step grid of
                       more than this many workgroups a one-workgroup kernel after each launch
                       folds them into one value instead, which the next launch reads. Results
                       are bitwise the same. 0 = 2048; -1 = never */
} vklb_options;

typedef struct vklb_solver vklb_solver;

typedef struct {
  double t;            /* current time */
  int64_t steps;       /* steps taken since vklb_init / vklb_set_state */
  double xi;           /* streaming speed the next step will use */
  double lambda_max;   /* global max |lambda| of the current state */
  double ch;           /* MHD cleaning speed of the current state (0 otherwise) */
  int done;            /* end time or step limit reached */
  int nonphysical;     /* 1 if a non-physical state was produced */
  int64_t fail_step;   /* step that produced it (-1 if none) */
  int64_t fail_cell;   /* lowest cell index where it was seen (-1 if none) */
  double totals[9];    /* compensated (Neumaier) sum of each conserved field over the cells */
  double max_div_b;    /* MHD 2D: max |dBx/dx + dBy/dy| by central differences; 0 otherwise */
} vklb_diag;

/* Bytes of device memory a solve needs (state, FP64 staging of U, two
 * population buffers, reduction partials), for the largest stored basis of the
 * precision, so it suffices for any vklb_options. 0 if the arguments are invalid. */
size_t vklb_workspace_bytes(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid, vklb_precision prec);

/* Create a solver. device_buf (>= vklb_workspace_bytes, 256-byte aligned) may be
 * NULL, in which case the library allocates it with hipMalloc and frees it in
 * vklb_destroy. hip_stream (a hipStream_t) may be NULL for the null stream.
 * opt may be NULL for defaults. Checks: 0 < omega <= 2 (Sec. 2.3), 0 < nu <= 1
 * (Sec. 3.2), c >= 0, k >= 0, dx == dy in 2D, lattice dimension == grid
 * dimension; c > (1 - nu)/2 (Sec. 4.2) is accepted with a note in
 * vklb_last_error. */
vklb_status vklb_create(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid, const vklb_speed* lambda,
                        double omega, const vklb_bc bc[2], const vklb_equilibrium* eq, vklb_precision prec,
                        const vklb_options* opt, void* device_buf, size_t buf_bytes, void* hip_stream,
                        vklb_solver** out);

/* Set the end condition: steps past time T (T = INFINITY: none) or past
 * max_steps (< 0: none) become no-ops. Before vklb_init it is stored for the
 * init; after it, it applies from the next vklb_step on (the call waits for
 * the solver's stream). VKLB_ERR_ARG for T = NaN. */
vklb_status vklb_set_end(vklb_solver* s, double T, int64_t max_steps);

/* Initialization (Sec. 3.5): xi^0 and c_h^0 from U0, f_q = f_q^eq(U0), t = 0.
 * U0_host: FP64 SoA [p][cells] in host memory (copied before return). */
vklb_status vklb_init(vklb_solver* s, const double* U0_host);

/* As vklb_init, with U0 already in device memory (FP64 SoA [p][cells]); the
 * copy and the initialization are enqueued on the solver's stream. */
vklb_status vklb_init_device(vklb_solver* s, const double* U0_device);

/* Advance n steps on the solver's stream (collision, streaming, moments and
 * the CFL update of Sec. 3.5, one fused kernel per step). No host sync. */
vklb_status vklb_step(vklb_solver* s, int64_t n);

/* Copy U = sum_q f_q to U_host (FP64 SoA [p][cells]); t and steps may be NULL.
 * Synchronizes; returns VKLB_ERR_NONPHYSICAL if such a state was produced. */
vklb_status vklb_moments(vklb_solver* s, double* U_host, double* t, int64_t* steps);

/* Time, step count and whether the end condition has been reached (no more
 * steps will run). Synchronizes; reports non-physical states like vklb_moments. */
vklb_status vklb_progress(vklb_solver* s, double* t, int64_t* steps, int* done);

/* Scalars and compensated totals of the current state. Synchronizes. */
vklb_status vklb_diagnostics(vklb_solver* s, vklb_diag* d);

/* Checkpoint / resume. The blob (vklb_state_bytes bytes) holds the stored
 * populations in the device's block layout (blocks of 256 cells, each holding its
 * [slot][var][256] values; the solver's precision and basis; 2D rows padded to a
 * multiple of 64 cells) with the rows in grid order, whatever the band height,
 * followed by a 128-byte trailer with t, the step count, xi, Lambda, c_h, the
 * end-time landing flag and the solve's shape. vklb_set_state restores all of
 * it, so a resumed run continues bit for bit; it rejects (VKLB_ERR_ARG) a blob
 * written by a solver of another system, lattice, size, precision or basis. */
size_t vklb_state_bytes(const vklb_solver* s);
vklb_status vklb_get_state(vklb_solver* s, void* host, double* t, int64_t* steps);
vklb_status vklb_set_state(vklb_solver* s, const void* host);

/* Time of the last vklb_step call's kernels, from HIP events on the solver's
 * stream (ms; synchronizes). */
vklb_status vklb_last_step_ms(vklb_solver* s, double* ms);

void vklb_destroy(vklb_solver* s);

/* Autotuner of the tile shape. Times `steps` steps (after a short warm-up) of
 * the given solve from U0_host (FP64 SoA [p][cells], host) for each candidate
 * shape and writes the fastest options to *best (other fields copied from
 * base, which may be NULL) and its time per step to *best_step_us (may be
 * NULL).
 *  - 1D candidates: 256- or 512-lane workgroups; grids of up to 1024 cells
 *    (not MHD) that run in one workgroup: 256, 512 or 1024 lanes.
 *  - 2D candidates: strips of 64/128/256 columns, bands of 4..64 rows, halo
 *    batches of 2, 8, 16 or 32 rows.
 * All shapes give identical results, so the choice only affects speed. The
 * end condition is ignored while timing. Allocates one workspace
 * (vklb_workspace_bytes) for the duration of the call and synchronizes.
 * Errors: VKLB_ERR_ARG (steps outside 1..100000, NULL pointers, invalid
 * problem), VKLB_ERR_OOM, or the last candidate's error if none ran (for
 * example a state that turns non-physical within the timed steps). */
vklb_status vklb_tune(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid, const vklb_speed* lambda,
                      double omega, const vklb_bc bc[2], const vklb_equilibrium* eq, vklb_precision prec,
                      const vklb_options* base, const double* U0_host, int steps, void* hip_stream,
                      vklb_options* best, double* best_step_us);

/* ------------------------------------------------------------------------
 * Allocation-free solve, for callers that cannot allocate device memory:
 * code being captured into a HIP graph, serving loops that forbid
 * allocation, harnesses that do not allow hipMalloc.
 *
 * vklb_run_static does what vklb_create (default options, no graph chunks)
 * + vklb_set_end(T, n_steps) + vklb_init_device + vklb_step(n_steps) + the
 * moments of vklb_moments do, with the same kernels and so the same bits,
 * but its workspace is a fixed array of VKLB_STATIC_BYTES inside the library
 * (one per GPU, held from the library's first use on that GPU until the
 * process ends). It calls no hipMalloc, hipFree or other allocating routine
 * and does not synchronize: everything is enqueued on hip_stream, in order.
 *
 *  U0_device   FP64 SoA [p][cells] in device memory: the initial state (read).
 *  U_device    FP64 SoA [p][cells] in device memory: U after the run (written).
 *  info_device device memory for one vklb_run_info (written; may be NULL):
 *              time, steps taken, whether the end was reached, and the step
 *              and cell of a non-physical state (-1 if none).
 *  T, n_steps  end time (INFINITY: none) and number of step launches; steps
 *              past T are no-ops, and the step that reaches T lands on it.
 *
 * Errors (before anything is enqueued): VKLB_ERR_ARG for NULL arrays,
 * n_steps < 0, T = NaN or any argument vklb_create rejects; VKLB_ERR_OOM when
 * the solve's workspace (vklb_workspace_bytes of the same arguments) exceeds
 * VKLB_STATIC_BYTES; VKLB_ERR_DEVICE when a launch fails. The message is
 * left for vklb_last_error(NULL).
 *
 * Every call on one GPU shares that GPU's array and overwrites what the
 * previous call left there (every value a run reads is written by the run
 * first). Calls that overlap on one GPU (on two streams, or from two
 * threads) race on the array and give undefined results: serialize them.
 * ------------------------------------------------------------------------ */
#define VKLB_STATIC_BYTES (64u * 1024u * 1024u)

typedef struct {
  double t;            /* time reached */
  int64_t steps;       /* steps taken */
  int64_t fail_step;   /* step that produced a non-physical state (-1 if none) */
  int64_t fail_cell;   /* lowest cell where it was seen (-1 if none) */
  int done;            /* end time or n_steps reached, or stopped by a non-physical state */
  int nonphysical;     /* 1 if a non-physical state was produced */
} vklb_run_info;

vklb_status vklb_run_static(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid,
                            const vklb_speed* lambda, double omega, const vklb_bc bc[2], const vklb_equilibrium* eq,
                            vklb_precision prec, double T, int64_t n_steps, const double* U0_device,
                            double* U_device, vklb_run_info* info_device, void* hip_stream);

/* ------------------------------------------------------------------------
 * Serving: a pool of concurrent solves in one device arena.
 *
 * Requests are admitted in submission order when their workspace fits in
 * the arena (continuous batching: admission happens at every vklb_pool_run,
 * while other solves are in flight). Each round advances every resident
 * solve by one time step with one batched launch per system class, whose
 * workgroups run tiles of many solves; the per-tile arithmetic is the same as
 * vklb_step's, so a solve gives the same bits alone and in a batch.
 * Finished solves are harvested by vklb_pool_poll, which copies U to the
 * request's output buffer and frees its memory. Not thread safe.
 * ------------------------------------------------------------------------ */
typedef struct vklb_pool vklb_pool;

typedef struct {
  vklb_system sys;
  vklb_lattice lat;
  vklb_grid grid;
  vklb_speed lambda;
  double omega;
  vklb_bc bc[2];
  vklb_equilibrium eq;
  double T;             /* end time (INFINITY: none) */
  int64_t max_steps;    /* step limit (< 0: none); a request needs T or max_steps */
  const double* U0;     /* host FP64 SoA [p][cells]; copied by vklb_pool_submit */
  double* U_out;        /* host FP64 SoA [p][cells]; written when the solve completes */
  uint64_t tag;         /* caller's tag, returned with the completion */
} vklb_request;

typedef struct {
  uint64_t ticket;
  uint64_t tag;
  vklb_status status;   /* VKLB_OK or VKLB_ERR_NONPHYSICAL */
  double t;
  int64_t steps;
  int64_t fail_step, fail_cell;
} vklb_completion;

typedef struct {
  int64_t submitted, admitted, completed, queued, resident;
  int64_t rounds;
  size_t arena_bytes, arena_used, arena_peak;
  int64_t graph_launches;  /* class round chunks replayed from a captured HIP graph */
  int64_t graph_captures;  /* class round chunks captured */
} vklb_pool_stats;

/* One tuned 2D shape of the pool (vklb_pool_autotune). */
typedef struct {
  int kind;           /* vklb_system_kind */
  int64_t n;          /* grid side of the sample it was tuned on */
  int size_class;     /* round(2 log2 n): the grids that use it are those of the nearest class */
  int band_rows, halo_rows;
  double step_us;     /* the sample's time per step in that shape, alone */
} vklb_pool_tile;

/* hbm_budget: bytes of the device arena (allocated here); prec: precision of
 * every solve in the pool; hip_stream may be NULL. */
vklb_status vklb_pool_create(size_t hbm_budget, vklb_precision prec, void* hip_stream, vklb_pool** out);
/* Validate and queue a request (VKLB_ERR_OOM if it can never fit the arena). */
vklb_status vklb_pool_submit(vklb_pool* p, const vklb_request* r, uint64_t* ticket);
/* Admit queued requests that fit, then enqueue `rounds` rounds (asynchronous). */
vklb_status vklb_pool_run(vklb_pool* p, int rounds);
/* Synchronize, harvest finished solves (up to max completions written to out,
 * count in *n; the rest are kept for the next call) and free their memory. */
vklb_status vklb_pool_poll(vklb_pool* p, vklb_completion* out, int max, int* n);
vklb_status vklb_pool_get_stats(const vklb_pool* p, vklb_pool_stats* st);
/* Tile shapes of the batched 2D kernel (128-column strips; band and halo
 * heights) by the autotuner (vklb_tune over those shapes), once per sample
 * request: each 2D sample is timed alone for `steps` steps per candidate and
 * its fastest shape is kept for its (system, half-octave size class of n);
 * later admissions take the entry of their class, or the nearest tuned class
 * of their system. The entries are kept for the process (per device and
 * precision), so pools created later use them too. 1D samples are skipped
 * (the batched 1D kernel has one shape). Call it before any request is
 * submitted to this pool (VKLB_ERR_STATE otherwise),
 * so that no other work disturbs the timing. Synchronizes; allocates one
 * workspace per sample for the duration of its tuning. Up to *n_out entries
 * are written to out (may be NULL); *n_out receives the count. */
vklb_status vklb_pool_autotune(vklb_pool* p, const vklb_request* samples, int n, int steps, vklb_pool_tile* out,
                               int* n_out);
void vklb_pool_destroy(vklb_pool* p);

/* Measurement utility (not a step of the method): copies `bytes` from src to
 * dst, both device memory, with one streaming kernel that reads and writes
 * every byte once, 16 bytes per lane access (non_temporal != 0: the
 * non-temporal loads and stores the step kernels use for their populations).
 * Enqueued on hip_stream; no sync. It gives the copy ceiling that the step
 * kernels' HBM bandwidth is compared with, and a kernel of known traffic for
 * scaling hardware byte counters. VKLB_ERR_ARG for NULL pointers or a size or
 * address that is not a multiple of 16. */
vklb_status vklb_stream_copy(void* dst, const void* src, size_t bytes, int non_temporal, void* hip_stream);

const char* vklb_status_str(vklb_status st);
const char* vklb_last_error(const vklb_solver* s); /* s may be NULL: last create error */

#ifdef __cplusplus
}
#endif

#endif /* VKLB_H */
