// Device kernels of the WU-VKLB step for gfx950 (one fused kernel per step).
//
// Data layout in HBM: cell = j * sx + i, with the row stride sx = nx in 1D and
// nx rounded up to a multiple of 64 in 2D (the padding cells are never read),
// so that every wavefront's 64 cells of a row start at a multiple of 64 and
// each of its plane loads is one aligned run; cells are grouped in blocks of
// 256 consecutive cells and each block stores its stored values plane after plane
// (plane = slot * P + var, 256 values each): structure of arrays inside a
// block, so every load and store of a wavefront is one contiguous 256-byte
// (FP32) run and a workgroup row touches one region, not Q * P far-apart
// streams. In 2D the rows of the whole bands are stored interleaved in march
// order (mem_row below), so that the bands of a launch, which march in step,
// work in one compact stretch of the buffers at a time rather than in as many
// stretches as there are bands. Two population buffers ping-pong by step
// parity. In the "delta" basis the rest-population plane holds U instead (the
// rest population is U minus the moving ones), which keeps FP32 rounding
// relative to the small per-step change of U rather than to U itself.
//
// Per-step global quantities (Sec. 3.2 CFL speed, Sec. 5.3 cleaning speed)
// need the max over every cell of the NEW state. Each workgroup therefore
// recomputes the collision of a one-cell halo, finishes U^{n+1} of its own
// cells inside the same kernel and stores its block maxima of |lambda| (and
// c_f) with plain stores into a partials array. The kernel boundary is the
// global synchronization: every workgroup of the next launch reduces all the
// partials itself and derives the same xi, Lambda, c_h and end condition.
// That costs every workgroup one load per workgroup of the grid; above a few
// thousand workgroups the runtime instead folds each launch's partials into
// one entry with a one-workgroup kernel, and the next launch reads that.
// Scalars (t, n) and partials are double buffered by launch parity, so the
// step needs no fence, no atomic and no "last workgroup" election.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vklb_cell.hpp"

namespace vklb {

// Scalars of one solve between launches. S[p] is read by launches of parity p
// and written (by workgroup 0) for the next launch, of parity 1 - p.
struct Scal {
  double t;      // time t^n
  long long n;   // step index
  int done;      // 1: end reached or a non-physical state was seen
  int pad;
};

struct DevState {
  Scal S[2];
  double T;                       // end time (inf: none)
  long long max_steps;
  unsigned long long err_word;    // min over detections of (step << 32 | cell); ~0 if none
  double pad[3];
};

// Everything a kernel needs to know about one solve (passed by value).
// Cells per storage block of the population buffers.
constexpr int kBlockLog2 = 8;
constexpr int kBlock = 1 << kBlockLog2;

struct SolveDesc {
  void* fa;
  void* fb;
  DevState* st;
  const double* stage;   // FP64 SoA [p][cells] (init source / moments target)
  double* part;          // block maxima: [parity][lam | cf][nblocks]
  Phys ph;
  double dx;
  double nu;
  double xi_fixed;
  int xi_mode;           // 0 CFL, 1 fixed
  int nx, ny;            // ny = 1 in 1D
  int sx;                // population buffers: cells from one row to the next (row_stride)
  long long stride;      // population buffers: cells (sx * ny) rounded up to whole 256-cell blocks
  int bcx, bcy;          // 0 periodic, 1 zero gradient
  int nblocks;           // workgroups per step launch (= number of partials)
  int band;              // 2D rows per band
  int nfull;             // 2D: whole bands (ny / band), whose rows are stored interleaved (mem_row)
  int par;               // launch parity
  int halo;              // 2D rows of halo columns collided per batch (1..32)
  int npar;              // parity of the step index at launches of parity 0
  int nred;              // partials a step launch reduces at entry: nblocks, or 1 when
                         // each launch's partials are folded into entry 0 after it
};

// Row of the population buffers that holds grid row r (2D). March step i of
// whole band b sits at row i * nfull + b: the bands of one launch advance
// together, so at any time they read and write neighbouring rows of the
// buffers. Bands that march down (odd MHD bands) count their steps from the
// top. The rows of a last, partial band keep their place. With nfull = 0 the
// rows are in grid order. The map is a permutation of the ny rows.
__host__ __device__ inline long long mem_row(int r, int band, int nfull, bool down_odd) {
  if (r >= nfull * band) return r;
  const int b = r / band, i = r - b * band;
  return (long long)((down_odd && (b & 1)) ? band - 1 - i : i) * nfull + b;
}

// Global-memory views of a solve's device pointers. The single-solve kernels
// take the descriptor as a kernel argument, whose pointers the compiler
// already treats as global memory; the batched kernel reads descriptors from
// a table in memory, and through plain pointers its loads and stores would be
// flat instructions, which also count against the LDS wait counter, so every
// LDS read of the row march would wait for the row loads in flight. All
// accesses of the per-step path go through these views.
template <class T>
using gmem = __attribute__((address_space(1))) T;
template <class T>
__device__ inline gmem<T>* gl(T* p) {
  return (gmem<T>*)p;
}
// Scalars of parity p: load and store field by field (address-space-qualified
// structs have no implicit copy).
__device__ inline Scal load_scal(const gmem<DevState>* st, int p) {
  Scal r;
  r.t = st->S[p].t;
  r.n = st->S[p].n;
  r.done = st->S[p].done;
  r.pad = 0;
  return r;
}
__device__ inline void store_scal(gmem<DevState>* st, int p, const Scal& v) {
  st->S[p].t = v.t;
  st->S[p].n = v.n;
  st->S[p].done = v.done;
  st->S[p].pad = v.pad;
}
__device__ inline void report_cell(const SolveDesc& sd, unsigned long long word) {
  __hip_atomic_fetch_min(&gl(sd.st)->err_word, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Values every workgroup derives at the start of a step.
struct Step {
  double t, xi, lam, ch, T;
  long long n;
  int landing, done;
};

// Sec. 3.5 flow chart, between two launches: cleaning speed c_h = factor * max
// c_f (Sec. 5.3), Lambda = max |lambda|, xi = Lambda / nu (Sec. 3.2) or the fixed
// speed, and the end condition; the step that reaches T uses xi = dx / (T - t).
// Shared by device and host so both derive identical values.
__host__ __device__ inline Step derive_step(const Scal& S, double T, long long max_steps, bool err, double lam7,
                                            double cfm, double ch_factor, int xi_mode, double nu, double xi_fixed,
                                            double dx) {
  Step r;
  r.t = S.t;
  r.n = S.n;
  r.T = T;
  r.ch = ch_factor > 0.0 ? ch_factor * cfm : 0.0;
  r.lam = fmax(lam7, r.ch);
  r.xi = xi_mode == 0 ? r.lam / nu : xi_fixed;
  r.landing = 0;
  r.done = S.done || S.n >= max_steps || !(S.t < T) || err || !(r.xi > 0.0) || !isfinite(r.xi);
  if (!r.done && isfinite(T)) {
    const double dt = dx / r.xi;
    const double tol = 1e-9 * dt;
    const double thr = T - tol;
    if (S.t + dt >= thr) {
      r.xi = dx / (T - S.t);
      r.landing = 1;
    }
  }
  return r;
}

__device__ inline int map_index(int x, int n, int bc) {
  if (x >= 0 && x < n) return x;
  if (bc == 0) {
    int r = x % n;
    return r < 0 ? r + n : r;
  }
  return x < 0 ? 0 : n - 1;
}

// Block id remap so that consecutive logical tiles share an XCD (blocks are
// dispatched to the 8 XCDs round robin); neighbouring tiles then meet in the
// same L2 when they re-read each other's halo.
__device__ inline int xcd_remap(int b, int nb) {
  const int per = nb / 8, rem = nb % 8;
  const int xcd = b % 8, idx = b / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}


// Max over the 64 lanes of a wavefront, in every lane, with DPP row
// operations (quad permutes, row mirrors, the row broadcasts of lanes 15 and
// 31) and no LDS round trip; the result is read from lane 63. Every lane of
// the wavefront must be active.
__device__ inline unsigned wave_umax(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Max of non-negative doubles (negatives and NaN count as 0): the IEEE bit
// patterns of non-negative doubles order like unsigned integers, so the max
// is the max high word, then the max low word among the lanes holding it.
__device__ inline double wave_max(double v) {
  v = v >= 0.0 ? v : 0.0;
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned hi = unsigned(b >> 32), lo = unsigned(b);
  const unsigned hm = wave_umax(hi);
  const unsigned lm = wave_umax(hi == hm ? lo : 0u);
  return __longlong_as_double((long long)(((unsigned long long)hm << 32) | lm));
}

// Block max of (a, b) into lane 0 of wave 0 for a workgroup of `lanes`
// lanes; `red` needs 2 * (lanes/64) doubles. TWO = false (systems without a
// cleaning speed, whose fast-speed maxima are identically 0) reduces a alone
// and leaves b as it is.
template <bool TWO = true>
__device__ inline void block_max2(double& a, double& b, double* red, int lanes) {
  a = wave_max(a);
  if (TWO) b = wave_max(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = lanes >> 6;
  if (lane == 0) {
    red[wid] = a;
    if (TWO) red[nw + wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < nw; ++w) {
      a = fmax(a, red[w]);
      if (TWO) b = fmax(b, red[nw + w]);
    }
  }
}

// Block max of (a, b) broadcast to every lane; `red` needs 2 * (lanes/64)
// doubles and is not written again by this workgroup (no trailing barrier).
template <bool TWO = true>
__device__ inline void block_max2_all(double& a, double& b, double* red, int lanes) {
  a = wave_max(a);
  if (TWO) b = wave_max(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = lanes >> 6;
  if (lane == 0) {
    red[wid] = a;
    if (TWO) red[nw + wid] = b;
  }
  __syncthreads();
  for (int w = 0; w < nw; ++w) {
    a = fmax(a, red[w]);
    if (TWO) b = fmax(b, red[nw + w]);
  }
}

// Solve state a step reads, loaded once at the start of a launch so that no
// later stage of the step waits on a scalar load.
struct StateIn {
  Scal S;
  double T;
  long long max_steps;
  bool err;
};

__device__ inline StateIn read_state(const SolveDesc& sd) {
  const gmem<DevState>* st = gl(sd.st);
  StateIn r;
  r.S = load_scal(st, sd.par);
  r.T = st->T;
  r.max_steps = st->max_steps;
  r.err = st->err_word != ~0ull;
  return r;
}

// This lane's first two partials of the previous launch (lanes: the
// workgroup size), loaded without a loop so that the loads issue together
// with the cell loads. Lanes past the end re-read the last partial, which
// leaves the max unchanged.
template <bool TWO = true>
__device__ inline void load_partials(const SolveDesc& sd, int lanes, double& a, double& b) {
  const gmem<double>* pl = gl(sd.part) + (long long)sd.par * 2 * sd.nblocks;
  const int last = sd.nred - 1;
  const int i0 = min((int)threadIdx.x, last), i1 = min((int)threadIdx.x + lanes, last);
  a = fmax(pl[i0], pl[i1]);
  b = TWO ? fmax(pl[sd.nblocks + i0], pl[sd.nblocks + i1]) : 0.0;
}

// Reduce the partials of the previous launch (a, b: this lane's first two,
// from load_partials; the first nred of them) and derive the step scalars
// from the state read at entry. `red` is this reduction's own LDS scratch (2 * blockDim/64 doubles).
// With TWO = false the fast-speed partials (all 0) are not read.
template <bool TWO = true>
__device__ inline Step begin_step(const SolveDesc& sd, double* red, int lanes, const StateIn& in, double a,
                                  double b) {
  const gmem<double>* pl = gl(sd.part) + (long long)sd.par * 2 * sd.nblocks;
  const gmem<double>* pc = pl + sd.nblocks;
  for (int i = threadIdx.x + 2 * lanes; i < sd.nred; i += lanes) {
    a = fmax(a, pl[i]);
    if (TWO) b = fmax(b, pc[i]);
  }
  block_max2_all<TWO>(a, b, red, lanes);
  return derive_step(in.S, in.T, in.max_steps, in.err, a, b, sd.ph.ch_factor, sd.xi_mode, sd.nu, sd.xi_fixed, sd.dx);
}

// The same for kernels off the per-step path, which read the state themselves.
template <bool TWO = true>
__device__ inline Step begin_step(const SolveDesc& sd, double* red) {
  const StateIn in = read_state(sd);
  double a, b;
  load_partials<TWO>(sd, blockDim.x, a, b);
  return begin_step<TWO>(sd, red, blockDim.x, in, a, b);
}

// Population buffer of step n: fa for even n, fb for odd. While a solve
// advances, launch parity and step parity alternate together, so the buffer
// a launch reads is predicted as (par ^ npar) and its loads need not wait for
// n; a launch that finds n of the other parity (a solve resumed after a
// pause) loads again from the buffer of n.
__device__ inline int predicted_parity(const SolveDesc& sd) { return (sd.par ^ sd.npar) & 1; }

// End of a step: store this workgroup's maxima for the next launch; workgroup 0
// advances (t, n) for it, or carries a finished state over unchanged.
__device__ inline void end_step(const SolveDesc& sd, const Step& S, int tile, double lam, double cfm) {
  const int np = sd.par ^ 1;
  gmem<double>* pl = gl(sd.part) + (long long)np * 2 * sd.nblocks;
  if (threadIdx.x == 0) {
    pl[tile] = lam;
    pl[sd.nblocks + tile] = cfm;
    if (tile == 0) {
      Scal nx;
      nx.t = S.landing ? S.T : S.t + sd.dx / S.xi;
      nx.n = S.n + 1;
      nx.done = 0;
      nx.pad = 0;
      store_scal(gl(sd.st), np, nx);
    }
  }
}

// A finished solve: workgroup 0 carries the scalars and the partials (the
// maxima of the final state) over to the other parity unchanged.
__device__ inline void carry_done(const SolveDesc& sd, const Step& S, int tile) {
  if (tile != 0) return;
  const gmem<double>* src = gl(sd.part) + (long long)sd.par * 2 * sd.nblocks;
  gmem<double>* dst = gl(sd.part) + (long long)(sd.par ^ 1) * 2 * sd.nblocks;
  for (int i = threadIdx.x; i < 2 * sd.nblocks; i += blockDim.x) dst[i] = src[i];
  if (threadIdx.x == 0) {
    Scal nx;
    nx.t = S.t;
    nx.n = S.n;
    nx.done = 1;
    nx.pad = 0;
    store_scal(gl(sd.st), sd.par ^ 1, nx);
  }
}

// Split arithmetic type (the FP32 MHD split switches to FP64 per direction
// near coinciding speeds, inside Cell<K_MHD, DIM, float>::split).
template <int KIND, class T> struct SplitType { using type = T; };

// Stored bases of a cell (BASIS): 0 the Q populations; 1 the moving
// populations and U in the rest slot ("delta": U^{n+1} = U^n plus the
// differences of the moving populations, which keeps the small per-step
// increment out of a large FP32 sum); 2 as 1 with U kept as an unevaluated
// FP32 pair hi + lo, lo in an extra slot Q (compensated update), so the
// rounding of U does not accumulate over many steps.
template <int KIND, int DIM, class T, int BASIS>
struct Kern {
  static constexpr int P = SysInfo<KIND, DIM>::P;
  static constexpr int Q = DIM == 1 ? 3 : 5;
  static constexpr int REST = DIM == 1 ? 1 : 2;
  static constexpr bool DELTA = BASIS >= 1;
  static constexpr bool COMP = BASIS == 2;
  static constexpr int PLANES = (Q + (COMP ? 1 : 0)) * P;  // stored values per cell
  using ST = typename SplitType<KIND, T>::type;

  // Element index of stored plane `plane` (slot * P + variable) of `cell`:
  // cells are grouped in blocks of kBlock consecutive cells, and a block holds
  // all its planes one after another, so the rows a workgroup reads and
  // writes are few contiguous regions rather than PLANES far-apart streams.
  __device__ static inline long long pidx(int plane, long long cell) {
    return ((cell >> kBlockLog2) * PLANES + plane) * kBlock + (cell & (kBlock - 1));
  }

  // (SP: a pointer to const T, plain or global; see gmem)
  template <class SP>
  __device__ static inline void load(SP __restrict__ src, long long cell, T (&f)[Q][P]) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int v = 0; v < P; ++v) f[q][v] = src[pidx(q * P + v, cell)];
  }

  // 2D rows of the strip's own cells, which no other workgroup of the launch
  // reads: non-temporal loads, so those lines leave L2 before the halo-column
  // and edge-row lines that neighbouring workgroups read again. (1D steps keep
  // plain loads: their cells stay cache-resident from one launch to the next.)
  template <class SP>
  __device__ static inline void load_stream(SP __restrict__ src, long long cell, T (&f)[Q][P], T (&lo)[P]) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int v = 0; v < P; ++v) f[q][v] = __builtin_nontemporal_load(&src[pidx(q * P + v, cell)]);
#pragma unroll
    for (int v = 0; v < P; ++v) lo[v] = COMP ? __builtin_nontemporal_load(&src[pidx(Q * P + v, cell)]) : T(0);
  }

  // Low part of U (compensated basis only).
  template <class SP>
  __device__ static inline void load_lo(SP __restrict__ src, long long cell, T (&lo)[P]) {
#pragma unroll
    for (int v = 0; v < P; ++v) lo[v] = COMP ? src[pidx(Q * P + v, cell)] : T(0);
  }

  // U^{n+1} = U^n + d in the delta bases; the compensated one adds d and the
  // carried low part to hi with an error-free sum (Knuth's TwoSum), keeping
  // the rounding error as the new low part.
  __device__ static inline T advance(T hi, T d, T lo, T& lo_new) {
    if (!COMP) {
      lo_new = T(0);
      return hi + d;
    }
    const T b = d + lo;
    const T s = hi + b;
    const T bb = s - hi;
    lo_new = (hi - (s - bb)) + (b - bb);
    return s;
  }

  // From a cell's stored values form U^n and the post-collision populations
  // f* = f - omega (f - f^eq(U^n)) (Sec. 3.5 collision). In the delta basis U
  // is stored and the rest population is not formed.
  __device__ static inline void relax(const T (&f)[Q][P], const Phys& ph, double ixi, double Lam, double ch,
                                      T (&fs)[Q][P], T (&U)[P]) {
#pragma unroll
    for (int v = 0; v < P; ++v) {
      if (DELTA) {
        U[v] = f[REST][v];
      } else {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < Q; ++q) s += f[q][v];
        U[v] = s;
      }
    }
    ST Us[P];
#pragma unroll
    for (int v = 0; v < P; ++v) Us[v] = ST(U[v]);
    ST fe[Q][P];
    Equilibrium<KIND, DIM, ST>::eval(Us, ph, ST(ixi), ST(Lam), ST(ch), fe);
    const T om = T(ph.omega);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (DELTA && q == REST) continue;
#pragma unroll
      for (int v = 0; v < P; ++v) fs[q][v] = f[q][v] - om * (f[q][v] - T(fe[q][v]));
    }
  }

  // Delta bases, 2D: load only U (rest slot) and population q of a cell.
  template <class SP>
  __device__ static inline void load_one(SP __restrict__ src, long long cell, int q, T (&Ur)[P], T (&fq)[P]) {
#pragma unroll
    for (int v = 0; v < P; ++v) {
      Ur[v] = src[pidx(REST * P + v, cell)];
      fq[v] = src[pidx(q * P + v, cell)];
    }
  }

  // Delta bases, 2D: post-collision population of velocity +AXIS (plus) or
  // -AXIS from U and that population alone, with the split of that axis
  // only; bitwise what relax gives for it.
  template <int AXIS>
  __device__ static inline void relax_one(const T (&Ur)[P], const T (&fq)[P], bool plus, const Phys& ph,
                                          double ixi, double Lam, double ch, T (&out)[P]) {
    ST Us[P], fp[P], fm[P];
#pragma unroll
    for (int v = 0; v < P; ++v) Us[v] = ST(Ur[v]);
    Equilibrium<KIND, DIM, ST>::eval_axis(Us, ph, ST(ixi), ST(Lam), ST(ch), AXIS, fp, fm);
    const T om = T(ph.omega);
#pragma unroll
    for (int v = 0; v < P; ++v) out[v] = fq[v] - om * (fq[v] - T(plus ? fp[v] : fm[v]));
  }

  // One stored slot (p values) of a strip row, non-temporal (see load_stream).
  template <class SP>
  __device__ static inline void load_slot_stream(SP __restrict__ src, long long cell, int slot, T (&f)[P]) {
#pragma unroll
    for (int v = 0; v < P; ++v) f[v] = __builtin_nontemporal_load(&src[pidx(slot * P + v, cell)]);
  }

  // Delta bases, 2D: both post-collision populations of axis AXIS (+AXIS
  // from fplus, -AXIS from fminus) with one split of that axis; bitwise what
  // relax gives for them.
  template <int AXIS>
  __device__ static inline void relax_axis(const T (&Ur)[P], const T (&fplus)[P], const T (&fminus)[P],
                                           const Phys& ph, double ixi, double Lam, double ch, T (&outp)[P],
                                           T (&outm)[P]) {
    ST Us[P], fp[P], fm[P];
#pragma unroll
    for (int v = 0; v < P; ++v) Us[v] = ST(Ur[v]);
    Equilibrium<KIND, DIM, ST>::eval_axis(Us, ph, ST(ixi), ST(Lam), ST(ch), AXIS, fp, fm);
    const T om = T(ph.omega);
#pragma unroll
    for (int v = 0; v < P; ++v) {
      outp[v] = fplus[v] - om * (fplus[v] - T(fp[v]));
      outm[v] = fminus[v] - om * (fminus[v] - T(fm[v]));
    }
  }

  // U of a stored cell: the rest slot in the delta bases, else the sum of
  // the populations (in the order relax takes them).
  template <class SP>
  __device__ static inline void moments_of(SP __restrict__ src, long long cell, T (&U)[P]) {
#pragma unroll
    for (int v = 0; v < P; ++v) {
      if (DELTA) {
        U[v] = src[pidx(REST * P + v, cell)];
      } else {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < Q; ++q) s += src[pidx(q * P + v, cell)];
        U[v] = s;
      }
    }
  }

  template <class SP>
  __device__ static inline void collide(SP __restrict__ src, long long cell, const Phys& ph, double ixi,
                                        double Lam, double ch, T (&fs)[Q][P], T (&U)[P]) {
    T f[Q][P];
    load(src, cell, f);
    relax(f, ph, ixi, Lam, ch, fs, U);
  }

  // Speeds of a finished cell for the global maxima; flags non-physical
  // states (the error word, and the return value).
  __device__ static inline bool new_state(const SolveDesc& sd, const T (&U)[P], long long cell, long long step,
                                          double& lam, double& cfm) {
    ST Us[P];
#pragma unroll
    for (int v = 0; v < P; ++v) Us[v] = ST(U[v]);
    ST l, c;
    Cell<KIND, DIM, ST>::speeds(Us, sd.ph, &l, &c);
    const bool bad = !Cell<KIND, DIM, ST>::admissible(Us, sd.ph);
    if (bad) {
      report_cell(sd, ((unsigned long long)step << 32) | (unsigned long long)cell);
      l = ST(0);
      c = ST(0);
    }
    lam = fmax(lam, double(l));
    cfm = fmax(cfm, double(c));
    return bad;
  }
};

// ---------------------------------------------------------------------------
// 1D step: workgroups of B lanes own B - 2 consecutive output cells plus one
// halo cell on each side whose collision they recompute. The solve state, the
// previous launch's partials and the cell's stored values are all loaded at
// entry (the cell from the predicted buffer), so no load waits on another.
// The tiles holding the end cells apply characteristic boundaries in place.
// ---------------------------------------------------------------------------
template <int KIND, class T, int BASIS, int B, bool CHARBC>
__device__ inline void step1d_tile(const SolveDesc& sd, int tile) {
  using K = Kern<KIND, 1, T, BASIS>;
  using ST = typename K::ST;
  constexpr bool DELTA = K::DELTA;
  constexpr int P = K::P, Q = 3, TW = B - 2;
  __shared__ double red[2 * (B / 64) + 2], red_end[2 * (B / 64) + 2];
  const int N = sd.nx;
  const int tid = threadIdx.x;
  const int x = tile * TW - 1 + tid;
  const int xl = map_index(x < N + 1 ? x : N, N, sd.bcx);
  const StateIn in = read_state(sd);
  const int bp = predicted_parity(sd);
  T f[Q][P], lo[P];
  K::load(gl((const T*)(bp ? sd.fb : sd.fa)), xl, f);
  K::load_lo(gl((const T*)(bp ? sd.fb : sd.fa)), xl, lo);
  double pa, pb;
  load_partials<KIND == K_MHD>(sd, B, pa, pb);
  const Step S = begin_step<KIND == K_MHD>(sd, red, B, in, pa, pb);
  if (S.done) {
    carry_done(sd, S, tile);
    return;
  }
  const long long n = S.n;
  if (int(n & 1) != bp) {
    K::load(gl((const T*)((n & 1) ? sd.fb : sd.fa)), xl, f);
    K::load_lo(gl((const T*)((n & 1) ? sd.fb : sd.fa)), xl, lo);
  }
  gmem<T>* __restrict__ dst = gl((T*)((n & 1) ? sd.fa : sd.fb));
  const double ixi = 1.0 / S.xi, Lam = S.lam, ch = S.ch;

  __shared__ T s_plus[P][B], s_minus[P][B];
  __shared__ T s_unb[2][P];  // characteristic boundaries: U^n of cells 1 and N - 2

  T fs[Q][P], U[P];
  K::relax(f, sd.ph, ixi, Lam, ch, fs, U);
#pragma unroll
  for (int v = 0; v < P; ++v) { s_plus[v][tid] = fs[0][v]; s_minus[v][tid] = fs[2][v]; }
  // Characteristic boundaries (CHARBC: compiled in, applied when the solve
  // uses them). The tile holding a boundary cell also holds its interior
  // neighbour (as an own or a halo cell), whose U^n the condition needs.
  // With N = 3 the middle cell is the neighbour of both boundaries, so one
  // lane fills both slots.
  const bool charbc = CHARBC && sd.bcx == 2 && N >= 2;
  if (charbc && x == 1) {
#pragma unroll
    for (int v = 0; v < P; ++v) s_unb[0][v] = U[v];
  }
  if (charbc && x == N - 2) {
#pragma unroll
    for (int v = 0; v < P; ++v) s_unb[1][v] = U[v];
  }
  __syncthreads();

  double lam = 0.0, cfm = 0.0;
  if (tid >= 1 && tid <= TW && x < N) {
    T Un[P];
    if (!(charbc && (x == 0 || x == N - 1))) {
#pragma unroll
      for (int v = 0; v < P; ++v) {
        const T a = s_plus[v][tid - 1];
        const T b = s_minus[v][tid + 1];
        dst[K::pidx(0 * P + v, x)] = a;
        dst[K::pidx(2 * P + v, x)] = b;
        if (DELTA) {
          T lo_new;
          Un[v] = K::advance(U[v], (a - fs[0][v]) + (b - fs[2][v]), lo[v], lo_new);
          dst[K::pidx(1 * P + v, x)] = Un[v];
          if (K::COMP) dst[K::pidx(Q * P + v, x)] = lo_new;
        } else {
          dst[K::pidx(1 * P + v, x)] = fs[1][v];
          Un[v] = ((T(0) + a) + fs[1][v]) + b;
        }
      }
    } else {
      // Characteristic (non-reflecting) boundary of Sec. 3.3: from U^n of the
      // boundary cell b and of its interior neighbour, the characteristic
      // variables advance with the outgoing waves only (first-order one-sided
      // difference, linearized about b), U_b^{n+1} = U_b - P (Lambda dW)' / xi,
      // and b's populations become f^eq(U_b^{n+1}) with this step's xi and
      // Lambda (the compensated low part 0); its speeds join the tile's maxima.
      const int side = x == 0 ? 0 : 1;
      ST us[P], du[P], corr[P], unew[P];
#pragma unroll
      for (int v = 0; v < P; ++v) {
        us[v] = ST(U[v]);
        const ST nb = ST(s_unb[side][v]);
        du[v] = side == 1 ? ST(U[v]) - nb : nb - ST(U[v]);
      }
      Cell<KIND, 1, ST>::char_correction(us, du, sd.ph, ST(ch), side == 1, corr);
#pragma unroll
      for (int v = 0; v < P; ++v) unew[v] = us[v] - corr[v] * ST(ixi);
      ST fe[Q][P];
      Equilibrium<KIND, 1, ST>::eval(unew, sd.ph, ST(ixi), ST(Lam), ST(ch), fe);
#pragma unroll
      for (int v = 0; v < P; ++v) Un[v] = T(unew[v]);
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int v = 0; v < P; ++v) dst[K::pidx(q * P + v, x)] = (DELTA && q == K::REST) ? Un[v] : T(fe[q][v]);
      if (K::COMP) {
#pragma unroll
        for (int v = 0; v < P; ++v) dst[K::pidx(Q * P + v, x)] = T(0);
      }
    }
    K::new_state(sd, Un, x, n + 1, lam, cfm);
  }
  block_max2<KIND == K_MHD>(lam, cfm, red_end, B);
  end_step(sd, S, tile, lam, cfm);
}

// ---------------------------------------------------------------------------
// Small 1D grids (N <= B R cells): one workgroup of B lanes runs `count`
// whole steps in a loop, lane tid holding cells r * B + tid (r < R) in
// registers. The workgroup barrier is the global synchronization, so the
// steps need no launches: a step costs its arithmetic and three barriers
// instead of a launch. Every cell value and maximum comes from the same code
// as step1d_tile (and the max is exact), so the results are bitwise those of
// `count` step launches, and the kernel leaves the scalars, partials and
// populations as those launches would (parity sd.par ^ (count & 1)).
// ---------------------------------------------------------------------------
template <int KIND, class T, int BASIS, int R, int B>
__global__ void __launch_bounds__(B) k_run1d_wg(const SolveDesc sd, int count) {
  using K = Kern<KIND, 1, T, BASIS>;
  using ST = typename K::ST;
  constexpr bool DELTA = K::DELTA;
  constexpr bool MHD = KIND == K_MHD;
  constexpr int P = K::P, Q = 3;
  __shared__ T s_plus[P][B * R], s_minus[P][B * R];
  __shared__ T s_unb[2][P];   // characteristic boundaries: U^n of cells 1 and N - 2
  __shared__ double red[2 * (B / 64) + 2];
  const int N = sd.nx;
  const int tid = threadIdx.x;
  DevState* st = sd.st;
  // scalars and maxima left by the previous launch (parity sd.par)
  const Scal s0 = st->S[sd.par];
  double t = s0.t;
  long long n = s0.n;
  int done = s0.done;
  bool err = st->err_word != ~0ull;
  double lam = 0.0, cfm = 0.0;
  {
    const double* pl = sd.part + (long long)sd.par * 2 * sd.nblocks;
    for (int i = tid; i < sd.nblocks; i += B) {
      lam = fmax(lam, pl[i]);
      if (MHD) cfm = fmax(cfm, pl[sd.nblocks + i]);
    }
    block_max2_all<MHD>(lam, cfm, red, B);
  }
  T f[R][Q][P], lo[R][P];
  {
    const T* __restrict__ src = (const T*)((n & 1) ? sd.fb : sd.fa);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = r * B + tid;
      if (c < N) {
        K::load(src, c, f[r]);
        K::load_lo(src, c, lo[r]);
      }
    }
  }
  const int left_ghost = sd.bcx == 0 ? N - 1 : 0, right_ghost = sd.bcx == 0 ? 0 : N - 1;
  const bool charbc = sd.bcx == 2;
  for (int it = 0; it < count; ++it) {
    Scal sc;
    sc.t = t;
    sc.n = n;
    sc.done = done;
    sc.pad = 0;
    const Step S = derive_step(sc, st->T, st->max_steps, err, lam, cfm, sd.ph.ch_factor, sd.xi_mode, sd.nu,
                               sd.xi_fixed, sd.dx);
    if (S.done) {
      done = 1;
      break;
    }
    const double ixi = 1.0 / S.xi;
    T fs[R][Q][P], U[R][P];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = r * B + tid;
      if (c < N) {
        K::relax(f[r], sd.ph, ixi, S.lam, S.ch, fs[r], U[r]);
#pragma unroll
        for (int v = 0; v < P; ++v) {
          s_plus[v][c] = fs[r][0][v];
          s_minus[v][c] = fs[r][2][v];
        }
        if (charbc && c == 1) {
#pragma unroll
          for (int v = 0; v < P; ++v) s_unb[0][v] = U[r][v];
        }
        if (charbc && c == N - 2) {
#pragma unroll
          for (int v = 0; v < P; ++v) s_unb[1][v] = U[r][v];
        }
      }
    }
    __syncthreads();
    double lm = 0.0, cm = 0.0;
    int bad = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = r * B + tid;
      if (c < N) {
        const int cl = c > 0 ? c - 1 : left_ghost, cr = c < N - 1 ? c + 1 : right_ghost;
        T Un[P];
#pragma unroll
        for (int v = 0; v < P; ++v) {
          const T a = s_plus[v][cl];
          const T b = s_minus[v][cr];
          if (DELTA) {
            T lo_new;
            Un[v] = K::advance(U[r][v], (a - fs[r][0][v]) + (b - fs[r][2][v]), lo[r][v], lo_new);
            f[r][1][v] = Un[v];
            if (K::COMP) lo[r][v] = lo_new;
          } else {
            f[r][1][v] = fs[r][1][v];
            Un[v] = ((T(0) + a) + fs[r][1][v]) + b;
          }
          f[r][0][v] = a;
          f[r][2][v] = b;
        }
        if (charbc && (c == 0 || c == N - 1)) {
          // characteristic boundary (Sec. 3.3), as step1d_tile does it: from
          // U^n of the cell and of its interior neighbour,
          // U_b^{n+1} = U_b - P (Lambda dW)' / xi, populations f^eq(U_b^{n+1})
          const int side = c == 0 ? 0 : 1;
          ST us[P], du[P], corr[P], unew[P];
#pragma unroll
          for (int v = 0; v < P; ++v) {
            us[v] = ST(U[r][v]);
            const ST nb = ST(s_unb[side][v]);
            du[v] = side == 1 ? ST(U[r][v]) - nb : nb - ST(U[r][v]);
          }
          Cell<KIND, 1, ST>::char_correction(us, du, sd.ph, ST(S.ch), side == 1, corr);
#pragma unroll
          for (int v = 0; v < P; ++v) unew[v] = us[v] - corr[v] * ST(ixi);
          ST fe[Q][P];
          Equilibrium<KIND, 1, ST>::eval(unew, sd.ph, ST(ixi), ST(S.lam), ST(S.ch), fe);
#pragma unroll
          for (int v = 0; v < P; ++v) Un[v] = T(unew[v]);
#pragma unroll
          for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int v = 0; v < P; ++v) f[r][q][v] = (DELTA && q == K::REST) ? Un[v] : T(fe[q][v]);
          if (K::COMP) {
#pragma unroll
            for (int v = 0; v < P; ++v) lo[r][v] = T(0);
          }
        }
        bad |= K::new_state(sd, Un, c, S.n + 1, lm, cm) ? 1 : 0;
      }
    }
    // the barriers inside keep the LDS arrays and `red` from being rewritten
    // by the next step while a lane still reads them
    err = __syncthreads_or(bad) != 0 || err;
    block_max2_all<MHD>(lm, cm, red, B);
    lam = lm;
    cfm = cm;
    t = S.landing ? st->T : S.t + sd.dx / S.xi;
    n = S.n + 1;
  }
  T* __restrict__ dst = (T*)((n & 1) ? sd.fb : sd.fa);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int c = r * B + tid;
    if (c < N) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int v = 0; v < P; ++v) dst[K::pidx(q * P + v, c)] = f[r][q][v];
      if (K::COMP) {
#pragma unroll
        for (int v = 0; v < P; ++v) dst[K::pidx(Q * P + v, c)] = lo[r][v];
      }
    }
  }
  const int pf = sd.par ^ (count & 1);
  double* pl = sd.part + (long long)pf * 2 * sd.nblocks;
  for (int i = tid; i < sd.nblocks; i += B) {
    pl[i] = lam;
    pl[sd.nblocks + i] = cfm;
  }
  if (tid == 0) {
    Scal o;
    o.t = t;
    o.n = n;
    o.done = done;
    o.pad = 0;
    st->S[pf] = o;
  }
}


template <int KIND, class T, int BASIS, int B, bool CHARBC>
__global__ void __launch_bounds__(B) k_step1d(const SolveDesc sd) {
  step1d_tile<KIND, T, BASIS, B, CHARBC>(sd, blockIdx.x);
}

// ---------------------------------------------------------------------------
// 2D step: a workgroup of W lanes owns a strip of W columns and `band` rows and
// marches up the rows. Row r is collided, its +x/-x populations go through LDS
// (triple buffered, one barrier per row) to the lanes on either side, and row
// r-1 is finished with the +y population kept from row r-2 and the -y
// population of row r. The columns left and right of the strip are collided
// by wave 0 in batches of `halo` rows; the rows below and above the band are
// collided by the whole workgroup (only their y-moving populations are used).
// The new populations are written with non-temporal stores: nothing reads
// them again in this launch, and keeping them out of L2 leaves it to the
// halo and next-row loads (2-3% per step on MI355X at 2048^2 and 1024^2).
// ---------------------------------------------------------------------------
template <int KIND, class T, int BASIS, int W>
__device__ inline void step2d_tile_rows(const SolveDesc& sd, int tile) {
  using K = Kern<KIND, 2, T, BASIS>;
  constexpr bool DELTA = K::DELTA;
  constexpr int P = K::P, Q = 5, REST = 2;
  __shared__ double red[2 * (W / 64) + 2], red_end[2 * (W / 64) + 2];
  const int nx = sd.nx, ny = sd.ny, H = sd.band;
  const long long rs = sd.sx;  // row stride of the population buffers
  const int nsx = (nx + W - 1) / W;
  const int sx = tile % nsx, sy = tile / nsx;
  const int x0 = sx * W, y0 = sy * H, y1 = min(y0 + H, ny), nr = y1 - y0;
  const int tid = threadIdx.x;
  const int x = x0 + tid;
  const int xl = map_index(x < nx + 1 ? x : nx, nx, sd.bcx);
  // MHD bands march up (even sy) or down (odd sy) their rows, so two
  // neighbouring bands reach the row pair they share at the same time, both
  // at the start or both at the end: one band's read of the other's edge row
  // then comes from L2. Those reads are a tenth of an 8-row MHD band's; in
  // the 32-row bands of the other systems they are a fortieth, and there
  // alternating measured slower, so those bands all march up. Row of march
  // index i:
  constexpr bool ALTERNATE = KIND == K_MHD;
  const bool down = ALTERNATE && (sy & 1) != 0;
  auto row_of = [&](int i) { return down ? y1 - 1 - i : y0 + i; };
  // Row of the population buffers that holds march index i (mem_row).
  const bool whole = sy < sd.nfull;
  auto mem_of = [&](int i) -> long long { return whole ? (long long)i * sd.nfull + sy : row_of(i); };
  const StateIn in = read_state(sd);
  const int bp = predicted_parity(sd);
  const gmem<T>* __restrict__ src = gl((const T*)(bp ? sd.fb : sd.fa));
  // Systems with few values per cell (SW, Euler) load the next row while a
  // row is collided, so a row's memory latency overlaps the previous row's
  // work; MHD has no registers to spare for it.
  constexpr bool PREFETCH = Q * P <= 20;
  // Rows whose loads are in flight ahead of the one being collided (SW and
  // Euler): each lane keeps this many rows of stored values in registers.
  constexpr int AHEAD = PREFETCH ? 2 : 0;
  // In the delta bases the rows next to the band and the halo columns use one
  // population each: they load only U and that population and collide it with
  // the split of its axis alone.
  constexpr bool PARTIAL = DELTA;
  // The row before the band in march order streams one population into its
  // first row (y0 - 1: +y up; y1: -y down); the row after it, into its last.
  const long long below = mem_row(map_index(y0 - 1, ny, sd.bcy), H, sd.nfull, ALTERNATE) * rs + xl;
  const long long above = mem_row(map_index(y1, ny, sd.bcy), H, sd.nfull, ALTERNATE) * rs + xl;
  const long long pre = down ? above : below, post = down ? below : above;
  const int qpre = down ? 4 : 3, qpost = down ? 3 : 4;
  // Array slot that receives the row after the band's population (fixed, so
  // no register array is indexed at run time).
  constexpr int PS = ALTERNATE ? 3 : 4;
  // Stored values of the row before the band (its population in slot 3 of
  // the array whichever it is) and of the first row.
  T fpre[Q][P], fraw[Q][P], lo[P], fnext[Q][P], lonext[P], fnext2[Q][P], lonext2[P];
  auto load_first = [&]() {
    if (PARTIAL) K::load_one(src, pre, qpre, fpre[REST], fpre[3]);
    else K::load(src, pre, fpre);
    K::load_stream(src, mem_of(0) * rs + xl, fraw, lo);
    if (AHEAD == 2) {
      // the second row (or, in a one-row band, the row after the band)
      if (nr > 1) {
        K::load_stream(src, mem_of(1) * rs + xl, fnext, lonext);
      } else {
        if (PARTIAL) K::load_one(src, post, qpost, fnext[REST], fnext[PS]);
        else K::load(src, post, fnext);
      }
    }
  };
  load_first();
  double pa, pb;
  load_partials<KIND == K_MHD>(sd, W, pa, pb);
  const Step S = begin_step<KIND == K_MHD>(sd, red, W, in, pa, pb);
  if (S.done) {
    carry_done(sd, S, tile);
    return;
  }
  const long long n = S.n;
  if (int(n & 1) != bp) {
    src = gl((const T*)((n & 1) ? sd.fb : sd.fa));
    load_first();
  }
  gmem<T>* __restrict__ dst = gl((T*)((n & 1) ? sd.fa : sd.fb));
  const double ixi = 1.0 / S.xi, Lam = S.lam, ch = S.ch;

  __shared__ T s_ex[3][2][P][W];      // march slot, (+x, -x), var, lane
  __shared__ T s_halo[3][2][32][P];   // batch buffer, (left +x, right -x), row, var

  T fs[Q][P], U[P];
  // The population the row before the band streams into the first row; then
  // the one of the row two back in march order (+y up, -y down).
  T prevm[P];
  if (PARTIAL) {
    K::template relax_one<1>(fpre[REST], fpre[3], !down, sd.ph, ixi, Lam, ch, prevm);
  } else {
    K::relax(fpre, sd.ph, ixi, Lam, ch, fs, U);
#pragma unroll
    for (int v = 0; v < P; ++v) prevm[v] = down ? fs[4][v] : fs[3][v];
  }
  // Values of the previous row (march order) carried into the next iteration.
  T c_rest[P], c4[P], c5[P], c_lo[P];
  double lam = 0.0, cfm = 0.0;
  // The halo columns are collided by wave 0 in batches of hb rows (lanes
  // 0..hb-1 left, 32..32+hb-1 right), hb rows ahead of the strip: a short
  // batch reads them close in time to the neighbouring strips' own reads of
  // the same cells, so those come from L2. Three batch buffers keep a batch
  // from being overwritten while a slower wave still reads it.
  const int hb = sd.halo;

  // Finish the row of march index j, collided one iteration before: gather
  // the populations streaming into it (+x/-x from LDS; +y and -y from the
  // current row in fs and the row two back in prevm), store them and
  // U^{n+1}, and take the new state's speeds.
  auto finish = [&](int j) {
    const int rr = row_of(j);
    const int ps = (ALTERNATE ? j : rr) % 3;
    const int rb = j / hb;
    const int hbuf = rb % 3, hr = j - rb * hb;
    const long long cell = (long long)rr * nx + x;  // reported for a non-physical state
    const long long pc = mem_of(j) * rs + x;        // in the population buffers
    T Un[P];
#pragma unroll
    for (int v = 0; v < P; ++v) {
      const T a1 = tid > 0 ? s_ex[ps][0][v][tid - 1] : s_halo[hbuf][0][hr][v];
      const T a2 = tid < W - 1 ? s_ex[ps][1][v][tid + 1] : s_halo[hbuf][1][hr][v];
      const T a4 = down ? fs[3][v] : prevm[v];
      const T a5 = down ? prevm[v] : fs[4][v];
      __builtin_nontemporal_store(a1, &dst[K::pidx(0 * P + v, pc)]);
      __builtin_nontemporal_store(a2, &dst[K::pidx(1 * P + v, pc)]);
      __builtin_nontemporal_store(a4, &dst[K::pidx(3 * P + v, pc)]);
      __builtin_nontemporal_store(a5, &dst[K::pidx(4 * P + v, pc)]);
      if (DELTA) {
        const T b1 = s_ex[ps][0][v][tid], b2 = s_ex[ps][1][v][tid];
        T lo_new;
        Un[v] = K::advance(c_rest[v], ((a1 - b1) + (a2 - b2)) + ((a4 - c4[v]) + (a5 - c5[v])), c_lo[v], lo_new);
        if (K::COMP) __builtin_nontemporal_store(lo_new, &dst[K::pidx(Q * P + v, pc)]);
      } else {
        Un[v] = ((((T(0) + a1) + a2) + c_rest[v]) + a4) + a5;
      }
      __builtin_nontemporal_store(DELTA ? Un[v] : c_rest[v], &dst[K::pidx(REST * P + v, pc)]);
    }
    K::new_state(sd, Un, cell, n + 1, lam, cfm);
  };

  // One row: r, at march index i.
  auto row_step = [&](int i, int r) {
    const int bq = i / hb;
    if (i == bq * hb && tid < 64) {
      const int buf = bq % 3;
      const int side = tid >> 5;
      const int k = i + (tid & 31);
      if ((tid & 31) < hb && k < nr) {
        const long long hrow = mem_of(k) * rs;
        const int hx = map_index(side == 0 ? x0 - 1 : x0 + W, nx, sd.bcx);
        if (PARTIAL) {
          T hU[P], hq[P], hs[P];
          K::load_one(src, hrow + hx, side, hU, hq);
          K::template relax_one<0>(hU, hq, side == 0, sd.ph, ixi, Lam, ch, hs);
#pragma unroll
          for (int v = 0; v < P; ++v) s_halo[buf][side][tid & 31][v] = hs[v];
        } else {
          T hf[Q][P], hU[P];
          K::collide(src, hrow + hx, sd.ph, ixi, Lam, ch, hf, hU);
#pragma unroll
          for (int v = 0; v < P; ++v) s_halo[buf][side][tid & 31][v] = side == 0 ? hf[0][v] : hf[1][v];
        }
      }
    }
    // collide row r; the first row was loaded before the partials reduction
    if (PREFETCH) {
      // the row AHEAD rows on (row i + 1 came with the previous iteration
      // when AHEAD is 2), or the row after the band
      const int k = i + AHEAD;
      T(&dstf)[Q][P] = AHEAD == 2 ? fnext2 : fnext;
      T(&dstl)[P] = AHEAD == 2 ? lonext2 : lonext;
      if (k < nr) {
        __builtin_amdgcn_s_setprio(2);  // prefetch at raised wave priority, as in step2d_tile_axes
        K::load_stream(src, mem_of(k) * rs + xl, dstf, dstl);
        __builtin_amdgcn_s_setprio(0);
      } else if (k == nr) {
        if (PARTIAL) K::load_one(src, post, qpost, dstf[REST], dstf[PS]);
        else K::load(src, post, dstf);
      }
    } else if (i > 0) {
      K::load_stream(src, mem_of(i) * rs + xl, fraw, lo);
    }
    K::relax(fraw, sd.ph, ixi, Lam, ch, fs, U);
    const int slot = (ALTERNATE ? i : r) % 3;
#pragma unroll
    for (int v = 0; v < P; ++v) { s_ex[slot][0][v][tid] = fs[0][v]; s_ex[slot][1][v][tid] = fs[1][v]; }
    __syncthreads();
    if (i > 0 && x < nx) finish(i - 1);
    if (i > 0) {
#pragma unroll
      for (int v = 0; v < P; ++v) prevm[v] = down ? c5[v] : c4[v];
    }
#pragma unroll
    for (int v = 0; v < P; ++v) {
      c_rest[v] = DELTA ? U[v] : fs[REST][v];
      c_lo[v] = lo[v];
      c4[v] = fs[3][v];
      c5[v] = fs[4][v];
    }
    if (PREFETCH) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int v = 0; v < P; ++v) {
          fraw[q][v] = fnext[q][v];
          if (AHEAD == 2) fnext[q][v] = fnext2[q][v];
        }
      if (K::COMP) {
#pragma unroll
        for (int v = 0; v < P; ++v) {
          lo[v] = lonext[v];
          if (AHEAD == 2) lonext[v] = lonext2[v];
        }
      }
    }
  };
  // (The loop takes the form each system measured fastest with.)
  if (ALTERNATE) {
    for (int i = 0; i < nr; ++i) row_step(i, row_of(i));
  } else {
    for (int r = y0; r < y1; ++r) row_step(r - y0, r);
  }
  // The row after the band in march order: only the population it streams
  // into the last row is used; it finishes that row (whose LDS values were
  // published before the last barrier).
  if (!PREFETCH) {
    if (PARTIAL) K::load_one(src, post, qpost, fraw[REST], fraw[PS]);
    else K::load(src, post, fraw);
  }
  if (PARTIAL) {
    K::template relax_one<1>(fraw[REST], fraw[PS], down, sd.ph, ixi, Lam, ch, fs[PS]);
    if (ALTERNATE) {
#pragma unroll
      for (int v = 0; v < P; ++v) fs[4][v] = fs[3][v];
    }
  } else {
    K::relax(fraw, sd.ph, ixi, Lam, ch, fs, U);
  }
  if (x < nx) finish(nr - 1);
  block_max2<KIND == K_MHD>(lam, cfm, red_end, W);
  end_step(sd, S, tile, lam, cfm);
}

// ---------------------------------------------------------------------------
// 2D step of the delta bases for MHD, whose per-cell split holds most of the
// registers: a row's two axes are split at different points of its march
// iteration, and the row before it is finished in between, so the values a
// lane keeps live never include both axes' populations and the carried row at
// once. Wave 0 first collides the band's halo cells (one batch, whatever the
// solve's halo_rows). Iteration i of the march:
//   2. split row i's y axis: its +y and -y populations;
//   3. finish row i - 1 (the population row i streams into it is one of them);
//   4. issue the loads of row i + 1; split row i's x axis: +x and -x into LDS;
//   5. barrier.
// A row's +-x values are written in step 4 of its own iteration and read in
// step 3 of the next, with the barrier between, and every wave has passed the
// reads of iteration i before any writes of iteration i + 2: two LDS slots
// suffice (three in step2d_tile_rows, which finishes a row after the barrier).
// Per cell, every value is computed by the same expressions as in
// step2d_tile_rows, so the results are bitwise the same.
// ---------------------------------------------------------------------------
template <int KIND, class T, int BASIS, int W>
__device__ inline void step2d_tile_axes(const SolveDesc& sd, int tile) {
  using K = Kern<KIND, 2, T, BASIS>;
  static_assert(K::DELTA, "the axis-split march needs U stored in the rest slot");
  constexpr int P = K::P, Q = 5, REST = 2;
  __shared__ double red[2 * (W / 64) + 2], red_end[2 * (W / 64) + 2];
  const int nx = sd.nx, ny = sd.ny, H = sd.band;
  const long long rs = sd.sx;  // row stride of the population buffers
  const int nsx = (nx + W - 1) / W;
  const int sx = tile % nsx, sy = tile / nsx;
  const int x0 = sx * W, y0 = sy * H, y1 = min(y0 + H, ny), nr = y1 - y0;
  const int tid = threadIdx.x;
  const int x = x0 + tid;
  const int xl = map_index(x < nx + 1 ? x : nx, nx, sd.bcx);
  // bands march up (even sy) or down (odd sy), as in step2d_tile_rows
  const bool down = (sy & 1) != 0;
  auto row_of = [&](int i) { return down ? y1 - 1 - i : y0 + i; };
  // Row of the population buffers that holds march index i (mem_row).
  const bool whole = sy < sd.nfull;
  auto mem_of = [&](int i) -> long long { return whole ? (long long)i * sd.nfull + sy : row_of(i); };
  const StateIn in = read_state(sd);
  const int bp = predicted_parity(sd);
  const gmem<T>* __restrict__ src = gl((const T*)(bp ? sd.fb : sd.fa));
  const long long below = mem_row(map_index(y0 - 1, ny, sd.bcy), H, sd.nfull, true) * rs + xl;
  const long long above = mem_row(map_index(y1, ny, sd.bcy), H, sd.nfull, true) * rs + xl;
  const long long pre = down ? above : below, post = down ? below : above;
  const int qpre = down ? 4 : 3, qpost = down ? 3 : 4;
  // the row before the band (U and its population into the first row); the
  // stored values of row i (r*) and of row i + 1 (n*), which are loaded
  // while row i's x axis is split, so their memory latency overlaps that work
  T preU[P], preq[P], rU[P], rlo[P], ry3[P], ry4[P], rx0[P], rx1[P];
  T nU[P], nlo[P], ny3[P], ny4[P], nx0[P], nx1[P];
  auto load_next = [&](int i) {
    const long long cell = mem_of(i) * rs + xl;
    K::load_slot_stream(src, cell, REST, nU);
    if (K::COMP) K::load_slot_stream(src, cell, Q, nlo);
    K::load_slot_stream(src, cell, 3, ny3);
    K::load_slot_stream(src, cell, 4, ny4);
    K::load_slot_stream(src, cell, 0, nx0);
    K::load_slot_stream(src, cell, 1, nx1);
  };
  auto take_next = [&]() {
#pragma unroll
    for (int v = 0; v < P; ++v) {
      rU[v] = nU[v];
      rlo[v] = K::COMP ? nlo[v] : T(0);
      ry3[v] = ny3[v];
      ry4[v] = ny4[v];
      rx0[v] = nx0[v];
      rx1[v] = nx1[v];
    }
  };
  auto load_first = [&]() {
    K::load_one(src, pre, qpre, preU, preq);
    load_next(0);
    take_next();
  };
  load_first();
  double pa, pb;
  load_partials<true>(sd, W, pa, pb);
  const Step S = begin_step<true>(sd, red, W, in, pa, pb);
  if (S.done) {
    carry_done(sd, S, tile);
    return;
  }
  const long long n = S.n;
  if (int(n & 1) != bp) {
    src = gl((const T*)((n & 1) ? sd.fb : sd.fa));
    load_first();
  }
  gmem<T>* __restrict__ dst = gl((T*)((n & 1) ? sd.fa : sd.fb));
  const double ixi = 1.0 / S.xi, Lam = S.lam, ch = S.ch;

  constexpr int HMAX = 64;            // band rows (vklb_options.band_rows <= 64 here)
  __shared__ T s_ex[2][2][P][W];      // row parity, (+x, -x), var, lane
  __shared__ T s_halo[2][HMAX][P];    // (left +x, right -x), march index, var

  // 1. the band's halo cells: lanes 0-31 the left column, 32-63 the right,
  // 32 rows at a time (read after the first iteration's barrier)
  if (tid < 64) {
    const int side = tid >> 5;
    const int hx = map_index(side == 0 ? x0 - 1 : x0 + W, nx, sd.bcx);
    for (int k = tid & 31; k < nr; k += 32) {
      T hU[P], hq[P], hs[P];
      K::load_one(src, mem_of(k) * rs + hx, side, hU, hq);
      K::template relax_one<0>(hU, hq, side == 0, sd.ph, ixi, Lam, ch, hs);
#pragma unroll
      for (int v = 0; v < P; ++v) s_halo[side][k][v] = hs[v];
    }
  }
  // the population the row before the band streams into the first row; then
  // that of the row before the one being finished
  T prevm[P];
  K::template relax_one<1>(preU, preq, !down, sd.ph, ixi, Lam, ch, prevm);
  // the row being finished: its U, low part and its own y populations
  T c_rest[P], c_lo[P], c4[P], c5[P];
  double lam = 0.0, cfm = 0.0;

  // Finish the row of march index j (its +-x values are in LDS slot j & 1);
  // ym: the population the row after it streams into it.
  auto finish = [&](int j, const T (&ym)[P]) {
    const int rr = row_of(j);
    const int ps = j & 1;
    const long long cell = (long long)rr * nx + x;  // reported for a non-physical state
    const long long pc = mem_of(j) * rs + x;        // in the population buffers
    T Un[P];
#pragma unroll
    for (int v = 0; v < P; ++v) {
      const T a1 = tid > 0 ? s_ex[ps][0][v][tid - 1] : s_halo[0][j][v];
      const T a2 = tid < W - 1 ? s_ex[ps][1][v][tid + 1] : s_halo[1][j][v];
      const T a4 = down ? ym[v] : prevm[v];
      const T a5 = down ? prevm[v] : ym[v];
      __builtin_nontemporal_store(a1, &dst[K::pidx(0 * P + v, pc)]);
      __builtin_nontemporal_store(a2, &dst[K::pidx(1 * P + v, pc)]);
      __builtin_nontemporal_store(a4, &dst[K::pidx(3 * P + v, pc)]);
      __builtin_nontemporal_store(a5, &dst[K::pidx(4 * P + v, pc)]);
      const T b1 = s_ex[ps][0][v][tid], b2 = s_ex[ps][1][v][tid];
      T lo_new;
      Un[v] = K::advance(c_rest[v], ((a1 - b1) + (a2 - b2)) + ((a4 - c4[v]) + (a5 - c5[v])), c_lo[v], lo_new);
      if (K::COMP) __builtin_nontemporal_store(lo_new, &dst[K::pidx(Q * P + v, pc)]);
      __builtin_nontemporal_store(Un[v], &dst[K::pidx(REST * P + v, pc)]);
    }
    K::new_state(sd, Un, cell, n + 1, lam, cfm);
  };

  for (int i = 0; i < nr; ++i) {
    // 2. row i's y split (row i came with the previous iteration, row 0 at entry)
    if (i > 0) take_next();
    T fs3[P], fs4[P];
    K::template relax_axis<1>(rU, ry3, ry4, sd.ph, ixi, Lam, ch, fs3, fs4);
    // 3. finish the row before
    if (i > 0) {
      if (x < nx) finish(i - 1, down ? fs3 : fs4);
#pragma unroll
      for (int v = 0; v < P; ++v) prevm[v] = down ? c5[v] : c4[v];
    }
#pragma unroll
    for (int v = 0; v < P; ++v) {
      c_rest[v] = rU[v];
      c_lo[v] = K::COMP ? rlo[v] : T(0);
      c4[v] = fs3[v];
      c5[v] = fs4[v];
    }
    // 4. load row i + 1; row i's x split, into LDS
    {
      T fs0[P], fs1[P];
      // issued at raised wave priority: the SIMD's other wave is usually in
      // its split, and these loads should not wait behind its arithmetic
      // (Orszag-Tang 1024^2 82.0 -> 79.0 us per step)
      __builtin_amdgcn_s_setprio(2);
      if (i + 1 < nr) load_next(i + 1);
      __builtin_amdgcn_s_setprio(0);
      K::template relax_axis<0>(rU, rx0, rx1, sd.ph, ixi, Lam, ch, fs0, fs1);
      const int slot = i & 1;
#pragma unroll
      for (int v = 0; v < P; ++v) { s_ex[slot][0][v][tid] = fs0[v]; s_ex[slot][1][v][tid] = fs1[v]; }
    }
    // 5.
    __syncthreads();
  }
  // The row after the band in march order: only the population it streams
  // into the last row is used; it finishes that row.
  {
    T postU[P], postq[P], ym[P];
    K::load_one(src, post, qpost, postU, postq);
    K::template relax_one<1>(postU, postq, down, sd.ph, ixi, Lam, ch, ym);
    if (x < nx) finish(nr - 1, ym);
  }
  block_max2<true>(lam, cfm, red_end, W);
  end_step(sd, S, tile, lam, cfm);
}

// 2D step of one tile: the axis-split march for MHD in the delta bases,
// else the row march.
template <int KIND, class T, int BASIS, int W>
__device__ inline void step2d_tile(const SolveDesc& sd, int tile) {
  if constexpr (KIND == K_MHD && BASIS >= 1) step2d_tile_axes<KIND, T, BASIS, W>(sd, tile);
  else step2d_tile_rows<KIND, T, BASIS, W>(sd, tile);
}

template <int KIND, class T, int BASIS, int W>
__global__ void __launch_bounds__(W) k_step2d(const SolveDesc sd) {
  step2d_tile<KIND, T, BASIS, W>(sd, xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Batched step for serving: one launch advances every resident solve of one
// system class by one time step. Work item i = (solve slot, tile); the tile
// runs the same code as in the single-solve kernels, so a solve gives the
// same bits alone and in a batch. Items beyond nwork exit.
// ---------------------------------------------------------------------------
struct WorkItem {
  int slot;
  int tile;
};

template <int KIND, int DIM, class T, int BASIS, int W>
__global__ void __launch_bounds__(W) k_step_batched(const SolveDesc* __restrict__ descs,
                                                    const WorkItem* __restrict__ work, const int* __restrict__ nwork,
                                                    int par) {
  const int i = blockIdx.x;
  if (i >= *nwork) return;
  const WorkItem w = work[i];
  SolveDesc sd = descs[w.slot];
  sd.par = par;
  if constexpr (DIM == 1) step1d_tile<KIND, T, BASIS, 256, true>(sd, w.tile);
  else step2d_tile<KIND, T, BASIS, W>(sd, w.tile);
}

// ---------------------------------------------------------------------------
// One workgroup folds the per-workgroup maxima of parity `par` into entry 0
// of each half (max |lambda|, max c_f). The max is exact and independent of
// order, so a step launch that reads entry 0 alone derives the step every
// workgroup would derive from all the entries. Eight loads per lane and
// iteration keep enough of them in flight for a million workgroups.
template <int LANES = 1024>
__global__ void __launch_bounds__(LANES) k_fold_partials(const SolveDesc sd, int par) {
  __shared__ double red[2 * (LANES / 64) + 2];
  double* pl = sd.part + (long long)par * 2 * sd.nblocks;
  const double* pc = pl + sd.nblocks;
  const int nb = sd.nblocks;
  double a = 0.0, b = 0.0;
  for (int i0 = threadIdx.x; i0 < nb; i0 += 8 * LANES) {
    double x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * LANES;
      x[u] = i < nb ? pl[i] : 0.0;
      y[u] = i < nb ? pc[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a = fmax(a, x[u]);
      b = fmax(b, y[u]);
    }
  }
  block_max2_all<true>(a, b, red, LANES);
  if (threadIdx.x == 0) {
    pl[0] = a;
    pl[nb] = b;
  }
}

// ---------------------------------------------------------------------------
// Initialization: (1) reduction of max|lambda| and max c_f over U0 (FP64
// staging) giving xi^0, Lambda^0, c_h^0; (2) f_q = f_q^eq(U0) (Sec. 3.5).
// ---------------------------------------------------------------------------
template <int KIND, int DIM>
__global__ void __launch_bounds__(256) k_init_reduce(const SolveDesc sd) {
  // Grid = the step grid: block b writes partial b of parity sd.par.
  constexpr int P = SysInfo<KIND, DIM>::P;
  __shared__ double red[10];
  const long long cells = (long long)sd.nx * sd.ny;
  double lam = 0.0, cfm = 0.0;
  for (long long c = blockIdx.x * 256ll + threadIdx.x; c < cells; c += (long long)gridDim.x * 256) {
    double U[P];
#pragma unroll
    for (int v = 0; v < P; ++v) U[v] = sd.stage[v * cells + c];
    double l, f;
    Cell<KIND, DIM, double>::speeds(U, sd.ph, &l, &f);
    if (!Cell<KIND, DIM, double>::admissible(U, sd.ph)) {
      atomicMin(&sd.st->err_word, (unsigned long long)c);
      l = 0.0;
      f = 0.0;
    }
    lam = fmax(lam, l);
    cfm = fmax(cfm, f);
  }
  block_max2(lam, cfm, red, blockDim.x);
  if (threadIdx.x == 0) {
    double* pl = sd.part + (long long)sd.par * 2 * sd.nblocks;
    pl[blockIdx.x] = lam;
    pl[sd.nblocks + blockIdx.x] = cfm;
  }
}

// Population-buffer index of natural cell c = j * nx + i (2D: rows padded to
// sx and placed by mem_row; down_odd: the solve's odd bands march down).
__device__ inline long long pcell(const SolveDesc& sd, long long c, bool down_odd) {
  if (sd.sx == sd.nx && sd.nfull == 0) return c;
  const long long j = c / sd.nx;
  return mem_row(int(j), sd.band, sd.nfull, down_odd) * sd.sx + (c - j * sd.nx);
}

template <int KIND, int DIM, class T, int BASIS>
__global__ void __launch_bounds__(256) k_init_feq(const SolveDesc sd) {
  using K = Kern<KIND, DIM, T, BASIS>;
  constexpr bool DELTA = K::DELTA;
  constexpr int P = K::P, Q = K::Q;
  using ST = typename K::ST;
  __shared__ double red[10];
  const Step S = begin_step(sd, red);
  T* __restrict__ f = (T*)sd.fa;
  const long long cells = (long long)sd.nx * sd.ny;
  const double ixi = 1.0 / S.xi;
  for (long long c = blockIdx.x * 256ll + threadIdx.x; c < cells; c += (long long)gridDim.x * 256) {
    T U[P];
    ST Us[P];
#pragma unroll
    for (int v = 0; v < P; ++v) { U[v] = T(sd.stage[v * cells + c]); Us[v] = ST(U[v]); }
    ST fe[Q][P];
    Equilibrium<KIND, DIM, ST>::eval(Us, sd.ph, ST(ixi), ST(S.lam), ST(S.ch), fe);
    const long long pc = pcell(sd, c, KIND == K_MHD);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int v = 0; v < P; ++v)
        f[K::pidx(q * P + v, pc)] = (DELTA && q == K::REST) ? U[v] : T(fe[q][v]);
    if (K::COMP) {
#pragma unroll
      for (int v = 0; v < P; ++v)
        f[K::pidx(Q * P + v, pc)] = T(sd.stage[v * cells + c] - double(U[v]));
    }
  }
}

// U = sum_q f_q (or the stored U, hi + lo when compensated) into the FP64 staging.
template <int KIND, int DIM, class T, int BASIS>
__global__ void __launch_bounds__(256) k_moments(const SolveDesc sd) {
  using K = Kern<KIND, DIM, T, BASIS>;
  constexpr bool DELTA = K::DELTA;
  constexpr int P = K::P, Q = K::Q;
  const long long n = sd.st->S[sd.par].n;
  const T* __restrict__ f = (const T*)((n & 1) ? sd.fb : sd.fa);
  double* out = const_cast<double*>(sd.stage);
  const long long cells = (long long)sd.nx * sd.ny;
  for (long long c = blockIdx.x * 256ll + threadIdx.x; c < cells; c += (long long)gridDim.x * 256) {
    const long long pc = pcell(sd, c, KIND == K_MHD);
#pragma unroll
    for (int v = 0; v < P; ++v) {
      T s;
      if (DELTA) {
        s = f[K::pidx(K::REST * P + v, pc)];
      } else {
        s = T(0);
#pragma unroll
        for (int q = 0; q < Q; ++q) s += f[K::pidx(q * P + v, pc)];
      }
      out[v * cells + c] = K::COMP ? double(s) + double(f[K::pidx(Q * P + v, pc)]) : double(s);
    }
  }
}

}  // namespace vklb
