// Host runtime behind include/vklb.h: argument checks, workspace layout,
// kernel dispatch, HIP-graph chunks of step launches, diagnostics.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vklb.h"
#include "vklb_host.hpp"

using namespace vklb;

namespace {

std::mutex g_err_mu;
// Message of the last failed call that has no solver handle (vklb_create,
// vklb_tune, vklb_run_static). A fixed buffer, so that reporting an error
// allocates nothing.
char g_create_error[512] = "";

void set_create_error(const char* msg) {
  std::lock_guard<std::mutex> lk(g_err_mu);
  snprintf(g_create_error, sizeof g_create_error, "%s", msg);
}

__global__ void k_totals_partial(const double* __restrict__ U, long long cells, int p, double* __restrict__ part) {
  // Neumaier partial sums of each field over a grid-stride range, combined per
  // block in a fixed lane order (deterministic for a fixed grid).
  __shared__ double ss[256], sc[256];
  for (int v = 0; v < p; ++v) {
    double s = 0.0, comp = 0.0;
    for (long long c = blockIdx.x * 256ll + threadIdx.x; c < cells; c += (long long)gridDim.x * 256) {
      const double x = U[v * cells + c];
      const double t = s + x;
      comp += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
      s = t;
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = comp;
    __syncthreads();
    if (threadIdx.x == 0) {
      double S = 0.0, C = 0.0;
      for (int i = 0; i < 256; ++i) {
        const double x = ss[i];
        const double t = S + x;
        C += fabs(S) >= fabs(x) ? (S - t) + x : (x - t) + S;
        S = t;
        C += sc[i];
      }
      part[(blockIdx.x * 9 + v) * 2 + 0] = S;
      part[(blockIdx.x * 9 + v) * 2 + 1] = C;
    }
    __syncthreads();
  }
}

__global__ void k_totals_final(const double* __restrict__ part, int nblk, int p, double* __restrict__ out) {
  const int v = threadIdx.x;
  if (v >= p) return;
  double S = 0.0, C = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double x = part[(b * 9 + v) * 2];
    const double t = S + x;
    C += fabs(S) >= fabs(x) ? (S - t) + x : (x - t) + S;
    S = t;
    C += part[(b * 9 + v) * 2 + 1];
  }
  out[v] = S + C;
}

// max |dBx/dx + dBy/dy| by central differences on the FP64 moments; ghosts
// follow the boundary rule (periodic wrap or copy of the boundary cell).
__global__ void k_divb(const double* __restrict__ U, int nx, int ny, double dx, int bcx, int bcy,
                       unsigned long long* __restrict__ out) {
  const long long cells = (long long)nx * ny;
  double m = 0.0;
  for (long long c = blockIdx.x * 256ll + threadIdx.x; c < cells; c += (long long)gridDim.x * 256) {
    const int i = int(c % nx), j = int(c / nx);
    const int ip = map_index(i + 1, nx, bcx), im = map_index(i - 1, nx, bcx);
    const int jp = map_index(j + 1, ny, bcy), jm = map_index(j - 1, ny, bcy);
    const double* Bx = U + 5 * cells;
    const double* By = U + 6 * cells;
    const double d = (Bx[(long long)j * nx + ip] - Bx[(long long)j * nx + im]) / (2.0 * dx) +
                     (By[(long long)jp * nx + i] - By[(long long)jm * nx + i]) / (2.0 * dx);
    m = fmax(m, fabs(d));
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// Workspace of vklb_run_static: one per GPU, held from the library's load on
// that GPU until the process ends. Host code never takes this name's address
// for device use: it is a host-side stand-in; the device address comes from
// hipGetSymbolAddress (static_workspace below).
static __device__ __align__(256) char scratch[VKLB_STATIC_BYTES];

// Solve scalars of a fresh run (what vklb_init's host copy writes), written by
// a kernel so that the allocation-free path enqueues no host-to-device copy.
__global__ void k_static_reset(DevState* st, double T, long long max_steps) {
  if (threadIdx.x != 0) return;
  for (int p = 0; p < 2; ++p) {
    st->S[p].t = 0.0;
    st->S[p].n = 0;
    st->S[p].done = 0;
    st->S[p].pad = 0;
  }
  st->T = T;
  st->max_steps = max_steps;
  st->err_word = ~0ull;
}

// Time, step count and error report of a finished vklb_run_static, read from
// the scalars of the launch parity `par` the next launch would use.
__global__ void k_static_info(const DevState* st, int par, vklb_run_info* out) {
  if (threadIdx.x != 0) return;
  const Scal S = st->S[par];
  const unsigned long long ew = st->err_word;
  const bool err = ew != ~0ull;
  out->t = S.t;
  out->steps = S.n;
  out->nonphysical = err ? 1 : 0;
  out->fail_step = err ? (long long)(ew >> 32) : -1;
  out->fail_cell = err ? (long long)(ew & 0xffffffffull) : -1;
  out->done = (S.done || S.n >= st->max_steps || !(S.t < st->T) || err) ? 1 : 0;
}

// Streaming copy of n16 16-byte words, one word per lane and one workgroup
// per 4 KiB: every wave issues its load and its store and ends, so the
// dispatcher keeps the compute units full of fresh waves and their loads in
// flight. Measured on MI355X (2 GiB): 6.14 TB/s read + write, against
// 5.0-5.5 TB/s for grid-stride or per-workgroup chunked loops with four or
// eight words per lane and 4.9 TB/s for hipMemcpyAsync. NT: non-temporal
// load and store (the step kernels' population stores and 2D row loads).
typedef float v4f __attribute__((ext_vector_type(4)));
template <bool NT>
__global__ void __launch_bounds__(256) k_stream_copy(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                     long long n16) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n16) return;
  if (NT) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
  else dst[i] = src[i];
}

}  // namespace

// Trailer of a checkpoint blob (see vklb_state_bytes).
struct CkptTrailer {
  unsigned long long magic;
  int kind, dim, prec, basis;
  long long nx, ny;
  double t, lam7, cfm, pad0;
  long long n;
  int done, pad;
  char reserved[128 - 8 - 16 - 16 - 32 - 8 - 8];
};
static_assert(sizeof(CkptTrailer) == 128, "trailer is 128 bytes");

struct vklb_solver {
  vklb_system sys;
  vklb_lattice lat;
  vklb_grid grid;
  vklb_speed speed;
  double omega;
  vklb_bc bc[2];
  vklb_equilibrium eq;
  vklb_precision prec;
  vklb_options opt;
  Layout L;
  char* buf = nullptr;
  bool own_buf = false;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  Launchers K;
  SolveDesc sd;
  int step_grid = 0;
  double T = INFINITY;
  long long max_steps = (1ll << 62);
  bool inited = false;
  int chunk = 64;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  std::string err;
  int device = 0;
  int basis = 0;
  long long launches = 0;   // step launches since init (selects the parity)
  int wg_cells = 0;         // > 0: 1D steps run in one workgroup, this many cells per lane
  int wg_lanes = 0;         // and this many lanes
};

namespace {

vklb_status fail(vklb_solver* s, vklb_status st, const std::string& msg) {
  if (s) s->err = msg;
  else set_create_error(msg.c_str());
  return st;
}

vklb_status hip_fail(vklb_solver* s, hipError_t e, const char* what) {
  return fail(s, VKLB_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(s, call)                                    \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail((s), e_, #call); \
  } while (0)

// The step graph holds copies of the kernel descriptor; it is rebuilt on the
// next use after the descriptor changes.
static void drop_graph(vklb_solver* s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->gexec = nullptr;
  s->graph = nullptr;
}

// Launches of parity 0 run steps of parity npar (the step kernels predict
// their source buffer from it).
static vklb_status set_npar(vklb_solver* s, int npar) {
  if (s->sd.npar == npar) return VKLB_OK;
  s->sd.npar = npar;
  if (s->gexec) HIPCHK(s, hipStreamSynchronize(s->stream));  // no replay in flight
  drop_graph(s);
  return VKLB_OK;
}

vklb_status reset_state(vklb_solver* s, double t, long long n, int done) {
  vklb_status st = set_npar(s, int(n & 1));
  if (st != VKLB_OK) return st;
  DevState h;
  memset(&h, 0, sizeof h);
  h.S[0].t = t;
  h.S[0].n = n;
  h.S[0].done = done;
  h.S[1] = h.S[0];
  h.T = s->T;
  h.max_steps = s->max_steps;
  h.err_word = ~0ull;
  HIPCHK(s, hipMemcpyAsync(s->buf + s->L.state_off, &h, sizeof(h), hipMemcpyHostToDevice, s->stream));
  s->launches = 0;
  return VKLB_OK;
}

// Folds the partials of parity `par` into entry 0 when the solve's step
// launches read that entry alone.
vklb_status fold_partials(vklb_solver* s, hipStream_t st, int par) {
  HIPCHK(s, launch_fold(s->sd, par, st));
  return VKLB_OK;
}

// n step launches, the first of launch index first_launch, each followed by
// the fold of its partials when the solve folds them.
hipError_t enqueue_steps(const SolveDesc& sd, const Launchers& K, long long n, long long first_launch, hipStream_t st) {
  SolveDesc d = sd;
  for (long long i = 0; i < n; ++i) {
    d.par = int((first_launch + i) & 1);
    hipError_t e = K.step(d, d.nblocks, st);
    if (e == hipSuccess) e = launch_fold(d, d.par ^ 1, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Small 1D grids: n steps in launches of up to 1024 steps of one workgroup;
// each stands for that many step launches (it leaves their parity).
hipError_t enqueue_wg_steps(const SolveDesc& sd, const Launchers& K, int wg_cells, int wg_lanes, long long n,
                            long long first_launch, hipStream_t st) {
  long long done = 0;
  while (done < n) {
    const int count = int(std::min<long long>(n - done, 1024));
    SolveDesc d = sd;
    d.par = int((first_launch + done) & 1);
    hipError_t e = K.run_wg(d, count, wg_cells, wg_lanes, st);
    if (e != hipSuccess) return e;
    done += count;
  }
  return hipSuccess;
}

vklb_status launch_steps(vklb_solver* s, hipStream_t st, long long n, long long first_launch) {
  HIPCHK(s, enqueue_steps(s->sd, s->K, n, first_launch, st));
  return VKLB_OK;
}

vklb_status ensure_graph(vklb_solver* s) {
  if (s->gexec) return VKLB_OK;
  if (!s->cap_stream) HIPCHK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
  HIPCHK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  vklb_status st = launch_steps(s, s->cap_stream, s->chunk, 0);  // parities 0, 1, 0, 1, ...
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s->cap_stream, &g);
  if (st != VKLB_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != VKLB_OK ? st : hip_fail(s, e, "hipStreamEndCapture");
  }
  s->graph = g;
  HIPCHK(s, hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0));
  return VKLB_OK;
}

CkptTrailer make_trailer(const vklb_solver* s) {
  CkptTrailer tr;
  memset(&tr, 0, sizeof tr);
  tr.magic = 0x564b4c4243505432ull;  // "VKLBCPT2"
  tr.kind = s->sys.kind;
  tr.dim = s->grid.dim;
  tr.prec = s->prec;
  tr.basis = s->basis;
  tr.nx = s->grid.n[0];
  tr.ny = s->grid.dim == 2 ? s->grid.n[1] : 1;
  return tr;
}

// Host view of the latest state: scalars, partial maxima and the derived step.
struct HostView {
  DevState h;
  Scal S;
  double lam7, cfm;
  Step step;
  bool err;
  long long err_step, err_cell;
};

vklb_status read_view(vklb_solver* s, HostView* v) {
  const int par = int(s->launches & 1);
  std::vector<double> part(size_t(2) * s->sd.nblocks);
  HIPCHK(s, hipMemcpyAsync(&v->h, s->buf + s->L.state_off, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(part.data(), s->sd.part + size_t(par) * 2 * s->sd.nblocks, part.size() * 8,
                           hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  v->S = v->h.S[par];
  double a = 0.0, b = 0.0;
  for (int i = 0; i < s->sd.nblocks; ++i) {
    a = fmax(a, part[i]);
    b = fmax(b, part[s->sd.nblocks + i]);
  }
  v->lam7 = a;
  v->cfm = b;
  v->err = v->h.err_word != ~0ull;
  v->err_step = v->err ? (long long)(v->h.err_word >> 32) : -1;
  v->err_cell = v->err ? (long long)(v->h.err_word & 0xffffffffull) : -1;
  const SolveDesc& d = s->sd;
  v->step = derive_step(v->S, v->h.T, v->h.max_steps, v->err, a, b, d.ph.ch_factor, d.xi_mode, d.nu, d.xi_fixed, d.dx);
  return VKLB_OK;
}

vklb_status check_err(vklb_solver* s, const HostView& v) {
  if (v.err) {
    char msg[160];
    snprintf(msg, sizeof msg, "non-physical state produced at step %lld, cell %lld", v.err_step, v.err_cell);
    return fail(s, VKLB_ERR_NONPHYSICAL, msg);
  }
  return VKLB_OK;
}

// Everything vklb_create derives from its arguments, before any memory
// exists: the layout, the kernels and the descriptor (bound to a workspace
// by bind()). Allocates nothing.
struct Plan {
  Layout L;
  Launchers K;
  vklb_grid grid;     // n[1] = 1 in 1D
  vklb_bc bc[2];      // bc[1] = bc[0] in 1D
  vklb_system sys;
  vklb_speed lambda;
  vklb_equilibrium eq;
  double omega;
  int basis = 0, width = 0, band = 0, halo = 0;
  int nred_one = 0;   // fold each launch's partials into one entry
  int wg_cells = 0, wg_lanes = 0;

  SolveDesc bind(char* buf) const {
    SolveDesc d = make_desc(buf, L, &sys, &grid, &lambda, omega, bc, &eq, width, band, halo);
    if (nred_one) d.nred = 1;
    return d;
  }
};

vklb_status plan_solve(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid, const vklb_speed* lambda,
                       double omega, const vklb_bc bc[2], const vklb_equilibrium* eq, vklb_precision prec,
                       const vklb_options& o, Plan* pl, const char** msg) {
  vklb_status vst = validate(sys, lat, grid, lambda, omega, bc, eq, prec, msg);
  if (vst != VKLB_OK) return vst;
  pl->basis = resolve_basis(o.basis, prec, grid->dim);
  if (pl->basis < 0) {
    *msg = "basis must be 0..3 (3, compensated, needs FP32)";
    return VKLB_ERR_ARG;
  }
  layout_of(sys, lat, grid, prec, pl->basis, &pl->L);
  pl->grid = *grid;
  if (grid->dim == 1) pl->grid.n[1] = 1;
  pl->bc[0] = bc[0];
  pl->bc[1] = grid->dim == 2 ? bc[1] : bc[0];
  pl->sys = *sys;
  pl->lambda = *lambda;
  pl->eq = *eq;
  pl->omega = omega;
  int width = o.strip_width;
  if (grid->dim == 1 ? (width != 256 && width != 512) : (width != 64 && width != 128 && width != 256))
    width = default_width(grid->dim, grid->n[0]);
  pl->width = width;
  pl->K = pick_launchers(sys->kind, grid->dim, prec == VKLB_FP32 ? 1 : 0, pl->basis, width);
  int band = o.band_rows;
  if (band < 1) band = default_band(grid, width);
  if (band > max_band(sys->kind, grid->dim, pl->basis)) band = max_band(sys->kind, grid->dim, pl->basis);
  pl->band = band;
  int halo = o.halo_rows;
  if (halo < 1 || halo > 32) halo = default_halo(sys->kind);
  pl->halo = halo;
  // Grids of many workgroups: every workgroup reading every partial costs
  // nblocks^2 loads per step (10^12 at a million workgroups), so above the
  // threshold each launch's partials are folded into one entry instead.
  const int fold = o.fold_partials == 0 ? kFoldAbove : o.fold_partials;
  pl->nred_one = fold > 0 && step_grid_of(&pl->grid, width, band) > fold;
  // small 1D grids: whole step sequences in one workgroup (bitwise the same)
  pl->wg_cells = pl->wg_lanes = 0;
  if (grid->dim == 1 && o.small_grid >= 0 && pl->K.run_wg && grid->n[0] <= pl->K.wg_max_cells) {
    const long long n = grid->n[0];
    // 512 lanes measured fastest for every N <= 1024 (1 or 2 cells per lane);
    // MHD holds too many registers for more than 256 lanes of one cell each
    int lanes = o.small_grid;
    if (lanes != 256 && lanes != 512 && lanes != 1024) lanes = 512;
    if (sys->kind == VKLB_MHD_GLM) lanes = 256;
    int cells = int((n + lanes - 1) / lanes);
    if (cells == 3) cells = 4;
    pl->wg_lanes = lanes;
    pl->wg_cells = cells;
  }
  return VKLB_OK;
}

}  // namespace

extern "C" {

size_t vklb_workspace_bytes(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid, vklb_precision prec) {
  Layout L;
  // the largest stored basis of the precision, so any basis fits
  return layout_of(sys, lat, grid, prec, prec == VKLB_FP32 ? 2 : 0, &L) ? L.total : 0;
}

vklb_status vklb_create(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid, const vklb_speed* lambda,
                        double omega, const vklb_bc bc[2], const vklb_equilibrium* eq, vklb_precision prec,
                        const vklb_options* opt, void* device_buf, size_t buf_bytes, void* hip_stream,
                        vklb_solver** out) {
  if (!out) return fail(nullptr, VKLB_ERR_ARG, "out is NULL");
  *out = nullptr;
  vklb_options o;
  if (opt) o = *opt;
  else memset(&o, 0, sizeof o);
  Plan pl;
  const char* msg = "";
  vklb_status vst = plan_solve(sys, lat, grid, lambda, omega, bc, eq, prec, o, &pl, &msg);
  if (vst != VKLB_OK) return fail(nullptr, vst, msg);
  if (device_buf && buf_bytes < pl.L.total) return fail(nullptr, VKLB_ERR_OOM, "device buffer smaller than vklb_workspace_bytes");
  if (device_buf && (reinterpret_cast<uintptr_t>(device_buf) % kAlign) != 0)
    return fail(nullptr, VKLB_ERR_ARG, "device buffer must be 256-byte aligned");

  vklb_solver* s = new vklb_solver();
  s->sys = *sys;
  s->lat = lat;
  s->grid = pl.grid;
  s->speed = *lambda;
  s->omega = omega;
  s->bc[0] = pl.bc[0];
  s->bc[1] = pl.bc[1];
  s->eq = *eq;
  s->prec = prec;
  s->opt = o;
  s->L = pl.L;
  s->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (lambda->mode == VKLB_XI_CFL && eq->set == VKLB_EQ_WEIGHTED && eq->c > 0.5 * (1.0 - lambda->nu))
    s->err = "note: c exceeds (1 - nu)/2, the monotonicity bound of Sec. 4.2";
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) {
    delete s;
    return fail(nullptr, VKLB_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  if (device_buf) {
    s->buf = static_cast<char*>(device_buf);
  } else {
    e = hipMalloc(&s->buf, pl.L.total);
    if (e != hipSuccess) {
      delete s;
      return fail(nullptr, VKLB_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    s->own_buf = true;
  }
  s->K = pl.K;
  s->basis = pl.basis;
  s->chunk = o.graph_chunk == 0 ? 512 : o.graph_chunk;  // 512: 1-2% per 1D step over 64
  if (s->chunk > 0) s->chunk = (s->chunk + 1) / 2 * 2;  // even: replays start on parity 0
  s->sd = pl.bind(s->buf);
  s->step_grid = s->sd.nblocks;
  s->wg_lanes = pl.wg_lanes;
  s->wg_cells = pl.wg_cells;
  *out = s;
  return VKLB_OK;
}

vklb_status vklb_set_end(vklb_solver* s, double T, int64_t max_steps) {
  if (!s) return VKLB_ERR_ARG;
  if (isnan(T)) return fail(s, VKLB_ERR_ARG, "T is NaN");
  s->T = T;
  s->max_steps = max_steps < 0 ? (1ll << 62) : max_steps;
  if (s->inited) {
    // after init the device copy is updated too, in stream order: steps
    // already queued keep the old end condition, later ones see the new one.
    // The finished flag of the scalars the next launch reads is cleared, so a
    // solve that had reached its old end goes on (a non-physical state still
    // stops it: that comes from the error word).
    HIPCHK(s, hipSetDevice(s->device));
    char* st = s->buf + s->L.state_off;
    const int zero = 0;
    const size_t done_off = offsetof(DevState, S) + size_t(s->launches & 1) * sizeof(Scal) + offsetof(Scal, done);
    HIPCHK(s, hipMemcpyAsync(st + offsetof(DevState, T), &s->T, sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(st + offsetof(DevState, max_steps), &s->max_steps, sizeof(long long),
                             hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(st + done_off, &zero, sizeof(int), hipMemcpyHostToDevice, s->stream));
    // launches that found the solve finished did not step, so the step
    // parity of the coming launches is read back
    long long n = 0;
    const size_t n_off = offsetof(DevState, S) + size_t(s->launches & 1) * sizeof(Scal) + offsetof(Scal, n);
    HIPCHK(s, hipMemcpyAsync(&n, st + n_off, sizeof(long long), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return set_npar(s, int((n ^ s->launches) & 1));
  }
  return VKLB_OK;
}

static vklb_status init_from(vklb_solver* s, const double* U0, hipMemcpyKind kind) {
  if (!s || !U0) return VKLB_ERR_ARG;
  HIPCHK(s, hipSetDevice(s->device));
  const long long cells = (long long)s->sd.nx * s->sd.ny;
  HIPCHK(s, hipMemcpyAsync(const_cast<double*>(s->sd.stage), U0, size_t(s->L.p) * cells * 8, kind, s->stream));
  vklb_status st = reset_state(s, 0.0, 0, 0);
  if (st != VKLB_OK) return st;
  SolveDesc d = s->sd;
  d.par = 0;
  HIPCHK(s, s->K.init_reduce(d, d.nblocks, s->stream));
  st = fold_partials(s, s->stream, 0);
  if (st != VKLB_OK) return st;
  HIPCHK(s, s->K.init_feq(d, grid_for_cells(cells), s->stream));
  s->inited = true;
  return VKLB_OK;
}

vklb_status vklb_init(vklb_solver* s, const double* U0_host) { return init_from(s, U0_host, hipMemcpyHostToDevice); }

vklb_status vklb_init_device(vklb_solver* s, const double* U0_device) {
  return init_from(s, U0_device, hipMemcpyDeviceToDevice);
}

vklb_status vklb_step(vklb_solver* s, int64_t n) {
  if (!s) return VKLB_ERR_ARG;
  if (!s->inited) return fail(s, VKLB_ERR_STATE, "vklb_step before vklb_init");
  if (n < 0) return fail(s, VKLB_ERR_ARG, "n < 0");
  if (n == 0) return VKLB_OK;
  HIPCHK(s, hipSetDevice(s->device));
  if (!s->ev0) {
    HIPCHK(s, hipEventCreate(&s->ev0));
    HIPCHK(s, hipEventCreate(&s->ev1));
  }
  HIPCHK(s, hipEventRecord(s->ev0, s->stream));
  long long rem = n;
  vklb_status st;
  if (s->wg_cells > 0) {
    HIPCHK(s, enqueue_wg_steps(s->sd, s->K, s->wg_cells, s->wg_lanes, rem, s->launches, s->stream));
    s->launches += rem;
    rem = 0;
  }
  if (s->chunk > 0 && rem >= s->chunk + 1) {
    st = ensure_graph(s);
    if (st != VKLB_OK) return st;
    if (s->launches & 1) {  // the graph starts on parity 0
      st = launch_steps(s, s->stream, 1, s->launches);
      if (st != VKLB_OK) return st;
      s->launches += 1;
      rem -= 1;
    }
    while (rem >= s->chunk) {
      HIPCHK(s, hipGraphLaunch(s->gexec, s->stream));
      rem -= s->chunk;
      s->launches += s->chunk;
    }
  }
  st = launch_steps(s, s->stream, rem, s->launches);
  if (st != VKLB_OK) return st;
  s->launches += rem;
  HIPCHK(s, hipEventRecord(s->ev1, s->stream));
  s->timed = true;
  return VKLB_OK;
}

vklb_status vklb_last_step_ms(vklb_solver* s, double* ms) {
  if (!s || !ms) return VKLB_ERR_ARG;
  if (!s->timed) return fail(s, VKLB_ERR_STATE, "no timed vklb_step yet");
  HIPCHK(s, hipEventSynchronize(s->ev1));
  float f = 0.f;
  HIPCHK(s, hipEventElapsedTime(&f, s->ev0, s->ev1));
  *ms = f;
  return VKLB_OK;
}

vklb_status vklb_moments(vklb_solver* s, double* U_host, double* t, int64_t* steps) {
  if (!s) return VKLB_ERR_ARG;
  if (!s->inited) return fail(s, VKLB_ERR_STATE, "vklb_moments before vklb_init");
  HIPCHK(s, hipSetDevice(s->device));
  const long long cells = (long long)s->sd.nx * s->sd.ny;
  if (U_host) {
    SolveDesc d = s->sd;
    d.par = int(s->launches & 1);
    HIPCHK(s, s->K.moments(d, grid_for_cells(cells), s->stream));
    HIPCHK(s, hipMemcpyAsync(U_host, s->sd.stage, size_t(s->L.p) * cells * 8, hipMemcpyDeviceToHost, s->stream));
  }
  HostView v;
  vklb_status st = read_view(s, &v);
  if (st != VKLB_OK) return st;
  if (t) *t = v.S.t;
  if (steps) *steps = v.S.n;
  return check_err(s, v);
}

vklb_status vklb_progress(vklb_solver* s, double* t, int64_t* steps, int* done) {
  if (!s) return VKLB_ERR_ARG;
  if (!s->inited) return fail(s, VKLB_ERR_STATE, "vklb_progress before vklb_init");
  HIPCHK(s, hipSetDevice(s->device));
  HostView v;
  vklb_status st = read_view(s, &v);
  if (st != VKLB_OK) return st;
  if (t) *t = v.S.t;
  if (steps) *steps = v.S.n;
  if (done) *done = v.step.done;
  return check_err(s, v);
}

vklb_status vklb_diagnostics(vklb_solver* s, vklb_diag* dg) {
  if (!s || !dg) return VKLB_ERR_ARG;
  if (!s->inited) return fail(s, VKLB_ERR_STATE, "vklb_diagnostics before vklb_init");
  HIPCHK(s, hipSetDevice(s->device));
  memset(dg, 0, sizeof *dg);
  const long long cells = (long long)s->sd.nx * s->sd.ny;
  const int p = s->L.p;
  SolveDesc dm = s->sd;
  dm.par = int(s->launches & 1);
  HIPCHK(s, s->K.moments(dm, grid_for_cells(cells), s->stream));
  const int nb = int(std::min<long long>(kDiagBlocks, (cells + 255) / 256));
  double* dpart = reinterpret_cast<double*>(s->buf + s->L.diag_off);
  hipLaunchKernelGGL(k_totals_partial, dim3(nb), dim3(256), 0, s->stream, s->sd.stage, cells, p, dpart);
  HIPCHK(s, hipGetLastError());
  double* tot_dev = dpart + kDiagBlocks * 9 * 2;
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, s->stream, dpart, nb, p, tot_dev);
  HIPCHK(s, hipGetLastError());
  unsigned long long* divb = reinterpret_cast<unsigned long long*>(tot_dev + 9);
  HIPCHK(s, hipMemsetAsync(divb, 0, 8, s->stream));
  if (s->sys.kind == VKLB_MHD_GLM && s->grid.dim == 2) {
    hipLaunchKernelGGL(k_divb, dim3(grid_for_cells(cells)), dim3(256), 0, s->stream, s->sd.stage, s->sd.nx, s->sd.ny,
                       s->sd.dx, s->sd.bcx, s->sd.bcy, divb);
    HIPCHK(s, hipGetLastError());
  }
  double host[10];
  HIPCHK(s, hipMemcpyAsync(host, tot_dev, sizeof host, hipMemcpyDeviceToHost, s->stream));
  HostView v;
  vklb_status st = read_view(s, &v);
  if (st != VKLB_OK) return st;
  for (int v = 0; v < p; ++v) dg->totals[v] = host[v];
  unsigned long long db;
  memcpy(&db, &host[9], 8);
  double dbv;
  memcpy(&dbv, &db, 8);
  dg->max_div_b = dbv;
  dg->t = v.S.t;
  dg->steps = v.S.n;
  dg->xi = v.step.xi;
  dg->lambda_max = v.step.lam;
  dg->ch = v.step.ch;
  dg->done = v.step.done;
  dg->nonphysical = v.err ? 1 : 0;
  dg->fail_step = v.err_step;
  dg->fail_cell = v.err_cell;
  return VKLB_OK;
}

size_t vklb_state_bytes(const vklb_solver* s) {
  if (!s) return 0;
  return size_t(s->L.slots) * s->L.p * size_t(s->L.stride) * s->L.elem + sizeof(CkptTrailer);
}

vklb_status vklb_get_state(vklb_solver* s, void* host, double* t, int64_t* steps) {
  if (!s || !host) return VKLB_ERR_ARG;
  if (!s->inited) return fail(s, VKLB_ERR_STATE, "vklb_get_state before vklb_init");
  HIPCHK(s, hipSetDevice(s->device));
  HostView v;
  vklb_status st = read_view(s, &v);
  if (st != VKLB_OK) return st;
  const size_t pop = vklb_state_bytes(s) - sizeof(CkptTrailer);
  const char* src = (v.S.n & 1) ? static_cast<const char*>(s->sd.fb) : static_cast<const char*>(s->sd.fa);
  HIPCHK(s, hipMemcpyAsync(host, src, pop, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  if (s->sd.nfull > 1) {  // rows to grid order
    std::vector<char> dev(static_cast<const char*>(host), static_cast<const char*>(host) + pop);
    reorder_rows(dev.data(), static_cast<char*>(host), s->sd, s->L, s->sys.kind == VKLB_MHD_GLM, true);
  }
  CkptTrailer tr = make_trailer(s);
  tr.t = v.S.t;
  tr.n = v.S.n;
  tr.lam7 = v.lam7;
  tr.cfm = v.cfm;
  tr.done = v.S.done;
  memcpy(static_cast<char*>(host) + pop, &tr, sizeof tr);
  if (t) *t = v.S.t;
  if (steps) *steps = v.S.n;
  return check_err(s, v);
}

vklb_status vklb_set_state(vklb_solver* s, const void* host) {
  if (!s || !host) return VKLB_ERR_ARG;
  HIPCHK(s, hipSetDevice(s->device));
  const size_t pop = vklb_state_bytes(s) - sizeof(CkptTrailer);
  CkptTrailer tr;
  memcpy(&tr, static_cast<const char*>(host) + pop, sizeof tr);
  const CkptTrailer me = make_trailer(s);
  if (tr.magic != me.magic || tr.kind != me.kind || tr.dim != me.dim || tr.prec != me.prec ||
      tr.basis != me.basis || tr.nx != me.nx || tr.ny != me.ny || tr.n < 0)
    return fail(s, VKLB_ERR_ARG, "checkpoint does not belong to a solver of this shape");
  char* dst = (tr.n & 1) ? static_cast<char*>(s->sd.fb) : static_cast<char*>(s->sd.fa);
  if (s->sd.nfull > 1) {  // rows to the device's order
    std::vector<char> dev(pop, 0);
    reorder_rows(static_cast<const char*>(host), dev.data(), s->sd, s->L, s->sys.kind == VKLB_MHD_GLM, false);
    HIPCHK(s, hipMemcpyAsync(dst, dev.data(), pop, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
  } else {
    HIPCHK(s, hipMemcpyAsync(dst, host, pop, hipMemcpyHostToDevice, s->stream));
  }
  vklb_status st = reset_state(s, tr.t, tr.n, tr.done);
  if (st != VKLB_OK) return st;
  // The saved maxima stand in for the partials of parity 0 (the max is exact).
  std::vector<double> part(size_t(2) * s->sd.nblocks, 0.0);
  part[0] = tr.lam7;
  part[s->sd.nblocks] = tr.cfm;
  HIPCHK(s, hipMemcpyAsync(s->sd.part, part.data(), part.size() * 8, hipMemcpyHostToDevice, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  s->inited = true;
  return VKLB_OK;
}

}  // extern "C"

// vklb_tune over the shapes of a single solve, or (pool_2d) over the band and
// halo heights of the serving pool's batched 2D kernel, whose strips are 128
// columns wide.
static vklb_status tune_impl(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid, const vklb_speed* lambda,
                             double omega, const vklb_bc bc[2], const vklb_equilibrium* eq, vklb_precision prec,
                             const vklb_options* base, const double* U0_host, int steps, void* hip_stream,
                             bool pool_2d, vklb_options* best, double* best_step_us) {
  if (!U0_host || !best || steps < 1 || steps > 100000) return fail(nullptr, VKLB_ERR_ARG, "vklb_tune: bad arguments");
  const char* msg = "";
  vklb_status vst = validate(sys, lat, grid, lambda, omega, bc, eq, prec, &msg);
  if (vst != VKLB_OK) return fail(nullptr, vst, msg);
  if (pool_2d && grid->dim != 2) return fail(nullptr, VKLB_ERR_ARG, "vklb_tune: the pool's tuned shapes are 2D");
  vklb_options b0;
  if (base) b0 = *base;
  else memset(&b0, 0, sizeof b0);
  // candidate tile shapes
  std::vector<vklb_options> cand;
  if (pool_2d) {
    const long long ny = grid->n[1];
    for (int band : {4, 8, 16, 32, 64}) {
      if (band > 4 && band / 2 >= ny) continue;
      for (int halo : {2, 8, 16, 32}) {
        if (halo > band) continue;
        vklb_options o = b0;
        o.strip_width = 128;
        o.band_rows = band;
        o.halo_rows = halo;
        cand.push_back(o);
      }
    }
  } else if (grid->dim == 1) {
    for (int w : {256, 512}) {
      vklb_options o = b0;
      o.strip_width = w;
      cand.push_back(o);
    }
    // grids that run in one workgroup: its lane count (MHD has one shape)
    if (grid->n[0] <= 1024 && sys->kind != VKLB_MHD_GLM && b0.small_grid >= 0) {
      cand.clear();
      for (int lanes : {256, 512, 1024}) {
        vklb_options o = b0;
        o.small_grid = lanes;
        cand.push_back(o);
      }
    }
  } else {
    const long long nx = grid->n[0], ny = grid->n[1];
    for (int w : {64, 128, 256}) {
      if (w > 64 && (nx + w - 1) / w * w - nx >= w / 2) continue;  // mostly idle lanes
      // the default rule's band too, where it is taller than these (large grids)
      std::vector<int> bands = {4, 8, 16, 32, 64};
      const int rule = std::min(default_band(grid, w), max_band(sys->kind, 2, resolve_basis(b0.basis, prec, 2)));
      if (rule > 64) bands.push_back(rule);
      for (int band : bands) {
        if (band > 4 && band / 2 >= ny) continue;
        for (int halo : {2, 8, 16, 32}) {
          if (halo > band) continue;
          vklb_options o = b0;
          o.strip_width = w;
          o.band_rows = band;
          o.halo_rows = halo;
          cand.push_back(o);
        }
      }
    }
  }
  const size_t bytes = vklb_workspace_bytes(sys, lat, grid, prec);
  void* buf = nullptr;
  hipError_t e = hipMalloc(&buf, bytes);
  if (e != hipSuccess) return fail(nullptr, VKLB_ERR_OOM, std::string("vklb_tune: hipMalloc: ") + hipGetErrorString(e));
  double best_us = INFINITY;
  vklb_status last = VKLB_OK;
  for (const vklb_options& o : cand) {
    vklb_solver* s = nullptr;
    vklb_status st = vklb_create(sys, lat, grid, lambda, omega, bc, eq, prec, &o, buf, bytes, hip_stream, &s);
    if (st == VKLB_OK) st = vklb_set_end(s, INFINITY, -1);
    if (st == VKLB_OK) st = vklb_init(s, U0_host);
    if (st == VKLB_OK) st = vklb_step(s, std::min(steps, 8));  // warm-up (and graph capture)
    if (st == VKLB_OK) st = vklb_step(s, steps);
    double ms = 0.0;
    if (st == VKLB_OK) st = vklb_last_step_ms(s, &ms);
    int done = 0;
    if (st == VKLB_OK) st = vklb_progress(s, nullptr, nullptr, &done);  // non-physical -> error
    if (st == VKLB_OK && !done && ms > 0.0) {
      const double us = 1e3 * ms / steps;
      if (us < best_us) {
        best_us = us;
        *best = o;
      }
    } else if (st != VKLB_OK) {
      last = st;
    }
    vklb_destroy(s);
  }
  (void)hipFree(buf);
  if (!(best_us < INFINITY))
    return fail(nullptr, last != VKLB_OK ? last : VKLB_ERR_STATE, "vklb_tune: no candidate ran");
  if (best_step_us) *best_step_us = best_us;
  return VKLB_OK;
}

namespace vklb {
vklb_status tune_pool_shape(const vklb_request* r, vklb_precision prec, int steps, void* hip_stream, int* band,
                            int* halo, double* step_us) {
  vklb_options best;
  memset(&best, 0, sizeof best);
  vklb_status st = tune_impl(&r->sys, r->lat, &r->grid, &r->lambda, r->omega, r->bc, &r->eq, prec, nullptr, r->U0,
                             steps, hip_stream, true, &best, step_us);
  if (st != VKLB_OK) return st;
  *band = best.band_rows;
  *halo = best.halo_rows;
  return VKLB_OK;
}
}  // namespace vklb

extern "C" {

vklb_status vklb_tune(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid, const vklb_speed* lambda,
                      double omega, const vklb_bc bc[2], const vklb_equilibrium* eq, vklb_precision prec,
                      const vklb_options* base, const double* U0_host, int steps, void* hip_stream,
                      vklb_options* best, double* best_step_us) {
  return tune_impl(sys, lat, grid, lambda, omega, bc, eq, prec, base, U0_host, steps, hip_stream, false, best,
                   best_step_us);
}

void vklb_destroy(vklb_solver* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->own_buf && s->buf) (void)hipFree(s->buf);
  delete s;
}

// Device address of the static workspace on the current device, found once
// per device (each GPU holds its own copy of the array).
static vklb_status static_workspace(char** out) {
  static std::mutex mu;
  static char* ptr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_create_error("vklb_run_static: hipGetDevice failed");
    return VKLB_ERR_DEVICE;
  }
  if (dev < 0 || dev >= 64) {
    set_create_error("vklb_run_static: device index above 63");
    return VKLB_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_create_error("vklb_run_static: hipGetSymbolAddress of the static workspace failed");
      return VKLB_ERR_DEVICE;
    }
    ptr[dev] = static_cast<char*>(p);
  }
  *out = ptr[dev];
  return VKLB_OK;
}

vklb_status vklb_run_static(const vklb_system* sys, vklb_lattice lat, const vklb_grid* grid,
                            const vklb_speed* lambda, double omega, const vklb_bc bc[2], const vklb_equilibrium* eq,
                            vklb_precision prec, double T, int64_t n_steps, const double* U0_device,
                            double* U_device, vklb_run_info* info_device, void* hip_stream) {
  if (!U0_device || !U_device) {
    set_create_error("vklb_run_static: U0_device and U_device must not be NULL");
    return VKLB_ERR_ARG;
  }
  if (n_steps < 0) {
    set_create_error("vklb_run_static: n_steps < 0");
    return VKLB_ERR_ARG;
  }
  if (isnan(T)) {
    set_create_error("vklb_run_static: T is NaN");
    return VKLB_ERR_ARG;
  }
  vklb_options o;
  memset(&o, 0, sizeof o);
  Plan pl;
  const char* msg = "";
  vklb_status st = plan_solve(sys, lat, grid, lambda, omega, bc, eq, prec, o, &pl, &msg);
  if (st != VKLB_OK) {
    set_create_error(msg);
    return st;
  }
  if (pl.L.total > size_t(VKLB_STATIC_BYTES)) {
    char m[200];
    snprintf(m, sizeof m, "vklb_run_static: the solve needs %zu bytes of workspace, above the static %zu",
             pl.L.total, size_t(VKLB_STATIC_BYTES));
    set_create_error(m);
    return VKLB_ERR_OOM;
  }
  char* ws = nullptr;
  st = static_workspace(&ws);
  if (st != VKLB_OK) return st;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  SolveDesc sd = pl.bind(ws);
  const long long cells = (long long)sd.nx * sd.ny;
  // vklb_init: scalars, xi^0 / c_h^0 from U0, f = f^eq(U0); U0 is read in
  // place, so the staging area is not used.
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(k_static_reset, dim3(1), dim3(64), 0, stream, sd.st, T, n_steps);
  e = hipGetLastError();
  SolveDesc d0 = sd;
  d0.stage = U0_device;
  d0.par = 0;
  if (e == hipSuccess) e = pl.K.init_reduce(d0, d0.nblocks, stream);
  if (e == hipSuccess) e = launch_fold(d0, 0, stream);
  if (e == hipSuccess) e = pl.K.init_feq(d0, grid_for_cells(cells), stream);
  // vklb_step(n_steps): the end condition turns the launches past it into no-ops
  if (e == hipSuccess) {
    e = pl.wg_cells > 0 ? enqueue_wg_steps(sd, pl.K, pl.wg_cells, pl.wg_lanes, n_steps, 0, stream)
                        : enqueue_steps(sd, pl.K, n_steps, 0, stream);
  }
  // vklb_moments, written to the caller's device array
  SolveDesc dm = sd;
  dm.stage = U_device;
  dm.par = int(n_steps & 1);
  if (e == hipSuccess) e = pl.K.moments(dm, grid_for_cells(cells), stream);
  if (e == hipSuccess && info_device) {
    hipLaunchKernelGGL(k_static_info, dim3(1), dim3(64), 0, stream, sd.st, int(n_steps & 1), info_device);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    char m[200];
    snprintf(m, sizeof m, "vklb_run_static: launch failed: %s", hipGetErrorString(e));
    set_create_error(m);
    return VKLB_ERR_DEVICE;
  }
  return VKLB_OK;
}

vklb_status vklb_stream_copy(void* dst, const void* src, size_t bytes, int non_temporal, void* hip_stream) {
  if (!dst || !src || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16) {
    set_create_error("vklb_stream_copy: NULL pointer, or size or address not a multiple of 16 bytes");
    return VKLB_ERR_ARG;
  }
  const long long n16 = (long long)(bytes / 16);
  if (n16 == 0) return VKLB_OK;
  const long long blocks = (n16 + 255) / 256;
  if (blocks > 0x7fffffffll) {
    set_create_error("vklb_stream_copy: more than 2^31 workgroups of 4 KiB");
    return VKLB_ERR_ARG;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if (non_temporal)
    hipLaunchKernelGGL(k_stream_copy<true>, dim3(unsigned(blocks)), dim3(256), 0, st, static_cast<const v4f*>(src),
                       static_cast<v4f*>(dst), n16);
  else
    hipLaunchKernelGGL(k_stream_copy<false>, dim3(unsigned(blocks)), dim3(256), 0, st, static_cast<const v4f*>(src),
                       static_cast<v4f*>(dst), n16);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    char m[160];
    snprintf(m, sizeof m, "vklb_stream_copy: launch failed: %s", hipGetErrorString(e));
    set_create_error(m);
    return VKLB_ERR_DEVICE;
  }
  return VKLB_OK;
}

const char* vklb_status_str(vklb_status st) {
  switch (st) {
    case VKLB_OK: return "ok";
    case VKLB_ERR_ARG: return "invalid argument";
    case VKLB_ERR_UNSUPPORTED: return "unsupported";
    case VKLB_ERR_OOM: return "out of memory";
    case VKLB_ERR_DEVICE: return "device error";
    case VKLB_ERR_NONPHYSICAL: return "non-physical state";
    case VKLB_ERR_STATE: return "call out of order";
  }
  return "unknown status";
}

const char* vklb_last_error(const vklb_solver* s) {
  if (s) return s->err.c_str();
  std::lock_guard<std::mutex> lk(g_err_mu);
  return g_create_error;
}

}  // extern "C"
