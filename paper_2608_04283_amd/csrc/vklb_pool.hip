// Serving pool (include/vklb.h, vklb_pool_*): many solves of different
// systems and sizes resident in one device arena, advanced together.
//
// Memory: one hipMalloc'd arena; each admitted solve gets a first-fit block
// holding its own workspace (same layout as a single solver). Admission is in
// submission order and stops at the first request that does not fit, so large
// requests are not starved by later small ones.
// Execution: a round is one batched launch per system class over the work
// list of (solve slot, tile) items of every resident solve of that class.
// While a class's resident set stays the same from one vklb_pool_run to the
// next, its chunk of rounds is captured once into a HIP graph and replayed;
// an admission or completion in the class drops its graph.
// Tile shapes: 1D tiles are 256 lanes; 2D strips are 128 columns, with band
// and halo heights per (system, size class) from vklb_pool_autotune when it
// was called in the process, else the single-solve defaults.
// All resident solves share the round parity; a solve admitted before round
// r is initialized into parity r & 1. A class's round depends only on that
// class's previous round, so each class runs on a stream of its own and small
// 1D rounds overlap the large 2D ones; the caller's stream (admission,
// initialization, status, harvest) and the class streams are joined by events
// at both ends of vklb_pool_run.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <array>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "vklb_host.hpp"

using namespace vklb;

namespace {

constexpr int kClasses = 8;   // (system kind) x (dimension)
constexpr int kMaxSlots = 4096;

inline int class_of(int kind, int dim) { return kind * 2 + (dim - 1); }

// First-fit allocator over [0, size) with coalescing of freed neighbours.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
    used_ = 0;
    peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

struct Req {
  uint64_t ticket = 0, tag = 0;
  vklb_system sys;
  vklb_lattice lat;
  vklb_grid grid;
  vklb_speed speed;
  double omega;
  vklb_bc bc[2];
  vklb_equilibrium eq;
  double T;
  long long max_steps;
  std::vector<double> U0;
  double* U_out = nullptr;
  Layout L;
  int cls = 0;
  int band = 32;
  int halo = 32;
  size_t off = 0;
  SolveDesc sd;
  int slot = -1;
};

struct SlotStatus {
  double t;
  long long n;
  int done;
  int pad;
  unsigned long long err_word;
};

__global__ void __launch_bounds__(256) k_gather_status(const SolveDesc* __restrict__ descs,
                                                       const int* __restrict__ slots, int nslots, int par,
                                                       SlotStatus* __restrict__ out) {
  const int i = blockIdx.x;
  if (i >= nslots) return;
  SolveDesc sd = descs[slots[i]];
  sd.par = par;
  __shared__ double red[10];
  const Step S = begin_step(sd, red);
  if (threadIdx.x == 0) {
    SlotStatus r;
    r.t = S.t;
    r.n = S.n;
    r.done = S.done;
    r.pad = 0;
    r.err_word = sd.st->err_word;
    out[i] = r;
  }
}

double now_s() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

}  // namespace

struct vklb_pool {
  char* base = nullptr;
  size_t budget = 0;
  Arena arena;
  vklb_precision prec = VKLB_FP32;
  int basis[3] = {0, 0, 0};  // stored basis per dimension (index 1, 2)
  hipStream_t stream = nullptr;
  hipStream_t cls_stream[kClasses] = {};   // default priority, non-blocking
  hipEvent_t ev_main = nullptr;
  hipEvent_t ev_cls[kClasses] = {};
  int device = 0;
  uint64_t next_ticket = 1;
  std::deque<Req*> queue;
  std::vector<Req*> slots;          // kMaxSlots entries
  Launchers cls_launch[kClasses];
  SolveDesc* d_descs = nullptr;
  WorkItem* d_work[kClasses] = {};
  int* d_nwork = nullptr;           // kClasses counters
  int cap_work[kClasses] = {};
  int nwork[kClasses] = {};
  int* d_slot_list = nullptr;
  SlotStatus* d_status = nullptr;
  SlotStatus* h_status = nullptr;   // pinned
  long long round = 0;
  bool dirty = true;                // work lists need uploading
  bool changed[kClasses] = {};      // the class's resident set changed since its last rounds
  hipGraph_t graph[kClasses] = {};  // the class's captured chunk of rounds (stable resident set)
  hipGraphExec_t gexec[kClasses] = {};
  int graph_rounds[kClasses] = {};
  int graph_par[kClasses] = {};
  int stable_calls[kClasses] = {};  // consecutive vklb_pool_run calls with an unchanged resident set
  long long graph_launches = 0, graph_captures = 0;

  std::deque<vklb_completion> done;
  vklb_pool_stats stats;
  std::string err;
};

namespace {

vklb_status pfail(vklb_pool* p, vklb_status st, const std::string& m) {
  if (p) p->err = m;
  return st;
}

#define PCHK(p, call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return pfail((p), VKLB_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// Half-octave size class of a 2D grid side: round(2 log2 n).
int size_class(long long n) { return int(lround(2.0 * log2(double(n > 0 ? n : 1)))); }

// Tuned 2D shapes, kept for the process: (device, precision, kind, size
// class) -> (band, halo).
std::mutex g_tiles_mu;
std::map<std::array<int, 4>, std::pair<int, int>> g_tiles;

// Band and halo heights for a 2D solve of this kind and side: the tuned entry
// of its size class, else the nearest tuned class of the kind, else (no tuned
// entry) *band and *halo as given.
void pick_shape(const vklb_pool* p, int kind, long long n, int* band, int* halo) {
  const int want = size_class(n);
  int bestd = 1 << 30;
  std::lock_guard<std::mutex> lk(g_tiles_mu);
  for (const auto& kv : g_tiles) {
    if (kv.first[0] != p->device || kv.first[1] != int(p->prec) || kv.first[2] != kind) continue;
    const int d = abs(kv.first[3] - want);
    if (d < bestd) {
      bestd = d;
      *band = kv.second.first;
      *halo = kv.second.second;
    }
  }
}

void drop_class_graph(vklb_pool* p, int c) {
  if (p->gexec[c]) (void)hipGraphExecDestroy(p->gexec[c]);
  if (p->graph[c]) (void)hipGraphDestroy(p->graph[c]);
  p->gexec[c] = nullptr;
  p->graph[c] = nullptr;
}

vklb_status admit(vklb_pool* p) {
  std::vector<Req*> admitted;
  std::vector<DevState> heads;
  heads.reserve(p->queue.size());
  while (!p->queue.empty()) {
    Req* r = p->queue.front();
    int slot = -1;
    for (int i = 0; i < kMaxSlots; ++i)
      if (!p->slots[i]) { slot = i; break; }
    if (slot < 0) break;
    size_t off;
    if (!p->arena.alloc(r->L.total, &off)) break;
    p->queue.pop_front();
    r->off = off;
    r->slot = slot;
    p->slots[slot] = r;
    const int width = r->grid.dim == 1 ? 256 : 128;  // the batched kernels' tile widths
    r->sd = make_desc(p->base + off, r->L, &r->sys, &r->grid, &r->speed, r->omega, r->bc, &r->eq, width, r->band,
                      r->halo);
    r->sd.npar = int(p->round & 1);  // step 0 runs at the parity of the next round
    if (r->sd.nblocks > kFoldAbove) r->sd.nred = 1;  // as a single solve: partials folded after each round
    // initialization into the parity of the next round
    const long long cells = (long long)r->sd.nx * r->sd.ny;
    PCHK(p, hipMemcpyAsync(const_cast<double*>(r->sd.stage), r->U0.data(), r->U0.size() * 8, hipMemcpyHostToDevice,
                           p->stream));
    heads.emplace_back();
    DevState& h = heads.back();
    memset(&h, 0, sizeof h);
    h.T = r->T;
    h.max_steps = r->max_steps;
    h.err_word = ~0ull;
    PCHK(p, hipMemcpyAsync(r->sd.st, &h, sizeof h, hipMemcpyHostToDevice, p->stream));
    admitted.push_back(r);
    SolveDesc d = r->sd;
    d.par = int(p->round & 1);
    const Launchers& K = p->cls_launch[r->cls];
    PCHK(p, K.init_reduce(d, d.nblocks, p->stream));
    PCHK(p, launch_fold(d, d.par, p->stream));
    PCHK(p, K.init_feq(d, grid_for_cells(cells), p->stream));
    p->dirty = true;
    p->changed[r->cls] = true;
    p->stats.admitted++;
  }
  if (!admitted.empty()) {
    // the host sources of the copies above must outlive them
    PCHK(p, hipStreamSynchronize(p->stream));
    for (Req* r : admitted) std::vector<double>().swap(r->U0);
  }
  return VKLB_OK;
}

vklb_status upload_lists(vklb_pool* p) {
  if (!p->dirty) return VKLB_OK;
  std::vector<SolveDesc> descs(kMaxSlots);
  std::vector<WorkItem> work[kClasses];
  for (int i = 0; i < kMaxSlots; ++i) {
    Req* r = p->slots[i];
    if (!r) continue;
    descs[i] = r->sd;
    for (int tl = 0; tl < r->sd.nblocks; ++tl) work[r->cls].push_back(WorkItem{i, tl});
  }
  int highest = -1;
  for (int i = 0; i < kMaxSlots; ++i)
    if (p->slots[i]) highest = i;
  if (highest >= 0)
    PCHK(p, hipMemcpyAsync(p->d_descs, descs.data(), sizeof(SolveDesc) * (highest + 1), hipMemcpyHostToDevice,
                           p->stream));
  int counts[kClasses];
  for (int c = 0; c < kClasses; ++c) {
    counts[c] = int(work[c].size());
    p->nwork[c] = counts[c];
    if (counts[c] > p->cap_work[c]) {
      PCHK(p, hipStreamSynchronize(p->stream));
      if (p->d_work[c]) PCHK(p, hipFree(p->d_work[c]));
      int cap = std::max(counts[c], 2 * p->cap_work[c]);
      PCHK(p, hipMalloc(&p->d_work[c], sizeof(WorkItem) * cap));
      p->cap_work[c] = cap;
    }
    if (counts[c])
      PCHK(p, hipMemcpyAsync(p->d_work[c], work[c].data(), sizeof(WorkItem) * counts[c], hipMemcpyHostToDevice,
                             p->stream));
  }
  PCHK(p, hipMemcpyAsync(p->d_nwork, counts, sizeof counts, hipMemcpyHostToDevice, p->stream));
  PCHK(p, hipStreamSynchronize(p->stream));  // host vectors above go out of scope
  p->dirty = false;
  return VKLB_OK;
}

}  // namespace

extern "C" {

vklb_status vklb_pool_create(size_t hbm_budget, vklb_precision prec, void* hip_stream, vklb_pool** out) {
  if (!out) return VKLB_ERR_ARG;
  *out = nullptr;
  if (prec != VKLB_FP32 && prec != VKLB_FP64) return VKLB_ERR_ARG;
  if (hbm_budget < (1u << 20)) return VKLB_ERR_ARG;
  vklb_pool* p = new vklb_pool();
  p->prec = prec;
  p->basis[1] = resolve_basis(0, prec, 1);
  p->basis[2] = resolve_basis(0, prec, 2);
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  p->budget = hbm_budget / kAlign * kAlign;
  p->slots.assign(kMaxSlots, nullptr);
  memset(&p->stats, 0, sizeof p->stats);
  auto cleanup = [&](hipError_t e) {
    vklb_pool_destroy(p);
    return e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? VKLB_ERR_OOM : VKLB_ERR_DEVICE;
  };
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return cleanup(e);
  if ((e = hipMalloc(&p->base, p->budget)) != hipSuccess) return cleanup(e);
  if ((e = hipMalloc(&p->d_descs, sizeof(SolveDesc) * kMaxSlots)) != hipSuccess) return cleanup(e);
  if ((e = hipMalloc(&p->d_nwork, sizeof(int) * kClasses)) != hipSuccess) return cleanup(e);
  if ((e = hipMalloc(&p->d_slot_list, sizeof(int) * kMaxSlots)) != hipSuccess) return cleanup(e);
  if ((e = hipMalloc(&p->d_status, sizeof(SlotStatus) * kMaxSlots)) != hipSuccess) return cleanup(e);
  if ((e = hipHostMalloc(&p->h_status, sizeof(SlotStatus) * kMaxSlots, hipHostMallocDefault)) != hipSuccess)
    return cleanup(e);
  for (int c = 0; c < kClasses; ++c) {
    if ((e = hipStreamCreateWithFlags(&p->cls_stream[c], hipStreamNonBlocking)) != hipSuccess) return cleanup(e);
    if ((e = hipEventCreateWithFlags(&p->ev_cls[c], hipEventDisableTiming)) != hipSuccess) return cleanup(e);
  }
  if ((e = hipEventCreateWithFlags(&p->ev_main, hipEventDisableTiming)) != hipSuccess) return cleanup(e);
  p->arena.reset(p->budget);
  for (int kind = 0; kind < 4; ++kind)
    for (int dim = 1; dim <= 2; ++dim)
      p->cls_launch[class_of(kind, dim)] =
          pick_launchers(kind, dim, prec == VKLB_FP32 ? 1 : 0, p->basis[dim], dim == 1 ? 256 : 128);
  p->stats.arena_bytes = p->budget;
  *out = p;
  return VKLB_OK;
}

vklb_status vklb_pool_submit(vklb_pool* p, const vklb_request* rq, uint64_t* ticket) {
  if (!p || !rq || !rq->U0 || !rq->U_out) return VKLB_ERR_ARG;
  const char* msg = "";
  vklb_status st = validate(&rq->sys, rq->lat, &rq->grid, &rq->lambda, rq->omega, rq->bc, &rq->eq, p->prec, &msg);
  if (st != VKLB_OK) return pfail(p, st, msg);
  if (!isfinite(rq->T) && rq->max_steps < 0) return pfail(p, VKLB_ERR_ARG, "a request needs an end time or a step limit");
  Req* r = new Req();
  r->ticket = p->next_ticket++;
  r->tag = rq->tag;
  r->sys = rq->sys;
  r->lat = rq->lat;
  r->grid = rq->grid;
  if (r->grid.dim == 1) r->grid.n[1] = 1;
  r->speed = rq->lambda;
  r->omega = rq->omega;
  r->bc[0] = rq->bc[0];
  r->bc[1] = rq->grid.dim == 2 ? rq->bc[1] : rq->bc[0];
  r->eq = rq->eq;
  r->T = rq->T;
  r->max_steps = rq->max_steps < 0 ? (1ll << 62) : rq->max_steps;
  layout_of(&r->sys, r->lat, &r->grid, p->prec, p->basis[r->grid.dim], &r->L);
  if (align_up(r->L.total) > p->budget) {
    delete r;
    return pfail(p, VKLB_ERR_OOM, "request larger than the pool arena");
  }
  const long long cells = r->grid.n[0] * (r->grid.dim == 2 ? r->grid.n[1] : 1);
  r->U0.assign(rq->U0, rq->U0 + size_t(r->L.p) * cells);
  r->U_out = rq->U_out;
  r->cls = class_of(r->sys.kind, r->grid.dim);
  r->band = r->grid.dim == 2 ? default_band(&r->grid, 128) : 32;  // the batched 2D strips are 128 columns
  r->halo = default_halo(r->sys.kind);
  if (r->grid.dim == 2) pick_shape(p, r->sys.kind, r->grid.n[0], &r->band, &r->halo);
  r->band = std::min(r->band, max_band(r->sys.kind, r->grid.dim, p->basis[r->grid.dim]));
  p->queue.push_back(r);
  p->stats.submitted++;
  if (ticket) *ticket = r->ticket;
  return VKLB_OK;
}

vklb_status vklb_pool_run(vklb_pool* p, int rounds) {
  if (!p || rounds < 0) return VKLB_ERR_ARG;
  PCHK(p, hipSetDevice(p->device));
  vklb_status st = admit(p);
  if (st != VKLB_OK) return st;
  st = upload_lists(p);
  if (st != VKLB_OK) return st;
  if (rounds == 0) return VKLB_OK;
  // class streams start after the caller's stream (admission, lists) ...
  PCHK(p, hipEventRecord(p->ev_main, p->stream));
  const int par0 = int(p->round & 1);
  for (int c = 0; c < kClasses; ++c) {
    if (p->changed[c]) {
      drop_class_graph(p, c);
      p->stable_calls[c] = 0;
    } else {
      p->stable_calls[c]++;
    }
    p->changed[c] = false;
    if (!p->nwork[c]) continue;
    hipStream_t cs = p->cls_stream[c];
    PCHK(p, hipStreamWaitEvent(cs, p->ev_main, 0));
    if (p->gexec[c] && (p->graph_rounds[c] != rounds || p->graph_par[c] != par0)) drop_class_graph(p, c);
    // a class whose resident set was the same at the previous call is captured
    // once (this call) and replayed while it stays the same
    const bool capture = !p->gexec[c] && p->stable_calls[c] >= 1;
    if (capture) {
      PCHK(p, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    }
    if (!p->gexec[c]) {
      std::vector<const SolveDesc*> fold;  // this class's solves whose partials are folded
      for (int i = 0; i < kMaxSlots; ++i)
        if (p->slots[i] && p->slots[i]->cls == c && p->slots[i]->sd.nred != p->slots[i]->sd.nblocks)
          fold.push_back(&p->slots[i]->sd);
      hipError_t e = hipSuccess;
      for (int k = 0; k < rounds && e == hipSuccess; ++k) {
        const int par = (par0 + k) & 1;
        e = p->cls_launch[c].batched(p->d_descs, p->d_work[c], p->d_nwork + c, par, p->nwork[c], cs);
        for (const SolveDesc* d : fold)
          if (e == hipSuccess) e = launch_fold(*d, par ^ 1, cs);
      }
      if (capture) {
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = ee;
        if (e == hipSuccess) e = hipGraphInstantiate(&p->gexec[c], g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          p->gexec[c] = nullptr;
          return pfail(p, VKLB_ERR_DEVICE, std::string("capture of a round chunk: ") + hipGetErrorString(e));
        }
        p->graph[c] = g;
        p->graph_rounds[c] = rounds;
        p->graph_par[c] = par0;
        p->graph_captures++;
      } else if (e != hipSuccess) {
        return pfail(p, VKLB_ERR_DEVICE, std::string("batched launch: ") + hipGetErrorString(e));
      }
    }
    if (p->gexec[c]) {
      PCHK(p, hipGraphLaunch(p->gexec[c], cs));
      p->graph_launches++;
    }
    // ... and the caller's stream continues after every class's rounds
    PCHK(p, hipEventRecord(p->ev_cls[c], cs));
    PCHK(p, hipStreamWaitEvent(p->stream, p->ev_cls[c], 0));
  }
  p->round += rounds;
  p->stats.rounds = p->round;
  return VKLB_OK;
}

vklb_status vklb_pool_poll(vklb_pool* p, vklb_completion* out, int max, int* n) {
  if (!p || (max > 0 && !out)) return VKLB_ERR_ARG;
  PCHK(p, hipSetDevice(p->device));
  std::vector<int> live;
  for (int i = 0; i < kMaxSlots; ++i)
    if (p->slots[i]) live.push_back(i);
  if (!live.empty()) {
    vklb_status st = upload_lists(p);
    if (st != VKLB_OK) return st;
    const int par = int(p->round & 1);
    PCHK(p, hipMemcpyAsync(p->d_slot_list, live.data(), sizeof(int) * live.size(), hipMemcpyHostToDevice, p->stream));
    hipLaunchKernelGGL(k_gather_status, dim3(live.size()), dim3(256), 0, p->stream, p->d_descs, p->d_slot_list,
                       int(live.size()), par, p->d_status);
    PCHK(p, hipGetLastError());
    PCHK(p, hipMemcpyAsync(p->h_status, p->d_status, sizeof(SlotStatus) * live.size(), hipMemcpyDeviceToHost,
                           p->stream));
    PCHK(p, hipStreamSynchronize(p->stream));
    std::vector<int> fin;
    for (size_t k = 0; k < live.size(); ++k)
      if (p->h_status[k].done) fin.push_back(int(k));
    for (int k : fin) {
      Req* r = p->slots[live[k]];
      SolveDesc d = r->sd;
      d.par = par;
      const long long cells = (long long)d.nx * d.ny;
      PCHK(p, p->cls_launch[r->cls].moments(d, grid_for_cells(cells), p->stream));
      PCHK(p, hipMemcpyAsync(r->U_out, d.stage, size_t(r->L.p) * cells * 8, hipMemcpyDeviceToHost, p->stream));
    }
    if (!fin.empty()) PCHK(p, hipStreamSynchronize(p->stream));
    for (int k : fin) {
      Req* r = p->slots[live[k]];
      const SlotStatus& s = p->h_status[k];
      vklb_completion c;
      c.ticket = r->ticket;
      c.tag = r->tag;
      const bool bad = s.err_word != ~0ull;
      c.status = bad ? VKLB_ERR_NONPHYSICAL : VKLB_OK;
      c.t = s.t;
      c.steps = s.n;
      c.fail_step = bad ? (long long)(s.err_word >> 32) : -1;
      c.fail_cell = bad ? (long long)(s.err_word & 0xffffffffull) : -1;
      p->done.push_back(c);
      p->arena.release(r->off, r->L.total);
      p->slots[live[k]] = nullptr;
      p->changed[r->cls] = true;
      delete r;
      p->dirty = true;
      p->stats.completed++;
    }
  }
  int cnt = 0;
  while (cnt < max && !p->done.empty()) {
    out[cnt++] = p->done.front();
    p->done.pop_front();
  }
  if (n) *n = cnt;
  return VKLB_OK;
}

vklb_status vklb_pool_get_stats(const vklb_pool* p, vklb_pool_stats* st) {
  if (!p || !st) return VKLB_ERR_ARG;
  *st = p->stats;
  st->queued = (int64_t)p->queue.size();
  int64_t res = 0;
  for (Req* r : p->slots)
    if (r) ++res;
  st->resident = res;
  st->arena_used = p->arena.used();
  st->arena_peak = p->arena.peak();
  st->graph_launches = p->graph_launches;
  st->graph_captures = p->graph_captures;
  return VKLB_OK;
}

vklb_status vklb_pool_autotune(vklb_pool* p, const vklb_request* samples, int n, int steps, vklb_pool_tile* out,
                               int* n_out) {
  if (!p || (n > 0 && !samples) || n < 0 || steps < 1 || steps > 100000) return VKLB_ERR_ARG;
  if (!p->queue.empty()) return pfail(p, VKLB_ERR_STATE, "vklb_pool_autotune: requests are queued");
  for (Req* r : p->slots)
    if (r) return pfail(p, VKLB_ERR_STATE, "vklb_pool_autotune: solves are resident");
  PCHK(p, hipSetDevice(p->device));
  int written = 0;
  for (int i = 0; i < n; ++i) {
    const vklb_request& r = samples[i];
    if (r.grid.dim != 2) continue;  // 1D tiles have one shape in the batched kernel
    int band = 0, halo = 0;
    double us = 0.0;
    vklb_status st = tune_pool_shape(&r, p->prec, steps, p->stream, &band, &halo, &us);
    if (st != VKLB_OK) return pfail(p, st, std::string("vklb_pool_autotune: ") + vklb_last_error(nullptr));
    {
      std::lock_guard<std::mutex> lk(g_tiles_mu);
      g_tiles[{p->device, int(p->prec), int(r.sys.kind), size_class(r.grid.n[0])}] = {band, halo};
    }
    if (out && n_out && written < *n_out) {
      vklb_pool_tile& t = out[written++];
      t.kind = r.sys.kind;
      t.n = r.grid.n[0];
      t.size_class = size_class(r.grid.n[0]);
      t.band_rows = band;
      t.halo_rows = halo;
      t.step_us = us;
    }
  }
  if (n_out) *n_out = written;
  return VKLB_OK;
}

void vklb_pool_destroy(vklb_pool* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  for (Req* r : p->queue) delete r;
  for (Req* r : p->slots) delete r;
  for (int c = 0; c < kClasses; ++c) drop_class_graph(p, c);
  for (int c = 0; c < kClasses; ++c) {
    if (p->cls_stream[c]) {
      (void)hipStreamSynchronize(p->cls_stream[c]);
      (void)hipStreamDestroy(p->cls_stream[c]);
    }
    if (p->ev_cls[c]) (void)hipEventDestroy(p->ev_cls[c]);
  }
  if (p->ev_main) (void)hipEventDestroy(p->ev_main);
  for (int c = 0; c < kClasses; ++c)
    if (p->d_work[c]) (void)hipFree(p->d_work[c]);
  if (p->d_descs) (void)hipFree(p->d_descs);
  if (p->d_nwork) (void)hipFree(p->d_nwork);
  if (p->d_slot_list) (void)hipFree(p->d_slot_list);
  if (p->d_status) (void)hipFree(p->d_status);
  if (p->h_status) (void)hipHostFree(p->h_status);
  if (p->base) (void)hipFree(p->base);
  delete p;
}

}  // extern "C"
