// Host-side evaluation of the per-cell arithmetic in vklb_cell.hpp, and of
// the 2D row placement of the population buffers (mem_row, reorder_rows in
// vklb_host.hpp), for the CPU test suite only (it lets the closed-form splits
// be compared with the oracle, and the layout be checked, without a GPU).
// Nothing in the library's entry points calls it.
#include "vklb_cell.hpp"
#include "vklb_host.hpp"

using namespace vklb;

namespace {

template <class S>
Phys make_phys(const double* prm) {
  // prm: g, gamma, ch_factor, adv0, adv1, omega, c, k, kinf, alpha_local
  Phys ph{};
  ph.g = prm[0];
  ph.gamma = prm[1];
  ph.ch_factor = prm[2];
  ph.adv[0] = prm[3];
  ph.adv[1] = prm[4];
  ph.omega = prm[5];
  ph.c = prm[6];
  ph.k = prm[7];
  ph.kinf = int(prm[8]);
  ph.alpha_local = int(prm[9]);
  return ph;
}

template <int KIND, int DIM, class S>
int run_split(int d, const double* U, const double* prm, double Lam, double ch, double* F, double* D) {
  using C = Cell<KIND, DIM, S>;
  S u[C::P], f[C::P], dd[C::P];
  for (int i = 0; i < C::P; ++i) u[i] = S(U[i]);
  C::split(d, u, make_phys<S>(prm), S(Lam), S(ch), f, dd);
  for (int i = 0; i < C::P; ++i) { F[i] = double(f[i]); D[i] = double(dd[i]); }
  return C::P;
}

template <int KIND, int DIM, class S>
int run_feq(const double* U, const double* prm, double xi, double Lam, double ch, double* out) {
  using E = Equilibrium<KIND, DIM, S>;
  S u[E::P], fe[E::Q][E::P];
  for (int i = 0; i < E::P; ++i) u[i] = S(U[i]);
  E::eval(u, make_phys<S>(prm), S(1.0 / xi), S(Lam), S(ch), fe);
  for (int q = 0; q < E::Q; ++q)
    for (int i = 0; i < E::P; ++i) out[q * E::P + i] = double(fe[q][i]);
  return E::P;
}

template <int KIND, int DIM, class S>
int run_speeds(const double* U, const double* prm, double* lam, double* cfm) {
  using C = Cell<KIND, DIM, S>;
  S u[C::P], a, b;
  for (int i = 0; i < C::P; ++i) u[i] = S(U[i]);
  C::speeds(u, make_phys<S>(prm), &a, &b);
  *lam = double(a);
  *cfm = double(b);
  return C::P;
}

#define DISPATCH(FN, ...)                                                   \
  switch (kind * 10 + dim) {                                                \
    case K_SW * 10 + 1: return FN<K_SW, 1, S>(__VA_ARGS__);                 \
    case K_SW * 10 + 2: return FN<K_SW, 2, S>(__VA_ARGS__);                 \
    case K_EULER * 10 + 1: return FN<K_EULER, 1, S>(__VA_ARGS__);           \
    case K_EULER * 10 + 2: return FN<K_EULER, 2, S>(__VA_ARGS__);           \
    case K_MHD * 10 + 1: return FN<K_MHD, 1, S>(__VA_ARGS__);               \
    case K_MHD * 10 + 2: return FN<K_MHD, 2, S>(__VA_ARGS__);               \
    case K_LINEAR * 10 + 1: return FN<K_LINEAR, 1, S>(__VA_ARGS__);         \
    case K_LINEAR * 10 + 2: return FN<K_LINEAR, 2, S>(__VA_ARGS__);         \
  }                                                                         \
  return -1;

template <class S>
int split_any(int kind, int dim, int d, const double* U, const double* prm, double Lam, double ch, double* F,
              double* D) {
  DISPATCH(run_split, d, U, prm, Lam, ch, F, D)
}
template <class S>
int feq_any(int kind, int dim, const double* U, const double* prm, double xi, double Lam, double ch, double* out) {
  DISPATCH(run_feq, U, prm, xi, Lam, ch, out)
}
template <class S>
int speeds_any(int kind, int dim, const double* U, const double* prm, double* lam, double* cfm) {
  DISPATCH(run_speeds, U, prm, lam, cfm)
}

template <int KIND, class S>
int run_char(const double* U, const double* dU, const double* prm, double ch, int right, double* out) {
  using C = Cell<KIND, 1, S>;
  S u[C::P], du[C::P], o[C::P];
  for (int i = 0; i < C::P; ++i) { u[i] = S(U[i]); du[i] = S(dU[i]); }
  if (!C::char_correction(u, du, make_phys<S>(prm), S(ch), right != 0, o)) return -1;
  for (int i = 0; i < C::P; ++i) out[i] = double(o[i]);
  return C::P;
}
template <class S>
int char_any(int kind, const double* U, const double* dU, const double* prm, double ch, int right, double* out) {
  switch (kind) {
    case K_SW: return run_char<K_SW, S>(U, dU, prm, ch, right, out);
    case K_EULER: return run_char<K_EULER, S>(U, dU, prm, ch, right, out);
    case K_MHD: return run_char<K_MHD, S>(U, dU, prm, ch, right, out);
    case K_LINEAR: return run_char<K_LINEAR, S>(U, dU, prm, ch, right, out);
  }
  return -1;
}

}  // namespace

extern "C" {
// Characteristic boundary correction P (Lambda dW)' of a 1D system (SW,
// Euler, MHD with cleaning speed ch, linear). Returns p, or -1.
int vklb_cc_char(int prec, int kind, const double* U, const double* dU, const double* prm, double ch, int right,
                 double* out) {
  return prec == 4 ? char_any<float>(kind, U, dU, prm, ch, right, out)
                   : char_any<double>(kind, U, dU, prm, ch, right, out);
}
// prec: 8 -> double arithmetic, 4 -> float arithmetic. Returns p, or -1.
int vklb_cc_split(int prec, int kind, int dim, int d, const double* U, const double* prm, double Lam, double ch,
                  double* F, double* D) {
  return prec == 4 ? split_any<float>(kind, dim, d, U, prm, Lam, ch, F, D)
                   : split_any<double>(kind, dim, d, U, prm, Lam, ch, F, D);
}
int vklb_cc_feq(int prec, int kind, int dim, const double* U, const double* prm, double xi, double Lam, double ch,
                double* out) {
  return prec == 4 ? feq_any<float>(kind, dim, U, prm, xi, Lam, ch, out)
                   : feq_any<double>(kind, dim, U, prm, xi, Lam, ch, out);
}
int vklb_cc_speeds(int prec, int kind, int dim, const double* U, const double* prm, double* lam, double* cfm) {
  return prec == 4 ? speeds_any<float>(kind, dim, U, prm, lam, cfm)
                   : speeds_any<double>(kind, dim, U, prm, lam, cfm);
}
// Buffer row of grid row r (mem_row) for bands of `band` rows, of which
// nfull are whole; down_odd: odd bands march down (MHD).
long long vklb_cc_mem_row(int r, int band, int nfull, int down_odd) { return mem_row(r, band, nfull, down_odd != 0); }
// reorder_rows over a population buffer of `planes` planes of elem-byte
// values for a 2D grid of row stride sx (a multiple of 64) and ny rows:
// to_grid = 1 from the device's row order to grid order, 0 the reverse.
// `from` and `to` hold stride * planes values, stride = sx * ny rounded up to
// whole 256-cell blocks.
void vklb_cc_reorder_rows(const void* from, void* to, int sx, int ny, int band, int nfull, int down_odd, int planes,
                          int elem, int to_grid) {
  SolveDesc d;
  memset(&d, 0, sizeof d);
  d.sx = sx;
  d.ny = ny;
  d.band = band;
  d.nfull = nfull;
  Layout L;
  memset(&L, 0, sizeof L);
  L.slots = planes;
  L.p = 1;
  L.elem = elem;
  reorder_rows(static_cast<const char*>(from), static_cast<char*>(to), d, L, down_odd != 0, to_grid != 0);
}
}
