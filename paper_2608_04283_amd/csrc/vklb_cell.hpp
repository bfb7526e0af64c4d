// Per-cell arithmetic of the weighted-upwind vector kinetic lattice Boltzmann
// step: physical fluxes, characteristic speeds, the sigmoid-weighted flux
// split and the weighted-upwind equilibrium. Host+device functions; the GPU
// kernels and the host-side cell check both include this header.
//
// The split is written as F+ = F/2 + D and F- = F/2 - D with
//   D = sum_j beta(lambda_j) phi_j r_j,  beta = alpha - 1/2 = tanh(k lambda / (2 Lambda)) / 2,
// which is the weighted splitting of Sec. 3.1 (alpha = 1/(1+exp(-k lambda/Lambda)))
// rearranged; D is evaluated per system in closed form, without forming
// the eigenvector matrix P or solving P Phi = F:
//   * linear advection: one wave;
//   * shallow water (Sec. 5.1): the two acoustic waves (the shear wave of the
//     2D system carries no flux);
//   * Euler (Sec. 5.2): the flux is homogeneous of degree one, so
//     D = P diag(beta_j lambda_j) P^-1 U, the Steger-Warming formula with each
//     eigenvalue scaled by its weight;
//   * ideal MHD with divergence cleaning (Sec. 5.3): the Jacobian is block
//     triangular, [[A7, C], [0, G]] with the (B_n, psi) pair in G. D on the
//     seven-wave block uses Roe-Balsara normalized primitive eigenvectors
//     (well defined at coinciding speeds); the coupling through C uses divided
//     differences of beta between each seven-wave speed and +-c_h; on the
//     cleaning pair D = beta(c_h) c_h (B_n, psi). In FP32, the eigenstructure
//     (speeds and normalization) of directions whose speeds nearly coincide is
//     evaluated in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace vklb {

enum Kind { K_SW = 0, K_EULER = 1, K_MHD = 2, K_LINEAR = 3 };

// Physical and method parameters of one solve (read-only in kernels).
struct Phys {
  double g, gamma, ch_factor;
  double adv[2];
  double omega, c, k;
  int kinf;         // 1: discontinuous split (k = infinity)
  int alpha_local;  // 1: normalize the sigmoid by the cell's own max |lambda|
};

template <int KIND, int DIM>
struct SysInfo;
template <> struct SysInfo<K_SW, 1> { static constexpr int P = 2; };
template <> struct SysInfo<K_SW, 2> { static constexpr int P = 3; };
template <> struct SysInfo<K_EULER, 1> { static constexpr int P = 3; };
template <> struct SysInfo<K_EULER, 2> { static constexpr int P = 4; };
template <> struct SysInfo<K_MHD, 1> { static constexpr int P = 9; };
template <> struct SysInfo<K_MHD, 2> { static constexpr int P = 9; };
template <> struct SysInfo<K_LINEAR, 1> { static constexpr int P = 1; };
template <> struct SysInfo<K_LINEAR, 2> { static constexpr int P = 1; };

template <class S>
__host__ __device__ inline S sq(S a) { return a * a; }

// beta(lambda) = alpha(lambda) - 1/2 for the sigmoid of Sec. 3.1.
// Division, reciprocal and square root of the per-cell arithmetic. FP32
// device code uses the hardware reciprocal and square root (about 1 ulp),
// as plain operations the compiler cannot fuse differently in different
// places, so every inlined copy still rounds identically; FP64, and host
// code, use the correctly rounded operations.
template <class S>
__host__ __device__ inline S qrcp(S b) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (sizeof(S) == 4) return __builtin_amdgcn_rcpf(b);
#endif
  return S(1) / b;
}
template <class S>
__host__ __device__ inline S qdiv(S a, S b) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (sizeof(S) == 4) return a * __builtin_amdgcn_rcpf(b);
#endif
  return a / b;
}
template <class S>
__host__ __device__ inline S qsqrt(S x) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (sizeof(S) == 4) return __builtin_amdgcn_sqrtf(x);
#endif
  return sqrt(x);
}

// tanh for the weights. FP32 device code evaluates it from its exponential
// form, tanh z = sign(z) (1 - e^{-2|z|}) / (1 + e^{-2|z|}), with the hardware
// base-2 exponential and reciprocal: a few units in the last place (absolute
// error ~1e-7 near z = 0), far inside the FP32 path's tolerance, and an odd
// function exactly as tanh is. FP64 device code uses the same identity through
// expm1, tanh z = sign(z) (-m) / (2 + m) with m = e^{-2|z|} - 1: about two
// units in the last place at every z (no cancellation near 0), in 68 vector
// instructions where the library tanh takes 165. Host code calls tanh.
template <class S>
__host__ __device__ inline S wtanh(S z) {
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (sizeof(S) == 4) {
    const float t = __builtin_amdgcn_exp2f(-2.8853900817779268f * fabsf(z));  // e^{-2|z|}
    return copysignf((1.0f - t) * __builtin_amdgcn_rcpf(1.0f + t), z);
  } else {
    const double m = expm1(-2.0 * fabs(double(z)));
    return S(copysign(-m / (2.0 + m), double(z)));
  }
#endif
  return tanh(z);
}

template <class S>
__host__ __device__ inline S beta_w(S lam, S half_k_over_L, int kinf) {
  if (kinf) return lam >= S(0) ? S(0.5) : S(-0.5);
  return S(0.5) * wtanh(lam * half_k_over_L);
}

// Divided difference (beta(a) - beta(b)) / (a - b) from the weights ba, bb
// already evaluated, with the derivative when the two speeds nearly coincide.
template <class S>
__host__ __device__ inline S beta_dd(S a, S ba, S b, S bb, S half_k_over_L, int kinf) {
  const S d = a - b;
  const S rel = sizeof(S) == 4 ? S(1e-3) : S(1e-6);
  if (fabs(d) > rel * (fabs(a) + fabs(b)) || kinf) return d != S(0) ? qdiv(ba - bb, d) : S(0);
  const S tm = wtanh(S(0.5) * (a + b) * half_k_over_L);
  return S(0.5) * half_k_over_L * (S(1) - tm * tm);
}

// ---------------------------------------------------------------------------
// Cell speeds: max |lambda| over directions and (MHD) the max fast speed.
// ---------------------------------------------------------------------------
template <int KIND, int DIM, class S>
struct Cell;

// ----------------------------- linear advection ----------------------------
template <int DIM, class S>
struct Cell<K_LINEAR, DIM, S> {
  static constexpr int P = 1;
  // Characteristic boundary of Sec. 3.3 (1D): out = g(a) dU with g(a) = a for
  // an outgoing wave (a > 0 at the right boundary, a < 0 at the left), else 0.
  __host__ __device__ static bool char_correction(const S* Ub, const S* dU, const Phys& ph, S, bool right, S* out) {
    (void)Ub;
    const S a = S(ph.adv[0]);
    out[0] = (right ? a > S(0) : a < S(0)) ? a * dU[0] : S(0);
    return true;
  }
  __host__ __device__ static void speeds(const S* U, const Phys& ph, S* lam, S* cfm) {
    S m = S(0);
    for (int d = 0; d < DIM; ++d) m = fmax(m, fabs(S(ph.adv[d])));
    *lam = m;
    *cfm = S(0);
  }
  __host__ __device__ static bool admissible(const S* U, const Phys&) { return isfinite(U[0]); }
  // F^(d) and D^(d); Lam normalizes the sigmoid (global max |lambda|), ch unused.
  __host__ __device__ static void split(int d, const S* U, const Phys& ph, S Lam, S, S* F, S* D) {
    S a = S(ph.adv[d]);
    S L = ph.alpha_local ? fabs(a) : Lam;
    S hk = L > S(0) ? qdiv(S(0.5 * ph.k), L) : S(0);
    F[0] = a * U[0];
    D[0] = beta_w(a, hk, ph.kinf) * a * U[0];
  }
};

// ------------------------------- shallow water -----------------------------
template <int DIM, class S>
struct Cell<K_SW, DIM, S> {
  static constexpr int P = DIM + 1;
  // Characteristic boundary of Sec. 3.3 (1D): out = sum_j g(lambda_j) (l_j . dU) r_j
  // over u -+ c, with r = (1, u -+ c), l = (+-(u +- c), -+1) / (2c) and g the
  // speed for outgoing waves, 0 for incoming ones.
  __host__ __device__ static bool char_correction(const S* Ub, const S* dU, const Phys& ph, S, bool right, S* out) {
    const S h = Ub[0];
    const S u = qdiv(Ub[1], h);
    const S c = qsqrt(S(ph.g) * h);
    const S l1 = u - c, l2 = u + c;
    const S i2c = qrcp(S(2) * c);
    const S w1 = ((u + c) * dU[0] - dU[1]) * i2c;
    const S w2 = (dU[1] - (u - c) * dU[0]) * i2c;
    const S g1 = (right ? l1 > S(0) : l1 < S(0)) ? l1 : S(0);
    const S g2 = (right ? l2 > S(0) : l2 < S(0)) ? l2 : S(0);
    out[0] = g1 * w1 + g2 * w2;
    out[1] = g1 * w1 * l1 + g2 * w2 * l2;
    return isfinite(out[0]) && isfinite(out[1]);
  }
  __host__ __device__ static void speeds(const S* U, const Phys& ph, S* lam, S* cfm) {
    S h = U[0];
    S c = qsqrt(S(ph.g) * h);
    S m = S(0);
    for (int d = 0; d < DIM; ++d) m = fmax(m, fabs(qdiv(U[1 + d], h)) + c);
    *lam = m;
    *cfm = S(0);
  }
  __host__ __device__ static bool admissible(const S* U, const Phys&) {
    bool ok = U[0] > S(0);
    for (int i = 0; i < P; ++i) ok = ok && isfinite(U[i]);
    return ok;
  }
  __host__ __device__ static void split(int d, const S* U, const Phys& ph, S Lam, S, S* F, S* D) {
    const S h = U[0];
    const S g = S(ph.g);
    const S ud = qdiv(U[1 + d], h);
    const S c = qsqrt(g * h);
    F[0] = U[1 + d];
    for (int kk = 0; kk < DIM; ++kk) F[1 + kk] = U[1 + kk] * ud;
    F[1 + d] += S(0.5) * g * h * h;
    const S lm = ud - c, lp = ud + c;
    const S L = ph.alpha_local ? fmax(fabs(lm), fabs(lp)) : Lam;
    const S hk = L > S(0) ? qdiv(S(0.5 * ph.k), L) : S(0);
    // coefficients of the two acoustic waves: phi = h (2 u_d -+ c) / 4
    const S wm = beta_w(lm, hk, ph.kinf) * h * (S(2) * ud - c) * S(0.25);
    const S wp = beta_w(lp, hk, ph.kinf) * h * (S(2) * ud + c) * S(0.25);
    D[0] = wm + wp;
    for (int kk = 0; kk < DIM; ++kk) D[1 + kk] = qdiv(U[1 + kk], h) * (wm + wp);
    D[1 + d] = lm * wm + lp * wp;
  }
};

// ----------------------------------- Euler ---------------------------------
template <int DIM, class S>
struct Cell<K_EULER, DIM, S> {
  static constexpr int P = DIM + 2;
  // Characteristic boundary of Sec. 3.3 (1D): out = sum_j g(lambda_j) (l_j . dU) r_j
  // over u - a, u, u + a with the textbook eigenvectors r = (1, u -+ a, H -+ ua),
  // (1, u, u^2/2) and left eigenvectors (b1 = (gamma-1)/a^2, b2 = b1 u^2/2)
  // l_1,3 = (b2 +- u/a, -(b1 u +- 1/a), b1)/2, l_2 = (1 - b2, b1 u, -b1);
  // g is the speed for outgoing waves, 0 for incoming ones.
  __host__ __device__ static bool char_correction(const S* Ub, const S* dU, const Phys& ph, S, bool right, S* out) {
    const S gamma = S(ph.gamma);
    const S rho = Ub[0];
    const S u = qdiv(Ub[1], rho);
    const S E = Ub[2];
    const S p = (gamma - S(1)) * (E - S(0.5) * rho * u * u);
    const S a = qsqrt(qdiv(gamma * p, rho));
    const S H = qdiv(E + p, rho);
    const S ia = qrcp(a);
    const S b1 = (gamma - S(1)) * ia * ia, b2 = S(0.5) * b1 * u * u;
    const S w1 = S(0.5) * ((b2 + u * ia) * dU[0] - (b1 * u + ia) * dU[1] + b1 * dU[2]);
    const S w2 = (S(1) - b2) * dU[0] + b1 * u * dU[1] - b1 * dU[2];
    const S w3 = S(0.5) * ((b2 - u * ia) * dU[0] - (b1 * u - ia) * dU[1] + b1 * dU[2]);
    const S lam[3] = {u - a, u, u + a};
    S g[3];
    for (int j = 0; j < 3; ++j) g[j] = (right ? lam[j] > S(0) : lam[j] < S(0)) ? lam[j] : S(0);
    const S c1 = g[0] * w1, c2 = g[1] * w2, c3 = g[2] * w3;
    out[0] = c1 + c2 + c3;
    out[1] = c1 * (u - a) + c2 * u + c3 * (u + a);
    out[2] = c1 * (H - u * a) + c2 * (S(0.5) * u * u) + c3 * (H + u * a);
    return isfinite(out[0]) && isfinite(out[1]) && isfinite(out[2]);
  }
  __host__ __device__ static S pressure(const S* U, S gamma) {
    S m2 = S(0);
    for (int kk = 0; kk < DIM; ++kk) m2 += U[1 + kk] * U[1 + kk];
    return (gamma - S(1)) * (U[DIM + 1] - S(0.5) * qdiv(m2, U[0]));
  }
  __host__ __device__ static void speeds(const S* U, const Phys& ph, S* lam, S* cfm) {
    const S gamma = S(ph.gamma);
    const S rho = U[0];
    const S c = qsqrt(qdiv(gamma * pressure(U, gamma), rho));
    S m = S(0);
    for (int d = 0; d < DIM; ++d) m = fmax(m, fabs(qdiv(U[1 + d], rho)) + c);
    *lam = m;
    *cfm = S(0);
  }
  __host__ __device__ static bool admissible(const S* U, const Phys& ph) {
    bool ok = U[0] > S(0) && pressure(U, S(ph.gamma)) > S(0);
    for (int i = 0; i < P; ++i) ok = ok && isfinite(U[i]);
    return ok;
  }
  __host__ __device__ static void split(int d, const S* U, const Phys& ph, S Lam, S, S* F, S* D) {
    const S gamma = S(ph.gamma);
    const S rho = U[0];
    const S irho = qrcp(rho);
    S vel[DIM];
    S v2 = S(0);
    for (int kk = 0; kk < DIM; ++kk) { vel[kk] = U[1 + kk] * irho; v2 += vel[kk] * vel[kk]; }
    const S E = U[DIM + 1];
    const S p = (gamma - S(1)) * (E - S(0.5) * rho * v2);
    const S c = qsqrt(gamma * p * irho);
    const S ud = vel[d];
    F[0] = U[1 + d];
    for (int kk = 0; kk < DIM; ++kk) F[1 + kk] = U[1 + kk] * ud;
    F[1 + d] += p;
    F[DIM + 1] = (E + p) * ud;
    const S l1 = ud - c, l3 = ud + c;
    const S L = ph.alpha_local ? fmax(fabs(l1), fabs(l3)) : Lam;
    const S hk = L > S(0) ? qdiv(S(0.5 * ph.k), L) : S(0);
    const S mu1 = beta_w(l1, hk, ph.kinf) * l1;
    const S mu2 = beta_w(ud, hk, ph.kinf) * ud;
    const S mu3 = beta_w(l3, hk, ph.kinf) * l3;
    const S H = (E + p) * irho;
    const S s = qdiv(rho, S(2) * gamma);
    const S ent = S(2) * (gamma - S(1)) * mu2;
    D[0] = s * (ent + mu1 + mu3);
    for (int kk = 0; kk < DIM; ++kk) D[1 + kk] = s * (ent + mu1 + mu3) * vel[kk];
    D[1 + d] += s * c * (mu3 - mu1);
    D[DIM + 1] = s * (ent * S(0.5) * v2 + mu1 * (H - ud * c) + mu3 * (H + ud * c));
  }
};

// ------------------------- ideal MHD with GLM cleaning ----------------------
// Conserved order: rho, m_x, m_y, m_z, E, B_x, B_y, B_z, psi (3-vectors in 1D/2D).
template <int DIM, class S>
struct Cell<K_MHD, DIM, S> {
  static constexpr int P = 9;
  // Characteristic boundary of Sec. 3.3 (1D, normal x): out = g(A) dU with
  // g(lambda) = lambda for waves leaving through the boundary and 0 for the
  // others, over the nine waves of the GLM system: the seven MHD waves through
  // the primitive eigenvectors of the split below, the cleaning pair +-c_h on
  // (B_n, psi), and the pair's coupling into the seven-wave block through the
  // B_n column of the Jacobian, by divided differences of g (the Jacobian is
  // block triangular). Computed in FP64 in both precisions: it runs on two
  // cells per step.
  __host__ __device__ static bool char_correction(const S* Ub, const S* dU, const Phys& ph, S ch, bool right,
                                                  S* out) {
    double U[9], dv[9], o[9];
    for (int i = 0; i < 9; ++i) {
      U[i] = double(Ub[i]);
      dv[i] = double(dU[i]);
    }
    if (!char64(U, dv, ph, double(ch), right, o)) return false;
    bool ok = true;
    for (int i = 0; i < 9; ++i) {
      out[i] = S(o[i]);
      ok = ok && isfinite(out[i]);
    }
    return ok;
  }
  __host__ __device__ static bool char64(const double* Ug, const double* dv, const Phys& ph, double ch, bool right,
                                         double* out) {
    using C = Cell<K_MHD, DIM, double>;
    if (!(ch > 0.0)) return false;
    const double gamma = ph.gamma, gm1 = gamma - 1.0;
    const double rho = Ug[0], irho = 1.0 / rho;
    const double u = Ug[1] * irho, v = Ug[2] * irho, w = Ug[3] * irho;
    const double Bn = Ug[5], By = Ug[6], Bz = Ug[7];
    const double uu = u * u + v * v + w * w;
    const double p = gm1 * (Ug[4] - 0.5 * rho * uu - 0.5 * (Bn * Bn + By * By + Bz * Bz));
    double eg[9];
    C::template eigenstructure<double>(rho, p, Bn, By, Bz, gamma, eg);
    typename C::Waves W;
    W.rho = rho;
    W.sr = sqrt(rho);
    W.a2 = eg[0];
    W.a = eg[1];
    W.cf = eg[2];
    W.cs = eg[3];
    const double ca = eg[4];
    W.af = eg[5];
    W.as = eg[6];
    W.by = eg[7];
    W.bz = eg[8];
    W.sgn = Bn >= 0.0 ? 1.0 : -1.0;
    const double lam[7] = {u - W.cf, u - ca, u - W.cs, u, u + W.cs, u + ca, u + W.cf};
    auto out_ = [right](double l) { return right ? l > 0.0 : l < 0.0; };
    auto g = [&](double l) { return out_(l) ? l : 0.0; };
    auto dd = [&](double a, double b) { return a != b ? (g(a) - g(b)) / (a - b) : (out_(a) ? 1.0 : 0.0); };
    // primitive images (B_n held fixed) of the seven-wave part of dU and of
    // the B_n column of the Jacobian
    double x[7], xC[7];
    x[0] = dv[0];
    x[1] = (dv[1] - u * dv[0]) * irho;
    x[2] = (dv[2] - v * dv[0]) * irho;
    x[3] = (dv[3] - w * dv[0]) * irho;
    x[4] = gm1 * (dv[4] + 0.5 * uu * dv[0] - (u * dv[1] + v * dv[2] + w * dv[3]) - By * dv[6] - Bz * dv[7]);
    x[5] = dv[6];
    x[6] = dv[7];
    xC[0] = 0.0;
    xC[1] = -gamma * Bn * irho;
    xC[2] = -By * irho;
    xC[3] = -Bz * irho;
    xC[4] = gm1 * (v * By + w * Bz);
    xC[5] = -v;
    xC[6] = -w;
    double c[7], cC[7], cD[7];
    C::project(W, x, c);
    C::project(W, xC, cC);
    // cleaning pair: eigenvalues +-c_h, eigenvectors (1, +-c_h) on (B_n, psi)
    const double qp = 0.5 * (dv[5] + dv[8] / ch), qm = 0.5 * (dv[5] - dv[8] / ch);
    for (int j = 0; j < 7; ++j) cD[j] = g(lam[j]) * c[j] + (dd(lam[j], ch) * qp + dd(lam[j], -ch) * qm) * cC[j];
    double y[7];
    C::combine(W, cD, y);
    out[0] = y[0];
    out[1] = u * y[0] + rho * y[1];
    out[2] = v * y[0] + rho * y[2];
    out[3] = w * y[0] + rho * y[3];
    out[4] = y[4] / gm1 + 0.5 * uu * y[0] + rho * (u * y[1] + v * y[2] + w * y[3]) + By * y[5] + Bz * y[6];
    out[6] = y[5];
    out[7] = y[6];
    out[5] = g(ch) * qp + g(-ch) * qm;
    out[8] = ch * (g(ch) * qp - g(-ch) * qm);
    return true;
  }

  __host__ __device__ static S pressure(const S* U, S gamma) {
    S m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
    S B2 = U[5] * U[5] + U[6] * U[6] + U[7] * U[7];
    return (gamma - S(1)) * (U[4] - S(0.5) * qdiv(m2, U[0]) - S(0.5) * B2);
  }
  // fast speed along direction d
  __host__ __device__ static S fast(const S* U, S gamma, int d) {
    const S rho = U[0];
    const S a2 = qdiv(gamma * pressure(U, gamma), rho);
    const S bn2 = qdiv(U[5 + d] * U[5 + d], rho);
    const S bt2 = qdiv(U[5] * U[5] + U[6] * U[6] + U[7] * U[7], rho) - bn2;
    const S disc = qsqrt(sq(a2 - bn2) + bt2 * (S(2) * a2 + S(2) * bn2 + bt2));
    return qsqrt(S(0.5) * (a2 + bn2 + bt2 + disc));
  }
  __host__ __device__ static void speeds(const S* U, const Phys& ph, S* lam, S* cfm) {
    const S gamma = S(ph.gamma);
    S m = S(0), cm = S(0);
    for (int d = 0; d < DIM; ++d) {
      const S cf = fast(U, gamma, d);
      m = fmax(m, fabs(qdiv(U[1 + d], U[0])) + cf);
      cm = fmax(cm, cf);
    }
    *lam = m;   // seven-wave max; the cleaning speed joins it globally
    *cfm = cm;
  }
  __host__ __device__ static bool admissible(const S* U, const Phys& ph) {
    bool ok = U[0] > S(0) && pressure(U, S(ph.gamma)) > S(0);
    for (int i = 0; i < P; ++i) ok = ok && isfinite(U[i]);
    return ok;
  }

  // Primitive-variable wave decomposition along the normal direction.
  struct Waves {
    S rho, sr, a, a2, cf, cs, af, as, by, bz, sgn;
  };

  // Coefficients (f-, a-, s-, e, s+, a+, f+) of a primitive 7-vector
  // x = (rho, u_n, u_t1, u_t2, p, B_t1, B_t2) in the right eigenvectors.
  __host__ __device__ static void project(const Waves& w, const S* x, S* c) {
    const S xvp = w.by * x[2] + w.bz * x[3];
    const S xvq = -w.bz * x[2] + w.by * x[3];
    const S xbp = w.by * x[5] + w.bz * x[6];
    const S xbq = -w.bz * x[5] + w.by * x[6];
    const S X = qdiv(x[4], w.rho * w.a2);
    const S Y = qdiv(xbp, w.a * w.sr);
    const S Fp = w.af * X + w.as * Y;
    const S Sp = w.as * X - w.af * Y;
    const S Z1 = x[1], Z2 = w.sgn * xvp;
    const S ia2 = qrcp(w.a2);
    const S Fm = (w.af * w.cf * Z1 - w.as * w.cs * Z2) * ia2;
    const S Sm = (w.as * w.cs * Z1 + w.af * w.cf * Z2) * ia2;
    const S Ap = qdiv(xbq, w.sr), Am = -w.sgn * xvq;
    c[0] = S(0.5) * (Fp - Fm);
    c[6] = S(0.5) * (Fp + Fm);
    c[2] = S(0.5) * (Sp - Sm);
    c[4] = S(0.5) * (Sp + Sm);
    c[1] = S(0.5) * (Ap - Am);
    c[5] = S(0.5) * (Ap + Am);
    c[3] = x[0] - x[4] * ia2;
  }
  // sum_j c_j r_j (primitive 7-vector) for the same eigenvectors.
  __host__ __device__ static void combine(const Waves& w, const S* c, S* y) {
    const S Fp = c[6] + c[0], Fm = c[6] - c[0];
    const S Sp = c[4] + c[2], Sm = c[4] - c[2];
    const S Ap = c[5] + c[1], Am = c[5] - c[1];
    const S pf = w.af * Fp + w.as * Sp;
    y[0] = c[3] + w.rho * pf;
    y[1] = w.af * w.cf * Fm + w.as * w.cs * Sm;
    const S vp = w.sgn * (-w.as * w.cs * Fm + w.af * w.cf * Sm);
    const S vq = -w.sgn * Am;
    y[2] = w.by * vp - w.bz * vq;
    y[3] = w.bz * vp + w.by * vq;
    y[4] = w.rho * w.a2 * pf;
    const S bp = w.a * w.sr * (w.as * Fp - w.af * Sp);
    const S bq = w.sr * Ap;
    y[5] = w.by * bp - w.bz * bq;
    y[6] = w.bz * bp + w.by * bq;
  }

  // Directions near the triple point, where the fast and slow speeds nearly
  // meet (c_f^2 - c_s^2 = disc small: transverse field -> 0 and a^2 -> b_n^2
  // together): the FP32 split computes their eigenstructure in FP64. Near the
  // other coincidences (transverse field -> 0 alone, where the fast or slow
  // speed meets the Alfven speed, or normal field -> 0) the FP32 closed form
  // with the Roe-Balsara normalization stays at FP32 rounding of the FP64
  // split at every distance, so those stay in FP32; near the triple point it
  // loses up to ~1e-6 without FP64.
  __host__ __device__ static bool near_degenerate(int d, const S* U, S gamma) {
    const S rho = U[0];
    const S a2 = qdiv(gamma * pressure(U, gamma), rho);
    const S bn2 = qdiv(U[5 + d] * U[5 + d], rho);
    const S bt2 = qdiv(U[5] * U[5] + U[6] * U[6] + U[7] * U[7], rho) - bn2;
    const S tot = a2 + bn2 + bt2;
    const S disc2 = sq(a2 - bn2) + bt2 * (S(2) * a2 + S(2) * bn2 + bt2);
    return disc2 < S(1e-4) * tot * tot;
  }

  // Wave speeds and Roe-Balsara normalization of one direction, in precision R.
  template <class R>
  __host__ __device__ static void eigenstructure(R rho, R p, R Bn, R By, R Bz, R gamma, R* out) {
    const R irho = qrcp(rho);
    const R a2 = gamma * p * irho;
    const R bn2 = Bn * Bn * irho;
    const R bt2r = By * By + Bz * Bz;
    const R bt2 = bt2r * irho;
    const R b2 = bn2 + bt2;
    const R disc = qsqrt(sq(a2 - bn2) + bt2 * (R(2) * a2 + R(2) * bn2 + bt2));
    const R cf2 = R(0.5) * (a2 + b2 + disc);
    const R cs2 = cf2 > R(0) ? qdiv(a2 * bn2, cf2) : R(0);
    R af, as, by, bz;
    if (disc > R(0)) {
      const R diff = a2 - b2;
      const R nf = diff >= R(0) ? R(0.5) * (diff + disc) : qdiv(R(2) * a2 * bt2, disc - diff);
      const R ns = diff <= R(0) ? R(0.5) * (disc - diff) : qdiv(R(2) * a2 * bt2, disc + diff);
      af = qsqrt(fmin(R(1), fmax(R(0), qdiv(nf, disc))));
      as = qsqrt(fmin(R(1), fmax(R(0), qdiv(ns, disc))));
    } else {
      af = R(1);
      as = R(0);
    }
    if (bt2r > R(0)) {
      const R ibt = qrcp(qsqrt(bt2r));
      by = By * ibt;
      bz = Bz * ibt;
    } else {
      by = R(0.70710678118654752440);
      bz = R(0.70710678118654752440);
    }
    out[0] = a2;
    out[1] = qsqrt(a2);
    out[2] = qsqrt(cf2);
    out[3] = qsqrt(cs2);
    out[4] = qsqrt(bn2);
    out[5] = af;
    out[6] = as;
    out[7] = by;
    out[8] = bz;
  }

  __host__ __device__ static void split(int d, const S* Ug, const Phys& ph, S Lam, S ch, S* Fg, S* Dg) {
    const S gamma = S(ph.gamma);
    const S gm1 = gamma - S(1);
    // local frame: n = d, t1 = the other in-plane axis, t2 = z
    const int n = d, t1 = 1 - d, t2 = 2;
    const S rho = Ug[0];
    const S irho = qrcp(rho);
    const S u = Ug[1 + n] * irho, v = Ug[1 + t1] * irho, w = Ug[1 + t2] * irho;
    const S E = Ug[4];
    const S Bn = Ug[5 + n], By = Ug[5 + t1], Bz = Ug[5 + t2];
    const S psi = Ug[8];
    const S uu = u * u + v * v + w * w;
    const S BB = Bn * Bn + By * By + Bz * Bz;
    const S uB = u * Bn + v * By + w * Bz;
    const S p = gm1 * (E - S(0.5) * rho * uu - S(0.5) * BB);
    const S pt = p + S(0.5) * BB;
    // flux in the local frame
    S F[9];
    F[0] = rho * u;
    F[1] = rho * u * u + pt - Bn * Bn;
    F[2] = rho * u * v - Bn * By;
    F[3] = rho * u * w - Bn * Bz;
    F[4] = (E + pt) * u - uB * Bn;
    F[5] = psi;
    F[6] = u * By - Bn * v;
    F[7] = u * Bz - Bn * w;
    F[8] = ch * ch * Bn;
    // wave speeds and Roe-Balsara normalization; in FP32 the directions whose
    // speeds nearly coincide get this eigenstructure in FP64
    Waves W;
    W.rho = rho;
    W.sr = qsqrt(rho);
    S eg[9];
    if (sizeof(S) == 4 && near_degenerate(d, Ug, gamma)) {
      double e64[9];
      eigenstructure<double>(double(rho), double(p), double(Bn), double(By), double(Bz), double(gamma), e64);
      for (int i = 0; i < 9; ++i) eg[i] = S(e64[i]);
    } else {
      eigenstructure<S>(rho, p, Bn, By, Bz, gamma, eg);
    }
    W.a2 = eg[0];
    W.a = eg[1];
    W.cf = eg[2];
    W.cs = eg[3];
    const S ca = eg[4];
    W.af = eg[5];
    W.as = eg[6];
    W.by = eg[7];
    W.bz = eg[8];
    W.sgn = Bn >= S(0) ? S(1) : S(-1);
    // speeds (f-, a-, s-, e, s+, a+, f+)
    S lam[7] = {u - W.cf, u - ca, u - W.cs, u, u + W.cs, u + ca, u + W.cf};
    const S L = ph.alpha_local ? fmax(fmax(fabs(lam[0]), fabs(lam[6])), ch) : Lam;
    const S hk = L > S(0) ? qdiv(S(0.5 * ph.k), L) : S(0);
    // primitive images of the seven-wave flux and of the B_n column of the Jacobian
    S xF[7], xC[7];
    xF[0] = F[0];
    xF[1] = (F[1] - u * F[0]) * irho;
    xF[2] = (F[2] - v * F[0]) * irho;
    xF[3] = (F[3] - w * F[0]) * irho;
    xF[4] = gm1 * (F[4] + S(0.5) * uu * F[0] - (u * F[1] + v * F[2] + w * F[3]) - By * F[6] - Bz * F[7]);
    xF[5] = F[6];
    xF[6] = F[7];
    xC[0] = S(0);
    xC[1] = -gamma * Bn * irho;
    xC[2] = -By * irho;
    xC[3] = -Bz * irho;
    xC[4] = gm1 * (v * By + w * Bz);
    xC[5] = -v;
    xC[6] = -w;
    S cF[7], cC[7], cD[7];
    project(W, xF, cF);
    project(W, xC, cC);
    const S qp = S(0.5) * (psi + ch * Bn), qm = S(0.5) * (psi - ch * Bn);
    const S bcp = beta_w(ch, hk, ph.kinf), bcm = beta_w(-ch, hk, ph.kinf);
    for (int j = 0; j < 7; ++j) {
      const S bj = beta_w(lam[j], hk, ph.kinf);
      const S sj = beta_dd(lam[j], bj, ch, bcp, hk, ph.kinf) * qp + beta_dd(lam[j], bj, -ch, bcm, hk, ph.kinf) * qm;
      cD[j] = bj * cF[j] + sj * cC[j];
    }
    S y[7];
    combine(W, cD, y);
    // back to conserved variables (B_n fixed in the seven-wave block)
    S D[9];
    D[0] = y[0];
    D[1] = u * y[0] + rho * y[1];
    D[2] = v * y[0] + rho * y[2];
    D[3] = w * y[0] + rho * y[3];
    D[4] = qdiv(y[4], gm1) + S(0.5) * uu * y[0] + rho * (u * y[1] + v * y[2] + w * y[3]) + By * y[5] + Bz * y[6];
    D[6] = y[5];
    D[7] = y[6];
    const S eta = bcp * ch;
    D[5] = eta * Bn;
    D[8] = eta * psi;
    // scatter from the local frame
    const int perm[3] = {n, t1, t2};
    Fg[0] = F[0];
    Dg[0] = D[0];
    for (int kk = 0; kk < 3; ++kk) {
      Fg[1 + perm[kk]] = F[1 + kk];
      Dg[1 + perm[kk]] = D[1 + kk];
      Fg[5 + perm[kk]] = F[5 + kk];
      Dg[5 + perm[kk]] = D[5 + kk];
    }
    Fg[4] = F[4];
    Dg[4] = D[4];
    Fg[8] = F[8];
    Dg[8] = D[8];
  }
};

// ---------------------------------------------------------------------------
// Equilibrium populations from U and the per-direction (F, D).
// 1D order (+xi, 0, -xi); 2D order (+x, -x, 0, +y, -y) (Sec. 3.1, Sec. 3.4).
// With F+ = F/2 + D and F- = F/2 - D per direction:
//   moving populations  f = c U + F+/xi  (along +d)  and  f = c U - F-/xi  (along -d),
//   rest population     f = (1 - 2 D c) U - sum_d (F+ - F-)/xi   (D = lattice dimension).
// ---------------------------------------------------------------------------
template <int KIND, int DIM, class S>
struct Equilibrium {
  using C = Cell<KIND, DIM, S>;
  static constexpr int P = C::P;
  static constexpr int Q = DIM == 1 ? 3 : 5;
  // feq[q][v]
  __host__ __device__ static void eval(const S* U, const Phys& ph, S ixi, S Lam, S ch, S (*feq)[C::P]) {
    const S c = S(ph.c);
    if (DIM == 1) {
      S F[P], D[P];
      C::split(0, U, ph, Lam, ch, F, D);
      for (int v = 0; v < P; ++v) {
        const S Fp = S(0.5) * F[v] + D[v];
        const S Fm = S(0.5) * F[v] - D[v];
        feq[0][v] = c * U[v] + Fp * ixi;
        feq[1][v] = (S(1) - S(2) * c) * U[v] - (Fp - Fm) * ixi;
        feq[2][v] = c * U[v] - Fm * ixi;
      }
    } else {
      S F1[P], D1[P], F2[P], D2[P];
      C::split(0, U, ph, Lam, ch, F1, D1);
      C::split(1, U, ph, Lam, ch, F2, D2);
      for (int v = 0; v < P; ++v) {
        const S F1p = S(0.5) * F1[v] + D1[v], F1m = S(0.5) * F1[v] - D1[v];
        const S F2p = S(0.5) * F2[v] + D2[v], F2m = S(0.5) * F2[v] - D2[v];
        feq[0][v] = c * U[v] + F1p * ixi;
        feq[1][v] = c * U[v] - F1m * ixi;
        feq[2][v] = (S(1) - S(4) * c) * U[v] - (F1p + F2p - F1m - F2m) * ixi;
        feq[3][v] = c * U[v] + F2p * ixi;
        feq[4][v] = c * U[v] - F2m * ixi;
      }
    }
  }

  // 2D: the two equilibria moving along axis d (+d into fplus, -d into
  // fminus), needing only that direction's split; the same expressions as
  // eval, so the results are bitwise those of eval.
  __host__ __device__ static void eval_axis(const S* U, const Phys& ph, S ixi, S Lam, S ch, int d, S* fplus,
                                            S* fminus) {
    const S c = S(ph.c);
    S F[P], D[P];
    C::split(d, U, ph, Lam, ch, F, D);
    for (int v = 0; v < P; ++v) {
      const S Fp = S(0.5) * F[v] + D[v], Fm = S(0.5) * F[v] - D[v];
      fplus[v] = c * U[v] + Fp * ixi;
      fminus[v] = c * U[v] - Fm * ixi;
    }
  }
};

}  // namespace vklb
