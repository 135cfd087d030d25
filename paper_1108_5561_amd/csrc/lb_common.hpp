// Shared host/device definitions: EoS table layout and interpolation,
// per-context constants passed to the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmi {

constexpr double kHbarC = 0.1973269804;           // GeV fm
constexpr double kPi = 3.14159265358979323846;

// Fields of one EoS table point (uniform grid in u = ln T).
enum EosField : int {
  kLnEk = 0,    // ln(eps - B) = ln eps_kin,eq(T)        [GeV^4]
  kLnEeos = 1,  // ln eps_EoS(T)                          [GeV^4]
  kZ = 2,       // z = M(T)/T
  kBeta = 3,    // beta = dB/d(eps - B)
  kQ = 4,       // q = T tau_R / (hbar c eta/s) = T s/h (CE) or 5 (massless)
  kBt4 = 5,     // B(T)/T^4
  kLnN = 6,     // ln n0(T), the particle density at mu = 0          [GeV^3]
  kNq = 7,      // T n0/h (CE; 0 for the massless rule): q(T, mu) = q - (mu/T) kNq
  kFields = 8   // 64 bytes per point
};

// Fields of one point of the table on a uniform grid in g = ln(eps - B),
// read by the stage kernels' matching: no root finding on the device.
enum EosGField : int { kGT = 0, kGZ = 1, kGBeta = 2, kGQ = 3, kGBt4 = 4, kGFields = 8 };

struct EosTable {
  const double* pts;     // [n][kFields]
  const double* inv_ek;  // [n_inv]: u with lnEk(u) = gk0 + i gk_h
  const double* inv_ee;  // [n_inv]: u with lnEeos(u) = ge0 + i ge_h
  int32_t n, n_inv;
  double u0, h, inv_h;   // u_i = u0 + i h
  double gk0, gk_h, gk_inv_h;
  double ge0, ge_h, ge_inv_h;
  double u_lo, u_hi;     // accepted range ln T_min .. ln T_max
  const double* gpts;    // [gn][kGFields]: T, M/T, beta, q, B/T^4 at g_i = gg0 + i gg_h
  int32_t gn, gpad_;
  double gg0, gg_h, gg_inv_h;
};

// 4-point Lagrange weights on nodes -1, 0, 1, 2 at t in [0, 1), and their
// t-derivatives.
__host__ __device__ inline void lagrange4(double t, double w[4], double dw[4]) {
  const double tm1 = t - 1.0, tm2 = t - 2.0, tp1 = t + 1.0;
  w[0] = -t * tm1 * tm2 * (1.0 / 6.0);
  w[1] = tp1 * tm1 * tm2 * 0.5;
  w[2] = -tp1 * t * tm2 * 0.5;
  w[3] = tp1 * t * tm1 * (1.0 / 6.0);
  // derivatives of the cubic products
  dw[0] = -(3.0 * t * t - 6.0 * t + 2.0) * (1.0 / 6.0);
  dw[1] = (3.0 * t * t - 4.0 * t - 1.0) * 0.5;
  dw[2] = -(3.0 * t * t - 2.0 * t - 2.0) * 0.5;
  dw[3] = (3.0 * t * t - 1.0) * (1.0 / 6.0);
}

// Locate u on the grid: base index i (stencil i-1..i+2) and fraction t.
__host__ __device__ inline int eos_locate(const EosTable& tb, double u, double* t) {
  double s = (u - tb.u0) * tb.inv_h;
  int i = (int)floor(s);
  if (i < 1) i = 1;
  if (i > tb.n - 3) i = tb.n - 3;
  *t = s - (double)i;
  return i;
}

__host__ __device__ inline double eos_field(const EosTable& tb, int i, const double w[4], int f) {
  const double* p = tb.pts + (size_t)(i - 1) * kFields + f;
  return w[0] * p[0] + w[1] * p[kFields] + w[2] * p[2 * kFields] + w[3] * p[3 * kFields];
}

// Solve field(u) = g for u (field monotone increasing in u): initial guess
// from the inverse table, then Newton on the interpolant.  Returns false if g
// is outside the inverse table.
__host__ __device__ inline bool eos_invert(const EosTable& tb, int field, const double* inv, double g0,
                                           double gh, double gh_inv, double g, double* u_out,
                                           int newton_iters = 4) {
  double s = (g - g0) * gh_inv;
  if (!(s >= 0.0) || !(s <= (double)(tb.n_inv - 1))) return false;
  int j = (int)s;
  if (j > tb.n_inv - 2) j = tb.n_inv - 2;
  double f = s - (double)j;
  double u = inv[j] + f * (inv[j + 1] - inv[j]);
  double w[4], dw[4], t;
  for (int it = 0; it < newton_iters; ++it) {
    int i = eos_locate(tb, u, &t);
    lagrange4(t, w, dw);
    double val = eos_field(tb, i, w, field);
    double der = eos_field(tb, i, dw, field) * tb.inv_h;
    u -= (val - g) / der;
  }
  *u_out = u;
  (void)gh;
  return true;
}

// Per-context lattice constants in the node arithmetic type R, passed by
// value to the kernels (kernel argument space, read with scalar loads).
// NXI x NTH nodes per phi slice; eight slices (n_phi = 4).
template <typename R, int NXI, int NTH>
struct LatticeConst {
  R x[NXI];          // gamma_k = cosh xi_k
  R inv_x[NXI];      // 1/gamma_k
  R sh2[NXI];        // sinh^2 xi_k
  R sig[NXI * NTH];  // |v_perp| = sinh xi_k sin theta_j
  R sigi[NXI * NTH]; // |v_perp| / gamma
  R sig2[NXI * NTH]; // |v_perp|^2
  R vY[NXI * NTH];   // v^Y = sinh xi_k cos theta_j
  R mu2[NTH];        // cos^2 theta_j
  R w[NXI * NTH];    // w_n (the same on every phi slice)
  R wx2[NXI * NTH];  // w_n gamma^2
  R wxs[NXI * NTH];  // w_n gamma |v_perp|
  R ws2[NXI * NTH];  // w_n |v_perp|^2
  R wvY2[NXI * NTH]; // w_n (v^Y)^2
  R wx[NXI * NTH];   // w_n gamma
  R A1[NXI * NXI];   // S1 radial part
  R A2[NXI * NXI];   // S2 (radial)
  R Ath[NTH * NTH];  // S1 polar part
  R cosl[8], sinl[8];
};

// Constants of one stage-kernel launch (5 x 5 nodes per phi slice).  The
// polar nodes are mirror pairs, mu_{4-j} = -mu_j, and every per-node
// quantity the stage needs (weights, |v_perp|, gamma) is even under the
// mirror, so it is stored once per (k, p): pair p = 0 holds j = 0, 4, p = 1
// holds j = 1, 3 and p = 2 is j = 2 (mu = 0).  The Milne factor 1/tau of S1
// is folded into A1 and the polar blocks (0 for the Minkowski metric).
template <typename R>
struct StageConst {
  static constexpr int NXI = 5, NP = 3;
  R x[NXI], inv_x[NXI], sh2[NXI];
  R sig[NXI * NP];   // |v_perp|
  R sigi[NXI * NP];  // |v_perp| / gamma
  R sig2[NXI * NP];  // |v_perp|^2
  R w[NXI * NP], wx2[NXI * NP], wxs[NXI * NP], ws2[NXI * NP];  // w, w gamma^2, w gamma |v_perp|, w |v_perp|^2
  R mu2[2];          // mu_j^2 of pairs 0 and 1
  R A1[NXI * NXI];   // radial part of S1, times 1/tau
  R A2[NXI * NXI];   // S2 (radial)
  // Polar part of S1, -Ath/tau, split by the mirror: for output pair p < 2,
  // Ev[p] acts on (f_0 + f_4, f_1 + f_3, f_2) and Od[p] on (f_0 - f_4,
  // f_1 - f_3), each with the factor 1/2 of the recombination; Mid acts on
  // (f_0 + f_4, f_1 + f_3, f_2) for j = 2.
  R Ev[2][3], Od[2][2], Mid[3];
  R cosl[8], sinl[8];
  // Weak-form 3-D mass-gradient force (weak_force), per node q = k * 5 + j
  // of a slice (s = sinh xi_k, x = cosh xi_k, mu = cos theta_j):
  R fw[25];      // w_n
  R finvw[25];   // 1/w_n
  R fa[25];      // sin theta x               (radial part)
  R fb[25];      // -mu sin theta / (s x)     (polar part)
  R fc[25];      // 1 / (s sin theta x)       (azimuthal part)
  R fy[25];      // 2 s sin theta / x
  R fDxT[25];    // [k][k']: derivative of the k-th Lagrange polynomial of the radial nodes at x_k'
  R fDmT[25];    // [j][j']: the same for the polar nodes mu
  R frho0[5], frho1[5], fsig1[5];  // s/x, s^2/x, 1/s per radial node
  R fst[2];      // sin theta of polar pairs 0 and 1 (pair 2: mu = 0, sin theta = 1)
  R fmr[5];      // mu / (1 - mu^2) per polar node
  R fphi[64];    // [l][r]: the Fourier function of lane r at phi_l; lane r holds
                 // mode 0, cos 4 phi, cos phi, sin phi, cos 2 phi, sin 2 phi,
                 // cos 3 phi, sin 3 phi for r = 0 .. 7
};

}  // namespace lbmi
