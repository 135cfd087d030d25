// Device helpers shared by the step kernels and the adjoint kernels:
// periodic wrap, the eight-lane DPP sum, the error flag, Landau matching of
// a 3x3 (tau, x, y) tensor and the EoS evaluation at lambda = eps - B.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "lb_common.hpp"

namespace lbmi {

// Periodic index for i within two of [0, n), n >= 1 (two corrections on
// each side cover n = 1); compare-and-select, no integer division.
__device__ __forceinline__ int wrap(int i, int n) {
  i = i < 0 ? i + n : i;
  i = i < 0 ? i + n : i;
  i = i >= n ? i - n : i;
  i = i >= n ? i - n : i;
  return i;
}
// The same for i within two of [0, n) where one correction on each side
// suffices for every n >= 2 (n = 1 has the single index 0).
__device__ __forceinline__ int wrap_near(int i, int n) {
  if (n == 1) return 0;
  i = i < 0 ? i + n : i;
  return i >= n ? i - n : i;
}
// The stage kernels' choice: wrap_near for FP32, wrap for FP64 (whose
// register allocation at one or two waves per SIMD was tuned with it).
template <typename R>
__device__ __forceinline__ int wrap_s(int i, int n) {
  if constexpr (sizeof(R) == 4) return wrap_near(i, n);
  else return wrap(i, n);
}

// Sum over the eight lanes of a site (lanes 8s .. 8s + 7) with DPP moves:
// swap neighbours, swap pairs, then mirror within the eight.  Every lane
// ends with the same bits (each step adds two equal-rank partial sums, and
// floating-point addition is commutative).
__device__ __forceinline__ int dpp8(int x, int step) {
  switch (step) {
    case 0: return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    case 1: return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    default: return __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false); // row_half_mirror
  }
}
__device__ __forceinline__ float sum8(float v) {
#pragma unroll
  for (int st = 0; st < 3; ++st) v += __int_as_float(dpp8(__float_as_int(v), st));
  return v;
}
__device__ __forceinline__ double sum8(double v) {
#pragma unroll
  for (int st = 0; st < 3; ++st) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)dpp8((int)(uint32_t)b, st), hi = (uint32_t)dpp8((int)(uint32_t)(b >> 32), st);
    v += __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  }
  return v;
}

__device__ __forceinline__ void flag(int* err, int bit) { atomicOr(err, bit); }

// Landau matching (eq. (sanity)) of the 3x3 (tau, x, y) block.  t = {Ttt, Ttx,
// Tty, Txx, Txy, Tyy}.  lambda is the largest root of det(lambda - T g), by
// Newton from T^{tau tau} (an upper bound, reached monotonically from
// above); u is the null vector of T g - lambda (a cross product of two rows),
// normalised to u.u = 1, u^tau > 0.
__device__ inline bool landau3(const double t[6], double* lam_out, double u[3]) {
  const double t00 = t[0], t01 = t[1], t02 = t[2], t11 = t[3], t12 = t[4], t22 = t[5];
  const double c2 = t00 - t11 - t22;
  const double c1 = (t01 * t01 - t00 * t11) + (t02 * t02 - t00 * t22) + (t11 * t22 - t12 * t12);
  const double c0 = t00 * (t11 * t22 - t12 * t12) - t01 * (t01 * t22 - t12 * t02) + t02 * (t01 * t12 - t11 * t02);
  // start: the ideal-fluid value T00 - |T0i|^2 / (T00 + (Txx + Tyy)/2), exact
  // for isotropic transverse pressure; above the inflection point c2/3 of the
  // cubic Newton converges to the largest root (after at most one overshoot),
  // otherwise start from the upper bound T00
  double lam = t00 - (t01 * t01 + t02 * t02) / (t00 + 0.5 * (t11 + t22));
  if (!(lam > c2 * (1.0 / 3.0)) || !(lam <= t00)) lam = t00;
  for (int it = 0; it < 40; ++it) {
    const double p = ((lam - c2) * lam + c1) * lam - c0;
    const double dp = (3.0 * lam - 2.0 * c2) * lam + c1;
    // Newton step; the update needs no correctly rounded quotient (the
    // residual p is evaluated exactly), so the hardware reciprocal serves
    const double d = p * __builtin_amdgcn_rcp(dp);
    lam -= d;
    if (!(fabs(d) > 4e-16 * fabs(lam))) break;
  }
  const double r0[3] = {t00 - lam, -t01, -t02};
  const double r1[3] = {t01, -t11 - lam, -t12};
  const double r2[3] = {t02, -t12, -t22 - lam};
  double c[3][3];
  c[0][0] = r0[1] * r1[2] - r0[2] * r1[1];
  c[0][1] = r0[2] * r1[0] - r0[0] * r1[2];
  c[0][2] = r0[0] * r1[1] - r0[1] * r1[0];
  c[1][0] = r0[1] * r2[2] - r0[2] * r2[1];
  c[1][1] = r0[2] * r2[0] - r0[0] * r2[2];
  c[1][2] = r0[0] * r2[1] - r0[1] * r2[0];
  c[2][0] = r1[1] * r2[2] - r1[2] * r2[1];
  c[2][1] = r1[2] * r2[0] - r1[0] * r2[2];
  c[2][2] = r1[0] * r2[1] - r1[1] * r2[0];
  int best = 0;
  double bn = -1.0;
  for (int i = 0; i < 3; ++i) {
    const double n2 = c[i][0] * c[i][0] + c[i][1] * c[i][1] + c[i][2] * c[i][2];
    if (n2 > bn) { bn = n2; best = i; }
  }
  const double mn = c[best][0] * c[best][0] - c[best][1] * c[best][1] - c[best][2] * c[best][2];
  *lam_out = lam;
  if (!(mn > 0.0) || !(lam > 0.0)) {
    u[0] = 1.0; u[1] = 0.0; u[2] = 0.0;
    return false;
  }
  double sc = 1.0 / sqrt(mn);
  if (c[best][0] < 0.0) sc = -sc;
  u[0] = c[best][0] * sc;
  u[1] = c[best][1] * sc;
  u[2] = c[best][2] * sc;
  return true;
}

// Temperature from lambda = eps_kin,eq(T) and the EoS functions there.
struct EosAt {
  double T, M_eq, beta, q, Bt4;
};

__device__ inline bool eos_from_lambda(const EosTable& tb, double lam, EosAt* o) {
  double u;
  bool ok = (lam > 0.0) && eos_invert(tb, kLnEk, tb.inv_ek, tb.gk0, tb.gk_h, tb.gk_inv_h, log(lam), &u, 2);
  if (!ok) u = (lam > 0.0 && log(lam) > tb.gk0) ? tb.u_hi : tb.u_lo;
  if (u < tb.u_lo) { u = tb.u_lo; ok = false; }
  if (u > tb.u_hi) { u = tb.u_hi; ok = false; }
  double t, w[4], dw[4];
  const int i = eos_locate(tb, u, &t);
  lagrange4(t, w, dw);
  o->T = exp(u);
  o->M_eq = eos_field(tb, i, w, kZ) * o->T;
  o->beta = eos_field(tb, i, w, kBeta);
  o->q = eos_field(tb, i, w, kQ);
  o->Bt4 = eos_field(tb, i, w, kBt4);
  return ok;
}

// Conserved particle number (eqs. (sanity), (epsp); constant mass): the
// fugacity exp(mu/T) multiplies eps - B and n alike, so T solves
// ln(eps_kin/n) = lnEk(u) - lnN(u), increasing and convex in u = ln T;
// Newton starts from the bound eps/n > 3T (above the root) and converges
// from above.  Then alpha = mu/T = ln n - lnN(u) and, for the CE rule,
// q(T, mu) = T s(T, mu)/h(T, mu) = q - alpha T n0/h.  False if lambda or
// n is not positive, the root leaves the table, or s(T, mu) <= 0.
__device__ inline bool eos_mu(const EosTable& tb, double lam, double n, EosAt* o, double* alpha) {
  bool ok = lam > 0.0 && n > 0.0 && isfinite(lam) && isfinite(n);
  const double g = ok ? log(lam / n) : 0.0;
  double u = ok ? log(lam / (3.0 * n)) : tb.u_lo;
  u = fmin(fmax(u, tb.u_lo), tb.u_hi);
  double t, w[4], dw[4], res = 0.0;
  int i = 0;
  for (int it = 0; it < 60; ++it) {
    i = eos_locate(tb, u, &t);
    lagrange4(t, w, dw);
    res = eos_field(tb, i, w, kLnEk) - eos_field(tb, i, w, kLnN) - g;
    const double der = (eos_field(tb, i, dw, kLnEk) - eos_field(tb, i, dw, kLnN)) * tb.inv_h;
    const double un = fmin(fmax(u - res / der, tb.u_lo), tb.u_hi);
    const bool done = fabs(un - u) < 1e-14;
    u = un;
    if (done) break;
  }
  i = eos_locate(tb, u, &t);
  lagrange4(t, w, dw);
  res = eos_field(tb, i, w, kLnEk) - eos_field(tb, i, w, kLnN) - g;
  ok = ok && fabs(res) < 1e-9;
  o->T = exp(u);
  o->M_eq = eos_field(tb, i, w, kZ) * o->T;
  o->beta = eos_field(tb, i, w, kBeta);
  o->Bt4 = eos_field(tb, i, w, kBt4);
  *alpha = ok ? log(n) - eos_field(tb, i, w, kLnN) : 0.0;
  o->q = eos_field(tb, i, w, kQ) - *alpha * eos_field(tb, i, w, kNq);
  ok = ok && o->q > 0.0;
  if (!ok) o->q = 1.0;
  return ok;
}

// EoS at lambda = eps - B for the stage kernels' matching, given
// g = ln(lambda) (lam_pos: lambda > 0): one read of the 4-point stencil of
// the table on the uniform g grid and a cubic interpolation of T, M_eq/T,
// beta, q and B/T^4 (the table holds the u-table's inversion at its nodes,
// so the two agree to the interpolation error).  False if lambda is outside
// the accepted range.
__device__ inline bool eos_g(const EosTable& tb, double g, bool lam_pos, EosAt* o) {
  double s = (g - tb.gg0) * tb.gg_inv_h;
  const bool ok = lam_pos && (s >= 0.0) && (s <= (double)(tb.gn - 1));
  if (!ok) s = (s > 0.0) ? (double)(tb.gn - 1) : 0.0;
  int i = (int)s;
  if (i < 1) i = 1;
  if (i > tb.gn - 3) i = tb.gn - 3;
  const double t = s - (double)i;
  double w[4], dw[4];
  lagrange4(t, w, dw);
  const double* p = tb.gpts + (size_t)(i - 1) * kGFields;
  double T = 0, z = 0, be = 0, q = 0, b4 = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double* r = p + k * kGFields;
    T += w[k] * r[kGT];
    z += w[k] * r[kGZ];
    be += w[k] * r[kGBeta];
    q += w[k] * r[kGQ];
    b4 += w[k] * r[kGBt4];
  }
  o->T = T;
  o->M_eq = z * T;
  o->beta = be;
  o->q = q;
  o->Bt4 = b4;
  return ok;
}

// u-derivatives of the interpolated EoS at the solution of eos_cell (for the
// adjoint): du/dlambda = 1/(lambda d lnEk/du), and dz/du, dbeta/du, dq/du of
// the same cubic.
struct EosDer {
  double du_dlam, dz, dbeta, dq;
};

// ---------------------------------------------------------------------------
// EoS at lambda = eps - B from one table cell: an initial u = ln T from the
// inverse table, the 4-point stencil around it loaded once, Newton on that
// cell's cubic, then M_eq/T, beta, q and B/T^4 from the same stencil.  With
// d != nullptr also the derivatives of EosDer.
__device__ inline bool eos_cell(const EosTable& tb, double lam, EosAt* o, EosDer* d = nullptr) {
  const double g = log(lam);
  double s = (g - tb.gk0) * tb.gk_inv_h;
  bool ok = (lam > 0.0) && (s >= 0.0) && (s <= (double)(tb.n_inv - 1));
  if (!ok) s = (s > 0.0) ? (double)(tb.n_inv - 1) : 0.0;
  int j = (int)s;
  if (j > tb.n_inv - 2) j = tb.n_inv - 2;
  const double u_guess = tb.inv_ek[j] + (s - (double)j) * (tb.inv_ek[j + 1] - tb.inv_ek[j]);
  double t;
  const int i = eos_locate(tb, u_guess, &t);
  double e[4], zz[4], bb[4], qq[4], b4[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double* p = tb.pts + (size_t)(i - 1 + k) * kFields;
    e[k] = p[kLnEk];
    zz[k] = p[kZ];
    bb[k] = p[kBeta];
    qq[k] = p[kQ];
    b4[k] = p[kBt4];
  }
  double w[4], dw[4];
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    lagrange4(t, w, dw);
    const double val = w[0] * e[0] + w[1] * e[1] + w[2] * e[2] + w[3] * e[3];
    const double der = dw[0] * e[0] + dw[1] * e[1] + dw[2] * e[2] + dw[3] * e[3];
    t -= (val - g) / der;
  }
  double u = tb.u0 + ((double)i + t) * tb.h;
  if (!(u >= tb.u_lo)) { u = tb.u_lo; ok = false; t = (u - tb.u0) * tb.inv_h - (double)i; }
  if (!(u <= tb.u_hi)) { u = tb.u_hi; ok = false; t = (u - tb.u0) * tb.inv_h - (double)i; }
  lagrange4(t, w, dw);
  o->T = exp(u);
  o->M_eq = (w[0] * zz[0] + w[1] * zz[1] + w[2] * zz[2] + w[3] * zz[3]) * o->T;
  o->beta = w[0] * bb[0] + w[1] * bb[1] + w[2] * bb[2] + w[3] * bb[3];
  o->q = w[0] * qq[0] + w[1] * qq[1] + w[2] * qq[2] + w[3] * qq[3];
  o->Bt4 = w[0] * b4[0] + w[1] * b4[1] + w[2] * b4[2] + w[3] * b4[3];
  if (d) {
    const double ih = tb.inv_h;
    d->du_dlam = 1.0 / (lam * ((dw[0] * e[0] + dw[1] * e[1] + dw[2] * e[2] + dw[3] * e[3]) * ih));
    d->dz = (dw[0] * zz[0] + dw[1] * zz[1] + dw[2] * zz[2] + dw[3] * zz[3]) * ih;
    d->dbeta = (dw[0] * bb[0] + dw[1] * bb[1] + dw[2] * bb[2] + dw[3] * bb[3]) * ih;
    d->dq = (dw[0] * qq[0] + dw[1] * qq[1] + dw[2] * qq[2] + dw[3] * qq[3]) * ih;
  }
  return ok;
}

}  // namespace lbmi
