// Discrete adjoint (reverse mode) of the Heun step of Sec. IV.D, FP64, for
// the differentiable form: gradients of a function of the final state with
// respect to the initial energy density e0 and to eta/s.
//
// The step differentiated is the FP64 step of the stage kernels, written out
// here per site in the canonical layout F[n][site], n = q 8 + l
// (q = k N_theta + j): for state (F, ln M) at time tau the right-hand side is
//   R0_n = A_n + S1_n/tau + F_eq,n ((u.V)/gamma r - poly_n) - (u.V)/gamma r F_n
//   X    = -beta sum w (u.V)^2 R0 / (sum w F + beta sum w (u.V)^2 (4F + S2))
//   K_n  = R0_n + X S2_n
// (streaming A, Milne term S1/tau, equilibrium with the mass-gradient force
// and BGK of eqs. (Bmilne), (newBeq), (bgk); mass evolution of eqs.
// (edchange), (masschange)), where r = 1/tau_R, u, T and M_eq come from the
// Landau matching (eq. (sanity)) of the state's own moments (eq. (emtnew))
// and the EoS inversion.  The reverse sweep of one right-hand side is one
// thread per site: a forward pass for the site sums, a second pass that
// recomputes each phi slice and propagates the adjoint through the
// collision, equilibrium, force and operator terms, the implicit-function
// adjoints of the eigenproblem and of the EoS root, and a third pass for the
// moments' adjoint.  The transposed streaming stencil and the transposed
// centred ln M gradient are gathers over the neighbours (adj_gather_kernel).
#include <hip/hip_runtime.h>

#include "../../include/lb.h"
#include "device_common.hpp"
#include "kernels.hpp"
#include "lb_common.hpp"

namespace lbmi {

namespace {

constexpr int kAdjBlock = 128;
constexpr int kQ = 25;  // nodes per phi slice
constexpr int kL = 8;   // phi slices
using LC = LatticeConst<double, 5, 5>;

__device__ __forceinline__ size_t cix(int q, int l, int site, int ns) {
  return (size_t)(q * kL + l) * (size_t)ns + (size_t)site;
}

// Upwind direction and streaming coefficients of slice l (as in the stage
// kernels: second-order upwind along +(cos phi, sin phi)).
struct SliceGeom {
  double cl, sl, ax, ay;
  int dxr, dyr;
};
__device__ __forceinline__ SliceGeom slice_geom(const LC& C, const StageArgs& a, int l) {
  SliceGeom g;
  g.cl = C.cosl[l];
  g.sl = C.sinl[l];
  g.dxr = (g.cl > 0.0) ? 1 : ((g.cl < 0.0) ? -1 : 0);
  g.dyr = (g.sl > 0.0) ? 1 : ((g.sl < 0.0) ? -1 : 0);
  g.ax = fabs(g.cl) * a.inv2dx;
  g.ay = fabs(g.sl) * a.inv2dx;
  return g;
}

// Site quantities of a state: moments, Landau matching, EoS.
struct SiteFwd {
  double m[3][3];  // sum_n w F V^a V^b, a, b in (tau, x, y)
  double M, G;     // mass and M^4/(2 pi^2)
  double lam, u[3];
  EosAt E;
  EosDer D;
  double invT, MT, rate, beta;
  double gx, gy;   // centred gradient of ln M
};

__device__ void site_fwd(const double* __restrict__ F, const double* __restrict__ lnM, int x, int y,
                         const LC& C, const EosTable& tb, const StageArgs& a, SiteFwd* s,
                         int* __restrict__ err) {
  const int ns = a.n_sites, site = y * a.nx + x;
  double p00 = 0, p01 = 0, p02 = 0, p11 = 0, p12 = 0, p22 = 0;
  for (int l = 0; l < kL; ++l) {
    double q0 = 0, q1 = 0, q2 = 0;
    for (int q = 0; q < kQ; ++q) {
      const double f = F[cix(q, l, site, ns)];
      q0 += C.wx2[q] * f;
      q1 += C.wxs[q] * f;
      q2 += C.ws2[q] * f;
    }
    const double cl = C.cosl[l], sl = C.sinl[l];
    p00 += q0;
    p01 += q1 * cl;
    p02 += q1 * sl;
    p11 += q2 * cl * cl;
    p12 += q2 * cl * sl;
    p22 += q2 * sl * sl;
  }
  s->m[0][0] = p00;
  s->m[0][1] = s->m[1][0] = p01;
  s->m[0][2] = s->m[2][0] = p02;
  s->m[1][1] = p11;
  s->m[1][2] = s->m[2][1] = p12;
  s->m[2][2] = p22;
  const double lm = lnM[site];
  s->M = exp(lm);
  s->G = s->M * s->M * s->M * s->M * (1.0 / (2.0 * kPi * kPi));
  const double tk[6] = {s->G * p00, s->G * p01, s->G * p02, s->G * p11, s->G * p12, s->G * p22};
  const bool matched = landau3(tk, &s->lam, s->u);
  const bool eos_ok = eos_cell(tb, s->lam, &s->E, &s->D);
  bool finite = true;
  for (int i = 0; i < 6; ++i) finite = finite && isfinite(tk[i]);
  if (!finite) flag(err, kErrNonfinite);
  else if (!matched) flag(err, kErrMatch);
  else if (!eos_ok) flag(err, kErrEos);
  s->invT = 1.0 / s->E.T;
  s->MT = s->M * s->invT;
  s->rate = s->E.T * a.inv_eta_hbarc / s->E.q;
  s->beta = s->E.beta;
  const int xp = wrap(x + 1, a.nx), xm = wrap(x - 1, a.nx), yp = wrap(y + 1, a.ny), ym = wrap(y - 1, a.ny);
  s->gx = (lnM[y * a.nx + xp] - lnM[y * a.nx + xm]) * a.inv2dx;
  s->gy = (lnM[yp * a.nx + x] - lnM[ym * a.nx + x]) * a.inv2dx;
}

// Per-slice forward of the right-hand side: R0 and S2 of the 25 nodes of
// slice l, and the slice's contributions to the three site sums.
struct SliceFwd {
  double f[kQ], R0[kQ], S2[kQ];
  double feq[kQ], uvg[kQ], poly[kQ];
  double Eeq[5], al[5], be[5], ga[5];
  double cu, Gl, gu;
};

__device__ void slice_fwd(const double* __restrict__ F, int x, int y, int l, const SiteFwd& s, const LC& C,
                          const StageArgs& a, SliceFwd* o, double* nsum, double* dsum, double* wsum) {
  const int ns = a.n_sites, site = y * a.nx + x;
  const SliceGeom g = slice_geom(C, a, l);
  for (int q = 0; q < kQ; ++q) o->f[q] = F[cix(q, l, site, ns)];
  // streaming (3 F_i - 4 F_{i-1} + F_{i-2}) |cos phi| / (2 dx), periodic
  const int x1 = wrap(x - g.dxr, a.nx), x2 = wrap(x - 2 * g.dxr, a.nx);
  const int y1 = wrap(y - g.dyr, a.ny), y2 = wrap(y - 2 * g.dyr, a.ny);
  const int s_x1 = y * a.nx + x1, s_x2 = y * a.nx + x2, s_y1 = y1 * a.nx + x, s_y2 = y2 * a.nx + x;
  for (int q = 0; q < kQ; ++q) {
    const double tr = 3.0 * (g.ax + g.ay) * o->f[q] - 4.0 * g.ax * F[cix(q, l, s_x1, ns)] +
                      g.ax * F[cix(q, l, s_x2, ns)] - 4.0 * g.ay * F[cix(q, l, s_y1, ns)] +
                      g.ay * F[cix(q, l, s_y2, ns)];
    o->R0[q] = -C.sigi[q] * tr;
  }
  // S2 (radial) and, for the Milne metric, S1/tau
  const bool milne = a.metric == LB_METRIC_MILNE;
  const double itau = 1.0 / a.tau;
  for (int k = 0; k < 5; ++k)
    for (int j = 0; j < 5; ++j) {
      double s2 = 0, s1r = 0, s1p = 0;
      for (int kp = 0; kp < 5; ++kp) {
        s2 += C.A2[k * 5 + kp] * o->f[kp * 5 + j];
        s1r += C.A1[k * 5 + kp] * o->f[kp * 5 + j];
      }
      for (int jp = 0; jp < 5; ++jp) s1p += C.Ath[j * 5 + jp] * o->f[k * 5 + jp];
      o->S2[k * 5 + j] = s2;
      if (milne) o->R0[k * 5 + j] += (C.mu2[j] * s1r - s1p) * itau;
    }
  const double ut = s.u[0], ux = s.u[1], uy = s.u[2];
  o->cu = ux * g.cl + uy * g.sl;
  o->Gl = s.gx * g.cl + s.gy * g.sl;
  o->gu = s.gx * ux + s.gy * uy;
  const double Meq = s.E.M_eq, M = s.M;
  for (int k = 0; k < 5; ++k) {
    o->Eeq[k] = sqrt(Meq * Meq + M * M * C.sh2[k]);
    o->al[k] = s.MT * o->Gl * ut * M * C.x[k] / o->Eeq[k];
    o->be[k] = s.MT * o->Gl * o->cu * C.inv_x[k];
    o->ga[k] = s.MT * o->gu * C.inv_x[k];
  }
  for (int q = 0; q < kQ; ++q) {
    const int k = q / 5;
    const double sg = C.sig[q];
    o->feq[q] = a.Z * exp((sg * M * o->cu - ut * o->Eeq[k]) * s.invT);
    o->uvg[q] = ut - C.sigi[q] * o->cu;
    o->poly[q] = o->al[k] * sg - o->be[k] * C.sig2[q] - o->ga[k];
    const double ru = s.rate * o->uvg[q];
    o->R0[q] += o->feq[q] * (ru - o->poly[q]) - ru * o->f[q];
    const double wuv2 = C.wx2[q] * o->uvg[q] * o->uvg[q];
    *nsum += wuv2 * o->R0[q];
    *dsum += wuv2 * (4.0 * o->f[q] + o->S2[q]);
    *wsum += C.w[q] * o->f[q];
  }
}

// ---------------------------------------------------------------------------
// One Heun stage of the FP64 step in the canonical layout: stage 0 writes
// Fout = Fin + dtau K(Fin), stage 1 Fout = (Fbase + Fin)/2 + dtau/2 K(Fin);
// ln M likewise with X.
__global__ __launch_bounds__(kAdjBlock) void adj_fwd_kernel(const double* __restrict__ Fin,
                                                            const double* __restrict__ Lin,
                                                            const double* __restrict__ Fbase,
                                                            const double* __restrict__ Lbase,
                                                            double* __restrict__ Fout, double* __restrict__ Lout,
                                                            int stage, const LC C, const EosTable tb,
                                                            const StageArgs a, int* __restrict__ err) {
  const int site = blockIdx.x * kAdjBlock + threadIdx.x;
  if (site >= a.n_sites) return;
  const int x = site % a.nx, y = site / a.nx, ns = a.n_sites;
  SiteFwd s;
  site_fwd(Fin, Lin, x, y, C, tb, a, &s, err);
  double nsum = 0, dsum = 0, wsum = 0;
  for (int l = 0; l < kL; ++l) {
    SliceFwd o;
    slice_fwd(Fin, x, y, l, s, C, a, &o, &nsum, &dsum, &wsum);
  }
  const double X = -s.beta * nsum / (wsum + s.beta * dsum);
  for (int l = 0; l < kL; ++l) {
    double d0 = 0, d1 = 0, d2 = 0;
    SliceFwd o;
    slice_fwd(Fin, x, y, l, s, C, a, &o, &d0, &d1, &d2);
    for (int q = 0; q < kQ; ++q) {
      const double K = o.R0[q] + X * o.S2[q];
      const size_t i = cix(q, l, site, ns);
      Fout[i] = stage == 0 ? o.f[q] + a.dtau * K : 0.5 * (Fbase[i] + o.f[q]) + 0.5 * a.dtau * K;
    }
  }
  const double lm = Lin[site];
  Lout[site] = stage == 0 ? lm + a.dtau * X : 0.5 * (Lbase[site] + lm) + 0.5 * a.dtau * X;
}

// ---------------------------------------------------------------------------
// Reverse sweep of one right-hand side at state (F, ln M), time a.tau, with
// K_bar = scale seedF and X_bar = scale seedL.  Writes (accumulate = 0) or
// adds (accumulate = 1) the site-local part of the state's adjoint into
// (outF, outL) and the site's eta/s adjoint into eta_part; writes R0_bar
// (for the transposed streaming) into Rb and the ln M gradient adjoint into
// gb[2][site].
__global__ __launch_bounds__(kAdjBlock) void adj_local_kernel(
    const double* __restrict__ F, const double* __restrict__ Lm, const double* __restrict__ seedF,
    const double* __restrict__ seedL, double scale, double* __restrict__ outF, double* __restrict__ outL,
    double* __restrict__ Rb, double* __restrict__ gb, double* __restrict__ eta_part, int accumulate,
    const LC C, const EosTable tb, const StageArgs a, int* __restrict__ err) {
  const int site = blockIdx.x * kAdjBlock + threadIdx.x;
  if (site >= a.n_sites) return;
  const int x = site % a.nx, y = site / a.nx, ns = a.n_sites;
  SiteFwd s;
  site_fwd(F, Lm, x, y, C, tb, a, &s, err);
  // pass 1: the site sums and sum_n K_bar S2
  double nsum = 0, dsum = 0, wsum = 0, kS2 = 0;
  for (int l = 0; l < kL; ++l) {
    SliceFwd o;
    slice_fwd(F, x, y, l, s, C, a, &o, &nsum, &dsum, &wsum);
    for (int q = 0; q < kQ; ++q) kS2 += scale * seedF[cix(q, l, site, ns)] * o.S2[q];
  }
  const double beta = s.beta, D = wsum + beta * dsum, X = -beta * nsum / D;
  const double Xb = scale * seedL[site] + kS2;
  const double nb = -beta * Xb / D;           // d/d nsum
  const double Db = -X * Xb / D;              // d/d (wsum + beta dsum)
  double betab = -nsum * Xb / D + Db * dsum;  // d/d beta
  const double wsb = Db, dsb = beta * Db;
  // pass 2: per slice, the adjoint of R0, S2 and of everything they use
  double utb = 0, uxb = 0, uyb = 0, Mb = 0, invTb = 0, MTb = 0, rateb = 0, Meqb = 0, gxb = 0, gyb = 0;
  const double ut = s.u[0], ux = s.u[1], uy = s.u[2], M = s.M, Meq = s.E.M_eq;
  const bool milne = a.metric == LB_METRIC_MILNE;
  const double itau = 1.0 / a.tau;
  for (int l = 0; l < kL; ++l) {
    double d0 = 0, d1 = 0, d2 = 0;
    SliceFwd o;
    slice_fwd(F, x, y, l, s, C, a, &o, &d0, &d1, &d2);
    const SliceGeom g = slice_geom(C, a, l);
    double R0b[kQ], S2b[kQ], fb[kQ];
    double cub = 0, Glb = 0, gub = 0;
    double alb[5] = {0, 0, 0, 0, 0}, beb[5] = {0, 0, 0, 0, 0}, gab[5] = {0, 0, 0, 0, 0};
    double Eeqb[5] = {0, 0, 0, 0, 0};
    for (int q = 0; q < kQ; ++q) {
      const int k = q / 5;
      const double Kb = scale * seedF[cix(q, l, site, ns)];
      const double uv = o.uvg[q], wuv2 = C.wx2[q] * uv * uv;
      R0b[q] = Kb + wuv2 * nb;
      S2b[q] = X * Kb + wuv2 * dsb;
      const double ru = s.rate * uv;
      fb[q] = 4.0 * wuv2 * dsb + C.w[q] * wsb - ru * R0b[q];
      double uvb = 2.0 * C.wx2[q] * uv * ((4.0 * o.f[q] + o.S2[q]) * dsb + o.R0[q] * nb) +
                   s.rate * (o.feq[q] - o.f[q]) * R0b[q];
      rateb += uv * (o.feq[q] - o.f[q]) * R0b[q];
      const double feqb = (ru - o.poly[q]) * R0b[q];
      const double polyb = -o.feq[q] * R0b[q];
      alb[k] += C.sig[q] * polyb;
      beb[k] -= C.sig2[q] * polyb;
      gab[k] -= polyb;
      // F_eq = Z exp((sig M cu - ut E_eq) / T)
      const double e = o.feq[q] * feqb, sg = C.sig[q];
      Mb += e * sg * o.cu * s.invT;
      cub += e * sg * M * s.invT;
      invTb += e * (sg * M * o.cu - ut * o.Eeq[k]);
      utb -= e * o.Eeq[k] * s.invT;
      Eeqb[k] -= e * ut * s.invT;
      // (u.V)/gamma = ut - (|v_perp|/gamma) cu
      utb += uvb;
      cub -= C.sigi[q] * uvb;
      Rb[cix(q, l, site, ns)] = R0b[q];
    }
    // transposed operators: S2 = A2 f, S1 = (mu^2 A1 f - Ath f)/tau
    for (int k = 0; k < 5; ++k)
      for (int j = 0; j < 5; ++j) {
        double acc = 0;
        for (int kk = 0; kk < 5; ++kk) {
          acc += C.A2[kk * 5 + k] * S2b[kk * 5 + j];
          if (milne) acc += C.mu2[j] * C.A1[kk * 5 + k] * R0b[kk * 5 + j] * itau;
        }
        if (milne)
          for (int jj = 0; jj < 5; ++jj) acc -= C.Ath[jj * 5 + j] * R0b[k * 5 + jj] * itau;
        fb[k * 5 + j] += acc;
      }
    for (int k = 0; k < 5; ++k) {
      const double c = C.x[k] / o.Eeq[k];
      // al = MT Gl ut M x / E_eq
      MTb += alb[k] * o.Gl * ut * M * c;
      Glb += alb[k] * s.MT * ut * M * c;
      utb += alb[k] * s.MT * o.Gl * M * c;
      Mb += alb[k] * s.MT * o.Gl * ut * c;
      Eeqb[k] -= alb[k] * o.al[k] / o.Eeq[k];
      // be = MT Gl cu / x, ga = MT gu / x
      MTb += beb[k] * o.Gl * o.cu * C.inv_x[k] + gab[k] * o.gu * C.inv_x[k];
      Glb += beb[k] * s.MT * o.cu * C.inv_x[k];
      cub += beb[k] * s.MT * o.Gl * C.inv_x[k];
      gub += gab[k] * s.MT * C.inv_x[k];
      // E_eq = sqrt(M_eq^2 + M^2 sinh^2 xi)
      Meqb += Eeqb[k] * Meq / o.Eeq[k];
      Mb += Eeqb[k] * M * C.sh2[k] / o.Eeq[k];
    }
    // cu = u_perp.(cos, sin), Gl = grad ln M.(cos, sin), gu = grad ln M.u_perp
    uxb += cub * g.cl + gub * s.gx;
    uyb += cub * g.sl + gub * s.gy;
    gxb += Glb * g.cl + gub * ux;
    gyb += Glb * g.sl + gub * uy;
    for (int q = 0; q < kQ; ++q) {
      const size_t i = cix(q, l, site, ns);
      outF[i] = accumulate ? outF[i] + fb[q] : fb[q];
    }
  }
  // site chain: M/T, 1/T, r = T/(q hbar c eta/s), then u = ln T
  Mb += MTb * s.invT;
  invTb += MTb * M;
  const double T = s.E.T, qv = s.E.q;
  double Tb = -invTb * s.invT * s.invT + rateb * a.inv_eta_hbarc / qv;
  const double qb = -rateb * s.rate / qv;
  const double etab = -rateb * s.rate * a.inv_eta_hbarc * kHbarC;  // dr/d(eta/s) = -r/(eta/s)
  const double z = Meq / T;
  const double uub = Tb * T + Meqb * (s.D.dz * T + z * T) + betab * s.D.dbeta + qb * s.D.dq;
  const double lamb = uub * s.D.du_dlam;
  // eigenproblem A u = lambda u, A = T_kin g, u.u = 1: with u_low = g u and
  // B = A - lambda + u u_low^T, solve B^T w = u_bar - (u_bar.u) u_low; then
  // T_kin_bar = -w u_low^T + (w.u + lambda_bar) u_low u_low^T
  const double ub[3] = {utb, uxb, uyb};
  const double ul[3] = {s.u[0], -s.u[1], -s.u[2]};
  const double gsg[3] = {1.0, -1.0, -1.0};
  const double al_ = ub[0] * s.u[0] + ub[1] * s.u[1] + ub[2] * s.u[2];
  double rhs[3], Bt[3][3];
  for (int i = 0; i < 3; ++i) rhs[i] = ub[i] - al_ * ul[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)  // Bt[j][i] = B[i][j]
      Bt[j][i] = s.G * s.m[i][j] * gsg[j] - (i == j ? s.lam : 0.0) + s.u[i] * ul[j];
  // Cramer's rule
  const double det = Bt[0][0] * (Bt[1][1] * Bt[2][2] - Bt[1][2] * Bt[2][1]) -
                     Bt[0][1] * (Bt[1][0] * Bt[2][2] - Bt[1][2] * Bt[2][0]) +
                     Bt[0][2] * (Bt[1][0] * Bt[2][1] - Bt[1][1] * Bt[2][0]);
  double w[3];
  for (int c = 0; c < 3; ++c) {
    double Mx[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Mx[i][j] = (j == c) ? rhs[i] : Bt[i][j];
    w[c] = (Mx[0][0] * (Mx[1][1] * Mx[2][2] - Mx[1][2] * Mx[2][1]) -
            Mx[0][1] * (Mx[1][0] * Mx[2][2] - Mx[1][2] * Mx[2][0]) +
            Mx[0][2] * (Mx[1][0] * Mx[2][1] - Mx[1][1] * Mx[2][0])) / det;
  }
  const double wu = w[0] * s.u[0] + w[1] * s.u[1] + w[2] * s.u[2] + lamb;
  double mb[3][3], Gb = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double tb_ = -w[i] * ul[j] + wu * ul[i] * ul[j];
      mb[i][j] = s.G * tb_;
      Gb += tb_ * s.m[i][j];
    }
  Mb += Gb * 4.0 * s.G / M;
  // pass 3: the moments' adjoint, m^{ab} = sum_n w F V^a V^b
  for (int l = 0; l < kL; ++l) {
    const double cl = C.cosl[l], sl = C.sinl[l];
    const double c00 = mb[0][0], c01 = (mb[0][1] + mb[1][0]) * cl + (mb[0][2] + mb[2][0]) * sl;
    const double c11 = mb[1][1] * cl * cl + (mb[1][2] + mb[2][1]) * cl * sl + mb[2][2] * sl * sl;
    for (int q = 0; q < kQ; ++q) {
      const size_t i = cix(q, l, site, ns);
      outF[i] += c00 * C.wx2[q] + c01 * C.wxs[q] + c11 * C.ws2[q];
    }
  }
  const double lb = Mb * M;  // M = exp(ln M)
  outL[site] = accumulate ? outL[site] + lb : lb;
  gb[site] = gxb;
  gb[ns + site] = gyb;
  eta_part[site] = accumulate ? eta_part[site] + etab : etab;
}

// Transposed streaming stencil and transposed centred ln M gradient:
// outF_n(s) += sum over the sites s' whose stencil reads s of the stencil
// weight times Rb_n(s'); outL(s) += (gb_x(s - 1) - gb_x(s + 1) + ...)/(2 dx).
__global__ __launch_bounds__(kAdjBlock) void adj_gather_kernel(const double* __restrict__ Rb,
                                                               const double* __restrict__ gb,
                                                               double* __restrict__ outF,
                                                               double* __restrict__ outL, const LC C,
                                                               const StageArgs a) {
  const int site = blockIdx.x * kAdjBlock + threadIdx.x;
  if (site >= a.n_sites) return;
  const int x = site % a.nx, y = site / a.nx, ns = a.n_sites;
  for (int l = 0; l < kL; ++l) {
    const SliceGeom g = slice_geom(C, a, l);
    const int s1 = y * a.nx + wrap(x + g.dxr, a.nx), s2 = y * a.nx + wrap(x + 2 * g.dxr, a.nx);
    const int s3 = wrap(y + g.dyr, a.ny) * a.nx + x, s4 = wrap(y + 2 * g.dyr, a.ny) * a.nx + x;
    for (int q = 0; q < kQ; ++q) {
      const double t = 3.0 * (g.ax + g.ay) * Rb[cix(q, l, site, ns)] - 4.0 * g.ax * Rb[cix(q, l, s1, ns)] +
                       g.ax * Rb[cix(q, l, s2, ns)] - 4.0 * g.ay * Rb[cix(q, l, s3, ns)] +
                       g.ay * Rb[cix(q, l, s4, ns)];
      outF[cix(q, l, site, ns)] -= C.sigi[q] * t;
    }
  }
  const int xm = y * a.nx + wrap(x - 1, a.nx), xp = y * a.nx + wrap(x + 1, a.nx);
  const int ym = wrap(y - 1, a.ny) * a.nx + x, yp = wrap(y + 1, a.ny) * a.nx + x;
  outL[site] += (gb[xm] - gb[xp] + gb[ns + ym] - gb[ns + yp]) * a.inv2dx;
}

// y += c x and, if z != nullptr, z *= cz, over n values.
__global__ __launch_bounds__(256) void adj_axpy_kernel(double* __restrict__ y, const double* __restrict__ x,
                                                       double c, double* __restrict__ z, double cz, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  y[i] += c * x[i];
  if (z) z[i] *= cz;
}

// *out += sum of v[0..n) (one block, fixed order: deterministic).
__global__ __launch_bounds__(256) void adj_sum_kernel(const double* __restrict__ v, int n,
                                                      double* __restrict__ out) {
  __shared__ double part[256];
  double acc = 0;
  for (int i = threadIdx.x; i < n; i += 256) acc += v[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += part[0];
}

// Adjoint of the initial state of lb_init: T0 from eps_EoS(T0) = e0, M =
// z(T0) T0, F_n = Z exp(-z (u^tau gamma - u_perp.v_perp)) (z = M/T0, flow
// held fixed).  grad_e0 = d/d e0 of (adjF . F + adjL . ln M).
__global__ __launch_bounds__(kAdjBlock) void adj_init_kernel(const double* __restrict__ e0,
                                                             const double* __restrict__ ux0,
                                                             const double* __restrict__ uy0,
                                                             const double* __restrict__ aF,
                                                             const double* __restrict__ aL,
                                                             double* __restrict__ grad_e0, const LC C,
                                                             const EosTable tb, const StageArgs a,
                                                             int* __restrict__ err) {
  const int site = blockIdx.x * kAdjBlock + threadIdx.x;
  if (site >= a.n_sites) return;
  const int ns = a.n_sites;
  const double e = e0[site] * (kHbarC * kHbarC * kHbarC);
  const double vx = ux0 ? ux0[site] : 0.0, vy = uy0 ? uy0[site] : 0.0;
  double uu = tb.u_lo;
  if (!(e > 0.0) || !eos_invert(tb, kLnEeos, tb.inv_ee, tb.ge0, tb.ge_h, tb.ge_inv_h, log(e), &uu)) {
    flag(err, kErrEos);
    grad_e0[site] = 0.0;
    return;
  }
  double t, w[4], dw[4];
  const int i = eos_locate(tb, uu, &t);
  lagrange4(t, w, dw);
  const double z = eos_field(tb, i, w, kZ);
  const double dz = eos_field(tb, i, dw, kZ) * tb.inv_h;
  const double dlnE = eos_field(tb, i, dw, kLnEeos) * tb.inv_h;  // d ln eps_EoS / du
  const double ut = sqrt(1.0 + vx * vx + vy * vy);
  double zb = 0;
  for (int l = 0; l < kL; ++l) {
    const double cu = vx * C.cosl[l] + vy * C.sinl[l];
    for (int q = 0; q < kQ; ++q) {
      const double h = ut * C.x[q / 5] - cu * C.sig[q];
      const double f = a.Z * exp(-z * h);
      zb += aF[cix(q, l, site, ns)] * f * (-h);
    }
  }
  // ln M = ln z + u
  zb += aL[site] / z;
  const double ub = aL[site] + zb * dz;
  grad_e0[site] = ub / (dlnE * e0[site]);
}

dim3 sites_grid(int n) { return dim3((unsigned)((n + kAdjBlock - 1) / kAdjBlock)); }

}  // namespace

hipError_t launch_adj_stage_fwd(const double* Fin, const double* Lin, const double* Fbase, const double* Lbase,
                                double* Fout, double* Lout, int stage, const void* lc, const EosTable& tb,
                                const StageArgs& a, int* err, hipStream_t s) {
  hipLaunchKernelGGL(adj_fwd_kernel, sites_grid(a.n_sites), dim3(kAdjBlock), 0, s, Fin, Lin, Fbase, Lbase, Fout,
                     Lout, stage, *static_cast<const LC*>(lc), tb, a, err);
  return hipGetLastError();
}

hipError_t launch_adj_rhs(const double* F, const double* Lm, const double* seedF, const double* seedL,
                          double scale, double* outF, double* outL, double* Rb, double* gb, double* eta_part,
                          int accumulate, const void* lc, const EosTable& tb, const StageArgs& a, int* err,
                          hipStream_t s) {
  const LC& C = *static_cast<const LC*>(lc);
  hipLaunchKernelGGL(adj_local_kernel, sites_grid(a.n_sites), dim3(kAdjBlock), 0, s, F, Lm, seedF, seedL, scale,
                     outF, outL, Rb, gb, eta_part, accumulate, C, tb, a, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adj_gather_kernel, sites_grid(a.n_sites), dim3(kAdjBlock), 0, s, Rb, gb, outF, outL, C, a);
  return hipGetLastError();
}

hipError_t launch_adj_axpy(double* y, const double* x, double c, double* z, double cz, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(adj_axpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, x, c, z, cz, n);
  return hipGetLastError();
}

hipError_t launch_adj_sum(const double* v, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(adj_sum_kernel, dim3(1), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

hipError_t launch_adj_init(const double* e0, const double* ux0, const double* uy0, const double* aF,
                           const double* aL, double* grad_e0, const void* lc, const EosTable& tb,
                           const StageArgs& a, int* err, hipStream_t s) {
  hipLaunchKernelGGL(adj_init_kernel, sites_grid(a.n_sites), dim3(kAdjBlock), 0, s, e0, ux0, uy0, aF, aL, grad_e0,
                     *static_cast<const LC*>(lc), tb, a, err);
  return hipGetLastError();
}

}  // namespace lbmi
