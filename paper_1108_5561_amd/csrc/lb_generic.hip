// The Heun step on a momentum lattice other than 5 x 5 x 8 nodes (paper
// Sec. IV.C: N_xi radial nodes, the roots of R_{N_xi}; N_theta polar
// Gauss-Legendre nodes; 2 N_phi azimuths phi_l = l pi / N_phi), FP64, in the
// canonical layout F[n][site], n = (k N_theta + j) 2 N_phi + l.  The paper
// names N_xi as the lever for accuracy away from the reference temperature
// (Sec. IV.E); this path lets a caller raise or lower it and the angular
// resolution at run time.  Same method as the stage kernels of
// lb_device.hip (streaming, Milne term S1/tau, mass change X S2, BGK of
// eq. (bgk) with the equilibrium of eq. (feq), the mass-gradient force on
// F_eq, eqs. (edchange)/(masschange)), but with a plain work mapping: one
// thread per (site, phi slice), 32 sites per block, sums over a site's
// slices through LDS in a fixed slice order, and the Landau matching and
// EoS inversion of the stage's input state done at the start of the stage
// by every thread of the site (no site records).
#include <hip/hip_runtime.h>

#include "../../include/lb.h"
#include "device_common.hpp"
#include "generic.hpp"
#include "kernels.hpp"
#include "lb_common.hpp"

namespace lbmi {

namespace {

constexpr int kGSites = 32;  // sites per block

template <int NL>
struct GLane {
  int l, sl, site, x, y;
  bool valid;
};
template <int NL>
__device__ __forceinline__ GLane<NL> glane(const StageArgs& a) {
  GLane<NL> g;
  g.l = threadIdx.x / kGSites;
  g.sl = threadIdx.x % kGSites;
  const int s = blockIdx.x * kGSites + g.sl;
  g.valid = s < a.n_sites;
  g.site = g.valid ? s : a.n_sites - 1;
  g.x = g.site % a.nx;
  g.y = g.site / a.nx;
  return g;
}

// v[k] <- sum over the NL slices of the site of v[k] (order l = 0..NL-1).
template <int K, int NL>
__device__ __forceinline__ void gsum(double v[K], double (*red)[NL][kGSites], const GLane<NL>& g) {
#pragma unroll
  for (int k = 0; k < K; ++k) red[k][g.l][g.sl] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0;
#pragma unroll
    for (int l = 0; l < NL; ++l) s += red[k][l][g.sl];
    v[k] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ size_t gix(int q, int l, int NL, int site, int ns) {
  return (size_t)(q * NL + l) * (size_t)ns + (size_t)site;
}

// One Heun stage: stage 0 Fout = Fin + dtau K(Fin), stage 1
// Fout = (Fbase + Fin)/2 + dtau/2 K(Fin); ln M likewise with X.
template <int NXI, int NTH, int NL>
__global__ __launch_bounds__(kGSites * NL) void gen_stage_kernel(
    const double* __restrict__ Fin, const double* __restrict__ Lin, const double* __restrict__ Fbase,
    const double* __restrict__ Lbase, double* __restrict__ Fout, double* __restrict__ Lout, int stage,
    const GenConst* __restrict__ Cg, const EosTable* __restrict__ tbg, const StageArgs a, int* __restrict__ err) {
  constexpr int Q = NXI * NTH;
  __shared__ double red[6][NL][kGSites];
  const GenConst& C = *Cg;
  const GLane<NL> g = glane<NL>(a);
  const int ns = a.n_sites, l = g.l;
  double f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = Fin[gix(q, l, NL, g.site, ns)];
  const double cl = C.cosl[l], sl = C.sinl[l];

  // moments of the input state (eq. (emtnew)), Landau matching (eq.
  // (sanity)) and the EoS at lambda = eps - B
  double v[6];
  {
    double q0 = 0, q1 = 0, q2 = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      q0 += C.wx2[q] * f[q];
      q1 += C.wxs[q] * f[q];
      q2 += C.ws2[q] * f[q];
    }
    v[0] = q0;
    v[1] = q1 * cl;
    v[2] = q1 * sl;
    v[3] = q2 * cl * cl;
    v[4] = q2 * cl * sl;
    v[5] = q2 * sl * sl;
  }
  gsum<6, NL>(v, red, g);
  const double lnM = Lin[g.site];
  const double M = exp(lnM);
  const double G = M * M * M * M * (1.0 / (2.0 * kPi * kPi));
  double tk[6];
  bool finite = isfinite(lnM);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    tk[i] = G * v[i];
    finite = finite && isfinite(tk[i]);
  }
  double lam, u[3];
  const bool matched = landau3(tk, &lam, u);
  EosAt E;
  const bool eos_ok = eos_g(*tbg, log(lam), lam > 0.0, &E);
  if (g.valid && l == 0) {
    if (!finite) flag(err, kErrNonfinite);
    else if (!matched) flag(err, kErrMatch);
    else if (!eos_ok) flag(err, kErrEos);
  }
  const double ut = u[0], ux = u[1], uy = u[2], T = E.T, invT = 1.0 / T, Meq = E.M_eq, beta = E.beta;
  const double rate = T * a.inv_eta_hbarc / E.q;  // 1/tau_R [fm^-1]
  const double MT = M * invT;

  // gradient of ln M: centred, or the streaming's upwind difference
  const int dxr = cl > 0.0 ? 1 : (cl < 0.0 ? -1 : 0);
  const int dyr = sl > 0.0 ? 1 : (sl < 0.0 ? -1 : 0);
  const int x = g.x, y = g.y;
  const double lxp = Lin[y * a.nx + wrap(x + 1, a.nx)], lxm = Lin[y * a.nx + wrap(x - 1, a.nx)];
  const double lyp = Lin[wrap(y + 1, a.ny) * a.nx + x], lym = Lin[wrap(y - 1, a.ny) * a.nx + x];
  double gx = (lxp - lxm) * a.inv2dx, gy = (lyp - lym) * a.inv2dx;
  if (a.grad_form == LB_GRAD_UPWIND) {
    if (dxr != 0)
      gx = (double)dxr * (3.0 * lnM - 4.0 * (dxr > 0 ? lxm : lxp) + Lin[y * a.nx + wrap(x - 2 * dxr, a.nx)]) * a.inv2dx;
    if (dyr != 0)
      gy = (double)dyr * (3.0 * lnM - 4.0 * (dyr > 0 ? lym : lyp) + Lin[wrap(y - 2 * dyr, a.ny) * a.nx + x]) * a.inv2dx;
  }

  // right-hand side of the slice (Sec. IV.D, eqs. (Bmilne), (newBeq), (bgk))
  const int s_x1 = y * a.nx + wrap(x - dxr, a.nx), s_x2 = y * a.nx + wrap(x - 2 * dxr, a.nx);
  const int s_y1 = wrap(y - dyr, a.ny) * a.nx + x, s_y2 = wrap(y - 2 * dyr, a.ny) * a.nx + x;
  const double ax = fabs(cl) * a.inv2dx, ay = fabs(sl) * a.inv2dx;
  const bool milne = a.metric == LB_METRIC_MILNE;
  const double itau = milne ? 1.0 / a.tau : 0.0;
  const double cu = ux * cl + uy * sl, Gl = gx * cl + gy * sl, gu = gx * ux + gy * uy;
  double R0[Q], S2[Q];
  double sums[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < NXI; ++k) {
    const double Eeq = sqrt(Meq * Meq + M * M * C.sh2[k]);
    const double al = MT * Gl * ut * M * C.x[k] / Eeq, be = MT * Gl * cu / C.x[k], ga = MT * gu / C.x[k];
#pragma unroll
    for (int j = 0; j < NTH; ++j) {
      const int q = k * NTH + j;
      // streaming: second-order upwind along (cos phi, sin phi), periodic
      const double tr = 3.0 * (ax + ay) * f[q] - 4.0 * ax * Fin[gix(q, l, NL, s_x1, ns)] +
                        ax * Fin[gix(q, l, NL, s_x2, ns)] - 4.0 * ay * Fin[gix(q, l, NL, s_y1, ns)] +
                        ay * Fin[gix(q, l, NL, s_y2, ns)];
      double s2 = 0, s1r = 0, s1p = 0;
#pragma unroll
      for (int kp = 0; kp < NXI; ++kp) {
        s2 += C.A2[k * NXI + kp] * f[kp * NTH + j];
        s1r += C.A1[k * NXI + kp] * f[kp * NTH + j];
      }
#pragma unroll
      for (int jp = 0; jp < NTH; ++jp) s1p += C.Ath[j * NTH + jp] * f[k * NTH + jp];
      S2[q] = s2;
      const double sg = C.sig[q];
      const double feq = a.Z * exp((sg * M * cu - ut * Eeq) * invT);  // eq. (feq) with flow
      const double uvg = ut - C.sigi[q] * cu;                         // (u.V)/gamma
      const double poly = al * sg - be * C.sig2[q] - ga;              // force on F_eq
      double r = -C.sigi[q] * tr + (C.mu2[j] * s1r - s1p) * itau - feq * poly - rate * uvg * (f[q] - feq);
      R0[q] = r;
      const double wuv2 = C.wx2[q] * uvg * uvg;
      sums[0] += wuv2 * r;
      sums[1] += wuv2 * (4.0 * f[q] + s2);
      sums[2] += C.w[q] * f[q];
    }
  }
  gsum<3, NL>(sums, red, g);
  // mass evolution (eq. (masschange))
  const double X = -beta * sums[0] / (sums[2] + beta * sums[1]);
  if (!g.valid) return;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double K = R0[q] + X * S2[q];
    const size_t i = gix(q, l, NL, g.site, ns);
    Fout[i] = stage == 0 ? f[q] + a.dtau * K : 0.5 * (Fbase[i] + f[q]) + 0.5 * a.dtau * K;
  }
  if (l == 0) Lout[g.site] = stage == 0 ? lnM + a.dtau * X : 0.5 * (Lbase[g.site] + lnM) + 0.5 * a.dtau * X;
}

// Initial local equilibrium (Sec. IV.D): T0 from eps_EoS(T0) = e0, M = M(T0),
// F = Z exp(-(u . P)/T0); one thread per site.
template <int NXI, int NTH, int NL>
__global__ __launch_bounds__(128) void gen_init_kernel(const double* __restrict__ e0,
                                                       const double* __restrict__ ux0,
                                                       const double* __restrict__ uy0, double* __restrict__ F,
                                                       double* __restrict__ lnM, const GenConst* __restrict__ Cg,
                                                       const EosTable* __restrict__ tbg, const StageArgs a,
                                                       int* __restrict__ err) {
  constexpr int Q = NXI * NTH;
  const int site = blockIdx.x * 128 + threadIdx.x;
  if (site >= a.n_sites) return;
  const GenConst& C = *Cg;
  const EosTable& tb = *tbg;
  const double e = e0[site] * (kHbarC * kHbarC * kHbarC);
  const double vx = ux0 ? ux0[site] : 0.0, vy = uy0 ? uy0[site] : 0.0;
  int bad = 0;
  if (!isfinite(e) || !(e > 0.0) || !isfinite(vx) || !isfinite(vy)) bad = kErrNonfinite;
  double uu = tb.u_lo;
  if (!bad && !eos_invert(tb, kLnEeos, tb.inv_ee, tb.ge0, tb.ge_h, tb.ge_inv_h, log(e), &uu)) bad = kErrEos;
  if (!bad && (uu < tb.u_lo || uu > tb.u_hi)) bad = kErrEos;
  if (bad) {
    uu = tb.u_lo;
    flag(err, bad);
  }
  double t, w[4], dw[4];
  const int i = eos_locate(tb, uu, &t);
  lagrange4(t, w, dw);
  const double T0 = exp(uu);
  const double M = eos_field(tb, i, w, kZ) * T0;
  const double ut = sqrt(1.0 + vx * vx + vy * vy);
  for (int l = 0; l < NL; ++l) {
    const double cu = vx * C.cosl[l] + vy * C.sinl[l];
    for (int q = 0; q < Q; ++q) {
      const double uP = M * (ut * C.x[q / NTH] - cu * C.sig[q]);
      F[gix(q, l, NL, site, a.n_sites)] = a.Z * exp(-uP / T0);
    }
  }
  lnM[site] = log(M);
}

// Observables (eqs. (emtnew), (NTdisc), (sanity)), as lb_moments documents;
// one thread per site.
template <int NXI, int NTH, int NL>
__global__ __launch_bounds__(128) void gen_moments_kernel(const double* __restrict__ F,
                                                          const double* __restrict__ lnMv, double* __restrict__ out,
                                                          const GenConst* __restrict__ Cg,
                                                          const EosTable* __restrict__ tbg, const StageArgs a,
                                                          int* __restrict__ err) {
  constexpr int Q = NXI * NTH;
  const int site = blockIdx.x * 128 + threadIdx.x;
  if (site >= a.n_sites) return;
  const GenConst& C = *Cg;
  const int ns = a.n_sites;
  double m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0, mYY = 0, n0 = 0, n1 = 0, n2 = 0;
  for (int l = 0; l < NL; ++l) {
    const double cl = C.cosl[l], sl = C.sinl[l];
    double p0 = 0, p1 = 0, p2 = 0, p3 = 0, p4 = 0, p5 = 0;
    for (int q = 0; q < Q; ++q) {
      const double fq = F[gix(q, l, NL, site, ns)];
      p0 += C.wx2[q] * fq;
      p1 += C.wxs[q] * fq;
      p2 += C.ws2[q] * fq;
      p3 += C.wvY2[q] * fq;
      p4 += C.wx[q] * fq;
      p5 += C.wsig[q] * fq;
    }
    m00 += p0;
    m01 += p1 * cl;
    m02 += p1 * sl;
    m11 += p2 * cl * cl;
    m12 += p2 * cl * sl;
    m22 += p2 * sl * sl;
    mYY += p3;
    n0 += p4;
    n1 += p5 * cl;
    n2 += p5 * sl;
  }
  const double lnM = lnMv[site];
  const double M = exp(lnM);
  const double G = M * M * M * M / (2.0 * kPi * kPi);
  const double G3 = M * M * M / (2.0 * kPi * kPi);
  const double tk[6] = {G * m00, G * m01, G * m02, G * m11, G * m12, G * m22};
  double lam, u[3];
  const bool matched = landau3(tk, &lam, u);
  EosAt E;
  const bool eos_ok = eos_from_lambda(*tbg, lam, &E);
  bool finite = true;
  for (int i = 0; i < 6; ++i) finite = finite && isfinite(tk[i]);
  if (!finite) flag(err, kErrNonfinite);
  else if (!matched) flag(err, kErrMatch);
  else if (!eos_ok) flag(err, kErrEos);
  const double B = E.Bt4 * E.T * E.T * E.T * E.T;
  const double c3 = 1.0 / (kHbarC * kHbarC * kHbarC);
  const size_t n = (size_t)ns;
  out[0 * n + site] = (tk[0] + B) * c3;
  out[1 * n + site] = tk[1] * c3;
  out[2 * n + site] = tk[2] * c3;
  out[3 * n + site] = (tk[3] - B) * c3;
  out[4 * n + site] = tk[4] * c3;
  out[5 * n + site] = (tk[5] - B) * c3;
  out[6 * n + site] = (G * mYY - B) * c3;
  out[7 * n + site] = G3 * n0 * c3;
  out[8 * n + site] = G3 * n1 * c3;
  out[9 * n + site] = G3 * n2 * c3;
  out[10 * n + site] = E.T;
  out[11 * n + site] = u[1];
  out[12 * n + site] = u[2];
  out[13 * n + site] = M;
}

enum GenKernel { kGenStage, kGenInit, kGenMoments };

struct GenLaunch {
  const double *Fin, *Lin, *Fbase, *Lbase;
  double *Fout, *Lout;
  int stage;
  const double *e0, *ux0, *uy0;
  double* out;
};

template <int NXI, int NTH, int NL>
hipError_t gen_launch_t(GenKernel k, const GenLaunch& p, const GenConst* C, const EosTable* tb, const StageArgs& a,
                        int* err, hipStream_t s) {
  const unsigned n = (unsigned)a.n_sites;
  switch (k) {
    case kGenStage:
      hipLaunchKernelGGL((gen_stage_kernel<NXI, NTH, NL>), dim3((n + kGSites - 1) / kGSites), dim3(kGSites * NL), 0, s,
                         p.Fin, p.Lin, p.Fbase, p.Lbase, p.Fout, p.Lout, p.stage, C, tb, a, err);
      break;
    case kGenInit:
      hipLaunchKernelGGL((gen_init_kernel<NXI, NTH, NL>), dim3((n + 127) / 128), dim3(128), 0, s, p.e0, p.ux0, p.uy0,
                         p.Fout, p.Lout, C, tb, a, err);
      break;
    case kGenMoments:
      hipLaunchKernelGGL((gen_moments_kernel<NXI, NTH, NL>), dim3((n + 127) / 128), dim3(128), 0, s, p.Fin, p.Lin,
                         p.out, C, tb, a, err);
      break;
  }
  return hipGetLastError();
}

template <int NXI, int NTH>
hipError_t gen_launch_l(int nl, GenKernel k, const GenLaunch& p, const GenConst* C, const EosTable* tb,
                        const StageArgs& a, int* err, hipStream_t s) {
  switch (nl) {
    case 6: return gen_launch_t<NXI, NTH, 6>(k, p, C, tb, a, err, s);
    case 8: return gen_launch_t<NXI, NTH, 8>(k, p, C, tb, a, err, s);
    case 10: return gen_launch_t<NXI, NTH, 10>(k, p, C, tb, a, err, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NXI>
hipError_t gen_launch_th(int nth, int nl, GenKernel k, const GenLaunch& p, const GenConst* C, const EosTable* tb,
                         const StageArgs& a, int* err, hipStream_t s) {
  switch (nth) {
    case 3: return gen_launch_l<NXI, 3>(nl, k, p, C, tb, a, err, s);
    case 5: return gen_launch_l<NXI, 5>(nl, k, p, C, tb, a, err, s);
    case 7: return gen_launch_l<NXI, 7>(nl, k, p, C, tb, a, err, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t gen_launch(int nxi, int nth, int nl, GenKernel k, const GenLaunch& p, const GenConst* C, const EosTable* tb,
                      const StageArgs& a, int* err, hipStream_t s) {
  if (a.n_sites <= 0) return hipSuccess;
  switch (nxi) {
    case 3: return gen_launch_th<3>(nth, nl, k, p, C, tb, a, err, s);
    case 5: return gen_launch_th<5>(nth, nl, k, p, C, tb, a, err, s);
    case 7: return gen_launch_th<7>(nth, nl, k, p, C, tb, a, err, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_gen_stage(int nxi, int nth, int nl, int stage, const double* Fin, const double* Lin,
                            const double* Fbase, const double* Lbase, double* Fout, double* Lout, const GenConst* C,
                            const EosTable* tb, const StageArgs& a, int* err, hipStream_t s) {
  GenLaunch p{};
  p.Fin = Fin;
  p.Lin = Lin;
  p.Fbase = Fbase;
  p.Lbase = Lbase;
  p.Fout = Fout;
  p.Lout = Lout;
  p.stage = stage;
  return gen_launch(nxi, nth, nl, kGenStage, p, C, tb, a, err, s);
}

hipError_t launch_gen_init(int nxi, int nth, int nl, const double* e0, const double* ux0, const double* uy0, double* F,
                           double* lnM, const GenConst* C, const EosTable* tb, const StageArgs& a, int* err,
                           hipStream_t s) {
  GenLaunch p{};
  p.e0 = e0;
  p.ux0 = ux0;
  p.uy0 = uy0;
  p.Fout = F;
  p.Lout = lnM;
  return gen_launch(nxi, nth, nl, kGenInit, p, C, tb, a, err, s);
}

hipError_t launch_gen_moments(int nxi, int nth, int nl, const double* F, const double* lnM, double* out,
                              const GenConst* C, const EosTable* tb, const StageArgs& a, int* err, hipStream_t s) {
  GenLaunch p{};
  p.Fin = F;
  p.Lin = lnM;
  p.out = out;
  return gen_launch(nxi, nth, nl, kGenMoments, p, C, tb, a, err, s);
}

}  // namespace lbmi
