// Discrete adjoint (reverse mode) of the Heun step of Sec. IV.D for the
// differentiable form: gradients of a function of the final state with
// respect to the initial energy density e0 and to eta/s.
//
// The step differentiated is the step of the stage kernels, written out
// here in the canonical layout F[n][site], n = q 8 + l (q = k N_theta + j):
// for state (F, ln M) at time tau the right-hand side is
//   R0_n = A_n + S1_n/tau + F_eq,n ((u.V)/gamma r - poly_n) - (u.V)/gamma r F_n
//   X    = -beta sum w (u.V)^2 R0 / (sum w F + beta sum w (u.V)^2 (4F + S2))
//   K_n  = R0_n + X S2_n
// (streaming A, Milne term S1/tau, equilibrium with the mass-gradient force
// and BGK of eqs. (Bmilne), (newBeq), (bgk); mass evolution of eqs.
// (edchange), (masschange)), where r = 1/tau_R, u, T and M_eq come from the
// Landau matching (eq. (sanity)) of the state's own moments (eq. (emtnew))
// and the EoS inversion (with the conserved particle number also n =
// u_a N^a, mu/T and the fugacity of F_eq; beta = 0 there).
//
// Work mapping: a block of 256 threads covers 32 sites; thread t owns phi
// slice l = t / 32 of site t % 32, so a wavefront reads 64 consecutive
// sites of one node (coalesced); each XCD takes a contiguous band of
// blocks.  Sums over a site's eight slices go through LDS in a fixed order
// (every thread of the site gets the same bits).  FP64 kernels
// (adj_fwd_kernel, adj_local_kernel): the per-site work (matching, EoS,
// their adjoints) is repeated by the eight threads of a site; the reverse
// sweep of one right-hand side evaluates the slice forward once, keeps R0
// and S2 in registers, propagates the adjoint through the collision,
// equilibrium, force and operator terms, reduces the site adjoints over the
// slices, runs the implicit-function adjoints of the EoS root and of the
// eigenproblem, and adds the moments' adjoint.  FP32 kernels
// (adj_fwd32_kernel, adj_local32_kernel, for contexts whose forward runs in
// FP32): the node arithmetic in FP32, the per-site chain once per site in
// FP64.  The transposed streaming stencil and the transposed centred ln M
// gradient are gathers over the neighbours (adj_gather_kernel).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "../../include/lb.h"
#include "device_common.hpp"
#include "kernels.hpp"
#include "lb_common.hpp"

namespace lbmi {

namespace {

constexpr int kQ = 25;                     // nodes per phi slice
constexpr int kL = 8;                      // phi slices
constexpr int kSites = 32;                 // sites per block
constexpr int kAdjThreads = kSites * kL;   // 256
constexpr int kRed = 11;                   // most values reduced at once
constexpr int kInitBlock = 128;           // adj_init_kernel: one thread per site
using LC = LatticeConst<double, 5, 5>;
typedef double RedBuf[kRed][kL][kSites];

__device__ __forceinline__ size_t cix(int q, int l, int site, int ns) {
  return (size_t)(q * kL + l) * (size_t)ns + (size_t)site;
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b on XCD
// b mod 8).  Each XCD is given one contiguous band of blocks instead, so
// that the stencil neighbours (two rows up and down) of a block were read
// by blocks on the same XCD and are in its L2: XCD x takes blocks
// [x base + min(x, rem), ...) with base = nb / 8, rem = nb % 8, which maps
// the nb workgroups one-to-one onto the nb blocks.
__device__ __forceinline__ int xcd_band_block() {
  const int nb = gridDim.x, b = blockIdx.x, x = b & 7;
  const int base = nb >> 3, rem = nb & 7;
  return x * base + (x < rem ? x : rem) + (b >> 3);
}

// The slice and site of this thread (sites past the grid repeat the last
// site and store nothing, but take part in the block's reductions).
struct Lane {
  int l, sl, site, x, y;
  bool valid;
};
__device__ __forceinline__ Lane lane_of(const StageArgs& a) {
  Lane g;
  g.l = threadIdx.x / kSites;
  g.sl = threadIdx.x % kSites;
  const int s = xcd_band_block() * kSites + g.sl;
  g.valid = s < a.n_sites;
  g.site = g.valid ? s : a.n_sites - 1;
  g.x = g.site % a.nx;
  g.y = g.site / a.nx;
  return g;
}

// v[k] <- sum over the eight slices of the site of v[k], k < K, in the
// order l = 0..7 (identical in every thread of the site).
template <int K>
__device__ __forceinline__ void slice_sum(double v[K], RedBuf& red, const Lane& g) {
#pragma unroll
  for (int k = 0; k < K; ++k) red[k][g.l][g.sl] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0;
#pragma unroll
    for (int l = 0; l < kL; ++l) s += red[k][l][g.sl];
    v[k] = s;
  }
  __syncthreads();
}

// Upwind direction and streaming coefficients of slice l (as in the stage
// kernels: second-order upwind along +(cos phi, sin phi)).
struct SliceGeom {
  double cl, sl, ax, ay;
  int dxr, dyr;
};
template <typename LCT>
__device__ __forceinline__ SliceGeom slice_geom(const LCT& C, const StageArgs& a, int l) {
  SliceGeom g;
  // cos and sin of phi_l by selects over constant indices: no dynamic
  // index into the kernel-argument struct (which would put it in scratch)
  g.cl = C.cosl[0];
  g.sl = C.sinl[0];
#pragma unroll
  for (int i = 1; i < kL; ++i) {
    g.cl = l == i ? C.cosl[i] : g.cl;
    g.sl = l == i ? C.sinl[i] : g.sl;
  }
  g.dxr = (g.cl > 0.0) ? 1 : ((g.cl < 0.0) ? -1 : 0);
  g.dyr = (g.sl > 0.0) ? 1 : ((g.sl < 0.0) ? -1 : 0);
  g.ax = fabs(g.cl) * a.inv2dx;
  g.ay = fabs(g.sl) * a.inv2dx;
  return g;
}

// Derivatives in u = ln T of the table fields that eos_mu uses, at the T it
// returned (for the adjoint of the n matching; the
// table fields by their qualified names, kQ being the node count here): ln eps0_kin, ln n0, z, q
// and T n0/h.
struct EosMuDer {
  double dlnEk, dlnN, dz, dQ, dNq, Nq;
};
__device__ inline void eos_mu_der(const EosTable& tb, double T, EosMuDer* d) {
  double t, w[4], dw[4];
  const int i = eos_locate(tb, log(T), &t);
  lagrange4(t, w, dw);
  const double ih = tb.inv_h;
  d->dlnEk = eos_field(tb, i, dw, ::lbmi::kLnEk) * ih;
  d->dlnN = eos_field(tb, i, dw, ::lbmi::kLnN) * ih;
  d->dz = eos_field(tb, i, dw, ::lbmi::kZ) * ih;
  d->dQ = eos_field(tb, i, dw, ::lbmi::kQ) * ih;
  d->dNq = eos_field(tb, i, dw, ::lbmi::kNq) * ih;
  d->Nq = eos_field(tb, i, w, ::lbmi::kNq);
}

// Site quantities of a state: moments, Landau matching, EoS.  With the
// conserved particle number (mu): the current sums c, n = u_a N^a, alpha =
// mu/T and the table derivatives of the n matching.
struct SiteFwd {
  double m[3][3];  // sum_n w F V^a V^b, a, b in (tau, x, y)
  double M, G;     // mass and M^4/(2 pi^2)
  double lam, u[3];
  EosAt E;
  EosDer D;
  double invT, MT, rate, beta;
  double gx, gy;   // centred gradient of ln M
  bool mu;
  double c[3], nd, alpha;  // sum_n w F V^a; n; mu/T
  EosMuDer Dm;
};

__device__ void site_fwd(const double f[kQ], const double* __restrict__ lnM, const Lane& g, const LC& C,
                         const EosTable& tb, const StageArgs& a, RedBuf& red, SiteFwd* s,
                         int* __restrict__ err) {
  double q0 = 0, q1 = 0, q2 = 0;
  for (int q = 0; q < kQ; ++q) {
    q0 += C.wx2[q] * f[q];
    q1 += C.wxs[q] * f[q];
    q2 += C.ws2[q] * f[q];
  }
  const double cl = C.cosl[g.l], sl = C.sinl[g.l];
  double v[9] = {q0, q1 * cl, q1 * sl, q2 * cl * cl, q2 * cl * sl, q2 * sl * sl, 0.0, 0.0, 0.0};
  s->mu = a.mu_mode != 0;
  if (s->mu) {
    // the particle current N^a = M^3/(2 pi^2) sum w F V^a (eq. (NTdisc))
    double n0 = 0, n1 = 0;
    for (int q = 0; q < kQ; ++q) {
      n0 += C.wx[q] * f[q];
      n1 += C.w[q] * C.sig[q] * f[q];
    }
    v[6] = n0;
    v[7] = n1 * cl;
    v[8] = n1 * sl;
    slice_sum<9>(v, red, g);
  } else {
    slice_sum<6>(v, red, g);
  }
  s->m[0][0] = v[0];
  s->m[0][1] = s->m[1][0] = v[1];
  s->m[0][2] = s->m[2][0] = v[2];
  s->m[1][1] = v[3];
  s->m[1][2] = s->m[2][1] = v[4];
  s->m[2][2] = v[5];
  s->M = exp(lnM[g.site]);
  s->G = s->M * s->M * s->M * s->M * (1.0 / (2.0 * kPi * kPi));
  const double tk[6] = {s->G * v[0], s->G * v[1], s->G * v[2], s->G * v[3], s->G * v[4], s->G * v[5]};
  const bool matched = landau3(tk, &s->lam, s->u);
  bool eos_ok;
  s->alpha = 0.0;
  if (s->mu) {
    // n matching (eq. (sanity)): T and alpha from lambda and n; the mass is
    // constant (beta = 0), as in the stage kernels' mu mode
    s->c[0] = v[6];
    s->c[1] = v[7];
    s->c[2] = v[8];
    s->nd = s->G / s->M * (s->u[0] * v[6] - s->u[1] * v[7] - s->u[2] * v[8]);
    eos_ok = eos_mu(tb, s->lam, s->nd, &s->E, &s->alpha);
    eos_mu_der(tb, s->E.T, &s->Dm);
    s->E.beta = 0.0;
  } else {
    eos_ok = eos_cell(tb, s->lam, &s->E, &s->D);
  }
  bool finite = true;
  for (int i = 0; i < 6; ++i) finite = finite && isfinite(tk[i]);
  if (g.valid && g.l == 0) {
    if (!finite) flag(err, kErrNonfinite);
    else if (!matched) flag(err, kErrMatch);
    else if (!eos_ok) flag(err, kErrEos);
  }
  s->invT = 1.0 / s->E.T;
  s->MT = s->M * s->invT;
  s->rate = s->E.T * a.inv_eta_hbarc / s->E.q;
  s->beta = s->E.beta;
  const int x = g.x, y = g.y;
  const int xp = wrap(x + 1, a.nx), xm = wrap(x - 1, a.nx), yp = wrap(y + 1, a.ny), ym = wrap(y - 1, a.ny);
  s->gx = (lnM[y * a.nx + xp] - lnM[y * a.nx + xm]) * a.inv2dx;
  s->gy = (lnM[yp * a.nx + x] - lnM[ym * a.nx + x]) * a.inv2dx;
}

// The ln M gradient that the force on F_eq of a slice uses: the site's
// centred one (gxc, gyc), or with the upwind gradient (LB_GRAD_UPWIND) the
// streaming's second-order upwind difference along the slice's direction
// of motion, centred along an axis it does not move on (as the stage
// kernels).
__device__ __forceinline__ void slice_grad(const double* __restrict__ Lm, const Lane& g, const SliceGeom& gm,
                                           const StageArgs& a, double gxc, double gyc, double* gx, double* gy,
                                           bool upwind) {
  *gx = gxc;
  *gy = gyc;
  if (!upwind) return;
  const int x = g.x, y = g.y;
  const double L0 = Lm[g.site];
  if (gm.dxr != 0)
    *gx = gm.dxr * (3.0 * L0 - 4.0 * Lm[y * a.nx + wrap(x - gm.dxr, a.nx)] + Lm[y * a.nx + wrap(x - 2 * gm.dxr, a.nx)]) *
          a.inv2dx;
  if (gm.dyr != 0)
    *gy = gm.dyr * (3.0 * L0 - 4.0 * Lm[wrap(y - gm.dyr, a.ny) * a.nx + x] + Lm[wrap(y - 2 * gm.dyr, a.ny) * a.nx + x]) *
          a.inv2dx;
}

// Per-slice factors of the equilibrium and the mass-gradient force (gx, gy:
// the slice's ln M gradient).
struct SliceAux {
  double cu, Gl, gu, gx, gy;
  double Eeq[5], al[5], be[5], ga[5];
};
// With the weak-form 3-D force (f3) the force acts on F instead (force_row)
// and the polynomial on F_eq vanishes: Gl = gu = 0.
__device__ __forceinline__ void slice_aux(const SiteFwd& s, const SliceGeom& gm, const LC& C, bool f3,
                                          const double* __restrict__ Lm, const Lane& g, const StageArgs& a,
                                          SliceAux* o) {
  const double ut = s.u[0], ux = s.u[1], uy = s.u[2], Meq = s.E.M_eq, M = s.M;
  slice_grad(Lm, g, gm, a, s.gx, s.gy, &o->gx, &o->gy, a.grad_form == LB_GRAD_UPWIND);
  o->cu = ux * gm.cl + uy * gm.sl;
  o->Gl = f3 ? 0.0 : o->gx * gm.cl + o->gy * gm.sl;
  o->gu = f3 ? 0.0 : o->gx * ux + o->gy * uy;
  for (int k = 0; k < 5; ++k) {
    o->Eeq[k] = sqrt(Meq * Meq + M * M * C.sh2[k]);
    o->al[k] = s.MT * o->Gl * ut * M * C.x[k] / o->Eeq[k];
    o->be[k] = s.MT * o->Gl * o->cu * C.inv_x[k];
    o->ga[k] = s.MT * o->gu * C.inv_x[k];
  }
}

// F_eq, (u.V)/gamma and the force polynomial of node q.
__device__ __forceinline__ void node_terms(const SiteFwd& s, const SliceAux& o, const LC& C, const StageArgs& a,
                                           int q, double* feq, double* uvg, double* poly) {
  const int k = q / 5;
  const double sg = C.sig[q];
  *feq = a.Z * exp(s.alpha + (sg * s.M * o.cu - s.u[0] * o.Eeq[k]) * s.invT);
  *uvg = s.u[0] - C.sigi[q] * o.cu;
  *poly = o.al[k] * sg - o.be[k] * C.sig2[q] - o.ga[k];
}

// Row n of the weak-form 3-D force operators applied to the site's state:
// (G_x F)_n and (G_y F)_n, with g3 = G [2][kN][kN] (canonical node order)
// and F in the canonical layout.
constexpr int kN = kQ * kL;  // nodes per site
__device__ __forceinline__ void force_row(const double* __restrict__ g3, const double* __restrict__ F, int site,
                                          int ns, int n, double* gxf, double* gyf) {
  const double* rx = g3 + (size_t)n * kN;
  const double* ry = rx + (size_t)kN * kN;
  double ax = 0, ay = 0;
  for (int m = 0; m < kN; ++m) {
    const double fm = F[(size_t)m * ns + site];
    ax += rx[m] * fm;
    ay += ry[m] * fm;
  }
  *gxf = ax;
  *gyf = ay;
}

// R0 and S2 of the thread's slice and its parts of the three site sums.
__device__ void slice_rhs(const double* __restrict__ F, const double f[kQ], const Lane& g, const SliceGeom& gm,
                          const SiteFwd& s, const SliceAux& o, const LC& C, const StageArgs& a,
                          const double* __restrict__ g3, double R0[kQ], double S2[kQ], double sums[3]) {
  const int ns = a.n_sites, x = g.x, y = g.y, l = g.l;
  // streaming (3 F_i - 4 F_{i-1} + F_{i-2}) |cos phi| / (2 dx), periodic
  const int x1 = wrap(x - gm.dxr, a.nx), x2 = wrap(x - 2 * gm.dxr, a.nx);
  const int y1 = wrap(y - gm.dyr, a.ny), y2 = wrap(y - 2 * gm.dyr, a.ny);
  const int s_x1 = y * a.nx + x1, s_x2 = y * a.nx + x2, s_y1 = y1 * a.nx + x, s_y2 = y2 * a.nx + x;
  for (int q = 0; q < kQ; ++q) {
    const double tr = 3.0 * (gm.ax + gm.ay) * f[q] - 4.0 * gm.ax * F[cix(q, l, s_x1, ns)] +
                      gm.ax * F[cix(q, l, s_x2, ns)] - 4.0 * gm.ay * F[cix(q, l, s_y1, ns)] +
                      gm.ay * F[cix(q, l, s_y2, ns)];
    R0[q] = -C.sigi[q] * tr;
  }
  // S2 (radial) and, for the Milne metric, S1/tau
  const bool milne = a.metric == LB_METRIC_MILNE;
  const double itau = 1.0 / a.tau;
  for (int k = 0; k < 5; ++k)
    for (int j = 0; j < 5; ++j) {
      double s2 = 0, s1r = 0, s1p = 0;
      for (int kp = 0; kp < 5; ++kp) {
        s2 += C.A2[k * 5 + kp] * f[kp * 5 + j];
        s1r += C.A1[k * 5 + kp] * f[kp * 5 + j];
      }
      for (int jp = 0; jp < 5; ++jp) s1p += C.Ath[j * 5 + jp] * f[k * 5 + jp];
      S2[k * 5 + j] = s2;
      if (milne) R0[k * 5 + j] += (C.mu2[j] * s1r - s1p) * itau;
    }
  if (g3)  // weak-form 3-D force on F: g_x G_x F + g_y G_y F
    for (int q = 0; q < kQ; ++q) {
      double gxf, gyf;
      force_row(g3, F, g.site, ns, q * kL + l, &gxf, &gyf);
      R0[q] += s.gx * gxf + s.gy * gyf;
    }
  sums[0] = sums[1] = sums[2] = 0;
  for (int q = 0; q < kQ; ++q) {
    double feq, uvg, poly;
    node_terms(s, o, C, a, q, &feq, &uvg, &poly);
    const double ru = s.rate * uvg;
    R0[q] += feq * (ru - poly) - ru * f[q];
    const double wuv2 = C.wx2[q] * uvg * uvg;
    sums[0] += wuv2 * R0[q];
    sums[1] += wuv2 * (4.0 * f[q] + S2[q]);
    sums[2] += C.w[q] * f[q];
  }
}

// ---------------------------------------------------------------------------
// One Heun stage of the FP64 step in the canonical layout: stage 0 writes
// Fout = Fin + dtau K(Fin), stage 1 Fout = (Fbase + Fin)/2 + dtau/2 K(Fin);
// ln M likewise with X.
__global__ __launch_bounds__(kAdjThreads) void adj_fwd_kernel(const double* __restrict__ Fin,
                                                              const double* __restrict__ Lin,
                                                              const double* __restrict__ Fbase,
                                                              const double* __restrict__ Lbase,
                                                              double* __restrict__ Fout,
                                                              double* __restrict__ Lout, int stage, const LC C,
                                                              const double* __restrict__ g3, const EosTable tb,
                                                              const StageArgs a, int* __restrict__ err) {
  __shared__ RedBuf red;
  const Lane g = lane_of(a);
  const int ns = a.n_sites;
  double f[kQ];
  for (int q = 0; q < kQ; ++q) f[q] = Fin[cix(q, g.l, g.site, ns)];
  SiteFwd s;
  site_fwd(f, Lin, g, C, tb, a, red, &s, err);
  const SliceGeom gm = slice_geom(C, a, g.l);
  SliceAux o;
  slice_aux(s, gm, C, g3 != nullptr, Lin, g, a, &o);
  double R0[kQ], S2[kQ], sums[3];
  slice_rhs(Fin, f, g, gm, s, o, C, a, g3, R0, S2, sums);
  slice_sum<3>(sums, red, g);
  const double X = -s.beta * sums[0] / (sums[2] + s.beta * sums[1]);
  if (!g.valid) return;
  for (int q = 0; q < kQ; ++q) {
    const double K = R0[q] + X * S2[q];
    const size_t i = cix(q, g.l, g.site, ns);
    Fout[i] = stage == 0 ? f[q] + a.dtau * K : 0.5 * (Fbase[i] + f[q]) + 0.5 * a.dtau * K;
  }
  if (g.l == 0) {
    const double lm = Lin[g.site];
    Lout[g.site] = stage == 0 ? lm + a.dtau * X : 0.5 * (Lbase[g.site] + lm) + 0.5 * a.dtau * X;
  }
}

// ---------------------------------------------------------------------------
// Reverse sweep of one right-hand side at state (F, ln M), time a.tau, with
// K_bar = scale seedF and X_bar = scale seedL.  Writes (accumulate = 0) or
// adds (accumulate = 1) the site-local part of the state's adjoint into
// (outF, outL) and the site's eta/s adjoint into eta_part; writes R0_bar
// (for the transposed streaming) into Rb and the ln M gradient adjoint into
// gb[2][site].
// (seven 25-value slice arrays per thread: one wave per SIMD, so that the
// compiler may use the whole register file rather than scratch)
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void adj_local_kernel(
    const double* __restrict__ F, const double* __restrict__ Lm, const double* __restrict__ seedF,
    const double* __restrict__ seedL, double scale, double* __restrict__ outF, double* __restrict__ outL,
    double* __restrict__ Rb, double* __restrict__ gb, double* __restrict__ eta_part, int accumulate,
    const LC C, const double* __restrict__ g3, const EosTable tb, const StageArgs a, int* __restrict__ err) {
  __shared__ RedBuf red;
  const Lane g = lane_of(a);
  const int ns = a.n_sites, l = g.l;
  double f[kQ];
  for (int q = 0; q < kQ; ++q) f[q] = F[cix(q, l, g.site, ns)];
  SiteFwd s;
  site_fwd(f, Lm, g, C, tb, a, red, &s, err);
  const SliceGeom gm = slice_geom(C, a, l);
  SliceAux o;
  slice_aux(s, gm, C, g3 != nullptr, Lm, g, a, &o);
  double R0[kQ], S2[kQ], Kb[kQ];
  double sums[4];
  slice_rhs(F, f, g, gm, s, o, C, a, g3, R0, S2, sums);
  sums[3] = 0;
  for (int q = 0; q < kQ; ++q) {
    Kb[q] = scale * seedF[cix(q, l, g.site, ns)];
    sums[3] += Kb[q] * S2[q];
  }
  slice_sum<4>(sums, red, g);
  const double nsum = sums[0], dsum = sums[1], wsum = sums[2];
  const double beta = s.beta, D = wsum + beta * dsum, X = -beta * nsum / D;
  const double Xb = scale * seedL[g.site] + sums[3];
  const double nb = -beta * Xb / D;           // d/d nsum
  const double Db = -X * Xb / D;              // d/d (wsum + beta dsum)
  const double betab = -nsum * Xb / D + Db * dsum;
  const double wsb = Db, dsb = beta * Db;
  // the slice's adjoint: R0, S2 and everything they use
  const double ut = s.u[0], M = s.M, Meq = s.E.M_eq;
  double R0b[kQ], S2b[kQ], fb[kQ];
  double cub = 0, Glb = 0, gub = 0, utb = 0, Mb = 0, invTb = 0, rateb = 0, alphab = 0;
  double alb[5] = {0, 0, 0, 0, 0}, beb[5] = {0, 0, 0, 0, 0}, gab[5] = {0, 0, 0, 0, 0};
  double Eeqb[5] = {0, 0, 0, 0, 0};
  double g3xb = 0, g3yb = 0;  // 3-D force: this slice's part of d/d g_x, d/d g_y
  for (int q = 0; q < kQ; ++q) {
    const int k = q / 5;
    double feq, uv, poly;
    node_terms(s, o, C, a, q, &feq, &uv, &poly);
    const double wuv2 = C.wx2[q] * uv * uv;
    R0b[q] = Kb[q] + wuv2 * nb;
    if (g3) {
      double gxf, gyf;
      force_row(g3, F, g.site, ns, q * kL + l, &gxf, &gyf);
      g3xb += R0b[q] * gxf;
      g3yb += R0b[q] * gyf;
    }
    S2b[q] = X * Kb[q] + wuv2 * dsb;
    const double ru = s.rate * uv;
    fb[q] = 4.0 * wuv2 * dsb + C.w[q] * wsb - ru * R0b[q];
    const double uvb = 2.0 * C.wx2[q] * uv * ((4.0 * f[q] + S2[q]) * dsb + R0[q] * nb) +
                       s.rate * (feq - f[q]) * R0b[q];
    rateb += uv * (feq - f[q]) * R0b[q];
    const double feqb = (ru - poly) * R0b[q];
    const double polyb = -feq * R0b[q];
    alb[k] += C.sig[q] * polyb;
    beb[k] -= C.sig2[q] * polyb;
    gab[k] -= polyb;
    // F_eq = Z exp(alpha + (sig M cu - ut E_eq) / T)
    const double e = feq * feqb, sg = C.sig[q];
    alphab += e;
    Mb += e * sg * o.cu * s.invT;
    cub += e * sg * M * s.invT;
    invTb += e * (sg * M * o.cu - ut * o.Eeq[k]);
    utb -= e * o.Eeq[k] * s.invT;
    Eeqb[k] -= e * ut * s.invT;
    // (u.V)/gamma = ut - (|v_perp|/gamma) cu
    utb += uvb;
    cub -= C.sigi[q] * uvb;
  }
  // transposed operators: S2 = A2 f, S1 = (mu^2 A1 f - Ath f)/tau
  const bool milne = a.metric == LB_METRIC_MILNE;
  const double itau = 1.0 / a.tau;
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
  double MTb = 0, Meqb = 0;
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
  // (zero with the 3-D force, whose gradient adjoint is g3xb, g3yb); then
  // the site totals over the eight slices
  if (g3) {
    Glb = 0;
    gub = 0;
  }
  double v[kRed] = {utb,
                    cub * gm.cl + gub * o.gx,
                    cub * gm.sl + gub * o.gy,
                    Mb,
                    invTb,
                    MTb,
                    rateb,
                    Meqb,
                    Glb * gm.cl + gub * s.u[1] + g3xb,
                    Glb * gm.sl + gub * s.u[2] + g3yb,
                    alphab};
  // with the upwind gradient the slice's own gradient adjoint goes out per
  // slice ([2][8][sites]); otherwise the site totals below ([2][sites])
  const bool upw = a.grad_form == LB_GRAD_UPWIND;
  if (upw && g.valid) {
    gb[(size_t)l * ns + g.site] = v[8];
    gb[(size_t)(kL + l) * ns + g.site] = v[9];
  }
  slice_sum<kRed>(v, red, g);
  utb = v[0];
  double uxb = v[1], uyb = v[2];
  Mb = v[3];
  invTb = v[4];
  MTb = v[5];
  rateb = v[6];
  Meqb = v[7];
  const double gxb = v[8], gyb = v[9];
  // site chain: M/T, 1/T, r = T/(q hbar c eta/s), then u = ln T
  Mb += MTb * s.invT;
  invTb += MTb * M;
  const double T = s.E.T, qv = s.E.q;
  const double Tb = -invTb * s.invT * s.invT + rateb * a.inv_eta_hbarc / qv;
  const double qb = -rateb * s.rate / qv;
  const double etab = -rateb * s.rate * a.inv_eta_hbarc * kHbarC;  // dr/d(eta/s) = -r/(eta/s)
  const double z = Meq / T;
  double lamb, cnb[3] = {0.0, 0.0, 0.0};
  if (s.mu) {
    // n matching: u = ln T from ln eps0_kin(u) - ln n0(u) = ln lambda - ln n,
    // alpha = ln n - ln n0(u), q = q0(u) - alpha Nq(u); beta = 0
    const double ab = v[10] - qb * s.Dm.Nq;
    const double uub = Tb * T + Meqb * (s.Dm.dz * T + z * T) + qb * (s.Dm.dQ - s.alpha * s.Dm.dNq) -
                       ab * s.Dm.dlnN;
    const double Dd = s.Dm.dlnEk - s.Dm.dlnN;
    lamb = uub / (Dd * s.lam);
    const double nb_ = ab / s.nd - uub / (Dd * s.nd);
    // n = (M^3 / (2 pi^2)) (u^tau c^tau - u^x c^x - u^y c^y)
    const double gmv = s.G / s.M;
    utb += nb_ * gmv * s.c[0];
    uxb -= nb_ * gmv * s.c[1];
    uyb -= nb_ * gmv * s.c[2];
    cnb[0] = nb_ * gmv * s.u[0];
    cnb[1] = -nb_ * gmv * s.u[1];
    cnb[2] = -nb_ * gmv * s.u[2];
    Mb += nb_ * 3.0 * s.nd / M;
  } else {
    const double uub = Tb * T + Meqb * (s.D.dz * T + z * T) + betab * s.D.dbeta + qb * s.D.dq;
    lamb = uub * s.D.du_dlam;
  }
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
  if (!g.valid) return;
  // the moments' adjoint, m^{ab} = sum_n w F V^a V^b, and the stores
  const double c00 = mb[0][0], c01 = (mb[0][1] + mb[1][0]) * gm.cl + (mb[0][2] + mb[2][0]) * gm.sl;
  const double c11 = mb[1][1] * gm.cl * gm.cl + (mb[1][2] + mb[2][1]) * gm.cl * gm.sl + mb[2][2] * gm.sl * gm.sl;
  // and the particle current's adjoint (mu mode; zero otherwise)
  const double n00 = cnb[0], n01 = cnb[1] * gm.cl + cnb[2] * gm.sl;
  for (int q = 0; q < kQ; ++q) {
    const size_t i = cix(q, l, g.site, ns);
    const double v_ = fb[q] + c00 * C.wx2[q] + c01 * C.wxs[q] + c11 * C.ws2[q] + n00 * C.wx[q] +
                      n01 * C.w[q] * C.sig[q];
    outF[i] = accumulate ? outF[i] + v_ : v_;
    Rb[i] = R0b[q];
  }
  if (l == 0) {
    const double lb = Mb * M;  // M = exp(ln M)
    outL[g.site] = accumulate ? outL[g.site] + lb : lb;
    if (!upw) {
      gb[g.site] = gxb;
      gb[ns + g.site] = gyb;
    }
    eta_part[g.site] = accumulate ? eta_part[g.site] + etab : etab;
  }
}

// The reverse sweep of adj_local_kernel for contexts whose forward runs in
// FP32: the same arithmetic with the node values in FP32, the site sums
// reduced in FP64 and the per-site FP64 chain (moments -> Landau matching ->
// EoS, and its reverse through the implicit-function adjoints) done once
// per site, by the thread of slice 0, and handed to the site's other seven
// threads through LDS.  The forward values S2, F_eq and R0 of a node are
// evaluated again where the reverse sweep needs them rather than held (the
// part of R0 read from the stencil neighbours is read once and kept), and
// the transposed operators S1^T and S2^T are applied to the slice's R0b and
// S2b after the sweep, so the register footprint allows two waves per
// SIMD.  The lattice constants come in FP32 (LCf); R0b goes out in FP32
// (Rb).
using LCf = LatticeConst<float, 5, 5>;
struct SiteLds {
  double m[6];  // sum w F V^a V^b: tau tau, tau x, tau y, xx, xy, yy
  double M, G, lam, u[3];
  double T, Meq, beta, q, invT, MT, rate;
  double du_dlam, dz, dbeta, dq;
  double gx, gy;
  double mb[6];  // the moments' adjoint: 00, 01 + 10, 02 + 20, 11, 12 + 21, 22
};

// The slice's share of the moments (eq. (emtnew)), summed over the slices
// in FP64, and the site's Landau matching and EoS by the slice-0 thread.
__device__ __forceinline__ void site_chain32(const float f[kQ], const double* __restrict__ Lm, const Lane& g,
                                             const LCf& C, double cl, double sl, const EosTable& tb,
                                             const StageArgs& a, RedBuf& red, SiteLds* sd,
                                             int* __restrict__ err) {
  float q0 = 0, q1 = 0, q2 = 0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    q0 += C.wx2[q] * f[q];
    q1 += C.wxs[q] * f[q];
    q2 += C.ws2[q] * f[q];
  }
  double v[6] = {(double)q0, (double)q1 * cl, (double)q1 * sl, (double)q2 * cl * cl, (double)q2 * cl * sl,
                 (double)q2 * sl * sl};
  slice_sum<6>(v, red, g);
  if (g.l == 0) {
    SiteLds& S = sd[g.sl];
#pragma unroll
    for (int i = 0; i < 6; ++i) S.m[i] = v[i];
    S.M = exp(Lm[g.site]);
    S.G = S.M * S.M * S.M * S.M * (1.0 / (2.0 * kPi * kPi));
    const double tk[6] = {S.G * v[0], S.G * v[1], S.G * v[2], S.G * v[3], S.G * v[4], S.G * v[5]};
    double u[3], lam;
    const bool matched = landau3(tk, &lam, u);
    EosAt E;
    EosDer D;
    const bool eos_ok = eos_cell(tb, lam, &E, &D);
    bool finite = true;
#pragma unroll
    for (int i = 0; i < 6; ++i) finite = finite && isfinite(tk[i]);
    if (g.valid) {
      if (!finite) flag(err, kErrNonfinite);
      else if (!matched) flag(err, kErrMatch);
      else if (!eos_ok) flag(err, kErrEos);
    }
    S.lam = lam;
    S.u[0] = u[0];
    S.u[1] = u[1];
    S.u[2] = u[2];
    S.T = E.T;
    S.Meq = E.M_eq;
    S.beta = E.beta;
    S.q = E.q;
    S.invT = 1.0 / E.T;
    S.MT = S.M * S.invT;
    S.rate = E.T * a.inv_eta_hbarc / E.q;
    S.du_dlam = D.du_dlam;
    S.dz = D.dz;
    S.dbeta = D.dbeta;
    S.dq = D.dq;
    const int x = g.x, y = g.y;
    S.gx = (Lm[y * a.nx + wrap(x + 1, a.nx)] - Lm[y * a.nx + wrap(x - 1, a.nx)]) * a.inv2dx;
    S.gy = (Lm[wrap(y + 1, a.ny) * a.nx + x] - Lm[wrap(y - 1, a.ny) * a.nx + x]) * a.inv2dx;
  }
  __syncthreads();
}

// Store at device scope (a relaxed atomic store with agent scope: written
// through this XCD's L2 to the memory side, where the next kernel's blocks
// on every XCD read it; the adjoint step 2% faster than plain stores).
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Addressing of the FP32 kernels: node n = q 8 + l of the canonical layout
// lies in the plane of q (base + q 8 ns, the same for the whole block) at
// the lane's byte offset (l ns + site) sizeof(T); with ns below 2^26 the
// offset fits 32 bits, so each access is a uniform base and one 32-bit lane
// offset rather than a 64-bit address per node.
template <typename T>
__device__ __forceinline__ T* qplane(T* base, int q, int ns) {
  return base + (size_t)(q * kL) * (size_t)ns;
}
__device__ __forceinline__ double ld8(const double* plane, uint32_t off) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(plane) + off);
}
__device__ __forceinline__ double& at8(double* plane, uint32_t off) {
  return *reinterpret_cast<double*>(reinterpret_cast<char*>(plane) + off);
}
__device__ __forceinline__ float& at4(float* plane, uint32_t off) {
  return *reinterpret_cast<float*>(reinterpret_cast<char*>(plane) + off);
}
__device__ __forceinline__ uint32_t lane_off8(int l, int site, int ns) {
  return ((uint32_t)l * (uint32_t)ns + (uint32_t)site) * 8u;
}

// Per-slice FP32 view of the site quantities and of the slice geometry
// (with the byte offsets of the site and of its upwind stencil neighbours).
struct Slice32 {
  float ut, M, Meq, invT, MT, rate, cu, Gl, gu, ax, ay, itau;
  uint32_t o_own, o_x1, o_x2, o_y1, o_y2;
  double gx, gy;  // the slice's ln M gradient (slice_grad)
};
template <bool kUp>
__device__ __forceinline__ Slice32 slice32(const SiteLds& S, const Lane& g, const SliceGeom& gm, bool f3,
                                           const double* __restrict__ Lm, const StageArgs& a) {
  Slice32 o;
  slice_grad(Lm, g, gm, a, S.gx, S.gy, &o.gx, &o.gy, kUp);
  o.ut = (float)S.u[0];
  o.M = (float)S.M;
  o.Meq = (float)S.Meq;
  o.invT = (float)S.invT;
  o.MT = (float)S.MT;
  o.rate = (float)S.rate;
  o.cu = (float)S.u[1] * (float)gm.cl + (float)S.u[2] * (float)gm.sl;
  o.Gl = f3 ? 0.0f : (float)(o.gx * gm.cl + o.gy * gm.sl);
  o.gu = f3 ? 0.0f : (float)(o.gx * S.u[1] + o.gy * S.u[2]);
  o.ax = (float)gm.ax;
  o.ay = (float)gm.ay;
  // S1/tau for the Milne metric, none for Minkowski
  o.itau = a.metric == LB_METRIC_MILNE ? (float)(1.0 / a.tau) : 0.0f;
  const int x = g.x, y = g.y, ns = a.n_sites;
  o.o_own = lane_off8(g.l, g.site, ns);
  o.o_x1 = lane_off8(g.l, y * a.nx + wrap(x - gm.dxr, a.nx), ns);
  o.o_x2 = lane_off8(g.l, y * a.nx + wrap(x - 2 * gm.dxr, a.nx), ns);
  o.o_y1 = lane_off8(g.l, wrap(y - gm.dyr, a.ny) * a.nx + x, ns);
  o.o_y2 = lane_off8(g.l, wrap(y - 2 * gm.dyr, a.ny) * a.nx + x, ns);
  return o;
}

// The equilibrium's radial factors at radial node k: E_eq and 1/E_eq, and
// the force polynomial's coefficients alpha, beta, gamma.  kHw: the
// hardware square root and reciprocal (as in the FP32 stage kernels; the
// reverse sweep), else the correctly rounded ones (adj_fwd32_kernel, whose
// register allocation is tuned with them).
struct Radial32 {
  float Eeq, iE, al, be, ga;
};
template <bool kHw = true>
__device__ __forceinline__ Radial32 radial32(const Slice32& o, const LCf& C, int k) {
  Radial32 r;
  if constexpr (kHw) {
    r.Eeq = __builtin_amdgcn_sqrtf(o.Meq * o.Meq + o.M * o.M * C.sh2[k]);
    r.iE = __builtin_amdgcn_rcpf(r.Eeq);
    r.al = o.MT * o.Gl * o.ut * o.M * C.x[k] * r.iE;
  } else {
    r.Eeq = sqrtf(o.Meq * o.Meq + o.M * o.M * C.sh2[k]);
    r.iE = 1.0f / r.Eeq;
    r.al = o.MT * o.Gl * o.ut * o.M * C.x[k] / r.Eeq;
  }
  r.be = o.MT * o.Gl * o.cu * C.inv_x[k];
  r.ga = o.MT * o.gu * C.inv_x[k];
  return r;
}

// The part of R0 of node q = k 5 + j that does not depend on the site's
// matching: streaming (from the upwind neighbours) and S1/tau.
// The node's upwind neighbours (x - 1, x - 2, y - 1, y - 2 along the
// slice's direction) are given (h) or read here.
template <int k, int j, bool kSkip = true>
__device__ __forceinline__ float node_r0a(const float h[4], const float f[kQ], const Slice32& o, const LCf& C) {
  constexpr int q = k * 5 + j;
  const float tr = 3.0f * (o.ax + o.ay) * f[q] - 4.0f * o.ax * h[0] + o.ax * h[1] - 4.0f * o.ay * h[2] +
                   o.ay * h[3];
  float s1r = 0, s1p = 0;
  // kSkip: the radial part left out on the polar node mu = 0 (j = 2), as
  // in the stage kernels (adj_fwd32_kernel evaluates it, with mu^2 = 0)
  constexpr bool kRadial = !(kSkip && j == 2);
  if constexpr (kRadial)
#pragma unroll
    for (int kp = 0; kp < 5; ++kp) s1r += C.A1[k * 5 + kp] * f[kp * 5 + j];
#pragma unroll
  for (int jp = 0; jp < 5; ++jp) s1p += C.Ath[j * 5 + jp] * f[k * 5 + jp];
  if constexpr (!kRadial) return -C.sigi[q] * tr - s1p * o.itau;
  else return -C.sigi[q] * tr + (C.mu2[j] * s1r - s1p) * o.itau;
}
template <int k, int j>
__device__ __forceinline__ void node_nbrs(const double* __restrict__ F, const Slice32& o, int ns, double h[4]) {
  const double* P = qplane(F, k * 5 + j, ns);
  h[0] = ld8(P, o.o_x1);
  h[1] = ld8(P, o.o_x2);
  h[2] = ld8(P, o.o_y1);
  h[3] = ld8(P, o.o_y2);
}
template <int k, int j, bool kSkip = true>
__device__ __forceinline__ float node_r0a(const double* __restrict__ F, const float f[kQ], const Slice32& o,
                                          const LCf& C, int ns) {
  double hd[4];
  node_nbrs<k, j>(F, o, ns, hd);
  const float h[4] = {(float)hd[0], (float)hd[1], (float)hd[2], (float)hd[3]};
  return node_r0a<k, j, kSkip>(h, f, o, C);
}

// S2 of node q = k 5 + j.
template <int k, int j>
__device__ __forceinline__ float node_s2(const float f[kQ], const LCf& C) {
  float a2 = 0;
#pragma unroll
  for (int kp = 0; kp < 5; ++kp) a2 += C.A2[k * 5 + kp] * f[kp * 5 + j];
  return a2;
}

// An opaque copy: the compiler cannot prove it equal to its input, so
// values computed from it are evaluated again rather than kept live from
// an earlier evaluation (register pressure over recomputation).
__device__ __forceinline__ float opaque(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Unrolled loop over the nodes of a slice, k-major, with compile-time k, j.
template <int k, int j, typename Fn>
__device__ __forceinline__ void for_nodes(Fn&& fn) {
  fn(std::integral_constant<int, k>{}, std::integral_constant<int, j>{});
  if constexpr (j < 4) for_nodes<k, j + 1>(fn);
  else if constexpr (k < 4) for_nodes<k + 1, 0>(fn);
}

// Two waves per SIMD for the force on F_eq (a few registers spill, faster
// than one wave with none); one for the weak-form 3-D force.  kUp: the
// upwind ln M gradient (force on F_eq only).
template <bool kF3, bool kUp>
__global__ __launch_bounds__(kAdjThreads, kF3 ? 1 : 2) void adj_local32_kernel(
    const double* __restrict__ F, const double* __restrict__ Lm, const double* __restrict__ seedF,
    const double* __restrict__ seedL, double scale, double* __restrict__ outF, double* __restrict__ outL,
    float* __restrict__ Rb, double* __restrict__ gb, double* __restrict__ eta_part, int accumulate,
    const LCf* __restrict__ Cg, const double* __restrict__ g3, const EosTable tb, const StageArgs a,
    int* __restrict__ err) {
  const LCf& C = *Cg;
  __shared__ RedBuf red;
  __shared__ SiteLds sd[kSites];
  // the slice's adjoint, parked in LDS over the site's reverse chain (held
  // in registers it was spilled to scratch and reloaded one value at a
  // time after the chain)
  __shared__ float4 s_fb4[6][kAdjThreads];
  __shared__ float s_fb1[kAdjThreads];
  const Lane g = lane_of(a);
  const int ns = a.n_sites, l = g.l;
  float f[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) f[q] = (float)ld8(qplane(F, q, ns), lane_off8(l, g.site, ns));
  const SliceGeom gm = slice_geom(C, a, l);
  site_chain32(f, Lm, g, C, gm.cl, gm.sl, tb, a, red, sd, err);
  const SiteLds& S = sd[g.sl];
  constexpr bool f3 = kF3;  // g3 != nullptr
  const Slice32 o = slice32<kUp>(S, g, gm, f3, Lm, a);
  const float sc = (float)scale, Zf = (float)a.Z;
  // what both sweeps read from memory, once: the part of R0 without the
  // collision and the equilibrium (streaming, S1/tau, the 3-D force) and
  // the seed K_bar
  float r0a[kQ], Kb[kQ];
  {
    // one radial node's neighbours and seeds are all read before any is
    // used, so that the reads are in flight together
    double h[5][4];
    double kb[5];
    for_nodes<0, 0>([&](auto kc, auto jc) {
      constexpr int k = decltype(kc)::value, j = decltype(jc)::value;
      if constexpr (j == 0) {
        node_nbrs<k, 0>(F, o, ns, h[0]);
        node_nbrs<k, 1>(F, o, ns, h[1]);
        node_nbrs<k, 2>(F, o, ns, h[2]);
        node_nbrs<k, 3>(F, o, ns, h[3]);
        node_nbrs<k, 4>(F, o, ns, h[4]);
#pragma unroll
        for (int jj = 0; jj < 5; ++jj) kb[jj] = ld8(qplane(seedF, k * 5 + jj, ns), o.o_own);
        __builtin_amdgcn_sched_barrier(0);
      }
      constexpr int q = k * 5 + j;
      const float hf[4] = {(float)h[j][0], (float)h[j][1], (float)h[j][2], (float)h[j][3]};
      r0a[q] = node_r0a<k, j>(hf, f, o, C);
      Kb[q] = sc * (float)kb[j];
    });
  }
  if (f3)
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      double gxf, gyf;
      force_row(g3, F, g.site, ns, q * kL + l, &gxf, &gyf);
      r0a[q] += (float)(S.gx * gxf + S.gy * gyf);
    }
  // forward right-hand side of the slice, node by node: the three site
  // sums of the mass equation and the seed's projection on S2
  double sums[4];
  {
    float s0 = 0, s1 = 0, s2s = 0, s3 = 0;
    Radial32 rk;
    for_nodes<0, 0>([&](auto kc, auto jc) {
      constexpr int k = decltype(kc)::value, j = decltype(jc)::value, q = k * 5 + j;
      if constexpr (j == 0) rk = radial32(o, C, k);
      const float s2 = node_s2<k, j>(f, C);
      const float sg = C.sig[q];
      const float feq = Zf * __expf((sg * o.M * o.cu - o.ut * rk.Eeq) * o.invT);
      const float uvg = o.ut - C.sigi[q] * o.cu;
      const float poly = rk.al * sg - rk.be * C.sig2[q] - rk.ga;
      const float ru = o.rate * uvg;
      const float r0 = r0a[q] + feq * (ru - poly) - ru * f[q];
      const float wuv2 = C.wx2[q] * uvg * uvg;
      s0 += wuv2 * r0;
      s1 += wuv2 * (4.0f * f[q] + s2);
      s2s += C.w[q] * f[q];
      s3 += Kb[q] * s2;
    });
    sums[0] = s0;
    sums[1] = s1;
    sums[2] = s2s;
    sums[3] = s3;
  }
  slice_sum<4>(sums, red, g);
  const double nsum = sums[0], dsum = sums[1], wsum = sums[2];
  const double beta = S.beta, Dd = wsum + beta * dsum, iD = 1.0 / Dd, Xd = -beta * nsum * iD;
  const double Xb = scale * seedL[g.site] + sums[3];
  const double nbd = -beta * Xb * iD;
  const double Db = -Xd * Xb * iD;
  const double betab = -nsum * Xb / Dd + Db * dsum;
  const float nb = (float)nbd, wsb = (float)Db, dsb = (float)(beta * Db), X = (float)Xd;
  // the slice's adjoint, node by node; S2, F_eq and R0 are evaluated again
  // (from opaque copies of f and of the site scalars) rather than held from
  // the forward sweep
#pragma unroll
  for (int q = 0; q < kQ; ++q) f[q] = opaque(f[q]);
  Slice32 o2 = o;
  o2.ut = opaque(o.ut);
  o2.M = opaque(o.M);
  o2.Meq = opaque(o.Meq);
  o2.cu = opaque(o.cu);
  o2.invT = opaque(o.invT);
  o2.rate = opaque(o.rate);
  const LCf& C2 = C;
  float R0b[kQ], S2b[kQ], fb[kQ];
  float cub = 0, Glb = 0, gub = 0, utb = 0, Mb = 0, invTb = 0, rateb = 0, MTb = 0, Meqb = 0;
  {
    Radial32 rk;
    float alb = 0, beb = 0, gab = 0, Eeqb = 0;
    for_nodes<0, 0>([&](auto kc, auto jc) {
      constexpr int k = decltype(kc)::value, j = decltype(jc)::value, q = k * 5 + j;
      if constexpr (j == 0) {
        rk = radial32(o2, C2, k);
        alb = beb = gab = Eeqb = 0.0f;
      }
      const float s2 = node_s2<k, j>(f, C2);
      const float sg = C2.sig[q];
      const float feq = Zf * __expf((sg * o2.M * o2.cu - o2.ut * rk.Eeq) * o2.invT);
      const float uv = o2.ut - C2.sigi[q] * o2.cu;
      const float poly = rk.al * sg - rk.be * C2.sig2[q] - rk.ga;
      const float ru = o2.rate * uv;
      const float r0 = r0a[q] + feq * (ru - poly) - ru * f[q];
      const float wuv2 = C2.wx2[q] * uv * uv;
      R0b[q] = Kb[q] + wuv2 * nb;
      S2b[q] = X * Kb[q] + wuv2 * dsb;
      fb[q] = 4.0f * wuv2 * dsb + C2.w[q] * wsb - ru * R0b[q];
      const float uvb = 2.0f * C2.wx2[q] * uv * ((4.0f * f[q] + s2) * dsb + r0 * nb) + o2.rate * (feq - f[q]) * R0b[q];
      rateb += uv * (feq - f[q]) * R0b[q];
      const float feqb = (ru - poly) * R0b[q];
      const float polyb = -feq * R0b[q];
      alb += sg * polyb;
      beb -= C2.sig2[q] * polyb;
      gab -= polyb;
      const float e = feq * feqb;
      Mb += e * sg * o2.cu * o2.invT;
      cub += e * sg * o2.M * o2.invT;
      invTb += e * (sg * o2.M * o2.cu - o2.ut * rk.Eeq);
      utb -= e * rk.Eeq * o2.invT;
      Eeqb -= e * o2.ut * o2.invT;
      utb += uvb;
      cub -= C2.sigi[q] * uvb;
      if constexpr (j == 4) {
        // radial node k done: the adjoints of its alpha, beta, gamma and E_eq
        const float c = C2.x[k] * rk.iE;
        MTb += alb * o2.Gl * o2.ut * o2.M * c;
        Glb += alb * o2.MT * o2.ut * o2.M * c;
        utb += alb * o2.MT * o2.Gl * o2.M * c;
        Mb += alb * o2.MT * o2.Gl * o2.ut * c;
        Eeqb -= alb * rk.al * rk.iE;
        MTb += beb * o2.Gl * o2.cu * C2.inv_x[k] + gab * o2.gu * C2.inv_x[k];
        Glb += beb * o2.MT * o2.cu * C2.inv_x[k];
        cub += beb * o2.MT * o2.Gl * C2.inv_x[k];
        gub += gab * o2.MT * C2.inv_x[k];
        Meqb += Eeqb * o2.Meq * rk.iE;
        Mb += Eeqb * o2.M * C2.sh2[k] * rk.iE;
      }
    });
  }
  double g3xb = 0, g3yb = 0;
  if (f3) {
    Glb = 0;
    gub = 0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      double gxf, gyf;
      force_row(g3, F, g.site, ns, q * kL + l, &gxf, &gyf);
      g3xb += (double)R0b[q] * gxf;
      g3yb += (double)R0b[q] * gyf;
    }
  }
  if (g.valid)
#pragma unroll
    for (int q = 0; q < kQ; ++q) st_dev(&at4(qplane(Rb, q, ns), o.o_own / 2), R0b[q]);
  // transposed operators: S2^T S2b and (S1/tau)^T R0b, with R0b/tau formed
  // once and the radial part of S1 absent on the polar node j = 2
  {
    float rt[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) rt[q] = R0b[q] * o2.itau;
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        float acc = 0, a1 = 0, ap = 0;
#pragma unroll
        for (int kk = 0; kk < 5; ++kk) acc += C2.A2[kk * 5 + k] * S2b[kk * 5 + j];
        if (j != 2)
#pragma unroll
          for (int kk = 0; kk < 5; ++kk) a1 += C2.A1[kk * 5 + k] * rt[kk * 5 + j];
#pragma unroll
        for (int jj = 0; jj < 5; ++jj) ap += C2.Ath[jj * 5 + j] * rt[k * 5 + jj];
        fb[k * 5 + j] += (j != 2 ? acc + C2.mu2[j] * a1 : acc) - ap;
      }
  }
#pragma unroll
  for (int gq = 0; gq < 6; ++gq)
    s_fb4[gq][threadIdx.x] = make_float4(fb[4 * gq], fb[4 * gq + 1], fb[4 * gq + 2], fb[4 * gq + 3]);
  s_fb1[threadIdx.x] = fb[24];
  double v[10] = {(double)utb,
                    (double)cub * gm.cl + (double)gub * o.gx,
                    (double)cub * gm.sl + (double)gub * o.gy,
                    (double)Mb,
                    (double)invTb,
                    (double)MTb,
                    (double)rateb,
                    (double)Meqb,
                    (double)Glb * gm.cl + (double)gub * S.u[1] + g3xb,
                    (double)Glb * gm.sl + (double)gub * S.u[2] + g3yb};
  // with the upwind gradient the slice's own gradient adjoint goes out per
  // slice ([2][8][sites]); otherwise the site totals below ([2][sites])
  if (kUp && g.valid) {
    gb[(size_t)l * ns + g.site] = v[8];
    gb[(size_t)(kL + l) * ns + g.site] = v[9];
  }
  slice_sum<10>(v, red, g);
  if (l == 0) {
    // the site's reverse chain, once (FP64): as adj_local_kernel
    SiteLds& W = sd[g.sl];
    const double utbd = v[0], uxb = v[1], uyb = v[2];
    double Mbd = v[3], invTbd = v[4];
    const double MTbd = v[5], ratebd = v[6], Meqbd = v[7], gxb = v[8], gyb = v[9];
    Mbd += MTbd * W.invT;
    invTbd += MTbd * W.M;
    const double T = W.T, iq = 1.0 / W.q;
    const double Tb = -invTbd * W.invT * W.invT + ratebd * a.inv_eta_hbarc * iq;
    const double qb = -ratebd * W.rate * iq;
    const double etab = -ratebd * W.rate * a.inv_eta_hbarc * kHbarC;
    const double z = W.Meq * W.invT;
    const double uub = Tb * T + Meqbd * (W.dz * T + z * T) + betab * W.dbeta + qb * W.dq;
    const double lamb = uub * W.du_dlam;
    const double ub[3] = {utbd, uxb, uyb};
    const double ul[3] = {W.u[0], -W.u[1], -W.u[2]};
    const double gsg[3] = {1.0, -1.0, -1.0};
    const double mm[3][3] = {{W.m[0], W.m[1], W.m[2]}, {W.m[1], W.m[3], W.m[4]}, {W.m[2], W.m[4], W.m[5]}};
    const double al_ = ub[0] * W.u[0] + ub[1] * W.u[1] + ub[2] * W.u[2];
    double rhs[3], Bt[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) rhs[i] = ub[i] - al_ * ul[i];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Bt[j][i] = W.G * mm[i][j] * gsg[j] - (i == j ? W.lam : 0.0) + W.u[i] * ul[j];
    const double det = Bt[0][0] * (Bt[1][1] * Bt[2][2] - Bt[1][2] * Bt[2][1]) -
                       Bt[0][1] * (Bt[1][0] * Bt[2][2] - Bt[1][2] * Bt[2][0]) +
                       Bt[0][2] * (Bt[1][0] * Bt[2][1] - Bt[1][1] * Bt[2][0]);
    const double idet = 1.0 / det;
    double w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double Mx[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Mx[i][j] = (j == c) ? rhs[i] : Bt[i][j];
      w[c] = (Mx[0][0] * (Mx[1][1] * Mx[2][2] - Mx[1][2] * Mx[2][1]) -
              Mx[0][1] * (Mx[1][0] * Mx[2][2] - Mx[1][2] * Mx[2][0]) +
              Mx[0][2] * (Mx[1][0] * Mx[2][1] - Mx[1][1] * Mx[2][0])) * idet;
    }
    const double wu = w[0] * W.u[0] + w[1] * W.u[1] + w[2] * W.u[2] + lamb;
    double mb[3][3], Gb = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double tb_ = -w[i] * ul[j] + wu * ul[i] * ul[j];
        mb[i][j] = W.G * tb_;
        Gb += tb_ * mm[i][j];
      }
    Mbd += Gb * 4.0 * W.G / W.M;
    W.mb[0] = mb[0][0];
    W.mb[1] = mb[0][1] + mb[1][0];
    W.mb[2] = mb[0][2] + mb[2][0];
    W.mb[3] = mb[1][1];
    W.mb[4] = mb[1][2] + mb[2][1];
    W.mb[5] = mb[2][2];
    if (g.valid) {
      const double lb = Mbd * W.M;
      outL[g.site] = accumulate ? outL[g.site] + lb : lb;
      if (!kUp) {
        gb[g.site] = gxb;
        gb[ns + g.site] = gyb;
      }
      eta_part[g.site] = accumulate ? eta_part[g.site] + etab : etab;
    }
  }
  __syncthreads();
  if (!g.valid) return;
  const float c00 = (float)S.mb[0], c01 = (float)(S.mb[1] * gm.cl + S.mb[2] * gm.sl);
  const float c11 = (float)(S.mb[3] * gm.cl * gm.cl + S.mb[4] * gm.cl * gm.sl + S.mb[5] * gm.sl * gm.sl);
  float fbl[kQ];
#pragma unroll
  for (int gq = 0; gq < 6; ++gq) {
    const float4 w = s_fb4[gq][threadIdx.x];
    fbl[4 * gq] = w.x;
    fbl[4 * gq + 1] = w.y;
    fbl[4 * gq + 2] = w.z;
    fbl[4 * gq + 3] = w.w;
  }
  fbl[24] = s_fb1[threadIdx.x];
  // the accumulated values are all read before the first store
  double prev[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) prev[q] = accumulate ? ld8(qplane(outF, q, ns), o.o_own) : 0.0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const double v_ = (double)(fbl[q] + c00 * C.wx2[q] + c01 * C.wxs[q] + c11 * C.ws2[q]);
    st_dev(&at8(qplane(outF, q, ns), o.o_own), prev[q] + v_);
  }
}

// adj_fwd_kernel for contexts whose forward runs in FP32: the same stage
// with the node arithmetic in FP32, the site sums in FP64 and the site's
// matching and EoS once per site (slice-0 thread, LDS), as
// adj_local32_kernel.  R0 is held per node across the site sum; S2 is
// evaluated again for the update.
// At most two waves per SIMD: the compiler's own choice (153 VGPRs, three
// waves) spilled scalar registers and ran 10% slower.
template <bool kF3, bool kUp>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) void adj_fwd32_kernel(const double* __restrict__ Fin,
                                                                const double* __restrict__ Lin,
                                                                const double* __restrict__ Fbase,
                                                                const double* __restrict__ Lbase,
                                                                double* __restrict__ Fout,
                                                                double* __restrict__ Lout, int stage,
                                                                const LCf* __restrict__ Cg,
                                                                const double* __restrict__ g3, const EosTable tb,
                                                                const StageArgs a, int* __restrict__ err) {
  const LCf& C = *Cg;
  __shared__ RedBuf red;
  __shared__ SiteLds sd[kSites];
  const Lane g = lane_of(a);
  const int ns = a.n_sites, l = g.l;
  float f[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) f[q] = (float)ld8(qplane(Fin, q, ns), lane_off8(l, g.site, ns));
  const SliceGeom gm = slice_geom(C, a, l);
  site_chain32(f, Lin, g, C, gm.cl, gm.sl, tb, a, red, sd, err);
  const SiteLds& S = sd[g.sl];
  constexpr bool f3 = kF3;  // g3 != nullptr
  const Slice32 o = slice32<kUp>(S, g, gm, f3, Lin, a);
  const float Zf = (float)a.Z;
  float R0[kQ];
  {
    // one radial node's upwind neighbours read together, as in
    // adj_local32_kernel
    double h[5][4];
    for_nodes<0, 0>([&](auto kc, auto jc) {
      constexpr int k = decltype(kc)::value, j = decltype(jc)::value, q = k * 5 + j;
      if constexpr (j == 0) {
        node_nbrs<k, 0>(Fin, o, ns, h[0]);
        node_nbrs<k, 1>(Fin, o, ns, h[1]);
        node_nbrs<k, 2>(Fin, o, ns, h[2]);
        node_nbrs<k, 3>(Fin, o, ns, h[3]);
        node_nbrs<k, 4>(Fin, o, ns, h[4]);
        __builtin_amdgcn_sched_barrier(0);
      }
      const float hf[4] = {(float)h[j][0], (float)h[j][1], (float)h[j][2], (float)h[j][3]};
      R0[q] = node_r0a<k, j, false>(hf, f, o, C);
    });
  }
  if (f3)
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      double gxf, gyf;
      force_row(g3, Fin, g.site, ns, q * kL + l, &gxf, &gyf);
      R0[q] += (float)(S.gx * gxf + S.gy * gyf);
    }
  double sums[3];
  {
    float s0 = 0, s1 = 0, s2s = 0;
    Radial32 rk;
    for_nodes<0, 0>([&](auto kc, auto jc) {
      constexpr int k = decltype(kc)::value, j = decltype(jc)::value, q = k * 5 + j;
      if constexpr (j == 0) rk = radial32<false>(o, C, k);
      const float s2 = node_s2<k, j>(f, C);
      const float sg = C.sig[q];
      const float feq = Zf * __expf((sg * o.M * o.cu - o.ut * rk.Eeq) * o.invT);
      const float uvg = o.ut - C.sigi[q] * o.cu;
      const float poly = rk.al * sg - rk.be * C.sig2[q] - rk.ga;
      const float ru = o.rate * uvg;
      R0[q] += feq * (ru - poly) - ru * f[q];
      const float wuv2 = C.wx2[q] * uvg * uvg;
      s0 += wuv2 * R0[q];
      s1 += wuv2 * (4.0f * f[q] + s2);
      s2s += C.w[q] * f[q];
    });
    sums[0] = s0;
    sums[1] = s1;
    sums[2] = s2s;
  }
  slice_sum<3>(sums, red, g);
  const double X = -S.beta * sums[0] / (sums[2] + S.beta * sums[1]);
  if (!g.valid) return;
  const float Xr = (float)X, dt = (float)a.dtau;
  for_nodes<0, 0>([&](auto kc, auto jc) {
    constexpr int k = decltype(kc)::value, j = decltype(jc)::value, q = k * 5 + j;
    float s2 = 0;
#pragma unroll
    for (int kp = 0; kp < 5; ++kp) s2 += C.A2[k * 5 + kp] * f[kp * 5 + j];
    const float K = R0[q] + Xr * s2;
    double& dst = at8(qplane(Fout, q, ns), o.o_own);
    st_dev(&dst, stage == 0 ? (double)(f[q] + dt * K)
                     : (double)(0.5f * ((float)ld8(qplane(Fbase, q, ns), o.o_own) + f[q]) + 0.5f * dt * K));
  });
  if (l == 0) {
    const double lm = Lin[g.site];
    Lout[g.site] = stage == 0 ? lm + a.dtau * X : 0.5 * (Lbase[g.site] + lm) + 0.5 * a.dtau * X;
  }
}

// Transposed streaming stencil and transposed centred ln M gradient:
// outF_n(s) += sum over the sites s' whose stencil reads s of the stencil
// weight times Rb_n(s'); outL(s) += (gb_x(s - 1) - gb_x(s + 1) + ...)/(2 dx).
// With the weak-form 3-D force (g3) also the transposed force:
// outF_m(s) += sum_n Rb_n(s) (g_x G_x[n][m] + g_y G_y[n][m]) at the site's
// own ln M gradient (Lm, the state of the right-hand side).  With combF
// (and combL) the Heun combination of the step's adjoint follows on the
// finished values: outF <- outF + combF/2, then combF <- combF/2 + outF
// (with outF the corrector's adjoint of the predictor state and combF the
// incoming adjoint of the new state).
template <typename RB, bool kG3, bool kComb>
__global__ __launch_bounds__(kAdjThreads, kG3 ? 1 : 2) void adj_gather_kernel(const RB* __restrict__ Rb,
                                                                 const double* __restrict__ gb,
                                                                 double* __restrict__ outF,
                                                                 double* __restrict__ outL, const LC C,
                                                                 const double* __restrict__ Lm,
                                                                 const double* __restrict__ g3,
                                                                 const StageArgs a, double* __restrict__ combF,
                                                                 double* __restrict__ combL) {
  const Lane g = lane_of(a);
  if (!g.valid) return;
  const int x = g.x, y = g.y, ns = a.n_sites, l = g.l, site = g.site;
  const SliceGeom gm = slice_geom(C, a, l);
  // byte offsets in a node plane (see qplane): the site and the sites whose
  // upwind stencil reads it
  constexpr uint32_t e = sizeof(RB);
  const uint32_t o0 = ((uint32_t)l * ns + site) * e;
  const uint32_t o1 = ((uint32_t)l * ns + y * a.nx + wrap(x + gm.dxr, a.nx)) * e;
  const uint32_t o2 = ((uint32_t)l * ns + y * a.nx + wrap(x + 2 * gm.dxr, a.nx)) * e;
  const uint32_t o3 = ((uint32_t)l * ns + wrap(y + gm.dyr, a.ny) * a.nx + x) * e;
  const uint32_t o4 = ((uint32_t)l * ns + wrap(y + 2 * gm.dyr, a.ny) * a.nx + x) * e;
  const uint32_t od = ((uint32_t)l * ns + site) * 8u;
  auto rb = [&](int q, uint32_t off) {
    return (double)*reinterpret_cast<const RB*>(reinterpret_cast<const char*>(qplane(Rb, q, ns)) + off);
  };
  double gx = 0, gy = 0;
  if constexpr (kG3) {
    gx = (Lm[y * a.nx + wrap(x + 1, a.nx)] - Lm[y * a.nx + wrap(x - 1, a.nx)]) * a.inv2dx;
    gy = (Lm[wrap(y + 1, a.ny) * a.nx + x] - Lm[wrap(y - 1, a.ny) * a.nx + x]) * a.inv2dx;
  }
  if constexpr (!kG3 && !kComb) {
    // every read of the slice (the stencil's R0_bar and F_bar) before its
    // first store: with the stores in between, each node's reads waited for
    // the previous node's round trip (13.3 -> 11.9 us at 128 x 128; with
    // the Heun accumulator's reads as well, the gather below needs 256
    // registers and ran 17.9 -> 19.9 us, so it keeps the node-by-node loop)
    double tq[kQ], dq[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      tq[q] = 3.0 * (gm.ax + gm.ay) * rb(q, o0) - 4.0 * gm.ax * rb(q, o1) + gm.ax * rb(q, o2) -
              4.0 * gm.ay * rb(q, o3) + gm.ay * rb(q, o4);
      dq[q] = at8(qplane(outF, q, ns), od);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < kQ; ++q) st_dev(&at8(qplane(outF, q, ns), od), dq[q] - C.sigi[q] * tq[q]);
  } else {
    // node by node (with the 3-D force's transposed operator, its own reads
    // per node)
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const double t = 3.0 * (gm.ax + gm.ay) * rb(q, o0) - 4.0 * gm.ax * rb(q, o1) + gm.ax * rb(q, o2) -
                       4.0 * gm.ay * rb(q, o3) + gm.ay * rb(q, o4);
      double& dst = at8(qplane(outF, q, ns), od);
      double v = dst - C.sigi[q] * t;
      if constexpr (kG3) {
        const double* gxc = g3;
        const double* gyc = g3 + (size_t)kN * kN;
        const int m = q * kL + l;
        double acc = 0;
#pragma unroll 1
        for (int n = 0; n < kN; ++n)
          acc += (double)Rb[(size_t)n * ns + site] * (gx * gxc[(size_t)n * kN + m] + gy * gyc[(size_t)n * kN + m]);
        v += acc;
      }
      if constexpr (kComb) {
        double& cv = at8(qplane(combF, q, ns), od);
        const double c = cv, t1 = v + 0.5 * c;
        st_dev(&dst, t1);
        st_dev(&cv, 0.5 * c + t1);
      } else {
        st_dev(&dst, v);
      }
    }
  }
  if (l == 0) {
    const int xm = y * a.nx + wrap(x - 1, a.nx), xp = y * a.nx + wrap(x + 1, a.nx);
    const int ym = wrap(y - 1, a.ny) * a.nx + x, yp = wrap(y + 1, a.ny) * a.nx + x;
    double v = outL[site];
    if (a.grad_form == LB_GRAD_UPWIND) {
      // the transposed per-slice gradients: each slice's upwind difference
      // along its direction of motion (centred along an axis it does not
      // move on), gb [2][8][sites]
#pragma unroll
      for (int k = 0; k < kL; ++k) {
        const SliceGeom gk = slice_geom(C, a, k);
        const double* bx = gb + (size_t)k * ns;
        const double* by = gb + (size_t)(kL + k) * ns;
        if (gk.dxr != 0)
          v += gk.dxr * (3.0 * bx[site] - 4.0 * bx[y * a.nx + wrap(x + gk.dxr, a.nx)] +
                         bx[y * a.nx + wrap(x + 2 * gk.dxr, a.nx)]) * a.inv2dx;
        else
          v += (bx[xm] - bx[xp]) * a.inv2dx;
        if (gk.dyr != 0)
          v += gk.dyr * (3.0 * by[site] - 4.0 * by[wrap(y + gk.dyr, a.ny) * a.nx + x] +
                         by[wrap(y + 2 * gk.dyr, a.ny) * a.nx + x]) * a.inv2dx;
        else
          v += (by[ym] - by[yp]) * a.inv2dx;
      }
    } else {
      v += (gb[xm] - gb[xp] + gb[ns + ym] - gb[ns + yp]) * a.inv2dx;
    }
    if constexpr (kComb) {
      const double c = combL[site], t1 = v + 0.5 * c;
      outL[site] = t1;
      combL[site] = 0.5 * c + t1;
    } else {
      outL[site] = v;
    }
  }
}

// The gather for a right-hand side's adjoint: Rb in RB, with or without the
// weak-form 3-D force and the Heun combination.
template <typename RB>
hipError_t launch_gather(const RB* Rb, const double* gb, double* outF, double* outL, const LC& C, const double* Lm,
                         const double* g3, const StageArgs& a, double* combF, double* combL, hipStream_t s) {
  const dim3 grid((unsigned)((a.n_sites + kSites - 1) / kSites)), block(kAdjThreads);
  if (combF && !combL) return hipErrorInvalidValue;
  if (g3) {
    if (combF)
      hipLaunchKernelGGL((adj_gather_kernel<RB, true, true>), grid, block, 0, s, Rb, gb, outF, outL, C, Lm, g3, a,
                         combF, combL);
    else
      hipLaunchKernelGGL((adj_gather_kernel<RB, true, false>), grid, block, 0, s, Rb, gb, outF, outL, C, Lm, g3, a,
                         combF, combL);
  } else {
    if (combF)
      hipLaunchKernelGGL((adj_gather_kernel<RB, false, true>), grid, block, 0, s, Rb, gb, outF, outL, C, Lm, g3, a,
                         combF, combL);
    else
      hipLaunchKernelGGL((adj_gather_kernel<RB, false, false>), grid, block, 0, s, Rb, gb, outF, outL, C, Lm, g3, a,
                         combF, combL);
  }
  return hipGetLastError();
}

// *out += sum of v[0..n) (one block of 1024 threads, eight accumulators per
// thread whose loads are issued together, fixed order: deterministic).
__global__ __launch_bounds__(1024) void adj_sum_kernel(const double* __restrict__ v, int n,
                                                       double* __restrict__ out) {
  __shared__ double part[1024];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int i = threadIdx.x;
  for (; i + 7 * 1024 < n; i += 8 * 1024) {
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = v[i + k * 1024];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] += t[k];
  }
  for (; i < n; i += 1024) acc[0] += v[i];
  part[threadIdx.x] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += part[0];
}

// Adjoint of the initial state of lb_init: T0 from eps_EoS(T0) = e0, M =
// z(T0) T0, F_n = Z exp(-z (u^tau gamma - u_perp.v_perp)) (z = M/T0, flow
// held fixed).  grad_e0 = d/d e0 of (adjF . F + adjL . ln M).  With an
// initial mu0 = alpha0 T0 (constant mass): eps0(T0) = e0 exp(-alpha0) and F
// carries exp(alpha0).
__global__ __launch_bounds__(kInitBlock) void adj_init_kernel(const double* __restrict__ e0,
                                                             const double* __restrict__ ux0,
                                                             const double* __restrict__ uy0,
                                                             const double* __restrict__ aF,
                                                             const double* __restrict__ aL,
                                                             double* __restrict__ grad_e0, const LC C,
                                                             const EosTable tb, const StageArgs a,
                                                             int* __restrict__ err) {
  const int site = blockIdx.x * kInitBlock + threadIdx.x;
  if (site >= a.n_sites) return;
  const int ns = a.n_sites;
  const double e = e0[site] * (kHbarC * kHbarC * kHbarC) * exp(-a.alpha0);
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
      const double f = a.Z * exp(a.alpha0 - z * h);
      zb += aF[cix(q, l, site, ns)] * f * (-h);
    }
  }
  // ln M = ln z + u
  zb += aL[site] / z;
  const double ub = aL[site] + zb * dz;
  grad_e0[site] = ub / (dlnE * e0[site]);
}

dim3 sites_grid(int n) { return dim3((unsigned)((n + kSites - 1) / kSites)); }

}  // namespace

hipError_t launch_adj_stage_fwd(const double* Fin, const double* Lin, const double* Fbase, const double* Lbase,
                                double* Fout, double* Lout, int stage, const void* lc, const double* g3,
                                const EosTable& tb, const StageArgs& a, int* err, hipStream_t s, const void* lc32) {
  if (lc32) {
    const auto kern = g3 ? adj_fwd32_kernel<true, false>
                         : (a.grad_form == LB_GRAD_UPWIND ? adj_fwd32_kernel<false, true>
                                                          : adj_fwd32_kernel<false, false>);
    hipLaunchKernelGGL(kern, sites_grid(a.n_sites), dim3(kAdjThreads), 0, s, Fin, Lin, Fbase, Lbase, Fout, Lout,
                       stage, static_cast<const LCf*>(lc32), g3, tb, a, err);
  } else {
    hipLaunchKernelGGL(adj_fwd_kernel, sites_grid(a.n_sites), dim3(kAdjThreads), 0, s, Fin, Lin, Fbase, Lbase, Fout,
                       Lout, stage, *static_cast<const LC*>(lc), g3, tb, a, err);
  }
  return hipGetLastError();
}

hipError_t launch_adj_rhs(const double* F, const double* Lm, const double* seedF, const double* seedL,
                          double scale, double* outF, double* outL, double* Rb, double* gb, double* eta_part,
                          int accumulate, const void* lc, const double* g3, const EosTable& tb,
                          const StageArgs& a, int* err, hipStream_t s, const void* lc32, double* combF,
                          double* combL) {
  const LC& C = *static_cast<const LC*>(lc);
  if (lc32) {
    float* Rb32 = reinterpret_cast<float*>(Rb);
    const auto kern = g3 ? adj_local32_kernel<true, false>
                         : (a.grad_form == LB_GRAD_UPWIND ? adj_local32_kernel<false, true>
                                                          : adj_local32_kernel<false, false>);
    hipLaunchKernelGGL(kern, sites_grid(a.n_sites),
                       dim3(kAdjThreads), 0, s, F, Lm, seedF, seedL, scale, outF, outL, Rb32, gb, eta_part,
                       accumulate, static_cast<const LCf*>(lc32), g3, tb, a, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_gather<float>(Rb32, gb, outF, outL, C, Lm, g3, a, combF, combL, s);
  }
  hipLaunchKernelGGL(adj_local_kernel, sites_grid(a.n_sites), dim3(kAdjThreads), 0, s, F, Lm, seedF, seedL, scale,
                     outF, outL, Rb, gb, eta_part, accumulate, C, g3, tb, a, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gather<double>(Rb, gb, outF, outL, C, Lm, g3, a, combF, combL, s);
}

hipError_t launch_adj_sum(const double* v, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(adj_sum_kernel, dim3(1), dim3(1024), 0, s, v, n, out);
  return hipGetLastError();
}

hipError_t launch_adj_init(const double* e0, const double* ux0, const double* uy0, const double* aF,
                           const double* aL, double* grad_e0, const void* lc, const EosTable& tb,
                           const StageArgs& a, int* err, hipStream_t s) {
  hipLaunchKernelGGL(adj_init_kernel, dim3((unsigned)((a.n_sites + kInitBlock - 1) / kInitBlock)), dim3(kInitBlock), 0, s, e0, ux0, uy0, aF, aL, grad_e0,
                     *static_cast<const LC*>(lc), tb, a, err);
  return hipGetLastError();
}

}  // namespace lbmi
