// C ABI of the lattice-Boltzmann library: parameter validation, workspace
// carving, host setup upload, kernel launches (declarations in include/lb.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lb.h"
#include "generic.hpp"
#include "host_setup.hpp"
#include "kernels.hpp"

using namespace lbmi;

struct lb_ctx {
  lb_params p;
  hipStream_t stream = nullptr;
  int device = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  void* F[3] = {nullptr, nullptr, nullptr};
  double* lnM[3] = {nullptr, nullptr, nullptr};
  double* sc[3] = {nullptr, nullptr, nullptr};  // site scalars of each state
  void* cst = nullptr;                          // device copy of the stage constants
  EosTable* tbd = nullptr;                      // device copy of the EoS table descriptor
  int cur = 0;  // index of the current state
  int* err = nullptr;
  EosTable tb{};
  HostLattice lat;
  LatticeConst<float, 5, 5> cf{};
  LatticeConst<double, 5, 5> cd{};
  void* lc32 = nullptr;  // device copy of cf (the adjoint's FP32 kernels)
  double* g3 = nullptr;  // dense weak-form force operators [2][N][N] (3-D force only)
  double tau = 0;
  bool initialised = false;
  bool generic = false;  // momentum lattice other than 5 x 5 x 8: FP64 kernels of lb_generic.hip
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev;  // 3 per step
  size_t ev_used = 0;
  double prof_ms[2] = {0, 0};
  int64_t prof_n[2] = {0, 0};
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t F[3], lnM[3], sc[3], cst, tbd, pts, inv_ek, inv_ee, gpts, err, lc32, cst64, g3, total;
};

std::string validate(const lb_params* p) {
  if (!p) return "params is NULL";
  if (!(p->n_xi == 5 && p->n_theta == 5 && p->n_phi == 4)) {
    // other lattices run on the generic FP64 kernels
    if (!gen_supported(p->n_xi, p->n_theta, p->n_phi))
      return "momentum lattice: n_xi and n_theta in {3, 5, 7}, n_phi in {3, 4, 5}";
    if (p->precision != LB_FP64) return "a momentum lattice other than 5 x 5 x 8 runs in precision LB_FP64";
    if (p->force_form != LB_FORCE_FEQ) return "a momentum lattice other than 5 x 5 x 8 takes force_form LB_FORCE_FEQ";
    if (p->particle_number != LB_N_FREE) return "a momentum lattice other than 5 x 5 x 8 takes particle_number LB_N_FREE";
  }
  if (!(p->z0 > 0) || !std::isfinite(p->z0)) return "z0 must be finite and > 0";
  if (!(p->Z > 0) || !std::isfinite(p->Z)) return "Z must be finite and > 0";
  if (p->nx < 1 || p->ny < 1) return "nx and ny must be >= 1";
  // a node plane (8 slices x sites, FP64) must be addressable with 32-bit byte offsets
  if ((int64_t)p->nx * p->ny >= ((int64_t)1 << 26)) return "grid too large (nx*ny must be below 2^26 sites)";
  {
    // the kernels address one distribution buffer with 32-bit byte offsets
    const int64_t elt = p->precision == LB_FP64 ? 8 : 4;
    const int64_t nodes = (int64_t)p->n_xi * p->n_theta * 2 * p->n_phi;
    if ((int64_t)p->nx * p->ny * nodes * elt > (int64_t)0xFFFFFFFF)
      return "grid too large: one distribution buffer (nx*ny*N values) must stay below 4 GiB";
  }
  if (!(p->dx_fm > 0) || !std::isfinite(p->dx_fm)) return "dx_fm must be finite and > 0";
  if (!std::isfinite(p->tau0_fm)) return "tau0_fm must be finite";
  if (p->metric == LB_METRIC_MILNE && !(p->tau0_fm > 0)) return "tau0_fm must be > 0 for the Milne metric";
  if (p->metric != LB_METRIC_MILNE && p->metric != LB_METRIC_MINKOWSKI) return "unknown metric";
  if (!(p->eta_over_s > 0)) return "eta_over_s must be > 0 (or +inf)";
  if (p->taur_rule != LB_TAUR_CE && p->taur_rule != LB_TAUR_MASSLESS) return "unknown taur_rule";
  if (p->precision != LB_FP64 && p->precision != LB_FP32_FP64MATCH) return "unknown precision";
  if (p->eos_kind == LB_EOS_TANH_P || p->eos_kind == LB_EOS_TANH_S) {
    if (!(p->eos_g > 0) || !(p->eos_width_GeV > 0) || !std::isfinite(p->eos_Tc_GeV))
      return "tanh EoS needs g > 0, width > 0, finite Tc";
  } else if (p->eos_kind == LB_EOS_CONST_MASS) {
    if (!(p->eos_mass_GeV > 0) || !std::isfinite(p->eos_mass_GeV)) return "constant-mass EoS needs mass > 0";
  } else if (p->eos_kind == LB_EOS_TABLE) {
    if (!p->eos_T_GeV || !p->eos_s_GeV3 || p->eos_n < 4) return "tabulated EoS needs eos_T, eos_s and eos_n >= 4";
    for (int i = 0; i < p->eos_n; ++i) {
      if (!(p->eos_T_GeV[i] > 0) || !std::isfinite(p->eos_T_GeV[i]) || !(p->eos_s_GeV3[i] > 0) ||
          !std::isfinite(p->eos_s_GeV3[i]))
        return "tabulated EoS: T and s must be finite and > 0";
      if (i > 0 && !(p->eos_T_GeV[i] > p->eos_T_GeV[i - 1])) return "tabulated EoS: T must increase strictly";
    }
    if (!std::isfinite(p->eos_p0_GeV4)) return "tabulated EoS: eos_p0 must be finite";
    if (!(p->T_min_GeV >= p->eos_T_GeV[0]) || !(p->T_max_GeV <= p->eos_T_GeV[p->eos_n - 1]))
      return "tabulated EoS: [T_min, T_max] must lie inside the table";
  } else {
    return "unknown eos_kind";
  }
  if (!(p->T_min_GeV > 0) || !(p->T_max_GeV > 2 * p->T_min_GeV) || !std::isfinite(p->T_max_GeV))
    return "need 0 < T_min and T_max > 2 T_min";
  if (p->operator_form != LB_OPS_WEAK && p->operator_form != LB_OPS_STRONG) return "unknown operator_form";
  if (p->force_form != LB_FORCE_FEQ && p->force_form != LB_FORCE_WEAK3D) return "unknown force_form";
  if (p->particle_number != LB_N_FREE && p->particle_number != LB_N_CONSERVED) return "unknown particle_number";
  if (p->particle_number == LB_N_CONSERVED && p->eos_kind != LB_EOS_CONST_MASS)
    return "particle_number LB_N_CONSERVED needs eos_kind LB_EOS_CONST_MASS";
  if (!std::isfinite(p->mu_over_T0) || std::fabs(p->mu_over_T0) > 20.0)
    return "mu_over_T0 must be finite and within +-20";
  if (p->mu_over_T0 != 0.0 && p->particle_number != LB_N_CONSERVED)
    return "mu_over_T0 needs particle_number LB_N_CONSERVED";
  if (p->gradient_form != LB_GRAD_CENTRED && p->gradient_form != LB_GRAD_UPWIND) return "unknown gradient_form";
  if (p->gradient_form == LB_GRAD_UPWIND && p->force_form != LB_FORCE_FEQ)
    return "gradient_form LB_GRAD_UPWIND needs force_form LB_FORCE_FEQ";
  return "";
}

Layout layout(const lb_params* p) {
  Layout L;
  const size_t sites = (size_t)p->nx * p->ny;
  const size_t nodes = (size_t)p->n_xi * p->n_theta * 2 * p->n_phi;
  const size_t elt = p->precision == LB_FP64 ? 8 : 4;
  size_t off = 0;
  for (int i = 0; i < 3; ++i) {
    L.F[i] = off;
    off = align_up(off + nodes * sites * elt);
  }
  for (int i = 0; i < 3; ++i) {
    L.lnM[i] = off;
    off = align_up(off + sites * 8);
  }
  for (int i = 0; i < 3; ++i) {
    L.sc[i] = off;
    off = align_up(off + site_scalar_bytes(sites, elt));
  }
  L.cst = off;
  off = align_up(off + std::max(sizeof(StageConst<double>), sizeof(GenConst)));
  L.tbd = off;
  off = align_up(off + sizeof(EosTable));
  L.pts = off;
  off = align_up(off + (size_t)kTablePoints * kFields * 8);
  L.inv_ek = off;
  off = align_up(off + (size_t)kInvPoints * 8);
  L.inv_ee = off;
  off = align_up(off + (size_t)kInvPoints * 8);
  L.gpts = off;
  off = align_up(off + (size_t)kGPoints * kGFields * 8);
  L.err = off;
  off = align_up(off + 256);
  L.lc32 = off;  // FP32 lattice constants of the adjoint's FP32 kernels
  off = align_up(off + sizeof(LatticeConst<float, 5, 5>));
  // the weak-form 3-D force: FP64 stage constants and the dense operators
  // [2][N][N] of the FP64 adjoint
  L.cst64 = L.g3 = 0;
  if (p->force_form == LB_FORCE_WEAK3D) {
    const size_t nodes = (size_t)p->n_xi * p->n_theta * 2 * p->n_phi;
    L.cst64 = off;
    off = align_up(off + sizeof(StageConst<double>));
    L.g3 = off;
    off = align_up(off + 2 * nodes * nodes * sizeof(double));
  }
  L.total = off;
  return L;
}

template <typename R>
void fill_const(const HostLattice& L, LatticeConst<R, 5, 5>* C) {
  const int nxi = 5, nth = 5;
  for (int k = 0; k < nxi; ++k) {
    C->x[k] = (R)L.x[k];
    C->inv_x[k] = (R)(1.0 / L.x[k]);
    C->sh2[k] = (R)(L.x[k] * L.x[k] - 1.0);
  }
  for (int j = 0; j < nth; ++j) C->mu2[j] = (R)(L.mu[j] * L.mu[j]);
  for (int k = 0; k < nxi; ++k)
    for (int j = 0; j < nth; ++j) {
      const int q = k * nth + j;
      const double sh = std::sqrt(L.x[k] * L.x[k] - 1.0);
      const double sth = std::sqrt(1.0 - L.mu[j] * L.mu[j]);
      const double sig = sh * sth, vY = sh * L.mu[j];
      const double w = std::exp(L.z0 * L.x[k]) * L.wxi[k] * L.wth[j] / (4.0 * L.nphi);
      C->sig[q] = (R)sig;
      C->sigi[q] = (R)(sig / L.x[k]);
      C->sig2[q] = (R)(sig * sig);
      C->vY[q] = (R)vY;
      C->w[q] = (R)w;
      C->wx2[q] = (R)(w * L.x[k] * L.x[k]);
      C->wxs[q] = (R)(w * L.x[k] * sig);
      C->ws2[q] = (R)(w * sig * sig);
      C->wvY2[q] = (R)(w * vY * vY);
      C->wx[q] = (R)(w * L.x[k]);
    }
  for (int i = 0; i < nxi * nxi; ++i) {
    C->A1[i] = (R)L.A1[i];
    C->A2[i] = (R)L.A2[i];
  }
  for (int i = 0; i < nth * nth; ++i) C->Ath[i] = (R)L.Ath[i];
  for (int l = 0; l < 8; ++l) {
    C->cosl[l] = (R)L.cosl[l];
    C->sinl[l] = (R)L.sinl[l];
  }
}

// Constants of the generic-lattice kernels (lb_generic.hip).
void fill_gen_const(const HostLattice& L, GenConst* C) {
  *C = GenConst{};
  const int nxi = L.nxi, nth = L.nth, nl = 2 * L.nphi;
  for (int k = 0; k < nxi; ++k) {
    C->x[k] = L.x[k];
    C->sh2[k] = L.x[k] * L.x[k] - 1.0;
  }
  for (int j = 0; j < nth; ++j) C->mu2[j] = L.mu[j] * L.mu[j];
  for (int k = 0; k < nxi; ++k)
    for (int j = 0; j < nth; ++j) {
      const int q = k * nth + j;
      const double sh = std::sqrt(L.x[k] * L.x[k] - 1.0), sth = std::sqrt(1.0 - L.mu[j] * L.mu[j]);
      const double sig = sh * sth, vY = sh * L.mu[j];
      const double w = std::exp(L.z0 * L.x[k]) * L.wxi[k] * L.wth[j] / (4.0 * L.nphi);
      C->w[q] = w;
      C->sig[q] = sig;
      C->sigi[q] = sig / L.x[k];
      C->sig2[q] = sig * sig;
      C->wx2[q] = w * L.x[k] * L.x[k];
      C->wxs[q] = w * L.x[k] * sig;
      C->ws2[q] = w * sig * sig;
      C->wvY2[q] = w * vY * vY;
      C->wx[q] = w * L.x[k];
      C->wsig[q] = w * sig;
    }
  for (int i = 0; i < nxi * nxi; ++i) {
    C->A1[i] = L.A1[i];
    C->A2[i] = L.A2[i];
  }
  for (int i = 0; i < nth * nth; ++i) C->Ath[i] = L.Ath[i];
  for (int l = 0; l < nl; ++l) {
    C->cosl[l] = L.cosl[l];
    C->sinl[l] = L.sinl[l];
  }
}

// Derivative matrix of polynomial interpolation through the nodes z:
// D[a][b] = l_b'(z_a), l_b the Lagrange polynomial of node b.
void lagrange_derivative(const std::vector<double>& z, double* D) {
  const int n = (int)z.size();
  std::vector<double> c(n, 1.0);
  for (int a = 0; a < n; ++a)
    for (int m = 0; m < n; ++m)
      if (m != a) c[a] *= z[a] - z[m];
  for (int a = 0; a < n; ++a) {
    double diag = 0.0;
    for (int b = 0; b < n; ++b) {
      if (b == a) continue;
      D[a * n + b] = (c[a] / c[b]) / (z[a] - z[b]);
      diag += 1.0 / (z[a] - z[b]);
    }
    D[a * n + a] = diag;
  }
}

// Constants of the weak-form 3-D force.  The weak operator is minus the
// w-weighted transpose of the strong-form derivatives on the test space,
//   sum_i g_i G_i F = -(1/w) [Ds^T (g_r sin(theta) x w F) + Dmu^T (-g_r mu sin(theta) w F / (s x))
//                             + Dphi^T (g_t w F / (s sin(theta) x)) + 2 g_r s sin(theta) w F / x],
// g_r = g_x cos phi + g_y sin phi, g_t = g_y cos phi - g_x sin phi, with
// Ds, Dmu, Dphi the partial derivatives (s, mu, phi) of the interpolant in
// the test space; per Fourier mode m of phi these are a radial matrix on
// s^e P(x) (e = parity of m + the mu-parity), the polar matrix on
// (1 - mu^2)^{m/2} P(mu) and a cos/sin swap times m.
template <typename R>
void fill_force_const(const HostLattice& L, StageConst<R>* S) {
  const int nxi = 5, nth = 5;
  double Dx[25], Dm[25];
  lagrange_derivative(L.x, Dx);
  lagrange_derivative(L.mu, Dm);
  for (int a = 0; a < 5; ++a)
    for (int b = 0; b < 5; ++b) {
      S->fDxT[a * 5 + b] = (R)Dx[b * 5 + a];
      S->fDmT[a * 5 + b] = (R)Dm[b * 5 + a];
    }
  for (int k = 0; k < nxi; ++k) {
    const double x = L.x[k], sh = std::sqrt(x * x - 1.0);
    S->frho0[k] = (R)(sh / x);
    S->frho1[k] = (R)(sh * sh / x);
    S->fsig1[k] = (R)(1.0 / sh);
    for (int j = 0; j < nth; ++j) {
      const int q = k * nth + j;
      const double mu = L.mu[j], st = std::sqrt(1.0 - mu * mu);
      const double w = std::exp(L.z0 * x) * L.wxi[k] * L.wth[j] / (4.0 * L.nphi);
      S->fw[q] = (R)w;
      S->finvw[q] = (R)(1.0 / w);
      S->fa[q] = (R)(st * x);
      S->fb[q] = (R)(-mu * st / (sh * x));
      S->fc[q] = (R)(1.0 / (sh * st * x));
      S->fy[q] = (R)(2.0 * sh * st / x);
    }
  }
  for (int pr = 0; pr < 2; ++pr) S->fst[pr] = (R)std::sqrt(1.0 - L.mu[pr] * L.mu[pr]);
  for (int j = 0; j < nth; ++j) S->fmr[j] = (R)(L.mu[j] / (1.0 - L.mu[j] * L.mu[j]));
  // cos and sin of multiples of pi/4, exact where they are 0 or +-1
  const double h = std::sqrt(0.5);
  const double c8[8] = {1, h, 0, -h, -1, -h, 0, h}, s8[8] = {0, h, 1, h, 0, -h, -1, -h};
  const int mode[8] = {0, 4, 1, 1, 2, 2, 3, 3};
  const bool sine[8] = {false, false, false, true, false, true, false, true};
  for (int l = 0; l < 8; ++l)
    for (int r = 0; r < 8; ++r) {
      const int i = (mode[r] * l) % 8;
      S->fphi[l * 8 + r] = (R)(sine[r] ? s8[i] : c8[i]);
    }
}

// Stage constants (mirror-pair form, see StageConst) with S1 unscaled.
template <typename R>
void fill_stage_const(const HostLattice& L, StageConst<R>* S) {
  const int nxi = 5, nth = 5;
  for (int k = 0; k < nxi; ++k) {
    S->x[k] = (R)L.x[k];
    S->inv_x[k] = (R)(1.0 / L.x[k]);
    S->sh2[k] = (R)(L.x[k] * L.x[k] - 1.0);
  }
  for (int pr = 0; pr < 2; ++pr) S->mu2[pr] = (R)(L.mu[pr] * L.mu[pr]);
  for (int k = 0; k < nxi; ++k)
    for (int pr = 0; pr < 3; ++pr) {
      const int i = k * 3 + pr;
      const double sh = std::sqrt(L.x[k] * L.x[k] - 1.0);
      const double sig = sh * std::sqrt(1.0 - L.mu[pr] * L.mu[pr]);
      const double w = std::exp(L.z0 * L.x[k]) * L.wxi[k] * L.wth[pr] / (4.0 * L.nphi);
      S->sig[i] = (R)sig;
      S->sigi[i] = (R)(sig / L.x[k]);
      S->sig2[i] = (R)(sig * sig);
      S->w[i] = (R)w;
      S->wx2[i] = (R)(w * L.x[k] * L.x[k]);
      S->wxs[i] = (R)(w * L.x[k] * sig);
      S->ws2[i] = (R)(w * sig * sig);
    }
  for (int i = 0; i < nxi * nxi; ++i) {
    S->A1[i] = (R)L.A1[i];
    S->A2[i] = (R)L.A2[i];
  }
  // -Ath split by the mirror j -> 4 - j (Ath is mirror symmetric):
  // (Ath f)_j +- (Ath f)_{4-j} = sum_j' Ath_{jj'} (f_j' +- f_{4-j'}).
  const auto A = [&](int j, int jp) { return L.Ath[j * nth + jp]; };
  for (int pr = 0; pr < 2; ++pr) {
    S->Ev[pr][0] = (R)(-0.5 * (A(pr, 0) + A(pr, 4)));
    S->Ev[pr][1] = (R)(-0.5 * (A(pr, 1) + A(pr, 3)));
    S->Ev[pr][2] = (R)(-A(pr, 2));
    S->Od[pr][0] = (R)(-0.5 * (A(pr, 0) - A(pr, 4)));
    S->Od[pr][1] = (R)(-0.5 * (A(pr, 1) - A(pr, 3)));
  }
  S->Mid[0] = (R)(-A(2, 0));
  S->Mid[1] = (R)(-A(2, 1));
  S->Mid[2] = (R)(-A(2, 2));
  for (int l = 0; l < 8; ++l) {
    S->cosl[l] = (R)L.cosl[l];
    S->sinl[l] = (R)L.sinl[l];
  }
  fill_force_const(L, S);
}

// The stage constants of a context: as built for the Milne metric (the
// kernel supplies the 1/tau of S1), with the S1 parts zero for Minkowski.
template <typename R>
StageConst<R> metric_stage_const(const StageConst<R>& base, int metric) {
  StageConst<R> S = base;
  if (metric == LB_METRIC_MILNE) return S;
  for (int i = 0; i < 25; ++i) S.A1[i] = 0;
  for (int pr = 0; pr < 2; ++pr) {
    for (int i = 0; i < 3; ++i) S.Ev[pr][i] = 0;
    for (int i = 0; i < 2; ++i) S.Od[pr][i] = 0;
  }
  for (int i = 0; i < 3; ++i) S.Mid[i] = 0;
  return S;
}

StageArgs stage_args(const lb_ctx* c, double tau, double dtau);

// Site scalars of the current state (after lb_init / lb_set_state).
hipError_t prime_site_scalars(lb_ctx* c) {
  if (c->generic) return hipSuccess;  // the generic kernels match at the start of each stage
  const StageArgs a = stage_args(c, c->tau, 0.0);
  const int cur = c->cur;
  return launch_site(c->p.precision, c->F[cur], c->lnM[cur], c->sc[cur], c->cst, c->tbd, a, c->err, c->stream);
}

// Time of a stage; tau_s = tau multiplies the S1-free terms of a Milne stage.
void set_tau(StageArgs* a, const lb_ctx* c, double tau) {
  a->tau = tau;
  a->tau_s = c->p.metric == LB_METRIC_MILNE ? tau : 1.0;
  a->inv_tau_s = 1.0 / a->tau_s;
}

StageArgs params_args(const lb_params& p, double tau, double dtau) {
  StageArgs a;
  a.nx = p.nx;
  a.ny = p.ny;
  a.n_sites = p.nx * p.ny;
  a.metric = p.metric;
  a.force_form = p.force_form;
  a.mu_mode = p.particle_number == LB_N_CONSERVED ? 1 : 0;
  a.alpha0 = p.mu_over_T0;
  a.grad_form = p.gradient_form;
  a.inv2dx = 0.5 / p.dx_fm;
  a.inv_dx = 1.0 / p.dx_fm;
  a.dtau = dtau;
  a.tau = tau;
  a.tau_s = p.metric == LB_METRIC_MILNE ? tau : 1.0;
  a.inv_tau_s = 1.0 / a.tau_s;
  a.inv_eta_hbarc = std::isinf(p.eta_over_s) ? 0.0 : 1.0 / (p.eta_over_s * kHbarC);
  a.Z = p.Z;
  a.log2Z = std::log2(p.Z);
  return a;
}

StageArgs stage_args(const lb_ctx* c, double tau, double dtau) { return params_args(c->p, tau, dtau); }

const void* lat_const(const lb_ctx* c) {
  return c->p.precision == LB_FP64 ? (const void*)&c->cd : (const void*)&c->cf;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(LB_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Adjoint workspace: the predictor state, the adjoint of the predictor
// state, R0_bar, the ln M gradient adjoint and the per-site eta/s adjoint.
struct AdjLayout {
  size_t Fp, Lp, aF1, aL1, Rb, gb, eta, total;
};
AdjLayout adj_layout(const lb_params& p) {
  const size_t ns = (size_t)p.nx * (size_t)p.ny;
  const size_t nF = ns * (size_t)p.n_xi * (size_t)p.n_theta * 2 * (size_t)p.n_phi * sizeof(double);
  AdjLayout L;
  size_t off = 0;
  L.Fp = off;
  off = align_up(off + nF);
  L.Lp = off;
  off = align_up(off + ns * sizeof(double));
  L.aF1 = off;
  off = align_up(off + nF);
  L.aL1 = off;
  off = align_up(off + ns * sizeof(double));
  L.Rb = off;
  off = align_up(off + nF);
  L.gb = off;  // the ln M gradient's adjoint: per site, or per phi slice with the upwind gradient
  off = align_up(off + 2 * ns * sizeof(double) * (p.gradient_form == LB_GRAD_UPWIND ? (size_t)(2 * p.n_phi) : 1));
  L.eta = off;
  off = align_up(off + ns * sizeof(double));
  L.total = off;
  return L;
}
struct AdjBufs {
  double *Fp, *Lp, *aF1, *aL1, *Rb, *gb, *eta;
};
int adj_check(lb_ctx* c, double tau, double dtau, void* ws, size_t bytes, AdjBufs* B) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  if (c->generic) return fail(LB_E_NOTIMPL, "the adjoint step has the 5 x 5 x 8 momentum lattice only");
  if (!(dtau > 0) || !std::isfinite(dtau)) return fail(LB_E_ARG, "dtau must be finite and > 0");
  if (!std::isfinite(tau) || (c->p.metric == LB_METRIC_MILNE && !(tau > 0)))
    return fail(LB_E_ARG, "tau must be finite (and > 0 for the Milne metric)");
  const double cfl = c->lat.vsum_max * dtau / c->p.dx_fm;
  if (cfl > 0.5)
    return fail(LB_E_ARG, "CFL number " + std::to_string(cfl) + " > 0.5 (reduce dtau or increase dx)");
  const AdjLayout L = adj_layout(c->p);
  if (!ws || ((uintptr_t)ws % kAlign) != 0 || bytes < L.total)
    return fail(LB_E_ARG, "adjoint workspace NULL, not 256-byte aligned or smaller than lb_adjoint_workspace_bytes");
  char* w = (char*)ws;
  B->Fp = (double*)(w + L.Fp);
  B->Lp = (double*)(w + L.Lp);
  B->aF1 = (double*)(w + L.aF1);
  B->aL1 = (double*)(w + L.aL1);
  B->Rb = (double*)(w + L.Rb);
  B->gb = (double*)(w + L.gb);
  B->eta = (double*)(w + L.eta);
  return LB_OK;
}

int read_err_word(int* d_err, hipStream_t stream) {
  int h = 0;
  hipError_t e = hipMemcpyAsync(&h, d_err, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(error word)");
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (h & kErrNonfinite) return fail(LB_E_NONFINITE, "device: non-finite value in the state or input");
  if (h & kErrMatch) return fail(LB_E_MATCH, "device: Landau matching found no timelike eigenvector");
  if (h & kErrEos) return fail(LB_E_EOS, "device: temperature or energy density outside the EoS table");
  return LB_OK;
}

int read_err(lb_ctx* c) { return read_err_word(c->err, c->stream); }

}  // namespace

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

size_t lb_workspace_bytes(const lb_params* p) {
  std::string m = validate(p);
  if (!m.empty()) {
    fail(LB_E_ARG, m);
    return 0;
  }
  return layout(p).total;
}

int lb_init(lb_ctx** out, const lb_params* p, void* d_workspace, size_t ws_bytes, const double* d_e0,
            const double* d_ux0, const double* d_uy0, void* hip_stream) {
  g_err.clear();
  if (!out) return fail(LB_E_ARG, "out is NULL");
  *out = nullptr;
  std::string m = validate(p);
  if (!m.empty()) return fail(LB_E_ARG, m);
  if (!d_workspace) return fail(LB_E_ARG, "workspace is NULL");
  if ((uintptr_t)d_workspace % kAlign) return fail(LB_E_ARG, "workspace must be 256-byte aligned");
  if (!d_e0) return fail(LB_E_ARG, "e0 is NULL");
  Layout L = layout(p);
  if (ws_bytes < L.total)
    return fail(LB_E_ARG, "workspace too small: need " + std::to_string(L.total) + " bytes");

  lb_ctx* c = new lb_ctx();
  c->p = *p;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)d_workspace;
  c->ws_bytes = ws_bytes;
  m = build_lattice(*p, &c->lat);
  if (!m.empty()) {
    delete c;
    return fail(LB_E_ARG, m);
  }
  HostTables T;
  m = build_tables(*p, &T);
  if (!m.empty()) {
    delete c;
    return fail(LB_E_EOS, m);
  }
  fill_const(c->lat, &c->cf);
  fill_const(c->lat, &c->cd);
  for (int i = 0; i < 3; ++i) {
    c->F[i] = c->ws + L.F[i];
    c->lnM[i] = (double*)(c->ws + L.lnM[i]);
    c->sc[i] = (double*)(c->ws + L.sc[i]);
  }
  c->cst = c->ws + L.cst;
  c->tbd = (EosTable*)(c->ws + L.tbd);
  double* d_pts = (double*)(c->ws + L.pts);
  double* d_iek = (double*)(c->ws + L.inv_ek);
  double* d_iee = (double*)(c->ws + L.inv_ee);
  double* d_gpts = (double*)(c->ws + L.gpts);
  c->err = (int*)(c->ws + L.err);
  c->tb = T.desc;
  c->tb.pts = d_pts;
  c->tb.inv_ek = d_iek;
  c->tb.inv_ee = d_iee;
  c->tb.gpts = d_gpts;
  hipError_t e;
  if ((e = hipGetDevice(&c->device)) != hipSuccess) { delete c; return hip_fail(e, "hipGetDevice"); }
  // synchronous copies: the host staging buffers die with this call
  if ((e = hipMemcpy(d_pts, T.pts.data(), T.pts.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_iek, T.inv_ek.data(), T.inv_ek.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_iee, T.inv_ee.data(), T.inv_ee.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(d_gpts, T.gpts.data(), T.gpts.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->tbd, &c->tb, sizeof(EosTable), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemsetAsync(c->err, 0, sizeof(int), c->stream)) != hipSuccess) {
    delete c;
    return hip_fail(e, "upload of EoS tables");
  }
  c->generic = !(p->n_xi == 5 && p->n_theta == 5 && p->n_phi == 4);
  if (c->generic) {
    GenConst gc;
    fill_gen_const(c->lat, &gc);
    if ((e = hipMemcpy(c->cst, &gc, sizeof(gc), hipMemcpyHostToDevice)) != hipSuccess) {
      delete c;
      return hip_fail(e, "upload of lattice constants");
    }
  } else {
    c->lc32 = c->ws + L.lc32;
    if ((e = hipMemcpy(c->lc32, &c->cf, sizeof(c->cf), hipMemcpyHostToDevice)) != hipSuccess) {
      delete c;
      return hip_fail(e, "upload of lattice constants");
    }
    StageConst<float> sf;
    StageConst<double> sd;
    if (p->precision == LB_FP32_FP64MATCH) {
      fill_stage_const(c->lat, &sf);
      sf = metric_stage_const(sf, p->metric);
      e = hipMemcpy(c->cst, &sf, sizeof(sf), hipMemcpyHostToDevice);
    } else {
      fill_stage_const(c->lat, &sd);
      sd = metric_stage_const(sd, p->metric);
      e = hipMemcpy(c->cst, &sd, sizeof(sd), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "upload of stage constants");
    }
    if (p->force_form == LB_FORCE_WEAK3D) {
      // the dense operators that the FP64 adjoint applies, from the same
      // device code as the stage kernels (FP64 constants for either precision)
      fill_stage_const(c->lat, &sd);
      c->g3 = (double*)(c->ws + L.g3);
      e = hipMemcpy(c->ws + L.cst64, &sd, sizeof(sd), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = launch_force_columns(c->ws + L.cst64, c->g3, c->stream);
      if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "dense force operators");
      }
    }
  }
  c->tau = p->tau0_fm;
  c->cur = 0;
  StageArgs a = stage_args(c, c->tau, 0.0);
  if (c->generic) {
    e = launch_gen_init(p->n_xi, p->n_theta, 2 * p->n_phi, d_e0, d_ux0, d_uy0, (double*)c->F[0], c->lnM[0],
                        (const GenConst*)c->cst, c->tbd, a, c->err, c->stream);
  } else {
    e = launch_init(p->precision, d_e0, d_ux0, d_uy0, c->F[0], c->lnM[0], lat_const(c), c->tb, a, c->err,
                    c->stream);
  }
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "init kernel launch");
  }
  if ((e = prime_site_scalars(c)) != hipSuccess) {
    delete c;
    return hip_fail(e, "site kernel launch");
  }
  int rc = read_err(c);
  if (rc != LB_OK) {
    delete c;
    return rc;
  }
  c->initialised = true;
  *out = c;
  return LB_OK;
}

int lb_step(lb_ctx* c, int32_t n_steps, double dtau) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  if (n_steps < 0) return fail(LB_E_ARG, "n_steps must be >= 0");
  if (!(dtau > 0) || !std::isfinite(dtau)) return fail(LB_E_ARG, "dtau must be finite and > 0");
  const double cfl = c->lat.vsum_max * dtau / c->p.dx_fm;
  if (cfl > 0.5)
    return fail(LB_E_ARG, "CFL number " + std::to_string(cfl) + " > 0.5 (reduce dtau or increase dx)");
  const int prec = c->p.precision;
  for (int s = 0; s < n_steps; ++s) {
    const int i0 = c->cur, i1 = (c->cur + 1) % 3, i2 = (c->cur + 2) % 3;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    if (c->prof) {
      while (c->ev.size() < c->ev_used + 3) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return fail(LB_E_HIP, "hipEventCreate");
        c->ev.push_back(ev);
      }
      e0 = c->ev[c->ev_used];
      e1 = c->ev[c->ev_used + 1];
      e2 = c->ev[c->ev_used + 2];
      c->ev_used += 3;
      hipEventRecord(e0, c->stream);
    }
    StageArgs a = stage_args(c, c->tau, dtau);
    hipError_t e;
    if (c->generic) {
      const int nxi = c->p.n_xi, nth = c->p.n_theta, nl = 2 * c->p.n_phi;
      const GenConst* gc = (const GenConst*)c->cst;
      e = launch_gen_stage(nxi, nth, nl, 0, (const double*)c->F[i0], c->lnM[i0], nullptr, nullptr, (double*)c->F[i1],
                           c->lnM[i1], gc, c->tbd, a, c->err, c->stream);
      if (e != hipSuccess) return hip_fail(e, "predictor launch");
      if (c->prof) hipEventRecord(e1, c->stream);
      set_tau(&a, c, c->tau + dtau);
      e = launch_gen_stage(nxi, nth, nl, 1, (const double*)c->F[i1], c->lnM[i1], (const double*)c->F[i0], c->lnM[i0],
                           (double*)c->F[i2], c->lnM[i2], gc, c->tbd, a, c->err, c->stream);
      if (e != hipSuccess) return hip_fail(e, "corrector launch");
      if (c->prof) hipEventRecord(e2, c->stream);
      c->cur = i2;
      c->tau += dtau;
      continue;
    }
    e = launch_stage(prec, 0, c->F[i0], nullptr, c->F[i1], c->lnM[i0], nullptr, c->lnM[i1], c->sc[i0],
                     c->sc[i1], c->cst, c->tbd, a, c->err, c->stream);
    if (e != hipSuccess) return hip_fail(e, "predictor launch");
    if (c->prof) hipEventRecord(e1, c->stream);
    set_tau(&a, c, c->tau + dtau);
    e = launch_stage(prec, 1, c->F[i1], c->F[i0], c->F[i2], c->lnM[i1], c->lnM[i0], c->lnM[i2], c->sc[i1],
                     c->sc[i2], c->cst, c->tbd, a,
                     c->err, c->stream);
    if (e != hipSuccess) return hip_fail(e, "corrector launch");
    if (c->prof) hipEventRecord(e2, c->stream);
    c->cur = i2;
    c->tau += dtau;
  }
  return LB_OK;
}

int lb_moments(lb_ctx* c, double* d_out) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  if (!d_out) return fail(LB_E_ARG, "out is NULL");
  StageArgs a = stage_args(c, c->tau, 0.0);
  hipError_t e = c->generic ? launch_gen_moments(c->p.n_xi, c->p.n_theta, 2 * c->p.n_phi, (const double*)c->F[c->cur],
                                                 c->lnM[c->cur], d_out, (const GenConst*)c->cst, c->tbd, a, c->err,
                                                 c->stream)
                            : launch_moments(c->p.precision, c->F[c->cur], c->lnM[c->cur], d_out, lat_const(c), c->tb,
                                             a, c->err, c->stream);
  if (e != hipSuccess) return hip_fail(e, "moments launch");
  return LB_OK;
}

int lb_get_state(lb_ctx* c, double* d_F, double* d_lnM, double* tau_fm) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  const int n_sites = c->p.nx * c->p.ny, n_q = c->p.n_xi * c->p.n_theta;
  if (d_F) {
    // the generic kernels keep the canonical FP64 layout
    hipError_t e = c->generic ? hipMemcpyAsync(d_F, c->F[c->cur], (size_t)n_sites * n_q * 2 * c->p.n_phi * 8,
                                               hipMemcpyDeviceToDevice, c->stream)
                              : launch_get_state(c->p.precision, c->F[c->cur], d_F, n_q, n_sites, c->stream);
    if (e != hipSuccess) return hip_fail(e, "get_state launch");
  }
  if (d_lnM) {
    hipError_t e = hipMemcpyAsync(d_lnM, c->lnM[c->cur], (size_t)n_sites * 8, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "copy of ln M");
  }
  if (tau_fm) *tau_fm = c->tau;
  return LB_OK;
}

int lb_set_state(lb_ctx* c, const double* d_F, const double* d_lnM, double tau_fm) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  if (!d_F || !d_lnM) return fail(LB_E_ARG, "F and lnM must be given");
  if (!std::isfinite(tau_fm) || (c->p.metric == LB_METRIC_MILNE && !(tau_fm > 0)))
    return fail(LB_E_ARG, "tau must be finite (and > 0 for Milne)");
  const int n_sites = c->p.nx * c->p.ny, n_q = c->p.n_xi * c->p.n_theta;
  hipError_t e = c->generic ? hipMemcpyAsync(c->F[c->cur], d_F, (size_t)n_sites * n_q * 2 * c->p.n_phi * 8,
                                             hipMemcpyDeviceToDevice, c->stream)
                            : launch_set_state(c->p.precision, d_F, c->F[c->cur], n_q, n_sites, c->stream);
  if (e != hipSuccess) return hip_fail(e, "set_state launch");
  e = hipMemcpyAsync(c->lnM[c->cur], d_lnM, (size_t)n_sites * 8, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(e, "copy of ln M");
  c->tau = tau_fm;
  if ((e = prime_site_scalars(c)) != hipSuccess) return hip_fail(e, "site kernel launch");
  return LB_OK;
}

size_t lb_adjoint_workspace_bytes(const lb_params* p) {
  g_err.clear();
  const std::string m = validate(p);
  if (!m.empty()) {
    fail(LB_E_ARG, m);
    return 0;
  }
  return adj_layout(*p).total;
}

int lb_adjoint_forward_step(lb_ctx* c, double tau_fm, double dtau_fm, const double* d_F, const double* d_lnM,
                            double* d_F_out, double* d_lnM_out, void* d_adj_workspace, size_t adj_ws_bytes) {
  AdjBufs B;
  int rc = adj_check(c, tau_fm, dtau_fm, d_adj_workspace, adj_ws_bytes, &B);
  if (rc != LB_OK) return rc;
  if (!d_F || !d_lnM || !d_F_out || !d_lnM_out) return fail(LB_E_ARG, "state pointer is NULL");
  if (d_F_out == d_F || d_lnM_out == d_lnM) return fail(LB_E_ARG, "outputs must not alias the inputs");
  StageArgs a = stage_args(c, tau_fm, dtau_fm);
  hipError_t e =
      launch_adj_stage_fwd(d_F, d_lnM, nullptr, nullptr, B.Fp, B.Lp, 0, &c->cd, c->g3, c->tb, a, c->err, c->stream);
  if (e == hipSuccess) {
    set_tau(&a, c, tau_fm + dtau_fm);
    e = launch_adj_stage_fwd(B.Fp, B.Lp, d_F, d_lnM, d_F_out, d_lnM_out, 1, &c->cd, c->g3, c->tb, a, c->err, c->stream);
  }
  return e == hipSuccess ? LB_OK : hip_fail(e, "adjoint forward step");
}

int lb_adjoint_step(lb_ctx* c, double tau_fm, double dtau_fm, const double* d_F, const double* d_lnM,
                    double* d_adj_F, double* d_adj_lnM, double* d_grad_eta_over_s, void* d_adj_workspace,
                    size_t adj_ws_bytes) {
  g_err.clear();
  AdjBufs B;
  int rc = adj_check(c, tau_fm, dtau_fm, d_adj_workspace, adj_ws_bytes, &B);
  if (rc != LB_OK) return rc;
  if (!d_F || !d_lnM || !d_adj_F || !d_adj_lnM || !d_grad_eta_over_s)
    return fail(LB_E_ARG, "state, adjoint or gradient pointer is NULL");
  const size_t ns = (size_t)c->p.nx * c->p.ny;
  const StageArgs a0 = stage_args(c, tau_fm, dtau_fm);
  StageArgs a1 = a0;
  set_tau(&a1, c, tau_fm + dtau_fm);
  hipStream_t st = c->stream;
  // an FP32 context's reverse sweep runs its node arithmetic in FP32 (with
  // the FP32 lattice constants); with the conserved particle number the
  // FP64 reverse sweep serves both precisions
  const bool fp32 = c->p.precision == LB_FP32_FP64MATCH && c->p.particle_number == LB_N_FREE;
  // predictor state F* = F + dtau K(F)
  hipError_t e =
      launch_adj_stage_fwd(d_F, d_lnM, nullptr, nullptr, B.Fp, B.Lp, 0, &c->cd, c->g3, c->tb, a0, c->err, st,
                           fp32 ? c->lc32 : nullptr);
  // corrector F_new = (F + F*)/2 + dtau/2 K(F*): adjoint of F*, and F's share
  // with the Heun combination in the same pass: aF1 += adj_F/2 (the
  // corrector's share through F*), adj_F <- adj_F/2 + aF1 (F's direct share
  // and the predictor's identity)
  if (e == hipSuccess)
    e = launch_adj_rhs(B.Fp, B.Lp, d_adj_F, d_adj_lnM, 0.5 * dtau_fm, B.aF1, B.aL1, B.Rb, B.gb, B.eta, 0, &c->cd,
                       c->g3, c->tb, a1, c->err, st, fp32 ? c->lc32 : nullptr, d_adj_F, d_adj_lnM);
  // predictor: F* = F + dtau K(F)
  if (e == hipSuccess)
    e = launch_adj_rhs(d_F, d_lnM, B.aF1, B.aL1, dtau_fm, d_adj_F, d_adj_lnM, B.Rb, B.gb, B.eta, 1, &c->cd, c->g3,
                       c->tb, a0, c->err, st, fp32 ? c->lc32 : nullptr);
  if (e == hipSuccess) e = launch_adj_sum(B.eta, (int)ns, d_grad_eta_over_s, st);
  return e == hipSuccess ? LB_OK : hip_fail(e, "adjoint step");
}

int lb_adjoint_init(lb_ctx* c, const double* d_e0, const double* d_ux0, const double* d_uy0,
                    const double* d_adj_F, const double* d_adj_lnM, double* d_grad_e0) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  if (!d_e0 || !d_adj_F || !d_adj_lnM || !d_grad_e0) return fail(LB_E_ARG, "pointer is NULL");
  if ((d_ux0 == nullptr) != (d_uy0 == nullptr)) return fail(LB_E_ARG, "give both ux0 and uy0 or neither");
  if (c->generic) return fail(LB_E_NOTIMPL, "the adjoint of lb_init has the 5 x 5 x 8 momentum lattice only");
  const StageArgs a = stage_args(c, c->p.tau0_fm, 0.0);
  hipError_t e = launch_adj_init(d_e0, d_ux0, d_uy0, d_adj_F, d_adj_lnM, d_grad_e0, &c->cd, c->tb, a, c->err,
                                 c->stream);
  return e == hipSuccess ? LB_OK : hip_fail(e, "adjoint of the initial state");
}

int lb_status(lb_ctx* c) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  return read_err(c);
}

int lb_destroy(lb_ctx* c) {
  if (!c) return LB_OK;
  for (hipEvent_t e : c->ev) hipEventDestroy(e);
  delete c;
  return LB_OK;
}

int lb_profile(lb_ctx* c, int32_t enable) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  if (enable) {
    hipStreamSynchronize(c->stream);
    c->ev_used = 0;
  }
  c->prof = enable != 0;
  c->prof_ms[0] = c->prof_ms[1] = 0;
  c->prof_n[0] = c->prof_n[1] = 0;
  return LB_OK;
}

int lb_profile_read(lb_ctx* c, double* ms_out, int64_t* count_out) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (size_t i = 0; i + 2 < c->ev_used; i += 3) {
    float a = 0, b = 0;
    hipEventElapsedTime(&a, c->ev[i], c->ev[i + 1]);
    hipEventElapsedTime(&b, c->ev[i + 1], c->ev[i + 2]);
    c->prof_ms[0] += a;
    c->prof_ms[1] += b;
    c->prof_n[0] += 1;
    c->prof_n[1] += 1;
  }
  c->ev_used = 0;
  if (ms_out) {
    ms_out[0] = c->prof_ms[0];
    ms_out[1] = c->prof_ms[1];
  }
  if (count_out) {
    count_out[0] = c->prof_n[0];
    count_out[1] = c->prof_n[1];
  }
  return LB_OK;
}

int lb_profile_stage(lb_ctx* c, int32_t stage, int32_t n, double dtau_fm, double* ms_out) {
  if (!c || !c->initialised) return fail(LB_E_STATE, "context not initialised");
  if ((stage != 0 && stage != 1) || n < 1 || !ms_out) return fail(LB_E_ARG, "need stage 0 or 1, n >= 1, ms_out");
  if (c->generic) return fail(LB_E_NOTIMPL, "stage timing has the 5 x 5 x 8 momentum lattice only");
  if (!(dtau_fm > 0) || !std::isfinite(dtau_fm)) return fail(LB_E_ARG, "dtau must be finite and > 0");
  const int prec = c->p.precision;
  const int i0 = c->cur, i1 = (c->cur + 1) % 3, i2 = (c->cur + 2) % 3;
  StageArgs a = stage_args(c, c->tau, dtau_fm);
  // the corrector needs a predictor output to read: one untimed predictor
  hipError_t e = launch_stage(prec, 0, c->F[i0], nullptr, c->F[i1], c->lnM[i0], nullptr, c->lnM[i1], c->sc[i0],
                              c->sc[i1], c->cst, c->tbd, a, c->err, c->stream);
  if (e != hipSuccess) return hip_fail(e, "predictor launch");
  if (stage == 1) set_tau(&a, c, c->tau + dtau_fm);
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (auto& x : ev)
    if ((e = hipEventCreate(&x)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  hipEventRecord(ev[0], c->stream);
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    if (stage == 0)
      e = launch_stage(prec, 0, c->F[i0], nullptr, c->F[i1], c->lnM[i0], nullptr, c->lnM[i1], c->sc[i0], c->sc[i1],
                       c->cst, c->tbd, a, c->err, c->stream);
    else
      e = launch_stage(prec, 1, c->F[i1], c->F[i0], c->F[i2], c->lnM[i1], c->lnM[i0], c->lnM[i2], c->sc[i1],
                       c->sc[i2], c->cst, c->tbd, a, c->err, c->stream);
  }
  hipEventRecord(ev[1], c->stream);
  float ms = 0;
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  hipEventDestroy(ev[0]);
  hipEventDestroy(ev[1]);
  if (e != hipSuccess) return hip_fail(e, "stage timing");
  *ms_out = (double)ms / n;
  return read_err(c);
}

int64_t lb_lattice_info(const lb_params* p, double* out, int64_t n_out) {
  if (!p) return fail(LB_E_ARG, "params is NULL");
  if (p->n_xi < 1 || p->n_theta < 1 || p->n_phi < 1 || !(p->z0 > 0))
    return fail(LB_E_ARG, "need n_xi, n_theta, n_phi >= 1 and z0 > 0");
  const int64_t nxi = p->n_xi, nth = p->n_theta, nph = 2 * p->n_phi;
  const int64_t need = 2 * nxi + 2 * nth + 2 * nph + 2 * nxi * nxi + nth * nth;
  if (!out) return need;
  if (n_out < need) return fail(LB_E_ARG, "output too small");
  HostLattice L;
  std::string m = build_lattice(*p, &L);
  if (!m.empty()) return fail(LB_E_ARG, m);
  double* o = out;
  for (auto* v : {&L.x, &L.wxi, &L.mu, &L.wth, &L.cosl, &L.sinl, &L.A1, &L.A2, &L.Ath})
    for (double d : *v) *o++ = d;
  return need;
}

int64_t lb_node_table(const lb_params* p, double* out, int64_t n_out) {
  if (!p) return fail(LB_E_ARG, "params is NULL");
  if (p->n_xi < 1 || p->n_theta < 1 || p->n_phi < 1 || !(p->z0 > 0))
    return fail(LB_E_ARG, "need n_xi, n_theta, n_phi >= 1 and z0 > 0");
  const int64_t nph = 2 * (int64_t)p->n_phi, N = (int64_t)p->n_xi * p->n_theta * nph;
  const int64_t need = 5 * N;
  if (!out) return need;
  if (n_out < need) return fail(LB_E_ARG, "output too small");
  HostLattice L;
  std::string m = build_lattice(*p, &L);
  if (!m.empty()) return fail(LB_E_ARG, m);
  // Sec. IV.C: the product rule over (xi, theta, phi) with the radial
  // weight's exp(-z0 cosh xi) divided out, normalised so that the angular
  // weights sum to one (4 n_phi = 2 x the number of azimuths)
  for (int k = 0; k < p->n_xi; ++k) {
    const double x = L.x[k], sh = std::sqrt(std::max(x * x - 1.0, 0.0));
    for (int j = 0; j < p->n_theta; ++j) {
      const double st = std::sqrt(std::max(1.0 - L.mu[j] * L.mu[j], 0.0));
      for (int l = 0; l < nph; ++l) {
        const int64_t n = ((int64_t)k * p->n_theta + j) * nph + l;
        out[n] = std::exp(p->z0 * x) * L.wxi[k] * L.wth[j] / (2.0 * (double)nph);
        out[N + n] = x;
        out[2 * N + n] = sh * st * L.cosl[l];
        out[3 * N + n] = sh * st * L.sinl[l];
        out[4 * N + n] = sh * L.mu[j];
      }
    }
  }
  return need;
}

double lb_degeneracy(double kappa, double g) {
  // Stefan-Boltzmann limit of the Boltzmann gas: p = Z T^4/pi^2 against
  // g pi^2 T^4/90, times the factor kappa
  return kappa * g * kPi * kPi * kPi * kPi / 90.0;
}

int lb_eos_eval(const lb_params* p, int64_t n, const double* T, double* out, int32_t table) {
  std::string m = validate(p);
  if (!m.empty()) return fail(LB_E_ARG, m);
  if (n < 0 || (n > 0 && (!T || !out))) return fail(LB_E_ARG, "bad arrays");
  HostEos eos(*p);
  HostTables tabs;
  if (table) {
    m = build_tables(*p, &tabs);
    if (!m.empty()) return fail(LB_E_EOS, m);
  }
  double zg = 2.0;
  for (int64_t i = 0; i < n; ++i) {
    HostEos::Point pt;
    double zu;
    if (!(T[i] > 0) || !eos.eval(T[i], zg, &pt, &zu)) return fail(LB_E_EOS, "no quasiparticle mass at T");
    zg = zu;
    double tauR = std::isinf(p->eta_over_s) ? INFINITY : p->eta_over_s * kHbarC * pt.q / T[i];
    if (table) {
      double t, w[4], dw[4];
      const double u = std::log(T[i]);
      const int j = eos_locate(tabs.desc, u, &t);
      lagrange4(t, w, dw);
      pt.M = eos_field(tabs.desc, j, w, kZ) * T[i];
      pt.B = eos_field(tabs.desc, j, w, kBt4) * T[i] * T[i] * T[i] * T[i];
      pt.ekin = std::exp(eos_field(tabs.desc, j, w, kLnEk));
      pt.beta = eos_field(tabs.desc, j, w, kBeta);
      const double q = eos_field(tabs.desc, j, w, kQ);
      tauR = std::isinf(p->eta_over_s) ? INFINITY : p->eta_over_s * kHbarC * q / T[i];
    }
    double* o = out + 8 * i;
    o[0] = pt.eps;
    o[1] = pt.p;
    o[2] = pt.s;
    o[3] = pt.M;
    o[4] = pt.B;
    o[5] = pt.ekin;
    o[6] = pt.beta;
    o[7] = tauR;
  }
  return LB_OK;
}

}  // extern "C"

// Internal hooks for the entry point without allocation (lb_noalloc.hip),
// which brings its own device scratch in place of the adjoint workspace.
namespace lbmi {
int set_error(int code, const char* msg) { return fail(code, msg); }
int context_device(const lb_ctx* c) { return c ? c->device : -1; }
size_t context_adjoint_bytes(const lb_ctx* c) { return c && c->initialised ? adj_layout(c->p).total : 0; }
}  // namespace lbmi

// ---------------------------------------------------------------------------
// Batched form: many events advanced together (lb_batch_* in lb.h).

struct lb_batch {
  lb_params p{};                 // shared parameters (grid fields per event)
  std::vector<lb_event> events;
  std::vector<BatchEvent> ev;    // host copy of the device event table
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;     // private stream the graphs are captured on
  char* ws = nullptr;
  HostLattice lat;
  EosTable tb{};                 // with device table pointers
  EosTable* tbd = nullptr;
  void* cst = nullptr;
  LatticeConst<float, 5, 5> cf{};
  LatticeConst<double, 5, 5> cd{};
  int* err = nullptr;
  BatchEvent* d_ev = nullptr;
  int32_t* d_tile_event = nullptr;
  StageTime* d_times = nullptr;  // [2][2 kBatchGraphSteps]
  StageTime* h_times = nullptr;  // pinned host staging of the same
  hipEvent_t copied[2] = {nullptr, nullptr};
  double vsum_over_dx = 0;       // max over events of max_n (|v^x|+|v^y|)/gamma / dx
  double tau = 0;
  int cur = 0;
  int variant = -1, n_tiles = 0;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int graph_variant = -1;
  double graph_dtau = 0;
  int slot = 0;
};

namespace {

constexpr int kBatchGraphSteps = 48;  // steps per captured graph (a multiple of 3)

struct BatchLayout {
  size_t cst, tbd, pts, inv_ek, inv_ee, gpts, err, ev, tile_event, times, total;
  std::vector<size_t> F, lnM, sc;  // [event * 3 + i]
};

lb_params event_params(const lb_params& p, const lb_event& e) {
  lb_params q = p;
  q.nx = e.nx;
  q.ny = e.ny;
  q.dx_fm = e.dx_fm;
  q.eta_over_s = e.eta_over_s;
  return q;
}

std::string validate_batch(const lb_params* p, const lb_event* ev, int32_t n) {
  if (!p) return "params is NULL";
  if (!ev || n < 1) return "need at least one event";
  if (!(p->n_xi == 5 && p->n_theta == 5 && p->n_phi == 4)) return "the batched form has the 5 x 5 x 8 momentum lattice only";
  int64_t tiles = 0;
  for (int i = 0; i < n; ++i) {
    const lb_params q = event_params(*p, ev[i]);
    std::string m = validate(&q);
    if (!m.empty()) return "event " + std::to_string(i) + ": " + m;
    tiles += batch_tiles(ev[i].nx, ev[i].ny, kBatchTileRows[0]);
  }
  if (tiles >= ((int64_t)1 << 30)) return "too many tiles in the batch";
  return "";
}

BatchLayout batch_layout(const lb_params* p, const lb_event* ev, int32_t n) {
  BatchLayout L;
  const size_t elt = p->precision == LB_FP64 ? 8 : 4;
  const size_t nodes = (size_t)p->n_xi * p->n_theta * 2 * p->n_phi;
  size_t off = 0;
  L.cst = off;
  off = align_up(off + sizeof(StageConst<double>));
  L.tbd = off;
  off = align_up(off + sizeof(EosTable));
  L.pts = off;
  off = align_up(off + (size_t)kTablePoints * kFields * 8);
  L.inv_ek = off;
  off = align_up(off + (size_t)kInvPoints * 8);
  L.inv_ee = off;
  off = align_up(off + (size_t)kInvPoints * 8);
  L.gpts = off;
  off = align_up(off + (size_t)kGPoints * kGFields * 8);
  L.err = off;
  off = align_up(off + 256);
  L.ev = off;
  off = align_up(off + (size_t)n * sizeof(BatchEvent));
  size_t max_tiles = 0;
  for (int r = 0; r < 3; ++r) {
    size_t t = 0;
    for (int i = 0; i < n; ++i) t += (size_t)batch_tiles(ev[i].nx, ev[i].ny, kBatchTileRows[r]);
    max_tiles = std::max(max_tiles, t);
  }
  L.tile_event = off;
  off = align_up(off + max_tiles * 4);
  L.times = off;
  off = align_up(off + 2 * 2 * kBatchGraphSteps * sizeof(StageTime));
  L.F.resize(3 * n);
  L.lnM.resize(3 * n);
  L.sc.resize(3 * n);
  for (int i = 0; i < n; ++i) {
    const size_t sites = (size_t)ev[i].nx * ev[i].ny;
    for (int k = 0; k < 3; ++k) {
      L.F[3 * i + k] = off;
      off = align_up(off + nodes * sites * elt);
      L.lnM[3 * i + k] = off;
      off = align_up(off + sites * 8);
      L.sc[3 * i + k] = off;
      off = align_up(off + site_scalar_bytes(sites, elt));
    }
  }
  L.total = off;
  return L;
}

// Tile numbering of a kernel variant: event tile offsets and the map from
// tile to event, uploaded to the device.
hipError_t set_variant(lb_batch* b, int variant) {
  const int rows = batch_tile_rows(variant);
  std::vector<int32_t> te;
  int t0 = 0;
  for (size_t i = 0; i < b->ev.size(); ++i) {
    b->ev[i].tile0 = t0;
    const int nt = batch_tiles(b->ev[i].nx, b->ev[i].ny, rows);
    te.insert(te.end(), (size_t)nt, (int32_t)i);
    t0 += nt;
  }
  hipError_t e = hipMemcpyAsync(b->d_ev, b->ev.data(), b->ev.size() * sizeof(BatchEvent), hipMemcpyHostToDevice,
                                b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_tile_event, te.data(), te.size() * 4, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // te is a local staging vector
  if (e == hipSuccess) {
    b->variant = variant;
    b->n_tiles = t0;
  }
  return e;
}

StageArgs batch_shared_args(const lb_batch* b, double dtau) {
  StageArgs a = params_args(b->p, b->tau, dtau);  // grid / time fields are set per block
  return a;
}

StageTime stage_time(const lb_params& p, double tau) {
  StageTime t;
  t.tau = tau;
  t.tau_s = p.metric == LB_METRIC_MILNE ? tau : 1.0;
  t.inv_tau_s = 1.0 / t.tau_s;
  return t;
}

// One Heun step of every event with the kernel arguments of the stage times
// given directly (pred at b->tau, corr at b->tau + dtau).
hipError_t batch_step_direct(lb_batch* b, double dtau) {
  const int i0 = b->cur, i1 = (b->cur + 1) % 3, i2 = (b->cur + 2) % 3;
  const StageArgs a = batch_shared_args(b, dtau);
  hipError_t e = launch_batch_stage(b->p.precision, 0, b->variant, b->d_ev, b->d_tile_event, b->n_tiles,
                                    stage_time(b->p, b->tau), nullptr, 0, i0, i0, i1, b->cst, b->tbd, a, b->err,
                                    b->stream);
  if (e != hipSuccess) return e;
  e = launch_batch_stage(b->p.precision, 1, b->variant, b->d_ev, b->d_tile_event, b->n_tiles,
                         stage_time(b->p, b->tau + dtau), nullptr, 0, i1, i0, i2, b->cst, b->tbd, a, b->err,
                         b->stream);
  if (e != hipSuccess) return e;
  b->cur = i2;
  b->tau += dtau;
  return hipSuccess;
}

// Destroys the captured graphs.  A replay of them may still run on the
// caller's stream, so the stream is drained first.
void drop_graphs(lb_batch* b) {
  bool any = false;
  for (auto g : b->graph) any = any || g != nullptr;
  if (any) hipStreamSynchronize(b->stream);
  for (auto& g : b->graph)
    if (g) {
      hipGraphExecDestroy(g);
      g = nullptr;
    }
  b->graph_variant = -1;
}

// Capture kBatchGraphSteps steps starting from buffer rotation 0, reading
// the stage times from slot `slot` of the device time table.
hipError_t capture_graph(lb_batch* b, int slot, double dtau) {
  // captured on the batch's own stream (the caller's may be the legacy
  // default stream, which cannot be captured); launched on the caller's
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const StageArgs a = batch_shared_args(b, dtau);
  const StageTime* times = b->d_times + (size_t)slot * 2 * kBatchGraphSteps;
  int cur = 0;
  hipError_t le = hipSuccess;
  for (int k = 0; k < kBatchGraphSteps && le == hipSuccess; ++k) {
    const int i0 = cur, i1 = (cur + 1) % 3, i2 = (cur + 2) % 3;
    le = launch_batch_stage(b->p.precision, 0, b->variant, b->d_ev, b->d_tile_event, b->n_tiles, StageTime{}, times,
                            2 * k, i0, i0, i1, b->cst, b->tbd, a, b->err, b->cap);
    if (le == hipSuccess)
      le = launch_batch_stage(b->p.precision, 1, b->variant, b->d_ev, b->d_tile_event, b->n_tiles, StageTime{},
                              times, 2 * k + 1, i1, i0, i2, b->cst, b->tbd, a, b->err, b->cap);
    cur = i2;
  }
  e = hipStreamEndCapture(b->cap, &g);
  if (le != hipSuccess) e = le;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->graph[slot], g, nullptr, nullptr, 0);
  if (g) hipGraphDestroy(g);
  return e;
}

// kBatchGraphSteps steps (rotation 0 to 0) as one graph launch.
hipError_t batch_graph_steps(lb_batch* b, double dtau) {
  hipError_t e = hipSuccess;
  if (b->graph_variant != b->variant || b->graph_dtau != dtau) {
    drop_graphs(b);
    for (int sl = 0; sl < 2 && e == hipSuccess; ++sl) e = capture_graph(b, sl, dtau);
    if (e != hipSuccess) {
      drop_graphs(b);
      return e;
    }
    b->graph_variant = b->variant;
    b->graph_dtau = dtau;
  }
  const int sl = b->slot;
  // the pinned staging of this slot is free once its previous copy is done
  if ((e = hipEventSynchronize(b->copied[sl])) != hipSuccess) return e;
  StageTime* h = b->h_times + (size_t)sl * 2 * kBatchGraphSteps;
  double tau = b->tau;
  for (int k = 0; k < kBatchGraphSteps; ++k) {  // the times lb_step would use
    h[2 * k] = stage_time(b->p, tau);
    h[2 * k + 1] = stage_time(b->p, tau + dtau);
    tau += dtau;
  }
  e = hipMemcpyAsync(b->d_times + (size_t)sl * 2 * kBatchGraphSteps, h, 2 * kBatchGraphSteps * sizeof(StageTime),
                     hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->copied[sl], b->stream);
  if (e == hipSuccess) e = hipGraphLaunch(b->graph[sl], b->stream);
  if (e != hipSuccess) return e;
  b->tau = tau;
  b->slot ^= 1;
  return hipSuccess;
}

// Mean milliseconds of one predictor + corrector pair of variant v over n
// pairs, on the spare buffers (the state is unchanged).
hipError_t time_variant(lb_batch* b, int v, double dtau, int n, float* ms) {
  hipError_t e = set_variant(b, v);
  if (e != hipSuccess) return e;
  const int i0 = b->cur, i1 = (b->cur + 1) % 3, i2 = (b->cur + 2) % 3;
  const StageArgs a = batch_shared_args(b, dtau);
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (auto& x : ev)
    if ((e = hipEventCreate(&x)) != hipSuccess) return e;
  for (int k = -1; k < n && e == hipSuccess; ++k) {  // k = -1: untimed warm-up
    if (k == 0) hipEventRecord(ev[0], b->stream);
    e = launch_batch_stage(b->p.precision, 0, v, b->d_ev, b->d_tile_event, b->n_tiles, stage_time(b->p, b->tau),
                           nullptr, 0, i0, i0, i1, b->cst, b->tbd, a, b->err, b->stream);
    if (e == hipSuccess)
      e = launch_batch_stage(b->p.precision, 1, v, b->d_ev, b->d_tile_event, b->n_tiles,
                             stage_time(b->p, b->tau + dtau), nullptr, 0, i1, i0, i2, b->cst, b->tbd, a, b->err,
                             b->stream);
  }
  hipEventRecord(ev[1], b->stream);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, ev[0], ev[1]);
  if (e == hipSuccess) *ms /= n;
  hipEventDestroy(ev[0]);
  hipEventDestroy(ev[1]);
  return e;
}

int batch_tune(lb_batch* b, double dtau, int32_t* variant_out, double* ms_out) {
  const int nv = batch_variants(b->p.precision, b->p.force_form, b->p.particle_number, b->p.gradient_form);
  int best = -1;
  float best_ms = 0;
  for (int v = 0; v < nv; ++v) {
    float ms = 0;
    hipError_t e = time_variant(b, v, dtau, 5, &ms);
    if (e != hipSuccess) return hip_fail(e, "batch tuning");
    if (ms_out) ms_out[v] = ms;
    if (best < 0 || ms < best_ms) {
      best = v;
      best_ms = ms;
    }
  }
  hipError_t e = set_variant(b, best);
  if (e != hipSuccess) return hip_fail(e, "batch tile map");
  if (variant_out) *variant_out = best;
  return read_err_word(b->err, b->stream);
}

}  // namespace

extern "C" {

size_t lb_batch_workspace_bytes(const lb_params* p, const lb_event* events, int32_t n_events) {
  g_err.clear();
  std::string m = validate_batch(p, events, n_events);
  if (!m.empty()) {
    fail(LB_E_ARG, m);
    return 0;
  }
  return batch_layout(p, events, n_events).total;
}

int lb_batch_init(lb_batch** out, const lb_params* p, const lb_event* events, int32_t n_events, void* d_workspace,
                  size_t ws_bytes, const double* const* d_e0, void* hip_stream) {
  g_err.clear();
  if (!out) return fail(LB_E_ARG, "out is NULL");
  *out = nullptr;
  std::string m = validate_batch(p, events, n_events);
  if (!m.empty()) return fail(LB_E_ARG, m);
  if (!d_workspace || (uintptr_t)d_workspace % kAlign) return fail(LB_E_ARG, "workspace NULL or not 256-byte aligned");
  if (!d_e0) return fail(LB_E_ARG, "e0 pointer array is NULL");
  for (int i = 0; i < n_events; ++i)
    if (!d_e0[i]) return fail(LB_E_ARG, "e0 of event " + std::to_string(i) + " is NULL");
  const BatchLayout L = batch_layout(p, events, n_events);
  if (ws_bytes < L.total) return fail(LB_E_ARG, "workspace too small: need " + std::to_string(L.total) + " bytes");

  lb_batch* b = new lb_batch();
  b->p = *p;
  b->events.assign(events, events + n_events);
  b->stream = (hipStream_t)hip_stream;
  b->ws = (char*)d_workspace;
  m = build_lattice(*p, &b->lat);
  if (!m.empty()) {
    delete b;
    return fail(LB_E_ARG, m);
  }
  HostTables T;
  m = build_tables(*p, &T);
  if (!m.empty()) {
    delete b;
    return fail(LB_E_EOS, m);
  }
  fill_const(b->lat, &b->cf);
  fill_const(b->lat, &b->cd);
  b->cst = b->ws + L.cst;
  b->tbd = (EosTable*)(b->ws + L.tbd);
  b->err = (int*)(b->ws + L.err);
  b->d_ev = (BatchEvent*)(b->ws + L.ev);
  b->d_tile_event = (int32_t*)(b->ws + L.tile_event);
  b->d_times = (StageTime*)(b->ws + L.times);
  b->tb = T.desc;
  b->tb.pts = (double*)(b->ws + L.pts);
  b->tb.inv_ek = (double*)(b->ws + L.inv_ek);
  b->tb.inv_ee = (double*)(b->ws + L.inv_ee);
  b->tb.gpts = (double*)(b->ws + L.gpts);
  b->ev.resize(n_events);
  for (int i = 0; i < n_events; ++i) {
    BatchEvent& E = b->ev[i];
    E.nx = events[i].nx;
    E.ny = events[i].ny;
    E.n_sites = events[i].nx * events[i].ny;
    E.tile0 = 0;
    E.inv2dx = 0.5 / events[i].dx_fm;
    E.inv_eta_hbarc = std::isinf(events[i].eta_over_s) ? 0.0 : 1.0 / (events[i].eta_over_s * kHbarC);
    for (int k = 0; k < 3; ++k) {
      E.F[k] = b->ws + L.F[3 * i + k];
      E.lnM[k] = (double*)(b->ws + L.lnM[3 * i + k]);
      E.sc[k] = (double*)(b->ws + L.sc[3 * i + k]);
    }
    b->vsum_over_dx = std::max(b->vsum_over_dx, b->lat.vsum_max / events[i].dx_fm);
  }
  hipError_t e = hipSuccess;
  if ((e = hipHostMalloc((void**)&b->h_times, 2 * 2 * kBatchGraphSteps * sizeof(StageTime))) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->copied[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->copied[1], hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) {
    lb_batch_destroy(b);
    return hip_fail(e, "batch host staging");
  }
  if ((e = hipMemcpy((void*)b->tb.pts, T.pts.data(), T.pts.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy((void*)b->tb.inv_ek, T.inv_ek.data(), T.inv_ek.size() * 8, hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy((void*)b->tb.inv_ee, T.inv_ee.data(), T.inv_ee.size() * 8, hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy((void*)b->tb.gpts, T.gpts.data(), T.gpts.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->tbd, &b->tb, sizeof(EosTable), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemsetAsync(b->err, 0, sizeof(int), b->stream)) != hipSuccess) {
    lb_batch_destroy(b);
    return hip_fail(e, "upload of EoS tables");
  }
  if (p->precision == LB_FP32_FP64MATCH) {
    StageConst<float> sf;
    fill_stage_const(b->lat, &sf);
    sf = metric_stage_const(sf, p->metric);
    e = hipMemcpy(b->cst, &sf, sizeof(sf), hipMemcpyHostToDevice);
  } else {
    StageConst<double> sd;
    fill_stage_const(b->lat, &sd);
    sd = metric_stage_const(sd, p->metric);
    e = hipMemcpy(b->cst, &sd, sizeof(sd), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    lb_batch_destroy(b);
    return hip_fail(e, "upload of stage constants");
  }
  b->tau = p->tau0_fm;
  b->cur = 0;
  const void* lc = p->precision == LB_FP64 ? (const void*)&b->cd : (const void*)&b->cf;
  for (int i = 0; i < n_events && e == hipSuccess; ++i) {
    const StageArgs a = params_args(event_params(*p, events[i]), b->tau, 0.0);
    e = launch_init(p->precision, d_e0[i], nullptr, nullptr, b->ev[i].F[0], b->ev[i].lnM[0], lc, b->tb, a, b->err,
                    b->stream);
    if (e == hipSuccess)
      e = launch_site(p->precision, b->ev[i].F[0], b->ev[i].lnM[0], b->ev[i].sc[0], b->cst, b->tbd, a, b->err,
                      b->stream);
  }
  if (e == hipSuccess) e = set_variant(b, p->precision == LB_FP32_FP64MATCH ? 1 : 1);  // until tuned
  if (e != hipSuccess) {
    lb_batch_destroy(b);
    return hip_fail(e, "batch initial state");
  }
  b->variant = -1;  // not tuned yet (the tile map above is variant 1)
  int rc = read_err_word(b->err, b->stream);
  if (rc != LB_OK) {
    lb_batch_destroy(b);
    return rc;
  }
  *out = b;
  return LB_OK;
}

int lb_batch_tune(lb_batch* b, double dtau_fm, int32_t* variant_out, double* ms_out) {
  if (!b) return fail(LB_E_STATE, "batch not initialised");
  if (!(dtau_fm > 0) || !std::isfinite(dtau_fm)) return fail(LB_E_ARG, "dtau must be finite and > 0");
  return batch_tune(b, dtau_fm, variant_out, ms_out);
}

int lb_batch_set_variant(lb_batch* b, int32_t variant) {
  if (!b) return fail(LB_E_STATE, "batch not initialised");
  if (variant < 0 || variant >= batch_variants(b->p.precision, b->p.force_form, b->p.particle_number, b->p.gradient_form))
    return fail(LB_E_ARG, "no such kernel variant");
  hipError_t e = set_variant(b, variant);
  if (e != hipSuccess) return hip_fail(e, "batch tile map");
  return LB_OK;
}

int lb_batch_step(lb_batch* b, int32_t n_steps, double dtau_fm) {
  if (!b) return fail(LB_E_STATE, "batch not initialised");
  if (n_steps < 0) return fail(LB_E_ARG, "n_steps must be >= 0");
  if (!(dtau_fm > 0) || !std::isfinite(dtau_fm)) return fail(LB_E_ARG, "dtau must be finite and > 0");
  const double cfl = b->vsum_over_dx * dtau_fm;
  if (cfl > 0.5)
    return fail(LB_E_ARG, "CFL number " + std::to_string(cfl) + " > 0.5 in some event (reduce dtau)");
  if (n_steps == 0) return LB_OK;
  if (b->variant < 0) {
    int rc = batch_tune(b, dtau_fm, nullptr, nullptr);
    if (rc != LB_OK) return rc;
  }
  int left = n_steps;
  while (left > 0) {
    hipError_t e;
    if (b->cur == 0 && left >= kBatchGraphSteps) {
      e = batch_graph_steps(b, dtau_fm);
      left -= kBatchGraphSteps;
    } else {
      e = batch_step_direct(b, dtau_fm);
      left -= 1;
    }
    if (e != hipSuccess) return hip_fail(e, "batch step");
  }
  return LB_OK;
}

int lb_batch_moments(lb_batch* b, int32_t event, double* d_out) {
  if (!b) return fail(LB_E_STATE, "batch not initialised");
  if (event < 0 || event >= (int)b->ev.size() || !d_out) return fail(LB_E_ARG, "bad event index or out is NULL");
  const StageArgs a = params_args(event_params(b->p, b->events[event]), b->tau, 0.0);
  const void* lc = b->p.precision == LB_FP64 ? (const void*)&b->cd : (const void*)&b->cf;
  hipError_t e = launch_moments(b->p.precision, b->ev[event].F[b->cur], b->ev[event].lnM[b->cur], d_out, lc, b->tb,
                                a, b->err, b->stream);
  if (e != hipSuccess) return hip_fail(e, "moments launch");
  return LB_OK;
}

int lb_batch_get_state(lb_batch* b, int32_t event, double* d_F, double* d_lnM, double* tau_fm) {
  if (!b) return fail(LB_E_STATE, "batch not initialised");
  if (event < 0 || event >= (int)b->ev.size()) return fail(LB_E_ARG, "bad event index");
  const int n_sites = b->ev[event].n_sites, n_q = b->p.n_xi * b->p.n_theta;
  if (d_F) {
    hipError_t e = launch_get_state(b->p.precision, b->ev[event].F[b->cur], d_F, n_q, n_sites, b->stream);
    if (e != hipSuccess) return hip_fail(e, "get_state launch");
  }
  if (d_lnM) {
    hipError_t e = hipMemcpyAsync(d_lnM, b->ev[event].lnM[b->cur], (size_t)n_sites * 8, hipMemcpyDeviceToDevice,
                                  b->stream);
    if (e != hipSuccess) return hip_fail(e, "copy of ln M");
  }
  if (tau_fm) *tau_fm = b->tau;
  return LB_OK;
}

int lb_batch_status(lb_batch* b) {
  if (!b) return fail(LB_E_STATE, "batch not initialised");
  return read_err_word(b->err, b->stream);
}

int lb_batch_destroy(lb_batch* b) {
  if (!b) return LB_OK;
  if (b->stream) hipStreamSynchronize(b->stream);
  drop_graphs(b);
  for (auto& x : b->copied)
    if (x) hipEventDestroy(x);
  if (b->h_times) hipHostFree(b->h_times);
  if (b->cap) hipStreamDestroy(b->cap);
  delete b;
  return LB_OK;
}

}  // extern "C"
