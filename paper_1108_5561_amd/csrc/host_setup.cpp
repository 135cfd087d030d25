// Host-side setup: momentum lattice (Sec. IV.C), factored weak-form
// operators (Sec. IV.D) and EoS tables (Sec. III.A, IV.A).
#include "host_setup.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

namespace lbmi {

namespace {

using ld = long double;

// ---------------------------------------------------------------------------
// Gauss-Legendre on [-1, 1] (long double), ascending nodes.
void gauss_legendre(int n, std::vector<ld>* xs, std::vector<ld>* ws) {
  xs->assign(n, 0);
  ws->assign(n, 0);
  for (int i = 0; i < n; ++i) {
    ld x = std::cos(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
    ld dp = 1;
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = x;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p0 = 1; p1 = x; }
      dp = n * (p0 - x * p1) / (1 - x * x);
      ld dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-21L) break;
    }
    // recompute derivative at the final node
    ld p0 = 1, p1 = x;
    for (int k = 2; k <= n; ++k) {
      ld p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (p0 - x * p1) / (1 - x * x);
    (*xs)[n - 1 - i] = x;
    (*ws)[n - 1 - i] = 2 / ((1 - x * x) * dp * dp);
  }
}

// Legendre L_m and L_m' at mu.
void legendre(int m, ld mu, ld* L, ld* dL) {
  ld p0 = 1, p1 = mu;
  if (m == 0) { *L = 1; *dL = 0; return; }
  for (int k = 2; k <= m; ++k) {
    ld p2 = ((2 * k - 1) * mu * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *L = p1;
  *dL = m * (p0 - mu * p1) / (1 - mu * mu);
}

// Discretised radial measure: nodes x = cosh xi and weights of
// int dxi exp(-z0 cosh xi) sinh^2 xi (.) by composite Gauss-Legendre in xi.
void radial_discrete_measure(ld z0, std::vector<ld>* xd, std::vector<ld>* wd) {
  const int panels = 96, per = 20;
  std::vector<ld> gx, gw;
  gauss_legendre(per, &gx, &gw);
  ld xi_max = std::acosh(1 + 90 / z0);  // exp(-90) below long-double resolution
  xd->clear();
  wd->clear();
  for (int p = 0; p < panels; ++p) {
    ld a = xi_max * p / panels, b = xi_max * (p + 1) / panels;
    for (int i = 0; i < per; ++i) {
      ld t = 0.5L * (a + b) + 0.5L * (b - a) * gx[i];
      ld sh = std::sinh(t), ch = std::cosh(t);
      xd->push_back(ch);
      wd->push_back(0.5L * (b - a) * gw[i] * sh * sh * std::exp(-z0 * ch));
    }
  }
}

// Monic orthogonal polynomials by the Stieltjes procedure on a discrete
// measure: R_{l+1} = (x - a_l) R_l - b_l R_{l-1}.
void stieltjes(const std::vector<ld>& xd, const std::vector<ld>& wd, int n, std::vector<ld>* a,
               std::vector<ld>* b) {
  size_t m = xd.size();
  std::vector<ld> rm1(m, 0), r0(m, 1), r1(m);
  a->assign(n + 1, 0);
  b->assign(n + 1, 0);
  ld norm_prev = 1;
  for (int l = 0; l <= n; ++l) {
    ld nrm = 0, xn = 0;
    for (size_t i = 0; i < m; ++i) {
      nrm += wd[i] * r0[i] * r0[i];
      xn += wd[i] * xd[i] * r0[i] * r0[i];
    }
    (*a)[l] = xn / nrm;
    (*b)[l] = (l == 0) ? nrm : nrm / norm_prev;  // b_0 = mu_0
    norm_prev = nrm;
    for (size_t i = 0; i < m; ++i) {
      r1[i] = (xd[i] - (*a)[l]) * r0[i] - (l == 0 ? 0 : (*b)[l]) * rm1[i];
    }
    rm1.swap(r0);
    r0.swap(r1);
  }
}

// R_l(x) and R_l'(x), l = 0..n, from the recurrence.
void recur_eval(const std::vector<ld>& a, const std::vector<ld>& b, int n, ld x, std::vector<ld>* R,
                std::vector<ld>* dR) {
  R->assign(n + 1, 0);
  dR->assign(n + 1, 0);
  (*R)[0] = 1;
  (*dR)[0] = 0;
  if (n >= 1) {
    (*R)[1] = x - a[0];
    (*dR)[1] = 1;
  }
  for (int l = 1; l < n; ++l) {
    (*R)[l + 1] = (x - a[l]) * (*R)[l] - b[l] * (*R)[l - 1];
    (*dR)[l + 1] = (*R)[l] + (x - a[l]) * (*dR)[l] - b[l] * (*dR)[l - 1];
  }
}

// Number of roots of R_n below x: with q_0 = x - a_0 and
// q_l = (x - a_l) - b_l / q_{l-1} (the ratios R_{l+1}(x)/R_l(x)), the count
// of positive q_l is the number of eigenvalues of the Jacobi matrix below x.
int sturm_count(const std::vector<ld>& a, const std::vector<ld>& b, int n, ld x) {
  int cnt = 0;
  ld q = x - a[0];
  if (q > 0) ++cnt;
  for (int l = 1; l < n; ++l) {
    if (q == 0) q = 1e-300L;
    q = (x - a[l]) - b[l] / q;
    if (q > 0) ++cnt;
  }
  return cnt;
}

}  // namespace

// ---------------------------------------------------------------------------
std::string build_lattice(const lb_params& p, HostLattice* L) {
  const int nxi = p.n_xi, nth = p.n_theta, nphi = p.n_phi;
  if (nxi < 1 || nth < 1 || nphi < 1) return "n_xi, n_theta, n_phi must be >= 1";
  if (!(p.z0 > 0) || !std::isfinite(p.z0)) return "z0 must be finite and > 0";
  L->nxi = nxi;
  L->nth = nth;
  L->nphi = nphi;
  L->z0 = p.z0;
  const ld z0 = p.z0;

  // radial rule: Stieltjes on the discretised measure, roots by Sturm
  // bisection + Newton, Christoffel weights
  std::vector<ld> xd, wd, a, b;
  radial_discrete_measure(z0, &xd, &wd);
  stieltjes(xd, wd, nxi, &a, &b);
  ld hi = 0;
  for (int l = 0; l < nxi; ++l) hi = std::max(hi, a[l] + 2 * std::sqrt(b[l + 1]) + 2 * std::sqrt(l ? b[l] : 0));
  std::vector<ld> xk(nxi), wk(nxi), R, dR;
  for (int k = 0; k < nxi; ++k) {
    ld lo = 1, up = hi + 1;
    for (int it = 0; it < 200; ++it) {
      ld mid = 0.5L * (lo + up);
      if (sturm_count(a, b, nxi, mid) > k) up = mid; else lo = mid;
      if (up - lo < 1e-18L * up) break;
    }
    ld x = 0.5L * (lo + up);
    for (int it = 0; it < 3; ++it) {
      recur_eval(a, b, nxi, x, &R, &dR);
      if (dR[nxi] != 0) x -= R[nxi] / dR[nxi];
    }
    xk[k] = x;
  }
  // norms I(l) = mu_0 b_1 ... b_l
  std::vector<ld> I(nxi);
  I[0] = b[0];
  for (int l = 1; l < nxi; ++l) I[l] = I[l - 1] * b[l];
  for (int k = 0; k < nxi; ++k) {
    recur_eval(a, b, nxi, xk[k], &R, &dR);
    ld s = 0;
    for (int l = 0; l < nxi; ++l) s += R[l] * R[l] / I[l];
    wk[k] = 1 / s;
  }
  // the paper's I(l) = sum_k w_k R_l(x_k)^2 (equal to the norm up to rounding)
  std::vector<std::vector<ld>> Rk(nxi), dRk(nxi);
  for (int k = 0; k < nxi; ++k) recur_eval(a, b, nxi, xk[k], &Rk[k], &dRk[k]);
  for (int l = 0; l < nxi; ++l) {
    ld s = 0;
    for (int k = 0; k < nxi; ++k) s += wk[k] * Rk[k][l] * Rk[k][l];
    I[l] = s;
  }

  std::vector<ld> mu, wth;
  gauss_legendre(nth, &mu, &wth);

  L->x.resize(nxi);
  L->wxi.resize(nxi);
  for (int k = 0; k < nxi; ++k) {
    L->x[k] = (double)xk[k];
    L->wxi[k] = (double)wk[k];
  }
  L->mu.resize(nth);
  L->wth.resize(nth);
  for (int j = 0; j < nth; ++j) {
    L->mu[j] = (double)mu[j];
    L->wth[j] = (double)wth[j];
  }
  L->cosl.resize(2 * nphi);
  L->sinl.resize(2 * nphi);
  for (int l = 0; l < 2 * nphi; ++l) {
    if ((2 * l) % nphi == 0) {
      int q = ((2 * l) / nphi) % 4;
      const double cc[4] = {1, 0, -1, 0}, ss[4] = {0, 1, 0, -1};
      L->cosl[l] = cc[q];
      L->sinl[l] = ss[q];
    } else {
      ld ph = 3.14159265358979323846264338327950288L * l / nphi;
      L->cosl[l] = (double)std::cos(ph);
      L->sinl[l] = (double)std::sin(ph);
    }
  }

  // Factored weak-form operators.  On one phi slice with F_{kj}:
  //   S2[F]_{kj} = sum_k' A2_{kk'} F_{k'j}
  //   S1[F]_{kj} = mu_j^2 sum_k' A1_{kk'} F_{k'j} - sum_j' Ath_{jj'} F_{kj'}
  // with (exact discrete orthogonality of the Gauss rules used for the
  // polar sum over m and, in the second S1 term, the radial sum over l)
  //   A2_{kk'}  = -e^{-z0 x_k} sum_l R_l(x_k) b2_l(x_k') e^{z0 x_k'} w_k' / I(l)
  //   A1_{kk'}  = -e^{-z0 x_k} sum_l R_l(x_k) a1_l(x_k') e^{z0 x_k'} w_k' / I(l)
  //   Ath_{jj'} = sum_m (2m+1)/2 L_m(mu_j) lam_m(mu_j') w^theta_j'
  //   b2_l = R_l (2 + 1/x^2) + R_l' x t^2,  a1_l = (R_l' x - R_l) t^2,
  //   lam_m = L_m + L_m' (mu - mu^3),       t^2 = (x^2 - 1)/x^2.
  L->A1.assign(nxi * nxi, 0);
  L->A2.assign(nxi * nxi, 0);
  for (int k = 0; k < nxi; ++k) {
    for (int kp = 0; kp < nxi; ++kp) {
      ld x = xk[kp];
      ld t2 = (x * x - 1) / (x * x);
      ld s1 = 0, s2 = 0;
      for (int l = 0; l < nxi; ++l) {
        ld Rl = Rk[kp][l], dRl = dRk[kp][l];
        ld b2 = Rl * (2 + 1 / (x * x)) + dRl * x * t2;
        ld a1 = (dRl * x - Rl) * t2;
        s1 += Rk[k][l] * a1 / I[l];
        s2 += Rk[k][l] * b2 / I[l];
      }
      ld f = -std::exp(z0 * (xk[kp] - xk[k])) * wk[kp];
      L->A1[k * nxi + kp] = (double)(f * s1);
      L->A2[k * nxi + kp] = (double)(f * s2);
    }
  }
  L->Ath.assign(nth * nth, 0);
  for (int j = 0; j < nth; ++j) {
    for (int jp = 0; jp < nth; ++jp) {
      ld s = 0;
      for (int m = 0; m < nth; ++m) {
        ld Lj, dLj, Lp, dLp;
        legendre(m, mu[j], &Lj, &dLj);
        legendre(m, mu[jp], &Lp, &dLp);
        ld lam = Lp + dLp * (mu[jp] - mu[jp] * mu[jp] * mu[jp]);
        s += (2 * m + 1) * 0.5L * Lj * lam * wth[jp];
      }
      L->Ath[j * nth + jp] = (double)s;
    }
  }

  if (p.operator_form == LB_OPS_STRONG) {
    // Strong form: differentiate the interpolant exp(-z0 x) P(x, mu) through
    // the nodes.  With D the barycentric derivative matrix of the Lagrange
    // interpolant on a node set,
    //   S2 = p . d/dp = ((x^2 - 1)/x) d/dx:
    //     A2_{kk'} = ((x_k^2 - 1)/x_k) e^{-z0 x_k} (Dx_{kk'} - z0 delta_{kk'}) e^{z0 x_k'},
    //   S1 = p^Y d/dp^Y = mu^2 (x^2 - 1)/x d/dx + mu (1 - mu^2) d/dmu:
    //     A1 = A2,  Ath_{jj'} = -mu_j (1 - mu_j^2) Dmu_{jj'}.
    auto deriv_matrix = [](const std::vector<ld>& y) {
      const int n = (int)y.size();
      std::vector<ld> c(n, 1), D(n * n, 0);
      for (int i = 0; i < n; ++i)
        for (int m = 0; m < n; ++m)
          if (m != i) c[i] *= (y[i] - y[m]);
      for (int i = 0; i < n; ++i) {
        ld diag = 0;
        for (int j = 0; j < n; ++j) {
          if (j == i) continue;
          D[i * n + j] = (c[i] / c[j]) / (y[i] - y[j]);
          diag += 1 / (y[i] - y[j]);
        }
        D[i * n + i] = diag;
      }
      return D;
    };
    const std::vector<ld> Dx = deriv_matrix(xk), Dm = deriv_matrix(mu);
    for (int k = 0; k < nxi; ++k)
      for (int kp = 0; kp < nxi; ++kp) {
        const ld x = xk[k];
        const ld v = (x * x - 1) / x * std::exp(z0 * (xk[kp] - x)) * (Dx[k * nxi + kp] - (k == kp ? z0 : 0));
        L->A2[k * nxi + kp] = (double)v;
        L->A1[k * nxi + kp] = (double)v;
      }
    for (int j = 0; j < nth; ++j)
      for (int jp = 0; jp < nth; ++jp)
        L->Ath[j * nth + jp] = (double)(-mu[j] * (1 - mu[j] * mu[j]) * Dm[j * nth + jp]);
  }

  // streaming CFL factor
  double vm = 0;
  for (int k = 0; k < nxi; ++k)
    for (int j = 0; j < nth; ++j)
      for (int l = 0; l < 2 * nphi; ++l) {
        double sig = std::sqrt(std::max(0.0, L->x[k] * L->x[k] - 1.0)) * std::sqrt(std::max(0.0, 1 - L->mu[j] * L->mu[j]));
        vm = std::max(vm, sig * (std::fabs(L->cosl[l]) + std::fabs(L->sinl[l])) / L->x[k]);
      }
  L->vsum_max = vm;
  return "";
}

// ---------------------------------------------------------------------------
HostEos::HostEos(const lb_params& p)
    : kind_(p.eos_kind), Z_(p.Z), g_(p.eos_g), Tc_(p.eos_Tc_GeV), w_(p.eos_width_GeV),
      m0_(p.eos_mass_GeV), taur_rule_(p.taur_rule) {
  c_ = kPi * kPi / 90.0 * g_;
  if (kind_ != LB_EOS_TABLE) return;
  // cubic spline of y = ln(s/T^3) on x = ln T with not-a-knot ends (the
  // third derivative is continuous at the second and the second-to-last
  // points): second derivatives sigma from the tridiagonal system that
  // remains after the two end conditions are eliminated
  const int n = p.eos_n;
  tx_.resize(n);
  ty_.resize(n);
  td_.assign(n, 0.0);
  tp_.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    const double T = p.eos_T_GeV[i];
    tx_[i] = std::log(T);
    ty_[i] = std::log(p.eos_s_GeV3[i] / (T * T * T));
  }
  std::vector<double> h(n - 1), dl(n - 1);
  for (int k = 0; k + 1 < n; ++k) {
    h[k] = tx_[k + 1] - tx_[k];
    dl[k] = (ty_[k + 1] - ty_[k]) / h[k];
  }
  // rows i = 1 .. n-2: h_{i-1} s_{i-1} + 2 (h_{i-1} + h_i) s_i + h_i s_{i+1} = 6 (dl_i - dl_{i-1})
  const int m = n - 2;
  std::vector<double> a(m, 0.0), b(m, 0.0), c(m, 0.0), r(m, 0.0);
  for (int i = 1; i <= m; ++i) {
    a[i - 1] = h[i - 1];
    b[i - 1] = 2 * (h[i - 1] + h[i]);
    c[i - 1] = h[i];
    r[i - 1] = 6 * (dl[i] - dl[i - 1]);
  }
  // left: s_0 = ((h0 + h1) s_1 - h0 s_2) / h1; right likewise
  {
    const double h0 = h[0], h1 = h[1];
    b[0] += a[0] * (h0 + h1) / h1;
    c[0] -= a[0] * h0 / h1;
    a[0] = 0;
    const double hA = h[n - 2], hB = h[n - 3];  // last and second-to-last intervals
    b[m - 1] += c[m - 1] * (hA + hB) / hB;
    a[m - 1] -= c[m - 1] * hA / hB;
    c[m - 1] = 0;
  }
  for (int i = 1; i < m; ++i) {  // forward elimination (diagonally dominant)
    const double f = a[i] / b[i - 1];
    b[i] -= f * c[i - 1];
    r[i] -= f * r[i - 1];
  }
  std::vector<double> sg(n, 0.0);
  sg[m] = r[m - 1] / b[m - 1];
  for (int i = m - 2; i >= 0; --i) sg[i + 1] = (r[i] - c[i] * sg[i + 2]) / b[i];
  sg[0] = ((h[0] + h[1]) * sg[1] - h[0] * sg[2]) / h[1];
  sg[n - 1] = ((h[n - 2] + h[n - 3]) * sg[n - 2] - h[n - 2] * sg[n - 3]) / h[n - 3];
  td_ = sg;
  tp_[0] = p.eos_p0_GeV4;
  for (int k = 0; k + 1 < n; ++k) tp_[k + 1] = tp_[k] + tab_s_integral(k, std::exp(tx_[k + 1]));
}

int HostEos::tab_interval(double x) const {
  const int n = (int)tx_.size();
  int k = (int)(std::upper_bound(tx_.begin(), tx_.end(), x) - tx_.begin()) - 1;
  return std::max(0, std::min(n - 2, k));  // the end cubics extend outside
}

double HostEos::tab_y(double x, double* dy) const {
  const int k = tab_interval(x);
  const double h = tx_[k + 1] - tx_[k], t = x - tx_[k];
  const double s0 = td_[k], s1 = td_[k + 1];
  const double bb = (ty_[k + 1] - ty_[k]) / h - h * (2 * s0 + s1) / 6, cc = 0.5 * s0, dd = (s1 - s0) / (6 * h);
  if (dy) *dy = bb + t * (2 * cc + 3 * dd * t);
  return ty_[k] + t * (bb + t * (cc + dd * t));
}

// int_{T_k}^{T} s dT' = int exp(4 x + y(x)) dx over [x_k, ln T], 16-point
// Gauss-Legendre (the integrand is smooth on one interpolation interval)
double HostEos::tab_s_integral(int k, double T) const {
  static std::vector<ld> gx, gw;
  static std::once_flag once;
  std::call_once(once, [] { gauss_legendre(16, &gx, &gw); });
  const double a = tx_[k], b = std::log(T);
  double sum = 0;
  for (int i = 0; i < 16; ++i) {
    const double x = 0.5 * (a + b) + 0.5 * (b - a) * (double)gx[i];
    sum += (double)gw[i] * std::exp(4 * x + tab_y(x, nullptr));
  }
  return 0.5 * (b - a) * sum;
}

double HostEos::p(double T) const {
  if (kind_ == LB_EOS_TABLE) {
    const int k = tab_interval(std::log(T));
    return tp_[k] + tab_s_integral(k, T);
  }
  if (kind_ == LB_EOS_CONST_MASS) {
    double z = m0_ / T;
    return Z_ * m0_ * m0_ * T * T * std::cyl_bessel_k(2.0, z) / (2 * kPi * kPi);
  }
  if (kind_ == LB_EOS_TANH_S) {
    // p = int_0^T s dT' with s = 4 c T'^3 h(T'): 16-point Gauss-Legendre on
    // panels no wider than w/2 up to b = Tc + 30 w; above b, h = 1 to far
    // below double precision and the rest is 4 c (T^4 - b^4)/4.
    static std::vector<ld> gx, gw;
    static std::once_flag once;
    std::call_once(once, [] { gauss_legendre(16, &gx, &gw); });
    const double b = Tc_ + 30 * w_;
    const double top = std::min(T, b);
    const int panels = std::max(8, (int)std::ceil(top / (0.5 * w_)));
    double sum = 0;
    for (int k = 0; k < panels; ++k) {
      const double a0 = top * k / panels, a1 = top * (k + 1) / panels;
      double ps = 0;
      for (int i = 0; i < 16; ++i) {
        const double t = 0.5 * (a0 + a1) + 0.5 * (a1 - a0) * (double)gx[i];
        ps += (double)gw[i] * t * t * t * 0.5 * (1 + std::tanh((t - Tc_) / w_));
      }
      sum += 0.5 * (a1 - a0) * ps;
    }
    if (T > b) sum += 0.25 * (T * T * T * T - b * b * b * b);
    return 4 * c_ * sum;
  }
  double h0 = 0.5 * (1 + std::tanh((T - Tc_) / w_));
  return c_ * T * T * T * T * h0;
}

double HostEos::s(double T) const {
  if (kind_ == LB_EOS_TABLE) return T * T * T * std::exp(tab_y(std::log(T), nullptr));
  if (kind_ == LB_EOS_CONST_MASS) {
    double z = m0_ / T;
    return Z_ * m0_ * m0_ * m0_ * std::cyl_bessel_k(3.0, z) / (2 * kPi * kPi);
  }
  double th = std::tanh((T - Tc_) / w_);
  double h0 = 0.5 * (1 + th), h1 = 0.5 * (1 - th * th) / w_;
  if (kind_ == LB_EOS_TANH_S) return 4 * c_ * T * T * T * h0;
  return c_ * (4 * T * T * T * h0 + T * T * T * T * h1);
}

double HostEos::ds(double T) const {
  if (kind_ == LB_EOS_TABLE) {
    double dy;
    const double y = tab_y(std::log(T), &dy);
    return T * T * std::exp(y) * (3 + dy);  // d/dT [T^3 e^y] with dy/dx, x = ln T
  }
  if (kind_ == LB_EOS_CONST_MASS) {
    double z = m0_ / T;
    // d/dT K_3(m/T) = K_3'(z)(-m/T^2), K_3' = -K_2 - 3 K_3/z
    double k3p = -std::cyl_bessel_k(2.0, z) - 3 * std::cyl_bessel_k(3.0, z) / z;
    return -Z_ * m0_ * m0_ * m0_ * k3p * m0_ / (2 * kPi * kPi * T * T);
  }
  double th = std::tanh((T - Tc_) / w_);
  double sech2 = 1 - th * th;
  double h0 = 0.5 * (1 + th), h1 = 0.5 * sech2 / w_, h2 = -sech2 * th / (w_ * w_);
  if (kind_ == LB_EOS_TANH_S) return 4 * c_ * (3 * T * T * h0 + T * T * T * h1);
  return c_ * (12 * T * T * h0 + 8 * T * T * T * h1 + T * T * T * T * h2);
}

bool HostEos::z_of_T(double T, double z_guess, double* zout) const {
  if (kind_ == LB_EOS_CONST_MASS) {
    *zout = m0_ / T;
    return true;
  }
  // z^3 K_3(z) = c, decreasing from 8 (z -> 0) to 0
  double c = 2 * kPi * kPi * s(T) / (Z_ * T * T * T);
  if (!(c > 0) || !(c < 8)) return false;
  auto f = [&](double z) { return std::log(z * z * z * std::cyl_bessel_k(3.0, z)) - std::log(c); };
  double lo = 1e-6, hi = 200.0;
  double z = (z_guess > lo && z_guess < hi) ? z_guess : 2.0;
  // Newton on ln(z^3 K_3) with derivative -K_2/K_3, safeguarded by bisection
  for (int it = 0; it < 200; ++it) {
    double fz = f(z);
    if (fz > 0) lo = z; else hi = z;
    double k2 = std::cyl_bessel_k(2.0, z), k3 = std::cyl_bessel_k(3.0, z);
    double zn = z + fz * k3 / k2;
    if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
    if (std::fabs(zn - z) <= 2e-16 * z) { z = zn; break; }
    z = zn;
  }
  *zout = z;
  return std::isfinite(z);
}

namespace {
// int_0^inf sinh^6 xi / cosh xi exp(-z cosh xi) dxi, composite Gauss-Legendre
double h_integral(double z) {
  static std::vector<ld> gx, gw;
  static std::once_flag once;
  std::call_once(once, [] { gauss_legendre(16, &gx, &gw); });
  const int panels = 64;
  double xi_max = std::acosh(1 + 130 / z);
  double sum = 0;
  for (int p = 0; p < panels; ++p) {
    double a = xi_max * p / panels, b = xi_max * (p + 1) / panels;
    double ps = 0;
    for (int i = 0; i < 16; ++i) {
      double t = 0.5 * (a + b) + 0.5 * (b - a) * (double)gx[i];
      double sh = std::sinh(t), ch = std::cosh(t);
      double sh2 = sh * sh;
      ps += (double)gw[i] * sh2 * sh2 * sh2 / ch * std::exp(-z * ch);
    }
    sum += 0.5 * (b - a) * ps;
  }
  return sum;
}
}  // namespace

bool HostEos::eval(double T, double z_guess, Point* o, double* z_used) const {
  double z;
  if (!z_of_T(T, z_guess, &z)) return false;
  const double M = z * T;
  const double k1 = std::cyl_bessel_k(1.0, z), k2 = std::cyl_bessel_k(2.0, z), k3 = std::cyl_bessel_k(3.0, z);
  const double tp2 = 2 * kPi * kPi;
  o->p = p(T);
  o->s = s(T);
  o->eps = T * o->s - o->p;
  o->M = M;
  double pkin = Z_ * M * M * T * T * k2 / tp2;
  o->ekin = Z_ * M * M * T * T * (3 * k2 + z * k1) / tp2;
  if (kind_ == LB_EOS_CONST_MASS) {
    o->B = 0;
    o->beta = 0;
  } else {
    o->B = pkin - o->p;
    double dsT = ds(T);
    // M' from d/dT [Z M^3 K_3(M/T)/(2 pi^2)] = s'(T)
    double dM = z + 3 * k3 / k2 - tp2 * dsT * T / (Z_ * M * M * M * k2);
    double dB = -Z_ * M * M * T * k1 * dM / tp2;
    o->beta = dB / (T * dsT - dB);
  }
  o->n0 = pkin / T;  // n = Z M^2 T K_2/(2 pi^2) of eq. (epsp) at mu = 0
  if (taur_rule_ == LB_TAUR_MASSLESS) {
    o->q = 5.0;
    o->qn = 0.0;
  } else {
    // h = eta/tau_R = Z M^5/(30 pi^2 T) int sinh^6/cosh exp(-z cosh)
    double h = Z_ * std::pow(M, 5) / (30 * kPi * kPi * T) * h_integral(z);
    o->q = T * o->s / h;
    o->qn = T * o->n0 / h;
  }
  *z_used = z;
  return true;
}

// ---------------------------------------------------------------------------
namespace {
struct TableKey {
  int kind, rule;
  double Z, g, Tc, w, m0, tmin, tmax;
  bool operator==(const TableKey& o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
};
std::mutex g_cache_mu;
TableKey g_cache_key;
bool g_cache_valid = false;
HostTables g_cache;
}  // namespace

std::string build_tables(const lb_params& p, HostTables* out) {
  TableKey key;
  std::memset(&key, 0, sizeof(key));
  key.kind = p.eos_kind;
  key.rule = p.taur_rule;
  key.Z = p.Z;
  key.g = p.eos_g;
  key.Tc = p.eos_Tc_GeV;
  key.w = p.eos_width_GeV;
  key.m0 = p.eos_mass_GeV;
  key.tmin = p.T_min_GeV;
  key.tmax = p.T_max_GeV;
  const bool cacheable = p.eos_kind != LB_EOS_TABLE;  // a caller's table is not keyed
  if (cacheable) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (g_cache_valid && g_cache_key == key) {
      *out = g_cache;
      return "";
    }
  }
  HostEos eos(p);
  const int n = kTablePoints, ninv = kInvPoints;
  const double ulo = std::log(p.T_min_GeV), uhi = std::log(p.T_max_GeV);
  const int pad = 3;
  const double h = (uhi - ulo) / (n - 1 - 2 * pad);
  const double u0 = ulo - pad * h;
  HostTables T;
  T.pts.assign((size_t)n * kFields, 0.0);
  std::vector<char> okv(n, 1);
  std::vector<double> deps(n, 0.0);

  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t) {
    pool.emplace_back([&, t] {
      int i0 = (int)((long long)n * t / nth), i1 = (int)((long long)n * (t + 1) / nth);
      double zg = 2.0;
      for (int i = i0; i < i1; ++i) {
        double Tt = std::exp(u0 + i * h);
        HostEos::Point pt;
        double zu;
        if (!eos.eval(Tt, zg, &pt, &zu) || !(pt.ekin > 0) || !(pt.eps > 0)) {
          okv[i] = 0;
          continue;
        }
        zg = zu;
        double* d = &T.pts[(size_t)i * kFields];
        d[kLnEk] = std::log(pt.ekin);
        d[kLnEeos] = std::log(pt.eps);
        d[kZ] = zu;
        d[kBeta] = pt.beta;
        d[kQ] = pt.q;
        d[kBt4] = pt.B / (Tt * Tt * Tt * Tt);
        d[kLnN] = std::log(pt.n0);
        d[kNq] = pt.qn;
        deps[i] = Tt * eos.ds(Tt);
      }
    });
  }
  for (auto& th : pool) th.join();
  for (int i = 0; i < n; ++i) {
    double Tt = std::exp(u0 + i * h);
    if (!okv[i]) return "EoS: no quasiparticle mass M(T) at T = " + std::to_string(Tt) + " GeV (raise Z)";
    if (!(deps[i] > 0))
      return "EoS thermodynamically unstable: d eps/dT <= 0 at T = " + std::to_string(Tt) + " GeV";
    if (i > 0 && !(T.pts[(size_t)i * kFields + kLnEk] > T.pts[(size_t)(i - 1) * kFields + kLnEk]))
      return "EoS: eps - B not increasing at T = " + std::to_string(Tt) + " GeV";
    if (i > 0 && !(T.pts[(size_t)i * kFields + kLnEeos] > T.pts[(size_t)(i - 1) * kFields + kLnEeos]))
      return "EoS: eps not increasing at T = " + std::to_string(Tt) + " GeV";
  }

  // inverse tables on the accepted range [ulo, uhi]
  EosTable& D = T.desc;
  D.n = n;
  D.n_inv = ninv;
  D.u0 = u0;
  D.h = h;
  D.inv_h = 1.0 / h;
  D.u_lo = ulo;
  D.u_hi = uhi;
  D.pts = T.pts.data();
  auto fwd = [&](int field, double u) {
    double t, w[4], dw[4];
    int i = eos_locate(D, u, &t);
    lagrange4(t, w, dw);
    return eos_field(D, i, w, field);
  };
  auto build_inv = [&](int field, std::vector<double>* inv, double* g0, double* gh) {
    double ga = fwd(field, ulo), gb = fwd(field, uhi);
    *g0 = ga;
    *gh = (gb - ga) / (ninv - 1);
    inv->assign(ninv, 0.0);
    for (int j = 0; j < ninv; ++j) {
      double g = ga + j * (*gh);
      double lo = ulo - 2 * h, hi = uhi + 2 * h;
      for (int it = 0; it < 80; ++it) {
        double mid = 0.5 * (lo + hi);
        if (fwd(field, mid) < g) lo = mid; else hi = mid;
      }
      (*inv)[j] = 0.5 * (lo + hi);
    }
  };
  build_inv(kLnEk, &T.inv_ek, &D.gk0, &D.gk_h);
  build_inv(kLnEeos, &T.inv_ee, &D.ge0, &D.ge_h);
  D.gk_inv_h = 1.0 / D.gk_h;
  D.ge_inv_h = 1.0 / D.ge_h;
  D.inv_ek = T.inv_ek.data();
  D.inv_ee = T.inv_ee.data();
  // the g table: the u-table cubic inverted at each g_i = ln(eps - B) of a
  // uniform grid over the accepted range, and its fields there
  {
    const int gn = kGPoints;
    const double ga = D.gk0, gb = D.gk0 + (ninv - 1) * D.gk_h;
    D.gn = gn;
    D.gpad_ = 0;
    D.gg0 = ga;
    D.gg_h = (gb - ga) / (gn - 1);
    D.gg_inv_h = 1.0 / D.gg_h;
    T.gpts.assign((size_t)gn * kGFields, 0.0);
    for (int i = 0; i < gn; ++i) {
      const double g = ga + i * D.gg_h;
      double lo = ulo - 2 * h, hi = uhi + 2 * h;
      for (int it = 0; it < 80; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (fwd(kLnEk, mid) < g) lo = mid; else hi = mid;
      }
      const double u = 0.5 * (lo + hi);
      double* d = &T.gpts[(size_t)i * kGFields];
      d[kGT] = std::exp(u);
      d[kGZ] = fwd(kZ, u);
      d[kGBeta] = fwd(kBeta, u);
      d[kGQ] = fwd(kQ, u);
      d[kGBt4] = fwd(kBt4, u);
    }
    D.gpts = T.gpts.data();
  }
  if (cacheable) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache = T;
    g_cache.desc.pts = g_cache.pts.data();
    g_cache.desc.inv_ek = g_cache.inv_ek.data();
    g_cache.desc.inv_ee = g_cache.inv_ee.data();
    g_cache.desc.gpts = g_cache.gpts.data();
    g_cache_key = key;
    g_cache_valid = true;
  }
  *out = T;
  out->desc.pts = out->pts.data();
  out->desc.inv_ek = out->inv_ek.data();
  out->desc.inv_ee = out->inv_ee.data();
  out->desc.gpts = out->gpts.data();
  return "";
}

}  // namespace lbmi
