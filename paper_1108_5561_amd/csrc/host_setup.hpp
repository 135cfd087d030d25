// Host-side setup: momentum lattice, factored weak-form operators and EoS
// tables (paper Sec. III.A, IV.A, IV.C, IV.D).  Built in long double / double
// on the host once per context and copied to the device.
#pragma once

#include <string>
#include <vector>

#include "../../include/lb.h"
#include "lb_common.hpp"

namespace lbmi {

struct HostLattice {
  int nxi = 0, nth = 0, nphi = 0;
  double z0 = 0;
  std::vector<double> x, wxi, mu, wth, cosl, sinl;  // 1-D rules
  std::vector<double> A1, A2, Ath;                   // factored operators
  double vsum_max = 0;                               // max (|v^x|+|v^y|)/gamma
};

// Returns "" on success, else an error message.
std::string build_lattice(const lb_params& p, HostLattice* out);

// Quasiparticle equation of state on the host (exact functions).
class HostEos {
 public:
  explicit HostEos(const lb_params& p);
  double p(double T) const;
  double s(double T) const;
  double ds(double T) const;
  double eps(double T) const { return T * s(T) - p(T); }
  // z = M/T; returns false if no quasiparticle mass exists at T.
  bool z_of_T(double T, double z_guess, double* z) const;
  struct Point {
    double eps, p, s, M, B, ekin, beta, q;
    double n0, qn;  // particle density at mu = 0; T n0/h (0 for the massless rule)
  };
  bool eval(double T, double z_guess, Point* out, double* z_used) const;
  double Z() const { return Z_; }

 private:
  // tabulated s(T): y = ln(s/T^3) on x = ln T, the spline's second
  // derivatives, and p at the knots (p0 + the integral of s)
  std::vector<double> tx_, ty_, td_, tp_;
  int tab_interval(double x) const;
  double tab_y(double x, double* dy) const;
  double tab_s_integral(int k, double T) const;  // int_{T_k}^{T} s dT'
  int kind_;
  double Z_, g_, Tc_, w_, m0_, c_;
  int taur_rule_;
};

struct HostTables {
  std::vector<double> pts, inv_ek, inv_ee, gpts;
  EosTable desc;  // pointers filled in when copied to the device
};

// Builds (or reuses a cached copy of) the device tables.  "" on success.
std::string build_tables(const lb_params& p, HostTables* out);

// Expected table point count (for workspace sizing).
constexpr int kTablePoints = 32768;
constexpr int kInvPoints = 32768;
constexpr int kGPoints = 32768;

}  // namespace lbmi
