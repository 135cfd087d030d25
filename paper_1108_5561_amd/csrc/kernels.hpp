// Launchers of the device kernels (defined in lb_device.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lb_common.hpp"

namespace lbmi {

enum : int { kErrNonfinite = 1, kErrMatch = 2, kErrEos = 4 };

// Site scalars of a state (Landau matching and EoS of it): one record per
// site, 16-byte aligned: kScN values of the node type (u^tau, u^x, u^y, M,
// M_eq = M(T), 1/tau_R [fm^-1], M/T, log2(e)/T), then beta and ln M in FP64.
enum : int { kScUt = 0, kScUx, kScUy, kScM, kScMeq, kScRate, kScMinvT, kScL2invT, kScN };
inline size_t site_record_bytes(size_t elt) { return kScN * elt + 16; }
inline size_t site_scalar_bytes(size_t n_sites, size_t elt) { return n_sites * site_record_bytes(elt); }

struct StageArgs {
  int32_t nx, ny, n_sites;
  int32_t metric;
  double inv2dx;         // 1/(2 dx)    [fm^-1]
  double inv_dx;         // 1/dx
  double tau;            // time of this stage [fm]
  double tau_s;          // tau for the Milne metric (the S1 constants carry no 1/tau), 1 for Minkowski
  double inv_tau_s;      // 1/tau_s
  double dtau;           // step [fm]
  double inv_eta_hbarc;  // 1/((eta/s) hbar c), 0 for eta/s = inf
  double Z;
  double log2Z;          // log2(Z)
};

// One Heun stage.  stage 0: F* = F + dtau K(F); stage 1:
// F_new = (F + F*)/2 + dtau/2 K(F*).  precision 0 = FP64, 1 = FP32;
// scin / scout are the site scalars of the input and output states;
// stageconst is a device pointer to the context's StageConst<double> or
// StageConst<float>.
hipError_t launch_stage(int precision, int stage, const void* Fin, const void* Fbase, void* Fout,
                        const double* lnMin, const double* lnMbase, double* lnMout, const double* scin,
                        double* scout, const void* stageconst, const EosTable& tb, const StageArgs& a,
                        int* err, hipStream_t s);

// Site scalars of the state (F, lnM) into scout.
hipError_t launch_site(int precision, const void* F, const double* lnM, double* scout, const void* stageconst,
                       const EosTable& tb, const StageArgs& a, int* err, hipStream_t s);

hipError_t launch_init(int precision, const double* e0, const double* ux0, const double* uy0, void* F,
                       double* lnM, const void* latconst, const EosTable& tb, const StageArgs& a,
                       int* err, hipStream_t s);

hipError_t launch_moments(int precision, const void* F, const double* lnM, double* out,
                          const void* latconst, const EosTable& tb, const StageArgs& a, int* err,
                          hipStream_t s);

// Canonical [N][sites] FP64 <-> internal node layout (precision).
hipError_t launch_get_state(int precision, const void* F, double* Fc, int n_q, int n_sites,
                            hipStream_t s);
hipError_t launch_set_state(int precision, const double* Fc, void* F, int n_q, int n_sites,
                            hipStream_t s);

}  // namespace lbmi
