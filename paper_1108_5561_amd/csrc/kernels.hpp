// Launchers of the device kernels (defined in lb_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lb_common.hpp"

namespace lbmi {

enum : int { kErrNonfinite = 1, kErrMatch = 2, kErrEos = 4 };

struct StageArgs {
  int32_t nx, ny, n_sites;
  int32_t metric;
  double inv2dx;         // 1/(2 dx)    [fm^-1]
  double inv_dx;         // 1/dx
  double tau;            // time of this stage [fm]
  double dtau;           // step [fm]
  double inv_eta_hbarc;  // 1/((eta/s) hbar c), 0 for eta/s = inf
  double Z;
  double log2Z;          // log2(Z)
};

// One Heun stage.  stage 0: F* = F + dtau K(F); stage 1:
// F_new = (F + F*)/2 + dtau/2 K(F*).  precision 0 = FP64, 1 = FP32.
hipError_t launch_stage(int precision, int stage, const void* Fin, const void* Fbase, void* Fout,
                        const double* lnMin, const double* lnMbase, double* lnMout,
                        const void* latconst, const EosTable& tb, const StageArgs& a, int* err,
                        hipStream_t s);

hipError_t launch_init(int precision, const double* e0, const double* ux0, const double* uy0, void* F,
                       double* lnM, const void* latconst, const EosTable& tb, const StageArgs& a,
                       int* err, hipStream_t s);

hipError_t launch_moments(int precision, const void* F, const double* lnM, double* out,
                          const void* latconst, const EosTable& tb, const StageArgs& a, int* err,
                          hipStream_t s);

// Canonical [N][sites] FP64 <-> internal [q][sites][8] (precision).
hipError_t launch_get_state(int precision, const void* F, double* Fc, int n_q, int n_sites,
                            hipStream_t s);
hipError_t launch_set_state(int precision, const double* Fc, void* F, int n_q, int n_sites,
                            hipStream_t s);

}  // namespace lbmi
