// Constants and launchers of the momentum-lattice-generic FP64 step
// (lb_generic.hip): lattices N_xi, N_theta in {3, 5, 7}, N_phi in {3, 4, 5}.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "lb_common.hpp"

namespace lbmi {

constexpr int kGenMaxXi = 7, kGenMaxTh = 7, kGenMaxL = 10, kGenMaxQ = kGenMaxXi * kGenMaxTh;

// Per-node constants of one phi slice (node q = k N_theta + j; the same on
// every slice) and the azimuths; the Milne 1/tau of S1 is applied by the
// kernel.
struct GenConst {
  double x[kGenMaxXi];      // gamma_k = cosh xi_k
  double sh2[kGenMaxXi];    // sinh^2 xi_k
  double mu2[kGenMaxTh];    // cos^2 theta_j
  double w[kGenMaxQ];       // w_n (Sec. IV.C)
  double sig[kGenMaxQ];     // |v_perp| = sinh xi sin theta
  double sigi[kGenMaxQ];    // |v_perp| / gamma
  double sig2[kGenMaxQ];    // |v_perp|^2
  double wx2[kGenMaxQ];     // w gamma^2
  double wxs[kGenMaxQ];     // w gamma |v_perp|
  double ws2[kGenMaxQ];     // w |v_perp|^2
  double wvY2[kGenMaxQ];    // w (v^Y)^2
  double wx[kGenMaxQ];      // w gamma
  double wsig[kGenMaxQ];    // w |v_perp|
  double A1[kGenMaxXi * kGenMaxXi];   // S1 radial part
  double A2[kGenMaxXi * kGenMaxXi];   // S2
  double Ath[kGenMaxTh * kGenMaxTh];  // S1 polar part
  double cosl[kGenMaxL], sinl[kGenMaxL];
};

// True for the lattices the generic path has kernels for.
inline bool gen_supported(int nxi, int nth, int nphi) {
  return (nxi == 3 || nxi == 5 || nxi == 7) && (nth == 3 || nth == 5 || nth == 7) &&
         (nphi == 3 || nphi == 4 || nphi == 5);
}

hipError_t launch_gen_stage(int nxi, int nth, int nl, int stage, const double* Fin, const double* Lin,
                            const double* Fbase, const double* Lbase, double* Fout, double* Lout, const GenConst* C,
                            const EosTable* tb, const StageArgs& a, int* err, hipStream_t s);
hipError_t launch_gen_init(int nxi, int nth, int nl, const double* e0, const double* ux0, const double* uy0, double* F,
                           double* lnM, const GenConst* C, const EosTable* tb, const StageArgs& a, int* err,
                           hipStream_t s);
hipError_t launch_gen_moments(int nxi, int nth, int nl, const double* F, const double* lnM, double* out,
                              const GenConst* C, const EosTable* tb, const StageArgs& a, int* err, hipStream_t s);

}  // namespace lbmi
