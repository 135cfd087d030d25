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
  int32_t force_form;    // LB_FORCE_FEQ or LB_FORCE_WEAK3D (lb_step only)
  int32_t mu_mode;       // 1: conserved particle number (n matching; record slot beta holds mu/T)
  int32_t grad_form;     // LB_GRAD_CENTRED or LB_GRAD_UPWIND: d_i ln M of the force on F_eq
  double inv2dx;         // 1/(2 dx)    [fm^-1]
  double inv_dx;         // 1/dx
  double tau;            // time of this stage [fm]
  double tau_s;          // tau for the Milne metric (the S1 constants carry no 1/tau), 1 for Minkowski
  double inv_tau_s;      // 1/tau_s
  double dtau;           // step [fm]
  double inv_eta_hbarc;  // 1/((eta/s) hbar c), 0 for eta/s = inf
  double Z;
  double log2Z;          // log2(Z)
  double alpha0;         // mu/T of the initial state (lb_init)
};

// One Heun stage.  stage 0: F* = F + dtau K(F); stage 1:
// F_new = (F + F*)/2 + dtau/2 K(F*).  precision 0 = FP64, 1 = FP32;
// scin / scout are the site records of the input and output states; d_tb
// is the device copy of the EoS table descriptor;
// stageconst is a device pointer to the context's StageConst<double> or
// StageConst<float>.
hipError_t launch_stage(int precision, int stage, const void* Fin, const void* Fbase, void* Fout,
                        const double* lnMin, const double* lnMbase, double* lnMout, const double* scin,
                        double* scout, const void* stageconst, const EosTable* d_tb, const StageArgs& a,
                        int* err, hipStream_t s);

// ---- batched form: many events (own grid, spacing, eta/s, state) advanced
// by one launch per stage ----
struct BatchEvent {
  int32_t nx, ny, n_sites, tile0;  // tile0: first tile of the event in the launch
  double inv2dx, inv_eta_hbarc;
  void* F[3];
  double* lnM[3];
  double* sc[3];
};
// Time of one stage: tau, and tau_s / 1/tau_s of StageArgs.
struct StageTime {
  double tau, tau_s, inv_tau_s;
};
// Variants of the batched stage kernel (the tuning choices): variant v has
// kBatchTileRows[v % 3] tile rows (tiles are 8 sites wide) and, in FP32,
// 4 ((v / 3) % 2 = 0) or 3 waves per SIMD as occupancy target, with
// streaming (nontemporal) stores of the new state for v >= 6; FP64 has
// variants 0..2 at 2 waves per SIMD.  With the weak-form 3-D force, the
// conserved particle number (or both), or the upwind ln M gradient there
// are three variants, tile rows 2, 4, 8 at the occupancy of the
// single-event kernel.
constexpr int kBatchTileRows[3] = {2, 4, 8};
inline int batch_variants(int precision, int force_form = 0, int particle_number = 0, int gradient_form = 0) {
  return (force_form || particle_number || gradient_form) ? 3 : (precision == 1 ? 12 : 3);
}
inline int batch_tile_rows(int variant) { return kBatchTileRows[variant % 3]; }
inline int batch_tiles(int nx, int ny, int tile_rows) { return ((nx + 7) / 8) * ((ny + tile_rows - 1) / tile_rows); }

// One stage of every event.  ev [n_events], tile_event [n_tiles] (event of
// each tile, in the launch's tile numbering); the stage time is `time` or,
// if times != NULL, times[time_idx] (read by the kernel: graph replays
// refresh it); buffers i_in, i_base, i_out of each event.
hipError_t launch_batch_stage(int precision, int stage, int variant, const BatchEvent* ev,
                              const int32_t* tile_event, int n_tiles, StageTime time, const StageTime* times,
                              int time_idx, int i_in, int i_base, int i_out, const void* stageconst,
                              const EosTable* d_tb, const StageArgs& shared, int* err, hipStream_t s);

// Site scalars of the state (F, lnM) into scout.
hipError_t launch_site(int precision, const void* F, const double* lnM, double* scout, const void* stageconst,
                       const EosTable* d_tb, const StageArgs& a, int* err, hipStream_t s);

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

// Dense weak-form force operators G [2][200][200] (canonical node order,
// G_i[n][m]) from the stage kernels' weak_force, given a device
// StageConst<double> with the force constants.
hipError_t launch_force_columns(const void* cst64, double* G, hipStream_t s);

// Adjoint of the FP64 step (lb_adjoint.hip), canonical layout F[n][site].
// g3 is the dense force operator of launch_force_columns for the weak-form
// 3-D force, or nullptr for the force on F_eq.
// One stage of the step: stage 0 Fout = Fin + dtau K(Fin), stage 1
// Fout = (Fbase + Fin)/2 + dtau/2 K(Fin), ln M likewise; lc points to the
// context's LatticeConst<double, 5, 5> (host).  With lc32 (a device
// LatticeConst<float, 5, 5>) the per-node arithmetic runs in FP32 (site
// chain FP64, once per site).
hipError_t launch_adj_stage_fwd(const double* Fin, const double* Lin, const double* Fbase, const double* Lbase,
                                double* Fout, double* Lout, int stage, const void* lc, const double* g3,
                                const EosTable& tb, const StageArgs& a, int* err, hipStream_t s,
                                const void* lc32 = nullptr);
// Reverse sweep of one right-hand side at (F, ln M), time a.tau, with
// K_bar = scale seedF, X_bar = scale seedL, into (outF, outL) (written, or
// added with accumulate = 1), plus the per-site eta/s adjoint; Rb
// ([N][sites] doubles; FP32 values with lc32) and gb ([2][sites], or
// [2][8][sites] with the upwind ln M gradient: per phi slice) are
// scratch.  lc32 as for launch_adj_stage_fwd.  With combF (combL) the Heun
// combination follows in the same pass: outF <- outF + combF/2, then
// combF <- combF/2 + outF.
hipError_t launch_adj_rhs(const double* F, const double* Lm, const double* seedF, const double* seedL,
                          double scale, double* outF, double* outL, double* Rb, double* gb, double* eta_part,
                          int accumulate, const void* lc, const double* g3, const EosTable& tb,
                          const StageArgs& a, int* err, hipStream_t s, const void* lc32 = nullptr,
                          double* combF = nullptr, double* combL = nullptr);
// *out += sum of v[0..n), deterministic order.
hipError_t launch_adj_sum(const double* v, int n, double* out, hipStream_t s);
// d/d e0 of (aF . F0 + aL . ln M0) for the initial state of lb_init.
hipError_t launch_adj_init(const double* e0, const double* ux0, const double* uy0, const double* aF,
                           const double* aL, double* grad_e0, const void* lc, const EosTable& tb,
                           const StageArgs& a, int* err, hipStream_t s);

}  // namespace lbmi
