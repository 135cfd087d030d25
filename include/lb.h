/*
 * lb.h - C ABI of the relativistic quasiparticle lattice-Boltzmann step
 * (P. Romatschke, "Relativistic (Lattice) Boltzmann Equation with Non-Ideal
 * Equation of State", arXiv:1108.5561), for AMD Instinct MI355X (gfx950).
 *
 * The library advances the on-shell distribution F_n(x, y) of one uncharged
 * quasiparticle species with a temperature-dependent mass M(T), in
 * boost-invariant Milne coordinates (tau, x, y, eta_s) with a periodic
 * transverse (x, y) lattice.  Per lattice site and stage it forms T^{mu nu}
 * over the discrete momenta (eq. (emtnew)), Landau-matches (eq. (sanity)),
 * inverts the equation of state for T and M(T) (Sec. III.A), relaxes towards
 * the equilibrium with the BGK term (eq. (bgk)) and streams with the Milne and
 * mass-gradient force terms (eqs. (Bmilne), (newBeq)); a step is the
 * predictor / trapezoid-corrector pair of Sec. IV.D.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Units: GeV (T, M), fm (tau, dx), GeV/fm^3 (energy density, T^{mu nu}),
 *         fm^-3 (N^mu); hbar c = 0.1973269804 GeV fm.
 *  Memory: every pointer named d_* is device memory on the current HIP
 *         device, owned by the caller; the library never allocates or frees
 *         device memory (it carves its buffers out of the caller's
 *         workspace).  Host pointers (params, host arrays) are read during the
 *         call only.
 *  Streams: calls are asynchronous on the stream given to lb_init, except
 *         lb_init itself, lb_status, lb_profile_read and the host-only
 *         helpers, which return with the work finished.
 *  Errors: every function returns LB_OK (0) or a negative LB_E_* code.
 *         Argument errors are detected on the host before any device work
 *         and change no state.  Errors found by the kernels (non-finite
 *         values, no timelike eigenvector, temperature outside the table) set
 *         a sticky device error word which lb_status returns.  lb_last_error
 *         gives a thread-local message for the last failure.
 *  Node order (canonical, used by lb_get_state / lb_set_state):
 *         n = (k * n_theta + j) * (2 n_phi) + l, where k indexes the radial
 *         nodes xi_k, j the polar nodes theta_j and l the azimuthal nodes
 *         phi_l (Sec. IV.C).  Site order: site = y * nx + x.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_ctx lb_ctx; /* opaque, host memory owned by the library */

enum {
  LB_OK = 0,
  LB_E_ARG = -1,       /* invalid argument, size or workspace */
  LB_E_HIP = -2,       /* a HIP runtime call failed */
  LB_E_EOS = -3,       /* EoS has no quasiparticle mass, is unstable, or a
                          temperature left the table range */
  LB_E_MATCH = -4,     /* Landau matching found no timelike eigenvector */
  LB_E_NONFINITE = -5, /* non-finite input or state */
  LB_E_STATE = -6,     /* call out of order (e.g. context not initialised) */
  LB_E_NOTIMPL = -7    /* entry point not implemented in this build */
};

enum { LB_FP64 = 0, LB_FP32_FP64MATCH = 1 };          /* storage / node arithmetic */
enum { LB_TAUR_CE = 0, LB_TAUR_MASSLESS = 1 };        /* how tau_R follows eta/s */
enum { LB_METRIC_MILNE = 0, LB_METRIC_MINKOWSKI = 1 };
enum { LB_EOS_TANH_P = 0, LB_EOS_CONST_MASS = 1, LB_EOS_TANH_S = 2, LB_EOS_TABLE = 3 };
enum { LB_OPS_WEAK = 0, LB_OPS_STRONG = 1 };  /* momentum-derivative operators S1, S2 */
enum { LB_FORCE_FEQ = 0, LB_FORCE_WEAK3D = 1 };  /* mass-gradient force of eq. (Bmilne) */
enum { LB_N_FREE = 0, LB_N_CONSERVED = 1 };      /* particle number, eq. (sanity) */
enum { LB_GRAD_CENTRED = 0, LB_GRAD_UPWIND = 1 };  /* d_i ln M of the mass-gradient force */

/*
 * Problem statement (Sec. IV.D: an initial condition is the distribution plus
 * T and M; the step size; the relaxation time tau_R set through eta/s,
 * eq. (bgk) and Sec. IV.A; the EoS through M(T), B(T), Sec. III.A; the
 * momentum lattice N_xi, N_theta, N_phi, z0 = M0/T0, Sec. IV.C; the Milne
 * metric and tau, Sec. IV.D).
 */
typedef struct lb_params {
  int32_t n_xi;        /* radial nodes (roots of R_{N_xi}); this build: 5 */
  int32_t n_theta;     /* polar nodes (roots of L_{N_theta}); this build: 5 */
  int32_t n_phi;       /* azimuths phi_l = l pi / n_phi, l < 2 n_phi; this build: 4 */
  double z0;           /* reference M0/T0 of the radial weight exp(-z0 cosh xi) (> 0) */
  double Z;            /* degeneracy of eq. (feq) (> 0) */
  int32_t nx, ny;      /* periodic transverse lattice, >= 1 each */
  double dx_fm;        /* lattice spacing (> 0) */
  double tau0_fm;      /* initial Milne time (> 0; any value for Minkowski) */
  double eta_over_s;   /* > 0; +INFINITY means tau_R = infinity (free streaming) */
  int32_t taur_rule;   /* LB_TAUR_CE: tau_R = (eta/s) s(T)/h(T) with h the
                          Chapman-Enskog eta/tau_R of Sec. IV.A at M = M(T);
                          LB_TAUR_MASSLESS: tau_R = 5 (eta/s)/T */
  int32_t precision;   /* LB_FP64, or LB_FP32_FP64MATCH: FP32 distributions,
                          streaming and moment sums, FP64 Landau matching,
                          EoS inversion and mass evolution */
  int32_t metric;      /* LB_METRIC_MILNE, or LB_METRIC_MINKOWSKI (no
                          Christoffel term; for tests) */
  int32_t eos_kind;    /* LB_EOS_TABLE: tabulated s(T) (fields eos_T_GeV .. eos_n below);
                          LB_EOS_TANH_S: s/T^3 = (2 pi^2/45) g (1 + tanh((T - Tc)/w))/2,
                          p = int_0^T s dT' (c_s^2 in (0, 1/3] for any w);
                          LB_EOS_TANH_P: p/T^4 = (pi^2/90) g (1 + tanh((T - Tc)/w))/2
                          (c_s^2 > 1/3 above Tc; rejected where d eps/dT <= 0);
                          LB_EOS_CONST_MASS: Boltzmann gas of mass eos_mass (B = 0) */
  double eos_g;        /* g of the tanh EoS (Stefan-Boltzmann degrees of freedom) */
  double eos_Tc_GeV;   /* Tc of the tanh EoS */
  double eos_width_GeV;/* w of the tanh EoS */
  double eos_mass_GeV; /* mass of the constant-mass EoS */
  double T_min_GeV;    /* EoS table range; temperatures outside are an */
  double T_max_GeV;    /*   LB_E_EOS device error (typ. 0.05 and 3.0) */
  /* LB_EOS_TABLE: the caller's entropy density (Sec. III.A takes s(T) as
   * the input of the quasiparticle construction), host arrays read during
   * the calls that take params.  s(T) between the points is the cubic
   * spline with not-a-knot ends of ln(s/T^3) against ln T (twice
   * continuously differentiable, so beta and c_s^2, which involve s', are
   * continuous); p(T) = eos_p0 + the integral of s from eos_T[0];
   * [T_min, T_max] must lie inside [eos_T[0], eos_T[n-1]].  Ignored for the
   * other kinds (set to NULL / 0). */
  const double* eos_T_GeV;  /* [eos_n] strictly increasing, > 0 */
  const double* eos_s_GeV3; /* [eos_n] entropy density, > 0 */
  double eos_p0_GeV4;       /* pressure at eos_T_GeV[0] */
  int32_t eos_n;            /* >= 4 */
  /* S1 (p^Y d/dp^Y) and S2 (p . d/dp) on the momentum lattice (Sec. IV.D):
   * LB_OPS_WEAK, the paper's weak form (projection with the coefficients
   * s_1^{ml}, s_2^{ml}), or LB_OPS_STRONG, the derivatives of the
   * interpolant exp(-z0 cosh xi) P(cosh xi, cos theta) through the nodes
   * (exact on that span).  Both keep the discrete energy balance of
   * eq. (edchange); far from equilibrium (free streaming) the weak form is
   * the more accurate.  Both factor into radial and polar 5 x 5 parts, so
   * the cost is the same. */
  int32_t operator_form;
  /* The force term (1/2) d_i M^2 d^i_(p) of eq. (Bmilne) at fixed v = p~/M,
   * (d_i ln M / gamma) [v^i (v . d_v) + d_{v^i}] with d_i ln M by centred
   * differences, applied either to
   * LB_FORCE_FEQ: the local equilibrium F_eq, differentiated analytically
   *   (exact on F_eq; the lattice moments of the force follow the balance
   *   laws only for F = F_eq), or to
   * LB_FORCE_WEAK3D: F itself, through the weak form of the operator on the
   *   test space of eq. (fansatz) (solid harmonics of v/|v| times powers
   *   of sinh xi times polynomials in cosh xi, one factor sinh xi kept for
   *   odd degree; 2 n_phi x n_theta x n_xi functions on the same number of
   *   nodes).  Energy, momentum and particle-number moments of the force
   *   then follow the balance laws exactly for any F.  It mixes the phi
   *   slices (a real Fourier transform over them), so the stage does about
   *   twice the arithmetic.  lb_step, the batched form and the adjoint
   *   entry points (the FP64 adjoint applies the operators as two dense
   *   N x N matrices, built at lb_init from the stage kernels' own code;
   *   the context's workspace holds them, 2 N^2 doubles). */
  int32_t force_form;
  /* LB_N_FREE: the equilibrium is matched to the energy density only (mu = 0,
   * as in the paper's runs).  LB_N_CONSERVED: also to the particle density
   * n = u_a N^a (second condition of eq. (sanity)), so that the collisions
   * conserve the current N^a; each site then has a temperature and a
   * chemical potential mu, F_eq carries exp(mu/T) (eq. (epsp)) and the CE
   * relaxation time uses s(T, mu) and h(T, mu).  Requires eos_kind
   * LB_EOS_CONST_MASS: a mass depending on T alone is thermodynamically
   * consistent (eq. (cdef)) at mu != 0 only if it is constant.  The site's
   * mu/T follows from the outputs as ln(n / n0(T)), n0 the density at mu = 0.
   * lb_step, lb_moments and the batched form (not together with
   * LB_FORCE_WEAK3D there); the adjoint entry points return LB_E_NOTIMPL
   * for it. */
  int32_t particle_number;
  /* mu/T of the initial state (uniform; lb_init): eps(T0, mu0) = e0 and
   * F = Z exp(mu0/T0 - u.P/T0).  Must be 0 unless LB_N_CONSERVED. */
  double mu_over_T0;
  /* The transverse gradient d_i ln M in the mass-gradient force on F_eq:
   * LB_GRAD_CENTRED, (ln M_{i+1} - ln M_{i-1}) / (2 dx); or LB_GRAD_UPWIND,
   * per node the same second-order upwind difference the streaming of that
   * node uses, (3 ln M_i - 4 ln M_{i-1} + ln M_{i-2}) / (2 dx) along the
   * node's direction of motion (centred along an axis the node does not
   * move on).  The streaming and the force are the two halves of the
   * transport term P^mu d_mu at fixed v = p/M of eq. (Bmilne); with one
   * difference operator for both, ln M modes near the grid scale, which a
   * centred difference does not see, are held by the force (a white-noise
   * initial state at eta/s 0.2 on a 0.025 fm grid keeps its ln M spread
   * bounded instead of growing).  Requires force_form LB_FORCE_FEQ;
   * lb_step, lb_moments, the batched form and the adjoint entry points take
   * it. */
  int32_t gradient_form;
} lb_params;

/*
 * Device workspace size in bytes for these parameters, or 0 on an invalid
 * parameter set (message in lb_last_error).  Host only; no device call.
 */
size_t lb_workspace_bytes(const lb_params* p);

/*
 * Create a context and set the initial state (Sec. IV.D: the state is the
 * distribution plus T and M).  Per site, T0 is the root of eps_EoS(T0) = e0
 * on [T_min, T_max] (eps_EoS is monotone for an accepted EoS), M = M(T0), and
 * F_n is the local equilibrium Z exp(-(u . P_n)/T0) with P_n = M V_n and
 * u = (sqrt(1 + ux^2 + uy^2), ux, uy).
 *   out         receives the context (host memory; free with lb_destroy).
 *   p           parameters; copied.
 *   d_workspace device buffer of at least lb_workspace_bytes(p) bytes, 256-byte
 *               aligned, owned by the caller, not touched by anyone else
 *               while the context lives.
 *   d_e0        [ny][nx] FP64 energy density in GeV/fm^3 (read during the call).
 *   d_ux0, d_uy0 [ny][nx] FP64 initial transverse flow, or NULL for zero.
 *   hip_stream  the hipStream_t all later calls of this context run on
 *               (NULL = the null stream).
 * Builds the momentum lattice, the weak-form operators and the EoS tables on
 * the host in FP64/long double and copies them into the workspace.  Returns
 * LB_E_ARG on invalid parameters, LB_E_EOS if M(T) has no solution or the EoS
 * is thermodynamically unstable (d eps/dT <= 0) anywhere in [T_min, T_max],
 * LB_E_NONFINITE / LB_E_EOS if e0 is non-finite or outside the table; it
 * synchronises the stream before returning.
 */
int lb_init(lb_ctx** out, const lb_params* p, void* d_workspace, size_t ws_bytes,
            const double* d_e0, const double* d_ux0, const double* d_uy0, void* hip_stream);

/*
 * Advance n_steps >= 0 Heun steps of size dtau_fm > 0 (Sec. IV.D: predictor
 * F* = F + dtau K(F), corrector F_new = F + dtau/2 (K(F) + K(F*)), and the
 * same for ln M).  Each step is two kernel launches.  Returns LB_E_ARG if
 * dtau is not finite and positive or if the streaming CFL number
 * max_n (|v^x_n| + |v^y_n|)/gamma_n * dtau/dx exceeds 0.5 (the stability
 * limit of the second-order upwind transverse streaming under Heun).
 */
int lb_step(lb_ctx* c, int32_t n_steps, double dtau_fm);

/*
 * Per-site observables into d_out, FP64 [14][ny][nx]:
 *   T^{tau tau}, T^{tau x}, T^{tau y}, T^{xx}, T^{xy}, T^{yy}, T^{YY}  (GeV/fm^3,
 *     Milne-orthonormal components of eq. (emtnew), including B(T) g^{mu nu}),
 *   N^tau, N^x, N^y (fm^-3, eq. (NTdisc)),
 *   T (GeV) and u^x, u^y from Landau matching (eq. (sanity)), M (GeV).
 */
int lb_moments(lb_ctx* c, double* d_out);

/* Current state in canonical order, FP64: d_F [N][ny][nx], d_lnM [ny][nx]
 * (N = n_xi n_theta 2 n_phi), and the current Milne time (host). */
int lb_get_state(lb_ctx* c, double* d_F, double* d_lnM, double* tau_fm);

/* Replace the state (same layouts; FP32 contexts round to FP32) and the time.
 * For checkpoint / restart and for tests that start both precisions from one
 * state. */
int lb_set_state(lb_ctx* c, const double* d_F, const double* d_lnM, double tau_fm);

/* ---- differentiable form: discrete adjoint of the FP64 step ----
 *
 * The step differentiated is the FP64 Heun step of Sec. IV.D as lb_step
 * computes it for an LB_FP64 context (same right-hand side: streaming,
 * Milne term, BGK of eq. (bgk) with the equilibrium of eq. (feq) and the
 * mass-gradient force of either force_form, mass evolution of eqs.
 * (edchange), (masschange); T, u
 * and M_eq from the Landau matching of eq. (sanity) and the EoS inversion
 * of Sec. III.A, whose derivatives are taken by the implicit-function
 * theorem).  States and adjoints are in the canonical order of
 * lb_get_state, FP64: F [N][ny][nx], ln M [ny][nx].  The adjoint is that of
 * the FP64 step, evaluated on the states the caller passes (e.g. the FP32
 * trajectory of an LB_FP32_FP64MATCH context).  For an LB_FP64 context all
 * of its arithmetic is FP64; for an LB_FP32_FP64MATCH context the reverse
 * sweep's per-node arithmetic is FP32 (the per-site chain through the
 * matching and the EoS, and the site sums, stay FP64), as the forward.
 * With particle_number LB_N_CONSERVED (constant mass) the step is the one
 * with the n matching of eq. (sanity): T and mu/T from lambda and
 * n = u_a N^a, the fugacity in F_eq and tau_R at (T, mu), all
 * differentiated (the reverse sweep is then FP64 for either precision),
 * and lb_adjoint_init takes the initial mu0/T0.  The calls only read the
 * context's parameters, lattice and EoS tables; its state is not used or
 * changed.  The adjoint workspace is caller-owned device memory, 256-byte
 * aligned, of at least lb_adjoint_workspace_bytes(p) bytes, not touched by
 * anyone else during a call.  Calls are asynchronous on the context's
 * stream.  Either gradient_form (the upwind ln M gradient differentiated
 * per phi slice).  LB_E_NOTIMPL for momentum lattices other than
 * 5 x 5 x 8.
 */

/* Adjoint workspace size for these parameters (0 on invalid parameters). */
size_t lb_adjoint_workspace_bytes(const lb_params* p);

/*
 * One step of the differentiated FP64 step, from the state (d_F, d_lnM) at
 * tau_fm to (d_F_out, d_lnM_out) at tau_fm + dtau_fm (outputs must not
 * alias the inputs).  Equal to lb_step on an LB_FP64 context up to rounding
 * order; it is the forward map whose transpose lb_adjoint_step applies.
 * LB_E_ARG for NULL or aliasing pointers, a workspace that is too small, a
 * tau that is not finite (or <= 0 for the Milne metric), or a dtau that
 * lb_step would reject (CFL).
 */
int lb_adjoint_forward_step(lb_ctx* c, double tau_fm, double dtau_fm, const double* d_F, const double* d_lnM,
                            double* d_F_out, double* d_lnM_out, void* d_adj_workspace, size_t adj_ws_bytes);

/*
 * Reverse mode of one step at the forward state (d_F, d_lnM) at tau_fm:
 * on entry (d_adj_F, d_adj_lnM) hold dL/dF and dL/d ln M of the state at
 * tau_fm + dtau_fm; on return they hold dL/dF, dL/d ln M of the state at
 * tau_fm.  *d_grad_eta_over_s (one device double) is incremented by the
 * step's contribution to dL/d(eta/s) (tau_R depends on eta/s through
 * Sec. IV.A; zero for eta/s = infinity).  Errors as lb_adjoint_forward_step;
 * non-finite values or a failed matching set the device error word.
 */
int lb_adjoint_step(lb_ctx* c, double tau_fm, double dtau_fm, const double* d_F, const double* d_lnM,
                    double* d_adj_F, double* d_adj_lnM, double* d_grad_eta_over_s, void* d_adj_workspace,
                    size_t adj_ws_bytes);

/*
 * lb_adjoint_step without the adjoint workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the scratch lives in a static device
 * array of the library, 80 MiB per device (held from the library's load
 * until the process ends), enough for grids of up to about 17000 sites
 * (4840 bytes per site, 4952 with the upwind ln M gradient; the 128 x 128
 * gradient workload fits).  Arguments,
 * results and errors as lb_adjoint_step; LB_E_ARG with a message if the
 * grid needs more scratch than that.  Calls on one device share its array,
 * so calls that overlap on one device (other streams, other threads) race;
 * each call writes every scratch value before reading it.  Allocates
 * nothing (the array's address is looked up once per device).
 */
int lb_adjoint_step_noalloc(lb_ctx* c, double tau_fm, double dtau_fm, const double* d_F, const double* d_lnM,
                            double* d_adj_F, double* d_adj_lnM, double* d_grad_eta_over_s);

/*
 * Reverse mode of the initial state of lb_init (T0 from eps_EoS(T0) = e0,
 * M = M(T0), F_n = Z exp(-(u . P_n)/T0), the flow held fixed): writes
 * d_grad_e0[ny][nx] = dL/d e0 (per GeV/fm^3) given (d_adj_F, d_adj_lnM) =
 * dL/d(F, ln M) of the initial state.  d_e0, d_ux0, d_uy0 as passed to
 * lb_init (both flows NULL for zero flow).
 */
int lb_adjoint_init(lb_ctx* c, const double* d_e0, const double* d_ux0, const double* d_uy0,
                    const double* d_adj_F, const double* d_adj_lnM, double* d_grad_e0);

/* Synchronise the context's stream and return the sticky device error
 * (LB_OK if none). */
int lb_status(lb_ctx* c);

/* Release the context (the workspace stays the caller's). */
int lb_destroy(lb_ctx* c);

/* Thread-local message of the last failure ("" if none). */
const char* lb_last_error(void);

/* ---- host-only helpers (no device call) ---- */

/*
 * Momentum lattice and factored weak-form operators as built for the device
 * (Sec. IV.C, IV.D).  With out == NULL returns the number of doubles needed;
 * otherwise fills out with
 *   x_k = cosh xi_k [n_xi], w^xi_k [n_xi], mu_j = cos theta_j [n_theta],
 *   w^theta_j [n_theta], cos phi_l [2 n_phi], sin phi_l [2 n_phi],
 *   A1 [n_xi][n_xi], A2 [n_xi][n_xi], Ath [n_theta][n_theta]
 * where on every phi slice S2[F]_{kj} = sum_k' A2_{kk'} F_{k'j} and
 * S1[F]_{kj} = mu_j^2 sum_k' A1_{kk'} F_{k'j} - sum_j' Ath_{jj'} F_{kj'}.
 * Returns the count, or a negative LB_E_* code.
 */
int64_t lb_lattice_info(const lb_params* p, double* out, int64_t n_out);

/*
 * Per-node quantities of the momentum lattice in the canonical node order
 * (Sec. IV.C), for callers that form moments of lb_get_state's output
 * themselves.  With out == NULL returns the number of doubles needed (5 N);
 * otherwise fills out with five arrays of N values:
 *   w_n   the product weight e^{z0 x_k} w^xi_k w^theta_j / (4 n_phi) (the
 *         radial weight's exp(-z0 cosh xi) divided out, angular weights
 *         summing to one), so that T^{ab}_kin = M^4/(2 pi^2) sum_n w_n F_n
 *         V^a_n V^b_n (eq. (emtnew)) and N^a = M^3/(2 pi^2) sum_n w_n F_n V^a_n;
 *   gamma_n = cosh xi_k, v^x_n, v^y_n = sinh xi_k sin theta_j (cos, sin) phi_l,
 *   v^Y_n = sinh xi_k cos theta_j (V_n = (gamma, v^x, v^y, v^Y)_n).
 * Returns the count, or a negative LB_E_* code (n_out too small, invalid
 * lattice parameters).
 */
int64_t lb_node_table(const lb_params* p, double* out, int64_t n_out);

/*
 * Degeneracy Z of eq. (feq) whose Boltzmann gas has kappa times the
 * Stefan-Boltzmann pressure of g bosonic degrees of freedom (Sec. III: the
 * high-temperature limit of the quasiparticle pressure): Z = kappa g pi^4 / 90.
 * kappa = 1 is the paper's matching; a larger kappa keeps M(T) solvable where
 * the EoS's entropy exceeds the massless gas's.  Pure function, no errors.
 */
double lb_degeneracy(double kappa, double g);

/*
 * Host evaluation of the equation of state at n temperatures T_GeV[i]:
 * out[8 i + 0..7] = eps, p, s (GeV^4, GeV^4, GeV^3), M (GeV), B (GeV^4),
 * eps - B (GeV^4), beta = dB/d(eps - B), tau_R (fm).  table != 0 evaluates
 * the interpolated device tables instead of the exact functions (M, B,
 * eps - B, beta, tau_R only; eps, p, s are then the exact values).
 */
int lb_eos_eval(const lb_params* p, int64_t n, const double* T_GeV, double* out, int32_t table);

/* Kernel timing with HIP events on the context's stream: enable != 0 starts
 * recording (and clears totals); lb_profile_read synchronises and returns the
 * summed milliseconds and launch counts of the predictor [0] and corrector
 * [1] stage kernels. */
int lb_profile(lb_ctx* c, int32_t enable);
int lb_profile_read(lb_ctx* c, double* ms_out, int64_t* count_out);

/* Mean duration in milliseconds of one launch of the predictor (stage 0) or
 * corrector (stage 1) kernel, from HIP events around n >= 1 back-to-back
 * launches on the context's stream (after one untimed predictor).  The
 * launches read the current state and write only the two spare state
 * buffers, so the state, the time and the next lb_step are unchanged.
 * Synchronises the stream; returns the device error word like lb_status. */
int lb_profile_stage(lb_ctx* c, int32_t stage, int32_t n, double dtau_fm, double* ms_out);

/* ---- batched form: many events advanced together ----
 *
 * A batch advances n_events independent events (boost-invariant initial
 * conditions, e.g. fluctuating ones, on their own periodic transverse grids)
 * of one species, lattice and EoS, with one kernel launch per Heun stage
 * covering the tiles of all events; the library keeps one context-wide
 * state per event exactly as lb_step would (an event's result does not
 * depend on the batch it is in).  Runs of 48 steps that start at the first
 * buffer rotation are replayed from a captured HIP graph; the tile shape and
 * occupancy of the batched kernel are chosen by timing the candidates on the
 * batch itself (lb_batch_tune, or automatically at the first lb_batch_step).
 */
typedef struct lb_batch lb_batch; /* opaque, host memory owned by the library */

typedef struct lb_event {
  int32_t nx, ny;      /* periodic transverse lattice of the event, >= 1 each */
  double dx_fm;        /* its spacing (> 0) */
  double eta_over_s;   /* its eta/s (> 0, +INFINITY for free streaming) */
} lb_event;

/* Workspace bytes for the batch (0 on invalid input; message in
 * lb_last_error).  p gives everything but the per-event grid, spacing and
 * eta/s, whose fields in p are ignored. */
size_t lb_batch_workspace_bytes(const lb_params* p, const lb_event* events, int32_t n_events);

/* Create a batch: as lb_init for every event, with zero initial flow.
 * d_e0 is a host array of n_events device pointers, each [ny][nx] FP64
 * energy density in GeV/fm^3 of that event (read during the call).  The
 * library allocates 2 x 48 stage-time records of pinned host memory
 * (hipHostMalloc) for the graph replays; device memory is the caller's
 * workspace only.  Errors as lb_init. */
int lb_batch_init(lb_batch** out, const lb_params* p, const lb_event* events, int32_t n_events,
                  void* d_workspace, size_t ws_bytes, const double* const* d_e0, void* hip_stream);

/* Time every variant of the batched stage kernel (tile rows 2, 4, 8; in
 * FP32 with 4 or 3 waves per SIMD as occupancy target, with or without
 * streaming stores of the new state: variant v has kBatchTileRows
 * 2, 4, 8 for v % 3, 4 waves for (v / 3) % 2 == 0 else 3, streaming for
 * v >= 6) on the batch's own events for a few steps of size dtau_fm, on
 * the spare state buffers (the state is unchanged), and keep the fastest.
 * variant_out (may be NULL) receives its index; ms_out (may be NULL) the
 * mean milliseconds per step of each variant ([12] in FP32, [3] in FP64).
 * With LB_FORCE_WEAK3D, LB_N_CONSERVED (or both) or LB_GRAD_UPWIND there
 * are three variants, tile rows 2, 4, 8 (v = 0, 1, 2) at the single-event
 * kernel's occupancy.
 * Synchronous. */
int lb_batch_tune(lb_batch* b, double dtau_fm, int32_t* variant_out, double* ms_out);

/* Use kernel variant `variant` (0..11 in FP32, 0..2 in FP64 or with the 3-D
 * force, the conserved particle number or the upwind ln M gradient,
 * numbered as in lb_batch_tune)
 * without timing: pins a tuned choice. */
int lb_batch_set_variant(lb_batch* b, int32_t variant);

/* Advance every event n_steps Heun steps of dtau_fm (as lb_step; LB_E_ARG
 * if the CFL limit is exceeded in any event).  Tunes first if not tuned. */
int lb_batch_step(lb_batch* b, int32_t n_steps, double dtau_fm);

/* Observables of one event into d_out [14][ny][nx] (as lb_moments). */
int lb_batch_moments(lb_batch* b, int32_t event, double* d_out);

/* State of one event in canonical order (as lb_get_state). */
int lb_batch_get_state(lb_batch* b, int32_t event, double* d_F, double* d_lnM, double* tau_fm);

/* Synchronise and return the sticky device error of the batch. */
int lb_batch_status(lb_batch* b);

/* Release the batch (the workspace stays the caller's). */
int lb_batch_destroy(lb_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
