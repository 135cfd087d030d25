"""One Heun step of the boost-invariant Milne lattice-Boltzmann scheme on a
periodic transverse (x, y) lattice (paper Sec. IV.D, eqs. (Bmilne), (newBeq),
(bgk), (sanity), (emtnew), (edchange), (masschange)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

State per site: F_n (the on-shell distribution at fixed v = p~/M on the N
nodes) and ln M.  tau is global.  Units: fm for tau, dx; GeV for T, M.

Right-hand side at (F, ln M, tau), per site (step numbers used below):

 1. kinetic moments T^{ab}_kin = M^4/(2pi^2) sum w F V^a V^b, a, b in
    (tau, x, y) (eq. (emtnew) without B);
 2. Landau matching (eq. (sanity)): u is the timelike eigenvector (u.u = 1,
    u^tau > 0) of the mixed tensor T_kin^{ab} g_{bc}; its eigenvalue lambda
    is eps - B, because B g^{ab} only shifts the eigenvalues;
 3. T from eps_kin_eq(T) = lambda, then M_eq = M(T), beta(T), tau_R(T);
 4. equilibrium on the nodes, F_eq = Z exp(-[u^tau E_eq - M (u^x v^x + u^y v^y)]/T)
    with E_eq = sqrt(M_eq^2 + M^2 sinh^2 xi) (Sec. IV.D, last paragraph, with
    flow);
 5. BGK (eq. (bgk) divided by E): C = ((u.V)/gamma) (F - F_eq)/tau_R, where
    u.V = u^tau gamma - u^x v^x - u^y v^y;
 6. S1 = D1 F, S2 = D2 F on every phi slice (Sec. IV.D);
 7. transport -sum_i (v^i/gamma) dF/dx^i with second-order upwind differences,
    periodic boundaries;
 8. mass-gradient force of eq. (Bmilne), (1/2) d_i M^2 d^i_(p), at fixed v:
    Gr = sum_i (g_i/gamma) [v^i (v . d_v F_eq) + d_{v^i} F_eq], g_i = d_i ln M
    by centred differences (or, with Params.grad = "upwind", per node by the
    same upwind difference as its streaming in step 7, centred along an
    axis the node does not move on), derivatives of F_eq taken analytically (lattice
    force "feq"); or Gr = sum_i g_i G_i F with the weak-form operators of
    force3d acting on F itself (lattice force "weak3d");
 9. R0 = A + S1/tau + Gr - C (the S1/tau term is the Milne Christoffel term and
    is absent for the Minkowski metric);
10. X = d ln M/d tau from eq. (masschange) with the temperature fixed by
    lambda: (M^4/2pi^2) X sum w F = -dB/dtau = -beta d lambda/dtau and
    d lambda/dtau = u_a u_b dT^{ab}_kin/dtau give
    X = -beta sum w (u.V)^2 R0 / [sum w F + beta sum w (u.V)^2 (4 F + S2)];
11. K = R0 + X S2 (= dF/dtau at fixed v).

Heun: F* = F + dtau K, lnM* = lnM + dtau X; (K*, X*) at (F*, lnM*, tau + dtau);
F_new = F + dtau/2 (K + K*), lnM_new = lnM + dtau/2 (X + X*).

Readings (the paper gives the scheme without space dependence): the transverse
terms 7 and 8 follow eq. (Bmilne) in the fixed-v variables of eq. (newBeq);
with a uniform state they vanish and the step is the paper's 0+1-D algorithm
(u = (1, 0, 0), lambda = T^{tau tau}_kin, beta/(1+beta) = dB/deps).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import force3d
from .eos import HBARC

PI2 = np.pi ** 2
METRIC_MILNE = 0
METRIC_MINKOWSKI = 1


@dataclass
class Params:
    dx: float                 # fm
    eta_over_s: float         # may be inf (free streaming)
    taur_rule: str = "ce"     # "ce" or "massless"
    metric: int = METRIC_MILNE
    T_lo: float = 0.05
    T_hi: float = 3.0
    conserve_n: bool = False  # match n = u_a N^a as well: T and mu/T per site
    grad: str = "centred"     # d_i ln M of the force: "centred" or "upwind" (the streaming's stencil per node)


def landau(Tk3):
    """Timelike eigenvector u and eigenvalue lambda of T^{ab} g_{bc}, per site.

    Tk3 has shape (3, 3, ...sites).  Returns u (3, ...) and lam (...).
    numpy.linalg.eig solves each 3x3 mixed tensor; the eigenvector with
    u.u > 0 is selected and normalised to u.u = 1, u^tau > 0.
    """
    sh = Tk3.shape[2:]
    A = np.moveaxis(Tk3.reshape(3, 3, -1), -1, 0) * np.array([1.0, -1.0, -1.0])[None, None, :]
    evals, evecs = np.linalg.eig(A)
    evals = evals.real
    evecs = evecs.real
    norm = evecs[:, 0, :] ** 2 - evecs[:, 1, :] ** 2 - evecs[:, 2, :] ** 2   # (sites, 3)
    pick = np.argmax(norm, axis=1)
    idx = np.arange(A.shape[0])
    if np.any(norm[idx, pick] <= 0):
        raise FloatingPointError("no timelike eigenvector")
    u = evecs[idx, :, pick] / np.sqrt(norm[idx, pick])[:, None]
    u *= np.sign(u[:, 0])[:, None]
    lam = evals[idx, pick]
    return np.moveaxis(u, 0, -1).reshape((3,) + sh), lam.reshape(sh)


def upwind_derivative(F, axis, positive):
    """Second-order one-sided derivative (times dx) along a periodic axis.

    positive: (3 F_i - 4 F_{i-1} + F_{i-2}) / 2;  otherwise
    -(3 F_i - 4 F_{i+1} + F_{i+2}) / 2.
    """
    if positive:
        return 0.5 * (3 * F - 4 * np.roll(F, 1, axis) + np.roll(F, 2, axis))
    return -0.5 * (3 * F - 4 * np.roll(F, -1, axis) + np.roll(F, -2, axis))


def rhs(lat, eos, prm: Params, F, lnM, tau):
    """(K, X, diagnostics) at one stage; F (N, ny, nx), lnM (ny, nx)."""
    N = lat.N
    M = np.exp(lnM)
    bc = (slice(None), None, None)

    # 1. kinetic moments (tau, x, y block)
    Tk, _ = lat.moments(F, lnM)
    Tk3 = Tk[:3, :3]

    # 2. Landau matching
    u, lam = landau(Tk3)
    ut, ux, uy = u[0], u[1], u[2]

    # 3. temperature and EoS functions
    alpha = np.zeros_like(lam)
    if prm.conserve_n:
        T, alpha = _match_n(lat, eos, prm, F, lnM, u, lam)
    else:
        T = eos.T_from_eps_kin_eq(lam.ravel(), prm.T_lo, prm.T_hi).reshape(lam.shape)
    M_eq = eos.M(T)
    beta = eos.beta(T)
    if np.isinf(prm.eta_over_s):
        inv_tauR = np.zeros_like(T)
    elif prm.conserve_n:
        inv_tauR = 1.0 / eos.tau_R_mu(T.ravel(), alpha.ravel(), prm.eta_over_s, prm.taur_rule).reshape(T.shape)
    else:
        inv_tauR = 1.0 / eos.tau_R(T.ravel(), prm.eta_over_s, prm.taur_rule).reshape(T.shape)

    # 4. equilibrium on the nodes
    gam = lat.gamma[bc]
    vx, vy = lat.V[1][bc], lat.V[2][bc]
    sh2 = (lat.gamma ** 2 - 1.0)[bc]
    E_eq = np.sqrt(M_eq ** 2 + M ** 2 * sh2)
    uv = ux * vx + uy * vy
    F_eq = eos.Z * np.exp(alpha - (ut * E_eq - M * uv) / T)

    # 5. BGK
    uV = ut * gam - uv
    C = (uV / gam) * (F - F_eq) * inv_tauR

    # 6. momentum operators
    S1 = lat.apply_slices(lat.D1, F)
    S2 = lat.apply_slices(lat.D2, F)

    # 7. transport, second-order upwind, periodic
    A = np.zeros_like(F)
    for n in range(N):
        ax_v = lat.V[1, n]
        ay_v = lat.V[2, n]
        g = lat.gamma[n]
        if ax_v != 0.0:
            A[n] -= (ax_v / g) * upwind_derivative(F[n], 1, ax_v > 0) / prm.dx
        if ay_v != 0.0:
            A[n] -= (ay_v / g) * upwind_derivative(F[n], 0, ay_v > 0) / prm.dx

    # 8. mass-gradient force on F_eq
    gx = (np.roll(lnM, -1, 1) - np.roll(lnM, 1, 1)) / (2 * prm.dx)
    gy = (np.roll(lnM, -1, 0) - np.roll(lnM, 1, 0)) / (2 * prm.dx)
    if prm.grad == "upwind":
        # per node, the transport's own second-order upwind difference along
        # its direction of motion (centred along an axis it does not move on)
        if lat.force != "feq":
            raise ValueError("the upwind ln M gradient is defined for the force on F_eq")
        sx = np.sign(np.round(lat.V[1], 12))[bc]
        sy = np.sign(np.round(lat.V[2], 12))[bc]
        ux_p, ux_m = upwind_derivative(lnM, 1, True), upwind_derivative(lnM, 1, False)
        uy_p, uy_m = upwind_derivative(lnM, 0, True), upwind_derivative(lnM, 0, False)
        gx = np.where(sx > 0, ux_p / prm.dx, np.where(sx < 0, ux_m / prm.dx, gx))
        gy = np.where(sy > 0, uy_p / prm.dx, np.where(sy < 0, uy_m / prm.dx, gy))
    elif prm.grad != "centred":
        raise ValueError(f"unknown gradient {prm.grad!r}")
    gv = gx * vx + gy * vy
    gu = gx * ux + gy * uy
    # d F_eq / d v^i = -(F_eq/T)(u^tau M^2 v^i / E_eq - M u^i), i = x, y
    # v . d_v F_eq  = -(F_eq/T)(u^tau M^2 |v|^2 / E_eq - M (u_perp . v_perp))
    v_dFeq = -(F_eq / T) * (ut * M ** 2 * sh2 / E_eq - M * uv)
    g_dFeq = -(F_eq / T) * (ut * M ** 2 * gv / E_eq - M * gu)
    Gr = (gv * v_dFeq + g_dFeq) / gam
    if lat.force == "weak3d":
        Gr = force3d.apply(lat.Gx, lat.Gy, F, gx, gy)

    # 9. R0
    R0 = A + Gr - C
    if prm.metric == METRIC_MILNE:
        R0 = R0 + S1 / tau

    # 10. mass evolution
    w = lat.w[bc]
    wF = np.sum(w * F, axis=0)
    num = np.sum(w * uV ** 2 * R0, axis=0)
    den = wF + beta * np.sum(w * uV ** 2 * (4 * F + S2), axis=0)
    X = -beta * num / den

    # 11. dF/dtau
    K = R0 + X * S2
    diag = dict(T=T, u=u, lam=lam, M_eq=M_eq, beta=beta, inv_tauR=inv_tauR, alpha=alpha)
    return K, X, diag


def _match_n(lat, eos, prm, F, lnM, u, lam):
    """Conserved particle number (eq. (sanity), second condition): with the
    Landau u, n = u_a N^a (N^a of eq. (NTdisc)), and T, alpha = mu/T from
    eps_kin_eq(T, mu) = lambda, n(T, mu) = n (eq. (epsp)).  Only for a
    constant mass: a mass depending on T alone is thermodynamically
    consistent (eq. (cdef)) at mu != 0 only if it is constant."""
    if np.any(eos.beta(np.array([0.2, 0.4])) != 0):
        raise ValueError("conserved particle number needs the constant-mass equation of state")
    _, Nk = lat.moments(F, lnM)
    n = u[0] * Nk[0] - u[1] * Nk[1] - u[2] * Nk[2]
    T, alpha = eos.T_alpha_from_eps_n(lam.ravel(), n.ravel(), prm.T_lo, prm.T_hi)
    return T.reshape(lam.shape), alpha.reshape(lam.shape)


def heun_step(lat, eos, prm, F, lnM, tau, dtau):
    """One predictor / trapezoid-corrector step (Sec. IV.D)."""
    K0, X0, _ = rhs(lat, eos, prm, F, lnM, tau)
    Fp = F + dtau * K0
    lp = lnM + dtau * X0
    K1, X1, _ = rhs(lat, eos, prm, Fp, lp, tau + dtau)
    return F + 0.5 * dtau * (K0 + K1), lnM + 0.5 * dtau * (X0 + X1)


def init_state(lat, eos, e0_GeVfm3, ux0=None, uy0=None, T_lo=0.05, T_hi=3.0, alpha0=0.0):
    """Local equilibrium initial state (reading of Sec. IV.D: the initial
    condition consists of the distribution plus T and M).

    T0 is the largest root of eps_EoS(T) = e0; M = M(T0); u^tau = sqrt(1 + u_perp^2);
    F = Z exp(-(u . P_n)/T0) with P_n = M V_n.  With a chemical potential
    mu0 = alpha0 T0 (constant mass, B = 0) eps = exp(alpha0) eps0(T0) = e0 and
    F carries the factor exp(alpha0).
    """
    e0 = np.asarray(e0_GeVfm3, dtype=float) * HBARC ** 3 * np.exp(-alpha0)
    sh = e0.shape
    T0 = eos.T_from_eps_largest(e0.ravel(), T_lo, T_hi).reshape(sh)
    M = eos.M(T0)
    ux = np.zeros(sh) if ux0 is None else np.asarray(ux0, dtype=float)
    uy = np.zeros(sh) if uy0 is None else np.asarray(uy0, dtype=float)
    ut = np.sqrt(1.0 + ux ** 2 + uy ** 2)
    bc = (slice(None), None, None)
    uP = M * (ut * lat.gamma[bc] - ux * lat.V[1][bc] - uy * lat.V[2][bc])
    F = eos.Z * np.exp(alpha0 - uP / T0)
    return F, np.log(M)


def observables(lat, eos, prm, F, lnM):
    """The 14 per-site output fields (GeV/fm^3, fm^-3, GeV, lab frame).

    T^{ab} = T^{ab}_kin + B(T) g^{ab} with g = diag(1, -1, -1, -1) in the
    Milne-orthonormal frame (eq. (emtnew)); N^a from eq. (NTdisc).
    Order: Ttt, Ttx, Tty, Txx, Txy, Tyy, TYY, Nt, Nx, Ny, T, ux, uy, M.
    """
    Tk, Nk = lat.moments(F, lnM)
    u, lam = landau(Tk[:3, :3])
    if prm.conserve_n:
        T, _ = _match_n(lat, eos, prm, F, lnM, u, lam)
    else:
        T = eos.T_from_eps_kin_eq(lam.ravel(), prm.T_lo, prm.T_hi).reshape(lam.shape)
    B = eos.B(T)
    c3 = HBARC ** 3
    out = np.stack([
        (Tk[0, 0] + B) / c3, Tk[0, 1] / c3, Tk[0, 2] / c3,
        (Tk[1, 1] - B) / c3, Tk[1, 2] / c3, (Tk[2, 2] - B) / c3, (Tk[3, 3] - B) / c3,
        Nk[0] / c3, Nk[1] / c3, Nk[2] / c3,
        T, u[1], u[2], np.exp(lnM),
    ])
    return out
