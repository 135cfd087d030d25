"""Quasiparticle equation of state (paper Sec. III, III.A) and the BGK relaxation
time (Sec. IV.A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Units: GeV for T, M; GeV^4 for p, eps, B; GeV^3 for s.  hbar c converts to fm.

For a given pressure p(T) (zero chemical potential), the quasiparticle picture
of Sec. III.A fixes:

* s(T) = dp/dT and eps = T s - p (eq. (thermo) with mu = 0);
* M(T) from (eps + p)/T = Z M^3 K_3(M/T) / (2 pi^2) = s(T);
* B(T) from eq. (epsp): p = Z M^2 T^2 K_2(M/T)/(2 pi^2) - B.  Since s is
  matched exactly, B = p_kin - p solves the consistency ODE of eq. (cdef2)
  (dB/dT = -Z M^2 T K_1 M'/(2 pi^2)) and vanishes where p and p_kin do;
  this closed form is the reading of the "integrate up from small T" passage;
* the kinetic (Boltzmann-gas) part eps_kin = eps - B
  = Z M^2 T^2 [3 K_2 + (M/T) K_1] / (2 pi^2), which is what Landau matching of
  the kinetic T^{mu nu} returns (eq. (sanity) with T^{mu nu} of eq. (tmunufull)).

Readings (also in the design notes):
* Z for the synthetic QCD-like EoS is kappa * g pi^4 / 90.  With kappa = 1
  (the high-T limit the paper uses to fix Z) the entropy of the synthetic EoS
  exceeds the largest quasiparticle entropy Z M^3 K_3/(2 pi^2) <= 4 Z T^3/pi^2
  near T = 0.17 GeV and M(T) has no solution; kappa = 2 restores one.
* tau_R(T) makes the Chapman-Enskog shear viscosity of Sec. IV.A equal
  (eta/s) s(T): tau_R = (eta/s) s / h(T), with
  h = eta / tau_R = Z/(15 T) int d^3p/(2pi)^3 p^4/E^2 exp(-E/T) at M = M(T).
  The alternative rule tau_R = 5 (eta/s)/T is the massless limit
  eta = tau_R (eps + P)/5 of the same section.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad_vec
from scipy.optimize import elementwise
from scipy.special import kv

HBARC = 0.1973269804  # GeV fm
PI2 = np.pi ** 2

_TOL = dict(xatol=0.0, xrtol=4 * np.finfo(float).eps, fatol=0.0, frtol=0.0)


def _root(f, lo, hi, args=()):
    res = elementwise.find_root(f, (lo, hi), args=args, tolerances=_TOL)
    if not np.all(res.success):
        bad = np.flatnonzero(~np.atleast_1d(res.success))
        raise ValueError(f"root not bracketed/converged at {bad.size} points")
    return res.x


def _h_integral(z):
    """int_0^inf sinh^6(xi)/cosh(xi) exp(-z cosh xi) dxi for an array of z > 0.

    This is the xi form of int p^6 / E^2 exp(-E/T) dp with p = M sinh xi.
    The integrand is below 1e-160 of its size beyond z cosh xi = 400 + 6 ln(...)
    so a finite upper limit is exact to double precision.
    """
    z = np.atleast_1d(np.asarray(z, dtype=float))
    xi_max = np.arccosh(np.maximum(420.0 / z.min(), 2.0)) + 2.0

    def f(t):
        ch = np.cosh(t)
        return np.sinh(t) ** 6 / ch * np.exp(-z * ch)

    val, _ = quad_vec(f, 0.0, xi_max, epsabs=0.0, epsrel=1e-14, limit=400)
    return val


class QuasiparticleEoS:
    """Base class: everything below follows from p(T), s(T), s'(T) and Z."""

    Z: float

    # ---- the input equation of state (to be provided by subclasses) ----
    def p(self, T):
        raise NotImplementedError

    def s(self, T):
        raise NotImplementedError

    def ds(self, T):
        raise NotImplementedError

    # ---- thermodynamics (eq. (thermo), mu = 0) ----
    def eps(self, T):
        T = np.asarray(T, dtype=float)
        return T * self.s(T) - self.p(T)

    # ---- quasiparticle mass (Sec. III.A) ----
    def z_of_T(self, T):
        """z = M/T solving z^3 K_3(z) = 2 pi^2 s(T) / (Z T^3)."""
        T = np.atleast_1d(np.asarray(T, dtype=float))
        target = 2 * PI2 * self.s(T) / (self.Z * T ** 3)
        if np.any(target >= 8.0) or np.any(target <= 0.0):
            raise ValueError("entropy outside the quasiparticle range: no M(T)")
        f = lambda zz, c: zz ** 3 * kv(3, zz) - c
        return _root(f, np.full_like(T, 1e-8), np.full_like(T, 800.0), args=(target,))

    def M(self, T):
        T = np.asarray(T, dtype=float)
        return self.z_of_T(T).reshape(T.shape) * T

    def p_kin(self, T):
        T = np.asarray(T, dtype=float)
        z = self.z_of_T(T).reshape(T.shape)
        return self.Z * z ** 2 * T ** 4 * kv(2, z) / (2 * PI2)

    def B(self, T):
        """Bag function of eq. (tmunufull): B = p_kin - p (eq. (epsp))."""
        return self.p_kin(T) - self.p(T)

    def eps_kin_eq(self, T):
        """eps - B = Z M^2 T^2 [3 K_2(z) + z K_1(z)] / (2 pi^2) (eq. (epsp))."""
        T = np.asarray(T, dtype=float)
        z = self.z_of_T(T).reshape(T.shape)
        return self.Z * z ** 2 * T ** 4 * (3 * kv(2, z) + z * kv(1, z)) / (2 * PI2)

    def dM(self, T):
        """dM/dT from differentiating Z M^3 K_3(M/T) / (2 pi^2) = s(T) in T.

        Using K_3'(z) = -K_2(z) - 3 K_3(z)/z the derivative of the left side
        is Z/(2 pi^2) [-M^3 K_2 M'/T + M^4 K_2/T^2 + 3 M^3 K_3/T]; equating to
        s'(T) and solving for M' gives
        M' = M/T + 3 K_3/K_2 - 2 pi^2 s' T / (Z M^3 K_2).
        """
        T = np.asarray(T, dtype=float)
        z = self.z_of_T(T).reshape(T.shape)
        M = z * T
        return z + 3 * kv(3, z) / kv(2, z) - 2 * PI2 * self.ds(T) * T / (self.Z * M ** 3 * kv(2, z))

    def dB(self, T):
        """dB/dT = -Z M^2 T K_1(M/T) dM/dT / (2 pi^2), eq. (cdef2)."""
        T = np.asarray(T, dtype=float)
        z = self.z_of_T(T).reshape(T.shape)
        M = z * T
        return -self.Z * M ** 2 * T * kv(1, z) * self.dM(T) / (2 * PI2)

    def beta(self, T):
        """beta = B'/(eps' - B') = dB/d(eps_kin_eq), with eps' = T s'.

        beta/(1 + beta) = B'/eps' = dB/deps is the factor of the paper's mass
        predictor (Sec. IV.D); beta itself is what appears once the
        temperature is fixed by the kinetic energy density eps - B.
        """
        T = np.asarray(T, dtype=float)
        dB = self.dB(T)
        return dB / (T * self.ds(T) - dB)

    # ---- transport (Sec. IV.A) ----
    def h(self, T):
        """eta / tau_R = Z/(15 T) int d^3p/(2 pi)^3 p^4/E^2 exp(-E/T), at M = M(T).

        With p = M sinh(xi): = Z M^5 / (30 pi^2 T) int sinh^6/cosh exp(-z cosh) dxi.
        """
        T = np.atleast_1d(np.asarray(T, dtype=float))
        z = self.z_of_T(T)
        M = z * T
        return self.Z * M ** 5 / (30 * PI2 * T) * _h_integral(z)

    def tau_R(self, T, eta_over_s, rule="ce"):
        """BGK relaxation time in fm/c (eq. (bgk)); rule 'ce' or 'massless'."""
        T = np.atleast_1d(np.asarray(T, dtype=float))
        if rule == "massless":
            return 5.0 * eta_over_s / T * HBARC
        return eta_over_s * self.s(T) / self.h(T) * HBARC

    # ---- conserved particle number (eqs. (epsp), (sanity) with mu != 0) ----
    def n_kin_eq(self, T):
        """Particle density at mu = 0, n0 = Z M^2 T K_2(z) / (2 pi^2) (eq. (epsp)).
        At chemical potential mu the Boltzmann factor exp(mu/T) multiplies
        n, eps - B and p + B alike."""
        T = np.asarray(T, dtype=float)
        z = self.z_of_T(T).reshape(T.shape)
        return self.Z * z ** 2 * T ** 3 * kv(2, z) / (2 * PI2)

    def T_alpha_from_eps_n(self, e, n, T_lo=0.05, T_hi=3.0):
        """(T, alpha = mu/T) with eps_kin_eq = e and n = n_kin (eq. (sanity)).

        The fugacity exp(alpha) cancels in the ratio eps_kin_eq / n =
        eps0(T) / n0(T) (= 3 T + M K_1/K_2 for a constant mass, increasing in
        T), so T is its root and alpha = ln(n / n0(T))."""
        e = np.atleast_1d(np.asarray(e, dtype=float))
        n = np.atleast_1d(np.asarray(n, dtype=float))
        if np.any(n <= 0) or np.any(e <= 0):
            raise FloatingPointError("non-positive energy or particle density")
        f = lambda T, r: self.eps_kin_eq(T) / self.n_kin_eq(T) - r
        T = _root(f, np.full_like(e, T_lo), np.full_like(e, T_hi), args=(e / n,))
        return T, np.log(n / self.n_kin_eq(T))

    def tau_R_mu(self, T, alpha, eta_over_s, rule="ce"):
        """tau_R at chemical potential mu = alpha T in fm/c.  CE rule:
        eta = (eta/s) s(T, mu), eta/tau_R = h(T, mu); for the Boltzmann gas
        s(T, mu) = exp(alpha) (s0 - alpha n0) (s = dp/dT at fixed mu with
        p = exp(mu/T) p0(T), p0 = n0 T) and h(T, mu) = exp(alpha) h0(T)."""
        T = np.atleast_1d(np.asarray(T, dtype=float))
        alpha = np.atleast_1d(np.asarray(alpha, dtype=float))
        if rule == "massless":
            return 5.0 * eta_over_s / T * HBARC
        s_mu = self.s(T) - alpha * self.n_kin_eq(T)
        if np.any(s_mu <= 0):
            raise FloatingPointError("non-positive entropy density at this chemical potential")
        return eta_over_s * s_mu / self.h(T) * HBARC

    # ---- a mass depending on T and mu (eq. (cdef) at mu != 0, reading 26) ----
    #
    # Consistency, eq. (cdef), asks dB = -(1/2) int dchi f_eq dM^2 = -phi dM
    # with phi(T, mu, M) = Z exp(mu/T) M^2 T K_1(M/T) / (2 pi^2) (the scalar
    # density times M).  B(T, mu) exists only if this form is closed,
    # d(phi dM) = 0, i.e. phi_T M_mu = phi_mu M_T with the partial derivatives
    # of phi at fixed M: M is constant along the curves
    # dmu/dT = -phi_T/phi_mu, and then so is B (dB = -phi dM = 0 there).
    # With phi_mu = phi/T and phi_T = Z M^2 exp(mu/T) [(2 - mu/T) K_1 + x K_0]
    # / (2 pi^2) (x = M/T; d[T K_1(M/T)]/dT = 2 K_1 + x K_0), the curve in
    # alpha = mu/T is  d alpha / d ln T = -(2 + x K_0(x)/K_1(x)).  Each such
    # curve meets alpha = 0 at one temperature T0, where the mass and B are
    # those of the mu = 0 construction:
    #   M(T, mu) = M(T0),  B(T, mu) = B(T0),
    #   alpha = int_{ln T}^{ln T0} [2 + x K_0(x)/K_1(x)] d ln t,  x = M(T0)/t.
    def char_integrand(self, x):
        """2 + x K_0(x)/K_1(x): minus d alpha / d ln T at fixed M."""
        return 2.0 + x * kv(0, x) / kv(1, x)

    def alpha_on_char(self, T, T0, M):
        """alpha at T on the curve of constant mass M through (T0, alpha = 0)."""
        a, b = np.log(T), np.log(T0)
        f = lambda t: self.char_integrand(M / np.exp(t))
        from scipy.integrate import quad
        v, _ = quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=200)
        return v

    def T0_of_T_alpha(self, T, alpha):
        """The foot T0 of the constant-mass curve through (T, alpha).

        The integrand is at least 2, so |alpha| >= 2 |ln(T0/T)|: T0 lies
        between T and T exp(alpha/2), where the residual changes sign."""
        from scipy.optimize import brentq
        T, alpha = float(T), float(alpha)
        if alpha == 0.0:
            return T
        g = lambda T0: self.alpha_on_char(T, T0, float(self.M(np.array(T0)))) - alpha
        lo, hi = sorted((T, T * np.exp(alpha / 2.0)))
        return brentq(g, lo, hi, xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=200)

    def M_mu(self, T, alpha):
        """M(T, mu) at mu = alpha T."""
        return float(self.M(np.array(self.T0_of_T_alpha(T, alpha))))

    def B_mu(self, T, alpha):
        """B(T, mu) at mu = alpha T."""
        return float(self.B(np.array(self.T0_of_T_alpha(T, alpha))))

    def thermo_mu(self, T, alpha):
        """(p, eps, n) at (T, mu = alpha T) with M(T, mu) and B(T, mu), eq. (epsp)."""
        M = self.M_mu(T, alpha)
        B = self.B_mu(T, alpha)
        x = M / T
        c = self.Z * np.exp(alpha) * M ** 2 * T / (2 * PI2)
        p = c * T * kv(2, x) - B
        eps = c * T * (3 * kv(2, x) + x * kv(1, x)) + B
        n = c * kv(2, x)
        return p, eps, n

    # ---- inversions used by the lattice-Boltzmann step ----
    def T_from_eps_kin_eq(self, e, T_lo=0.05, T_hi=3.0):
        """Unique T with eps_kin_eq(T) = e (monotone in T), on [T_lo, T_hi]."""
        e = np.atleast_1d(np.asarray(e, dtype=float))
        f = lambda T, ee: self.eps_kin_eq(T) - ee
        return _root(f, np.full_like(e, T_lo), np.full_like(e, T_hi), args=(e,))

    def T_from_eps_largest(self, e, T_lo=0.05, T_hi=3.0, n_scan=6000):
        """Largest T in [T_lo, T_hi] with eps(T) = e.

        eps(T) of an EoS with an unstable band is not monotone; the largest
        root is the one on the upper branch.  A scan from the top of a fine
        grid brackets it, then a bracketing root finder refines it.
        """
        e = np.atleast_1d(np.asarray(e, dtype=float))
        grid = np.linspace(T_lo, T_hi, n_scan)
        eg = self.eps(grid)
        if np.any(e > eg[-1]) or np.any(e < eg.min()):
            raise ValueError("energy density outside the EoS table range")
        above = eg[None, :] > e[:, None]
        # largest index i with eps(grid[i]) <= e; the bracket is [grid[i], grid[i+1]]
        idx = np.where(~above, np.arange(n_scan)[None, :], -1).max(axis=1)
        idx = np.clip(idx, 0, n_scan - 2)
        f = lambda T, ee: self.eps(T) - ee
        return _root(f, grid[idx], grid[idx + 1], args=(e,))


class TanhEoS(QuasiparticleEoS):
    """Synthetic QCD-like EoS p/T^4 = (pi^2/90) g (1 + tanh((T - Tc)/w)) / 2.

    Degeneracy Z = kappa g pi^4/90 (for g = 37 this is kappa times the
    Z = (pi^4/180)(4 (Nc^2 - 1) + 7 Nc Nf) of Sec. III.A at Nc = 3, Nf = 2).
    """

    def __init__(self, g=37.0, Tc=0.17, width=0.02, kappa=2.0):
        self.g, self.Tc, self.width, self.kappa = float(g), float(Tc), float(width), float(kappa)
        self.Z = self.kappa * self.g * np.pi ** 4 / 90.0
        self.c = PI2 / 90.0 * self.g

    def _h(self, T):
        y = (T - self.Tc) / self.width
        th = np.tanh(y)
        h0 = 0.5 * (1 + th)
        sech2 = 1 - th * th
        h1 = 0.5 * sech2 / self.width
        h2 = -sech2 * th / self.width ** 2
        return h0, h1, h2

    def p(self, T):
        T = np.asarray(T, dtype=float)
        h0, _, _ = self._h(T)
        return self.c * T ** 4 * h0

    def s(self, T):
        T = np.asarray(T, dtype=float)
        h0, h1, _ = self._h(T)
        return self.c * (4 * T ** 3 * h0 + T ** 4 * h1)

    def ds(self, T):
        T = np.asarray(T, dtype=float)
        h0, h1, h2 = self._h(T)
        return self.c * (12 * T ** 2 * h0 + 8 * T ** 3 * h1 + T ** 4 * h2)


class TanhEntropyEoS(QuasiparticleEoS):
    """Synthetic QCD-like crossover on the entropy density:
    s/T^3 = (2 pi^2/45) g (1 + tanh((T - Tc)/w)) / 2, p(T) = int_0^T s dT'.

    The paper's quasiparticle construction takes s(T) as its input
    (Sec. III.A: (eps + p)/T = Z M^3 K_3/(2 pi^2) = s).  With the crossover
    on s/T^3 the speed of sound c_s^2 = s/(T s') = h/(3 h + T h') lies in
    (0, 1/3] for every width, as for QCD; a tanh on p/T^4 instead has
    c_s^2 > 1/3 above Tc (and d eps/dT < 0 for w = 0.02), where the
    Chapman-Enskog bulk viscosity of Sec. IV.A is negative.
    """

    def __init__(self, g=37.0, Tc=0.17, width=0.02, kappa=2.0):
        self.g, self.Tc, self.width, self.kappa = float(g), float(Tc), float(width), float(kappa)
        self.Z = self.kappa * self.g * np.pi ** 4 / 90.0
        self.cs = 4 * PI2 / 90.0 * self.g

    def _h(self, T):
        th = np.tanh((T - self.Tc) / self.width)
        return 0.5 * (1 + th), 0.5 * (1 - th * th) / self.width

    def s(self, T):
        T = np.asarray(T, dtype=float)
        return self.cs * T ** 3 * self._h(T)[0]

    def ds(self, T):
        T = np.asarray(T, dtype=float)
        h0, h1 = self._h(T)
        return self.cs * (3 * T ** 2 * h0 + T ** 3 * h1)

    def p(self, T):
        """p = int_0^T s dT' = cs T^4 int_0^1 t^3 h(t T) dt (adaptive quadrature)."""
        T = np.asarray(T, dtype=float)
        Tf = np.atleast_1d(T).ravel()
        f = lambda t: t ** 3 * self._h(t * Tf)[0]
        v, _ = quad_vec(f, 0.0, 1.0, epsabs=0.0, epsrel=1e-14, limit=4000)
        return (self.cs * Tf ** 4 * v).reshape(T.shape)


class TabulatedEoS(QuasiparticleEoS):
    """The caller's entropy density s(T_i) as the input of the quasiparticle
    construction (Sec. III.A builds M(T) and B(T) from s(T) and p(T)).

    Between the points s(T) = T^3 exp(y(ln T)), y the cubic spline with
    not-a-knot ends (scipy's CubicSpline, extended by its end cubics) of
    ln(s_i/T_i^3) against ln T_i; ds/dT follows from the same cubic; p(T) =
    p0 + int_{T_0}^T s dT' (adaptive quadrature in ln T).  The spline is
    twice continuously differentiable, so beta and c_s^2, which involve s',
    are continuous.
    """

    def __init__(self, T, s, p0, Z):
        from scipy.interpolate import CubicSpline
        T = np.asarray(T, dtype=float)
        s = np.asarray(s, dtype=float)
        self.T0, self.p0, self.Z = float(T[0]), float(p0), float(Z)
        self._y = CubicSpline(np.log(T), np.log(s / T ** 3), bc_type="not-a-knot", extrapolate=True)
        self._dy = self._y.derivative()

    def s(self, T):
        T = np.asarray(T, dtype=float)
        return T ** 3 * np.exp(self._y(np.log(T)))

    def ds(self, T):
        T = np.asarray(T, dtype=float)
        x = np.log(T)
        return T ** 2 * np.exp(self._y(x)) * (3.0 + self._dy(x))

    def p(self, T):
        T = np.asarray(T, dtype=float)
        b = np.log(np.atleast_1d(T).ravel())
        a = np.log(self.T0)
        # int_{T0}^{T} s dT' = int_a^b exp(4 x + y(x)) dx, x = a + t (b - a),
        # each component divided by T s(T) (~ its size) so that the common
        # error control of the vector quadrature is relative per component
        scale = np.exp(b) * self.s(np.exp(b))
        f = lambda t: (b - a) * np.exp(4.0 * (a + t * (b - a)) + self._y(a + t * (b - a))) / scale
        v, _ = quad_vec(f, 0.0, 1.0, epsabs=0.0, epsrel=1e-14, limit=4000)
        return (self.p0 + v * scale).reshape(T.shape)


class ConstMassEoS(QuasiparticleEoS):
    """Boltzmann gas of constant mass M0 (Sec. II.A): B = 0, M(T) = M0."""

    def __init__(self, Z, M0):
        self.Z, self.M0 = float(Z), float(M0)

    def p(self, T):
        T = np.asarray(T, dtype=float)
        z = self.M0 / T
        return self.Z * self.M0 ** 2 * T ** 2 * kv(2, z) / (2 * PI2)

    def s(self, T):
        T = np.asarray(T, dtype=float)
        z = self.M0 / T
        return self.Z * self.M0 ** 3 * kv(3, z) / (2 * PI2)

    def ds(self, T):
        # d/dT [Z M^3 K_3(M/T)/(2 pi^2)] = Z M^3/(2 pi^2) K_3'(z) (-M/T^2)
        T = np.asarray(T, dtype=float)
        z = self.M0 / T
        k3p = -kv(2, z) - 3 * kv(3, z) / z
        return -self.Z * self.M0 ** 3 * k3p * self.M0 / (2 * PI2 * T ** 2)

    def z_of_T(self, T):
        T = np.atleast_1d(np.asarray(T, dtype=float))
        return self.M0 / T

    def B(self, T):
        return np.zeros_like(np.asarray(T, dtype=float))

    def dM(self, T):
        return np.zeros_like(np.asarray(T, dtype=float))

    def beta(self, T):
        return np.zeros_like(np.asarray(T, dtype=float))
