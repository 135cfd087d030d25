"""Fluid-dynamics references for Bjorken (0+1-D Milne) flow (paper Sec. IV.A,
IV.E, eq. (hydroeq)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ideal:   d eps/d tau = -(eps + p)/tau
* first-order (Navier-Stokes) with the Chapman-Enskog eta and zeta of the
  BGK quasiparticle gas (Sec. IV.A):
           d eps/d tau = -(eps + p)/tau + (4 eta/3 + zeta)/tau^2

The state variable is T (eps(T) is monotone for a stable EoS); tau in fm,
so eta/(eps + p) etc. carry a factor hbar c.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad, solve_ivp

from .eos import HBARC


def zeta_over_tauR(eos, T):
    """zeta/tau_R = Z/(9T) int d^3p/(2pi)^3 p^2 [-M^2 + (1 - 3 c_s^2) E^2
    + 3 c_s^2 M T dM/dT] / E^2 exp(-E/T) at M = M(T) (Sec. IV.A), in GeV^4."""
    T = float(T)
    Ta = np.array([T])
    M = float(eos.M(Ta)[0])
    dM = float(eos.dM(Ta)[0])
    cs2 = float(eos.s(Ta)[0] / (T * eos.ds(Ta)[0]))

    def f(p):
        E2 = M * M + p * p
        return p ** 4 * (-M * M + (1 - 3 * cs2) * E2 + 3 * cs2 * M * T * dM) / E2 * np.exp(-np.sqrt(E2) / T)

    I, _ = quad(f, 0, 60 * T + 10 * M, epsabs=0, epsrel=1e-12, limit=400)
    return eos.Z / (9 * T) * I / (2 * np.pi ** 2)


def _dT_from_deps(eos, T, deps):
    return deps / (T * float(eos.ds(np.array([T]))[0]))


def ideal(eos, T0, tau0, taus):
    def f(tau, y):
        T = y[0]
        Ta = np.array([T])
        e, p = float(eos.eps(Ta)[0]), float(eos.p(Ta)[0])
        return [_dT_from_deps(eos, T, -(e + p) / tau)]

    sol = solve_ivp(f, (tau0, taus[-1]), [T0], t_eval=taus, rtol=1e-12, atol=1e-14, method="DOP853")
    return sol.y[0]


def navier_stokes(eos, T0, tau0, taus, eta_over_s, taur_rule="ce"):
    def f(tau, y):
        T = y[0]
        Ta = np.array([T])
        e, p, s = float(eos.eps(Ta)[0]), float(eos.p(Ta)[0]), float(eos.s(Ta)[0])
        eta = eta_over_s * s
        tauR = float(eos.tau_R(Ta, eta_over_s, taur_rule)[0]) / HBARC     # GeV^-1
        zeta = tauR * zeta_over_tauR(eos, T)
        # (4 eta/3 + zeta)/tau^2 with tau in fm: eta in GeV^3 -> GeV^4 fm via hbar c
        visc = (4 * eta / 3 + zeta) * HBARC / tau ** 2
        return [_dT_from_deps(eos, T, -(e + p) / tau + visc)]

    sol = solve_ivp(f, (tau0, taus[-1]), [T0], t_eval=taus, rtol=1e-10, atol=1e-13, method="DOP853")
    return sol.y[0]

