"""The paper's own 0+1-D lattice-Boltzmann algorithm for Milne spacetime
(paper Sec. IV.D, "Lattice Boltzmann Algorithm for Milne Spacetime").

TEST INFRASTRUCTURE ONLY (see the package docstring).

No space dependence, so U = (1, 0, 0, 0) and eps is the tau-tau component of
eq. (emtnew).  State: the distribution on the nodes, ln M and tau.  One step:

* temperature from the energy density through the EoS (Sec. IV.D, eq.
  (edchange)): the new T is the one at which eps(T) - B(T) equals the
  evolved eps_kin = T^{tau tau}_kin;
* f_eq = Z exp(-sqrt(M_eq^2 + M^2 sinh^2 xi)/T) with M_eq = M(T) and M the
  evolved mass (Sec. IV.D, last paragraph);
* d ln M / d tau = -(dB/deps) sum_n w_n cosh^2 xi_n [S1/tau - (f - f_eq)/tau_R]
  / sum_n w_n f_n;
* d f / d tau = S1/tau + (d ln M/d tau) S2 - (f - f_eq)/tau_R (eq. (newBeq));
* predictor (Euler) then trapezoid corrector (Heun).

Reading: the printed mass predictor has no cosh^2 xi_n in the numerator.
Eq. (edchange) together with eq. (masschange) gives
(M^4/2pi^2) d ln M/d tau sum w f = -dB/dtau = -(dB/deps) d eps/dtau with
d eps/dtau = (M^4/2pi^2) sum w cosh^2 xi [...], so the factor is restored here.
"""
from __future__ import annotations

import numpy as np

PI2 = np.pi ** 2


class Bjorken01:
    def __init__(self, lat, eos, eta_over_s, taur_rule="ce", T_lo=0.05, T_hi=3.0):
        self.lat, self.eos = lat, eos
        self.eta_over_s = float(eta_over_s)
        self.taur_rule = taur_rule
        self.T_lo, self.T_hi = T_lo, T_hi

    def init(self, T0):
        """Equilibrium at temperature T0 with M = M(T0)."""
        lat = self.lat
        M = float(self.eos.M(np.array([T0]))[0])
        f = self.eos.Z * np.exp(-M * lat.gamma / T0)
        return f, np.log(M)

    def temperature(self, f, lnM):
        lat = self.lat
        M = np.exp(lnM)
        eps_kin = M ** 4 / (2 * PI2) * np.sum(lat.w * f * lat.gamma ** 2)
        return float(self.eos.T_from_eps_kin_eq(np.array([eps_kin]), self.T_lo, self.T_hi)[0])

    def rates(self, f, lnM, tau):
        """(d f/d tau, d ln M/d tau) at the given state."""
        lat, eos = self.lat, self.eos
        M = np.exp(lnM)
        T = self.temperature(f, lnM)
        Ta = np.array([T])
        M_eq = float(eos.M(Ta)[0])
        if np.isinf(self.eta_over_s):
            inv_tauR = 0.0
        else:
            inv_tauR = 1.0 / float(eos.tau_R(Ta, self.eta_over_s, self.taur_rule)[0])
        dB = float(eos.dB(Ta)[0])
        deps = T * float(eos.ds(Ta)[0])
        dB_deps = dB / deps

        sh = np.sqrt(lat.gamma ** 2 - 1.0)
        f_eq = eos.Z * np.exp(-np.sqrt(M_eq ** 2 + M ** 2 * sh ** 2) / T)
        S1 = lat.apply_slices(lat.D1, f)
        S2 = lat.apply_slices(lat.D2, f)
        coll = (f - f_eq) * inv_tauR
        dlnM = -dB_deps * np.sum(lat.w * lat.gamma ** 2 * (S1 / tau - coll)) / np.sum(lat.w * f)
        df = S1 / tau + dlnM * S2 - coll
        return df, dlnM, T

    def step(self, f, lnM, tau, dtau):
        df0, dl0, _ = self.rates(f, lnM, tau)
        fp = f + dtau * df0
        lp = lnM + dtau * dl0
        df1, dl1, _ = self.rates(fp, lp, tau + dtau)
        return f + 0.5 * dtau * (df0 + df1), lnM + 0.5 * dtau * (dl0 + dl1)

    def energy_density(self, f, lnM):
        """Total eps = T^{tau tau}_kin + B(T), and P_L = T^{YY}_kin - B(T)."""
        lat = self.lat
        M = np.exp(lnM)
        G = M ** 4 / (2 * PI2)
        ek = G * np.sum(lat.w * f * lat.gamma ** 2)
        pl = G * np.sum(lat.w * f * lat.V[3] ** 2)
        T = self.temperature(f, lnM)
        B = float(self.eos.B(np.array([T]))[0])
        return ek + B, pl - B, T
