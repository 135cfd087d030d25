"""Sound waves in the transverse plane (pin of the 2+1-D terms: streaming,
mass-gradient force, collisions, against the hydrodynamic limit).

A small standing density wave on a periodic line at T0 = 0.35 GeV (where
the synthetic EoS is conformal, c_s^2 = 1/3, and M/T = 2.60), Minkowski
metric, eta/s = 0.02: the first zero crossing of the wave's amplitude comes
a quarter period after the start, t = L / (4 c_s) up to O(Gamma/omega)
(Gamma/omega < 0.02 here).  The lattice's reference z0 is the fluid's M/T,
so that its equilibrium moments are exact (Sec. IV.C); the sound speed of
the scheme is then that of the EoS.  Without the mass-gradient force of
eq. (Bmilne) the momentum balance lacks the gradient of the bag pressure
and the wave does not propagate at c_s.
"""
import numpy as np

from oracle import step as st
from oracle.eos import HBARC, TanhEntropyEoS
from oracle.lattice import Lattice

T0 = 0.35


def _quarter_period_speed(lat, eos, nx=32, dx=0.2, dt=0.04, eta=0.02):
    """L / (4 t0) with t0 the first zero crossing of the cos mode of T^{tt},
    or None if there is none within 1.3 times the EoS quarter period."""
    L = nx * dx
    xs = (np.arange(nx) + 0.5) * dx
    c = np.cos(2 * np.pi * xs / L)
    e_bg = float(eos.eps(T0)) / HBARC ** 3
    F, lnM = st.init_state(lat, eos, (e_bg * (1 + 0.01 * c))[None, :])
    prm = st.Params(dx=dx, eta_over_s=eta, metric=st.METRIC_MINKOWSKI)
    cs = np.sqrt(eos.s(np.array([T0]))[0] / (T0 * eos.ds(np.array([T0]))[0]))
    amp = []
    for _ in range(int(round(1.3 * L / (4 * cs) / dt))):
        Tk, _ = lat.moments(F, lnM)
        amp.append(np.sum(Tk[0, 0, 0] * c) / np.sum(c * c))
        F, lnM = st.heun_step(lat, eos, prm, F, lnM, 1.0, dt)
    amp = np.array(amp)
    k = np.where((amp[:-1] > 0) & (amp[1:] <= 0))[0]
    if k.size == 0:
        return cs, None
    k = k[0]
    t0 = (k + amp[k] / (amp[k] - amp[k + 1])) * dt
    return cs, L / (4 * t0)


def test_sound_speed_of_the_eos():
    eos = TanhEntropyEoS()
    z = float(eos.z_of_T(np.array([T0]))[0])
    assert abs(eos.s(np.array([T0]))[0] / (T0 * eos.ds(np.array([T0]))[0]) - 1 / 3) < 1e-6
    cs, c_lb = _quarter_period_speed(Lattice(5, 5, 4, z), eos)
    assert c_lb is not None and abs(c_lb / cs - 1) < 0.015


def test_sound_needs_the_mass_gradient_force():
    # planted in the oracle: the weak-form 3-D force with its operators zeroed
    eos = TanhEntropyEoS()
    z = float(eos.z_of_T(np.array([T0]))[0])
    lat = Lattice(5, 5, 4, z, force="weak3d")
    lat.Gx, lat.Gy = 0 * lat.Gx, 0 * lat.Gy
    cs, c_lb = _quarter_period_speed(lat, eos)
    assert c_lb is None or abs(c_lb / cs - 1) > 0.05


def test_sound_damping_rate_of_first_order_hydrodynamics():
    # P16, damping: a standing wave in a homogeneous fluid decays as
    # exp(-Gamma t) with Gamma = (4 eta/3 + zeta) k^2 / (2 (eps + p)) (eta =
    # (eta/s) s, zeta of Sec. IV.A; both from the Chapman-Enskog forms the
    # oracle's relaxation time is built on).  48 sites per wavelength
    # (dx 0.2 fm, L 9.6 fm), eta/s 0.06 (k tau_R = 0.14), one period;
    # a fit of a exp(-G t) cos(w t + ph) to the cos mode of T^{tt}.
    # Measured: G/Gamma = 1.017, w/(c_s k) = 1.003 (with 32 sites per
    # wavelength the upwind streaming adds 6% to G).
    from scipy.optimize import curve_fit
    from oracle import hydro
    eos = TanhEntropyEoS()
    z = float(eos.z_of_T(np.array([T0]))[0])
    lat = Lattice(5, 5, 4, z)
    nx, dx, dt, eta = 48, 0.2, 0.04, 0.06
    L = nx * dx
    xs = (np.arange(nx) + 0.5) * dx
    c = np.cos(2 * np.pi * xs / L)
    e_bg = float(eos.eps(T0)) / HBARC ** 3
    F, lnM = st.init_state(lat, eos, (e_bg * (1 + 0.01 * c))[None, :])
    prm = st.Params(dx=dx, eta_over_s=eta, metric=st.METRIC_MINKOWSKI)
    Ta = np.array([T0])
    e, p, s = (float(f(Ta)[0]) for f in (eos.eps, eos.p, eos.s))
    cs = np.sqrt(s / (T0 * eos.ds(Ta)[0]))
    k = 2 * np.pi / L
    tauR = float(eos.tau_R(Ta, eta)[0]) / HBARC          # GeV^-1
    zeta = tauR * hydro.zeta_over_tauR(eos, T0)
    Gamma = (4 * eta * s / 3 + zeta) * HBARC * k ** 2 / (2 * (e + p))   # fm^-1
    n = int(round(2 * np.pi / (cs * k) / dt))
    amp = []
    for _ in range(n + 1):
        Tk, _ = lat.moments(F, lnM)
        amp.append(np.sum((Tk[0, 0, 0] - np.mean(Tk[0, 0, 0])) * c) / np.sum(c * c))
        F, lnM = st.heun_step(lat, eos, prm, F, lnM, 1.0, dt)
    t = np.arange(n + 1) * dt
    fit = lambda t, a, G, w, ph: a * np.exp(-G * t) * np.cos(w * t + ph)
    (a, G, w, ph), _ = curve_fit(fit, t, np.array(amp), p0=[amp[0], Gamma, cs * k, 0.0])
    assert abs(G / Gamma - 1) < 0.04, G / Gamma
    assert abs(w / (cs * k) - 1) < 0.01, w / (cs * k)
