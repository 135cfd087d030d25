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
