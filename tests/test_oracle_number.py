"""Pins of the conserved particle number (chemical potential mu != 0; paper
eq. (sanity) second condition, eq. (epsp), eq. (NTdisc)) in the oracle.

* Matching: a lattice equilibrium exp(alpha - (M/T) gamma) built at
  M/T = z0, where the lattice moments of the equilibrium are exact (Sec.
  IV.C), is matched back to its T and alpha = mu/T.
* Conservation: on a uniform grid in Milne coordinates the particle
  current obeys d(tau N^tau)/d tau = 0 with collisions; the n matching keeps
  it to the equilibrium quadrature error, matching energy alone (mu = 0
  equilibrium) violates it at O(1) in dtau/tau_R.
* Initial state: lb_init's reading with alpha0 reproduces e0 and
  n = exp(alpha0) n0(T0).
"""
import numpy as np
import pytest

from oracle import step as st
from oracle.eos import HBARC, ConstMassEoS, TanhEntropyEoS
from oracle.lattice import Lattice


@pytest.fixture(scope="module")
def lat():
    return Lattice(5, 5, 4, 1.0)


@pytest.fixture(scope="module")
def eos():
    return ConstMassEoS(Z=3.0, M0=0.4)


@pytest.mark.parametrize("alpha", [0.7, -1.2, 0.0])
def test_matching_recovers_T_and_mu(lat, eos, alpha):
    T = 0.4   # M/T = z0 = 1
    F = (eos.Z * np.exp(alpha) * np.exp(-(eos.M0 / T) * lat.gamma))[:, None, None]
    lnM = np.full((1, 1), np.log(eos.M0))
    Tk, Nk = lat.moments(F, lnM)
    u, lam = st.landau(Tk[:3, :3])
    n = u[0] * Nk[0] - u[1] * Nk[1] - u[2] * Nk[2]
    Tr, ar = eos.T_alpha_from_eps_n(lam.ravel(), n.ravel())
    assert abs(Tr[0] - T) < 1e-13 * T
    assert abs(ar[0] - alpha) < 1e-12


def test_density_and_energy_of_the_boltzmann_gas(eos):
    # n0 T = p (eq. (epsp): n = p/T for B = 0); eps/n between the
    # nonrelativistic and ultrarelativistic limits M + 3T/2 and 3T
    T = np.array([0.1, 0.3, 1.0, 3.0])
    assert np.allclose(eos.n_kin_eq(T) * T, eos.p(T), rtol=1e-13)
    r = eos.eps_kin_eq(T) / eos.n_kin_eq(T)
    assert np.all(r > 3 * T) and np.all(r > eos.M0 + 1.5 * T) and np.all(r < eos.M0 + 3 * T)


def _tau_N_drift(lat, eos, conserve):
    prm = st.Params(dx=0.2, eta_over_s=0.1, conserve_n=conserve)
    e0 = np.full((2, 2), float(eos.eps(0.35)) / HBARC ** 3)
    F, lnM = st.init_state(lat, eos, e0, alpha0=0.4)
    tau, dt = 0.5, 0.01
    _, N0 = lat.moments(F, lnM)
    q0 = tau * N0[0, 0, 0]
    for _ in range(100):
        F, lnM = st.heun_step(lat, eos, prm, F, lnM, tau, dt)
        tau += dt
    _, N1 = lat.moments(F, lnM)
    return (tau * N1[0, 0, 0] - q0) / q0


def test_particle_number_conservation(lat, eos):
    with_n = _tau_N_drift(lat, eos, True)
    without = _tau_N_drift(lat, eos, False)
    assert abs(with_n) < 3e-4
    assert abs(without) > 100 * abs(with_n)


def test_initial_state_with_chemical_potential(lat, eos):
    e0 = np.array([[2.0, 5.0]])
    F, lnM = st.init_state(lat, eos, e0, alpha0=0.5)
    prm = st.Params(dx=0.2, eta_over_s=0.1, conserve_n=True)
    obs = st.observables(lat, eos, prm, F, lnM)
    T = obs[10]
    # eps = e0 up to the lattice quadrature of the equilibrium (Sec. IV.C)
    assert np.allclose(obs[0], e0, rtol=5e-3)
    assert np.allclose(obs[7] * HBARC ** 3, np.exp(0.5) * eos.n_kin_eq(T), rtol=5e-3)


def test_requires_constant_mass(lat):
    prm = st.Params(dx=0.2, eta_over_s=0.1, conserve_n=True)
    eos = TanhEntropyEoS()
    e0 = np.full((1, 1), float(eos.eps(0.35)) / HBARC ** 3)
    F, lnM = st.init_state(lat, eos, e0)
    with pytest.raises(ValueError):
        st.heun_step(lat, eos, prm, F, lnM, 0.5, 0.01)


@pytest.mark.parametrize("alpha", [0.8, -0.5, 0.0])
def test_relaxation_time_at_chemical_potential(eos, alpha):
    # Chapman-Enskog relaxation time with a chemical potential (reading of
    # Sec. IV.A at mu != 0): eta = (eta/s) s(T, mu) and eta / tau_R = h(T, mu).
    # Pinned independently of the oracle's closed forms:
    #  * s(T, mu) as the finite-difference derivative dp/dT at fixed mu of
    #    the Boltzmann-gas pressure p = exp(mu/T) Z M^2 T^2 K_2(M/T)/(2 pi^2)
    #    (Sec. II.A, eq. (epsp));
    #  * h(T, mu) = (1/15T) int d^3p/(2pi)^3 p^4/E^2 f_eq with the fugacity
    #    in f_eq = Z exp(mu/T - E/T), by adaptive quadrature.
    from scipy.integrate import quad
    from scipy.special import kv
    eta_s = 0.12
    for T in (0.25, 0.4, 0.7):
        mu = alpha * T
        M, Z = eos.M0, eos.Z

        def p_at(TT):
            return np.exp(mu / TT) * Z * M ** 2 * TT ** 2 * kv(2, M / TT) / (2 * np.pi ** 2)

        h = 1e-4 * T
        s_fd = (-p_at(T + 2 * h) + 8 * p_at(T + h) - 8 * p_at(T - h) + p_at(T - 2 * h)) / (12 * h)
        integ = lambda q: q ** 6 / (M * M + q * q) * np.exp(mu / T - np.sqrt(M * M + q * q) / T)
        I, _ = quad(integ, 0.0, 80 * T + 10 * M, epsabs=0, epsrel=1e-13, limit=400)
        h_mu = Z * I / (2 * np.pi ** 2) / (15 * T)
        tau_R = float(eos.tau_R_mu(np.array([T]), np.array([alpha]), eta_s)[0])   # fm
        assert abs(tau_R * h_mu / (eta_s * s_fd * HBARC) - 1) < 1e-9, (T, alpha)
