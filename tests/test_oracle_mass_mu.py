"""Pins of the quasiparticle mass at a chemical potential, M(T, mu) and
B(T, mu), built from the consistency condition eq. (cdef) (Sec. III) with
the mu = 0 construction of Sec. III.A as boundary values (oracle/eos.py,
reading 26 of the design notes).

The construction says: B(T, mu) exists only if -phi dM is a closed form
(phi = scalar density times M), which makes M and B constant along curves
d alpha / d ln T = -(2 + x K_0/K_1), x = M/T; each curve takes the mu = 0
values where it meets alpha = 0.  These tests check it against what the
paper fixes independently of that derivation:

* thermodynamic consistency, eq. (thermcons), at mu != 0 by central
  differences of p(T, mu) = p_kin - B: n = dp/dmu at fixed T, and
  eps + p = T dp/dT + mu n;
* the mu = 0 limit (M(T) and B(T) of Sec. III.A) and the constant-mass gas
  (M, B unchanged by mu);
* the scalar density int dchi f_eq (the weight of dM^2 in eq. (cdef)) by
  momentum quadrature, and dp_kin/dM = -phi, which ties eq. (cdef) to the
  densities of eq. (epsp);
* the constant-mass curves by integrating their ODE with a general-purpose
  integrator from alpha = 0 (a route independent of the quadrature and the
  root find that the oracle uses);
* planted mistakes in the curves' slope fail the consistency check.
"""
import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp
from scipy.special import kv

from oracle.eos import PI2, ConstMassEoS, TanhEntropyEoS

POINTS = [(0.2, 0.1), (0.3, 0.3), (0.25, -0.1), (0.45, 0.6), (0.19, 0.05)]  # (T, mu) in GeV


@pytest.fixture(scope="module")
def eos():
    return TanhEntropyEoS()


def _consistency(e, T, mu, h=1e-5):
    p, eps, n = e.thermo_mu(T, mu / T)
    pf = lambda T_, mu_: e.thermo_mu(T_, mu_ / T_)[0]
    dpdmu = (pf(T, mu + h) - pf(T, mu - h)) / (2 * h)
    dpdT = (pf(T + h, mu) - pf(T - h, mu)) / (2 * h)
    return (dpdmu - n) / n, (eps + p - T * dpdT - mu * dpdmu) / (eps + p)


@pytest.mark.parametrize("T,mu", POINTS)
def test_thermodynamic_consistency_at_a_chemical_potential(eos, T, mu):
    # central differences with h = 1e-5 GeV: truncation ~1e-10 relative
    rn, re = _consistency(eos, T, mu)
    assert abs(rn) < 1e-8, rn
    assert abs(re) < 1e-7, re


def test_mu_zero_limit_is_the_sec_IIIA_construction(eos):
    for T in (0.16, 0.2, 0.35, 0.8):
        assert eos.M_mu(T, 0.0) == float(eos.M(np.array(T)))
        assert eos.B_mu(T, 0.0) == float(eos.B(np.array(T)))
    # and continuity into mu = 0
    T = 0.3
    assert abs(eos.M_mu(T, 1e-7) - eos.M_mu(T, 0.0)) < 1e-6 * eos.M_mu(T, 0.0)


def test_constant_mass_gas_is_unchanged_by_mu():
    e = ConstMassEoS(Z=3.0, M0=0.4)
    for T, a in ((0.2, 0.5), (0.35, -0.8), (0.6, 1.5)):
        assert abs(e.M_mu(T, a) - 0.4) < 1e-14
        assert e.B_mu(T, a) == 0.0
        # and its consistency holds with B = 0
        rn, re = _consistency(e, T, a * T)
        assert abs(rn) < 1e-8 and abs(re) < 1e-7


def test_scalar_density_and_mass_derivative_of_the_pressure():
    # int dchi f_eq = int d^3p / ((2 pi)^3 E) Z exp(alpha) exp(-E/T)
    Z, M, T, a = 3.0, 0.55, 0.27, 0.4
    q, _ = quad(lambda k: k * k / np.sqrt(k * k + M * M) * np.exp(-np.sqrt(k * k + M * M) / T), 0, 60 * T,
                epsabs=0, epsrel=1e-13, limit=200)
    ns_quad = Z * np.exp(a) * q / (2 * PI2)
    ns_closed = Z * np.exp(a) * M * T * kv(1, M / T) / (2 * PI2)
    assert abs(ns_quad / ns_closed - 1) < 1e-11
    # d p_kin / dM = -phi = -M int dchi f_eq at fixed (T, mu)
    pk = lambda m: Z * np.exp(a) * m ** 2 * T ** 2 * kv(2, m / T) / (2 * PI2)
    h = 1e-6
    assert abs((pk(M + h) - pk(M - h)) / (2 * h) / (-M * ns_closed) - 1) < 1e-8


@pytest.mark.parametrize("T0,T", [(0.3, 0.22), (0.25, 0.33), (0.4, 0.2)])
def test_mass_is_constant_along_the_curves(eos, T0, T):
    M0 = float(eos.M(np.array(T0)))
    # d alpha / d ln t = -(2 + x K0/K1), x = M0/t, from alpha(ln T0) = 0
    rhs = lambda lt, y: [-(2.0 + (M0 / np.exp(lt)) * kv(0, M0 / np.exp(lt)) / kv(1, M0 / np.exp(lt)))]
    sol = solve_ivp(rhs, (np.log(T0), np.log(T)), [0.0], method="DOP853", rtol=1e-12, atol=1e-14)
    alpha = sol.y[0, -1]
    assert abs(eos.M_mu(T, alpha) / M0 - 1) < 1e-9
    assert abs(eos.B_mu(T, alpha) - float(eos.B(np.array(T0)))) < 1e-9 * abs(float(eos.B(np.array(T0)))) + 1e-15


class _PlantedKRatio(TanhEntropyEoS):
    # K_1/K_0 in place of K_0/K_1 in the curves' slope
    def char_integrand(self, x):
        return 2.0 + x * kv(1, x) / kv(0, x)


class _PlantedConstant(TanhEntropyEoS):
    # 1 in place of 2 (the d/dT of T in T K_1(M/T) dropped)
    def char_integrand(self, x):
        return 1.0 + x * kv(0, x) / kv(1, x)


@pytest.mark.parametrize("cls", [_PlantedKRatio, _PlantedConstant])
def test_planted_slope_mistakes_fail_consistency(cls):
    rn, _ = _consistency(cls(), 0.3, 0.3)
    assert abs(rn) > 1e-3, rn
