"""Pins of the oracle's quasiparticle EoS (paper Sec. II.A, III, III.A, IV.A)
against thermodynamics, the paper's closed forms and numerical derivatives."""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import kv

from oracle import hydro
from oracle.eos import HBARC, ConstMassEoS, TanhEntropyEoS, TanhEoS

T = np.array([0.08, 0.12, 0.16, 0.17, 0.19, 0.22, 0.3, 0.5, 1.0, 2.0])


def _fd(f, x, h):
    return (f(x + h) - f(x - h)) / (2 * h)


@pytest.fixture(scope="module", params=["entropy", "pressure"])
def eos(request):
    # crossover on s/T^3 (the workloads' EoS) and on p/T^4 (the printed form,
    # at the smallest width with d eps/dT > 0 and c_s^2 <= 1)
    return TanhEntropyEoS() if request.param == "entropy" else TanhEoS(width=0.03)


def test_entropy_and_its_derivative_are_derivatives_of_p(eos):
    # eq. (thermo) at mu = 0: s = dp/dT; the analytic s' is d s/dT
    h = 1e-6
    assert np.allclose(eos.s(T), _fd(eos.p, T, h), rtol=1e-7)
    assert np.allclose(eos.ds(T), _fd(eos.s, T, h), rtol=1e-6)


def test_bag_function_solves_consistency_ode(eos):
    # eq. (cdef2): dB/dT = -Z M^2 T K_1(M/T) M'(T)/(2 pi^2); B = p_kin - p
    h = 1e-6
    num = _fd(eos.B, T, h)
    ana = eos.dB(T)
    assert np.allclose(ana, num, rtol=2e-6, atol=1e-12)
    # the paper integrates up from small T where B ~ 0: |B| is below 1e-3 of
    # the Stefan-Boltzmann pressure of the same degrees of freedom there
    Tl = np.array([0.05, 0.06, 0.08, 0.1])
    p_sb = np.pi ** 2 / 90 * eos.g * Tl ** 4
    assert np.all(np.abs(eos.B(Tl)) < 1e-3 * p_sb)
    # M' from implicit differentiation against a numerical derivative of M(T)
    assert np.allclose(eos.dM(T), _fd(eos.M, T, h), rtol=1e-6)


def test_kinetic_energy_plus_bag_is_eos_energy(eos):
    # eq. (epsp): eps = Z M^2 T^2 [3 K2 + (M/T) K1]/(2 pi^2) + B, p = p_kin - B
    assert np.allclose(eos.eps_kin_eq(T) + eos.B(T), eos.eps(T), rtol=1e-12)
    # and the kinetic entropy Z M^3 K_3/(2 pi^2) is the input s(T) (Sec. III.A)
    M = eos.M(T)
    s_qp = eos.Z * M ** 3 * kv(3, M / T) / (2 * np.pi ** 2)
    assert np.allclose(s_qp, eos.s(T), rtol=1e-12)


def test_beta_is_dB_deps_kin(eos):
    # beta = dB/d(eps - B); beta/(1+beta) = dB/deps (mass predictor of Sec. IV.D)
    h = 1e-6
    dB = _fd(eos.B, T, h)
    deps = _fd(eos.eps, T, h)
    assert np.allclose(eos.beta(T) / (1 + eos.beta(T)), dB / deps, rtol=1e-5, atol=1e-9)


def test_high_temperature_mass_limit():
    # s -> 4 g pi^2 T^3/90 = (Z/kappa) 4 T^3/pi^2, so z^3 K_3(z) -> 8/kappa
    e = TanhEoS(width=0.03, kappa=2.0)
    z = e.z_of_T(np.array([3.0]))[0]
    assert abs(z ** 3 * kv(3, z) - 4.0) < 1e-10


def test_config_eos_is_unstable_and_stable_reading_is_not():
    # The width-0.02 EoS has d eps/dT < 0 on a band near 0.19 GeV (c_s^2 < 0);
    # the width-0.03 reading is stable and causal on [0.05, 3] GeV.
    Tg = np.linspace(0.05, 3.0, 60001)
    e02, e03 = TanhEoS(width=0.02), TanhEoS(width=0.03)
    d02 = Tg * e02.ds(Tg)
    assert np.any(d02 < 0)
    band = Tg[d02 < 0]
    assert 0.184 < band.min() < 0.185 and 0.196 < band.max() < 0.197
    cs2 = e03.s(Tg) / (Tg * e03.ds(Tg))
    assert np.all(cs2 > 0) and np.all(cs2 <= 1.0)
    # the matched quantity eps - B stays monotone for both
    for e in (e02, e03):
        assert np.all(np.diff(e.eps_kin_eq(Tg[::20])) > 0)


def test_constant_mass_gas_sound_speed_and_bessel_forms():
    # Sec. II.A: c_s^2 = (3 + (m/T) K2/K3)^-1 and n = p/T for a constant mass
    e = ConstMassEoS(Z=3.0, M0=0.5)
    h = 1e-6
    cs2 = _fd(e.p, T, h) / _fd(e.eps, T, h)
    z = 0.5 / T
    assert np.allclose(cs2, 1.0 / (3 + z * kv(2, z) / kv(3, z)), rtol=1e-7)
    eps_ref = 3.0 * 0.25 * T * (3 * T * kv(2, z) + 0.5 * kv(1, z)) / (2 * np.pi ** 2)
    assert np.allclose(e.eps(T), eps_ref, rtol=1e-12)
    assert np.allclose(e.beta(T), 0.0) and np.allclose(e.B(T), 0.0)


def test_shear_viscosity_limits():
    # Sec. IV.A: massless eta = tau_R (eps + P)/5; constant mass
    # eta = (tau_R/T) int_0^T dT' (eps + P)
    Tt = np.array([0.2, 0.4])
    e0 = ConstMassEoS(Z=3.0, M0=1e-4)
    assert np.allclose(e0.h(Tt), (e0.eps(Tt) + e0.p(Tt)) / 5.0, rtol=1e-6)
    e = ConstMassEoS(Z=3.0, M0=0.5)
    for t in Tt:
        I, _ = quad(lambda tp: e.eps(np.array([tp]))[0] + e.p(np.array([tp]))[0], 1e-3, t,
                    epsabs=0, epsrel=1e-12)
        assert abs(e.h(np.array([t]))[0] - I / t) < 1e-9 * I / t


def test_relaxation_time_rules(eos):
    Tt = np.array([0.2, 0.4, 1.0])
    assert np.allclose(eos.tau_R(Tt, 0.1, "massless"), 0.5 / Tt * HBARC, rtol=1e-15)
    # CE rule: eta = tau_R h(T) equals (eta/s) s
    tr = eos.tau_R(Tt, 0.1, "ce") / HBARC
    assert np.allclose(tr * eos.h(Tt), 0.1 * eos.s(Tt), rtol=1e-13)


def test_entropy_form_sound_speed_and_bulk_viscosity():
    # tanh on s/T^3: c_s^2 = h/(3h + T h') in (0, 1/3]; the Chapman-Enskog bulk
    # viscosity of Sec. IV.A stays non-negative (up to quadrature rounding
    # where M/T is constant at high T and zeta -> 0)
    e = TanhEntropyEoS()
    Tg = np.linspace(0.05, 3.0, 30001)
    cs2 = e.s(Tg) / (Tg * e.ds(Tg))
    assert np.all(cs2 > 0) and np.all(cs2 <= 1 / 3 + 1e-12)
    for t in (0.12, 0.16, 0.17, 0.18, 0.2, 0.25, 0.3, 0.4):
        z = hydro.zeta_over_tauR(e, t)
        assert z > -1e-6 * e.h(np.array([t]))[0], t
    # the printed p/T^4 form has c_s^2 > 1/3 above Tc, where the same formula
    # gives a negative bulk viscosity (a linearly unstable kinetic evolution)
    e_p = TanhEoS(width=0.03)
    assert hydro.zeta_over_tauR(e_p, 0.2) < -0.2 * e_p.h(np.array([0.2]))[0]


def test_inversions():
    e = TanhEoS(width=0.03)
    Tt = np.array([0.06, 0.15, 0.2, 0.4, 2.5])
    assert np.allclose(e.T_from_eps_kin_eq(e.eps_kin_eq(Tt)), Tt, rtol=1e-13)
    assert np.allclose(e.T_from_eps_largest(e.eps(Tt)), Tt, rtol=1e-13)
    # the unstable EoS: an energy density with three roots gives the largest
    e2 = TanhEoS(width=0.02)
    target = 3.19 * HBARC ** 3
    Tr = e2.T_from_eps_largest(np.array([target]))[0]
    assert abs(e2.eps(Tr) - target) < 1e-13 * target
    Tg = np.linspace(Tr + 1e-6, 3.0, 20000)
    assert np.all(e2.eps(Tg) > target)
    assert Tr > 0.196


# ---- tabulated entropy density (the caller's s(T), Sec. III.A) ----

def _power_table(b, A=5.0, T0=0.05, T1=3.2, n=40):
    T = np.exp(np.linspace(np.log(T0), np.log(T1), n))
    return T, A * T ** (3 + b)


@pytest.mark.parametrize("b", [0.0, -0.4, 0.7])
def test_tabulated_power_law_is_exact(b):
    # ln(s/T^3) = ln A + b ln T is linear in ln T, which the cubic spline
    # reproduces exactly, so s, s' and p = p0 + A (T^{4+b} - T0^{4+b})/(4+b)
    # hold off the knots
    from oracle.eos import TabulatedEoS
    A = 5.0
    T, s = _power_table(b, A)
    p0 = 0.01
    e = TabulatedEoS(T, s, p0, Z=20.0)
    Tq = np.array([0.051, 0.0777, 0.19, 0.333, 1.7, 3.1])
    assert np.allclose(e.s(Tq), A * Tq ** (3 + b), rtol=1e-13, atol=0)
    assert np.allclose(e.ds(Tq), (3 + b) * A * Tq ** (2 + b), rtol=1e-12, atol=0)
    p_exact = p0 + A * (Tq ** (4 + b) - T[0] ** (4 + b)) / (4 + b)
    assert np.allclose(e.p(Tq), p_exact, rtol=1e-12, atol=0)


def test_tabulated_cubic_in_log_t_is_exact():
    # a not-a-knot spline is exact on cubics: ln(s/T^3) = c0 + c1 x + c2 x^2
    # + c3 x^3 (x = ln T) on unevenly spaced points
    from oracle.eos import TabulatedEoS
    rng = np.random.default_rng(3)
    x = np.sort(rng.uniform(np.log(0.04), np.log(3.5), 30))
    x[0], x[-1] = np.log(0.04), np.log(3.5)
    y = lambda x: 1.0 + 0.3 * x - 0.2 * x ** 2 + 0.05 * x ** 3
    dy = lambda x: 0.3 - 0.4 * x + 0.15 * x ** 2
    T = np.exp(x)
    e = TabulatedEoS(T, T ** 3 * np.exp(y(x)), 1e-4, Z=40.0)
    xq = np.array([-3.1, -2.0, -0.5, 0.4, 1.2])
    Tq = np.exp(xq)
    assert np.allclose(e.s(Tq), Tq ** 3 * np.exp(y(xq)), rtol=1e-12, atol=0)
    assert np.allclose(e.ds(Tq), Tq ** 2 * np.exp(y(xq)) * (3 + dy(xq)), rtol=1e-11, atol=0)


def test_tabulated_conformal_gas_has_constant_mass_ratio():
    # s = A T^3 with p = A T^4 / 4: every temperature is the same state in
    # units of T, so z = M/T and B/T^4 are constants
    from oracle.eos import TabulatedEoS
    T, s = _power_table(0.0, A=20.0)
    e = TabulatedEoS(T, s, 20.0 * T[0] ** 4 / 4, Z=60.0)  # 2 pi^2 s/(Z T^3) = 6.6 < 8: M exists
    Tq = np.array([0.07, 0.2, 0.9, 2.5])
    z = e.z_of_T(Tq)
    assert np.max(np.abs(z / z[0] - 1)) < 1e-12
    bt4 = e.B(Tq) / Tq ** 4
    assert np.max(np.abs(bt4 - bt4[0])) < 1e-12 * np.max(e.p(Tq) / Tq ** 4)


def test_tabulated_tanh_converges_at_fourth_order():
    # the cubic spline of a smooth function converges like h^4; halving the
    # spacing of a table of the closed-form entropy EoS cuts the error of s
    # and M at least 12x
    from oracle.eos import TabulatedEoS
    ref = TanhEntropyEoS()
    Tq = np.exp(np.linspace(np.log(0.06), np.log(2.8), 97))
    errs = []
    for n in (150, 300, 600):
        T = np.exp(np.linspace(np.log(0.04), np.log(3.5), n))
        e = TabulatedEoS(T, ref.s(T), float(ref.p(T[:1])[0]), ref.Z)
        errs.append((np.max(np.abs(e.s(Tq) / ref.s(Tq) - 1)), np.max(np.abs(e.M(Tq) / ref.M(Tq) - 1))))
    for i in (0, 1):
        assert errs[0][i] / errs[1][i] > 12 and errs[1][i] / errs[2][i] > 12, errs
    assert errs[2][0] < 1e-6
