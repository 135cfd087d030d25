"""Pins of the weak-form three-dimensional mass-gradient force (oracle.force3d;
paper eq. (fansatz) test space, eq. (Bmilne) force term, eq. (sanity)).

What fixes the operator independently of its construction:
* balance laws: with dF/dtau += g_i G_i F the lattice moments of the force
  must give what energy, momentum and particle-number conservation demand
  once T^{ab} = M^4/(2 pi^2) sum w F V^a V^b is differentiated in space
  (the factor M^4 gives 4 g_i, M^3 in N^a gives 3 g_i) and
  d_j B = -M^4/(2 pi^2) g_j sum w F (eq. (sanity) in space):
      sum w gamma^2 G_i F     = -4 sum w gamma v^i F,
      sum w gamma v^j G_i F   = -4 sum w v^i v^j F - delta_ij sum w F,
      sum w gamma G_i F       = -3 sum w v^i F;
* the continuum value on the lattice's reference equilibrium
  F = exp(-z0 gamma): G_i F = -z0 v^i F;
* symmetry: rotations by pi/N_phi about the Y axis and the reflections
  y -> -y, Y -> -Y;
* dynamics: in free streaming with a space-dependent mass the total
  momentum of a periodic box drifts only at the order of the spatial
  discretisation (second order in dx), which the F_eq form does not do.
"""
import numpy as np
import pytest

from oracle import force3d
from oracle import step as st
from oracle.eos import HBARC, TanhEntropyEoS
from oracle.lattice import Lattice


@pytest.fixture(scope="module")
def lat():
    return Lattice(5, 5, 4, 1.0, force="weak3d")


def _random_state(lat, seed):
    rng = np.random.default_rng(seed)
    return np.exp(-1.3 * lat.gamma) * (1.0 + 0.4 * rng.standard_normal(lat.N))


def test_balance_laws(lat):
    w, g, V = lat.w, lat.gamma, lat.V
    for seed in range(3):
        F = _random_state(lat, seed)
        scale = np.sum(w * g * g * F)
        for i, G in ((1, lat.Gx), (2, lat.Gy)):
            GF = G @ F
            assert abs(np.sum(w * g * g * GF) + 4 * np.sum(w * g * V[i] * F)) < 1e-12 * scale
            assert abs(np.sum(w * g * GF) + 3 * np.sum(w * V[i] * F)) < 1e-12 * scale
            for j in (1, 2, 3):
                want = -4 * np.sum(w * V[i] * V[j] * F) - (i == j) * np.sum(w * F)
                assert abs(np.sum(w * g * V[j] * GF) - want) < 1e-12 * scale


def test_feq_form_breaks_the_momentum_balance(lat):
    # the force on F_eq only (analytic derivatives) carries the balance for
    # the equilibrium part: a state off equilibrium shows the difference
    # (here in the form the oracle's F_eq path uses at u = 0, M/T = 1.3)
    w, g, V = lat.w, lat.gamma, lat.V
    F = _random_state(lat, 7)
    Feq = np.exp(-1.3 * g)
    Gr_feq = -1.3 * V[1] * Feq           # (1/gamma)[v^x v.d_v + d_vx] exp(-1.3 gamma)
    want = -4 * np.sum(w * V[1] * V[1] * F) - np.sum(w * F)
    got = np.sum(w * g * V[1] * Gr_feq)
    assert abs(got - want) > 1e-2 * abs(want)


@pytest.mark.parametrize("z0", [1.0, 2.0])
def test_exact_on_reference_equilibrium(z0):
    lat = Lattice(5, 5, 4, z0, force="weak3d")
    F = np.exp(-z0 * lat.gamma)
    for i, G in ((1, lat.Gx), (2, lat.Gy)):
        want = -z0 * lat.V[i] * F
        assert np.max(np.abs(G @ F - want)) < 1e-10 * np.max(np.abs(want))


def test_rotation_and_reflections(lat):
    F = _random_state(lat, 11)
    nk, ns = lat.n_kj, lat.n_slice
    a = np.pi / lat.n_phi

    def rot(v):      # (R F)_l = F_{l-1}: the state turned by pi/N_phi
        return np.roll(v.reshape(nk, ns), 1, axis=1).ravel()

    def refl_y(v):   # phi -> -phi
        return v.reshape(nk, ns)[:, (-np.arange(ns)) % ns].ravel()

    def refl_Y(v):   # mu -> -mu
        return v.reshape(lat.n_xi, lat.n_theta, ns)[:, ::-1, :].ravel()

    Gx, Gy = lat.Gx, lat.Gy
    tol = 1e-12 * np.max(np.abs(Gx @ F))
    assert np.max(np.abs(Gx @ rot(F) - rot(np.cos(a) * (Gx @ F) - np.sin(a) * (Gy @ F)))) < tol
    assert np.max(np.abs(Gy @ rot(F) - rot(np.sin(a) * (Gx @ F) + np.cos(a) * (Gy @ F)))) < tol
    assert np.max(np.abs(Gx @ refl_y(F) - refl_y(Gx @ F))) < tol
    assert np.max(np.abs(Gy @ refl_y(F) + refl_y(Gy @ F))) < tol
    assert np.max(np.abs(Gx @ refl_Y(F) - refl_Y(Gx @ F))) < tol
    assert np.max(np.abs(Gy @ refl_Y(F) - refl_Y(Gy @ F))) < tol


def test_planted_mistake_breaks_the_energy_balance(lat):
    # a 3 v^i psi instead of 2 v^i psi in the integrated-by-parts bracket
    psi, vgrad, dx_, _ = force3d._test_functions(lat)
    W = np.diag(lat.w)
    vx = lat.V[1][:, None]
    b = -(vx * vgrad + dx_ + 3.0 * vx * psi) / lat.gamma[:, None]
    Gbad = np.linalg.solve(psi.T @ W, b.T @ W)
    F = _random_state(lat, 3)
    w, g, V = lat.w, lat.gamma, lat.V
    err = abs(np.sum(w * g * g * (Gbad @ F)) + 4 * np.sum(w * g * V[1] * F))
    assert err > 1e-3 * np.sum(w * g * g * F)


def _momentum_drift(lat, eos, nx):
    # 1-D periodic box, Minkowski metric, free streaming, mass varying in x
    L = 6.4
    dx = L / nx
    xs = (np.arange(nx) + 0.5) * dx
    e0 = (float(eos.eps(0.3)) / HBARC ** 3) * (1 + 0.5 * np.sin(2 * np.pi * xs / L)
                                              + 0.25 * np.sin(4 * np.pi * xs / L + 1.0))[None, :]
    ux = (0.1 + 0.2 * np.cos(2 * np.pi * xs / L + 0.5))[None, :]
    prm = st.Params(dx=dx, eta_over_s=np.inf, metric=st.METRIC_MINKOWSKI)
    F, l = st.init_state(lat, eos, e0, ux, None)
    T0, _ = lat.moments(F, l)
    tau, dt = 1.0, 0.25 * dx
    for _ in range(int(round(0.4 / dt))):
        F, l = st.heun_step(lat, eos, prm, F, l, tau, dt)
        tau += dt
    T1, _ = lat.moments(F, l)
    return (T1[0, 1].sum() - T0[0, 1].sum()) / T0[0, 0].sum()


def test_free_streaming_momentum_drift_is_second_order(lat):
    eos = TanhEntropyEoS()
    d16, d32 = _momentum_drift(lat, eos, 16), _momentum_drift(lat, eos, 32)
    assert 3.0 < d16 / d32 < 5.0
    feq = Lattice(5, 5, 4, 1.0)
    f16, f32 = _momentum_drift(feq, eos, 16), _momentum_drift(feq, eos, 32)
    assert abs(f32) > 5 * abs(d32)
    assert abs(f32) > 0.5 * abs(f16)   # no convergence with dx
