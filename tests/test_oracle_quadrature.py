"""Pins of the oracle's momentum lattice (paper Sec. IV.C) against closed forms
and independent library routines."""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import kv

from oracle import quadrature as q


@pytest.mark.parametrize("n", [3, 4, 5, 7])
def test_polar_rule_matches_library_gauss_legendre(n):
    # Sec. IV.C polar rule: roots of L_N, weights 2/[(1-mu^2) L'_N(mu)^2]
    mu, w = q.gauss_legendre(n)
    mu_ref, w_ref = np.polynomial.legendre.leggauss(n)
    assert np.allclose(mu, mu_ref, rtol=0, atol=2e-16)
    assert np.allclose(w, w_ref, rtol=2e-14, atol=0)
    for p in range(2 * n):
        exact = (1 - (-1) ** (p + 1)) / (p + 1)
        assert abs(np.sum(w * mu ** p) - exact) < 1e-14


@pytest.mark.parametrize("z0", [1.0, 2.6])
def test_radial_rule_sum_and_exactness(z0):
    # Sec. IV.C: sum_k w_k = K_1(z0)/z0, and exact for cosh^p with p <= 2 N - 1
    n = 5
    x, w = q.radial_rule(z0, n)
    assert abs(w.sum() - kv(1, z0) / z0) < 1e-15 * kv(1, z0) / z0 * 10
    for p in range(2 * n):
        f = lambda t: np.cosh(t) ** p * np.sinh(t) ** 2 * np.exp(-z0 * np.cosh(t))
        ref, _ = quad(f, 0, 12, epsabs=0, epsrel=1e-13, limit=200)
        assert abs(np.sum(w * x ** p) - ref) < 2e-13 * ref
    # degree 2N is not integrated exactly (sanity of the Gauss property)
    f = lambda t: np.cosh(t) ** (2 * n) * np.sinh(t) ** 2 * np.exp(-z0 * np.cosh(t))
    ref, _ = quad(f, 0, 12, epsabs=0, epsrel=1e-13, limit=200)
    assert abs(np.sum(w * x ** (2 * n)) - ref) > 1e-8 * ref


@pytest.mark.parametrize("z0", [1.0, 2.6])
def test_radial_polynomials_closed_forms(z0):
    # Sec. IV.C: R_1 = x - K_2/K_1; R_2 = x^2 + a R_1 + b with the printed a, b
    # (reading: the unbalanced parenthesis of a's denominator closes at its end)
    c = q.radial_polynomials(z0, 5)
    K0, K1, K2 = kv(0, z0), kv(1, z0), kv(2, z0)
    assert abs(c[1][0] - (-K2 / K1)) < 1e-14 * K2 / K1
    a = 6 * K1 * (-z0 ** 2 * K0 ** 2 + (4 + z0 ** 2) * K1 ** 2) / (
        z0 * (z0 ** 3 * K0 ** 3 + 8 * z0 ** 2 * K0 ** 2 * K1 + 14 * z0 * K0 * K1 ** 2
              + 2 * (2 - z0 ** 2) * K1 ** 3 - z0 ** 3 * K2 ** 3))
    b = -(3 * K2 + z0 * K1) / (z0 * K1)
    # R_2 = x^2 + a x + (b - a K2/K1)
    assert abs(c[2][1] - a) < 1e-12 * abs(a)
    assert abs(c[2][0] - (b - a * K2 / K1)) < 1e-12 * abs(b - a * K2 / K1)
    assert c[2][2] == 1.0


def test_radial_orthogonality_and_printed_weight_sums():
    # sum_k w_k R_m(x_k) = 0 for m = 1 .. N-1 (Sec. IV.C) and discrete orthogonality
    z0, n = 1.0, 5
    x, w = q.radial_rule(z0, n)
    R, _ = q.radial_values(z0, n, x)
    G = (R * w) @ R.T
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) < 1e-14 * np.max(np.diag(G))
    for m in range(1, n):
        assert abs(np.sum(w * R[m])) < 1e-14 * np.sqrt(G[m, m] * w.sum())
    # nodes are the roots of R_N
    c = q.radial_polynomials(z0, n)[n]
    vals = np.polynomial.polynomial.polyval(x, c)
    scale = np.polynomial.polynomial.polyval(x, np.abs(c))
    assert np.max(np.abs(vals) / scale) < 1e-13


@pytest.mark.parametrize("n_phi", [3, 4, 5])
def test_azimuth_rule_exact_on_trig_polynomials(n_phi):
    # Sec. IV.C: phi_l = l pi/N_phi integrates cos^a sin^b with a + b < 2 N_phi exactly
    phi, c, s = q.phi_nodes(n_phi)
    assert phi.size == 2 * n_phi
    for a in range(2 * n_phi):
        for b in range(2 * n_phi - a):
            ref, _ = quad(lambda t: np.cos(t) ** a * np.sin(t) ** b, 0, 2 * np.pi, epsabs=1e-14)
            assert abs(np.pi / n_phi * np.sum(c ** a * s ** b) - ref) < 1e-13


def test_angular_normalisation():
    # sum_{j,l} w_theta_j / (4 N_phi) = int dOmega/(4 pi) = 1 (Sec. IV.C)
    for n_phi in (3, 4, 5):
        _, wt = q.gauss_legendre(5)
        assert abs(np.sum(wt) * 2 * n_phi / (4 * n_phi) - 1.0) < 1e-15
