"""Momentum-lattice quadrature (paper Sec. IV.C, "Deriving the Momentum Lattice").

TEST INFRASTRUCTURE ONLY (see the package docstring).

Three one-dimensional rules make up the product lattice:

* azimuth: phi_l = l pi / N_phi, l = 0 .. 2 N_phi - 1, the zeros of
  sin(N_phi phi), each with weight pi / N_phi;
* polar: cos(theta_j) = the roots of the Legendre polynomial L_{N_theta}, with
  weights 2 / [(1 - mu^2) L'_{N_theta}(mu)^2] (the formula printed in the
  paper);
* radial: x_k = cosh(xi_k) = the roots of R_{N_xi}, where R_0, R_1, ... are
  the monic polynomials in x = cosh(xi) orthogonal with respect to
  int_0^inf dxi exp(-z0 cosh xi) sinh^2 xi, and w_k the Gauss (Christoffel)
  weights of that measure, so that sum_k w_k = K_1(z0)/z0.

The radial rule is built in 60-digit arithmetic (mpmath) straight from its
definition: moments of the measure by numerical integration, Gram-Schmidt
orthogonalisation of 1, x, x^2, ..., roots of R_{N_xi}, Christoffel weights.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

_DPS = 60


def phi_nodes(n_phi: int):
    """Azimuthal nodes phi_l = l pi / N_phi (paper Sec. IV.C, azimuth rule).

    Returns (phi, cos(phi), sin(phi)).  cos and sin are exact (0 or +-1) at
    multiples of pi/2, which the printed definition fixes; elsewhere they are
    the correctly rounded library values.
    """
    phi = np.arange(2 * n_phi) * np.pi / n_phi
    c = np.cos(phi)
    s = np.sin(phi)
    for l in range(2 * n_phi):
        # multiples of pi/2 are exact: 2 l / n_phi integer
        if (2 * l) % n_phi == 0:
            q = (2 * l) // n_phi % 4
            c[l] = [1.0, 0.0, -1.0, 0.0][q]
            s[l] = [0.0, 1.0, 0.0, -1.0][q]
    return phi, c, s


def _legendre_and_derivative(n: int, x):
    """L_n(x) and L_n'(x) by the three-term (Bonnet) recurrence."""
    x = np.asarray(x, dtype=float)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    # derivative: (1 - x^2) L_n' = n (L_{n-1} - x L_n)
    dp = n * (p0 - x * p1) / (1.0 - x * x)
    return p1, dp


def gauss_legendre(n_theta: int):
    """Polar nodes mu_j = cos(theta_j) and weights (paper Sec. IV.C, polar rule).

    Nodes: roots of L_{N_theta} found by Newton's method from the Chebyshev
    estimates cos(pi (j + 3/4) / (N + 1/2)).  Weights: the printed formula
    w_j = 2 / [(1 - mu_j^2) L'_N(mu_j)^2].  Nodes are returned in increasing
    order.
    """
    n = n_theta
    j = np.arange(n)
    x = np.cos(np.pi * (j + 0.75) / (n + 0.5))
    for _ in range(100):
        p, dp = _legendre_and_derivative(n, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p, dp = _legendre_and_derivative(n, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order], w[order]


@functools.lru_cache(maxsize=32)
def _radial_rule_mp(z0: float, n_xi: int):
    """Radial rule in 60-digit arithmetic, cached per (z0, N_xi).

    Returns (nodes, weights, coeffs, norms) as mpmath objects: coeffs[l] are
    the monomial coefficients (lowest degree first) of the monic R_l for
    l = 0 .. n_xi, norms[l] = int R_l^2 dmu.
    """
    with mp.workdps(_DPS):
        z = mp.mpf(z0)

        # the integrand falls like exp(-z0 cosh xi): beyond z0 cosh xi = 400 it
        # is below 1e-170 of its peak, far under the working precision
        xi_max = mp.acosh(400 / z + 1)
        pieces = mp.linspace(0, xi_max, 12)

        def moment(p):
            # int_0^inf cosh^p(xi) sinh^2(xi) exp(-z0 cosh xi) dxi
            f = lambda t: mp.cosh(t) ** p * mp.sinh(t) ** 2 * mp.exp(-z * mp.cosh(t))
            return mp.quad(f, pieces)

        nmom = 2 * n_xi + 1
        mom = [moment(p) for p in range(nmom)]

        def inner(a, b):
            # <a, b> for polynomials given by coefficient lists
            s = mp.mpf(0)
            for i, ai in enumerate(a):
                if ai == 0:
                    continue
                for k, bk in enumerate(b):
                    s += ai * bk * mom[i + k]
            return s

        coeffs, norms = [], []
        for l in range(n_xi + 1):
            c = [mp.mpf(0)] * l + [mp.mpf(1)]          # x^l
            for i in range(l):                         # Gram-Schmidt
                proj = inner(c, coeffs[i]) / norms[i]
                c = [ci - proj * (coeffs[i][k] if k < len(coeffs[i]) else 0)
                     for k, ci in enumerate(c)]
            coeffs.append(c)
            norms.append(inner(c, c))

        # nodes: roots of R_{n_xi}; mpmath.polyroots takes highest degree first
        roots = mp.polyroots(list(reversed(coeffs[n_xi])), maxsteps=200, extraprec=200)
        roots = sorted([mp.re(r) for r in roots])

        def rval(l, x):
            return mp.fsum(c * x ** i for i, c in enumerate(coeffs[l]))

        # Christoffel weights: w_k = 1 / sum_{l<N} R_l(x_k)^2 / I(l)
        weights = [1 / mp.fsum(rval(l, x) ** 2 / norms[l] for l in range(n_xi)) for x in roots]
        return roots, weights, coeffs, norms, mom


def radial_rule(z0: float, n_xi: int):
    """Radial nodes x_k = cosh(xi_k) and weights w^xi_k (paper Sec. IV.C).

    The weights satisfy sum_k w_k R_0(x_k) = K_1(z0)/z0 and sum_k w_k R_m(x_k) = 0
    for m = 1 .. N_xi - 1, as printed.
    """
    roots, weights, _, _, _ = _radial_rule_mp(float(z0), int(n_xi))
    return (np.array([float(r) for r in roots]), np.array([float(w) for w in weights]))


def radial_polynomials(z0: float, n_xi: int):
    """Monomial coefficients (lowest degree first) of the monic R_0..R_{N_xi}.

    Float64 copies of the 60-digit Gram-Schmidt result.  R_1 and R_2 have the
    closed forms printed in Sec. IV.C.
    """
    _, _, coeffs, _, _ = _radial_rule_mp(float(z0), int(n_xi))
    return [np.array([float(c) for c in cl]) for cl in coeffs]


def radial_values(z0: float, n_xi: int, x):
    """R_l(x) and R_l'(x) for l = 0 .. N_xi - 1, evaluated in 60-digit arithmetic.

    Returns two arrays of shape (N_xi, len(x)).
    """
    _, _, coeffs, _, _ = _radial_rule_mp(float(z0), int(n_xi))
    x = np.atleast_1d(np.asarray(x, dtype=float))
    R = np.zeros((n_xi, x.size))
    dR = np.zeros((n_xi, x.size))
    with mp.workdps(_DPS):
        for l in range(n_xi):
            c = coeffs[l]
            for i, xv in enumerate(x):
                xm = mp.mpf(xv)
                R[l, i] = float(mp.fsum(ck * xm ** k for k, ck in enumerate(c)))
                dR[l, i] = float(mp.fsum(k * ck * xm ** (k - 1) for k, ck in enumerate(c) if k > 0))
    return R, dR


def radial_moments(z0: float, n_xi: int):
    """The moments int cosh^p sinh^2 exp(-z0 cosh) dxi, p = 0 .. 2 N_xi (float64)."""
    _, _, _, _, mom = _radial_rule_mp(float(z0), int(n_xi))
    return np.array([float(m) for m in mom])
