"""Weak-form three-dimensional operator for the mass-gradient force
(paper Sec. IV.B, eq. (fansatz), and eq. (Bmilne)'s term (1/2) d_i M^2 d^i_(p)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

At fixed v = p~/M the force term of eq. (Bmilne) divided by E becomes, per
transverse direction i = x, y and with g_i = d_i ln M,
    dF/dtau  +=  g_i G_i F,   G_i F = (1/gamma) [v^i (v . d_v F) + d_{v^i} F].
Unlike S1 and S2 it mixes the phi slices, so it needs a test space over the
whole sphere of directions: the general ansatz of eq. (fansatz), solid
harmonics of v/|v| of degree n times sinh^n xi times polynomials R_k(cosh xi),
with even powers of sinh xi folded into the polynomials, so that odd degrees
keep one factor sinh xi.  On the product lattice with 2 N_phi azimuths,
N_theta polar and N_xi radial nodes this space is spanned by the N functions
    psi(v) = Phi_m(phi) (1 - mu^2)^{m/2} L_j(mu) s^{(m + j) mod 2} P_i(x),
with Phi_m = cos(m phi) (m = 0 .. N_phi) or sin(m phi) (m = 1 .. N_phi - 1),
L_j the Legendre polynomials (j < N_theta), P_i polynomials of degree
i < N_xi, s = sinh xi, x = cosh xi, mu = cos theta.  (Re (v^x + i v^y)^m
(v^Y)^j = s^{m+j} (1 - mu^2)^{m/2} mu^j e^{i m phi}: degree n = m + j.)

The weak form follows the construction of Sec. IV.D: G_i F is the node vector
whose projections on the test space equal those of the continuum operator
after integration by parts.  The lattice sum sum_n w_n (...) is the
quadrature of int d^3 v / (4 pi gamma) (...), so for every test function psi
    sum_n w_n psi(n) (G_i F)_n = sum_n w_n F_n b_i[psi](n),
    b_i[psi] = -(1/gamma) [v^i (v . grad psi) + d_{v^i} psi + 2 v^i psi]
(moving the derivatives of (psi/gamma^2) v^i v^j and psi/gamma^2 onto psi;
the surface terms vanish because F decays).  The N conditions fix the N
values of G_i F.

The test space holds 1, gamma, v^i, gamma^2, gamma v^i and v^i v^j, so the
lattice moments of the force obey the continuum balance laws exactly:
energy, momentum (with d_j B = -M^4/(2 pi^2) g_j sum w F from eq. (sanity))
and particle number.

Reading: the paper words the odd-degree reduction as one inverse power of
sinh xi.  With s^{-1} instead of s in the odd terms the balance laws still
hold, but the operator is then far from the continuum one even on the
lattice's reference equilibrium exp(-z0 cosh xi) (pointwise error above 100%),
whereas with one factor s it is exact there, as the paper's quadrature is
exact for that equilibrium.  The factor s is used.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as npcheb
from numpy.polynomial import legendre as npleg


def _test_functions(lat):
    """Values and gradients of the N test functions at the N nodes.

    Returns psi (N nodes, N functions), v.grad psi, d psi/dv^x, d psi/dv^y.
    Gradients in spherical variables (s, mu, phi):
        grad = n d_s + (theta_hat / s) d_theta + (phi_hat / (s sin theta)) d_phi,
        d_theta = -sin theta d_mu.
    """
    n_phi, nt, nx = lat.n_phi, lat.n_theta, lat.n_xi
    x = lat.gamma
    s = np.sqrt(x * x - 1.0)
    mu = lat.mu_j[lat.j_n]
    st = np.sqrt(1.0 - mu * mu)
    ph = lat.phi_l[lat.l_n]
    cph, sph = lat.cos_l[lat.l_n], lat.sin_l[lat.l_n]

    # radial polynomials: Chebyshev on the node interval (conditioning only)
    lo, hi = lat.x_k[0], lat.x_k[-1]
    t = (2.0 * x - (lo + hi)) / (hi - lo)

    modes = [(m, "c") for m in range(n_phi + 1)] + [(m, "s") for m in range(1, n_phi)]
    cols, cols_r, cols_x, cols_y = [], [], [], []
    for m, kind in modes:
        if kind == "c":
            Ph, dPh = np.cos(m * ph), -m * np.sin(m * ph)
        else:
            Ph, dPh = np.sin(m * ph), m * np.cos(m * ph)
        for j in range(nt):
            cj = np.eye(nt)[j]
            Lj = npleg.legval(mu, cj)
            dLj = npleg.legval(mu, npleg.legder(cj))
            A = st ** m * Lj
            # d/dmu [(1 - mu^2)^{m/2} L_j] = (1 - mu^2)^{m/2} L_j' - m mu (1 - mu^2)^{m/2 - 1} L_j
            dA = st ** m * dLj - m * mu * st ** (m - 2) * Lj if m > 0 else dLj
            e = (m + j) % 2
            for i in range(nx):
                ci = np.eye(nx)[i]
                P = npcheb.chebval(t, ci)
                dP = npcheb.chebval(t, npcheb.chebder(ci)) * 2.0 / (hi - lo)
                Rad = P * s ** e
                # d/ds [s^e P(x)], dx/ds = s/x
                dRad = dP * (s / x) * s ** e + e * P * s ** (e - 1)
                psi = Ph * A * Rad
                d_s = Ph * A * dRad
                d_mu = Ph * dA * Rad
                d_ph = dPh * A * Rad
                d_th = -st * d_mu
                gx = st * cph * d_s + mu * cph * d_th / s - sph * d_ph / (s * st)
                gy = st * sph * d_s + mu * sph * d_th / s + cph * d_ph / (s * st)
                cols.append(psi)
                cols_r.append(s * d_s)
                cols_x.append(gx)
                cols_y.append(gy)
    st_ = lambda c: np.stack(c, axis=1)
    return st_(cols), st_(cols_r), st_(cols_x), st_(cols_y)


def weak_force_operators(lat):
    """(G_x, G_y), each N x N: (G_i F)_n for F given on the N nodes in the
    lattice's canonical node order."""
    psi, vgrad, dx_, dy_ = _test_functions(lat)
    if psi.shape[0] != psi.shape[1]:
        raise ValueError("test space and node set differ in size")
    g = lat.gamma[:, None]
    vx, vy = lat.V[1][:, None], lat.V[2][:, None]
    W = np.diag(lat.w)
    out = []
    for vi, di in ((vx, dx_), (vy, dy_)):
        b = -(vi * vgrad + di + 2.0 * vi * psi) / g          # b_i[psi_a] at the nodes
        # sum_n w_n psi_a(n) (G F)_n = sum_n w_n F_n b_a(n) for every a
        out.append(np.linalg.solve(psi.T @ W, b.T @ W))
    return out[0], out[1]


def apply(Gx, Gy, F, gx, gy):
    """Force term g_x G_x F + g_y G_y F for F (N, ...sites), g (...sites)."""
    return (gx[None] * np.einsum("nm,m...->n...", Gx, F)
            + gy[None] * np.einsum("nm,m...->n...", Gy, F))
