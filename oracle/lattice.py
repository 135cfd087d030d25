"""Discrete momentum set and weak-form momentum-derivative operators
(paper Sec. IV.B-IV.D).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Node order (canonical): n = (k * N_theta + j) * (2 N_phi) + l with k the
radial index (xi_k), j the polar index (theta_j) and l the azimuthal index
(phi_l).  A "slice" is the set of N_xi * N_theta nodes with one phi_l; slice
vectors are ordered by q = k * N_theta + j.

Momentum of node n (Sec. IV.B, momentum parametrisation), in units of M and
in the Milne-orthonormal frame:
    V_n = (cosh xi_k, sinh xi_k sin theta_j cos phi_l,
           sinh xi_k sin theta_j sin phi_l, sinh xi_k cos theta_j),
so that P^mu_n = M V^mu_n and v = (V^x, V^y, V^Y) is the paper's bold v.

Weights (Sec. IV.C): w_n = exp(z0 x_k) w^xi_k w^theta_j / (4 N_phi), which make
sum_n w_n f(P_n) the quadrature of int dOmega/(4 pi) int dxi sinh^2 xi f.

Energy-momentum tensor (eq. (emtnew)): T^{ab} = M^4/(2 pi^2) sum_n w_n F_n
V^a_n V^b_n (+ B g^{ab}); particle current (eq. (NTdisc)) on the same lattice:
N^a = M^3/(2 pi^2) sum_n w_n F_n V^a_n.

Operators (Sec. IV.D, coefficients s_1^{ml}, s_2^{ml}): for one phi slice,
    (S F)_n = exp(-z0 x_n) sum_{m < N_theta} sum_{l < N_xi} L_m(mu_n) R_l(x_n) s^{ml},
    s^{ml} = -(2m+1)/I(l) sum_{n'} w'_{n'} F_{n'} b^{ml}(n'),
with w'_n = exp(z0 x_k) w^xi_k w^theta_j / 2 (the weight of one slice; summing
2 N_phi equal slices with w_n gives the same number), I(l) = sum_k w^xi_k R_l(x_k)^2
and, with mu = cos theta, x = cosh xi, t^2 = tanh^2 xi:
    b_1^{ml} = (L_m R_l' x - L_m R_l) mu^2 t^2 + R_l (L_m + L_m' (mu - mu^3)),
    b_2^{ml} = L_m R_l (2 + 1/x^2) + L_m R_l' x t^2.
S1 represents p^Y d/dp^Y (= v^Y d/dv^Y) and S2 represents p . d/dp (= v . d/dv),
both at fixed phi, so they act on each phi slice separately.

Readings: the printed s_1 bracket "(P_m R'_l cosh xi - R_l)" is read as
(L_m R'_l x - L_m R_l) (integration by parts of v^Y d/dv^Y against L_m R_l / E
gives exactly this); "\\hat f_1" in s_2 is read as the distribution of the
current stage; I(l) carries the weight exp(-z0 cosh xi) so that the projection
of a basis function returns coefficient 1.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg

from . import quadrature as quad

PI2 = np.pi ** 2


def weak_brackets(x, mu, Lm, dLm, R, dR):
    """The brackets b_1, b_2 of the coefficients s_1^{ml}, s_2^{ml} (Sec. IV.D)
    for the test function psi = L_m(mu) R(x), at points (x = cosh xi, mu =
    cos theta), given L_m, L_m', R, R' there.  They are what integration by
    parts against the measure sinh^2 xi d xi d mu leaves on psi:
        int psi (S F) = -int F b[psi]   for S1 = p^Y d/dp^Y, S2 = p . d/dp,
    with t^2 = tanh^2 xi = (x^2 - 1)/x^2:
        b_1 = (L_m R' x - L_m R) mu^2 t^2 + R (L_m + L_m' (mu - mu^3)),
        b_2 = L_m R (2 + 1/x^2) + L_m R' x t^2."""
    t2 = (x * x - 1.0) / (x * x)
    b1 = (Lm * dR * x - Lm * R) * mu ** 2 * t2 + R * (Lm + dLm * (mu - mu ** 3))
    b2 = Lm * R * (2.0 + 1.0 / x ** 2) + Lm * dR * x * t2
    return b1, b2


class Lattice:
    def __init__(self, n_xi=5, n_theta=5, n_phi=4, z0=1.0, form="weak", force="feq"):
        """form = "weak": the paper's weak-form S1, S2 (Sec. IV.D); "strong":
        the derivatives of the interpolant through the nodes (a comparison
        variant, see _strong_form_operators).
        force = "feq": the mass-gradient force acts on F_eq, differentiated
        analytically; "weak3d": it acts on F through the weak-form operators
        G_x, G_y over the whole sphere of directions (force3d)."""
        self.n_xi, self.n_theta, self.n_phi, self.z0 = int(n_xi), int(n_theta), int(n_phi), float(z0)
        self.form = form
        self.force = force
        self.n_slice = 2 * self.n_phi
        self.n_kj = self.n_xi * self.n_theta
        self.N = self.n_kj * self.n_slice

        # one-dimensional rules (Sec. IV.C)
        self.x_k, self.w_xi = quad.radial_rule(self.z0, self.n_xi)
        self.s_k = np.sqrt(self.x_k ** 2 - 1.0)
        self.mu_j, self.w_th = quad.gauss_legendre(self.n_theta)
        self.sin_j = np.sqrt(1.0 - self.mu_j ** 2)
        self.phi_l, self.cos_l, self.sin_l = quad.phi_nodes(self.n_phi)

        # product lattice in canonical order
        k, j, l = np.meshgrid(np.arange(self.n_xi), np.arange(self.n_theta),
                              np.arange(self.n_slice), indexing="ij")
        self.k_n, self.j_n, self.l_n = k.ravel(), j.ravel(), l.ravel()
        x = self.x_k[self.k_n]
        sh = self.s_k[self.k_n]
        self.gamma = x
        self.w = np.exp(self.z0 * x) * self.w_xi[self.k_n] * self.w_th[self.j_n] / (4 * self.n_phi)
        self.V = np.stack([
            x,
            sh * self.sin_j[self.j_n] * self.cos_l[self.l_n],
            sh * self.sin_j[self.j_n] * self.sin_l[self.l_n],
            sh * self.mu_j[self.j_n],
        ])  # (4, N)

        if form == "weak":
            self.D1, self.D2 = self._weak_form_operators()
        elif form == "strong":
            self.D1, self.D2 = self._strong_form_operators()
        else:
            raise ValueError(f"unknown operator form {form!r}")
        if force == "weak3d":
            from . import force3d
            self.Gx, self.Gy = force3d.weak_force_operators(self)
        elif force != "feq":
            raise ValueError(f"unknown force form {force!r}")

    # ------------------------------------------------------------------
    def _weak_form_operators(self):
        """Dense slice operators D1, D2 (n_kj x n_kj), built literally from the
        projection formula and the s_1, s_2 coefficients of Sec. IV.D."""
        nx, nt, z0 = self.n_xi, self.n_theta, self.z0
        q = np.arange(self.n_kj)
        kq, jq = q // nt, q % nt
        x = self.x_k[kq]
        mu = self.mu_j[jq]
        wslice = np.exp(z0 * x) * self.w_xi[kq] * self.w_th[jq] / 2.0

        Rv, dRv = quad.radial_values(z0, nx, self.x_k)       # (l, k)
        I = np.array([np.sum(self.w_xi * Rv[l] ** 2) for l in range(nx)])

        Phi = np.zeros((self.n_kj, nt * nx))      # basis at nodes, with exp(-z0 x)
        B1 = np.zeros((nt * nx, self.n_kj))       # -(2m+1)/I(l) w' b_1
        B2 = np.zeros((nt * nx, self.n_kj))
        for m in range(nt):
            cm = np.zeros(m + 1)
            cm[m] = 1.0
            Lm = npleg.legval(mu, cm)
            dLm = npleg.legval(mu, npleg.legder(cm))
            for l in range(nx):
                R = Rv[l, kq]
                dR = dRv[l, kq]
                col = m * nx + l
                Phi[:, col] = np.exp(-z0 * x) * Lm * R
                b1, b2 = weak_brackets(x, mu, Lm, dLm, R, dR)
                pref = -(2 * m + 1) / I[l]
                B1[col, :] = pref * wslice * b1
                B2[col, :] = pref * wslice * b2
        return Phi @ B1, Phi @ B2

    def _strong_form_operators(self):
        """Strong-form slice operators: on one phi slice the values F_{kj} are
        interpolated by exp(-z0 x) P(x, mu), P of degree < N_xi in x and
        < N_theta in mu through the nodes, and the continuum operators are
        applied to the interpolant at the nodes:
            S2 F = p . dF/dp = ((x^2 - 1)/x) dF/dx       (|p| = M sinh xi),
            S1 F = p^Y dF/dp^Y = mu^2 (x^2 - 1)/x dF/dx + mu (1 - mu^2) dF/dmu.
        P is written in Chebyshev polynomials of x mapped to [-1, 1] times
        Legendre polynomials of mu (a well-conditioned tensor basis) and its
        coefficients are solved for directly."""
        from numpy.polynomial import chebyshev as npcheb
        nx, nt, z0 = self.n_xi, self.n_theta, self.z0
        q = np.arange(self.n_kj)
        x = self.x_k[q // nt]
        mu = self.mu_j[q % nt]
        lo, hi = self.x_k[0], self.x_k[-1]
        t = (2.0 * x - (lo + hi)) / (hi - lo)
        dt_dx = 2.0 / (hi - lo)
        Vt = npcheb.chebvander(t, nx - 1)                       # (n_kj, nx)
        dVt = np.stack([npcheb.chebval(t, npcheb.chebder(np.eye(nx)[a])) for a in range(nx)], 1) * dt_dx
        Vm = npleg.legvander(mu, nt - 1)                        # (n_kj, nt)
        dVm = np.stack([npleg.legval(mu, npleg.legder(np.eye(nt)[b])) for b in range(nt)], 1)
        V = (Vt[:, :, None] * Vm[:, None, :]).reshape(self.n_kj, -1)
        Vx = (dVt[:, :, None] * Vm[:, None, :]).reshape(self.n_kj, -1)
        Vu = (Vt[:, :, None] * dVm[:, None, :]).reshape(self.n_kj, -1)
        # P coefficients of a slice vector F: P(nodes) = exp(z0 x) F
        C = np.linalg.solve(V, np.diag(np.exp(z0 * x)))
        E = np.diag(np.exp(-z0 * x))
        dFdx = E @ (Vx @ C - z0 * (V @ C))      # d/dx [exp(-z0 x) P] at the nodes
        dFdmu = E @ (Vu @ C)
        D2 = np.diag((x * x - 1.0) / x) @ dFdx
        D1 = np.diag(mu * mu) @ D2 + np.diag(mu * (1.0 - mu * mu)) @ dFdmu
        return D1, D2

    # ------------------------------------------------------------------
    def apply_slices(self, D, F):
        """Apply a slice operator to every phi slice of F (N, ...)."""
        sh = F.shape
        Fs = F.reshape(self.n_kj, self.n_slice, -1)
        out = np.einsum("pq,qsr->psr", D, Fs)
        return out.reshape(sh)

    def moments(self, F, lnM):
        """Kinetic T^{ab} (a, b in tau, x, y, Y) and N^a of eq. (emtnew) / (NTdisc).

        F has shape (N, ...sites); lnM has shape (...sites).  Returns
        Tk (4, 4, ...) in GeV^4 and Nk (4, ...) in GeV^3, without B.
        """
        M = np.exp(lnM)
        G = M ** 4 / (2 * PI2)
        wF = self.w.reshape((-1,) + (1,) * (F.ndim - 1)) * F
        Tk = np.einsum("an,bn,n...->ab...", self.V, self.V, wF) * G
        Nk = np.einsum("an,n...->a...", self.V, wF) * M ** 3 / (2 * PI2)
        return Tk, Nk
