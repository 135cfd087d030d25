"""C-ABI contract on the CPU: the library loads, exports every function the
header declares, validates on the host before any device call, and its
independently derived host setup (lattice, factored operators, EoS tables)
agrees with the oracle."""
import ctypes
import math

import numpy as np
import pytest

import paper_1108_5561_amd as lb
from oracle import quadrature as oq
from oracle.eos import HBARC, ConstMassEoS, TanhEntropyEoS, TanhEoS
from oracle.lattice import Lattice


def test_library_exports_every_header_function():
    names = lb.header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lb.lib, n), n


def test_workspace_bytes_and_validation():
    p = lb.make_params(32, 32, 0.2)
    n = lb.workspace_bytes(p)
    assert n >= 3 * 200 * 1024 * 8
    p32 = lb.make_params(32, 32, 0.2, precision=lb.LB_FP32_FP64MATCH)
    assert lb.workspace_bytes(p32) < n
    for bad in [dict(nx=0), dict(ny=-1), dict(dx_fm=0.0), dict(dx_fm=float("nan")), dict(eta_over_s=0.0),
                dict(n_xi=4), dict(n_phi=6), dict(n_theta=9), dict(z0=-1.0), dict(T_min_GeV=0.0), dict(eos_width_GeV=0.0),
                dict(tau0_fm=0.0), dict(precision=7), dict(metric=5), dict(taur_rule=3), dict(Z=0.0)]:
        q = lb.make_params(32, 32, 0.2)
        for k, v in bad.items():
            setattr(q, k, v)
        assert lb.lib.lb_workspace_bytes(ctypes.byref(q)) == 0, bad
        assert lb.last_error() != ""


def _init_rc(p, ws=256, e0=512):
    ctx = ctypes.c_void_p()
    return lb.lib.lb_init(ctypes.byref(ctx), ctypes.byref(p), ws, 1 << 40, e0, None, None, None), ctx


def test_init_rejects_on_host_before_device_work():
    p = lb.make_params(8, 8, 0.2)
    assert lb.lib.lb_init(None, ctypes.byref(p), 256, 1 << 40, 512, None, None, None) == lb.LB_E_ARG
    q = lb.make_params(8, 8, 0.2)
    q.nx = 0
    assert _init_rc(q)[0] == lb.LB_E_ARG
    assert _init_rc(p, ws=None)[0] == lb.LB_E_ARG
    assert _init_rc(p, ws=257)[0] == lb.LB_E_ARG            # misaligned
    assert _init_rc(p, e0=None)[0] == lb.LB_E_ARG
    ctx = ctypes.c_void_p()
    assert lb.lib.lb_init(ctypes.byref(ctx), ctypes.byref(p), 256, 1024, 512, None, None, None) == lb.LB_E_ARG


def test_unstable_or_massless_eos_is_rejected():
    # the tanh EoS of width 0.02 GeV has d eps/dT < 0 near 0.19 GeV: the mass
    # equation of the scheme is singular there
    p = lb.make_params(8, 8, 0.2, eos_kind=lb.LB_EOS_TANH_P, eos_width_GeV=0.02)
    rc, _ = _init_rc(p)
    assert rc == lb.LB_E_EOS and "unstable" in lb.last_error()
    # kappa = 1: the quasiparticle entropy cannot reach s(T), no M(T)
    p = lb.make_params(8, 8, 0.2, eos_kind=lb.LB_EOS_TANH_P, eos_width_GeV=0.03, kappa=1.0)
    rc, _ = _init_rc(p)
    assert rc == lb.LB_E_EOS and "mass" in lb.last_error()


def test_momentum_lattice_choices():
    # n_xi, n_theta in {3, 5, 7} and n_phi in {3, 4, 5}; lattices other than
    # 5 x 5 x 8 run on the generic FP64 kernels (force on F_eq, mu = 0)
    for nxi, nth, nph in [(3, 5, 4), (7, 5, 5), (5, 3, 3), (5, 7, 4), (3, 3, 3)]:
        p = lb.make_params(8, 8, 0.2, n_xi=nxi, n_theta=nth, n_phi=nph)
        n = lb.lib.lb_workspace_bytes(ctypes.byref(p))
        assert n >= 3 * nxi * nth * 2 * nph * 64 * 8, (nxi, nth, nph)
        for bad in (dict(precision=lb.LB_FP32_FP64MATCH), dict(force_form=lb.LB_FORCE_WEAK3D),
                    dict(particle_number=lb.LB_N_CONSERVED, eos_kind=lb.LB_EOS_CONST_MASS, eos_mass_GeV=0.4)):
            q = lb.make_params(8, 8, 0.2, n_xi=nxi, n_theta=nth, n_phi=nph, **bad)
            assert lb.lib.lb_workspace_bytes(ctypes.byref(q)) == 0 and "momentum lattice" in lb.last_error()
    p = lb.make_params(8, 8, 0.2, n_xi=3)
    assert lb.lib.lb_batch_workspace_bytes(ctypes.byref(p), (lb.lb_event * 1)(lb.lb_event(8, 8, 0.2, 0.1)), 1) == 0


def test_upwind_gradient_validation():
    # gradient_form LB_GRAD_UPWIND is defined for the force on F_eq only;
    # its adjoint keeps the gradient's adjoint per phi slice: 2 x 8 values
    # per site instead of 2 (112 more bytes per site)
    p = lb.make_params(8, 8, 0.2, gradient_form=lb.LB_GRAD_UPWIND)
    assert lb.lib.lb_workspace_bytes(ctypes.byref(p)) > 0
    c = lb.make_params(8, 8, 0.2)
    up, ce = lb.lib.lb_adjoint_workspace_bytes(ctypes.byref(p)), lb.lib.lb_adjoint_workspace_bytes(ctypes.byref(c))
    assert up - ce >= 14 * 8 * 64 and up - ce < 14 * 8 * 64 + 256
    q = lb.make_params(8, 8, 0.2, gradient_form=lb.LB_GRAD_UPWIND, force_form=lb.LB_FORCE_WEAK3D)
    assert lb.lib.lb_workspace_bytes(ctypes.byref(q)) == 0 and "gradient_form" in lb.last_error()
    q = lb.make_params(8, 8, 0.2, gradient_form=5)
    assert lb.lib.lb_workspace_bytes(ctypes.byref(q)) == 0


def test_calls_without_context():
    assert lb.lib.lb_step(None, 1, 0.01) == lb.LB_E_STATE
    assert lb.lib.lb_moments(None, None) == lb.LB_E_STATE
    assert lb.lib.lb_status(None) == lb.LB_E_STATE
    assert lb.lib.lb_destroy(None) == lb.LB_OK
    assert lb.lib.lb_adjoint_step(None, 0.5, 0.01, None, None, None, None, None, None, 0) == lb.LB_E_STATE
    assert lb.lib.lb_adjoint_forward_step(None, 0.5, 0.01, None, None, None, None, None, 0) == lb.LB_E_STATE
    assert lb.lib.lb_adjoint_init(None, None, None, None, None, None, None) == lb.LB_E_STATE


def test_adjoint_workspace_size():
    import ctypes
    p = lb.make_params(12, 10, 0.2)
    n = lb.lib.lb_adjoint_workspace_bytes(ctypes.byref(p))
    # predictor state, its adjoint and R0_bar (3 x N x sites doubles), two
    # per-site doubles, the gradient pair and the eta/s partials, 256-aligned
    assert n >= (3 * 200 + 5) * 120 * 8 and n % 256 == 0
    p.nx = 0
    assert lb.lib.lb_adjoint_workspace_bytes(ctypes.byref(p)) == 0


@pytest.mark.parametrize("z0", [1.0, 2.6])
def test_host_lattice_matches_oracle(z0):
    p = lb.make_params(8, 8, 0.2, z0=z0)
    info = lb.lattice_info(p)
    x, w = oq.radial_rule(z0, 5)
    mu, wt = oq.gauss_legendre(5)
    assert np.allclose(info["x"], x, rtol=1e-14, atol=0)
    assert np.allclose(info["w_xi"], w, rtol=1e-13, atol=0)
    assert np.allclose(info["mu"], mu, rtol=0, atol=1e-15)
    assert np.allclose(info["w_th"], wt, rtol=1e-13, atol=0)
    _, c, s = oq.phi_nodes(4)
    assert np.allclose(info["cos"], c, rtol=0, atol=3e-16)
    assert np.allclose(info["sin"], s, rtol=0, atol=3e-16)


@pytest.mark.parametrize("shape", [(5, 5, 4, 1.0), (3, 4, 3, 2.6), (7, 5, 5, 1.0)])
def test_node_table_matches_oracle(shape):
    # lb_node_table (the library's weights and node momenta) against the
    # oracle's lattice, canonical node order
    nxi, nth, nph, z0 = shape
    p = lb.make_params(8, 8, 0.2, z0=z0, n_xi=nxi, n_theta=nth, n_phi=nph)
    t = lb.node_table(p)
    lat = Lattice(nxi, nth, nph, z0)
    assert t.shape == (5, lat.N)
    assert np.allclose(t[0], lat.w, rtol=1e-12, atol=0)
    assert np.allclose(t[1], lat.gamma, rtol=1e-14, atol=0)
    for row, ref in zip(t[2:], (lat.V[1], lat.V[2], lat.V[3])):
        assert np.allclose(row, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))
    n = lb.lib.lb_node_table(ctypes.byref(p), None, 0)
    assert n == 5 * lat.N
    buf = (ctypes.c_double * 4)()
    assert lb.lib.lb_node_table(ctypes.byref(p), buf, 4) == lb.LB_E_ARG


def test_degeneracy():
    # Z T^4/pi^2 (massless Boltzmann gas) = kappa g pi^2 T^4/90
    for kappa, g in [(1.0, 37.0), (2.0, 37.0), (1.5, 16.0)]:
        Z = lb.degeneracy(kappa, g)
        assert abs(Z / math.pi ** 2 - kappa * g * math.pi ** 2 / 90.0) < 1e-14 * Z
    assert lb.make_params(4, 4, 0.1).Z == lb.degeneracy(2.0, 37.0)


@pytest.mark.parametrize("z0", [1.0, 2.6])
def test_factored_operators_equal_oracle_dense_operators(z0):
    # The device applies S1, S2 as mu^2 (A1 x) - (Ath x) and (A2 x) on each
    # phi slice; rebuilt densely they must equal the oracle's literal
    # weak-form matrices of Sec. IV.D.
    p = lb.make_params(8, 8, 0.2, z0=z0)
    info = lb.lattice_info(p)
    lat = Lattice(5, 5, 4, z0)
    I5 = np.eye(5)
    D2 = np.kron(info["A2"], I5)
    D1 = np.kron(info["A1"], I5) * np.tile(info["mu"] ** 2, 5)[:, None] - np.kron(I5, info["Ath"])
    scale1 = np.max(np.abs(lat.D1))
    scale2 = np.max(np.abs(lat.D2))
    assert np.max(np.abs(D1 - lat.D1)) < 1e-11 * scale1
    assert np.max(np.abs(D2 - lat.D2)) < 1e-11 * scale2


@pytest.mark.parametrize("kind", ["s", "p"])
def test_host_eos_matches_oracle(kind):
    if kind == "s":
        p = lb.make_params(8, 8, 0.2, eta_over_s=0.1)
        e = TanhEntropyEoS()
    else:
        p = lb.make_params(8, 8, 0.2, eta_over_s=0.1, eos_kind=lb.LB_EOS_TANH_P, eos_width_GeV=0.03)
        e = TanhEoS(width=0.03)
    T = np.array([0.06, 0.12, 0.17, 0.2, 0.35, 1.0, 2.9])
    out = lb.eos_eval(p, T)
    ref = [e.eps(T), e.p(T), e.s(T), e.M(T), e.B(T), e.eps_kin_eq(T), e.beta(T), e.tau_R(T, 0.1)]
    for i, r in enumerate(ref):
        scale = np.maximum(np.abs(r), 1e-300)
        if i == 4:  # B is a difference of nearly equal pressures at low T
            scale = np.maximum(np.abs(r), 1e-12 * e.p(T))
        assert np.all(np.abs(out[:, i] - r) <= 1e-10 * scale), (i, out[:, i], r)


def test_device_tables_interpolate_exact_eos():
    # The kernels read the EoS from tables on a uniform ln T grid with
    # 4-point Lagrange interpolation: error bound h^4 f''''/ (~43) with
    # h = 1.25e-4.  Check at off-grid temperatures.
    p = lb.make_params(8, 8, 0.2, eta_over_s=0.1)
    rng = np.random.default_rng(0)
    T = np.exp(rng.uniform(np.log(0.05), np.log(3.0), 400))
    ex = lb.eos_eval(p, T)
    tb = lb.eos_eval(p, T, table=True)
    rel = lambda a, b: np.max(np.abs(a - b) / np.abs(b))
    # measured at 2000 off-grid temperatures: ~5e-13 (M, tau_R, B, beta) and
    # ~7e-12 (eps - B, steepest in relative terms at low T)
    assert rel(tb[:, 3], ex[:, 3]) < 2e-12        # M
    assert rel(tb[:, 5], ex[:, 5]) < 2e-11        # eps - B
    assert rel(tb[:, 7], ex[:, 7]) < 2e-12        # tau_R
    assert np.max(np.abs(tb[:, 6] - ex[:, 6])) < 1e-11   # beta
    assert np.max(np.abs(tb[:, 4] - ex[:, 4]) / (np.abs(ex[:, 0]))) < 2e-12  # B relative to eps


def test_const_mass_eos():
    p = lb.make_params(8, 8, 0.2, eos_kind=lb.LB_EOS_CONST_MASS, eos_mass_GeV=0.4, Z=3.0)
    T = np.array([0.1, 0.3, 1.0])
    out = lb.eos_eval(p, T)
    e = ConstMassEoS(3.0, 0.4)
    assert np.allclose(out[:, 0], e.eps(T), rtol=1e-13)
    assert np.allclose(out[:, 3], 0.4) and np.all(out[:, 4] == 0) and np.all(out[:, 6] == 0)


def _tanh_table(n=1200):
    e = TanhEntropyEoS()
    T = np.exp(np.linspace(np.log(0.04), np.log(3.5), n))
    return e, (T, e.s(T), float(e.p(T[:1])[0]))


def test_host_tabulated_eos_matches_oracle():
    from oracle.eos import TabulatedEoS
    e, tab = _tanh_table()
    p = lb.make_params(8, 8, 0.2, eta_over_s=0.1, eos_table=tab)
    o = TabulatedEoS(*tab, Z=p.Z)
    T = np.array([0.06, 0.12, 0.17, 0.2, 0.35, 1.0, 2.9])
    out = lb.eos_eval(p, T)
    ref = [o.eps(T), o.p(T), o.s(T), o.M(T), o.B(T), o.eps_kin_eq(T), o.beta(T), o.tau_R(T, 0.1)]
    for i, r in enumerate(ref):
        scale = np.maximum(np.abs(r), 1e-300)
        if i == 4:
            scale = np.maximum(np.abs(r), 1e-12 * o.p(T))
        assert np.all(np.abs(out[:, i] - r) <= 1e-10 * scale), (i, out[:, i], r)
    # and it is the closed-form EoS to the interpolation error (1200 points)
    ex = lb.eos_eval(lb.make_params(8, 8, 0.2, eta_over_s=0.1), T)
    assert np.max(np.abs(out[:, :4] / ex[:, :4] - 1)) < 1e-6


@pytest.mark.parametrize("b", [0.0, 0.6])
def test_host_tabulated_power_law_is_exact(b):
    # the host's spline reproduces ln(s/T^3) linear in ln T exactly
    A, p0 = 10.0, 2e-5  # 2 pi^2 s/(Z T^3) < 8 on the queried range: M exists
    T = np.exp(np.linspace(np.log(0.04), np.log(3.5), 30))
    p = lb.make_params(8, 8, 0.2, Z=60.0, eos_table=(T, A * T ** (3 + b), p0))
    Tq = np.array([0.055, 0.21, 0.77, 3.3])
    out = lb.eos_eval(p, Tq)
    assert np.allclose(out[:, 2], A * Tq ** (3 + b), rtol=1e-13, atol=0)
    assert np.allclose(out[:, 1], p0 + A * (Tq ** (4 + b) - T[0] ** (4 + b)) / (4 + b), rtol=1e-12, atol=0)


def test_tabulated_eos_validation():
    import ctypes
    T = np.exp(np.linspace(np.log(0.04), np.log(3.5), 20))
    s = 10 * T ** 3
    bad = [
        (T[::-1].copy(), s),                     # not increasing
        (T, -s),                                 # s <= 0
        (T[5:], s[5:]),                          # does not cover T_min = 0.05
    ]
    for Tt, st in bad:
        p = lb.make_params(8, 8, 0.2, Z=60.0, eos_table=(Tt, st, 1e-5))
        assert lb.lib.lb_workspace_bytes(ctypes.byref(p)) == 0
    p = lb.make_params(8, 8, 0.2, Z=60.0, eos_table=(T[:3], s[:3], 1e-5))
    assert lb.lib.lb_workspace_bytes(ctypes.byref(p)) == 0   # fewer than 4 points


def test_host_tabulated_cubic_in_log_t_is_exact():
    # the host spline (its own tridiagonal solve) is exact on a cubic in ln T
    rng = np.random.default_rng(4)
    x = np.sort(rng.uniform(np.log(0.04), np.log(3.5), 25))
    x[0], x[-1] = np.log(0.04), np.log(3.5)
    y = lambda x: 0.5 + 0.3 * x - 0.2 * x ** 2 + 0.05 * x ** 3
    T = np.exp(x)
    p = lb.make_params(8, 8, 0.2, Z=60.0, eos_table=(T, T ** 3 * np.exp(y(x)), 1e-4))
    xq = np.array([-2.9, -1.7, -0.3, 0.9])
    out = lb.eos_eval(p, np.exp(xq))
    assert np.allclose(out[:, 2], np.exp(3 * xq + y(xq)), rtol=1e-12, atol=0)


@pytest.mark.parametrize("z0", [1.0, 2.6])
def test_host_strong_form_operators_match_oracle(z0):
    # LB_OPS_STRONG: the host's barycentric derivative matrices against the
    # oracle's tensor-interpolant construction
    p = lb.make_params(8, 8, 0.2, z0=z0, operator_form=lb.LB_OPS_STRONG)
    info = lb.lattice_info(p)
    lat = Lattice(5, 5, 4, z0, form="strong")
    I5 = np.eye(5)
    D2 = np.kron(info["A2"], I5)
    D1 = np.kron(info["A1"], I5) * np.tile(info["mu"] ** 2, 5)[:, None] - np.kron(I5, info["Ath"])
    assert np.max(np.abs(D1 - lat.D1)) < 1e-11 * np.max(np.abs(lat.D1))
    assert np.max(np.abs(D2 - lat.D2)) < 1e-11 * np.max(np.abs(lat.D2))
    p.operator_form = 7
    assert lb.lib.lb_workspace_bytes(ctypes.byref(p)) == 0


def test_force_form_validation():
    # LB_FORCE_WEAK3D is a valid parameter set; unknown force forms are not
    p = lb.make_params(8, 8, 0.2, force_form=lb.LB_FORCE_WEAK3D)
    assert lb.lib.lb_workspace_bytes(ctypes.byref(p)) > 0
    p.force_form = 2
    assert lb.lib.lb_workspace_bytes(ctypes.byref(p)) == 0
    assert "force_form" in lb.last_error()


def test_particle_number_validation():
    # LB_N_CONSERVED needs the constant-mass EoS; mu_over_T0 needs it too
    p = lb.make_params(8, 8, 0.2, eos_kind=lb.LB_EOS_CONST_MASS, eos_mass_GeV=0.4, Z=3.0,
                       particle_number=lb.LB_N_CONSERVED, mu_over_T0=0.5)
    assert lb.lib.lb_workspace_bytes(ctypes.byref(p)) > 0
    p.eos_kind = lb.LB_EOS_TANH_S
    assert lb.lib.lb_workspace_bytes(ctypes.byref(p)) == 0
    assert "LB_EOS_CONST_MASS" in lb.last_error()
    q = lb.make_params(8, 8, 0.2, mu_over_T0=0.5)
    assert lb.lib.lb_workspace_bytes(ctypes.byref(q)) == 0
    q.mu_over_T0, q.particle_number = 0.0, 2
    assert lb.lib.lb_workspace_bytes(ctypes.byref(q)) == 0
