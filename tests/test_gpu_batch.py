"""Batched form on the GPU: every event of a batch advances exactly as the
same event in a context of its own (lb_step, itself checked against the
oracle in test_gpu_parity.py), for every kernel variant, across the graph
replays of 48 steps and step counts that are not multiples of it."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1108_5561_amd as lb  # noqa: E402
from paper_1108_5561_amd import workloads as wl  # noqa: E402

DEV = "cuda:0"
EVENTS = [(8, 8, 0.3, 0.08), (13, 7, 0.25, 0.2), (20, 16, 0.2, 0.12), (1, 3, 0.3, 0.3)]
DTAU = 0.01


def _e0(params, nx, ny, dx, seed, T_bg=0.2):
    bg = lb.eos_eval(params, [T_bg])[0, 0] / lb.HBARC ** 3
    spots = wl.hot_spots(nx, ny, dx, n_spots=4, width=0.6, disk_radius=0.3 * max(nx, ny) * dx,
                         mean_amplitude=10.0, seed=seed)
    return torch.from_numpy(bg + spots).to(DEV)


def _setup(precision):
    p = lb.make_params(8, 8, 0.3, precision=precision)
    e0s = [_e0(p, nx, ny, dx, 100 + i) for i, (nx, ny, dx, _) in enumerate(EVENTS)]
    return p, e0s


def _single(precision, e0s, n_steps):
    out = []
    for (nx, ny, dx, eta), e0 in zip(EVENTS, e0s):
        q = lb.make_params(nx, ny, dx, eta_over_s=eta, precision=precision)
        c = lb.Context(q, e0)
        c.step(n_steps, DTAU)
        F, l, t = c.get_state()
        out.append((F, l, t, c.moments()))
        assert c.status() == lb.LB_OK
        c.close()
    return out


@pytest.mark.parametrize("precision", [lb.LB_FP64, lb.LB_FP32_FP64MATCH])
def test_batch_equals_single_contexts_every_variant(precision):
    p, e0s = _setup(precision)
    n1, n2 = 50, 47   # 48 + 2 direct steps, then 1 + 46 direct (rotation not at 0)
    ref = _single(precision, e0s, n1 + n2)
    nvar = 12 if precision == lb.LB_FP32_FP64MATCH else 3
    for v in range(nvar):
        b = lb.Batch(p, EVENTS, e0s)
        b.set_variant(v)
        b.step(n1, DTAU)
        b.step(n2, DTAU)
        for e, (F, l, t, obs) in enumerate(ref):
            Fb, lb_, tb = b.get_state(e)
            assert tb == t
            assert torch.equal(Fb, F), f"variant {v} event {e}"
            assert torch.equal(lb_, l)
            assert torch.equal(b.moments(e), obs)
        assert b.status() == lb.LB_OK
        b.close()


def _mode_params(mode, nx, ny, dx, eta, precision):
    if mode == "force3d":
        return lb.make_params(nx, ny, dx, eta_over_s=eta, precision=precision, force_form=lb.LB_FORCE_WEAK3D)
    if mode == "upwind":
        return lb.make_params(nx, ny, dx, eta_over_s=eta, precision=precision, gradient_form=lb.LB_GRAD_UPWIND)
    force = lb.LB_FORCE_WEAK3D if mode == "both" else lb.LB_FORCE_FEQ
    grad = lb.LB_GRAD_UPWIND if mode == "upwind_mu" else lb.LB_GRAD_CENTRED
    return lb.make_params(nx, ny, dx, eta_over_s=eta, precision=precision, eos_kind=lb.LB_EOS_CONST_MASS,
                          eos_mass_GeV=0.4, Z=3.0, particle_number=lb.LB_N_CONSERVED, mu_over_T0=0.3,
                          force_form=force, gradient_form=grad)


@pytest.mark.parametrize("mode", ["force3d", "mu", "both", "upwind", "upwind_mu"])
@pytest.mark.parametrize("precision", [lb.LB_FP64, lb.LB_FP32_FP64MATCH])
def test_batch_modes_equal_single_contexts(precision, mode):
    # the weak-form 3-D force and the conserved particle number in the
    # batched form: every variant, every event bitwise as lb_step
    p = _mode_params(mode, 8, 8, 0.3, 0.1, precision)
    # with the particle number conserved the heavy gas cools faster in the
    # expansion: a hotter background keeps the cold sites inside the EoS range
    T_bg = 0.35 if mode in ("mu", "both", "upwind_mu") else 0.2
    e0s = [_e0(p, nx, ny, dx, 200 + i, T_bg) for i, (nx, ny, dx, _) in enumerate(EVENTS)]
    n1, n2 = 50, 2
    ref = []
    for (nx, ny, dx, eta), e0 in zip(EVENTS, e0s):
        c = lb.Context(_mode_params(mode, nx, ny, dx, eta, precision), e0)
        c.step(n1 + n2, DTAU)
        assert c.status() == lb.LB_OK
        ref.append(c.get_state()[:2])
        c.close()
    for v in range(3):
        print(f"batch {mode} precision {precision} variant {v}", flush=True)
        b = lb.Batch(p, EVENTS, e0s)
        b.set_variant(v)
        b.step(n1, DTAU)
        b.step(n2, DTAU)
        assert b.status() == lb.LB_OK
        for e, (F, l) in enumerate(ref):
            Fb, lb_, _ = b.get_state(e)
            assert torch.equal(Fb, F), f"variant {v} event {e}"
            assert torch.equal(lb_, l)
        with pytest.raises(lb.LbError):
            b.set_variant(3)
        b.close()


def test_batch_graph_replays_match_direct_steps():
    """96 steps as two graph replays equal 96 steps taken one by one."""
    p, e0s = _setup(lb.LB_FP32_FP64MATCH)
    a = lb.Batch(p, EVENTS, e0s)
    b = lb.Batch(p, EVENTS, e0s)
    a.set_variant(1)
    b.set_variant(1)
    a.step(96, DTAU)
    for _ in range(96):
        b.step(1, DTAU)
    for e in range(len(EVENTS)):
        Fa, la, ta = a.get_state(e)
        Fb, lb_, tb = b.get_state(e)
        assert ta == tb and torch.equal(Fa, Fb) and torch.equal(la, lb_)


def test_batch_tune_and_errors():
    p, e0s = _setup(lb.LB_FP32_FP64MATCH)
    b = lb.Batch(p, EVENTS, e0s)
    v, ms = b.tune(DTAU)
    assert 0 <= v < 12 and len(ms) == 12 and all(m > 0 for m in ms) and ms[v] == min(ms)
    F0, l0, t0 = b.get_state(2)
    F1, l1, t1 = b.get_state(2)
    assert t0 == t1 and torch.equal(F0, F1)   # tuning left the state alone
    with pytest.raises(lb.LbError) as ei:
        b.step(1, 1.0)                         # CFL far above 0.5
    assert ei.value.code == lb.LB_E_ARG
    with pytest.raises(lb.LbError):
        b.get_state(len(EVENTS))
    with pytest.raises(lb.LbError):
        b.set_variant(12)
    assert b.status() == lb.LB_OK


def test_large_grid_mode_equals_cached_tiles():
    """A state above the last-level-cache threshold (3 x 800 B x sites >
    192 MiB) runs lb_step with 8-row tiles and streaming stores; its result
    equals the batched kernel's 4-row cached variant bit for bit."""
    nx, ny, dx = 320, 304, 0.05
    p = lb.make_params(nx, ny, dx, precision=lb.LB_FP32_FP64MATCH, eta_over_s=0.12)
    bg = lb.eos_eval(p, [0.25])[0, 0] / lb.HBARC ** 3
    e0 = torch.from_numpy(bg + wl.hot_spots(nx, ny, dx, n_spots=8, width=0.6, disk_radius=4.0, seed=41)).to(DEV)
    c = lb.Context(p, e0)
    c.step(3, DTAU)
    F, l, t = c.get_state()
    b = lb.Batch(p, [(nx, ny, dx, 0.12)], [e0])
    b.set_variant(1)
    b.step(3, DTAU)
    Fb, lb_, tb = b.get_state(0)
    assert tb == t and torch.equal(Fb, F) and torch.equal(lb_, l)
    assert c.status() == lb.LB_OK and b.status() == lb.LB_OK


def test_graph_replays_after_step_size_change():
    """48 steps replayed at one dtau, then 48 at another (the graphs are
    re-captured; the first replay may still be running when they are
    dropped), equal the same steps taken one by one."""
    p, e0s = _setup(lb.LB_FP32_FP64MATCH)
    a = lb.Batch(p, EVENTS, e0s)
    b = lb.Batch(p, EVENTS, e0s)
    a.set_variant(1)
    b.set_variant(1)
    for dt in (DTAU, 0.6 * DTAU, DTAU):
        a.step(48, dt)
        for _ in range(48):
            b.step(1, dt)
    assert a.status() == lb.LB_OK and b.status() == lb.LB_OK
    for e in range(len(EVENTS)):
        Fa, la, ta = a.get_state(e)
        Fb, lb_, tb = b.get_state(e)
        assert ta == tb and torch.equal(Fa, Fb) and torch.equal(la, lb_)


def test_full_batch_workload_sampled_events():
    """The 64-event batched workload at the bench's launch configuration
    (tuned variant, 96 steps as two 48-step graph replays): the smallest,
    the largest and two random events equal the same events advanced alone
    with lb_step, bit for bit; and one further batched step of the smallest
    and the largest event agrees with the FP64 oracle at sampled sites
    (9 x 9 periodic windows: the corrector reaches 4 sites) to the FP32
    one-step bar 1e-5."""
    w = wl.WORKLOADS["batch"]
    events = wl.batch_events(w["n_events"], w["n_min"], w["n_max"], w["box"])
    p = lb.make_params(8, 8, 0.1, tau0_fm=w["tau0"], precision=lb.LB_FP32_FP64MATCH)
    bg = lb.eos_eval(p, [0.25])[0, 0] / lb.HBARC ** 3
    spots = wl.batch_hot_spots(events)
    e0s = [torch.from_numpy(bg + h).to(DEV) for h in spots]
    dtau = (w["tau1"] - w["tau0"]) / w["steps"]
    b = lb.Batch(p, events, e0s)
    b.tune(dtau)
    b.step(96, dtau)
    assert b.status() == lb.LB_OK
    sizes = [nx * ny for nx, ny, _, _ in events]
    rng = np.random.default_rng(5)
    picks = {int(np.argmin(sizes)), int(np.argmax(sizes))} | set(int(i) for i in rng.integers(0, len(events), 2))
    for e in sorted(picks):
        nx, ny, dx, eta = events[e]
        q = lb.make_params(nx, ny, dx, tau0_fm=w["tau0"], eta_over_s=eta, precision=lb.LB_FP32_FP64MATCH)
        c = lb.Context(q, e0s[e])
        c.step(96, dtau)
        F, l, t = c.get_state()
        Fb, lb_, tb = b.get_state(e)
        assert tb == t and torch.equal(Fb, F) and torch.equal(lb_, l), f"event {e} ({nx}x{ny})"
        assert c.status() == lb.LB_OK
        c.close()
    # oracle contact: one more batched step from the replayed state
    from oracle import step as st
    from oracle.eos import TanhEntropyEoS
    from oracle.lattice import Lattice
    from _helpers import patch, tmunu_rel_err
    lat, eos = Lattice(5, 5, 4, 1.0), TanhEntropyEoS()
    small, large = int(np.argmin(sizes)), int(np.argmax(sizes))
    before = {e: b.get_state(e) for e in (small, large)}
    b.step(1, dtau)
    assert b.status() == lb.LB_OK
    for e in (small, large):
        nx, ny, dx, eta = events[e]
        F0, l0, tau = (x.cpu().numpy() if torch.is_tensor(x) else x for x in before[e])
        obs = b.moments(e).cpu().numpy()
        prm = st.Params(dx=dx, eta_over_s=eta)
        hot = np.unravel_index(np.argmax(e0s[e].cpu().numpy()), (ny, nx))
        rs = np.random.default_rng(100 + e)
        for (cy, cx) in [hot, (0, 0), (ny - 1, nx - 1)] + [tuple(rs.integers(0, min(nx, ny), 2)) for _ in range(3)]:
            Fp, lp = patch(F0, cy, cx, 4), patch(l0, cy, cx, 4)
            Fo, lo = st.heun_step(lat, eos, prm, Fp, lp, tau, dtau)
            ref = st.observables(lat, eos, prm, Fo, lo)[:, 4:5, 4:5]
            err = tmunu_rel_err(obs[:, cy:cy + 1, cx:cx + 1], ref)
            assert err < 1e-5, (e, cy, cx, err)
    b.close()
