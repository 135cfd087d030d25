"""lb_adjoint_step_noalloc (the adjoint step on the library's static device
scratch, for callers that cannot allocate) against lb_adjoint_step with a
caller's workspace, through the C ABI: two calls in a row on the same
device, the second on a smaller grid, each equal bit for bit (the same
kernels on the same inputs); a grid beyond the scratch's limit is refused
on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1108_5561_amd as lb  # noqa: E402
from paper_1108_5561_amd import workloads as wl  # noqa: E402

DEV = "cuda:0"


def _case(nx, ny, dx, seed, steps=3, dtau=0.005):
    p = lb.make_params(nx, ny, dx, eta_over_s=0.12)
    bg = lb.eos_eval(p, [0.25])[0, 0] / lb.HBARC ** 3
    e0 = bg + wl.hot_spots(nx, ny, dx, n_spots=5, width=0.4, disk_radius=0.3 * min(nx, ny) * dx, seed=seed)
    c = lb.Context(p, torch.from_numpy(e0).to(DEV))
    c.step(steps, dtau)
    F, L, tau = c.get_state()
    rng = np.random.default_rng(seed)
    aF = torch.from_numpy(rng.standard_normal(tuple(F.shape))).to(DEV)
    aL = torch.from_numpy(rng.standard_normal(tuple(L.shape))).to(DEV)
    return c, F, L, tau, aF, aL, dtau


def _both(c, F, L, tau, aF, aL, dtau):
    ws = c.adjoint_workspace()
    a1F, a1L = aF.clone(), aL.clone()
    g1 = torch.zeros(1, dtype=torch.float64, device=DEV)
    c.adjoint_step(tau, dtau, F, L, a1F, a1L, g1, ws)
    a2F, a2L = aF.clone(), aL.clone()
    g2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    rc = lb.lib.lb_adjoint_step_noalloc(c._ctx, float(tau), float(dtau), F.data_ptr(), L.data_ptr(),
                                        a2F.data_ptr(), a2L.data_ptr(), g2.data_ptr())
    assert rc == lb.LB_OK, lb.last_error()
    assert c.status() == lb.LB_OK
    return (a1F, a1L, g1), (a2F, a2L, g2)


def test_noalloc_adjoint_step_equals_workspace_step():
    for nx, ny, dx, seed in ((40, 36, 0.12, 1), (13, 9, 0.15, 2)):   # second call: smaller grid
        print(f"noalloc adjoint step on {nx}x{ny}", flush=True)
        c, F, L, tau, aF, aL, dtau = _case(nx, ny, dx, seed)
        ref, got = _both(c, F, L, tau, aF, aL, dtau)
        for r, g in zip(ref, got):
            assert torch.equal(r, g)
        assert float(ref[2]) != 0.0
        c.close()


def test_noalloc_rejects_grids_beyond_the_scratch():
    p = lb.make_params(140, 140, 0.1, eta_over_s=0.12)     # 19600 sites x 4840 B > 80 MiB
    e0 = torch.full((140, 140), float(lb.eos_eval(p, [0.3])[0, 0] / lb.HBARC ** 3), dtype=torch.float64,
                    device=DEV)
    c = lb.Context(p, e0)
    F, L, tau = c.get_state()
    aF, aL = torch.zeros_like(F), torch.zeros_like(L)
    g = torch.zeros(1, dtype=torch.float64, device=DEV)
    rc = lb.lib.lb_adjoint_step_noalloc(c._ctx, float(tau), 0.005, F.data_ptr(), L.data_ptr(), aF.data_ptr(),
                                        aL.data_ptr(), g.data_ptr())
    assert rc == lb.LB_E_ARG and "scratch" in lb.last_error()
    assert lb.lib.lb_adjoint_step_noalloc(None, 0.5, 0.005, None, None, None, None, None) == lb.LB_E_STATE
    c.close()
