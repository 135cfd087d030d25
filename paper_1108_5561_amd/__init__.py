"""Python binding of liblbmi.so, the C-ABI library of the relativistic
quasiparticle lattice-Boltzmann step (see include/lb.h for the contract).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  Importing this
module fails loudly if the library has not been built
(``python paper_1108_5561_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmi.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "lb.h")

LB_OK, LB_E_ARG, LB_E_HIP, LB_E_EOS, LB_E_MATCH, LB_E_NONFINITE, LB_E_STATE, LB_E_NOTIMPL = 0, -1, -2, -3, -4, -5, -6, -7
LB_FP64, LB_FP32_FP64MATCH = 0, 1
LB_TAUR_CE, LB_TAUR_MASSLESS = 0, 1
LB_METRIC_MILNE, LB_METRIC_MINKOWSKI = 0, 1
LB_EOS_TANH_P, LB_EOS_CONST_MASS, LB_EOS_TANH_S, LB_EOS_TABLE = 0, 1, 2, 3
LB_OPS_WEAK, LB_OPS_STRONG = 0, 1
LB_FORCE_FEQ, LB_FORCE_WEAK3D = 0, 1
LB_N_FREE, LB_N_CONSERVED = 0, 1
LB_GRAD_CENTRED, LB_GRAD_UPWIND = 0, 1
HBARC = 0.1973269804  # GeV fm
N_OBS = 14
OBS_NAMES = ("Ttt", "Ttx", "Tty", "Txx", "Txy", "Tyy", "TYY", "Nt", "Nx", "Ny", "T", "ux", "uy", "M")

_ERR_NAMES = {LB_E_ARG: "LB_E_ARG", LB_E_HIP: "LB_E_HIP", LB_E_EOS: "LB_E_EOS", LB_E_MATCH: "LB_E_MATCH",
              LB_E_NONFINITE: "LB_E_NONFINITE", LB_E_STATE: "LB_E_STATE", LB_E_NOTIMPL: "LB_E_NOTIMPL"}


class LbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class lb_params(ctypes.Structure):
    _fields_ = [
        ("n_xi", ctypes.c_int32), ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
        ("z0", ctypes.c_double), ("Z", ctypes.c_double),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx_fm", ctypes.c_double), ("tau0_fm", ctypes.c_double), ("eta_over_s", ctypes.c_double),
        ("taur_rule", ctypes.c_int32), ("precision", ctypes.c_int32), ("metric", ctypes.c_int32),
        ("eos_kind", ctypes.c_int32),
        ("eos_g", ctypes.c_double), ("eos_Tc_GeV", ctypes.c_double), ("eos_width_GeV", ctypes.c_double),
        ("eos_mass_GeV", ctypes.c_double), ("T_min_GeV", ctypes.c_double), ("T_max_GeV", ctypes.c_double),
        ("eos_T_GeV", ctypes.POINTER(ctypes.c_double)), ("eos_s_GeV3", ctypes.POINTER(ctypes.c_double)),
        ("eos_p0_GeV4", ctypes.c_double), ("eos_n", ctypes.c_int32),
        ("operator_form", ctypes.c_int32), ("force_form", ctypes.c_int32),
        ("particle_number", ctypes.c_int32), ("mu_over_T0", ctypes.c_double),
        ("gradient_form", ctypes.c_int32),
    ]


class lb_event(ctypes.Structure):
    """One event of a batch (include/lb.h)."""
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx_fm", ctypes.c_double),
                ("eta_over_s", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1108_5561_amd/build.py`")
    # torch bundles its own HIP runtime under the same soname
    # (libamdhip64.so.7).  Loading torch first makes the dynamic loader bind
    # the library to that copy, so one HIP runtime serves the process and
    # device pointers and streams from torch are valid in the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(lb_params)
    vp, dp, i32, i64, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "lb_workspace_bytes": (sz, [P]),
        "lb_init": (ctypes.c_int, [ctypes.POINTER(vp), P, vp, sz, vp, vp, vp, vp]),
        "lb_step": (ctypes.c_int, [vp, i32, ctypes.c_double]),
        "lb_moments": (ctypes.c_int, [vp, vp]),
        "lb_get_state": (ctypes.c_int, [vp, vp, vp, dp]),
        "lb_set_state": (ctypes.c_int, [vp, vp, vp, ctypes.c_double]),
        "lb_adjoint_workspace_bytes": (sz, [P]),
        "lb_adjoint_forward_step": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, vp, sz]),
        "lb_adjoint_step": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, vp, vp, sz]),
        "lb_adjoint_step_noalloc": (ctypes.c_int, [vp, ctypes.c_double, ctypes.c_double, vp, vp, vp, vp, vp]),
        "lb_adjoint_init": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "lb_status": (ctypes.c_int, [vp]),
        "lb_destroy": (ctypes.c_int, [vp]),
        "lb_last_error": (ctypes.c_char_p, []),
        "lb_lattice_info": (i64, [P, dp, i64]),
        "lb_node_table": (i64, [P, dp, i64]),
        "lb_degeneracy": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
        "lb_eos_eval": (ctypes.c_int, [P, i64, dp, dp, i32]),
        "lb_profile": (ctypes.c_int, [vp, i32]),
        "lb_profile_read": (ctypes.c_int, [vp, dp, ctypes.POINTER(i64)]),
        "lb_profile_stage": (ctypes.c_int, [vp, i32, i32, ctypes.c_double, dp]),
        "lb_batch_workspace_bytes": (sz, [P, ctypes.POINTER(lb_event), i32]),
        "lb_batch_init": (ctypes.c_int, [ctypes.POINTER(vp), P, ctypes.POINTER(lb_event), i32, vp, sz,
                                         ctypes.POINTER(vp), vp]),
        "lb_batch_tune": (ctypes.c_int, [vp, ctypes.c_double, ctypes.POINTER(i32), dp]),
        "lb_batch_step": (ctypes.c_int, [vp, i32, ctypes.c_double]),
        "lb_batch_set_variant": (ctypes.c_int, [vp, i32]),
        "lb_batch_moments": (ctypes.c_int, [vp, i32, vp]),
        "lb_batch_get_state": (ctypes.c_int, [vp, i32, vp, vp, dp]),
        "lb_batch_status": (ctypes.c_int, [vp]),
        "lb_batch_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def header_functions():
    """Names of the functions declared in include/lb.h."""
    txt = open(HEADER_PATH).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", txt)))


def last_error():
    return lib.lb_last_error().decode()


def check(rc):
    if rc != LB_OK:
        raise LbError(rc, last_error())
    return rc


def degeneracy(kappa, g):
    """Z of eq. (feq) for kappa times the Stefan-Boltzmann pressure of g
    degrees of freedom (lb_degeneracy)."""
    return float(lib.lb_degeneracy(float(kappa), float(g)))


def make_params(nx, ny, dx_fm, tau0_fm=0.5, eta_over_s=0.08, precision=LB_FP64, metric=LB_METRIC_MILNE,
                taur_rule=LB_TAUR_CE, eos_kind=LB_EOS_TANH_S, eos_g=37.0, eos_Tc_GeV=0.17, eos_width_GeV=0.02,
                eos_mass_GeV=0.0, kappa=2.0, Z=None, z0=1.0, n_xi=5, n_theta=5, n_phi=4,
                T_min_GeV=0.05, T_max_GeV=3.0, eos_table=None, operator_form=LB_OPS_WEAK,
                force_form=LB_FORCE_FEQ, particle_number=LB_N_FREE, mu_over_T0=0.0,
                gradient_form=LB_GRAD_CENTRED):
    """Parameters of a run.  eos_table = (T [GeV], s [GeV^3], p(T[0]) [GeV^4])
    selects LB_EOS_TABLE with the caller's entropy density (the arrays are
    kept alive by the returned object)."""
    p = lb_params()
    if eos_table is not None:
        import numpy as np
        Tt = np.ascontiguousarray(eos_table[0], dtype=np.float64)
        st = np.ascontiguousarray(eos_table[1], dtype=np.float64)
        dptr = ctypes.POINTER(ctypes.c_double)
        p.eos_T_GeV, p.eos_s_GeV3 = Tt.ctypes.data_as(dptr), st.ctypes.data_as(dptr)
        p.eos_p0_GeV4, p.eos_n = float(eos_table[2]), int(Tt.size)
        p._eos_keep = (Tt, st)
        eos_kind = LB_EOS_TABLE
    p.n_xi, p.n_theta, p.n_phi, p.z0 = n_xi, n_theta, n_phi, z0
    p.Z = degeneracy(kappa, eos_g) if Z is None else Z
    p.nx, p.ny, p.dx_fm, p.tau0_fm, p.eta_over_s = nx, ny, dx_fm, tau0_fm, eta_over_s
    p.taur_rule, p.precision, p.metric, p.eos_kind = taur_rule, precision, metric, eos_kind
    p.eos_g, p.eos_Tc_GeV, p.eos_width_GeV, p.eos_mass_GeV = eos_g, eos_Tc_GeV, eos_width_GeV, eos_mass_GeV
    p.T_min_GeV, p.T_max_GeV = T_min_GeV, T_max_GeV
    p.operator_form = operator_form
    p.force_form = force_form
    p.particle_number, p.mu_over_T0 = particle_number, mu_over_T0
    p.gradient_form = gradient_form
    return p


def workspace_bytes(p):
    n = lib.lb_workspace_bytes(ctypes.byref(p))
    if n == 0:
        raise LbError(LB_E_ARG, last_error())
    return n


def lattice_info(p):
    """dict of the lattice and factored operators (lb_lattice_info)."""
    import numpy as np
    n = lib.lb_lattice_info(ctypes.byref(p), None, 0)
    if n < 0:
        raise LbError(int(n), last_error())
    buf = (ctypes.c_double * n)()
    r = lib.lb_lattice_info(ctypes.byref(p), buf, n)
    if r < 0:
        raise LbError(int(r), last_error())
    a = np.frombuffer(buf, dtype=np.float64).copy()
    nxi, nth, nph = p.n_xi, p.n_theta, 2 * p.n_phi
    out, o = {}, 0
    for name, size, shape in [("x", nxi, None), ("w_xi", nxi, None), ("mu", nth, None), ("w_th", nth, None),
                              ("cos", nph, None), ("sin", nph, None), ("A1", nxi * nxi, (nxi, nxi)),
                              ("A2", nxi * nxi, (nxi, nxi)), ("Ath", nth * nth, (nth, nth))]:
        v = a[o:o + size]
        out[name] = v.reshape(shape) if shape else v
        o += size
    return out


def eos_eval(p, T, table=False):
    """(n, 8) array: eps, p, s, M, B, eps-B, beta, tau_R (lb_eos_eval)."""
    import numpy as np
    T = np.ascontiguousarray(np.atleast_1d(np.asarray(T, dtype=np.float64)))
    out = np.zeros((T.size, 8))
    dptr = ctypes.POINTER(ctypes.c_double)
    check(lib.lb_eos_eval(ctypes.byref(p), T.size, T.ctypes.data_as(dptr), out.ctypes.data_as(dptr), int(table)))
    return out


class Context:
    """One lattice-Boltzmann state on the current GPU (lb_init .. lb_destroy).

    Device memory (workspace, inputs, outputs) is held in torch tensors; the
    library runs on torch's current stream.
    """

    def __init__(self, params, e0, ux0=None, uy0=None, device=None):
        import torch
        self.torch = torch
        self.params = params
        dev = e0.device if device is None else torch.device(device)
        if dev.type != "cuda":
            raise LbError(LB_E_ARG, "inputs must be GPU tensors")
        for t in (e0, ux0, uy0):
            if t is not None and (t.dtype != torch.float64 or tuple(t.shape) != (params.ny, params.nx)
                                  or not t.is_contiguous() or t.device != dev):
                raise LbError(LB_E_ARG, "e0/ux0/uy0 must be contiguous float64 [ny, nx] on the same GPU")
        self.device = dev
        nbytes = workspace_bytes(params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        self._ctx = ctypes.c_void_p()
        check(lib.lb_init(ctypes.byref(self._ctx), ctypes.byref(params), self.workspace.data_ptr(), nbytes,
                          e0.data_ptr(), ux0.data_ptr() if ux0 is not None else None,
                          uy0.data_ptr() if uy0 is not None else None, self.stream.cuda_stream))
        self.N = params.n_xi * params.n_theta * 2 * params.n_phi

    def step(self, n_steps, dtau_fm):
        check(lib.lb_step(self._ctx, int(n_steps), float(dtau_fm)))

    def moments(self, out=None):
        torch = self.torch
        if out is None:
            out = torch.empty((N_OBS, self.params.ny, self.params.nx), dtype=torch.float64, device=self.device)
        check(lib.lb_moments(self._ctx, out.data_ptr()))
        return out

    def get_state(self):
        torch = self.torch
        F = torch.empty((self.N, self.params.ny, self.params.nx), dtype=torch.float64, device=self.device)
        lnM = torch.empty((self.params.ny, self.params.nx), dtype=torch.float64, device=self.device)
        tau = ctypes.c_double()
        check(lib.lb_get_state(self._ctx, F.data_ptr(), lnM.data_ptr(), ctypes.byref(tau)))
        return F, lnM, tau.value

    def set_state(self, F, lnM, tau_fm):
        torch = self.torch
        if F.dtype != torch.float64 or lnM.dtype != torch.float64 or not F.is_contiguous() or not lnM.is_contiguous():
            raise LbError(LB_E_ARG, "F and lnM must be contiguous float64")
        if tuple(F.shape) != (self.N, self.params.ny, self.params.nx) or tuple(lnM.shape) != (self.params.ny, self.params.nx):
            raise LbError(LB_E_ARG, "state shape mismatch")
        check(lib.lb_set_state(self._ctx, F.data_ptr(), lnM.data_ptr(), float(tau_fm)))

    def status(self):
        return lib.lb_status(self._ctx)

    def profile(self, enable):
        check(lib.lb_profile(self._ctx, int(enable)))

    def profile_read(self):
        ms = (ctypes.c_double * 2)()
        cnt = (ctypes.c_int64 * 2)()
        check(lib.lb_profile_read(self._ctx, ms, cnt))
        return (ms[0], ms[1]), (cnt[0], cnt[1])

    def profile_stage(self, stage, n, dtau_fm):
        """Mean milliseconds of one predictor (0) or corrector (1) launch over
        n back-to-back launches; the state is left unchanged."""
        ms = ctypes.c_double()
        check(lib.lb_profile_stage(self._ctx, int(stage), int(n), float(dtau_fm), ctypes.byref(ms)))
        return ms.value

    # ---- differentiable form (lb_adjoint_*) ----
    def _state_check(self, *ts):
        torch = self.torch
        shapes = [(self.N, self.params.ny, self.params.nx), (self.params.ny, self.params.nx)]
        for t in ts:
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device or tuple(t.shape) not in shapes:
                raise LbError(LB_E_ARG, "states and adjoints must be contiguous float64 [N, ny, nx] / [ny, nx] on the context's GPU")

    def adjoint_workspace(self):
        """A device buffer of lb_adjoint_workspace_bytes for this context."""
        n = lib.lb_adjoint_workspace_bytes(ctypes.byref(self.params))
        if n == 0:
            raise LbError(LB_E_ARG, last_error())
        return self.torch.empty(n, dtype=self.torch.uint8, device=self.device)

    def adjoint_forward_step(self, tau_fm, dtau_fm, F, lnM, ws):
        """The differentiated FP64 step from (F, lnM) at tau: new (F, lnM)."""
        self._state_check(F, lnM)
        Fo, Lo = self.torch.empty_like(F), self.torch.empty_like(lnM)
        check(lib.lb_adjoint_forward_step(self._ctx, float(tau_fm), float(dtau_fm), F.data_ptr(), lnM.data_ptr(),
                                          Fo.data_ptr(), Lo.data_ptr(), ws.data_ptr(), ws.numel()))
        return Fo, Lo

    def adjoint_step(self, tau_fm, dtau_fm, F, lnM, adj_F, adj_lnM, grad_eta, ws):
        """In place: (adj_F, adj_lnM) <- transpose of the step at (F, lnM, tau)
        applied to them; grad_eta (one float64 on the GPU) += d/d(eta/s)."""
        self._state_check(F, lnM, adj_F, adj_lnM)
        check(lib.lb_adjoint_step(self._ctx, float(tau_fm), float(dtau_fm), F.data_ptr(), lnM.data_ptr(),
                                  adj_F.data_ptr(), adj_lnM.data_ptr(), grad_eta.data_ptr(), ws.data_ptr(),
                                  ws.numel()))

    def adjoint_step_noalloc(self, tau_fm, dtau_fm, F, lnM, adj_F, adj_lnM, grad_eta):
        """As adjoint_step, with the library's static device scratch instead
        of a workspace (lb_adjoint_step_noalloc; allocates nothing)."""
        self._state_check(F, lnM, adj_F, adj_lnM)
        check(lib.lb_adjoint_step_noalloc(self._ctx, float(tau_fm), float(dtau_fm), F.data_ptr(), lnM.data_ptr(),
                                          adj_F.data_ptr(), adj_lnM.data_ptr(), grad_eta.data_ptr()))

    def adjoint_init(self, e0, adj_F, adj_lnM, ux0=None, uy0=None):
        """dL/d e0 [ny, nx] from the adjoint of the initial state."""
        self._state_check(e0, adj_F, adj_lnM)
        g = self.torch.empty_like(e0)
        check(lib.lb_adjoint_init(self._ctx, e0.data_ptr(), ux0.data_ptr() if ux0 is not None else None,
                                  uy0.data_ptr() if uy0 is not None else None, adj_F.data_ptr(),
                                  adj_lnM.data_ptr(), g.data_ptr()))
        return g

    def close(self):
        if self._ctx:
            lib.lb_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many events advanced together (lb_batch_init .. lb_batch_destroy):
    events is a list of (nx, ny, dx_fm, eta_over_s), e0s the matching list
    of contiguous float64 [ny, nx] GPU tensors; params gives the shared
    lattice, EoS, precision, metric and tau0."""

    def __init__(self, params, events, e0s):
        import torch
        self.torch = torch
        self.params = params
        if len(events) != len(e0s) or not events:
            raise LbError(LB_E_ARG, "need one e0 per event")
        dev = e0s[0].device
        for (nx, ny, _, _), t in zip(events, e0s):
            if t.dtype != torch.float64 or tuple(t.shape) != (ny, nx) or not t.is_contiguous() or t.device != dev:
                raise LbError(LB_E_ARG, "each e0 must be a contiguous float64 [ny, nx] GPU tensor")
        self.device = dev
        self.events = [tuple(e) for e in events]
        n = len(events)
        self._ev = (lb_event * n)(*[lb_event(int(a), int(b), float(c), float(d)) for a, b, c, d in events])
        nbytes = lib.lb_batch_workspace_bytes(ctypes.byref(params), self._ev, n)
        if nbytes == 0:
            raise LbError(LB_E_ARG, last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in e0s])
        self._b = ctypes.c_void_p()
        check(lib.lb_batch_init(ctypes.byref(self._b), ctypes.byref(params), self._ev, n, self.workspace.data_ptr(),
                                nbytes, ptrs, self.stream.cuda_stream))
        self.N = params.n_xi * params.n_theta * 2 * params.n_phi

    def tune(self, dtau_fm):
        """Time the kernel variants, keep the fastest; returns (variant, ms per step of each)."""
        plain = self.params.force_form == LB_FORCE_FEQ and self.params.particle_number == LB_N_FREE
        nv = 12 if self.params.precision == LB_FP32_FP64MATCH and plain else 3
        ms = (ctypes.c_double * nv)()
        v = ctypes.c_int32()
        check(lib.lb_batch_tune(self._b, float(dtau_fm), ctypes.byref(v), ms))
        return v.value, list(ms)

    def set_variant(self, variant):
        check(lib.lb_batch_set_variant(self._b, int(variant)))

    def step(self, n_steps, dtau_fm):
        check(lib.lb_batch_step(self._b, int(n_steps), float(dtau_fm)))

    def _grid(self, event):
        if not 0 <= int(event) < len(self.events):
            raise LbError(LB_E_ARG, f"no event {event} in a batch of {len(self.events)}")
        return self.events[int(event)][:2]

    def moments(self, event):
        nx, ny = self._grid(event)
        out = self.torch.empty((N_OBS, ny, nx), dtype=self.torch.float64, device=self.device)
        check(lib.lb_batch_moments(self._b, int(event), out.data_ptr()))
        return out

    def get_state(self, event):
        nx, ny = self._grid(event)
        torch = self.torch
        F = torch.empty((self.N, ny, nx), dtype=torch.float64, device=self.device)
        lnM = torch.empty((ny, nx), dtype=torch.float64, device=self.device)
        tau = ctypes.c_double()
        check(lib.lb_batch_get_state(self._b, int(event), F.data_ptr(), lnM.data_ptr(), ctypes.byref(tau)))
        return F, lnM, tau.value

    def status(self):
        return lib.lb_batch_status(self._b)

    def close(self):
        if self._b:
            lib.lb_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def node_table(p):
    """(5, N) float64 array of the per-node quantities in the canonical node
    order (lb_node_table): w_n, gamma_n, v^x_n, v^y_n, v^Y_n."""
    import numpy as np
    n = lib.lb_node_table(ctypes.byref(p), None, 0)
    if n < 0:
        raise LbError(int(n), last_error())
    buf = np.zeros(n, dtype=np.float64)
    r = lib.lb_node_table(ctypes.byref(p), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n)
    if r < 0:
        raise LbError(int(r), last_error())
    return buf.reshape(5, -1)


def node_tensors(p, device):
    """The node table of lb_node_table as five float64 tensors of shape [N]
    on device: w_n, gamma_n, v^x_n, v^y_n, v^Y_n."""
    import torch
    return tuple(torch.tensor(row, dtype=torch.float64, device=device) for row in node_table(p))


class _Evolve:
    """Checkpointed forward run and its adjoint (see evolve)."""

    @staticmethod
    def build():
        import torch

        class Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, e0, eta, params, n_steps, dtau, every):
                p = lb_params.from_buffer_copy(params)
                p.eta_over_s = float(eta)
                c = Context(p, e0.detach().contiguous())
                ckpt = []
                for k in range(n_steps):
                    if k % every == 0:
                        ckpt.append(c.get_state())
                    c.step(1, dtau)
                F, lnM, _ = c.get_state()
                if c.status() != LB_OK:
                    raise LbError(c.status(), last_error())
                ctx.c, ctx.ckpt, ctx.n, ctx.dtau, ctx.every = c, ckpt, n_steps, dtau, every
                ctx.save_for_backward(e0)
                ctx.eta_shape = eta.shape if torch.is_tensor(eta) else None
                return F, lnM

            @staticmethod
            def backward(ctx, gF, gL):
                (e0,) = ctx.saved_tensors
                c = ctx.c
                aF = (gF if gF is not None else torch.zeros((c.N, c.params.ny, c.params.nx), dtype=torch.float64,
                                                            device=c.device)).detach().clone().contiguous()
                aL = (gL if gL is not None else torch.zeros((c.params.ny, c.params.nx), dtype=torch.float64,
                                                            device=c.device)).detach().clone().contiguous()
                g_eta = torch.zeros(1, dtype=torch.float64, device=c.device)
                ws = c.adjoint_workspace()
                for seg in reversed(range(len(ctx.ckpt))):
                    k0 = seg * ctx.every
                    k1 = min(k0 + ctx.every, ctx.n)
                    F, L, tau = ctx.ckpt[seg]
                    c.set_state(F, L, tau)
                    states = [(F, L, tau)]
                    for _ in range(k0 + 1, k1):
                        c.step(1, ctx.dtau)
                        states.append(c.get_state())
                    for F, L, tau in reversed(states):
                        c.adjoint_step(tau, ctx.dtau, F, L, aF, aL, g_eta, ws)
                g_e0 = c.adjoint_init(e0.detach().contiguous(), aF, aL)
                if c.status() != LB_OK:
                    raise LbError(c.status(), last_error())
                ge = g_eta.reshape(ctx.eta_shape).to(e0.device) if ctx.eta_shape is not None else None
                return g_e0, ge, None, None, None, None

        return Fn


_evolve_fn = None


def evolve(params, e0, eta_over_s, n_steps, dtau_fm, checkpoint_every=50):
    """Differentiable run: the state (F [N, ny, nx], ln M [ny, nx]) after
    n_steps Heun steps from lb_init(e0) with the given eta/s, as a
    torch.autograd.Function of e0 (float64 [ny, nx] on the GPU) and eta_over_s
    (a float64 tensor with one element).  The backward pass re-runs the
    forward from checkpoints taken every checkpoint_every steps and applies
    lb_adjoint_step backwards, then lb_adjoint_init."""
    global _evolve_fn
    if _evolve_fn is None:
        _evolve_fn = _Evolve.build()
    return _evolve_fn.apply(e0, eta_over_s, params, int(n_steps), float(dtau_fm), int(checkpoint_every))
