"""Python face of the LB-SMRT library: a lattice context over caller-owned
torch device tensors.  PyTorch supplies device memory and the stream only."""
import atexit
import ctypes
import weakref

import torch

from . import _lib as C


# Every open context, so that all are destroyed while the HIP runtime is still up: at interpreter
# exit the atexit hook runs before module teardown, where __del__ would otherwise free device
# tables after the runtime (or a profiler attached to it) has been finalised.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    live = list(_LIVE)
    if not live:
        return
    try:
        torch.cuda.synchronize()
    except Exception:
        pass
    for lat in live:
        try:
            lat.close()
        except Exception:
            pass


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


class Lattice:
    """One LB-SMRT configuration: velocity set, truncation order, relaxation
    times and a list of domains (see include/lbsmrt.h for every field).

    tau: dict {(n, m): tau_nm} in time-step units at rho_ref.
    domains: list of dicts with nx, ny, nz, bc_x and, for bc_x = 1,
    rho_in, u_in, theta_in, rho_out, u_out, theta_out (lab frame).
    precision: "fp64_contract" (default: FP64 contractions, as fast as FP32 ones on gfx950)
    or "fp32" (FP32 contractions); the state is float32 in both.
    regularized: True (f* rebuilt from the relaxed moments) or False (additive collision
    f* = g + R (a' - a); FP64 contractions only).
    """

    def __init__(self, abscissae, degree, N, tau, domains, shift_k=(0, 0, 0), rho_ref=1.0,
                 tau_density_scaling=True, tau_offset_half=True, precision="fp64_contract", regularized=True):
        if not torch.cuda.is_available():
            raise RuntimeError("the LB-SMRT library runs on a gfx950 GPU; no GPU is visible")
        lib = C.lib()
        d = C.LatticeDesc()
        d.n_abscissa = len(abscissae)
        for i, a in enumerate(abscissae):
            d.abscissa[i] = int(a)
        d.degree = int(degree)
        d.order_N = int(N)
        for k in range(3):
            d.shift_k[k] = int(shift_k[k])
        for n in range(6):
            for m in range(3):
                d.tau[n][m] = float(tau.get((n, m), 1.0)) if (n >= 2 and 2 * m <= n) else 1.0
        d.rho_ref = float(rho_ref)
        d.tau_density_scaling = int(bool(tau_density_scaling))
        d.tau_offset_half = int(bool(tau_offset_half))
        d.regularized = 1 if regularized else 0
        d.precision = {"fp32": C.FP32, "split_bf16x3": C.SPLIT_BF16X3, "fp64_contract": C.FP64_CONTRACT}[precision]
        arr = (C.DomainDesc * len(domains))()
        for i, dom in enumerate(domains):
            x = arr[i]
            x.nx, x.ny, x.nz = int(dom["nx"]), int(dom.get("ny", 1)), int(dom.get("nz", 1))
            x.bc_x = int(dom.get("bc_x", 0))
            x.tau_scale = float(dom.get("tau_scale", 1.0))
            if x.bc_x == 1:
                x.rho_in, x.theta_in = float(dom["rho_in"]), float(dom["theta_in"])
                x.rho_out, x.theta_out = float(dom["rho_out"]), float(dom["theta_out"])
                for k in range(3):
                    x.u_in[k] = float(dom["u_in"][k])
                    x.u_out[k] = float(dom["u_out"][k])
        self.domains = [dict(dm) for dm in domains]
        self.precision = precision
        self.regularized = bool(regularized)
        self.tau = dict(tau)
        self.shift_k = tuple(int(v) for v in shift_k)
        h = ctypes.c_void_p()
        C.check(lib.lbsmrt_init_lattice(ctypes.byref(d), arr, len(domains), _stream_ptr(), ctypes.byref(h)),
                "lbsmrt_init_lattice")
        self._h = h
        info = C.Info()
        C.check(lib.lbsmrt_get_info(h, ctypes.byref(info)), "lbsmrt_get_info")
        self.Q, self.Q1, self.M, self.N = info.Q, info.Q1, info.M, info.N
        self.c_l = info.c_l
        self.w1d = [info.w1d[i] for i in range(self.Q1)]
        self.e1d = [info.e1d[i] for i in range(self.Q1)]
        self.n_nodes = info.n_nodes
        self.f_stride = info.f_stride
        offs = (ctypes.c_longlong * info.n_domains)()
        got = ctypes.c_int()
        C.check(lib.lbsmrt_get_domain_offsets(h, offs, info.n_domains, ctypes.byref(got)), "lbsmrt_get_domain_offsets")
        self.domain_offset = [offs[i] for i in range(got.value)]
        self.device = torch.device("cuda", torch.cuda.current_device())
        _LIVE.add(self)

    # -- buffers ------------------------------------------------------------
    def new_state(self):
        return torch.empty((self.Q, self.f_stride), dtype=torch.float32, device=self.device)

    # -- calls --------------------------------------------------------------
    def equilibrium(self, fields, out=None):
        """fields: float64 (5, n_nodes) rows rho, u_x, u_y, u_z, theta (lab frame)."""
        f = self.new_state() if out is None else out
        C.check(C.lib().lbsmrt_equilibrium(self._h, _dev_ptr(fields, torch.float64, "fields"),
                                           _dev_ptr(f, torch.float32, "f"), _stream_ptr()), "lbsmrt_equilibrium")
        return f

    def step(self, f_a, f_b, n_steps=1):
        """Advance n_steps; returns whichever of f_a, f_b holds the result."""
        C.check(C.lib().lbsmrt_step(self._h, _dev_ptr(f_a, torch.float32, "f_a"), _dev_ptr(f_b, torch.float32, "f_b"),
                                    int(n_steps), _stream_ptr()), "lbsmrt_step")
        return f_a if n_steps % 2 == 0 else f_b

    def moment_rows(self, mask):
        return C.lib().lbsmrt_moment_rows(self._h, mask)

    def moments(self, f, mask=C.MOM_BASIC, out=None):
        rows = self.moment_rows(mask)
        o = torch.empty((rows, self.n_nodes), dtype=torch.float64, device=self.device) if out is None else out
        C.check(C.lib().lbsmrt_moments(self._h, _dev_ptr(f, torch.float32, "f"), _dev_ptr(o, torch.float64, "out"),
                                       int(mask), _stream_ptr()), "lbsmrt_moments")
        return o

    def step_adjoint(self, f_t, lam_next, lam_t, dL_dtau):
        C.check(C.lib().lbsmrt_step_adjoint(self._h, _dev_ptr(f_t, torch.float32, "f_t"),
                                            _dev_ptr(lam_next, torch.float32, "lam_next"),
                                            _dev_ptr(lam_t, torch.float32, "lam_t"),
                                            _dev_ptr(dL_dtau, torch.float64, "dL_dtau"), _stream_ptr()),
                "lbsmrt_step_adjoint")
        return lam_t

    def step_adjoint_noalloc(self, f_t, lam_next, lam_t, dL_dtau):
        """step_adjoint through the allocation-free entry point (library-held scratch, one per GPU;
        calls that overlap on one GPU race).  LbsmrtError with E_LIMIT beyond its size limit."""
        C.check(C.lib().lbsmrt_step_adjoint_noalloc(self._h, _dev_ptr(f_t, torch.float32, "f_t"),
                                                    _dev_ptr(lam_next, torch.float32, "lam_next"),
                                                    _dev_ptr(lam_t, torch.float32, "lam_t"),
                                                    _dev_ptr(dL_dtau, torch.float64, "dL_dtau"), _stream_ptr()),
                "lbsmrt_step_adjoint_noalloc")
        return lam_t

    def loss_seed(self, f, target, scales, lam, loss):
        sc = (ctypes.c_double * 3)(*[float(s) for s in scales])
        C.check(C.lib().lbsmrt_loss_seed(self._h, _dev_ptr(f, torch.float32, "f"),
                                         _dev_ptr(target, torch.float64, "target"), sc,
                                         _dev_ptr(lam, torch.float32, "lam"), _dev_ptr(loss, torch.float64, "loss"),
                                         _stream_ptr()), "lbsmrt_loss_seed")
        return lam

    # -- moment-state form (periodic box contexts; see lbsmrt_step_moment_state) --------
    def moment_state_len(self):
        """(m_len, work_len) in floats."""
        m, w = ctypes.c_longlong(), ctypes.c_longlong()
        C.check(C.lib().lbsmrt_moment_state_len(self._h, ctypes.byref(m), ctypes.byref(w)), "lbsmrt_moment_state_len")
        return m.value, w.value

    def new_moment_state(self):
        return torch.empty((self.M, self.f_stride), dtype=torch.float32, device=self.device)

    def new_moment_work(self):
        return torch.empty(self.moment_state_len()[1], dtype=torch.float32, device=self.device)

    def equilibrium_moments(self, fields, out=None):
        """fields: float64 (5, n_nodes) rows rho, u_x, u_y, u_z, theta -> moment state (M, f_stride)."""
        m = self.new_moment_state() if out is None else out
        C.check(C.lib().lbsmrt_equilibrium_moments(self._h, _dev_ptr(fields, torch.float64, "fields"),
                                                   _dev_ptr(m, torch.float32, "m"), _stream_ptr()),
                "lbsmrt_equilibrium_moments")
        return m

    def project_state(self, f, out=None):
        """Own-node moments m_alpha = sum_i f_i He_alpha(c_i) of a population state."""
        m = self.new_moment_state() if out is None else out
        C.check(C.lib().lbsmrt_project_state(self._h, _dev_ptr(f, torch.float32, "f"), _dev_ptr(m, torch.float32, "m"),
                                             _stream_ptr()), "lbsmrt_project_state")
        return m

    def expand_state(self, m, out=None):
        """Population state f_i = w_i sum_alpha m_alpha He_alpha(c_i) / alpha! of a moment state."""
        f = self.new_state() if out is None else out
        C.check(C.lib().lbsmrt_expand_state(self._h, _dev_ptr(m, torch.float32, "m"), _dev_ptr(f, torch.float32, "f"),
                                            _stream_ptr()), "lbsmrt_expand_state")
        return f

    def step_moment_state(self, m_a, m_b, work, n_steps=1):
        """Advance a moment state n_steps; returns whichever of m_a, m_b holds the result."""
        C.check(C.lib().lbsmrt_step_moment_state(self._h, _dev_ptr(m_a, torch.float32, "m_a"),
                                                 _dev_ptr(m_b, torch.float32, "m_b"),
                                                 _dev_ptr(work, torch.float32, "work"), int(n_steps), _stream_ptr()),
                "lbsmrt_step_moment_state")
        return m_a if n_steps % 2 == 0 else m_b

    def set_tau(self, tau):
        """Replace the relaxation times ({(n, m): tau_nm}); missing entries keep their value."""
        self.tau.update({k: float(v) for k, v in tau.items()})
        arr = (ctypes.c_double * 18)()
        for n in range(6):
            for m in range(3):
                arr[n * 3 + m] = float(self.tau.get((n, m), 1.0))
        C.check(C.lib().lbsmrt_set_tau(self._h, arr), "lbsmrt_set_tau")

    def set_launch(self, mode="direct", block_size=0, graph_steps=64, lanes_per_node=0):
        """mode: 'direct', 'graph' or 'persistent'; block_size 64/128/256 (0 keeps it);
        lanes_per_node 1, 2, 4, 8 or 16 (0 keeps it; > 1 for shock contexts with FP64 contractions).
        See lbsmrt_set_launch in include/lbsmrt.h."""
        m = {"direct": C.LAUNCH_DIRECT, "graph": C.LAUNCH_GRAPH, "persistent": C.LAUNCH_PERSISTENT}[mode]
        C.check(C.lib().lbsmrt_set_launch(self._h, m, int(block_size), int(graph_steps), int(lanes_per_node)),
                "lbsmrt_set_launch")
        self.launch = (mode, block_size, graph_steps, lanes_per_node)

    def launch_settings(self):
        """{'mode', 'block', 'lanes_per_node'} as the library holds them."""
        m, b, k = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        C.check(C.lib().lbsmrt_get_launch(self._h, ctypes.byref(m), ctypes.byref(b), ctypes.byref(k)),
                "lbsmrt_get_launch")
        names = {C.LAUNCH_DIRECT: "direct", C.LAUNCH_GRAPH: "graph", C.LAUNCH_PERSISTENT: "persistent"}
        return {"mode": names[m.value], "block": b.value, "lanes_per_node": k.value}

    def sync(self):
        """Wait for the current stream; raise if a node left the validity region."""
        C.check(C.lib().lbsmrt_sync_status(self._h, _stream_ptr()), "lbsmrt_sync_status")

    def close(self):
        """Destroy the context (its device tables); the caller's buffers are untouched."""
        if getattr(self, "_h", None):
            C.lib().lbsmrt_destroy(self._h)
            self._h = None
        _LIVE.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
