"""ctypes binding of liblbsmrt.so (the C ABI declared in include/lbsmrt.h).

Argument marshalling only: every step of the method runs in the HIP library.
Loading fails loudly when the library has not been built.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbsmrt.so")

OK, E_ARG, E_QUADRATURE, E_STATE, E_HIP, E_NOMEM, E_UNSUPPORTED, E_LIMIT, E_TIMEOUT = range(9)
FP32, SPLIT_BF16X3, FP64_CONTRACT = 0, 1, 2
LAUNCH_DIRECT, LAUNCH_GRAPH, LAUNCH_PERSISTENT = 0, 1, 2
MOM_BASIC, MOM_SIGMA, MOM_Q, MOM_M3, MOM_R41, MOM_R42, MOM_DLOCAL, MOM_ALAB = (1, 2, 4, 8, 16, 32, 64, 128)


class LatticeDesc(ctypes.Structure):
    _fields_ = [
        ("n_abscissa", ctypes.c_int),
        ("abscissa", ctypes.c_int * 16),
        ("degree", ctypes.c_int),
        ("order_N", ctypes.c_int),
        ("shift_k", ctypes.c_int * 3),
        ("tau", (ctypes.c_double * 3) * 6),
        ("rho_ref", ctypes.c_double),
        ("tau_density_scaling", ctypes.c_int),
        ("tau_offset_half", ctypes.c_int),
        ("regularized", ctypes.c_int),
        ("precision", ctypes.c_int),
    ]


class DomainDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("bc_x", ctypes.c_int),
        ("rho_in", ctypes.c_double), ("u_in", ctypes.c_double * 3), ("theta_in", ctypes.c_double),
        ("rho_out", ctypes.c_double), ("u_out", ctypes.c_double * 3), ("theta_out", ctypes.c_double),
        ("tau_scale", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("Q", ctypes.c_int), ("Q1", ctypes.c_int), ("M", ctypes.c_int), ("N", ctypes.c_int),
        ("c_l", ctypes.c_double),
        ("w1d", ctypes.c_double * 17),
        ("e1d", ctypes.c_int * 17),
        ("n_nodes", ctypes.c_longlong),
        ("f_stride", ctypes.c_longlong),
        ("f_len", ctypes.c_longlong),
        ("n_domains", ctypes.c_int),
        ("domain_offset", ctypes.c_longlong * 64),
    ]


class LbsmrtError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "lbsmrt_init_lattice": (ctypes.c_int, [ctypes.POINTER(LatticeDesc), ctypes.POINTER(DomainDesc), ctypes.c_int,
                                           ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "lbsmrt_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "lbsmrt_get_domain_offsets": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong), ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_int)]),
    "lbsmrt_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "lbsmrt_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint,
                                      ctypes.c_void_p]),
    "lbsmrt_moment_rows": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint]),
    "lbsmrt_equilibrium": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbsmrt_step_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "lbsmrt_step_adjoint_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbsmrt_loss_seed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "lbsmrt_sync_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "lbsmrt_set_tau": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "lbsmrt_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "lbsmrt_test_flow_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint, ctypes.c_uint]),
    "lbsmrt_get_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int)]),
    "lbsmrt_moment_state_len": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_longlong),
                                               ctypes.POINTER(ctypes.c_longlong)]),
    "lbsmrt_equilibrium_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbsmrt_project_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbsmrt_expand_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "lbsmrt_step_moment_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_int, ctypes.c_void_p]),
    "lbsmrt_destroy": (None, [ctypes.c_void_p]),
    "lbsmrt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lbsmrt_solve_quadrature": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "lbsmrt_shock_states": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -m paper_2401_11086_amd.build); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status):
    try:
        return lib().lbsmrt_status_string(status).decode()
    except ImportError:
        return "library not loaded"


def check(status, what):
    if status != OK:
        raise LbsmrtError(status, what)


def solve_quadrature(abscissae, degree):
    """Host-side 1D quadrature of the library: returns (r, weights[p+1])."""
    p = len(abscissae)
    arr = (ctypes.c_int * p)(*abscissae)
    r = ctypes.c_double()
    w = (ctypes.c_double * (p + 1))()
    check(lib().lbsmrt_solve_quadrature(p, arr, degree, ctypes.byref(r), w), "solve_quadrature")
    return r.value, [w[i] for i in range(p + 1)]


def shock_states(Ma, gamma=5.0 / 3.0, theta1=0.0, theta2=0.0, c_l=0.0):
    out = (ctypes.c_double * 8)()
    check(lib().lbsmrt_shock_states(Ma, gamma, theta1, theta2, c_l, out), "shock_states")
    keys = ("rho1", "u1", "theta1", "rho2", "u2", "theta2", "u_mid", "k")
    return {k: out[i] for i, k in enumerate(keys)}
