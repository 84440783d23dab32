"""Normal-shock tube set-up for batched runs (Sec. 4.2, Table 3).

End states come from the library's Rankine-Hugoniot helper
(lbsmrt_shock_states); cells are half an up-stream mean free path
(l = tau sqrt(theta)), so each shock carries its own tau scale
tau_20 = 2 c_l / sqrt(theta_1).
"""
import math

from . import _lib as C
from . import workloads as W

# Table 3: down-stream temperature used at Ma = 1.5, 3, 5
TABLE3_THETA2 = ((1.5, 1.07), (3.0, 1.22), (5.0, 1.45))


def theta2_for(Ma):
    """Piecewise-linear in Ma through Table 3's theta_2, held constant outside [1.5, 5]."""
    pts = TABLE3_THETA2
    if Ma <= pts[0][0]:
        return pts[0][1]
    for (m0, t0), (m1, t1) in zip(pts, pts[1:]):
        if Ma <= m1:
            return t0 + (t1 - t0) * (Ma - m0) / (m1 - m0)
    return pts[-1][1]


def shock_domain(Ma, nx, c_l, width=5.0, theta2=None):
    """Domain dict (with tau_scale) and tanh initial fields (5, nx) of one shock."""
    st = C.shock_states(Ma, theta2=theta2 if theta2 else theta2_for(Ma), c_l=c_l)
    dom = dict(nx=int(nx), ny=1, nz=1, bc_x=1,
               rho_in=st["rho1"], u_in=(st["u1"], 0.0, 0.0), theta_in=st["theta1"],
               rho_out=st["rho2"], u_out=(st["u2"], 0.0, 0.0), theta_out=st["theta2"],
               tau_scale=2.0 * c_l / math.sqrt(st["theta1"]))
    fields = W.tanh_profile(int(nx), (st["rho1"], st["u1"], st["theta1"]), (st["rho2"], st["u2"], st["theta2"]),
                            width)
    return dom, fields, st
