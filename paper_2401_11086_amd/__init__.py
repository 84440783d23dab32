"""MI355X (gfx950) LB-SMRT collide-and-stream: HIP kernels behind a C ABI
(include/lbsmrt.h) with a thin Python binding."""
from ._lib import (MOM_ALAB, MOM_BASIC, MOM_DLOCAL, MOM_M3, MOM_Q, MOM_R41, MOM_R42, MOM_SIGMA,  # noqa: F401
                   LbsmrtError, shock_states, solve_quadrature)
from .lattice import Lattice  # noqa: F401
