// Host-side set-up helpers (quadrature, shock states).  Not part of the C ABI.
#pragma once
#include "lbsmrt.h"

namespace lbsmrt {
lbsmrt_status solve_quadrature(const int* abscissa, int p, int degree, double* r_out, double* w_out);
lbsmrt_status shock_states(double Ma, double gamma, double theta1, double theta2, double c_l, double* out);
}  // namespace lbsmrt
