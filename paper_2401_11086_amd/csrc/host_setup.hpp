// Host-side set-up helpers (quadrature, shock states).  Not part of the C ABI.
#pragma once
#include "lbsmrt.h"

namespace lbsmrt {
lbsmrt_status solve_quadrature(const int* abscissa, int p, int degree, double* r_out, double* w_out);
lbsmrt_status shock_states(double Ma, double gamma, double theta1, double theta2, double c_l, double* out);
// 1D projection weights dual to a float32 rebuild table: hd[j][m] (m = 0, 1, 2) closest to
// he[j][m] with sum_j hd[j][m] rw[j][n] = delta_mn for n = 0..N.  Tables are [17][6] row-major.
void dual_projection_table(const float (*rw)[6], const double (*he)[6], int Q1, int N, double (*hd)[3]);
}  // namespace lbsmrt
