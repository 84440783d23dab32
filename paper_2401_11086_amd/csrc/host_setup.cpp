// Host-side set-up of the LB-SMRT lattice: the 1D quadrature (Sec. 4.2,
// D1Qd rules and Table 3's lattice constants) and the normal-shock end
// states (eq:rankine).  Plain C++ (long double and binary128 arithmetic), no GPU.
#include <cmath>
#include <cstring>
#include <vector>

#include "lbsmrt.h"
#include "host_setup.hpp"

namespace lbsmrt {

namespace {

// The root is bracketed on a grid in long double and then bisected, and its weights solved, in
// binary128 (__float128, software arithmetic): at degree 19 the residual below is ill-conditioned
// enough that long double bisection left r ~2e-14 from the root and the weights' quadrature
// identity off by ~3e-13, while binary128 gives r and w correctly rounded to double.  Only basic
// operations are used (no powl: the x87 transcendental instructions behind it differ in their
// last bits between processor vendors), so the rule is the same on every host.
using quad = __float128;

template <typename T>
T abs_of(T x) { return x < 0 ? -x : x; }

template <typename T>
T gaussian_even_moment(int k) {  // (2k-1)!!
  T m = 1;
  for (int j = 1; j < 2 * k; j += 2) m *= j;
  return m;
}

template <typename T>
T even_power(T x, int k) {  // x^(2k)
  const T x2 = x * x;
  T v = 1;
  for (int i = 0; i < k; ++i) v *= x2;
  return v;
}

// Weights w_0, w_{a_j} matching the even moments 0..2(n_eq-1) for a given r;
// Gaussian elimination with partial pivoting.  Returns false if singular.
template <typename T>
bool weights_for(const std::vector<int>& ab, T r, int n_eq, std::vector<T>& w) {
  const int p = static_cast<int>(ab.size());
  const int n = p + 1;
  std::vector<T> A(n_eq * n), b(n_eq);
  for (int k = 0; k < n_eq; ++k) {
    A[k * n + 0] = (k == 0) ? T(1) : T(0);
    for (int j = 0; j < p; ++j) A[k * n + j + 1] = 2 * even_power<T>(ab[j] * r, k);
    b[k] = gaussian_even_moment<T>(k);
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int i = c + 1; i < n; ++i)
      if (abs_of(A[i * n + c]) > abs_of(A[piv * n + c])) piv = i;
    if (A[piv * n + c] == 0) return false;
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[piv * n + j]);
      std::swap(b[c], b[piv]);
    }
    for (int i = c + 1; i < n; ++i) {
      const T f = A[i * n + c] / A[c * n + c];
      for (int j = c; j < n; ++j) A[i * n + j] -= f * A[c * n + j];
      b[i] -= f * b[c];
    }
  }
  w.assign(n, T(0));
  for (int i = n - 1; i >= 0; --i) {
    T s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * w[j];
    w[i] = s / A[i * n + i];
  }
  return true;
}

template <typename T>
bool residual(const std::vector<int>& ab, T r, int k_top, T& res) {
  std::vector<T> w;
  if (!weights_for<T>(ab, r, k_top, w)) return false;
  T s = 0;
  for (size_t j = 0; j < ab.size(); ++j) s += 2 * w[j + 1] * even_power<T>(ab[j] * r, k_top);
  res = s - gaussian_even_moment<T>(k_top);
  return true;
}

}  // namespace

lbsmrt_status solve_quadrature(const int* abscissa, int p, int degree, double* r_out, double* w_out) {
  if (p < 1 || p > 16 || !abscissa || !r_out || !w_out) return LBSMRT_E_ARG;
  std::vector<int> ab(abscissa, abscissa + p);
  for (int j = 0; j < p; ++j) {
    if (ab[j] <= 0) return LBSMRT_E_ARG;
    if (j > 0 && ab[j] <= ab[j - 1]) return LBSMRT_E_ARG;
  }
  // p+1 weights and r are fixed by the p+2 even moments 0..2(p+1)
  if (degree / 2 + 1 != p + 2) return LBSMRT_E_QUADRATURE;
  const int k_top = p + 1;
  const int n_grid = 12000;
  const long double lo = 0.02L, hi = 6.0L;
  long double prev_r = lo, prev_f = 0.0L;
  bool have_prev = residual<long double>(ab, lo, k_top, prev_f);
  for (int i = 1; i < n_grid; ++i) {
    const long double r = lo + (hi - lo) * i / (n_grid - 1);
    long double f;
    if (!residual<long double>(ab, r, k_top, f)) { have_prev = false; continue; }
    if (have_prev && ((prev_f < 0) != (f < 0))) {
      quad a = prev_r, b = r, fa = 0;
      bool ok = residual<quad>(ab, a, k_top, fa);
      for (int it = 0; ok && it < 120; ++it) {
        const quad m = (a + b) / 2;
        quad fm;
        if (!residual<quad>(ab, m, k_top, fm)) break;
        if ((fm < 0) == (fa < 0)) { a = m; fa = fm; } else { b = m; }
      }
      const quad root = (a + b) / 2;
      std::vector<quad> w;
      if (ok && weights_for<quad>(ab, root, k_top, w)) {
        bool pos = true;
        for (const quad& x : w) pos = pos && (x > 0);
        if (pos) {
          *r_out = static_cast<double>(root);
          for (int j = 0; j <= p; ++j) w_out[j] = static_cast<double>(w[j]);
          return LBSMRT_OK;
        }
      }
    }
    prev_r = r;
    prev_f = f;
    have_prev = true;
  }
  return LBSMRT_E_QUADRATURE;
}

lbsmrt_status shock_states(double Ma, double gamma, double theta1, double theta2, double c_l, double* out) {
  if (!out || !(Ma >= 1.0) || !(gamma > 1.0)) return LBSMRT_E_ARG;
  const double M2 = Ma * Ma;
  const double dens = (gamma + 1.0) * M2 / ((gamma - 1.0) * M2 + 2.0);
  const double tratio = (2.0 * gamma * M2 - gamma + 1.0) * ((gamma - 1.0) * M2 + 2.0) /
                        ((gamma + 1.0) * (gamma + 1.0) * M2);
  if (!(theta1 > 0.0)) {
    if (!(theta2 > 0.0)) return LBSMRT_E_ARG;
    theta1 = theta2 / tratio;
  }
  theta2 = theta1 * tratio;
  const double u1 = Ma * std::sqrt(gamma * theta1);
  const double u2 = u1 / dens;
  const double umid = 0.5 * (u1 + u2);
  out[0] = 1.0; out[1] = u1; out[2] = theta1;
  out[3] = dens; out[4] = u2; out[5] = theta2;
  out[6] = umid;
  out[7] = (c_l > 0.0) ? std::floor(umid / c_l + 0.5) : 0.0;
  return LBSMRT_OK;
}

// FP32 contractions rebuild f* with float32 1D tables rw (the rounded w_j He_n(c_j)/n!), for
// which the quadrature identity sum_j He_m(c_j) rw[j][n] = delta_mn holds only to float32
// rounding: a projection with the exact He_m would then see the rebuilt mass, momentum and
// energy off by ~1e-8 per step, the same way at every step.  The FP64 sums of the conserved
// moments use instead the weights hd closest to He_m (m = 0, 1, 2) that are exactly dual to the
// float32 table: hd = he + rw (rw^T rw)^{-1} (e_m - rw^T he), in long double, refined once.  The
// 3D rebuild table is the tensor product of the 1D one and so is its dual, so the conserved
// moments of a rebuilt node come back exactly as they went in.
void dual_projection_table(const float (*rw)[6], const double (*he)[6], int Q1, int N, double (*hd)[3]) {
  const int n = N + 1;
  long double G[6][6];
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      long double s = 0.0L;
      for (int j = 0; j < Q1; ++j) s += static_cast<long double>(rw[j][a]) * rw[j][b];
      G[a][b] = s;
    }
  for (int m = 0; m < 3 && m <= N; ++m) {
    long double x[17];
    for (int j = 0; j < Q1; ++j) x[j] = he[j][m];
    for (int pass = 0; pass < 2; ++pass) {
      // residual r_b = delta_mb - sum_j x_j rw[j][b]; solve G y = r; x += rw y
      long double A[6][7];
      for (int b = 0; b < n; ++b) {
        long double s = (b == m) ? 1.0L : 0.0L;
        for (int j = 0; j < Q1; ++j) s -= x[j] * rw[j][b];
        for (int c = 0; c < n; ++c) A[b][c] = G[b][c];
        A[b][n] = s;
      }
      for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
          if (fabsl(A[i][c]) > fabsl(A[piv][c])) piv = i;
        for (int k = 0; k <= n; ++k) std::swap(A[c][k], A[piv][k]);
        for (int i = 0; i < n; ++i) {
          if (i == c || A[c][c] == 0.0L) continue;
          const long double f = A[i][c] / A[c][c];
          for (int k = c; k <= n; ++k) A[i][k] -= f * A[c][k];
        }
      }
      for (int b = 0; b < n; ++b) {
        const long double y = A[b][b] != 0.0L ? A[b][n] / A[b][b] : 0.0L;
        for (int j = 0; j < Q1; ++j) x[j] += static_cast<long double>(rw[j][b]) * y;
      }
    }
    for (int j = 0; j < Q1; ++j) hd[j][m] = static_cast<double>(x[j]);
  }
}

}  // namespace lbsmrt
