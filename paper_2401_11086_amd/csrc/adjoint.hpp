// Reverse mode of the per-node SMRT collision (device code).
//
// Forward map at one node (FP64 arithmetic, see kernels.hpp):
//   a = P g                       projection (eq:an)
//   rho = a_0, u = a_1 / rho, theta = (sum_k a_{2e_k} + 3 rho - rho |u|^2) / (3 rho)
//   d = Lambda^{-1} T_B(u, theta) a      lattice -> local frame (binomial transform)
//   d' = K(omega(rho)) d                 irreducible split + relaxation (eq:SMRT, App. A)
//   a' = T_A(u, theta) Lambda d'         local -> lattice frame
//   f* = R a'                            rebuild (eq:fi)
// The adjoint maps lambda = dL/df* to mu = dL/dg = P^T abar and accumulates
// dL/dtau_nm.  Derivatives of the shift polynomials follow from their
// generating functions: dA_j/du = j A_{j-1}, dA_j/dtheta = C(j,2) A_{j-2},
// dB_j/du = -j B_{j-1}, dB_j/dtheta = -C(j,2) B_{j-2}.
#pragma once
#include "kernels.hpp"

namespace lbsmrt {

// ---------------------------------------------------------------- transposed tensor operators
// transpose of sym_trace<L>: rank L -> rank L+2
template <int L>
__device__ __forceinline__ void sym_trace_T(const double* Tb, double* Xb) {
#pragma unroll
  for (int i = 0; i < n_sym(L + 2); ++i) Xb[i] = 0.0;
#pragma unroll
  for (int a = 0; a <= L; ++a)
#pragma unroll
    for (int b = 0; b <= L; ++b)
      if (a + b <= L) {
        const double t = Tb[sym_pos(L, a, b)];
        Xb[sym_pos(L + 2, a + 2, b)] += t;
        Xb[sym_pos(L + 2, a, b + 2)] += t;
        Xb[sym_pos(L + 2, a, b)] += t;
      }
}

// transpose of sym_delta<L>: rank L+2 -> rank L
template <int L>
__device__ __forceinline__ void sym_delta_T(const double* Pb, double* Yb) {
  constexpr double inv = 1.0 / binom(L + 2, 2);
#pragma unroll
  for (int i = 0; i < n_sym(L); ++i) Yb[i] = 0.0;
#pragma unroll
  for (int a = 0; a <= L + 2; ++a)
#pragma unroll
    for (int b = 0; b <= L + 2; ++b) {
      if (a + b > L + 2) continue;
      const int c = L + 2 - a - b;
      const double p = Pb[sym_pos(L + 2, a, b)] * inv;
      if (a >= 2) Yb[sym_pos(L, a - 2, b)] += binom(a, 2) * p;
      if (b >= 2) Yb[sym_pos(L, a, b - 2)] += binom(b, 2) * p;
      if (c >= 2) Yb[sym_pos(L, a, b)] += binom(c, 2) * p;
    }
}

// transpose of traceless<L>: Y' = Y + D(L,1) delta tr Y  ->  Yb += D(L,1) tr^T delta^T Yb'
template <int L>
__device__ __forceinline__ void traceless_T(double* Yb) {
  if constexpr (L >= 2) {
    double t[n_sym(L - 2)];
    double x[n_sym(L)];
    sym_delta_T<L - 2>(Yb, t);
    sym_trace_T<L - 2>(t, x);
    constexpr double dk = coefD(L, 1);
#pragma unroll
    for (int i = 0; i < n_sym(L); ++i) Yb[i] += dk * x[i];
  }
}

// transpose of irreducible_piece<n,m> (m >= 1): rank n -> rank n
template <int n, int m>
__device__ __forceinline__ void irreducible_piece_T(const double* Pb, double* Db) {
  constexpr int L = n - 2 * m;
  double part[n_sym(L)];
  if constexpr (m == 1) {
    sym_delta_T<L>(Pb, part);
  } else {
    double tmp[n_sym(L + 2)];
    sym_delta_T<L + 2>(Pb, tmp);
    sym_delta_T<L>(tmp, part);
  }
  constexpr double bnm = coefB(n, m);
#pragma unroll
  for (int i = 0; i < n_sym(L); ++i) part[i] *= bnm;
  traceless_T<L>(part);
  if constexpr (m == 1) {
    sym_trace_T<L>(part, Db);
  } else {
    double t1[n_sym(n - 2)];
    sym_trace_T<L>(part, t1);
    sym_trace_T<n - 2>(t1, Db);
  }
}

template <int n>
__device__ __forceinline__ double dotn(const double* x, const double* y) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < n_sym(n); ++i) s = fma(x[i], y[i], s);
  return s;
}

// Adjoint of relax_order<n>: in dpb = dL/dd'^(n), dn = d^(n) (forward input);
// out dpb <- dL/dd^(n); ob[m] += dL/domega_nm.
template <int n>
__device__ __forceinline__ void relax_order_T(double* dpb, const double* dn, const double* om, double* ob) {
  double acc[n_sym(n)];
#pragma unroll
  for (int i = 0; i < n_sym(n); ++i) acc[i] = (1.0 - om[0]) * dpb[i];
  double rest = dotn<n>(dpb, dn);  // d'.d  -> becomes d'.P_0 d after removing the pieces
  {
    double P[n_sym(n)], PT[n_sym(n)];
    irreducible_piece<n, 1>(dn, P);
    const double s1 = dotn<n>(dpb, P);
    ob[1] += -s1;
    rest -= s1;
    irreducible_piece_T<n, 1>(dpb, PT);
    const double c1 = om[1] - om[0];
#pragma unroll
    for (int i = 0; i < n_sym(n); ++i) acc[i] -= c1 * PT[i];
  }
  if constexpr (n >= 4) {
    double P[n_sym(n)], PT[n_sym(n)];
    irreducible_piece<n, 2>(dn, P);
    const double s2 = dotn<n>(dpb, P);
    ob[2] += -s2;
    rest -= s2;
    irreducible_piece_T<n, 2>(dpb, PT);
    const double c2 = om[2] - om[0];
#pragma unroll
    for (int i = 0; i < n_sym(n); ++i) acc[i] -= c2 * PT[i];
  }
  ob[0] += -rest;
#pragma unroll
  for (int i = 0; i < n_sym(n); ++i) dpb[i] = acc[i];
}

// Transpose of axis_transform<N,AXIS>:  xb_g = sum_{b >= g} C(b, g) P_{b-g} yb_b  (in place, bottom-up)
template <int N, int AXIS>
__device__ __forceinline__ void axis_transform_T(double* d, const double (&P)[N + 1]) {
#pragma unroll
  for (int o1 = 0; o1 <= N; ++o1)
#pragma unroll
    for (int o2 = 0; o2 <= N; ++o2)
#pragma unroll
      for (int g = 0; g <= N; ++g) {
        const int L = N - o1 - o2;
        if (L < 0 || g > L) continue;
        auto id = [&](int v) {
          return AXIS == 0 ? midx(v, o1, o2) : (AXIS == 1 ? midx(o1, v, o2) : midx(o1, o2, v));
        };
        double s = d[id(g)];
#pragma unroll
        for (int b = 1; b <= N; ++b)
          if (b > g && b <= L) s += binom(b, g) * P[b - g] * d[id(b)];
        d[id(g)] = s;
      }
}

__host__ __device__ constexpr int order_of(int i) {
  int n = 0;
  while (order_start(n + 1) <= i) ++n;
  return n;
}

// Decode multi-index i -> (a,b,c)
__host__ __device__ constexpr int mi_a(int i) {
  const int n = order_of(i);
  const int r = i - order_start(n);
  int a = n;
  int rem = r;
  while (rem >= n - a + 1) { rem -= n - a + 1; --a; }
  return a;
}
__host__ __device__ constexpr int mi_b(int i) {
  const int n = order_of(i);
  const int r = i - order_start(n);
  int a = n;
  int rem = r;
  while (rem >= n - a + 1) { rem -= n - a + 1; --a; }
  return (n - a) - rem;
}
__host__ __device__ constexpr int mi_c(int i) { return order_of(i) - mi_a(i) - mi_b(i); }

// Per-node reverse sweep.  d: local moments entering the relaxation (d_0 = rho, d_1 = 0).
// ab: in dL/da' (lattice frame, after collision); out dL/da (lattice frame, before).
// tb[n][m] += dL/dtau_nm.
template <int N>
__device__ __forceinline__ void node_adjoint(const LatticeConst& L, const Macro& mac, const double* d, double* ab,
                                             double (&tb)[kMaxN + 1][3]) {
  constexpr int M = n_moments(N);
  const double rho = mac.rho, th = mac.th;
  const double u[3] = {mac.ux, mac.uy, mac.uz};
  const double sc = L.density_scaling ? L.rho_ref / rho : 1.0;
  double om[kMaxN + 1][3];
#pragma unroll
  for (int n = 2; n <= N; ++n)
#pragma unroll
    for (int m = 0; m < 3; ++m) om[n][m] = (2 * m <= n) ? 1.0 / fma(L.tau[n][m], sc, L.tau_offset) : 0.0;
  om[2][1] = 0.0;

  double ubar[3] = {0.0, 0.0, 0.0};
  double thbar = 0.0, rhobar = 0.0;
  // powers of sqrt(theta)
  const double sq = sqrt(th);
  double sp[N + 1];
  sp[0] = 1.0;
#pragma unroll
  for (int n = 1; n <= N; ++n) sp[n] = sp[n - 1] * sq;

  // ---- a' = T_A Lambda d'  (reverse)
  {
    double dp[M];
#pragma unroll
    for (int i = 0; i < M; ++i) dp[i] = d[i];
    relax<N>(dp, L, rho);
    double ap[M];
#pragma unroll
    for (int i = 0; i < M; ++i) ap[i] = dp[i];
    to_lattice<N>(ap, mac);
    // u, theta through T_A
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const int a = mi_a(i), b = mi_b(i), c = mi_c(i);
      const double g = ab[i];
      if (a >= 1) ubar[0] += g * a * ap[midx(a - 1, b, c)];
      if (b >= 1) ubar[1] += g * b * ap[midx(a, b - 1, c)];
      if (c >= 1) ubar[2] += g * c * ap[midx(a, b, c - 1)];
      double t = 0.0;
      if (a >= 2) t += binom(a, 2) * ap[midx(a - 2, b, c)];
      if (b >= 2) t += binom(b, 2) * ap[midx(a, b - 2, c)];
      if (c >= 2) t += binom(c, 2) * ap[midx(a, b, c - 2)];
      thbar += g * t;
    }
    double Ax[N + 1], Ay[N + 1], Az[N + 1];
    shift_poly<N>(mac.ux, th - 1.0, Ax);
    shift_poly<N>(mac.uy, th - 1.0, Ay);
    shift_poly<N>(mac.uz, th - 1.0, Az);
    axis_transform_T<N, 2>(ab, Az);
    axis_transform_T<N, 1>(ab, Ay);
    axis_transform_T<N, 0>(ab, Ax);
    // theta through Lambda; then d'bar = Lambda zbar
#pragma unroll
    for (int i = 0; i < M; ++i) {
      const int n = order_of(i);
      if (n >= 1) thbar += ab[i] * (0.5 * n) * (sp[n] / th) * dp[i];
      ab[i] *= sp[n];
    }
  }
  // orders 0 and 1 of d' are rho and 0
  rhobar += ab[0];
  ab[0] = 0.0;
  ab[1] = ab[2] = ab[3] = 0.0;

  // ---- relaxation (reverse)
#pragma unroll
  for (int n = 2; n <= N; ++n) {
    double ob[3] = {0.0, 0.0, 0.0};
    double* dpb = ab + order_start(n);
    const double* dn = d + order_start(n);
    if (n == 2) relax_order_T<2>(dpb, dn, om[2], ob);
    if (n == 3) relax_order_T<3>(dpb, dn, om[3], ob);
    if constexpr (N >= 4) if (n == 4) relax_order_T<4>(dpb, dn, om[4], ob);
    if constexpr (N >= 5) if (n == 5) relax_order_T<5>(dpb, dn, om[5], ob);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (2 * m > n || (n == 2 && m == 1)) continue;
      const double w = om[n][m];
      tb[n][m] += ob[m] * (-sc * w * w);
      if (L.density_scaling) rhobar += ob[m] * (w * w * L.tau[n][m] * L.rho_ref / (rho * rho));
    }
  }

  // ---- d = Lambda^{-1} T_B a  (reverse); orders 0, 1 of d were set from rho and 0
  {
    const double ith = 1.0 / th;
    const double isq = 1.0 / sq;
#pragma unroll
    for (int i = 4; i < M; ++i) {
      const int a = mi_a(i), b = mi_b(i), c = mi_c(i);
      const int n = a + b + c;
      const double g = ab[i];
      if (a >= 1) ubar[0] -= isq * g * a * d[midx(a - 1, b, c)];
      if (b >= 1) ubar[1] -= isq * g * b * d[midx(a, b - 1, c)];
      if (c >= 1) ubar[2] -= isq * g * c * d[midx(a, b, c - 1)];
      double t = 0.0;
      if (a >= 2) t += binom(a, 2) * d[midx(a - 2, b, c)];
      if (b >= 2) t += binom(b, 2) * d[midx(a, b - 2, c)];
      if (c >= 2) t += binom(c, 2) * d[midx(a, b, c - 2)];
      thbar -= g * ((0.5 * n) * ith * d[i] + ith * t);
    }
#pragma unroll
    for (int i = 4; i < M; ++i) ab[i] /= sp[order_of(i)];
    double Bx[N + 1], By[N + 1], Bz[N + 1];
    shift_poly<N>(-mac.ux, 1.0 - th, Bx);
    shift_poly<N>(-mac.uy, 1.0 - th, By);
    shift_poly<N>(-mac.uz, 1.0 - th, Bz);
    axis_transform_T<N, 2>(ab, Bz);
    axis_transform_T<N, 1>(ab, By);
    axis_transform_T<N, 0>(ab, Bx);
  }

  // ---- rho, u, theta from a_0, a_1, a_2  (reverse)
  const double irho = 1.0 / rho;
  const double Ebar = thbar * (1.0 / 3.0) * irho;
  rhobar -= thbar * (th + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * (1.0 / 3.0)) * irho;
#pragma unroll
  for (int k = 0; k < 3; ++k) ubar[k] -= thbar * (2.0 / 3.0) * u[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) rhobar -= ubar[k] * u[k] * irho;
  ab[0] += rhobar + 3.0 * Ebar;
  ab[midx(1, 0, 0)] += ubar[0] * irho;
  ab[midx(0, 1, 0)] += ubar[1] * irho;
  ab[midx(0, 0, 1)] += ubar[2] * irho;
  ab[midx(2, 0, 0)] += Ebar;
  ab[midx(0, 2, 0)] += Ebar;
  ab[midx(0, 0, 2)] += Ebar;
}

}  // namespace lbsmrt
