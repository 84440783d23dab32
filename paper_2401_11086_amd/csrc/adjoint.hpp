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

// Compact index of the relaxation times that act: (2,0), (3,0), (3,1), (4,0), (4,1), (4,2), (5,0), (5,1), (5,2).
__host__ __device__ constexpr int tau_slot(int n, int m) { return n == 2 ? 0 : (n == 3 ? 1 + m : (n == 4 ? 3 + m : 6 + m)); }
__host__ __device__ constexpr int n_tau_slots(int N) { return N == 2 ? 1 : (N == 3 ? 3 : (N == 4 ? 6 : 9)); }

// Multiplicity n!/(a! b! c!) of component (a,b,c) of a symmetric tensor: the weight of the
// full-contraction inner product in the component representation.
__host__ __device__ constexpr double multiplicity(int a, int b, int c) {
  return factorial(a + b + c) / (factorial(a) * factorial(b) * factorial(c));
}

// Per-node reverse sweep.
//   dv: local moments d entering the relaxation (d_0 = rho, d_1 = 0), per work-item in LDS;
//   zv: per work-item LDS scratch of M doubles (receives z = Lambda d');
//   ab: in dL/da' (lattice frame, after collision); out dL/da (lattice frame, before);
//   tb[tau_slot(n,m)] += dL/dtau_nm.
// Two identities keep a single M-vector in registers:
//  * the shift operators commute with the raising operator (L y)_b = b y_{b-1}, so
//    dT_A/du_k = L_k T_A = T_A L_k and dT_A/dtheta = T_A (1/2) sum_k L_k^2: the u and theta
//    sensitivities of a' = T_A z are zbar . (L_k z) and zbar . (sum_k L_k^2 z)/2 with zbar = T_A^T abar;
//  * the irreducible projectors are self-adjoint in the full-contraction inner product
//    (weights W = n!/alpha!), so the transposed relaxation is W K W^{-1}.
template <int N, class V>
__device__ __forceinline__ void node_adjoint(const LatticeConst& L, const Macro& mac, const V& dv, const V& zv,
                                             double* ab, double* tb) {
  constexpr int M = n_moments(N);
  const double rho = mac.rho, th = mac.th;
  const double u[3] = {mac.ux, mac.uy, mac.uz};
  const double sc = mac.tsc * (L.density_scaling ? L.rho_ref / rho : 1.0);
  double ubar[3] = {0.0, 0.0, 0.0};
  double thbar = 0.0, rhobar = 0.0;
  const double sq = sqrt(th);
  double sp[N + 1];
  sp[0] = 1.0;
#pragma unroll
  for (int n = 1; n <= N; ++n) sp[n] = sp[n - 1] * sq;
  auto omegas = [&](int n, double (&om)[3]) {
#pragma unroll
    for (int m = 0; m < 3; ++m) om[m] = (2 * m <= n) ? 1.0 / fma(L.tau[n][m], sc, L.tau_offset) : 0.0;
    if (n == 2) om[1] = 0.0;   // the (2,1) part is left unrelaxed (it is zero)
  };

  // ---- z = Lambda d' = Lambda K d, into LDS
  zv.set(0, dv(0));
  zv.set(1, 0.0);
  zv.set(2, 0.0);
  zv.set(3, 0.0);
#pragma unroll
  for (int n = 2; n <= N; ++n) {
    double om[3];
    omegas(n, om);
    double t[n_sym(kMaxN)];
#pragma unroll
    for (int i = 0; i < n_sym(n); ++i) t[i] = dv(order_start(n) + i);
    if (n == 2) relax_order<2>(t, om);
    if (n == 3) relax_order<3>(t, om);
    if constexpr (N >= 4) if (n == 4) relax_order<4>(t, om);
    if constexpr (N >= 5) if (n == 5) relax_order<5>(t, om);
#pragma unroll
    for (int i = 0; i < n_sym(n); ++i) zv.set(order_start(n) + i, t[i] * sp[n]);
  }

  // ---- a' = T_A z  (reverse): zbar = T_A^T abar; u, theta sensitivities in z space
  {
    double Ax[N + 1], Ay[N + 1], Az[N + 1];
    shift_poly<N>(mac.ux, th - 1.0, Ax);
    shift_poly<N>(mac.uy, th - 1.0, Ay);
    shift_poly<N>(mac.uz, th - 1.0, Az);
    axis_transform_T<N, 2>(ab, Az);
    axis_transform_T<N, 1>(ab, Ay);
    axis_transform_T<N, 0>(ab, Ax);
  }
  {
    const double i2th = 0.5 / th;
#pragma unroll
    for (int a = 0; a <= N; ++a)
#pragma unroll
    for (int b = 0; b <= N; ++b)
#pragma unroll
    for (int c = 0; c <= N; ++c) {
      const int n = a + b + c;
      if (n == 0 || n > N) continue;
      const int i = midx(a, b, c);
      const double g = ab[i];
      if (a >= 1) ubar[0] += g * a * zv(midx(a - 1, b, c));
      if (b >= 1) ubar[1] += g * b * zv(midx(a, b - 1, c));
      if (c >= 1) ubar[2] += g * c * zv(midx(a, b, c - 1));
      double t = (n * i2th) * zv(i);
      if (a >= 2) t += binom(a, 2) * zv(midx(a - 2, b, c));
      if (b >= 2) t += binom(b, 2) * zv(midx(a, b - 2, c));
      if (c >= 2) t += binom(c, 2) * zv(midx(a, b, c - 2));
      thbar += g * t;
    }
  }
  // d'bar = Lambda zbar; orders 0 and 1 of d' are rho and 0
#pragma unroll
  for (int n = 2; n <= N; ++n)
#pragma unroll
    for (int i = order_start(n); i < order_start(n + 1); ++i) ab[i] *= sp[n];
  rhobar += ab[0];
  ab[0] = ab[1] = ab[2] = ab[3] = 0.0;

  // ---- relaxation (reverse):  dbar = W K W^{-1} d'bar,  omega_bar_m = -<P_m y, d>_W with y = W^{-1} d'bar
#pragma unroll
  for (int n = 2; n <= N; ++n) {
    double om[3];
    omegas(n, om);
    constexpr int S = n_sym(kMaxN);
    double y[S], wgt[S];
#pragma unroll
    for (int a = 0; a <= n; ++a)
#pragma unroll
      for (int b = 0; b <= n; ++b)
        if (a + b <= n) wgt[sym_pos(n, a, b)] = multiplicity(a, b, n - a - b);
#pragma unroll
    for (int i = 0; i < n_sym(n); ++i) y[i] = ab[order_start(n) + i] / wgt[i];
    double ob[3] = {0.0, 0.0, 0.0};
    double r[S];
#pragma unroll
    for (int i = 0; i < n_sym(n); ++i) r[i] = (1.0 - om[0]) * y[i];
    double p0d = 0.0;   // <y, d>_W
#pragma unroll
    for (int i = 0; i < n_sym(n); ++i) p0d += wgt[i] * y[i] * dv(order_start(n) + i);
#pragma unroll
    for (int m = 1; m <= 2; ++m) {
      if (2 * m > n) continue;
      double P[S];
      if (n == 2 && m == 1) irreducible_piece<2, 1>(y, P);
      if (n == 3 && m == 1) irreducible_piece<3, 1>(y, P);
      if constexpr (N >= 4) {
        if (n == 4 && m == 1) irreducible_piece<4, 1>(y, P);
        if (n == 4 && m == 2) irreducible_piece<4, 2>(y, P);
      }
      if constexpr (N >= 5) {
        if (n == 5 && m == 1) irreducible_piece<5, 1>(y, P);
        if (n == 5 && m == 2) irreducible_piece<5, 2>(y, P);
      }
      double pd = 0.0;
#pragma unroll
      for (int i = 0; i < n_sym(n); ++i) pd += wgt[i] * P[i] * dv(order_start(n) + i);
      ob[m] = -pd;
      p0d -= pd;
      const double cm = om[m] - om[0];
#pragma unroll
      for (int i = 0; i < n_sym(n); ++i) r[i] -= cm * P[i];
    }
    ob[0] = -p0d;
#pragma unroll
    for (int i = 0; i < n_sym(n); ++i) ab[order_start(n) + i] = r[i] * wgt[i];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (2 * m > n || (n == 2 && m == 1)) continue;
      const double w = om[m];
      tb[tau_slot(n, m)] += ob[m] * (-sc * w * w);
      if (L.density_scaling) rhobar += ob[m] * (w * w * L.tau[n][m] * mac.tsc * L.rho_ref / (rho * rho));
    }
  }

  // ---- d = Lambda^{-1} T_B a  (reverse); orders 0, 1 of d were set from rho and 0
  {
    const double ith = 1.0 / th;
    const double isq = 1.0 / sq;
#pragma unroll
    for (int a = 0; a <= N; ++a)
#pragma unroll
    for (int b = 0; b <= N; ++b)
#pragma unroll
    for (int c = 0; c <= N; ++c) {
      const int n = a + b + c;
      if (n < 2 || n > N) continue;
      const int i = midx(a, b, c);
      const double g = ab[i];
      if (a >= 1) ubar[0] -= isq * g * a * dv(midx(a - 1, b, c));
      if (b >= 1) ubar[1] -= isq * g * b * dv(midx(a, b - 1, c));
      if (c >= 1) ubar[2] -= isq * g * c * dv(midx(a, b, c - 1));
      double t = 0.0;
      if (a >= 2) t += binom(a, 2) * dv(midx(a - 2, b, c));
      if (b >= 2) t += binom(b, 2) * dv(midx(a, b - 2, c));
      if (c >= 2) t += binom(c, 2) * dv(midx(a, b, c - 2));
      thbar -= g * ((0.5 * n) * ith * dv(i) + ith * t);
    }
#pragma unroll
    for (int n = 2; n <= N; ++n) {
      const double inv = 1.0 / sp[n];
#pragma unroll
      for (int i = order_start(n); i < order_start(n + 1); ++i) ab[i] *= inv;
    }
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
