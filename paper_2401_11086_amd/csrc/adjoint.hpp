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

// Transpose of axis_transform<N,AXIS>:  xb_g = sum_{b >= g} C(b, g) P_{b-g} yb_b  (in place, bottom-up)
template <int N, int AXIS, class D>
__device__ __forceinline__ void axis_transform_T(D d, const double (&P)[N + 1]) {
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
template <int N, class V, class AB>
__device__ __forceinline__ void node_adjoint(const LatticeConst& L, const Macro& mac, const V& dv, const V& zv,
                                             AB ab, double* tb) {
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

  // The workgroup fences between phases make the compiler re-read d and z from LDS after each
  // fence instead of keeping the values of an earlier phase live in registers.
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
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

  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
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
    // each z_j is read once and feeds the components j + e_k and j + 2 e_k of abar
    const double i2th = 0.5 / th;
#pragma unroll
    for (int a = 0; a <= N; ++a)
#pragma unroll
    for (int b = 0; b <= N; ++b)
#pragma unroll
    for (int c = 0; c <= N; ++c) {
      const int m = a + b + c;
      if (m > N) continue;
      const double zj = zv(midx(a, b, c));
      if (m + 1 <= N) {
        ubar[0] += ab[midx(a + 1, b, c)] * (a + 1) * zj;
        ubar[1] += ab[midx(a, b + 1, c)] * (b + 1) * zj;
        ubar[2] += ab[midx(a, b, c + 1)] * (c + 1) * zj;
      }
      double t = (m >= 1) ? ab[midx(a, b, c)] * (m * i2th) : 0.0;
      if (m + 2 <= N)
        t += binom(a + 2, 2) * ab[midx(a + 2, b, c)] + binom(b + 2, 2) * ab[midx(a, b + 2, c)] +
             binom(c + 2, 2) * ab[midx(a, b, c + 2)];
      thbar += t * zj;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  // d'bar = Lambda zbar; orders 0 and 1 of d' are rho and 0
#pragma unroll
  for (int n = 2; n <= N; ++n)
#pragma unroll
    for (int i = order_start(n); i < order_start(n + 1); ++i) ab[i] *= sp[n];
  rhobar += ab[0];
  ab[0] = ab[1] = ab[2] = ab[3] = 0.0;

  // ---- relaxation (reverse):  dbar = W K W^{-1} d'bar,  omega_bar_m = -<P_m y, d>_W with y = W^{-1} d'bar.
  // With P_m y = delta^m part_m(y) and delta linear, K y = (1 - om_0) y - delta Y for the rank n-2
  // bracket Y = (om_1 - om_0) part_1(y) + (om_2 - om_0) delta part_2(y); the components of
  // delta part_1(y) and delta delta part_2(y) are formed one at a time.
#pragma unroll
  for (int n = 2; n <= N; ++n) {
    double om[3];
    omegas(n, om);
    // this order's components in a local array (ab may live in LDS): y = W^{-1} d'bar
    double y[n_sym(kMaxN)];
#pragma unroll
    for (int a = 0; a <= n; ++a)
#pragma unroll
      for (int b = 0; b <= n; ++b)
        if (a + b <= n) y[sym_pos(n, a, b)] = ab[order_start(n) + sym_pos(n, a, b)] * (1.0 / multiplicity(a, b, n - a - b));
    constexpr int S2 = n_sym(kMaxN - 2);
    double Y1[S2], Y2[S2];
    if (n == 2) irreducible_part<2, 1>(y, Y1);
    if (n == 3) irreducible_part<3, 1>(y, Y1);
    if constexpr (N >= 4) if (n == 4) irreducible_part<4, 1>(y, Y1);
    if constexpr (N >= 5) if (n == 5) irreducible_part<5, 1>(y, Y1);
    if (n >= 4) {
      double p2[n_sym(kMaxN - 4)];
      if constexpr (N >= 4) if (n == 4) { irreducible_part<4, 2>(y, p2); sym_delta<0>(p2, Y2); }
      if constexpr (N >= 5) if (n == 5) { irreducible_part<5, 2>(y, p2); sym_delta<1>(p2, Y2); }
    }
    const double c1 = om[1] - om[0], c2 = om[2] - om[0];
    double p0d = 0.0, pd1 = 0.0, pd2 = 0.0;
#pragma unroll
    for (int a = 0; a <= n; ++a)
#pragma unroll
      for (int b = 0; b <= n; ++b) {
        if (a + b > n) continue;
        const int i = sym_pos(n, a, b);
        const double w = multiplicity(a, b, n - a - b);
        const double di = dv(order_start(n) + i);
        double q1 = 0.0, q2 = 0.0;
        if (n == 2) q1 = sym_delta_at<0>(Y1, a, b);
        if (n == 3) q1 = sym_delta_at<1>(Y1, a, b);
        if constexpr (N >= 4) if (n == 4) { q1 = sym_delta_at<2>(Y1, a, b); q2 = sym_delta_at<2>(Y2, a, b); }
        if constexpr (N >= 5) if (n == 5) { q1 = sym_delta_at<3>(Y1, a, b); q2 = sym_delta_at<3>(Y2, a, b); }
        p0d += w * y[i] * di;
        pd1 += w * q1 * di;
        pd2 += w * q2 * di;
        ab[order_start(n) + i] = ((1.0 - om[0]) * y[i] - c1 * q1 - c2 * q2) * w;
      }
    const double ob[3] = {-(p0d - pd1 - pd2), -pd1, -pd2};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (2 * m > n || (n == 2 && m == 1)) continue;
      const double w = om[m];
      tb[tau_slot(n, m)] += ob[m] * (-sc * w * w);
      if (L.density_scaling) rhobar += ob[m] * (w * w * L.tau[n][m] * mac.tsc * L.rho_ref / (rho * rho));
    }
  }

  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  // ---- d = Lambda^{-1} T_B a  (reverse); orders 0, 1 of d were set from rho and 0
  {
    const double ith = 1.0 / th;
    const double isq = 1.0 / sq;
    // each d_j is read once and feeds the components j, j + e_k and j + 2 e_k of abar (orders 2..N)
#pragma unroll
    for (int a = 0; a <= N; ++a)
#pragma unroll
    for (int b = 0; b <= N; ++b)
#pragma unroll
    for (int c = 0; c <= N; ++c) {
      const int m = a + b + c;
      if (m > N) continue;
      const double dj = dv(midx(a, b, c));
      if (m + 1 >= 2 && m + 1 <= N) {
        ubar[0] -= isq * ab[midx(a + 1, b, c)] * (a + 1) * dj;
        ubar[1] -= isq * ab[midx(a, b + 1, c)] * (b + 1) * dj;
        ubar[2] -= isq * ab[midx(a, b, c + 1)] * (c + 1) * dj;
      }
      double t = (m >= 2) ? ab[midx(a, b, c)] * (0.5 * m) : 0.0;
      if (m + 2 <= N)
        t += binom(a + 2, 2) * ab[midx(a + 2, b, c)] + binom(b + 2, 2) * ab[midx(a, b + 2, c)] +
             binom(c + 2, 2) * ab[midx(a, b, c + 2)];
      thbar -= ith * t * dj;
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
