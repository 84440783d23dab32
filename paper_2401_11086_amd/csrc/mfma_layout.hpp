// Operand orderings of the split-BF16x3 contraction form (eq:an projection, eq:fi rebuild) on
// the gfx950 matrix cores, v_mfma_f32_32x32x16_bf16: D[32 x 32] += A[32 x 16] B[16 x 32], every
// operand lane l holding row / column l % 32 and the 8 consecutive k = 8 (l / 32) + e.
//
// A wave updates 64 nodes as two tiles of 32 (the MFMA columns).  Each contraction runs as three
// products on bf16 halves, hi.hi + hi.lo + lo.hi, accumulated in FP32.
//
// Projection a_alpha = sum_q He_alpha(c_q) g_q for the orders 2..N (rows: alpha - 4, so one
// 32-row tile at N = 4 and two at N = 5); orders 0 and 1 and the order-2 trace come from FP64
// sums instead.  Its k axis walks z lines of populations, KPX k-steps per x-slab ix (so that a
// k-step stays inside one slab: one source x per lane); in k-step p of a slab:
//   p < Q1 / 2 : lines (ix, iy = 2p) in the lower half-wave and (ix, 2p + 1) in the upper, iz = e
//                (with Q1 = 7 the last pair's upper line is empty);
//   Q1 = 9, p = 4: line (ix, 8), iz = e in the lower half-wave; iz = 8 of lines iy = e in the upper;
//   Q1 = 9, p = 5: population (ix, 8, 8) alone (lower half-wave, e = 0).
// Out-of-range positions are zero.
// Rebuild f_q = sum_K T[q][K] b_K: rows q (32-row tiles, Q padded), k axis K = the M moments
// a'_alpha followed by 5 correction coefficients (see mfma_tables.cpp), padded to a multiple of 16.
#pragma once
#include "smrt_node.hpp"

namespace lbsmrt {

template <int Q1, int N>
struct MfmaShape {
  static constexpr int Q = Q1 * Q1 * Q1;
  static constexpr int M = n_moments(N);
  static constexpr int KPX = Q1 <= 8 ? (Q1 + 1) / 2 : 6;     // k-steps per x-slab (D1Q7, D1Q9)
  static constexpr int KSTEPS_P = Q1 * KPX;                  // projection k-steps
  static constexpr int NA = M - 4;                           // projected rows (orders 2..N)
  static constexpr int ATILES = (NA + 31) / 32;
  static constexpr int QTILES = (Q + 31) / 32;
  static constexpr int KR = M + 5;                           // rebuild k: moments + corrections
  static constexpr int KSTEPS_R = (KR + 15) / 16;
  // element counts (8 bf16 per lane and operand) of the two tables, per bf16 half
  static constexpr long long PROJ_VEC = static_cast<long long>(ATILES) * KSTEPS_P * 64;
  static constexpr long long REB_VEC = static_cast<long long>(QTILES) * KSTEPS_R * 64;
};

// 1D indices (ix, iy, iz) of the population at projection k-position (s, half h, element e);
// false for a padding position.
// The two stencils the form is built for, 1D integers in ascending order (D1Q7 {0, +-1, +-2, +-3}
// and D1Q9 {0, +-1, +-2, +-3, +-5}, Table 3): the conserved sums weight populations by these
// integers, which as compile-time constants stay out of the register file.
template <int Q1>
struct MfmaStencil;
template <>
struct MfmaStencil<7> {
  static constexpr int e[7] = {-3, -2, -1, 0, 1, 2, 3};
};
template <>
struct MfmaStencil<9> {
  static constexpr int e[9] = {-5, -3, -2, -1, 0, 1, 2, 3, 5};
};

__host__ __device__ constexpr int proj_kpx(int Q1) { return Q1 <= 8 ? (Q1 + 1) / 2 : 6; }
__host__ __device__ constexpr bool proj_pop(int Q1, int s, int h, int e, int& ix, int& iy, int& iz) {
  const int kpx = proj_kpx(Q1);
  const int p = s % kpx;
  ix = s / kpx;
  if (Q1 <= 8 || p < 4) {
    iy = 2 * p + h;
    iz = e;
  } else if (p == 4) {
    iy = h == 0 ? 8 : e;
    iz = h == 0 ? e : 8;
  } else {
    iy = 8;
    iz = (h == 0 && e == 0) ? 8 : Q1;
  }
  return ix < Q1 && iy < Q1 && iz < Q1;
}

// Contents of the constant block that follows the two tables (FP64): for the five conserved
// sums P_k = (1, e_x, e_y, e_z, |e|^2) over the populations and each moment alpha < M, the ten
// values Phi[k][alpha] = P_k T_hi[:, alpha] (at 10 alpha + k) and Plo[k][alpha] = P_k T_lo[:, alpha]
// (at 10 alpha + 5 + k), then the inverse of the 5 x 5 matrix P_j T_hi[:, M + k] of the
// correction columns (row-major, at 10 M).
template <int N>
struct MfmaConsLayout {
  static constexpr int M = n_moments(N);
  static constexpr int MINV = 10 * M;
  static constexpr int SIZE = 10 * M + 25;
  static constexpr int phi(int k, int alpha) { return 10 * alpha + k; }
  static constexpr int plo(int k, int alpha) { return 10 * alpha + 5 + k; }
};

}  // namespace lbsmrt
