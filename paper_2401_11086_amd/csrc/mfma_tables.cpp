// Host-side tables of the split-BF16x3 contraction form: the bf16 halves of the projection
// table He_alpha(c_q) (eq:an) and of the rebuild table w_q He_alpha(c_q) / alpha! (eq:fi, with
// eq:hermite1's 1/n!), laid out as MFMA operands, and the FP64 constants with which the step
// kernel keeps the rebuild conservative.
//
// Why the constants: with bf16 halves the rebuilt populations f = T_hi (a_hi + a_lo) + T_lo a_hi
// carry the table roundings and the dropped lo.lo product.  Their conserved sums
// P_k f = sum_q P_k(q) f_q, P = (1, e_x, e_y, e_z, |e|^2), would then miss a'_0, a'_1 / c_l and
// (3 a'_0 + tr a'_2) / c_l^2 by ~1e-6 relative, the same way at every step, and mass, momentum and
// energy would drift.  Since T_hi and T_lo are fixed, those sums are known exactly in advance:
// P_k f = Phi_k (a_hi + a_lo) + Plo_k a_hi with Phi = P T_hi, Plo = P T_lo.  Five more k-columns
// phi_k(q) = bf16(w_q P_k(q)) carry a correction c, chosen per node in FP64 as
// c = (P phi)^{-1} (target - Phi (a_hi + a_lo) - Plo a_hi) and itself split into bf16 halves,
// so the rebuilt node hands exactly its conserved moments to the next step's FP64 sums (up to
// the FP32 accumulation and storage rounding).
#include "mfma_tables.hpp"

#include <cmath>
#include <cstring>

#include "mfma_layout.hpp"

namespace lbsmrt {

namespace {

uint16_t bf16_bits(double v) {   // round to float, then to bf16 (nearest, ties to even)
  const float f = static_cast<float>(v);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
double bf16_value(uint16_t b) {
  const uint32_t u = static_cast<uint32_t>(b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
double hermite(int n, double x) {
  double h0 = 1.0, h1 = x;
  if (n == 0) return h0;
  for (int k = 1; k < n; ++k) {
    const double h2 = x * h1 - k * h0;
    h0 = h1;
    h1 = h2;
  }
  return h1;
}
double fact(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

bool invert5(const long double (&m)[5][5], double (&inv)[5][5]) {
  long double a[5][10];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 10; ++j) a[i][j] = j < 5 ? m[i][j] : (j - 5 == i ? 1.0L : 0.0L);
  for (int c = 0; c < 5; ++c) {
    int piv = c;
    for (int i = c + 1; i < 5; ++i)
      if (fabsl(a[i][c]) > fabsl(a[piv][c])) piv = i;
    if (a[piv][c] == 0.0L) return false;
    for (int j = 0; j < 10; ++j) std::swap(a[c][j], a[piv][j]);
    const long double d = a[c][c];
    for (int j = 0; j < 10; ++j) a[c][j] /= d;
    for (int i = 0; i < 5; ++i) {
      if (i == c) continue;
      const long double f = a[i][c];
      for (int j = 0; j < 10; ++j) a[i][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) inv[i][j] = static_cast<double>(a[i][5 + j]);
  return true;
}

}  // namespace

bool build_mfma_tables(int Q1, int N, double r, const double* w1, const int* e1, MfmaHostTables& out) {
  const int Q = Q1 * Q1 * Q1;
  const int M = n_moments(N);
  const int kpx = proj_kpx(Q1);
  const int ksteps_p = Q1 * kpx;
  const int atiles = (M - 4 + 31) / 32;
  const int qtiles = (Q + 31) / 32;
  const int ksteps_r = (M + 5 + 15) / 16;
  // multi-indices in the library's order (by n, then a, then b descending)
  std::vector<int> al[3];
  for (int n = 0; n <= N; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) {
        al[0].push_back(a);
        al[1].push_back(b);
        al[2].push_back(n - a - b);
      }
  auto he_q = [&](int q, int alpha) {
    const int ix = q / (Q1 * Q1), iy = (q / Q1) % Q1, iz = q % Q1;
    return hermite(al[0][alpha], r * e1[ix]) * hermite(al[1][alpha], r * e1[iy]) * hermite(al[2][alpha], r * e1[iz]);
  };
  auto w_q = [&](int q) { return w1[q / (Q1 * Q1)] * w1[(q / Q1) % Q1] * w1[q % Q1]; };
  auto P_q = [&](int q, int k) -> long double {
    const int ex = e1[q / (Q1 * Q1)], ey = e1[(q / Q1) % Q1], ez = e1[q % Q1];
    switch (k) {
      case 0: return 1.0L;
      case 1: return ex;
      case 2: return ey;
      case 3: return ez;
      default: return static_cast<long double>(ex * ex + ey * ey + ez * ez);
    }
  };
  // projection table
  const long long pvec = static_cast<long long>(atiles) * ksteps_p * 64;
  out.proj.assign(2 * pvec * 8, 0);
  for (int a = 0; a < atiles; ++a)
    for (int s = 0; s < ksteps_p; ++s)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 8; ++e) {
          const int alpha = 4 + 32 * a + (lane & 31);
          int ix, iy, iz;
          if (alpha >= M || !proj_pop(Q1, s, lane >> 5, e, ix, iy, iz)) continue;
          const double v = he_q((ix * Q1 + iy) * Q1 + iz, alpha);
          const uint16_t hi = bf16_bits(v);
          const uint16_t lo = bf16_bits(v - bf16_value(hi));
          const long long at = ((static_cast<long long>(a) * ksteps_p + s) * 64 + lane) * 8 + e;
          out.proj[at] = hi;
          out.proj[pvec * 8 + at] = lo;
        }
  // rebuild table: T[q][K], K < M the rebuild weights, M <= K < M + 5 the correction columns
  std::vector<uint16_t> thi(static_cast<size_t>(Q) * (M + 5), 0), tlo(static_cast<size_t>(Q) * (M + 5), 0);
  for (int q = 0; q < Q; ++q) {
    for (int alpha = 0; alpha < M; ++alpha) {
      const double v = w_q(q) * he_q(q, alpha) / (fact(al[0][alpha]) * fact(al[1][alpha]) * fact(al[2][alpha]));
      thi[q * (M + 5) + alpha] = bf16_bits(v);
      tlo[q * (M + 5) + alpha] = bf16_bits(v - bf16_value(thi[q * (M + 5) + alpha]));
    }
    for (int k = 0; k < 5; ++k) thi[q * (M + 5) + M + k] = bf16_bits(w_q(q) * static_cast<double>(P_q(q, k)));
  }
  const long long rvec = static_cast<long long>(qtiles) * ksteps_r * 64;
  out.rebuild.assign(2 * rvec * 8, 0);
  for (int t = 0; t < qtiles; ++t)
    for (int kk = 0; kk < ksteps_r; ++kk)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 8; ++e) {
          const int q = 32 * t + (lane & 31);
          const int K = 16 * kk + 8 * (lane >> 5) + e;
          if (q >= Q || K >= M + 5) continue;
          const long long at = ((static_cast<long long>(t) * ksteps_r + kk) * 64 + lane) * 8 + e;
          out.rebuild[at] = thi[q * (M + 5) + K];
          out.rebuild[rvec * 8 + at] = tlo[q * (M + 5) + K];
        }
  // conserved sums of the table columns (exact: bf16 values times small integers, long double sums)
  out.cons.assign(10 * M + 25, 0.0);
  long double mphi[5][5] = {};
  for (int k = 0; k < 5; ++k) {
    for (int alpha = 0; alpha < M; ++alpha) {
      long double sh = 0.0L, sl = 0.0L;
      for (int q = 0; q < Q; ++q) {
        sh += P_q(q, k) * bf16_value(thi[q * (M + 5) + alpha]);
        sl += P_q(q, k) * bf16_value(tlo[q * (M + 5) + alpha]);
      }
      out.cons[10 * alpha + k] = static_cast<double>(sh);
      out.cons[10 * alpha + 5 + k] = static_cast<double>(sl);
    }
    for (int j = 0; j < 5; ++j) {
      long double s = 0.0L;
      for (int q = 0; q < Q; ++q) s += P_q(q, k) * bf16_value(thi[q * (M + 5) + M + j]);
      mphi[k][j] = s;
    }
  }
  double inv[5][5];
  if (!invert5(mphi, inv)) return false;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) out.cons[10 * M + i * 5 + j] = inv[i][j];
  return true;
}

}  // namespace lbsmrt
