// Per-node LB-SMRT arithmetic for gfx950 kernels (header-only, device code).
//
// Notation follows Yan & Shan (arXiv 2401.11086): absolute Hermite moments
// a_alpha (eq:an), local moments d_beta (rho absorbed, Sec. 3), irreducible
// parts d^(n,m) (App. A), relaxation times tau_nm (eq:SMRT, Table 4).
//
// Multi-index alpha = (a,b,c), |alpha| <= N, stored by order n, then a
// descending, then b descending.  A rank-n symmetric tensor is held as its
// (n+1)(n+2)/2 distinct components in the same (a desc, b desc) order.
#pragma once
#include <hip/hip_runtime.h>

// The large per-node phases are force-inlined; defining LBSMRT_PHASE as
// "__device__ __noinline__" gives per-phase register reports.
#ifndef LBSMRT_PHASE
#define LBSMRT_PHASE __device__ __forceinline__
#endif

namespace lbsmrt {

constexpr int kMaxQ1 = 17;   // D1Q17 {0, +-1..+-7, +-9} (Table 3, Ma 7)
constexpr int kMaxN = 5;

__host__ __device__ constexpr int n_moments(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
__host__ __device__ constexpr int n_sym(int n) { return (n + 1) * (n + 2) / 2; }
// position of (a,b,n-a-b) among the rank-n components
__host__ __device__ constexpr int sym_pos(int n, int a, int b) { return (n - a) * (n - a + 1) / 2 + (n - a - b); }
__host__ __device__ constexpr int order_start(int n) { return n * (n + 1) * (n + 2) / 6; }
__host__ __device__ constexpr int midx(int a, int b, int c) { return order_start(a + b + c) + sym_pos(a + b + c, a, b); }
// (ay, az) with ay + az <= N  -> simplex position
__host__ __device__ constexpr int pair_pos(int ay, int az) { return (ay + az) * (ay + az + 1) / 2 + az; }
__host__ __device__ constexpr double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}
__host__ __device__ constexpr double dfact(int k) {  // k!! for odd k >= -1
  double r = 1.0;
  for (int j = k; j > 1; j -= 2) r *= j;
  return r;
}
__host__ __device__ constexpr double factorial(int n) {
  double r = 1.0;
  for (int j = 2; j <= n; ++j) r *= j;
  return r;
}
// eq:bd (App. A)
__host__ __device__ constexpr double coefB(int n, int m) {
  return factorial(n) * dfact(2 * n - 4 * m + 1) /
         (factorial(m) * double(1 << m) * factorial(n - 2 * m) * dfact(2 * n - 2 * m + 1));
}
__host__ __device__ constexpr double coefD(int n, int m) {
  return ((m & 1) ? -1.0 : 1.0) * factorial(n) * dfact(2 * n - 2 * m - 1) /
         (factorial(m) * double(1 << m) * factorial(n - 2 * m) * dfact(2 * n - 1));
}

// Kernel-argument constants of a lattice (passed by value, lands in SGPRs).
struct LatticeConst {
  float  He[kMaxQ1][kMaxN + 1];   // He_n(c_j), c_j = r e_j
  float  Rw[kMaxQ1][kMaxN + 1];   // w_j He_n(c_j) / n!
  double He64[kMaxQ1][kMaxN + 1]; // the same two tables in FP64
  double Rw64[kMaxQ1][kMaxN + 1];
  double Hd[kMaxQ1][3];           // FP64 projection weights of orders 0..2 dual to the float32 Rw
  int    e[kMaxQ1];               // 1D integers, ascending
  double r;                       // lattice constant c_l
  int    k[3];                    // frame shift, ubar = r k
  double tau[kMaxN + 1][3];       // tau_nm at rho_ref
  double rho_ref;
  double tau_offset;              // 0.5 or 0
  int    density_scaling;
};

// He_n(0): 0 for odd n, (-1)^(n/2) (n-1)!! for even n
__host__ __device__ constexpr double hermite_at_zero(int n) {
  return (n & 1) ? 0.0 : (((n / 2) & 1) ? -1.0 : 1.0) * dfact(n - 1);
}

// ------------------------------------------------------------------ tensor algebra
// trace: rank L+2 -> rank L,   (tr X)_alpha = sum_k X_{alpha + 2 e_k}
template <int L>
__device__ __forceinline__ void sym_trace(const double* X, double* T) {
#pragma unroll
  for (int a = 0; a <= L; ++a)
#pragma unroll
    for (int b = 0; b <= L; ++b)
      if (a + b <= L)
        T[sym_pos(L, a, b)] = X[sym_pos(L + 2, a + 2, b)] + X[sym_pos(L + 2, a, b + 2)] +
                              X[sym_pos(L + 2, a, b)];
}

// symmetric product with delta: rank L -> rank L+2,
//   (delta Y)_alpha = sum_k C(alpha_k, 2) Y_{alpha - 2 e_k} / C(L+2, 2);
// sym_delta_at gives component (x, y, L+2-x-y).
template <int L>
__device__ __forceinline__ double sym_delta_at(const double* Y, int x, int y) {
  const int z = L + 2 - x - y;
  double s = 0.0;
  if (x >= 2) s += binom(x, 2) * Y[sym_pos(L, x - 2, y)];
  if (y >= 2) s += binom(y, 2) * Y[sym_pos(L, x, y - 2)];
  if (z >= 2) s += binom(z, 2) * Y[sym_pos(L, x, y)];
  return s * (1.0 / binom(L + 2, 2));
}

template <int L>
__device__ __forceinline__ void sym_delta(const double* Y, double* P) {
#pragma unroll
  for (int x = 0; x <= L + 2; ++x)
#pragma unroll
    for (int y = 0; y <= L + 2; ++y)
      if (x + y <= L + 2) P[sym_pos(L + 2, x, y)] = sym_delta_at<L>(Y, x, y);
}

// Traceless projector Q_0^(L) (App. A); for L <= 3 only the k <= 1 term exists.
template <int L>
__device__ __forceinline__ void traceless(double* Y) {
  static_assert(L <= 3, "traceless projector written for rank <= 3");
  if constexpr (L >= 2) {
    double t[n_sym(L - 2)];
    double p[n_sym(L)];
    sym_trace<L - 2>(Y, t);
    sym_delta<L - 2>(t, p);
    constexpr double dk = coefD(L, 1);
#pragma unroll
    for (int i = 0; i < n_sym(L); ++i) Y[i] += dk * p[i];
  }
}

// Irreducible part d^(n,m) = B(n,m) Q_0^(n-2m) tr^m d^(n), rank n-2m.
template <int n, int m>
__device__ __forceinline__ void irreducible_part(const double* dn, double* out) {
  constexpr int L = n - 2 * m;
  if constexpr (m == 0) {
#pragma unroll
    for (int i = 0; i < n_sym(n); ++i) out[i] = dn[i];
  } else if constexpr (m == 1) {
    sym_trace<L>(dn, out);
  } else {
    double t1[n_sym(n - 2)];
    sym_trace<n - 2>(dn, t1);
    sym_trace<L>(t1, out);
  }
  traceless<L>(out);
  constexpr double bnm = coefB(n, m);
#pragma unroll
  for (int i = 0; i < n_sym(L); ++i) out[i] *= bnm;
}

// D = a D - delta Y  (rank L -> rank L+2, in place on D)
template <int L>
__device__ __forceinline__ void sym_delta_update(const double* Y, double a, double* D) {
#pragma unroll
  for (int x = 0; x <= L + 2; ++x)
#pragma unroll
    for (int y = 0; y <= L + 2; ++y)
      if (x + y <= L + 2) D[sym_pos(L + 2, x, y)] = fma(a, D[sym_pos(L + 2, x, y)], -sym_delta_at<L>(Y, x, y));
}

// eq:SMRT on order n: d'^(n) = sum_m (1 - om_m) d^(n,m) delta^m
//   = (1 - om_0) d^(n) - sum_{m>=1} (om_m - om_0) sym(d^(n,m) delta^m)
//   = (1 - om_0) d^(n) - delta [ (om_1 - om_0) d^(n,1) + (om_2 - om_0) delta d^(n,2) ]
// (delta is linear), so only the rank n-2 bracket is held beside d^(n).
template <int n>
__device__ __forceinline__ void relax_order(double* dn, const double* om) {
  double Y[n_sym(n - 2)];
  irreducible_part<n, 1>(dn, Y);
  const double c1 = om[1] - om[0];
#pragma unroll
  for (int i = 0; i < n_sym(n - 2); ++i) Y[i] *= c1;
  if constexpr (n >= 4) {
    double part[n_sym(n - 4)];
    irreducible_part<n, 2>(dn, part);
    const double c2 = om[2] - om[0];
#pragma unroll
    for (int i = 0; i < n_sym(n - 4); ++i) part[i] *= c2;
    double dp[n_sym(n - 2)];
    sym_delta<n - 4>(part, dp);
#pragma unroll
    for (int i = 0; i < n_sym(n - 2); ++i) Y[i] += dp[i];
  }
  sym_delta_update<n - 2>(Y, 1.0 - om[0], dn);
}

// ------------------------------------------------------------------ frame shift
// Coefficients of the binomial transform between the lattice frame and the
// local frame (u', theta): with generating functions
//   sum_j A_j t^j / j! = exp(u t + (theta-1) t^2 / 2)   (App. B closed form)
//   sum_j B_j t^j / j! = exp(-u t + (1-theta) t^2 / 2)
// one has theta^{n/2} He_n((x-u)/sqrt(theta)) = sum_k C(n,k) B_{n-k} He_k(x) and
// He_n(u + sqrt(theta) y) = sum_k C(n,k) theta^{k/2} A_{n-k} He_k(y).
template <int N>
__device__ __forceinline__ void shift_poly(double u, double c, double (&P)[N + 1]) {
  P[0] = 1.0;
  if constexpr (N >= 1) P[1] = u;
#pragma unroll
  for (int j = 1; j < N; ++j) P[j + 1] = u * P[j] + double(j) * c * P[j - 1];
}

// In-place lower-triangular transform along one axis of the multi-index simplex:
//   y_{..b..} = sum_{g <= b} C(b, g) P_{b-g} x_{..g..}
template <int N, int AXIS>
__device__ __forceinline__ void axis_transform(double* d, const double (&P)[N + 1]) {
#pragma unroll
  for (int o1 = 0; o1 <= N; ++o1)
#pragma unroll
    for (int o2 = 0; o2 <= N; ++o2)
#pragma unroll
      for (int bb = 0; bb <= N; ++bb) {
        const int b = N - bb;             // top-down keeps the inputs g < b unmodified
        if (o1 + o2 + b > N) continue;
        auto id = [&](int v) {
          return AXIS == 0 ? midx(v, o1, o2) : (AXIS == 1 ? midx(o1, v, o2) : midx(o1, o2, v));
        };
        double s = d[id(b)];
#pragma unroll
        for (int g = 0; g < N; ++g)
          if (g < b) s += binom(b, g) * P[b - g] * d[id(g)];
        d[id(b)] = s;
      }
}

template <int N>
__device__ __forceinline__ void scale_by_order(double* d, double s) {
  double p[N + 1];
  p[0] = 1.0;
#pragma unroll
  for (int n = 1; n <= N; ++n) p[n] = p[n - 1] * s;
#pragma unroll
  for (int i = 0; i < n_moments(N); ++i) {
    int n = 0;
#pragma unroll
    for (int k = 1; k <= N; ++k) n += (i >= order_start(k)) ? 1 : 0;
    d[i] *= p[n];
  }
}

}  // namespace lbsmrt
