// Adjoint step, loss seed and the deterministic reduction of per-block partials.
#pragma once
#include "adjoint.hpp"

namespace lbsmrt {

constexpr int kTauCols = (kMaxN + 1) * 3;   // dL/dtau[n][m] flattened as n*3+m

// Scatter of mu = P^T abar to the streaming sources: out[q][x - s_q] = sum_alpha He_alpha(c_q) abar_alpha.
// Populations whose source was a ghost cell (shock ends) are skipped.
// Plain (temporal) stores: the shifted chunks of neighbouring wavefronts complete each other's
// partial cache lines in L2 (with the non-temporal hint they went out as partial-line writes).
// LPN > 1: each lane of a node's group scatters the slabs ix = sub, sub + LPN, ... with the
// uniform pass count of gather_project64; a lane with no slab left repeats the last one, storing
// the values its owner stores to the same addresses in the same instruction.
template <int Q1, int N, bool SHOCK, int LPN = 1, class AB>
LBSMRT_PHASE void scatter_transpose_projection(const LatticeConst& L, const Pull<Q1>& P, const AB& ab,
                                                             float* __restrict__ out, long long stride) {
  constexpr int p = Q1 / 2;
  constexpr int P2 = n_sym(N);
#pragma unroll 1
  for (int k = 0; k < (Q1 + LPN - 1) / LPN; ++k) {
    const int ixr = (LPN > 1 ? P.sub : 0) + k * LPN;
    const int ix = (LPN == 1 || ixr < Q1) ? ixr : Q1 - 1;
    const int xs = source_x_e<Q1>(L, P, abscissa_of<Q1, LPN>(L, ix));
    if (SHOCK && xs < 0) continue;
    const unsigned xoff = (LPN == 1 ? 0u : static_cast<unsigned>(ix * Q1 * Q1) * static_cast<unsigned>(stride) * 4u) +
                          static_cast<unsigned>(P.row + xs) * 4u;
    double hx[N + 1];
    table_row<Q1, N, LPN>(L.He64, ix, hx);
    double u2[P2];
#pragma unroll
    for (int ay = 0; ay <= N; ++ay)
#pragma unroll
      for (int az = 0; az <= N; ++az) {
        if (ay + az > N) continue;
        double s = 0.0;
#pragma unroll
        for (int ax = 0; ax <= N; ++ax)
          if (ax + ay + az <= N) s = fma(ab[midx(ax, ay, az)], hx[ax], s);
        u2[pair_pos(ay, az)] = s;
      }
    float* __restrict__ slab = LPN == 1 ? out + static_cast<size_t>(ix * Q1 * Q1) * stride : out;
    auto zline = [&](int iy, const double (&v)[N + 1]) {
      float* __restrict__ line = slab + static_cast<size_t>(iy * Q1) * stride;
      const unsigned yoff = xoff + P.yo[iy];
      {
        double s = 0.0;
#pragma unroll
        for (int az = 0; az <= N; az += 2) s = fma(v[az], hermite_at_zero(az), s);
        store_at(line + static_cast<size_t>(p) * stride, yoff + P.zo[p], static_cast<float>(s));
      }
#pragma unroll
      for (int j = 1; j <= p; ++j) {
        double e = 0.0, o = 0.0;
#pragma unroll
        for (int az = 0; az <= N; ++az) {
          if (az & 1) o = fma(v[az], L.He64[p + j][az], o);
          else e = fma(v[az], L.He64[p + j][az], e);
        }
        store_at(line + static_cast<size_t>(p + j) * stride, yoff + P.zo[p + j], static_cast<float>(e + o));
        store_at(line + static_cast<size_t>(p - j) * stride, yoff + P.zo[p - j], static_cast<float>(e - o));
      }
    };
    {
      double v[N + 1];
#pragma unroll
      for (int az = 0; az <= N; ++az) {
        double s = 0.0;
#pragma unroll
        for (int ay = 0; ay <= N; ay += 2)
          if (ay + az <= N) s = fma(u2[pair_pos(ay, az)], hermite_at_zero(ay), s);
        v[az] = s;
      }
      zline(p, v);
    }
#pragma unroll
    for (int j = 1; j <= p; ++j) {
      double vp[N + 1], vm[N + 1];
#pragma unroll
      for (int az = 0; az <= N; ++az) {
        double e = 0.0, o = 0.0;
#pragma unroll
        for (int ay = 0; ay <= N; ++ay) {
          if (ay + az > N) continue;
          if (ay & 1) o = fma(u2[pair_pos(ay, az)], L.He64[p + j][ay], o);
          else e = fma(u2[pair_pos(ay, az)], L.He64[p + j][ay], e);
        }
        vp[az] = e + o;
        vm[az] = e - o;
      }
      zline(p + j, vp);
      zline(p - j, vm);
    }
  }
}

// Shock tubes: populations of node x that stream out through an end of the domain
// influence nothing; their adjoint is zero.
template <int Q1>
__device__ __forceinline__ void zero_outflow(const LatticeConst& L, const Pull<Q1>& P, float* __restrict__ out,
                                             long long stride) {
  const unsigned off = static_cast<unsigned>(P.node) * 4u;
#pragma unroll 1
  for (int ix = 0; ix < Q1; ++ix) {
    const int xd = P.x + L.e[ix] + L.k[0];
    if (xd >= 0 && xd < P.nx) continue;
    float* __restrict__ slab = out + static_cast<size_t>(ix * Q1 * Q1) * stride;
#pragma unroll
    for (int qs = 0; qs < Q1 * Q1; ++qs) store_at(slab + static_cast<size_t>(qs) * stride, off, 0.0f);
  }
}

// Fixed-order tree reduction of C values per thread over the block (blockDim.x a power of two
// <= 256): every column in the same pass, so one ladder of barriers serves all of them.
// red holds C * blockDim.x doubles.  Thread 0 receives the block sums in v.
template <int C>
__device__ __forceinline__ void block_sum_cols(double (&v)[C], double* red) {
  const int t = threadIdx.x;
  const int B = blockDim.x;
#pragma unroll
  for (int c = 0; c < C; ++c) red[c * B + t] = v[c];
  __syncthreads();
  for (int s = B / 2; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int c = 0; c < C; ++c) red[c * B + t] += red[c * B + t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = red[c * B];
  }
  __syncthreads();
}

// Work-items per block of the adjoint kernels: one wavefront, or (periodic domains, N <= 4)
// kAdjRowBlock, so that a work-group scatters whole 256-node rows and its shifted stores cover
// whole cache lines.
constexpr int kAdjBlock = 64;
constexpr int kAdjRowBlock = 256;

// Vector of M doubles in dynamic LDS, one per node, strided by the number of nodes B of the
// work-group (conflict-free); the stride is a compile-time constant so that every element address
// is the node's base plus an immediate offset.  The LPN lanes of a node's group share it: they
// hold bit-identical values (the group's sums are all-reduced) and write the same values.
template <int B>
struct LdsVec {
  double* base;
  __device__ __forceinline__ double operator()(int i) const { return base[i * B]; }
  __device__ __forceinline__ void set(int i, double v) const { base[i * B] = v; }
  __device__ __forceinline__ double& operator[](int i) const { return base[i * B]; }
  __device__ __forceinline__ LdsVec operator+(int k) const { return LdsVec{base + k * B}; }
};

// Dynamic LDS of the adjoint step per work-group of B work-items: d and z for each of its B / LPN
// nodes, and at N >= 5 with a node split over lanes also the adjoint moments (56 doubles, which
// in registers spill about 1 KB per work-item; with one lane per node they stay in registers, as
// a third vector per work-item would leave one 64-item work-group per compute unit).
template <int N, int LPN>
constexpr bool adjoint_moments_in_lds() { return N >= 5 && LPN > 1; }
template <int N, int LPN, int B>
constexpr size_t adjoint_lds_bytes() {
  return (adjoint_moments_in_lds<N, LPN>() ? 3 : 2) * sizeof(double) * n_moments(N) * (B / LPN);
}

// One adjoint step: lam_t = (d f_{t+1} / d f_t)^T lam_next, per-block partials of dL/dtau.
// Dynamic LDS (adjoint_lds_bytes): per node the local moments d and z = Lambda d', and at
// N >= 5 with lanes per node the adjoint moments abar; blocks of kAdjBlock work-items.
template <int Q1, int N, bool SHOCK, int LPN = 1, int B = kAdjBlock>
__global__ __launch_bounds__(B) void k_adjoint(LatticeConst L, StepArgs A, const float* __restrict__ f_t,
                                                 const float* __restrict__ lam_next, float* __restrict__ lam_t,
                                                 double* __restrict__ partial) {
  constexpr int M = n_moments(N);
  constexpr int NT = n_tau_slots(N);
  extern __shared__ double lds[];
  __shared__ double red[NT * B];
  Pull<Q1> P;
  const bool active = make_pull<Q1, LPN>(L, A, P);
  double tb[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) tb[i] = 0.0;
  if (active) {
    constexpr int G = B / LPN;                       // nodes per work-group
    const int g = static_cast<int>(threadIdx.x) / LPN;
    const LdsVec<G> dv{lds + g};
    const LdsVec<G> zv{lds + M * G + g};
    Macro mac;
    {
      double d[M];
      double S[5];
      gather_project64<Q1, N, SHOCK, LPN>(L, A, f_t, P, d);
      sums_from_a<N>(d, L, S);
      mac = macro_from_sums(L, S, A.err);
      mac.tsc = P.tsc;
      to_local<N>(d, mac);
#pragma unroll
      for (int i = 0; i < M; ++i) dv.set(i, d[i]);
    }
    if constexpr (adjoint_moments_in_lds<N, LPN>()) {
      const LdsVec<G> av{lds + 2 * M * G + g};
      {
        double ab[M];
        own_project64<Q1, N, true, LPN>(L, lam_next, A.stride, P.node, ab, P.sub);
#pragma unroll
        for (int i = 0; i < M; ++i) av.set(i, ab[i]);
      }
      node_adjoint<N>(L, mac, dv, zv, av, tb);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      scatter_transpose_projection<Q1, N, SHOCK, LPN>(L, P, av, lam_t, A.stride);
    } else {
      double ab[M];
      own_project64<Q1, N, true, LPN>(L, lam_next, A.stride, P.node, ab, P.sub);
      node_adjoint<N>(L, mac, dv, zv, ab, tb);
      scatter_transpose_projection<Q1, N, SHOCK, LPN>(L, P, ab, lam_t, A.stride);
    }
    // every lane of a group zeroes the same out-flowing populations (identical stores)
    if (SHOCK && P.bc_x == 1) zero_outflow<Q1>(L, P, lam_t, A.stride);
    if (LPN > 1 && P.sub != 0) {
#pragma unroll
      for (int i = 0; i < NT; ++i) tb[i] = 0.0;   // the group's dL/dtau counted once
    }
  }
  block_sum_cols<NT>(tb, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT; ++i) partial[static_cast<size_t>(blockIdx.x) * NT + i] = tb[i];
  }
}

// Deterministic two-stage column sums of per-block partials [rows][cols], cols <= kTauCols.
// Stage 1 (kReduceBlocks work-groups of 256): work-item t of group g sums rows
// g + G t, g + G (t + 256), ... in that order for every column, then one fixed tree per
// group; writes stage[g][col].  Stage 2 sums the G rows of stage the same way in one group.
constexpr int kReduceBlocks = 256;

// (internal linkage: every translation unit that launches it holds its own copy)
static __global__ __launch_bounds__(256) void k_reduce_stage1(const double* __restrict__ partial, int rows, int cols,
                                                       double* __restrict__ stage) {
  __shared__ double red[kTauCols * 256];
  double s[kTauCols];
#pragma unroll
  for (int c = 0; c < kTauCols; ++c) s[c] = 0.0;
  for (int r = blockIdx.x + gridDim.x * static_cast<int>(threadIdx.x); r < rows;
       r += gridDim.x * static_cast<int>(blockDim.x)) {
#pragma unroll
    for (int c = 0; c < kTauCols; ++c)
      if (c < cols) s[c] += partial[static_cast<size_t>(r) * cols + c];
  }
  block_sum_cols<kTauCols>(s, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < kTauCols; ++c)
      if (c < cols) stage[static_cast<size_t>(blockIdx.x) * cols + c] = s[c];
  }
}

// Stage 2 (one group of kReduceBlocks work-items): column sums of stage[kReduceBlocks][NT].
template <int NT>
__device__ __forceinline__ void stage2_sums(const double* __restrict__ stage, double (&s)[NT], double* red) {
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < NT; ++c) s[c] = stage[static_cast<size_t>(t) * NT + c];
  block_sum_cols<NT>(s, red);
}

// Stage 2 for dL/dtau: out[n*3+m] += column tau_slot(n,m).  Launch: 1 x kReduceBlocks.
template <int N>
__global__ __launch_bounds__(kReduceBlocks) void k_reduce_tau(const double* __restrict__ stage,
                                                              double* __restrict__ out) {
  constexpr int NT = n_tau_slots(N);
  __shared__ double red[NT * kReduceBlocks];
  double s[NT];
  stage2_sums<NT>(stage, s, red);
  if (threadIdx.x == 0) {
    for (int nn = 2; nn <= N; ++nn)
      for (int mm = 0; 2 * mm <= nn; ++mm)
        if (!(nn == 2 && mm == 1)) out[nn * 3 + mm] += s[tau_slot(nn, mm)];
  }
}

// The same column sums in one launch when the partials are few (rows <= kSmallReduceRows): work-item
// t of one group sums rows t, t + 256, ... in that order, then one fixed tree.  (Small domains:
// the two-stage form cost two launches of about 9 and 5 us beside a ~45 us adjoint step.)
constexpr int kSmallReduceRows = 16 * kReduceBlocks;
template <int N>
__global__ __launch_bounds__(kReduceBlocks) void k_reduce_tau_rows(const double* __restrict__ partial, int rows,
                                                                   double* __restrict__ out) {
  constexpr int NT = n_tau_slots(N);
  __shared__ double red[NT * kReduceBlocks];
  double s[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) s[c] = 0.0;
  for (int r = static_cast<int>(threadIdx.x); r < rows; r += kReduceBlocks) {
#pragma unroll
    for (int c = 0; c < NT; ++c) s[c] += partial[static_cast<size_t>(r) * NT + c];
  }
  block_sum_cols<NT>(s, red);
  if (threadIdx.x == 0) {
    for (int nn = 2; nn <= N; ++nn)
      for (int mm = 0; 2 * mm <= nn; ++mm)
        if (!(nn == 2 && mm == 1)) out[nn * 3 + mm] += s[tau_slot(nn, mm)];
  }
}

// Seed of the adjoint for L = sum_x [s0^2 (rho - rho*)^2 + s1^2 (theta - theta*)^2 + s2^2 (q_x - q_x*)^2]
// on the pre-collision moments of state f.  lam[i][x - s_i] = dL/dg_i(x); per-block partial of L.
template <int Q1, int N, bool SHOCK>
__global__ __launch_bounds__(256) void k_loss_seed(LatticeConst L, StepArgs A, const float* __restrict__ f,
                                                   const double* __restrict__ target, long long n_nodes, double s0,
                                                   double s1, double s2, float* __restrict__ lam,
                                                   double* __restrict__ partial) {
  constexpr int M = n_moments(N);
  constexpr int p = Q1 / 2;
  __shared__ double red[256];
  Pull<Q1> P;
  const bool active = make_pull<Q1>(L, A, P);
  double ell = 0.0;
  if (active) {
    double d[M];
    double S[5];
    gather_project64<Q1, N, SHOCK>(L, A, f, P, d);
    sums_from_a<N>(d, L, S);
    const Macro mac = macro_from_sums(L, S, A.err);
    to_local<N>(d, mac);
    const double rho = mac.rho, th = mac.th;
    const double u[3] = {mac.ux, mac.uy, mac.uz};
    double t3[3];
    sym_trace<1>(d + order_start(3), t3);
    const double qx = 0.5 * th * sqrt(th) * t3[0];
    // pressure tensor P = theta (d2 + rho delta), row x: (xx, xy, xz)
    const double Pxx = th * (d[midx(2, 0, 0)] + rho), Pxy = th * d[midx(1, 1, 0)], Pxz = th * d[midx(1, 0, 1)];
    const double er = rho - target[P.node], et = th - target[n_nodes + P.node], eq = qx - target[2 * n_nodes + P.node];
    ell = s0 * s0 * er * er + s1 * s1 * et * et + s2 * s2 * eq * eq;
    const double cr = 2.0 * s0 * s0 * er, ct = 2.0 * s1 * s1 * et, cq = 2.0 * s2 * s2 * eq;
    const double ir = 1.0 / rho;
    const double kx = 1.5 * rho * th + Pxx;
#pragma unroll 1
    for (int ix = 0; ix < Q1; ++ix) {
      const int xs = source_x<Q1>(L, P, ix);
      if (SHOCK && xs < 0) continue;
      const unsigned xoff = static_cast<unsigned>(P.row + xs) * 4u;
      const double cx = L.r * L.e[ix] - u[0];
#pragma unroll
      for (int iy = 0; iy < Q1; ++iy) {
        const double cy = L.r * L.e[iy] - u[1];
#pragma unroll
        for (int iz = 0; iz < Q1; ++iz) {
          const double cz = L.r * L.e[iz] - u[2];
          const double c2 = cx * cx + cy * cy + cz * cz;
          const double dth = (c2 * (1.0 / 3.0) - th) * ir;
          const double dq = 0.5 * cx * c2 - (kx * cx + Pxy * cy + Pxz * cz) * ir;
          const double G = cr + ct * dth + cq * dq;
          const int q = (ix * Q1 + iy) * Q1 + iz;
          store_at(lam + static_cast<size_t>(q) * A.stride, xoff + P.yo[iy] + P.zo[iz], static_cast<float>(G));
        }
      }
    }
    if (SHOCK && P.bc_x == 1) zero_outflow<Q1>(L, P, lam, A.stride);
    (void)p;
  }
  double v[1] = {ell};
  block_sum_cols<1>(v, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

// Stage 2 for the loss (one column): out[0] (+)= sum over the kReduceBlocks rows of stage.
// Launch: 1 x kReduceBlocks.
static __global__ __launch_bounds__(kReduceBlocks) void k_reduce_loss(const double* __restrict__ stage,
                                                               double* __restrict__ out, int accumulate) {
  __shared__ double red[kReduceBlocks];
  double s[1];
  stage2_sums<1>(stage, s, red);
  if (threadIdx.x == 0) out[0] = accumulate ? out[0] + s[0] : s[0];
}

}  // namespace lbsmrt
