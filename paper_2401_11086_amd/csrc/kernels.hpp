// gfx950 kernels of the LB-SMRT step: fused pull-stream + SMRT collision,
// moments, equilibrium fill.  One work-item per lattice node; the f state is
// structure-of-arrays float32 [Q][stride], so for every population q the
// 64 lanes of a wave touch 64 consecutive nodes (coalesced 256-byte rows).
// The projection and reconstruction contractions are sum-factorised over the
// tensor-product velocity set (x, then y, then z), FP32 FMA with the 1D
// Hermite tables held in scalar registers; the conserved sums, the frame
// shift, the irreducible split and the relaxation run in FP64.
#pragma once
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "smrt_node.hpp"

namespace lbsmrt {

struct DomainDev {
  long long off;      // first node of the domain in the global node space
  int nx, ny, nz;
  int bc_x;           // 0 periodic, 1 fixed Maxwellian ends
  int ghost;          // column of the left ghost state in the ghost table (right = ghost+1)
  int pad;
  double tau_scale;   // multiplies every tau_nm of this domain
};

struct BlockDev {
  int dom;            // domain handled by this work-group
  int first;          // first local node of the work-group
};

struct StepArgs {
  const DomainDev* doms;
  const BlockDev* blocks;
  const float* ghosts;       // [Q][n_ghost]
  int n_ghost;
  long long stride;
  int* err;
  double* dtau;              // adjoint only: dL/dtau [6][3]
};

enum : int { kErrState = 1, kErrTimeout = 2 };

// Loads and stores at a wave-uniform base plus a 32-bit byte offset, so the
// compiler can use the scalar-base (saddr) form of global memory instructions.
__device__ __forceinline__ float load_at(const float* __restrict__ base, unsigned byte_off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ __forceinline__ void store_at(float* __restrict__ base, unsigned byte_off, float v) {
  *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// Store of a rebuilt population; NT marks it non-temporal (it is not read again in this step).
// Used for periodic boxes, where the step streams HBM (measured 1.8 % faster on a 256^3 box);
// the shock kernels keep plain stores, whose uniform-base addressing matters more to their
// VALU-bound wavefronts than the hint (the non-temporal form is addressed by 64-bit lane pointers).
template <bool NT>
__device__ __forceinline__ void store_pop(float* __restrict__ base, unsigned byte_off, float v) {
  float* ptr = reinterpret_cast<float*>(reinterpret_cast<char*>(base) + byte_off);
  if constexpr (NT) __builtin_nontemporal_store(v, ptr);
  else *ptr = v;
}

template <int Q1, int N>
struct Shape {
  static constexpr int M = n_moments(N);
  static constexpr int P2 = n_sym(N);
  static constexpr int Q = Q1 * Q1 * Q1;
};

// Node coordinates and source offsets of the pull stream g_i(x) = f*_i(x - e_i - k).
template <int Q1>
struct Pull {
  int node;                  // global node index of this work-item
  int row;                   // global node index of (x = 0, y, z) of this work-item
  int x, nx, bc_x;
  unsigned yo[Q1];           // byte offset of source row ys*nx per iy
  unsigned zo[Q1];           // byte offset of source plane zs*nx*ny per iz
  int gcol;                  // left ghost column
  int sub;                   // lane of this work-item within its node's group (0 .. LPN-1)
  double tsc;                // tau scale of the domain
};

// Node of this work-item: LPN consecutive work-items share one node (block b covers nodes
// first .. first + blockDim.x / LPN - 1 of its domain).
template <int Q1, int LPN = 1>
__device__ __forceinline__ bool make_pull(const LatticeConst& L, const StepArgs& A, Pull<Q1>& P,
                                          int work_block = -1) {
  const BlockDev bd = A.blocks[work_block < 0 ? static_cast<int>(blockIdx.x) : work_block];
  const DomainDev D = A.doms[bd.dom];
  const int local = bd.first + static_cast<int>(threadIdx.x) / LPN;
  P.sub = static_cast<int>(threadIdx.x) % LPN;
  const int nxy = D.nx * D.ny;
  if (local >= nxy * D.nz) return false;
  const int x = local % D.nx;
  const int y = (local / D.nx) % D.ny;
  const int z = local / nxy;
  P.node = static_cast<int>(D.off) + local;
  P.row = static_cast<int>(D.off);
  P.x = x;
  P.nx = D.nx;
  P.bc_x = D.bc_x;
  P.gcol = D.ghost;
  P.tsc = D.tau_scale;
#pragma unroll
  for (int j = 0; j < Q1; ++j) {
    int t = (y - (L.e[j] + L.k[1])) % D.ny;
    P.yo[j] = static_cast<unsigned>((t < 0 ? t + D.ny : t) * D.nx) * 4u;
    t = (z - (L.e[j] + L.k[2])) % D.nz;
    P.zo[j] = static_cast<unsigned>((t < 0 ? t + D.nz : t) * nxy) * 4u;
  }
  return true;
}


// Row ix of a per-abscissa table.  With ix uniform across the wavefront (LPN = 1) this is a
// plain (scalar) lookup; with ix differing between lanes it is a select over the Q1 rows, which
// keeps the table in scalar registers.
template <int Q1, int N, int LPN, class T, int R, int C>
__device__ __forceinline__ void table_row(const T (&tab)[R][C], int ix, T (&out)[N + 1]) {
  if constexpr (LPN == 1) {
#pragma unroll
    for (int n = 0; n <= N; ++n) out[n] = tab[ix][n];
  } else {
#pragma unroll
    for (int n = 0; n <= N; ++n) out[n] = tab[0][n];
#pragma unroll
    for (int j = 1; j < Q1; ++j) {
      const bool hit = ix == j;
#pragma unroll
      for (int n = 0; n <= N; ++n) out[n] = hit ? tab[j][n] : out[n];
    }
  }
}

template <int Q1, int LPN>
__device__ __forceinline__ int abscissa_of(const LatticeConst& L, int ix) {
  if constexpr (LPN == 1) {
    return L.e[ix];
  } else {
    int e = L.e[0];
#pragma unroll
    for (int j = 1; j < Q1; ++j) e = ix == j ? L.e[j] : e;
    return e;
  }
}

// Source x of the population column with 1D integer e: >= 0 inside, -1 / -2 for the left /
// right ghost.  source_x takes the column index ix.
template <int Q1>
__device__ __forceinline__ int source_x_e(const LatticeConst& L, const Pull<Q1>& P, int e) {
  int xs = P.x - (e + L.k[0]);
  if (P.bc_x == 0) {
    xs %= P.nx;
    if (xs < 0) xs += P.nx;
    return xs;
  }
  return xs < 0 ? -1 : (xs >= P.nx ? -2 : xs);
}

template <int Q1>
__device__ __forceinline__ int source_x(const LatticeConst& L, const Pull<Q1>& P, int ix) {
  return source_x_e<Q1>(L, P, L.e[ix]);
}

// Gather the streamed populations and project them (eq:an), sum-factorised:
//   a[ax,ay,az] = sum_ix He_ax(c_ix) sum_iy He_ay(c_iy) sum_iz He_az(c_iz) g[ix,iy,iz]
// in FP32, plus the conserved moments in FP64 through the weights Hd dual to the float32 rebuild
// table: S = (a_0, a_100, a_010, a_001, a_200 + a_020 + a_002), so that a node rebuilt with the
// float32 table hands the same rho, j and energy to the next step's projection.
// The x loop stays rolled (one 2D slab of Q1*Q1 populations per iteration).
template <int Q1, int N, bool SHOCK>
__device__ __forceinline__ void gather_project(const LatticeConst& L, const StepArgs& A,
                                               const float* __restrict__ f, const Pull<Q1>& P,
                                               float (&a)[Shape<Q1, N>::M], double (&S)[5]) {
  constexpr int P2 = Shape<Q1, N>::P2;
#pragma unroll
  for (int i = 0; i < Shape<Q1, N>::M; ++i) a[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) S[i] = 0.0;
#pragma unroll 1
  for (int ix = 0; ix < Q1; ++ix) {
    float t2[P2];
#pragma unroll
    for (int i = 0; i < P2; ++i) t2[i] = 0.f;
    // per slab: U0 = (0,0), U1y = (1,0), U1z = (0,1), U2 = (2,0) + (0,2) Hermite orders in (y, z)
    double U0 = 0.0, U1y = 0.0, U1z = 0.0, U2 = 0.0;
    const int xs = source_x<Q1>(L, P, ix);
    const float* __restrict__ fx = f + static_cast<size_t>(ix * Q1 * Q1) * A.stride;
    const unsigned xoff = static_cast<unsigned>(P.row + xs) * 4u;
    // issue the whole slab of Q1*Q1 loads before any use (memory-level parallelism)
    float gs[Q1 * Q1];
#pragma unroll
    for (int iy = 0; iy < Q1; ++iy) {
      const unsigned xyoff = xoff + P.yo[iy];
#pragma unroll
      for (int iz = 0; iz < Q1; ++iz) {
        const int qs = iy * Q1 + iz;   // population inside the slab
        if constexpr (SHOCK) {
          if (xs >= 0) {
            gs[qs] = load_at(fx + static_cast<size_t>(qs) * A.stride, xyoff + P.zo[iz]);
          } else {
            gs[qs] = A.ghosts[static_cast<size_t>(ix * Q1 * Q1 + qs) * A.n_ghost + P.gcol + (xs == -1 ? 0 : 1)];
          }
        } else {
          gs[qs] = load_at(fx + static_cast<size_t>(qs) * A.stride, xyoff + P.zo[iz]);
        }
      }
    }
#pragma unroll
    for (int iy = 0; iy < Q1; ++iy) {
      float t1[N + 1];
#pragma unroll
      for (int n = 0; n <= N; ++n) t1[n] = 0.f;
      double V0 = 0.0, V1 = 0.0, V2 = 0.0;
#pragma unroll
      for (int iz = 0; iz < Q1; ++iz) {
        const float g = gs[iy * Q1 + iz];
#pragma unroll
        for (int n = 0; n <= N; ++n) t1[n] = fmaf(g, L.He[iz][n], t1[n]);
        const double gd = static_cast<double>(g);
        V0 = fma(gd, L.Hd[iz][0], V0);
        V1 = fma(gd, L.Hd[iz][1], V1);
        V2 = fma(gd, L.Hd[iz][2], V2);
      }
#pragma unroll
      for (int ay = 0; ay <= N; ++ay)
#pragma unroll
        for (int az = 0; az <= N; ++az)
          if (ay + az <= N) t2[pair_pos(ay, az)] = fmaf(t1[az], L.He[iy][ay], t2[pair_pos(ay, az)]);
      U0 = fma(V0, L.Hd[iy][0], U0);
      U1y = fma(V0, L.Hd[iy][1], U1y);
      U1z = fma(V1, L.Hd[iy][0], U1z);
      U2 = fma(V0, L.Hd[iy][2], fma(V2, L.Hd[iy][0], U2));
    }
    float hx[N + 1];
#pragma unroll
    for (int n = 0; n <= N; ++n) hx[n] = L.He[ix][n];
#pragma unroll
    for (int ax = 0; ax <= N; ++ax)
#pragma unroll
      for (int ay = 0; ay <= N; ++ay)
#pragma unroll
        for (int az = 0; az <= N; ++az)
          if (ax + ay + az <= N) a[midx(ax, ay, az)] = fmaf(t2[pair_pos(ay, az)], hx[ax], a[midx(ax, ay, az)]);
    S[0] = fma(U0, L.Hd[ix][0], S[0]);
    S[1] = fma(U0, L.Hd[ix][1], S[1]);
    S[2] = fma(U1y, L.Hd[ix][0], S[2]);
    S[3] = fma(U1z, L.Hd[ix][0], S[3]);
    S[4] = fma(U0, L.Hd[ix][2], fma(U2, L.Hd[ix][0], S[4]));
  }
}

// ---------------------------------------------------------------- FP64 folded contractions
// The 1D stencil is symmetric (e_{p+j} = -e_{p-j}) and He_n has the parity of n,
// so sums over a +-e pair split into an even part (sum of the pair) and an odd
// part (difference): every 1D contraction over Q1 = 2p+1 points costs p+1
// multiply-adds per output instead of Q1.

// 1D table of a contraction: He_n(c_j) (RW = false) or w_j He_n(c_j) / n! (RW = true).
template <bool RW>
__device__ __forceinline__ double tab(const LatticeConst& L, int j, int n) {
  return RW ? L.Rw64[j][n] : L.He64[j][n];
}
template <bool RW>
__device__ __forceinline__ double tab_center(const LatticeConst& L, int p, int n) {
  return (n & 1) ? 0.0 : (RW ? L.Rw64[p][n] : hermite_at_zero(n));
}

// One z line of a slab: t1[n] = sum_iz T_n(c_iz) g[iz], FP64.
template <int Q1, int N, bool RW = false>
__device__ __forceinline__ void fold_line_project(const LatticeConst& L, const float* g, double (&t1)[N + 1]) {
  constexpr int p = Q1 / 2;
  double P[p], Mn[p];
#pragma unroll
  for (int j = 1; j <= p; ++j) {
    const double gp = static_cast<double>(g[p + j]);
    const double gm = static_cast<double>(g[p - j]);
    P[j - 1] = gp + gm;
    Mn[j - 1] = gp - gm;
  }
  const double g0 = static_cast<double>(g[p]);
#pragma unroll
  for (int n = 0; n <= N; ++n) {
    double s = (n & 1) ? 0.0 : tab_center<RW>(L, p, n) * g0;
#pragma unroll
    for (int j = 1; j <= p; ++j) s = fma(tab<RW>(L, p + j, n), (n & 1) ? Mn[j - 1] : P[j - 1], s);
    t1[n] = s;
  }
}

// One slab (fixed ix): t2[ay,az] = sum_{iy,iz} T_ay(c_iy) T_az(c_iz) g[iy][iz], FP64, folded in y and z.
template <int Q1, int N, bool RW = false>
__device__ __forceinline__ void fold_slab_project(const LatticeConst& L, const float (&gs)[Q1 * Q1],
                                                  double (&t2)[n_sym(N)]) {
  constexpr int p = Q1 / 2;
  {
    double tc[N + 1];
    fold_line_project<Q1, N, RW>(L, gs + p * Q1, tc);
#pragma unroll
    for (int ay = 0; ay <= N; ++ay)
#pragma unroll
      for (int az = 0; az <= N; ++az)
        if (ay + az <= N) t2[pair_pos(ay, az)] = (ay & 1) ? 0.0 : tab_center<RW>(L, p, ay) * tc[az];
  }
#pragma unroll
  for (int j = 1; j <= p; ++j) {
    double tp[N + 1], tm[N + 1];
    fold_line_project<Q1, N, RW>(L, gs + (p + j) * Q1, tp);
    fold_line_project<Q1, N, RW>(L, gs + (p - j) * Q1, tm);
#pragma unroll
    for (int az = 0; az <= N; ++az) {
      const double Pz = tp[az] + tm[az];
      const double Mz = tp[az] - tm[az];
#pragma unroll
      for (int ay = 0; ay <= N; ++ay)
        if (ay + az <= N) t2[pair_pos(ay, az)] = fma(tab<RW>(L, p + j, ay), (ay & 1) ? Mz : Pz, t2[pair_pos(ay, az)]);
    }
  }
}

// Sum over the LPN (2, 4 or 8) consecutive lanes of a group, every lane receiving the total, by
// DPP permutations: lane ^ 1, lane ^ 2 (quad_perm), then the mirror within each half-row of 8
// (after the first two steps each quad holds one value, so the mirror pairs the two quads).
// Floating-point addition is commutative, so all lanes of a group end with bit-identical sums.
template <int CTRL>
__device__ __forceinline__ double dpp_move_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                        static_cast<unsigned>(lo));
}

template <int LPN, int M>
__device__ __forceinline__ void group_allreduce(double (&a)[M]) {
  static_assert(LPN == 2 || LPN == 4 || LPN == 8 || LPN == 16, "groups of 2, 4, 8 or 16 lanes");
  constexpr int kSwap1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);   // quad_perm [1,0,3,2]
  constexpr int kSwap2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);   // quad_perm [2,3,0,1]
  constexpr int kHalfMirror = 0x141;                            // row_half_mirror
  constexpr int kMirror = 0x140;                                // row_mirror
#pragma unroll
  for (int i = 0; i < M; ++i) a[i] += dpp_move_f64<kSwap1>(a[i]);
  if constexpr (LPN >= 4) {
#pragma unroll
    for (int i = 0; i < M; ++i) a[i] += dpp_move_f64<kSwap2>(a[i]);
  }
  if constexpr (LPN >= 8) {
#pragma unroll
    for (int i = 0; i < M; ++i) a[i] += dpp_move_f64<kHalfMirror>(a[i]);
  }
  if constexpr (LPN == 16) {   // each lane's mirror lies in the other half-row, which holds its sum
#pragma unroll
    for (int i = 0; i < M; ++i) a[i] += dpp_move_f64<kMirror>(a[i]);
  }
}

// As fold_slab_project, with the populations of each z line fetched just before it is folded
// (load(iy, line) fills line[iz]); keeps at most two lines of a slab in registers.
template <int Q1, int N, bool RW, class LineLoad>
__device__ __forceinline__ void fold_slab_project_lines(const LatticeConst& L, const LineLoad& load,
                                                        double (&t2)[n_sym(N)]) {
  constexpr int p = Q1 / 2;
  {
    float g[Q1];
    load(p, g);
    double tc[N + 1];
    fold_line_project<Q1, N, RW>(L, g, tc);
#pragma unroll
    for (int ay = 0; ay <= N; ++ay)
#pragma unroll
      for (int az = 0; az <= N; ++az)
        if (ay + az <= N) t2[pair_pos(ay, az)] = (ay & 1) ? 0.0 : tab_center<RW>(L, p, ay) * tc[az];
  }
#pragma unroll
  for (int j = 1; j <= p; ++j) {
    float gp[Q1], gm[Q1];
    load(p + j, gp);
    load(p - j, gm);
    double tp[N + 1], tm[N + 1];
    fold_line_project<Q1, N, RW>(L, gp, tp);
    fold_line_project<Q1, N, RW>(L, gm, tm);
#pragma unroll
    for (int az = 0; az <= N; ++az) {
      const double Pz = tp[az] + tm[az];
      const double Mz = tp[az] - tm[az];
#pragma unroll
      for (int ay = 0; ay <= N; ++ay)
        if (ay + az <= N) t2[pair_pos(ay, az)] = fma(tab<RW>(L, p + j, ay), (ay & 1) ? Mz : Pz, t2[pair_pos(ay, az)]);
    }
  }
}

// FP64 projection of a node's own populations (no streaming) with table T:
//   out[ax,ay,az] = sum_{ix,iy,iz} T_ax(c_ix) T_ay(c_iy) T_az(c_iz) v[q]
template <int Q1, int N, bool RW, int LPN = 1>
LBSMRT_PHASE void own_project64(const LatticeConst& L, const float* __restrict__ v, long long stride,
                                              int node, double (&out)[n_moments(N)], int sub = 0) {
  constexpr int P2 = n_sym(N);
#pragma unroll
  for (int i = 0; i < n_moments(N); ++i) out[i] = 0.0;
  // LPN > 1: the slab split of gather_project64 (uniform pass count, zero weight on a repeat)
#pragma unroll 1
  for (int k = 0; k < (Q1 + LPN - 1) / LPN; ++k) {
    const int ixr = (LPN > 1 ? sub : 0) + k * LPN;
    const int ix = (LPN == 1 || ixr < Q1) ? ixr : Q1 - 1;
    const float* __restrict__ vx = LPN == 1 ? v + static_cast<size_t>(ix * Q1 * Q1) * stride : v;
    const unsigned off = (LPN == 1 ? 0u : static_cast<unsigned>(ix * Q1 * Q1) * static_cast<unsigned>(stride) * 4u) +
                         static_cast<unsigned>(node) * 4u;
    float gs[Q1 * Q1];
#pragma unroll
    for (int qs = 0; qs < Q1 * Q1; ++qs) gs[qs] = load_at(vx + static_cast<size_t>(qs) * stride, off);
    double t2[P2];
    fold_slab_project<Q1, N, RW>(L, gs, t2);
    double hx[N + 1];
    if constexpr (RW) table_row<Q1, N, LPN>(L.Rw64, ix, hx);
    else table_row<Q1, N, LPN>(L.He64, ix, hx);
    if (LPN > 1 && ixr >= Q1) {
#pragma unroll
      for (int n = 0; n <= N; ++n) hx[n] = 0.0;
    }
#pragma unroll
    for (int ax = 0; ax <= N; ++ax)
#pragma unroll
      for (int ay = 0; ay <= N; ++ay)
#pragma unroll
        for (int az = 0; az <= N; ++az)
          if (ax + ay + az <= N) out[midx(ax, ay, az)] = fma(t2[pair_pos(ay, az)], hx[ax], out[midx(ax, ay, az)]);
  }
  if constexpr (LPN > 1) group_allreduce<LPN, n_moments(N)>(out);
}

// Gather + FP64 projection (eq:an): a[ax,ay,az] = sum_ix He_ax(c_ix) t2_ix[ay,az].
// rho = a_0, j = a_1 and sum g |c|^2 = sum_k a_{2 e_k} + 3 rho come out exactly in FP64.
template <int Q1, int N, bool SHOCK, int LPN = 1>
LBSMRT_PHASE void gather_project64(const LatticeConst& L, const StepArgs& A,
                                                 const float* __restrict__ f, const Pull<Q1>& P,
                                                 double (&a)[Shape<Q1, N>::M]) {
  constexpr int P2 = Shape<Q1, N>::P2;
#pragma unroll
  for (int i = 0; i < Shape<Q1, N>::M; ++i) a[i] = 0.0;
#pragma unroll 1
  // With LPN > 1 every lane makes the same number of passes (uniform control flow); a lane with
  // no slab left repeats the last slab with zero weight.
  for (int k = 0; k < (Q1 + LPN - 1) / LPN; ++k) {
    const int ixr = (LPN > 1 ? P.sub : 0) + k * LPN;
    const int ix = (LPN == 1 || ixr < Q1) ? ixr : Q1 - 1;
    const int xs = source_x_e<Q1>(L, P, abscissa_of<Q1, LPN>(L, ix));
    // slab ix: a uniform base pointer when every lane works on the same slab; otherwise the
    // slab's offset goes into each lane's 32-bit byte offset (Q * stride * 4 < 2^32 then)
    const float* __restrict__ fx = LPN == 1 ? f + static_cast<size_t>(ix * Q1 * Q1) * A.stride : f;
    const unsigned slab_off = LPN == 1 ? 0u : static_cast<unsigned>(ix * Q1 * Q1) * static_cast<unsigned>(A.stride) * 4u;
    // shock ends: every lane loads from an in-domain address; lanes whose source is a ghost
    // cell then take the ghost value, on a path only waves that touch an end execute
    const bool ghost = SHOCK && xs < 0;
    const unsigned xoff = slab_off + static_cast<unsigned>(P.row + (ghost ? 0 : xs)) * 4u;
    const bool any_ghost = SHOCK && __any(ghost);
    // ghost value of population (ix, iy, iz): ghosts[(ix Q1^2 + iy Q1 + iz) n_ghost + column]
    const unsigned goff = static_cast<unsigned>(ix * Q1 * Q1 * A.n_ghost + P.gcol + (xs == -2 ? 1 : 0)) * 4u;
    auto load = [&](int iy, float (&line)[Q1]) {
      const unsigned xyoff = xoff + P.yo[iy];
#pragma unroll
      for (int iz = 0; iz < Q1; ++iz)
        line[iz] = load_at(fx + static_cast<size_t>(iy * Q1 + iz) * A.stride, xyoff + P.zo[iz]);
      if (any_ghost) {
#pragma unroll
        for (int iz = 0; iz < Q1; ++iz) {
          const float gv = load_at(A.ghosts + static_cast<size_t>(iy * Q1 + iz) * A.n_ghost, goff);
          line[iz] = ghost ? gv : line[iz];
        }
      }
    };
    double t2[P2];
    fold_slab_project_lines<Q1, N, false>(L, load, t2);
    double hx[N + 1];
    table_row<Q1, N, LPN>(L.He64, ix, hx);
    if (LPN > 1 && ixr >= Q1) {
#pragma unroll
      for (int n = 0; n <= N; ++n) hx[n] = 0.0;
    }
#pragma unroll
    for (int ax = 0; ax <= N; ++ax)
#pragma unroll
      for (int ay = 0; ay <= N; ++ay)
#pragma unroll
        for (int az = 0; az <= N; ++az)
          if (ax + ay + az <= N) a[midx(ax, ay, az)] = fma(t2[pair_pos(ay, az)], hx[ax], a[midx(ax, ay, az)]);
  }
  if constexpr (LPN > 1) group_allreduce<LPN, Shape<Q1, N>::M>(a);
}

// Per-slab source of the additive collision (no addition for the regularised rebuild).
struct NoAdd {
  static constexpr bool active = false;
  template <int Q1>
  __device__ void line(int, float (&)[Q1]) const {}
};
struct NoAddSource {
  __device__ NoAdd slab(int) const { return NoAdd{}; }
};

// Additive collision f* = g + R (a' - a): the pulled populations g of slab ix, loaded again at
// store time with the gather's addressing (uniform slab base, ghost columns at shock ends).
template <int Q1, bool SHOCK>
struct PulledSlab {
  static constexpr bool active = true;
  const float* __restrict__ fx;
  const float* __restrict__ ghosts;
  const Pull<Q1>* P;
  long long stride;
  int n_ghost;
  unsigned xoff, goff;
  bool ghost, any_ghost;
  // the pulled values of z line iy, all loaded before the line's stores (the compiler cannot
  // move a load past a store it does not know to be disjoint)
  __device__ void line(int iy, float (&g)[Q1]) const {
#pragma unroll
    for (int iz = 0; iz < Q1; ++iz)
      g[iz] = load_at(fx + static_cast<size_t>(iy * Q1 + iz) * stride, xoff + P->yo[iy] + P->zo[iz]);
    if (SHOCK && any_ghost) {
#pragma unroll
      for (int iz = 0; iz < Q1; ++iz) {
        const float gv = load_at(ghosts + static_cast<size_t>(iy * Q1 + iz) * n_ghost, goff);
        g[iz] = ghost ? gv : g[iz];
      }
    }
  }
};
template <int Q1, bool SHOCK>
struct PulledSource {
  const LatticeConst* L;
  const StepArgs* A;
  const float* __restrict__ f;
  const Pull<Q1>* P;
  __device__ PulledSlab<Q1, SHOCK> slab(int ix) const {
    PulledSlab<Q1, SHOCK> s;
    const int xs = source_x<Q1>(*L, *P, ix);
    s.fx = f + static_cast<size_t>(ix * Q1 * Q1) * A->stride;
    s.ghosts = A->ghosts;
    s.P = P;
    s.stride = A->stride;
    s.n_ghost = A->n_ghost;
    s.ghost = SHOCK && xs < 0;
    s.xoff = static_cast<unsigned>(P->row + (s.ghost ? 0 : xs)) * 4u;
    s.any_ghost = SHOCK && __any(s.ghost);
    s.goff = static_cast<unsigned>(ix * Q1 * Q1 * A->n_ghost + P->gcol + (xs == -2 ? 1 : 0)) * 4u;
    return s;
  }
};

// One z line of the rebuild: f[iz] = sum_az Rw_az(iz) v[az] (+ g[iy][iz] for the additive
// collision), stored as FP32.
template <int Q1, int N, bool NT = false, class SL = NoAdd>
__device__ __forceinline__ void fold_line_store(const LatticeConst& L, const double (&v)[N + 1],
                                                float* __restrict__ line_base, long long stride, unsigned off,
                                                const SL& add = SL{}, int iy = 0) {
  constexpr int p = Q1 / 2;
  // the additive source's line is loaded ahead of the stores (loaded one by one as they are
  // added, the values wait behind the stores: 1.7x the step time at D3Q343, 1.4x at D3Q729)
  float g[Q1];
  if constexpr (SL::active) add.line(iy, g);
  auto pulled = [&](int iz) -> double { return static_cast<double>(g[iz]); };
  {
    double s = 0.0;
#pragma unroll
    for (int az = 0; az <= N; az += 2) s = fma(v[az], L.Rw64[p][az], s);
    if constexpr (SL::active) s += pulled(p);
    store_pop<NT>(line_base + static_cast<size_t>(p) * stride, off, static_cast<float>(s));
  }
#pragma unroll
  for (int j = 1; j <= p; ++j) {
    double e = 0.0, o = 0.0;
#pragma unroll
    for (int az = 0; az <= N; ++az) {
      if (az & 1) o = fma(v[az], L.Rw64[p + j][az], o);
      else e = fma(v[az], L.Rw64[p + j][az], e);
    }
    double hi = e + o, lo = e - o;
    if constexpr (SL::active) {
      hi += pulled(p + j);
      lo += pulled(p - j);
    }
    store_pop<NT>(line_base + static_cast<size_t>(p + j) * stride, off, static_cast<float>(hi));
    store_pop<NT>(line_base + static_cast<size_t>(p - j) * stride, off, static_cast<float>(lo));
  }
}

// Rebuild (eq:fi with 1/alpha!) in FP64, folded in y and z, and store to the own node.  With an
// additive source (LPN = 1 only) every stored population also gets its pulled value g added.
template <int Q1, int N, int LPN = 1, bool NT = false, class SRC = NoAddSource>
LBSMRT_PHASE void reconstruct_store64(const LatticeConst& L, const double (&ap)[Shape<Q1, N>::M],
                                                    float* __restrict__ out, long long stride, int node,
                                                    int sub = 0, const SRC& src = SRC{}) {
  constexpr int p = Q1 / 2;
  constexpr int P2 = Shape<Q1, N>::P2;
  // With LPN > 1 every lane makes the same number of passes; a lane with no slab left rebuilds
  // and stores the last slab again: the same values the lane that owns it stores to the same
  // addresses in the same instruction.
#pragma unroll 1
  for (int k = 0; k < (Q1 + LPN - 1) / LPN; ++k) {
    const int ixr = (LPN > 1 ? sub : 0) + k * LPN;
    const int ix = (LPN == 1 || ixr < Q1) ? ixr : Q1 - 1;
    double rx[N + 1];
    table_row<Q1, N, LPN>(L.Rw64, ix, rx);
    // as in gather_project64: uniform slab pointer, or the slab offset in the lane's byte offset
    const unsigned off = (LPN == 1 ? 0u : static_cast<unsigned>(ix * Q1 * Q1) * static_cast<unsigned>(stride) * 4u) +
                         static_cast<unsigned>(node) * 4u;
    double u2[P2];
#pragma unroll
    for (int ay = 0; ay <= N; ++ay)
#pragma unroll
      for (int az = 0; az <= N; ++az) {
        if (ay + az > N) continue;
        double s = 0.0;
#pragma unroll
        for (int ax = 0; ax <= N; ++ax)
          if (ax + ay + az <= N) s = fma(ap[midx(ax, ay, az)], rx[ax], s);
        u2[pair_pos(ay, az)] = s;
      }
    float* __restrict__ slab = LPN == 1 ? out + static_cast<size_t>(ix * Q1 * Q1) * stride : out;
    const auto add = src.slab(ix);
    {
      double v[N + 1];
#pragma unroll
      for (int az = 0; az <= N; ++az) {
        double s = 0.0;
#pragma unroll
        for (int ay = 0; ay <= N; ay += 2)
          if (ay + az <= N) s = fma(u2[pair_pos(ay, az)], L.Rw64[p][ay], s);
        v[az] = s;
      }
      fold_line_store<Q1, N, NT>(L, v, slab + static_cast<size_t>(p * Q1) * stride, stride, off, add, p);
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
          if (ay & 1) o = fma(u2[pair_pos(ay, az)], L.Rw64[p + j][ay], o);
          else e = fma(u2[pair_pos(ay, az)], L.Rw64[p + j][ay], e);
        }
        vp[az] = e + o;
        vm[az] = e - o;
      }
      fold_line_store<Q1, N, NT>(L, vp, slab + static_cast<size_t>((p + j) * Q1) * stride, stride, off, add, p + j);
      fold_line_store<Q1, N, NT>(L, vm, slab + static_cast<size_t>((p - j) * Q1) * stride, stride, off, add, p - j);
    }
  }
}

// Conserved moments of an FP64 projection: rho = a_0, u' = a_1 / rho,
// theta = (sum_k a_{2e_k} + 3 rho - rho |u'|^2) / (3 rho).
template <int N>
__device__ __forceinline__ void sums_from_a(const double* a, const LatticeConst& L, double (&S)[5]) {
  const double ir = 1.0 / L.r;
  S[0] = a[0];
  S[1] = a[midx(1, 0, 0)] * ir;
  S[2] = a[midx(0, 1, 0)] * ir;
  S[3] = a[midx(0, 0, 1)] * ir;
  S[4] = (a[midx(2, 0, 0)] + a[midx(0, 2, 0)] + a[midx(0, 0, 2)] + 3.0 * a[0]) * ir * ir;
}

// Conserved moments -> rho, u' (relative to ubar), theta; validity (Sec. 4.1).
struct Macro {
  double rho, ux, uy, uz, th;
  double tsc = 1.0;   // tau scale of the node's domain
};

__device__ __forceinline__ Macro macro_from_sums(const LatticeConst& L, const double (&S)[5], int* err) {
  Macro m;
  m.rho = S[0];
  const double inv = 1.0 / m.rho;
  m.ux = L.r * S[1] * inv;
  m.uy = L.r * S[2] * inv;
  m.uz = L.r * S[3] * inv;
  const double E = L.r * L.r * S[4];
  m.th = (E * inv - (m.ux * m.ux + m.uy * m.uy + m.uz * m.uz)) * (1.0 / 3.0);
  if (!(m.rho > 0.0 && m.th > 0.0 && m.th < 2.0)) atomicOr(err, kErrState);
  return m;
}

// a (lattice frame, FP32 projection) -> d (local frame, FP64), rho absorbed:
//   d_beta = theta^{-|beta|/2} sum_{gamma <= beta} prod_k C(beta_k, gamma_k) B_{beta_k - gamma_k} a_gamma
template <int N>
__device__ __forceinline__ void to_local(double* d, const Macro& m) {
  double Bx[N + 1], By[N + 1], Bz[N + 1];
  shift_poly<N>(-m.ux, 1.0 - m.th, Bx);
  shift_poly<N>(-m.uy, 1.0 - m.th, By);
  shift_poly<N>(-m.uz, 1.0 - m.th, Bz);
  axis_transform<N, 0>(d, Bx);
  axis_transform<N, 1>(d, By);
  axis_transform<N, 2>(d, Bz);
  scale_by_order<N>(d, 1.0 / sqrt(m.th));
  d[0] = m.rho;
  d[1] = 0.0;
  d[2] = 0.0;
  d[3] = 0.0;
}

// d (local) -> a (lattice):  a_alpha = sum_{beta <= alpha} prod_k C(alpha_k, beta_k) A_{alpha_k - beta_k} theta^{|beta|/2} d_beta
template <int N>
__device__ __forceinline__ void to_lattice(double* d, const Macro& m) {
  double Ax[N + 1], Ay[N + 1], Az[N + 1];
  scale_by_order<N>(d, sqrt(m.th));
  shift_poly<N>(m.ux, m.th - 1.0, Ax);
  shift_poly<N>(m.uy, m.th - 1.0, Ay);
  shift_poly<N>(m.uz, m.th - 1.0, Az);
  axis_transform<N, 0>(d, Ax);
  axis_transform<N, 1>(d, Ay);
  axis_transform<N, 2>(d, Az);
}

// eq:SMRT with tau_nm(x) = tau_nm * (rho_ref / rho) [optional] and tau_bar = tau + offset.
template <int N>
__device__ __forceinline__ void relax(double* d, const LatticeConst& L, double rho, double tsc) {
  const double sc = tsc * (L.density_scaling ? L.rho_ref / rho : 1.0);
#pragma unroll
  for (int n = 2; n <= N; ++n) {
    double om[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) om[m] = (2 * m <= n) ? 1.0 / fma(L.tau[n][m], sc, L.tau_offset) : 0.0;
    if (n == 2) om[1] = 0.0;   // the (2,1) part is zero by the definition of theta
    double* dn = d + order_start(n);
    if (n == 2) relax_order<2>(dn, om);
    if (n == 3) relax_order<3>(dn, om);
    if constexpr (N >= 4) if (n == 4) relax_order<4>(dn, om);
    if constexpr (N >= 5) if (n == 5) relax_order<5>(dn, om);
  }
}

// Reconstruction (eq:fi with 1/alpha!), sum-factorised, and store to the own node.
template <int Q1, int N, bool NT = false>
__device__ __forceinline__ void reconstruct_store(const LatticeConst& L, const float (&ap)[Shape<Q1, N>::M],
                                                  float* __restrict__ out, long long stride, int node) {
  constexpr int P2 = Shape<Q1, N>::P2;
#pragma unroll 1
  for (int ix = 0; ix < Q1; ++ix) {
    float rx[N + 1];
#pragma unroll
    for (int n = 0; n <= N; ++n) rx[n] = L.Rw[ix][n];
    float u2[P2];
#pragma unroll
    for (int ay = 0; ay <= N; ++ay)
#pragma unroll
      for (int az = 0; az <= N; ++az) {
        if (ay + az > N) continue;
        float s = 0.f;
#pragma unroll
        for (int ax = 0; ax <= N; ++ax)
          if (ax + ay + az <= N) s = fmaf(ap[midx(ax, ay, az)], rx[ax], s);
        u2[pair_pos(ay, az)] = s;
      }
#pragma unroll
    for (int iy = 0; iy < Q1; ++iy) {
      float v[N + 1];
#pragma unroll
      for (int az = 0; az <= N; ++az) {
        float s = 0.f;
#pragma unroll
        for (int ay = 0; ay <= N; ++ay)
          if (ay + az <= N) s = fmaf(u2[pair_pos(ay, az)], L.Rw[iy][ay], s);
        v[az] = s;
      }
#pragma unroll
      for (int iz = 0; iz < Q1; ++iz) {
        float s = 0.f;
#pragma unroll
        for (int az = 0; az <= N; ++az) s = fmaf(v[az], L.Rw[iz][az], s);
        const int q = (ix * Q1 + iy) * Q1 + iz;
        store_pop<NT>(out + static_cast<size_t>(q) * stride, static_cast<unsigned>(node) * 4u, s);
      }
    }
  }
}

// ------------------------------------------------------------------ kernels

enum : int { kPrecFp32 = 0, kPrecFp64 = 2 };

// One node of the fused step (work-block `wb` of the block table, or blockIdx.x when wb < 0).
// LPN > 1 (FP64 contractions only): LPN lanes share a node, each gathering and storing the
// x-slabs ix = sub, sub + LPN, ...; the moments are summed across the group and every lane
// runs the (identical) collision.
// ADD: the additive collision f* = g + R (a' - a) instead of the rebuild f* = R a' (FP64
// contractions, one lane per node); g is loaded again at store time.
template <int Q1, int N, bool SHOCK, int PREC, int LPN = 1, bool ADD = false>
__device__ __forceinline__ void collide_stream_node(const LatticeConst& L, const StepArgs& A,
                                                    const float* __restrict__ fsrc, float* __restrict__ fdst,
                                                    int wb) {
  static_assert(LPN == 1 || PREC == kPrecFp64, "lanes per node > 1 needs the FP64 contractions");
  static_assert(!ADD || (PREC == kPrecFp64 && LPN == 1), "the additive collision runs with FP64 contractions, one lane");
  constexpr int M = Shape<Q1, N>::M;
  Pull<Q1> P;
  if (!make_pull<Q1, LPN>(L, A, P, wb)) return;
  double d[M];
  double S[5];
  [[maybe_unused]] double a0[ADD ? M : 1];
  if constexpr (PREC == kPrecFp64) {
    gather_project64<Q1, N, SHOCK, LPN>(L, A, fsrc, P, d);
    sums_from_a<N>(d, L, S);
    if constexpr (ADD) {
#pragma unroll
      for (int i = 0; i < M; ++i) a0[i] = d[i];
    }
  } else {
    float a[M];
    double H[5];
    gather_project<Q1, N, SHOCK>(L, A, fsrc, P, a, H);
#pragma unroll
    for (int i = 0; i < M; ++i) d[i] = static_cast<double>(a[i]);
    // orders 0 and 1 and the trace of order 2 from the FP64 sums: the FP32 trace would leave a
    // (2,1) part, which is not relaxed, and re-emit its rounding as energy every step
    d[0] = H[0];
    d[1] = H[1];
    d[2] = H[2];
    d[3] = H[3];
    const double dtr = (H[4] - (d[midx(2, 0, 0)] + d[midx(0, 2, 0)] + d[midx(0, 0, 2)])) * (1.0 / 3.0);
    d[midx(2, 0, 0)] += dtr;
    d[midx(0, 2, 0)] += dtr;
    d[midx(0, 0, 2)] += dtr;
    sums_from_a<N>(d, L, S);
  }
  Macro mac = macro_from_sums(L, S, A.err);
  mac.tsc = P.tsc;
  to_local<N>(d, mac);
  relax<N>(d, L, mac.rho, mac.tsc);
  to_lattice<N>(d, mac);
  if constexpr (ADD) {
#pragma unroll
    for (int i = 0; i < M; ++i) d[i] -= a0[i];
    reconstruct_store64<Q1, N, 1, !SHOCK>(L, d, fdst, A.stride, P.node, 0, PulledSource<Q1, SHOCK>{&L, &A, fsrc, &P});
  } else if constexpr (PREC == kPrecFp64) {
    reconstruct_store64<Q1, N, LPN, !SHOCK>(L, d, fdst, A.stride, P.node, P.sub);
  } else {
    float ap[M];
#pragma unroll
    for (int i = 0; i < M; ++i) ap[i] = static_cast<float>(d[i]);
    reconstruct_store<Q1, N, !SHOCK>(L, ap, fdst, A.stride, P.node);
  }
}

template <int Q1, int N, bool SHOCK, int PREC, int LPN = 1, bool ADD = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_collide_stream(
    LatticeConst L, StepArgs A, const float* __restrict__ fsrc, float* __restrict__ fdst) {
  collide_stream_node<Q1, N, SHOCK, PREC, LPN, ADD>(L, A, fsrc, fdst, -1);
}

// s_waitcnt immediate of gfx9 waiting for vmcnt = 0 only (expcnt 7, lgkmcnt 15 left open).
constexpr int kWaitVmcnt0 = 0x0F70;

// Per-block progress of the persistent launch on line domains: nbr[b] = the blocks b depends on
// (the neighbouring blocks of its domain within the pull reach, -1 for none), done[b] = the
// number of steps block b has completed (since the tables were built; compared with
// wrap-around), spin_limit = polls before a wait gives up.
struct FlowArgs {
  const int2* nbr;
  unsigned* done;
  unsigned spin_limit;
  unsigned skew;   // added to every wait's target: 0, or (tests of the give-up path) unreachable
};

// Wait (one work-item) until block b has completed `target` steps; gives up after spin_limit
// polls, or at once when another wait has given up, latching kErrTimeout (the launch then ends
// normally with wrong values, which lbsmrt_sync_status reports).
// Polls are relaxed (an acquire load would invalidate the caches at every poll); the caller
// fences once after its waits.
__device__ __forceinline__ void wait_block(const FlowArgs& F, int b, unsigned target, int* err) {
  if (b < 0) return;
  unsigned spins = 0;
  while (static_cast<int>(__hip_atomic_load(F.done + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrTimeout) return;
    if (++spins >= F.spin_limit) {
      atomicOr(err, kErrTimeout);
      return;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Persistent form (cooperative launch, so all work-groups are resident): every work-group strides
// over the block table, n_steps times.  Step t reads fa when t is even and fb when odd, as
// lbsmrt_step does.  FLOW = false: a grid-wide barrier between steps.  FLOW = true (line domains):
// no barrier; a block starts step t once the blocks it pulls from have completed step t - 1,
// which also means they no longer read the buffer it overwrites (step t writes the buffer step
// t - 1 read).  Each work-group takes its blocks in step order, and every wait is for a smaller
// step than the waiter's, so the work-group at the smallest step can always proceed.
template <int Q1, int N, bool SHOCK, int PREC, int LPN = 1, bool FLOW = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_collide_persistent(
    LatticeConst L, StepArgs A, float* fa, float* fb, int n_blocks, int n_steps, FlowArgs F) {
  if constexpr (!FLOW) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    for (int t = 0; t < n_steps; ++t) {
      const float* src = (t & 1) ? fb : fa;
      float* dst = (t & 1) ? fa : fb;
      for (int wb = blockIdx.x; wb < n_blocks; wb += gridDim.x)
        collide_stream_node<Q1, N, SHOCK, PREC, LPN>(L, A, src, dst, wb);
      grid.sync();
    }
  } else {
    // Every launch takes every block through all its steps and the counters start equal, so all
    // blocks hold the same count when a launch starts: each work-group reads it from its first
    // block (written only by itself, and by earlier launches).  Counting from there, the launch
    // depends on no step count kept by the host.
    if (static_cast<int>(blockIdx.x) >= n_blocks) return;
    unsigned base = 0;
    if (threadIdx.x == 0) base = __hip_atomic_load(F.done + blockIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int t = 0; t < n_steps; ++t) {
      const float* src = (t & 1) ? fb : fa;
      float* dst = (t & 1) ? fa : fb;
      for (int wb = blockIdx.x; wb < n_blocks; wb += gridDim.x) {
        if (t > 0) {
          if (threadIdx.x == 0) {
            const int2 nb = F.nbr[wb];
            wait_block(F, nb.x, base + F.skew + t, A.err);
            wait_block(F, nb.y, base + F.skew + t, A.err);
            // pairs with the neighbours' release stores; the barrier orders the other waves'
            // loads after it (they share this work-item's compute unit and caches)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          }
          __syncthreads();
        }
        collide_stream_node<Q1, N, SHOCK, PREC, LPN>(L, A, src, dst, wb);
        // every wave's stores acknowledged before the barrier, so the release store below (one
        // write-back of this XCD's L2 per block, not one per wave) publishes all of them
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
        if (threadIdx.x == 0)
          __hip_atomic_store(F.done + wb, base + t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// Moment fields of the pre-collision populations (see lbsmrt_moments).
template <int Q1, int N, bool SHOCK>
__global__ __launch_bounds__(256) void k_moments(LatticeConst L, StepArgs A, const float* __restrict__ f,
                                                 double* __restrict__ out, unsigned mask, long long n_nodes) {
  constexpr int M = Shape<Q1, N>::M;
  Pull<Q1> P;
  if (!make_pull<Q1>(L, A, P)) return;
  double aa[M], d[M];
  double S[5];
  gather_project64<Q1, N, SHOCK>(L, A, f, P, aa);
  sums_from_a<N>(aa, L, S);
  const Macro mac = macro_from_sums(L, S, A.err);
#pragma unroll
  for (int i = 0; i < M; ++i) d[i] = aa[i];
  to_local<N>(d, mac);
  double* o = out + P.node;
  long long row = 0;
  auto put = [&](double v) { o[row * n_nodes] = v; ++row; };
  if (mask & 1u) {
    put(mac.rho);
    put(L.r * L.k[0] + mac.ux);
    put(L.r * L.k[1] + mac.uy);
    put(L.r * L.k[2] + mac.uz);
    put(mac.th);
  }
  if (mask & 2u) {
#pragma unroll
    for (int i = 0; i < 6; ++i) put(mac.th * d[order_start(2) + i]);
  }
  if (mask & 4u) {
    double t[3];
    sym_trace<1>(d + order_start(3), t);
    const double c = 0.5 * mac.th * sqrt(mac.th);
#pragma unroll
    for (int i = 0; i < 3; ++i) put(c * t[i]);
  }
  if (mask & 8u) {
    double p[10];
    irreducible_part<3, 0>(d + order_start(3), p);
    constexpr double inv = 1.0 / coefD(3, 0);
#pragma unroll
    for (int i = 0; i < 10; ++i) put(p[i] * inv);
  }
  if constexpr (N >= 4) {
    if (mask & 16u) {
      double p[6];
      irreducible_part<4, 1>(d + order_start(4), p);
      constexpr double inv = 1.0 / coefD(4, 1);
#pragma unroll
      for (int i = 0; i < 6; ++i) put(p[i] * inv);
    }
    if (mask & 32u) {
      double p[1];
      irreducible_part<4, 2>(d + order_start(4), p);
      put(p[0] * (1.0 / coefD(4, 2)));
    }
  }
  if (mask & 64u) {
#pragma unroll
    for (int i = 0; i < M; ++i) put(d[i]);
  }
  if (mask & 128u) {
#pragma unroll
    for (int i = 0; i < M; ++i) put(aa[i]);
  }
}

// Truncated Maxwellian of lab-frame (rho, u, theta) rows; nodes 0..count-1 map to
// columns 0..count-1 of f (row stride `stride`).
template <int Q1, int N>
__global__ __launch_bounds__(256) void k_equilibrium(LatticeConst L, const double* __restrict__ fields, long long count,
                                                     float* __restrict__ f, long long stride) {
  constexpr int M = Shape<Q1, N>::M;
  const long long node = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (node >= count) return;
  const double rho = fields[node];
  const double ux = fields[count + node] - L.r * L.k[0];
  const double uy = fields[2 * count + node] - L.r * L.k[1];
  const double uz = fields[3 * count + node] - L.r * L.k[2];
  const double th = fields[4 * count + node];
  double Ax[N + 1], Ay[N + 1], Az[N + 1];
  shift_poly<N>(ux, th - 1.0, Ax);
  shift_poly<N>(uy, th - 1.0, Ay);
  shift_poly<N>(uz, th - 1.0, Az);
  double a[M];
#pragma unroll
  for (int ax = 0; ax <= N; ++ax)
#pragma unroll
    for (int ay = 0; ay <= N; ++ay)
#pragma unroll
      for (int az = 0; az <= N; ++az)
        if (ax + ay + az <= N) a[midx(ax, ay, az)] = rho * Ax[ax] * Ay[ay] * Az[az];
  reconstruct_store64<Q1, N>(L, a, f, stride, static_cast<int>(node));
}

}  // namespace lbsmrt
