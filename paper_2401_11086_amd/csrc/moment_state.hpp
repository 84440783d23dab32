// Moment-state form of the periodic LB-SMRT step (gfx950 kernels).
//
// With the regularised rebuild (eq:fi) the post-collision populations are fully determined by
// the M moments a'_alpha of each node: f*_i(x) = w_i sum_alpha a'_alpha(x) He_alpha(c_i) / alpha!.
// The pull stream followed by the projection (eq:an) is then a linear map of the moment fields,
//   a_beta(x) = sum_alpha sum_e prod_k K_{beta_k alpha_k}(e_k) a'_alpha(x - e - k),
//   K_{b a}(e) = He_b(c_e) w_e He_a(c_e) / a!      (1D tap of the tensor-product stencil),
// a separable convolution that is applied one axis at a time:
//   pass z:  a'[ax, ay, az]       -> t1[ax, ay, bz]   (P2 (N+1) fields)
//   pass y:  t1[ax, ay, bz]       -> t2[ax, by, bz]   ((N+1) P2 fields)
//   pass x:  t2[ax, by, bz]       -> a[bx, by, bz]    (M fields), then the SMRT collision of
//            Sec. 3 (frame shift, irreducible split, relaxation, shift back) and the store of a'.
// The state is float32 [M][stride] (moment index as in smrt_node.hpp); the two intermediates are
// float32 [P2 (N+1)][stride] each.  Every node of one periodic domain (x fastest).
//
// Passes z and y march each work-item along its line with a register ring of the last W rows
// (W = 2 max|e| + 1), so every input row is read once per line chunk of T rows (T a multiple of
// W, chosen by the host so that the launch has enough waves).  Pass x reads its row's shifted
// neighbours directly (same cache lines as the row itself).  Every pass applies a tap pair +-e_t
// factored through the populations (K(-e) = (-1)^(a+b) K(e)): the two sources are folded by
// parity in float32, v(x - e) + v(x + e) and v(x - e) - v(x + e) (exact where they agree, so a
// uniform state stays uniform), and F = sum_a Rw_a(c_t) fold_a and its projection with
// He_b(c_t) run in FP64 with FP64 tables, so the quadrature identity sum_e K_{b a}(e) =
// delta_ab, and with it the conservation of mass, momentum and energy, holds up to the float32
// storage of the fields.
#pragma once
#include "kernels.hpp"
#include "ms_std_tables.hpp"

namespace lbsmrt {

// Compile-time non-negative taps of the two stencils with a moment-state kernel:
// D1Q7 {0, +-1, +-2, +-3} and D1Q9 {0, +-1, +-2, +-3, +-5} (Sec. 4.2).
template <int Q1>
struct Taps1D;
template <>
struct Taps1D<7> {
  static constexpr int p = 3;
  static constexpr int H = 3;   // max |e|
  static constexpr int e[4] = {0, 1, 2, 3};
};
template <>
struct Taps1D<9> {
  static constexpr int p = 4;
  static constexpr int H = 5;
  static constexpr int e[5] = {0, 1, 2, 3, 5};
};
template <>
struct Taps1D<17> {   // D1Q17: the line kernel with one lane per node only (nine taps)
  static constexpr int p = 8;
  static constexpr int H = 9;
  static constexpr int e[9] = {0, 1, 2, 3, 4, 5, 6, 7, 9};
};

// 1D tables of the non-negative taps t (c = r e_t): He[t][b] = He_b(c), Rw[t][a] = w He_a(c) / a!,
// so K_{b a}(e_t) = He[t][b] Rw[t][a].  Stencils of up to nine points have every moment-state
// kernel, the 17-point stencil the line kernel (one lane per node) and the state conversions.
constexpr int kMsMaxTaps = 9;
struct MomentTables64 {
  double He[kMsMaxTaps][kMaxN + 1];
  double Rw[kMsMaxTaps][kMaxN + 1];
};

// Tap table entries of every moment-state pass: compile-time constants (the host has checked that they
// agree with the context's tables; with these taps the quadrature is unique), which the
// compiler rematerialises with scalar moves instead of holding up to 60 FP64 values in scalar
// registers and spilling them.
template <int Q1>
__device__ __forceinline__ double tab_he(int t, int n) { return MsStdTables<Q1>::He[t][n]; }
template <int Q1>
__device__ __forceinline__ double tab_rw(int t, int n) { return MsStdTables<Q1>::Rw[t][n]; }

struct MsGeom {
  int nx, ny, nz;
  int k[3];            // frame shift (integer), the pull source is x - e - k
  long long stride;    // row stride of every [fields][stride] buffer
  double tsc;          // tau scale of the domain
  int* err;            // validity flag (kErrState)
};

// March of one line: outputs at positions p0 .. p0 + T - 1 (< len) of the line whose position q
// has byte offset base + q * step.  Inputs: fields fin[a], a < NF (the 1D index a of the
// convolved axis); outputs: fields fout[b], b < no (1D index b).
template <int Q1, int N, int NF>
__device__ __forceinline__ void march_line(const float* __restrict__ in,
                                           float* __restrict__ out, long long stride, const int (&fin)[N + 1],
                                           const int (&fout)[N + 1], int no, unsigned base, unsigned step,
                                           int len, int p0, int T, int kshift) {
  constexpr int nf = NF;
  using S = Taps1D<Q1>;
  constexpr int H = S::H;
  constexpr int W = 2 * H + 1;   // T is a multiple of W (checked by the host)
  const float* __restrict__ src[N + 1];
#pragma unroll
  for (int a = 0; a <= N; ++a) src[a] = in + static_cast<size_t>(a < nf ? fin[a] : fin[0]) * stride;
  // ring slot r % W holds line position p0 - H - kshift + r (mod len)
  int q = (p0 - H - kshift) % len;
  if (q < 0) q += len;
  float ring[W][N + 1];
#pragma unroll
  for (int r = 0; r < W - 1; ++r) {
    const unsigned off = base + static_cast<unsigned>(q) * step;
#pragma unroll
    for (int a = 0; a <= N; ++a)
      if (a < nf) ring[r][a] = load_at(src[a], off);
    q = (q + 1 == len) ? 0 : q + 1;
  }
#pragma unroll 1
  for (int jb = 0; jb < T; jb += W) {
#pragma unroll
    for (int jj = 0; jj < W; ++jj) {
      {
        const unsigned off = base + static_cast<unsigned>(q) * step;
#pragma unroll
        for (int a = 0; a <= N; ++a)
          if (a < nf) ring[(jj + W - 1) % W][a] = load_at(src[a], off);
        q = (q + 1 == len) ? 0 : q + 1;
      }
      const int pos = p0 + jb + jj;
      if (pos < len) {
        double acc[N + 1];
#pragma unroll
        for (int b = 0; b <= N; ++b) acc[b] = 0.0;
        // centre tap (He and Rw vanish at c = 0 for odd orders): the tap e pulls line position
        // pos - e - kshift = ring slot (jj + H - e) % W
        {
          double c = 0.0;
#pragma unroll
          for (int a = 0; a <= N; a += 2)
            if (a < nf) c = fma(tab_rw<Q1>(0, a), static_cast<double>(ring[(jj + H) % W][a]), c);
#pragma unroll
          for (int b = 0; b <= N; b += 2) acc[b] = fma(tab_he<Q1>(0, b), c, acc[b]);
        }
#pragma unroll
        for (int t = 1; t <= S::p; ++t) {
          double ev = 0.0, od = 0.0;
#pragma unroll
          for (int a = 0; a <= N; ++a) {
            if (a >= nf) continue;
            // the fold is rounded in FP32 (unbiased); the tables and the sums stay FP64
            const float vp = ring[(jj + H - S::e[t]) % W][a];
            const float vm = ring[(jj + H + S::e[t]) % W][a];
            const double sm = static_cast<double>(vp + vm), df = static_cast<double>(vp - vm);
            ev = fma(tab_rw<Q1>(t, a), (a & 1) ? df : sm, ev);
            od = fma(tab_rw<Q1>(t, a), (a & 1) ? sm : df, od);
          }
#pragma unroll
          for (int b = 0; b <= N; ++b) acc[b] = fma(tab_he<Q1>(t, b), (b & 1) ? od : ev, acc[b]);
        }
        const unsigned off = base + static_cast<unsigned>(pos) * step;
#pragma unroll
        for (int b = 0; b <= N; ++b)
          if (b < no) store_at(out + static_cast<size_t>(fout[b]) * stride, off, static_cast<float>(acc[b]));
      }
    }
  }
}

// The input count as a compile-time constant (a uniform switch per line), so that the march
// carries no per-field guards and its work scales with the fields it actually reads.
template <int Q1, int N, int NF = N + 1>
__device__ __forceinline__ void march_line_n(const float* __restrict__ in,
                                             float* __restrict__ out, long long stride, const int (&fin)[N + 1],
                                             int nf, const int (&fout)[N + 1], int no, unsigned base, unsigned step,
                                             int len, int p0, int T, int kshift) {
  if constexpr (NF >= 1) {
    if (nf == NF) march_line<Q1, N, NF>(in, out, stride, fin, fout, no, base, step, len, p0, T, kshift);
    else march_line_n<Q1, N, NF - 1>(in, out, stride, fin, nf, fout, no, base, step, len, p0, T, kshift);
  }
}

// Pass z: a'[ax, ay, az] -> t1[pair(ax, ay) (N+1) + bz].  One work-item per z line (x, y), the
// lines numbered x fastest over the plane (so a wave reads contiguous 256 B); grid
// (ceil(nx ny / 256), ceil(nz / T)), each work-item marching T rows.
template <int Q1, int N>
__global__ __launch_bounds__(256) void k_ms_pass_z(MsGeom G, const float* __restrict__ m,
                                                   float* __restrict__ t1, int T) {
  const int line = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  if (line >= G.nx * G.ny) return;
  const int z0 = static_cast<int>(blockIdx.y) * T;
  const unsigned base = static_cast<unsigned>(line) * 4u;
  const unsigned step = static_cast<unsigned>(G.nx * G.ny) * 4u;
#pragma unroll 1
  for (int ax = 0; ax <= N; ++ax)
#pragma unroll 1
    for (int ay = 0; ax + ay <= N; ++ay) {
      int fin[N + 1], fout[N + 1];
#pragma unroll
      for (int a = 0; a <= N; ++a) fin[a] = midx(ax, ay, a <= N - ax - ay ? a : 0);
#pragma unroll
      for (int b = 0; b <= N; ++b) fout[b] = pair_pos(ax, ay) * (N + 1) + b;
      march_line_n<Q1, N>(m, t1, G.stride, fin, N - ax - ay + 1, fout, N + 1, base, step, G.nz, z0, T, G.k[2]);
    }
}

// Pass y: t1[pair(ax, ay) (N+1) + bz] -> t2[ax P2 + pair(by, bz)].  One work-item per y line
// (x, z), x fastest; grid (ceil(nx nz / 256), ceil(ny / T)).
template <int Q1, int N>
__global__ __launch_bounds__(256) void k_ms_pass_y(MsGeom G, const float* __restrict__ t1,
                                                   float* __restrict__ t2, int T) {
  constexpr int P2 = n_sym(N);
  const int line = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  if (line >= G.nx * G.nz) return;
  const int x = line % G.nx;
  const int z = line / G.nx;
  const int y0 = static_cast<int>(blockIdx.y) * T;
  const unsigned base = static_cast<unsigned>(x + G.nx * G.ny * z) * 4u;
  const unsigned step = static_cast<unsigned>(G.nx) * 4u;
#pragma unroll 1
  for (int ax = 0; ax <= N; ++ax)
#pragma unroll 1
    for (int bz = 0; bz <= N; ++bz) {
      int fin[N + 1], fout[N + 1];
#pragma unroll
      for (int a = 0; a <= N; ++a) fin[a] = pair_pos(ax, a <= N - ax ? a : 0) * (N + 1) + bz;
#pragma unroll
      for (int b = 0; b <= N; ++b) fout[b] = ax * P2 + pair_pos(b <= N - bz ? b : 0, bz);
      march_line_n<Q1, N>(t1, t2, G.stride, fin, N - ax + 1, fout, N - bz + 1, base, step, G.ny, y0, T, G.k[1]);
    }
}

// Groups (by, bz) in their compile-time order: index of (BY, BZ).
constexpr int group_index(int N, int BY, int BZ) {
  int g = 0;
  for (int by = 0; by < BY; ++by) g += N - by + 1;
  return g + BZ;
}

// Groups whose loads may be in flight together in pass x and the line kernel (a memory fence
// after every kGroupsPerPhase groups): fewer serial load round trips per node, more registers.
#ifndef LBSMRT_GROUPS_PER_PHASE
#define LBSMRT_GROUPS_PER_PHASE 3
#endif
constexpr int kGroupsPerPhase = LBSMRT_GROUPS_PER_PHASE;
// The line kernel's phase length per stencil: the 17-point stencil loads 17 values per field and
// tap group, so one group per phase (three held about 300 loads in flight and spilled).
template <int Q1>
constexpr int line_groups_per_phase() { return Q1 > 9 ? 1 : kGroupsPerPhase; }
#ifndef LBSMRT_GROUPS_PER_PHASE_ROW
#define LBSMRT_GROUPS_PER_PHASE_ROW 5
#endif
constexpr int kGroupsPerPhaseRow = LBSMRT_GROUPS_PER_PHASE_ROW;   // two loads per field instead of 2 p + 1
// Share of pass x's groups whose taps move across lanes on whole rows (the rest are loaded):
// measured on the 256^3 D3Q343 box, 0, 1/3, 1/2, 2/3 of the groups: 6.11, 6.01, 5.95, 5.74 ms
// per moment-state step (one unit, one run); the 160^3 D3Q729 box is unchanged (3.30 ms).
#ifndef LBSMRT_ROW_GROUPS_NUM
#define LBSMRT_ROW_GROUPS_NUM 2
#define LBSMRT_ROW_GROUPS_DEN 3
#endif

// One (by, bz) group of pass x: a[bx, by, bz] = sum_ax sum_e K_{bx ax}(e) t2[ax, by, bz](x - e - k_x)
// for bx <= N - by - bz, in FP64, each tap pair factored through the rebuilt populations.
// Row neighbours of a wave that covers 64 consecutive x of one row (nx a multiple of 64, no x
// shift): lane l holds v = row[x0 + l] and a halo value h (lanes 0 .. H-1: row[x0 - 1 - l], lanes
// 64 - H .. 63: row[x0 + 127 - l], periodic).  wave_shr:1 moves every lane's value one lane up and
// leaves lane 0 its old value, wave_shl:1 one lane down leaving lane 63's; so R[d] = row[x0 + l - d]
// and Lf[d] = row[x0 + l + d] are built d lanes at a time, the halo shifted into lanes 0 and 63.
__device__ __forceinline__ float wave_shr1(float old, float src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, src), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_shl1(float old, float src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, src), 0x130, 0xf, 0xf, false));
}
template <int H>
__device__ __forceinline__ void row_neighbours(float v, float h, float (&R)[H + 1], float (&Lf)[H + 1]) {
  R[0] = v;
  Lf[0] = v;
  float hl = h, hr = h;
#pragma unroll
  for (int d = 1; d <= H; ++d) {
    R[d] = wave_shr1(hl, R[d - 1]);
    Lf[d] = wave_shl1(hr, Lf[d - 1]);
    if (d < H) {
      hl = wave_shl1(hl, hl);
      hr = wave_shr1(hr, hr);
    }
  }
}

template <int Q1, int N, int BY, int BZ>
__device__ __forceinline__ void x_group(const LatticeConst& L, const float* __restrict__ t2, long long stride,
                                        const unsigned (&op)[Taps1D<Q1>::p + 1],
                                        const unsigned (&om)[Taps1D<Q1>::p + 1], float (&a32)[n_moments(N)]) {
  using S = Taps1D<Q1>;
  constexpr int P2 = n_sym(N);
  constexpr int NO = N - BY - BZ;
  const float* __restrict__ src[N + 1];
#pragma unroll
  for (int a = 0; a <= N; ++a) src[a] = t2 + static_cast<size_t>(a * P2 + pair_pos(BY, BZ)) * stride;
  double acc[NO + 1];
#pragma unroll
  for (int b = 0; b <= NO; ++b) acc[b] = 0.0;
  {
    double c = 0.0;                           // centre tap: even orders only
#pragma unroll
    for (int a = 0; a <= N; a += 2) c = fma(tab_rw<Q1>(0, a), static_cast<double>(load_at(src[a], op[0])), c);
#pragma unroll
    for (int b = 0; b <= NO; b += 2) acc[b] = fma(tab_he<Q1>(0, b), c, acc[b]);
  }
#pragma unroll
  for (int t = 1; t <= S::p; ++t) {
    double ev = 0.0, od = 0.0;
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      // fold in FP32 (unbiased rounding) so the loads in flight stay one register each
      const float vp = load_at(src[a], op[t]);
      const float vm = load_at(src[a], om[t]);
      const double sm = static_cast<double>(vp + vm), df = static_cast<double>(vp - vm);
      ev = fma(tab_rw<Q1>(t, a), (a & 1) ? df : sm, ev);
      od = fma(tab_rw<Q1>(t, a), (a & 1) ? sm : df, od);
    }
#pragma unroll
    for (int b = 0; b <= NO; ++b) acc[b] = fma(tab_he<Q1>(t, b), (b & 1) ? od : ev, acc[b]);
  }
  // Finish each group before later loads: the empty asm statements pin the sums here and fence
  // the loads every kGroupsPerPhase groups, otherwise every loaded value stays live until the
  // collision.  The moments wait for the collision as float32 (the collision returns the
  // conserved ones unchanged, and the store rounds them to float32 in any case), which keeps
  // enough registers free for the loads of a group to be in flight together.
#pragma unroll
  for (int b = 0; b <= NO; ++b) {
    float v = static_cast<float>(acc[b]);
    asm volatile("" : "+v"(v));
    a32[midx(b, BY, BZ)] = v;
  }
  if constexpr ((group_index(N, BY, BZ) + 1) % kGroupsPerPhase == 0) asm volatile("" ::: "memory");
}

// All groups (by, bz), by + bz <= N, in compile-time order.
template <int Q1, int N, int BY, int BZ>
__device__ __forceinline__ void x_groups(const LatticeConst& L, const float* __restrict__ t2, long long stride,
                                         const unsigned (&op)[Taps1D<Q1>::p + 1],
                                         const unsigned (&om)[Taps1D<Q1>::p + 1], float (&a32)[n_moments(N)]) {
  if constexpr (BY <= N) {
    if constexpr (BY + BZ <= N) {
      x_group<Q1, N, BY, BZ>(L, t2, stride, op, om, a32);
      x_groups<Q1, N, BY, BZ + 1>(L, t2, stride, op, om, a32);
    } else {
      x_groups<Q1, N, BY + 1, 0>(L, t2, stride, op, om, a32);
    }
  }
}

// ---- pass x on whole 64-lane rows: tap sources moved across lanes
// Group g (compile-time order of group_index) -> (by, bz).
// (g = n_sym(N), one past the last group, maps to (N + 1, 0).)
constexpr int group_by(int N, int g) {
  int by = 0;
  while (by <= N && g > N - by) {
    g -= N - by + 1;
    ++by;
  }
  return by;
}
constexpr int group_bz(int N, int g) {
  int by = 0;
  while (by <= N && g > N - by) {
    g -= N - by + 1;
    ++by;
  }
  return g;
}

// One group (BY, BZ) from this lane's row and halo values of its N + 1 input fields.
template <int Q1, int N, int BY, int BZ>
__device__ __forceinline__ void x_group_row(const float (&rv)[N + 1], const float (&rh)[N + 1],
                                            float (&a32)[n_moments(N)]) {
  using S = Taps1D<Q1>;
  constexpr int NO = N - BY - BZ;
  float Rn[N + 1][S::H + 1], Ln[N + 1][S::H + 1];
#pragma unroll
  for (int a = 0; a <= N; ++a) row_neighbours<S::H>(rv[a], rh[a], Rn[a], Ln[a]);
  double acc[NO + 1];
#pragma unroll
  for (int b = 0; b <= NO; ++b) acc[b] = 0.0;
  {
    double c = 0.0;                           // centre tap: even orders only
#pragma unroll
    for (int a = 0; a <= N; a += 2) c = fma(tab_rw<Q1>(0, a), static_cast<double>(rv[a]), c);
#pragma unroll
    for (int b = 0; b <= NO; b += 2) acc[b] = fma(tab_he<Q1>(0, b), c, acc[b]);
  }
#pragma unroll
  for (int t = 1; t <= S::p; ++t) {
    double ev = 0.0, od = 0.0;
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      // tap +e pulls from x - e (lane l - e), tap -e from x + e; folded in FP32 as in x_group
      const float vp = Rn[a][S::e[t]], vm = Ln[a][S::e[t]];
      const double sm = static_cast<double>(vp + vm), df = static_cast<double>(vp - vm);
      ev = fma(tab_rw<Q1>(t, a), (a & 1) ? df : sm, ev);
      od = fma(tab_rw<Q1>(t, a), (a & 1) ? sm : df, od);
    }
#pragma unroll
    for (int b = 0; b <= NO; ++b) acc[b] = fma(tab_he<Q1>(t, b), (b & 1) ? od : ev, acc[b]);
  }
#pragma unroll
  for (int b = 0; b <= NO; ++b) {
    float v = static_cast<float>(acc[b]);
    asm volatile("" : "+v"(v));
    a32[midx(b, BY, BZ)] = v;
  }
}

template <int Q1, int N, int G0, int I, int NG>
__device__ __forceinline__ void x_phase_groups(const float (&rv)[NG][N + 1], const float (&rh)[NG][N + 1],
                                               float (&a32)[n_moments(N)]) {
  if constexpr (I < NG) {
    x_group_row<Q1, N, group_by(N, G0 + I), group_bz(N, G0 + I)>(rv[I], rh[I], a32);
    x_phase_groups<Q1, N, G0, I + 1, NG>(rv, rh, a32);
  }
}

// Groups G0 .. G0 + G - 1 as one phase: the row and halo values of all their input fields are
// loaded first (two loads per field, all in flight together), then the groups are reduced; the
// sums' pins end the phase, so each phase is one memory round trip.
template <int Q1, int N, int G0, int G, int GEND>
__device__ __forceinline__ void x_phases_row(const float* __restrict__ t2, long long stride, unsigned own,
                                             unsigned hoff, float (&a32)[n_moments(N)]) {
  constexpr int P2 = n_sym(N);
  if constexpr (G0 < GEND) {
    constexpr int NG = G0 + G <= GEND ? G : GEND - G0;
    float rv[NG][N + 1], rh[NG][N + 1];
#pragma unroll
    for (int i = 0; i < NG; ++i)
#pragma unroll
      for (int a = 0; a <= N; ++a) {
        const float* __restrict__ row =
            t2 + static_cast<size_t>(a * P2 + pair_pos(group_by(N, G0 + i), group_bz(N, G0 + i))) * stride;
        rv[i][a] = load_at(row, own);
        rh[i][a] = load_at(row, hoff);
      }
    x_phase_groups<Q1, N, G0, 0, NG>(rv, rh, a32);
    x_phases_row<Q1, N, G0 + G, G, GEND>(t2, stride, own, hoff, a32);
  }
}

// Pass x + collision: t2[ax P2 + pair(by, bz)] -> a[bx, by, bz], SMRT collision (FP64), store a'.
// Grid (ceil(nx/256), ny, nz).  ROW (nx a multiple of 64, k_x = 0): the tap sources are moved
// across the wave's lanes (row_neighbours) instead of loaded one by one; every wave is then either
// entirely inside the row or entirely past its end.
template <int Q1, int N, bool ROW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(N >= 5 ? 2 : 1))) void k_ms_pass_x_collide(
    LatticeConst L, MsGeom G, const float* __restrict__ t2, float* __restrict__ m_out) {
  using S = Taps1D<Q1>;
  constexpr int M = n_moments(N);
  const int x = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  if (x >= G.nx) return;
  const int y = static_cast<int>(blockIdx.y);
  const int z = static_cast<int>(blockIdx.z);
  const int row = G.nx * (y + G.ny * z);
  unsigned hoff = 0;
  if constexpr (ROW) {
    const int l = static_cast<int>(threadIdx.x) & 63;
    const int x0 = x - l;
    int hx = l < S::H ? x0 - 1 - l : (l >= 64 - S::H ? x0 + 127 - l : x);
    hx %= G.nx;
    hx += hx < 0 ? G.nx : 0;
    hoff = static_cast<unsigned>(row + hx) * 4u;
  }
  // byte offsets of the sources x - e - k_x (tap +e) and x + e - k_x (tap -e)
  unsigned op[S::p + 1], om[S::p + 1];
#pragma unroll
  for (int t = 0; t <= S::p; ++t) {
    int sp = (x - S::e[t] - G.k[0]) % G.nx;
    int sm = (x + S::e[t] - G.k[0]) % G.nx;
    sp += sp < 0 ? G.nx : 0;
    sm += sm < 0 ? G.nx : 0;
    op[t] = static_cast<unsigned>(row + sp) * 4u;
    om[t] = static_cast<unsigned>(row + sm) * 4u;
  }
  float a32[M];
  if constexpr (ROW) {
    // the first kRowGroups groups take their taps across lanes (vector ALU), the rest by loads
    // (texture-address unit), so that neither unit carries the whole pass
    constexpr int kRowGroups = LBSMRT_ROW_GROUPS_NUM * n_sym(N) / LBSMRT_ROW_GROUPS_DEN;
    x_phases_row<Q1, N, 0, kGroupsPerPhaseRow, kRowGroups>(t2, G.stride, op[0], hoff, a32);
    x_groups<Q1, N, group_by(N, kRowGroups), group_bz(N, kRowGroups)>(L, t2, G.stride, op, om, a32);
  } else {
    x_groups<Q1, N, 0, 0>(L, t2, G.stride, op, om, a32);
  }
  double d[M];
#pragma unroll
  for (int i = 0; i < M; ++i) d[i] = static_cast<double>(a32[i]);
  double S5[5];
  sums_from_a<N>(d, L, S5);
  Macro mac = macro_from_sums(L, S5, G.err);
  mac.tsc = G.tsc;
  to_local<N>(d, mac);
  relax<N>(d, L, mac.rho, mac.tsc);
  to_lattice<N>(d, mac);
  const unsigned off = static_cast<unsigned>(row + x) * 4u;
#pragma unroll
  for (int i = 0; i < M; ++i) store_at(m_out + static_cast<size_t>(i) * G.stride, off, static_cast<float>(d[i]));
}

// ------------------------------------------------------------------ line domains
// A domain with ny = nz = 1 (a shock tube, or a periodic ring): every y and z tap pulls from the
// node itself, and sum_e K_{b a}(e) = sum_j He_b(c_j) w_j He_a(c_j) / a! is the Kronecker delta
// for a, b <= N (the quadrature is exact to degree 2N), so passes z and y are the identity and
// the step is the x-stage on the moment fields themselves, followed by the collision.  Pulls
// from beyond a shock tube's ends read the moments of its fixed end states.
//
// The x-stage is factored through the populations as in the box passes: for each tap pair +-e_t
// the two sources are folded by parity in float32, the rebuilt population of the fold (eq:fi)
// is formed and projected with He_b(c_t) (eq:an) in FP64 with FP64 tables.  The quadrature
// identity then holds to FP64 rounding, so a tube conserves mass, momentum and energy up to the
// float32 storage of the moments (float32 tables drift a steady shock by ~1e-6 of the mass per
// step).

// Sources of the x taps of one node: byte offset into a moment row, or a ghost column.
template <int Q1>
struct LineTaps {
  unsigned op[Taps1D<Q1>::p + 1], om[Taps1D<Q1>::p + 1];   // tap +e_t, tap -e_t
  int gp[Taps1D<Q1>::p + 1], gm[Taps1D<Q1>::p + 1];         // -1 inside, else the ghost column
};

// Moment field a of group (BY, BZ) at one tap source (ghost value past a tube's end).  GHOST is
// set when some node of the wave pulls from beyond its tube's ends (a wave-uniform choice made
// once per kernel, so that the taps themselves carry no branch and their loads stay in flight
// together).
template <bool GHOST>
__device__ __forceinline__ float line_tap(const float* __restrict__ row, unsigned off, int g,
                                          const float* __restrict__ ghost_col) {
  float v = load_at(row, off);
  if constexpr (GHOST) {
    const float gv = ghost_col[g < 0 ? 0 : g];
    v = g < 0 ? v : gv;
  }
  return v;
}

// One tap pair's contribution to group (BY, BZ): he[b] = He_b(c_t), rw[a] = Rw_a(c_t) (FP64),
// pair false for the centre tap.
template <int N, bool GHOST, int BY, int BZ>
__device__ __forceinline__ void line_tap_pair(const float* __restrict__ src, long long stride,
                                              const float* __restrict__ ghost_m, int n_ghost,
                                              unsigned op, int gp, unsigned om, int gm, bool pair,
                                              const double (&he)[N + 1], const double (&rw)[N + 1], double* acc) {
  constexpr int NO = N - BY - BZ;
  double ev = 0.0, od = 0.0;   // rebuilt population folded: even part (for even b), odd part
#pragma unroll
  for (int a = 0; a <= NO; ++a) {
    const int field = midx(a, BY, BZ);
    const float* __restrict__ row = src + static_cast<size_t>(field) * stride;
    const float* __restrict__ gcol = ghost_m + static_cast<size_t>(field) * n_ghost;
    // fold in FP32: exact where the two sources agree (a uniform state stays uniform), unbiased
    // elsewhere, and the loads in flight stay one register each
    const float vp = line_tap<GHOST>(row, op, gp, gcol);
    const float vm = pair ? line_tap<GHOST>(row, om, gm, gcol) : 0.f;
    const double s = static_cast<double>(vp + vm), dd = static_cast<double>(vp - vm);
    // K_{ba} uses s when a + b is even, d when odd
    ev = fma(rw[a], (a & 1) ? dd : s, ev);
    od = fma(rw[a], (a & 1) ? s : dd, od);
  }
#pragma unroll
  for (int b = 0; b <= NO; ++b) acc[b] = fma(he[b], (b & 1) ? od : ev, acc[b]);
}

template <int Q1, int N, bool GHOST, int BY, int BZ>
__device__ __forceinline__ void line_group(const LatticeConst& L, const float* __restrict__ src, long long stride,
                                           const float* __restrict__ ghost_m, int n_ghost,
                                           const LineTaps<Q1>& T, float (&a32)[n_moments(N)]) {
  using S = Taps1D<Q1>;
  constexpr int NO = N - BY - BZ;
  double acc[NO + 1];
#pragma unroll
  for (int b = 0; b <= NO; ++b) acc[b] = 0.0;
#pragma unroll
  for (int t = 0; t <= S::p; ++t) {
    double he[N + 1], rw[N + 1];
#pragma unroll
    for (int n = 0; n <= N; ++n) {
      he[n] = tab_he<Q1>(t, n);
      rw[n] = tab_rw<Q1>(t, n);
    }
    line_tap_pair<N, GHOST, BY, BZ>(src, stride, ghost_m, n_ghost, T.op[t], T.gp[t], T.om[t], T.gm[t],
                                    t > 0, he, rw, acc);
  }
  // pin the sums, and fence the loads after every phase of groups; the moments wait for
  // the collision as float32 (as in pass x)
#pragma unroll
  for (int b = 0; b <= NO; ++b) {
    float v = static_cast<float>(acc[b]);
    asm volatile("" : "+v"(v));
    a32[midx(b, BY, BZ)] = v;
  }
  if constexpr ((group_index(N, BY, BZ) + 1) % line_groups_per_phase<Q1>() == 0) asm volatile("" ::: "memory");
}

template <int Q1, int N, bool GHOST, int BY, int BZ>
__device__ __forceinline__ void line_groups(const LatticeConst& L, const float* __restrict__ src, long long stride,
                                            const float* __restrict__ ghost_m, int n_ghost,
                                            const LineTaps<Q1>& T, float (&a32)[n_moments(N)]) {
  if constexpr (BY <= N) {
    if constexpr (BY + BZ <= N) {
      line_group<Q1, N, GHOST, BY, BZ>(L, src, stride, ghost_m, n_ghost, T, a32);
      line_groups<Q1, N, GHOST, BY, BZ + 1>(L, src, stride, ghost_m, n_ghost, T, a32);
    } else {
      line_groups<Q1, N, GHOST, BY + 1, 0>(L, src, stride, ghost_m, n_ghost, T, a32);
    }
  }
}

// One tap pair's contribution to group (BY, BZ), its two sources read from the work-group's
// staged window (W slots per field, field-major) at slots wp (tap +e_t) and wm (tap -e_t);
// he[b] = He_b(c_t), rw[a] = Rw_a(c_t) (FP64), pair false for the centre tap.
template <int N, int W, int BY, int BZ>
__device__ __forceinline__ void win_tap_pair(const float* win, int wp, int wm, bool pair,
                                             const double (&he)[N + 1], const double (&rw)[N + 1], double* acc) {
  constexpr int NO = N - BY - BZ;
  double ev = 0.0, od = 0.0;   // rebuilt population folded: even part (for even b), odd part
#pragma unroll
  for (int a = 0; a <= NO; ++a) {
    const float* row = win + midx(a, BY, BZ) * W;
    // fold in FP32: exact where the two sources agree (a uniform state stays uniform)
    const float vp = row[wp];
    const float vm = pair ? row[wm] : 0.f;
    const double s = static_cast<double>(vp + vm), dd = static_cast<double>(vp - vm);
    // K_{ba} uses s when a + b is even, d when odd
    ev = fma(rw[a], (a & 1) ? dd : s, ev);
    od = fma(rw[a], (a & 1) ? s : dd, od);
  }
#pragma unroll
  for (int b = 0; b <= NO; ++b) acc[b] = fma(he[b], (b & 1) ? od : ev, acc[b]);
}

// Group (BY, BZ) and the groups after it in their compile-time order, for one lane's tap pair
// (its tables chosen at run time; zero beyond the taps) of the node at window slot wp - H + e.
template <int N, int W, int BY, int BZ>
__device__ __forceinline__ void win_groups_lane(const float* win, int wp, int wm, bool pair,
                                                const double (&he)[N + 1], const double (&rw)[N + 1],
                                                double (&d)[n_moments(N)]) {
  if constexpr (BY <= N) {
    if constexpr (BY + BZ <= N) {
      constexpr int NO = N - BY - BZ;
      double acc[NO + 1];
#pragma unroll
      for (int b = 0; b <= NO; ++b) acc[b] = 0.0;
      win_tap_pair<N, W, BY, BZ>(win, wp, wm, pair, he, rw, acc);
#pragma unroll
      for (int b = 0; b <= NO; ++b) d[midx(b, BY, BZ)] = acc[b];
      win_groups_lane<N, W, BY, BZ + 1>(win, wp, wm, pair, he, rw, d);
    } else {
      win_groups_lane<N, W, BY + 1, 0>(win, wp, wm, pair, he, rw, d);
    }
  }
}

// One node of a line domain per LPN work-items; work-groups of 64 work-items cover G = 64 / LPN
// consecutive nodes of one domain (a block of the block table; any number of line domains, each
// of its own length and end states; ghost_m: float32 [M][n_ghost] moments of the end states,
// columns 2 d, 2 d + 1 for domain d).
// LPN = 1: each work-item loads its taps' sources itself, a few groups' loads in flight at a time.
// LPN > 1 (short tubes, where each wave's serial load rounds set the step): the work-group first
// stages every moment field at the G + 2 H source positions its nodes pull from (x - e - k,
// |e| <= H) into LDS, one load per slot and eight in flight per work-item, with the periodic wrap
// of rings and the end states past a tube's ends resolved there; each lane then reads its tap
// pair from LDS.  (Staging with one lane per node was measured slower: 28.4 against 26.7 us on
// the 64-shock sweep.)
template <int Q1, int N, bool SHOCK, int LPN = 1>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(N >= 5 ? 2 : 1))) void k_ms_line_collide(
    LatticeConst L, StepArgs A, const float* __restrict__ ghost_m, const float* __restrict__ src,
    float* __restrict__ dst) {
  using S = Taps1D<Q1>;
  constexpr int M = n_moments(N);
  const BlockDev bd = A.blocks[blockIdx.x];
  const DomainDev D = A.doms[bd.dom];
  const int row0 = static_cast<int>(D.off);
  const int xl = static_cast<int>(threadIdx.x) / LPN;
  const int x = bd.first + xl;
  double d[M];
  if constexpr (LPN == 1) {
    if (x >= D.nx) return;
    bool ghost = false;
    auto source = [&](int xs, unsigned& off, int& g) {
      g = -1;
      if (D.bc_x == 0) {
        xs %= D.nx;
        if (xs < 0) xs += D.nx;
      } else if (xs < 0 || xs >= D.nx) {
        g = D.ghost + (xs < 0 ? 0 : 1);
        ghost = true;
        xs = x;                                 // an in-domain address; the ghost value replaces it
      }
      off = static_cast<unsigned>(row0 + xs) * 4u;
    };
    LineTaps<Q1> T;
#pragma unroll
    for (int t = 0; t <= S::p; ++t) {
      source(x - S::e[t] - L.k[0], T.op[t], T.gp[t]);
      source(x + S::e[t] - L.k[0], T.om[t], T.gm[t]);
    }
    float a32[M];
    if (SHOCK && __any(ghost)) line_groups<Q1, N, SHOCK, 0, 0>(L, src, A.stride, ghost_m, A.n_ghost, T, a32);
    else line_groups<Q1, N, false, 0, 0>(L, src, A.stride, ghost_m, A.n_ghost, T, a32);
#pragma unroll
    for (int i = 0; i < M; ++i) d[i] = static_cast<double>(a32[i]);
  } else {
    static_assert(LPN > S::p, "one tap pair per lane");
    constexpr int G = 64 / LPN;               // nodes per work-group
    constexpr int W = G + 2 * S::H;           // staged source positions per field
    __shared__ float win[M * W];
    const int w0 = bd.first - S::H - L.k[0]; // position of slot 0
    // source address of window slot i (field i / W)
    auto slot = [&](int i) -> const float* {
      const int f = i / W;
      int pos = w0 + (i - f * W);
      if (D.bc_x == 0 || !SHOCK) {
        pos %= D.nx;
        if (pos < 0) pos += D.nx;
      } else if (pos < 0 || pos >= D.nx) {
        return ghost_m + static_cast<size_t>(f) * A.n_ghost + D.ghost + (pos < 0 ? 0 : 1);
      }
      return src + static_cast<size_t>(f) * A.stride + row0 + pos;
    };
    constexpr int kIter = (M * W + 63) / 64;  // slots per work-item
    constexpr int kBatch = 8;                  // loads in flight per work-item
#pragma unroll 1
    for (int it0 = 0; it0 < kIter; it0 += kBatch) {
      float v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int i = (it0 + u) * 64 + static_cast<int>(threadIdx.x);
        v[u] = (it0 + u < kIter && i < M * W) ? *slot(i) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int i = (it0 + u) * 64 + static_cast<int>(threadIdx.x);
        if (it0 + u < kIter && i < M * W) win[i] = v[u];
      }
    }
    __syncthreads();
    if (x >= D.nx) return;                    // whole groups: the lanes of a node share x
    const int sub = static_cast<int>(threadIdx.x) % LPN;
    const int t = sub <= S::p ? sub : 0;
    int e = S::e[0];
#pragma unroll
    for (int j = 1; j <= S::p; ++j) e = t == j ? S::e[j] : e;
    double he[N + 1], rw[N + 1];
#pragma unroll
    for (int n = 0; n <= N; ++n) {
      double h = tab_he<Q1>(0, n), r = tab_rw<Q1>(0, n);
#pragma unroll
      for (int j = 1; j <= S::p; ++j) {
        h = t == j ? tab_he<Q1>(j, n) : h;
        r = t == j ? tab_rw<Q1>(j, n) : r;
      }
      he[n] = sub <= S::p ? h : 0.0;          // lanes beyond the taps contribute nothing
      rw[n] = r;
    }
    win_groups_lane<N, W, 0, 0>(win, xl + S::H - e, xl + S::H + e, t > 0, he, rw, d);
    group_allreduce<LPN, M>(d);
  }
  double S5[5];
  sums_from_a<N>(d, L, S5);
  Macro mac = macro_from_sums(L, S5, A.err);
  mac.tsc = D.tau_scale;
  to_local<N>(d, mac);
  relax<N>(d, L, mac.rho, mac.tsc);
  to_lattice<N>(d, mac);
  // with LPN > 1 every lane of the group stores the same values to the same addresses
  const unsigned off = static_cast<unsigned>(row0 + x) * 4u;
#pragma unroll
  for (int i = 0; i < M; ++i) store_at(dst + static_cast<size_t>(i) * A.stride, off, static_cast<float>(d[i]));
}

// Own-node projection of a population state: m[alpha] = sum_i f_i He_alpha(c_i) (FP64 sums).
template <int Q1, int N>
__global__ __launch_bounds__(256) void k_ms_project(LatticeConst L, const float* __restrict__ f,
                                                    float* __restrict__ m, long long stride, long long count) {
  constexpr int M = n_moments(N);
  const long long node = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (node >= count) return;
  double a[M];
  own_project64<Q1, N, false>(L, f, stride, static_cast<int>(node), a);
#pragma unroll
  for (int i = 0; i < M; ++i) m[static_cast<size_t>(i) * stride + node] = static_cast<float>(a[i]);
}

// Rebuild of the populations from a moment state: f_i = w_i sum_alpha m_alpha He_alpha(c_i) / alpha!.
template <int Q1, int N>
__global__ __launch_bounds__(256) void k_ms_expand(LatticeConst L, const float* __restrict__ m,
                                                   float* __restrict__ f, long long stride, long long count) {
  constexpr int M = n_moments(N);
  const long long node = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (node >= count) return;
  double a[M];
#pragma unroll
  for (int i = 0; i < M; ++i) a[i] = static_cast<double>(m[static_cast<size_t>(i) * stride + node]);
  reconstruct_store64<Q1, N>(L, a, f, stride, static_cast<int>(node));
}

// Moments of the truncated Maxwellian (App. B closed form per axis) of lab-frame (rho, u, theta).
template <int N>
__global__ __launch_bounds__(256) void k_ms_equilibrium(LatticeConst L, const double* __restrict__ fields,
                                                        long long count, float* __restrict__ m, long long stride) {
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
#pragma unroll
  for (int ax = 0; ax <= N; ++ax)
#pragma unroll
    for (int ay = 0; ay <= N; ++ay)
#pragma unroll
      for (int az = 0; az <= N; ++az)
        if (ax + ay + az <= N)
          m[static_cast<size_t>(midx(ax, ay, az)) * stride + node] = static_cast<float>(rho * Ax[ax] * Ay[ay] * Az[az]);
}

}  // namespace lbsmrt
