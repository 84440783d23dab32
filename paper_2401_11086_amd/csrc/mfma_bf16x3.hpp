// Split-BF16x3 form of the fused step on the gfx950 matrix cores: the eq:an projection and the
// eq:fi rebuild run as dense MFMA products (v_mfma_f32_32x32x16_bf16) of bf16 halves,
// hi.hi + hi.lo + lo.hi with FP32 accumulation; the conserved sums, the frame shift, the
// irreducible split and the relaxation stay in FP64 on the vector ALUs.  Operand orderings:
// mfma_layout.hpp; tables and conservation constants: mfma_tables.cpp.
//
// Work-group: 256 work-items = 4 waves, each wave two tiles of 32 consecutive nodes (the MFMA
// columns) of one domain; a periodic domain needs nx % 32 == 0 so that a tile stays in one x row
// (its y and z, hence its y and z stream offsets, are uniform).  Both half-waves gather for the
// same 32 nodes (the B operand holds 8 populations of one node per lane), and after the
// projection one v_permlane32_swap per register moves each node's moments into one lane: lanes
// 0..31 then hold the nodes of tile 0, lanes 32..63 those of tile 1, and the FP64 collision runs
// one node per lane.  The rebuilt moments go back to the MFMA layout by the same swap.
#pragma once
#include "kernels.hpp"
#include "mfma_layout.hpp"

namespace lbsmrt {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

struct MfmaArgs {
  const u32x4_t* proj;      // [2][ATILES][KSTEPS_P][64]
  const u32x4_t* rebuild;   // [2][QTILES][KSTEPS_R][64]
  const double* cons;       // MfmaConsLayout<N>
};

// Lanes 32..63 of a trade values with lanes 0..31 of b.
__device__ __forceinline__ void swap_halves(unsigned& a, unsigned& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
  a = r[0];
  b = r[1];
}
__device__ __forceinline__ void swap_halves(float& a, float& b) {
  unsigned ua = __float_as_uint(a), ub = __float_as_uint(b);
  swap_halves(ua, ub);
  a = __uint_as_float(ua);
  b = __uint_as_float(ub);
}
__device__ __forceinline__ void swap_halves(double& a, double& b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  unsigned al = static_cast<unsigned>(ua), ah = static_cast<unsigned>(ua >> 32);
  unsigned bl = static_cast<unsigned>(ub), bh = static_cast<unsigned>(ub >> 32);
  swap_halves(al, bl);
  swap_halves(ah, bh);
  a = __builtin_bit_cast(double, (static_cast<unsigned long long>(ah) << 32) | al);
  b = __builtin_bit_cast(double, (static_cast<unsigned long long>(bh) << 32) | bl);
}

__device__ __forceinline__ bf16x8_t as_bf16x8(const u32x4_t& v) { return __builtin_bit_cast(bf16x8_t, v); }
__device__ __forceinline__ u32x4_t as_u32x4(const bf16x8_t& v) { return __builtin_bit_cast(u32x4_t, v); }

// One node tile of the gather: where a lane's node pulls from in the current x-slab.
struct TilePull {
  unsigned xoff;   // byte offset of (domain start + source x), before the y/z and plane offsets
  bool ghost;      // shock tubes: the source lies beyond an end (take the ghost state)
  int gside;       // 0 left, 1 right ghost column
  bool any_ghost;  // some lane of the wave pulls from a ghost this slab
};

template <int Q1, int N, bool SHOCK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_collide_stream_bf16x3(LatticeConst L, StepArgs A, MfmaArgs T,
                                                               const float* __restrict__ fsrc,
                                                               float* __restrict__ fdst) {
  using S = MfmaShape<Q1, N>;
  constexpr int M = S::M;
  constexpr int KPX = S::KPX;
  constexpr int AT = S::ATILES;
  constexpr int KR = S::KSTEPS_R;
  constexpr int kFence = Q1 <= 8 ? 4 : 2;   // k-steps per group of loads
  constexpr bool kProjAhead = Q1 <= 8;
  constexpr bool kRebLds = Q1 <= 8;   // both rebuild-table halves fit in LDS (66 KB at N = 4)
  __shared__ u32x4_t reb_lds[kRebLds ? 2 * S::REB_VEC : 1];
  if constexpr (kRebLds) {
    constexpr int kPer = static_cast<int>((2 * S::REB_VEC + 255) / 256);
    u32x4_t tmp[kPer];   // every load in flight before the first LDS write
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = static_cast<int>(threadIdx.x) + 256 * k;
      if (i < 2 * S::REB_VEC) tmp[k] = T.rebuild[i];
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = static_cast<int>(threadIdx.x) + 256 * k;
      if (i < 2 * S::REB_VEC) reb_lds[i] = tmp[k];
    }
    __syncthreads();
  }
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int j = lane & 31;
  const int h = lane >> 5;
  // all ones in the upper half-wave: per-lane choices between two uniform values are taken as
  // a + (hmask & (b - a)), which keeps both values in scalar registers (a select of two table
  // reads is turned into a read through a per-lane address, which puts the table in scratch)
  const unsigned hmask = h ? ~0u : 0u;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const BlockDev bd = A.blocks[blockIdx.x];
  const DomainDev D = A.doms[bd.dom];
  const int nxy = D.nx * D.ny;
  const int ndom = nxy * D.nz;
  // tile t: local nodes tstart[t] + 0..31 (one x row); this lane's column is node tstart[t] + j
  int tstart[2], xl[2], ty[2], tz[2];
  bool valid[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    tstart[t] = bd.first + 64 * wave + 32 * t;
    const int local = tstart[t] + j;
    valid[t] = local < ndom;
    xl[t] = SHOCK ? local : (tstart[t] % D.nx) + j;
    ty[t] = SHOCK ? 0 : (tstart[t] / D.nx) % D.ny;
    tz[t] = SHOCK ? 0 : tstart[t] / nxy;
  }
  const unsigned sbytes = static_cast<unsigned>(A.stride) * 4u;
  // y and z source offsets (bytes) of each tile per 1D index: the pull from rows ty - e_iy - k_y
  // and planes tz - e_iz - k_z (periodic), uniform over the tile
  unsigned yo[2][Q1], zo[2][Q1];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int i = 0; i < Q1; ++i) {
      int ys = 0, zs = 0;
      if (!SHOCK) {
        ys = (ty[t] - (L.e[i] + L.k[1])) % D.ny;
        if (ys < 0) ys += D.ny;
        zs = (tz[t] - (L.e[i] + L.k[2])) % D.nz;
        if (zs < 0) zs += D.nz;
      }
      yo[t][i] = static_cast<unsigned>(ys * D.nx) * 4u;
      zo[t][i] = static_cast<unsigned>(zs * nxy) * 4u;
    }

  // ---------------------------------------------------------------- gather + projection
  f32x16_t acc[AT][2];
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[a][t] = f32x16_t{};
  // FP64 conserved sums of this lane's share of the node's populations: sum g, sum g e_x,
  // sum g e_y, sum g e_z, sum g |e|^2
  double Sg[2][5];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int k = 0; k < 5; ++k) Sg[t][k] = 0.0;

#pragma unroll 1
  for (int ix = 0; ix < Q1; ++ix) {
    const int ex = L.e[ix];
    TilePull tp[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      int xs = xl[t] - (ex + L.k[0]);
      bool gh = false;
      int side = 0;
      if (SHOCK) {
        gh = xs < 0 || xs >= D.nx;
        side = xs >= D.nx ? 1 : 0;
        xs = gh ? 0 : xs;
      } else {
        xs %= D.nx;
        if (xs < 0) xs += D.nx;
      }
      tp[t].xoff = static_cast<unsigned>(D.off + xs) * 4u;
      tp[t].ghost = gh;
      tp[t].gside = side;
      tp[t].any_ghost = SHOCK && __any(gh);
    }
    const float* __restrict__ fx = fsrc + static_cast<size_t>(ix * Q1 * Q1) * A.stride;
    // the per-element offsets below do not depend on ix; without this the compiler hoists all of
    // them (hundreds of scalars) out of the slab loop and spills them
    unsigned sb = sbytes;
    asm volatile("" : "+s"(sb));
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < Q1; ++i) asm volatile("" : "+s"(yo[t][i]), "+s"(zo[t][i]));
    // Groups of kFence k-steps: every load of the group is issued first, then the values are
    // consumed in order (the scheduling barrier keeps the consumers behind the loads, so one
    // memory round trip serves the whole group instead of one load after another).
#pragma unroll
    for (int p0 = 0; p0 < KPX; p0 += kFence) {
      float gv[kFence][2][8];
#pragma unroll
      for (int pp = 0; pp < kFence; ++pp) {
        const int p = p0 + pp;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            int ixA = 0, iyA = 0, izA = 0, ixB = 0, iyB = 0, izB = 0;
            const bool okA = p < KPX && proj_pop(Q1, p, 0, e, ixA, iyA, izA);
            const bool okB = p < KPX && proj_pop(Q1, p, 1, e, ixB, iyB, izB);
            gv[pp][t][e] = 0.f;
            if (okA || okB) {
              // where only one half-wave has a population here (okA, okB are compile-time), the
              // other loads the same address and zeroes the value below: no load sits in a
              // lane-divergent branch, where it would wait for its own return
              const int iyAc = okA ? iyA : iyB, izAc = okA ? izA : izB;
              const int iyBc = okB ? iyB : iyAc, izBc = okB ? izB : izAc;
              const unsigned oA = yo[t][iyAc] + zo[t][izAc] + static_cast<unsigned>(iyAc * Q1 + izAc) * sb;
              const unsigned oB = yo[t][iyBc] + zo[t][izBc] + static_cast<unsigned>(iyBc * Q1 + izBc) * sb;
              gv[pp][t][e] = load_at(fx, tp[t].xoff + oA + (hmask & (oB - oA)));
            }
          }
      }
      // the projection-table operands of the group's k-steps travel with the same round trip
      // (7-point stencil; with 9 points the registers they need would spill)
      u32x4_t pa[kFence][AT][2];
#pragma unroll
      for (int pp = 0; pp < (kProjAhead ? kFence : 0); ++pp) {
        const int s = ix * KPX + (p0 + pp < KPX ? p0 + pp : KPX - 1);
#pragma unroll
        for (int a = 0; a < AT; ++a) {
          pa[pp][a][0] = T.proj[(static_cast<long long>(a) * S::KSTEPS_P + s) * 64 + lane];
          pa[pp][a][1] = T.proj[S::PROJ_VEC + (static_cast<long long>(a) * S::KSTEPS_P + s) * 64 + lane];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int pp = 0; pp < kFence; ++pp) {
        const int p = p0 + pp;
        if (p >= KPX) break;
        const int s = ix * KPX + p;
        // when every element of a half-wave lies on one z line the conserved sums are taken per
        // line, else per element
        const bool lines = Q1 <= 8 || p < 4;
        bf16x8_t bh[2], bl[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          float g[8];
          double V0 = 0.0, V1 = 0.0, V2 = 0.0;
          double Se[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            // (iy, iz) depend only on the k-step p inside the slab: evaluated at compile time
            int ixA = 0, iyA = 0, izA = 0, ixB = 0, iyB = 0, izB = 0;
            const bool okA = proj_pop(Q1, p, 0, e, ixA, iyA, izA);
            const bool okB = proj_pop(Q1, p, 1, e, ixB, iyB, izB);
            float v = 0.f;
            if (okA || okB) {
              const int iyAc = okA ? iyA : iyB, izAc = okA ? izA : izB;
              const int iyBc = okB ? iyB : iyAc, izBc = okB ? izB : izAc;
              v = gv[pp][t][e];
              if (SHOCK && tp[t].any_ghost) {
                const int qs = h == 0 ? iyAc * Q1 + izAc : iyBc * Q1 + izBc;
                const float gh = A.ghosts[static_cast<size_t>(ix * Q1 * Q1 + qs) * A.n_ghost + D.ghost + tp[t].gside];
                v = tp[t].ghost ? gh : v;
              }
              if (!(okA && okB)) v = (okA ? h == 0 : h != 0) ? v : 0.f;
              const double vd = static_cast<double>(v);
              constexpr auto& kE = MfmaStencil<Q1>::e;
              const int hm = static_cast<int>(hmask);
              const double ez = static_cast<double>(kE[izAc] + (hm & (kE[izBc] - kE[izAc])));
              if (lines) {
                const int zA2 = kE[izAc] * kE[izAc], zB2 = kE[izBc] * kE[izBc];
                const double ez2 = static_cast<double>(zA2 + (hm & (zB2 - zA2)));
                V0 += vd;
                V1 = fma(vd, ez, V1);
                V2 = fma(vd, ez2, V2);
              } else {
                const double ey = static_cast<double>(kE[iyAc] + (hm & (kE[iyBc] - kE[iyAc])));
                const int sA = kE[iyAc] * kE[iyAc] + kE[izAc] * kE[izAc], sB = kE[iyBc] * kE[iyBc] + kE[izBc] * kE[izBc];
                const double e2 = static_cast<double>(sA + (hm & (sB - sA)));
                Se[0] += vd;
                Se[2] = fma(vd, ey, Se[2]);
                Se[3] = fma(vd, ez, Se[3]);
                Se[4] = fma(vd, e2, Se[4]);
              }
            }
            g[e] = v;
          }
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const __bf16 hi = static_cast<__bf16>(g[e]);
            bh[t][e] = hi;
            bl[t][e] = static_cast<__bf16>(g[e] - static_cast<float>(hi));
          }
          const double exd = static_cast<double>(ex);
          if (lines) {   // the half-wave's line (ix, iy): fold its sums with e_x and e_y
            int i0 = 0, yA = 0, z0 = 0, yB = 0;
            proj_pop(Q1, p, 0, 0, i0, yA, z0);
            proj_pop(Q1, p, 1, 0, i0, yB, z0);
            constexpr auto& kE = MfmaStencil<Q1>::e;
            const int eyA = kE[yA < Q1 ? yA : 0], eyB = kE[yB < Q1 ? yB : 0];
            const double ey = static_cast<double>(eyA + (static_cast<int>(hmask) & (eyB - eyA)));
            Sg[t][0] += V0;
            Sg[t][1] = fma(V0, exd, Sg[t][1]);
            Sg[t][2] = fma(V0, ey, Sg[t][2]);
            Sg[t][3] += V1;
            Sg[t][4] = fma(V0, exd * exd + ey * ey, Sg[t][4] + V2);
          } else {
            Sg[t][0] += Se[0];
            Sg[t][1] = fma(Se[0], exd, Sg[t][1]);
            Sg[t][2] += Se[2];
            Sg[t][3] += Se[3];
            Sg[t][4] = fma(Se[0], exd * exd, Sg[t][4] + Se[4]);
          }
        }
#pragma unroll
        for (int a = 0; a < AT; ++a) {
          const long long ta = (static_cast<long long>(a) * S::KSTEPS_P + s) * 64 + lane;
          const bf16x8_t ah = as_bf16x8(kProjAhead ? pa[pp][a][0] : T.proj[ta]);
          const bf16x8_t al = as_bf16x8(kProjAhead ? pa[pp][a][1] : T.proj[S::PROJ_VEC + ta]);
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            acc[a][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[t], acc[a][t], 0, 0, 0);
            acc[a][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[t], acc[a][t], 0, 0, 0);
            acc[a][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[t], acc[a][t], 0, 0, 0);
          }
        }
      }
    }
  }

  // ---------------------------------------------------------------- one node per lane
  // after the swaps, lane l holds node tstart[h] + j: rows r and r + 4 of each 32-row tile
  // (r = 8 (v / 4) + v % 4) in acc[a][0][v] and acc[a][1][v]; the FP64 sums of both halves add up
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float x0 = acc[a][0][v], x1 = acc[a][1][v];
      swap_halves(x0, x1);
      acc[a][0][v] = x0;
      acc[a][1][v] = x1;
    }
  double Ssum[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double s0 = Sg[0][k], s1 = Sg[1][k];
    swap_halves(s0, s1);
    Ssum[k] = s0 + s1;
  }
  const bool mine = h == 0 ? valid[0] : valid[1];
  double d[M];
#pragma unroll
  for (int a = 0; a < AT; ++a)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 8 * (v / 4) + (v % 4);
      const int alo = 4 + 32 * a + r, ahi = alo + 4;
      if (alo < M) d[alo] = static_cast<double>(acc[a][0][v]);
      if (ahi < M) d[ahi] = static_cast<double>(acc[a][1][v]);
    }
  if (!mine) {   // a column past the domain's end: a unit Maxwellian at rest, never stored
#pragma unroll
    for (int i = 4; i < M; ++i) d[i] = 0.0;
    Ssum[0] = 1.0;
    Ssum[1] = Ssum[2] = Ssum[3] = 0.0;
    Ssum[4] = 3.0 / (L.r * L.r);
  }
  // orders 0 and 1 and the trace of order 2 from the FP64 sums (the MFMA trace would leave an
  // unrelaxed (2,1) part and re-emit its rounding as energy every step)
  d[0] = Ssum[0];
  d[1] = L.r * Ssum[1];
  d[2] = L.r * Ssum[2];
  d[3] = L.r * Ssum[3];
  {
    const double tr = L.r * L.r * Ssum[4] - 3.0 * Ssum[0];
    const double dtr = (tr - (d[midx(2, 0, 0)] + d[midx(0, 2, 0)] + d[midx(0, 0, 2)])) * (1.0 / 3.0);
    d[midx(2, 0, 0)] += dtr;
    d[midx(0, 2, 0)] += dtr;
    d[midx(0, 0, 2)] += dtr;
  }
  Macro mac = macro_from_sums(L, Ssum, A.err);
  mac.tsc = D.tau_scale;
  to_local<N>(d, mac);
  relax<N>(d, L, mac.rho, mac.tsc);
  to_lattice<N>(d, mac);

  // ---------------------------------------------------------------- rebuild operands
  // b = (a'_hi | c_hi | 0) and (a'_lo | c_lo | 0), c the conservation correction (mfma_tables.cpp)
  using CL = MfmaConsLayout<N>;
  // the constants are the same for every lane: read them through the constant address space so
  // that they land in scalar registers (as vector loads they filled the register file)
  const __attribute__((address_space(4))) double* __restrict__ cons =
      (const __attribute__((address_space(4))) double*)(T.cons);
  double defect[5];
  {
    const double ir = 1.0 / L.r;
    defect[0] = d[0];
    defect[1] = d[1] * ir;
    defect[2] = d[2] * ir;
    defect[3] = d[3] * ir;
    defect[4] = (3.0 * d[0] + d[midx(2, 0, 0)] + d[midx(0, 2, 0)] + d[midx(0, 0, 2)]) * ir * ir;
  }
  __bf16 khi[16 * KR], klo[16 * KR];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const __bf16 hi = static_cast<__bf16>(static_cast<float>(d[i]));
    const double hd = static_cast<double>(static_cast<float>(hi));
    const __bf16 lo = static_cast<__bf16>(static_cast<float>(d[i] - hd));
    const double ld = static_cast<double>(static_cast<float>(lo));
    khi[i] = hi;
    klo[i] = lo;
#pragma unroll
    for (int k = 0; k < 5; ++k) defect[k] -= cons[CL::phi(k, i)] * (hd + ld) + cons[CL::plo(k, i)] * hd;
    if (i % 2 == 1) asm volatile("" ::: "memory");   // a few moments' constants in scalar registers at a time
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double c = 0.0;
#pragma unroll
    for (int m = 0; m < 5; ++m) c = fma(cons[CL::MINV + k * 5 + m], defect[m], c);
    const __bf16 hi = static_cast<__bf16>(static_cast<float>(c));
    khi[M + k] = hi;
    klo[M + k] = static_cast<__bf16>(static_cast<float>(c - static_cast<double>(static_cast<float>(hi))));
  }
#pragma unroll
  for (int i = M + 5; i < 16 * KR; ++i) {
    khi[i] = static_cast<__bf16>(0.f);
    klo[i] = static_cast<__bf16>(0.f);
  }
  // back to the MFMA layout: for k-step kk, tile 0 takes the lower 8 k-values of lanes 0..31 in
  // its lower half-wave and the upper 8 of the same nodes in its upper half-wave (and tile 1
  // likewise from lanes 32..63): one swap of (lower 8, upper 8) per k-step
  bf16x8_t B1[2][KR], B2[2][KR];
#pragma unroll
  for (int kk = 0; kk < KR; ++kk) {
    bf16x8_t lo1, up1, lo2, up2;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      lo1[e] = khi[16 * kk + e];
      up1[e] = khi[16 * kk + 8 + e];
      lo2[e] = klo[16 * kk + e];
      up2[e] = klo[16 * kk + 8 + e];
    }
    u32x4_t x0 = as_u32x4(lo1), x1 = as_u32x4(up1), y0 = as_u32x4(lo2), y1 = as_u32x4(up2);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      unsigned a0 = x0[w], a1 = x1[w], c0 = y0[w], c1 = y1[w];
      swap_halves(a0, a1);
      swap_halves(c0, c1);
      x0[w] = a0;
      x1[w] = a1;
      y0[w] = c0;
      y1[w] = c1;
    }
    B1[0][kk] = as_bf16x8(x0);
    B1[1][kk] = as_bf16x8(x1);
    B2[0][kk] = as_bf16x8(y0);
    B2[1][kk] = as_bf16x8(y1);
  }

  // ---------------------------------------------------------------- rebuild + store
  // tile t, register v: population q = 32 tau + 8 (v / 4) + 4 h + v % 4 of node tstart[t] + j.
  // The matrix cores drop low bits of addends much smaller than the running sum (measured: a
  // negative bias of ~0.1 ulp per population, which a long run turns into a mass and energy
  // drift).  So the first k-step's hi.hi product, which carries orders 0..2 and most of the
  // value, runs from a zero accumulator; every other product (higher orders, then the lo
  // halves and the correction columns) runs in a second chain of smaller values; one
  // round-to-nearest add per population joins them.
  // Rebuild tables: with the 7-point stencil both halves sit in LDS (copied there at the start of
  // the work-group), so their reads wait on the LDS counter alone.  Otherwise the tables of q-tile
  // tau are loaded from memory while tile tau - 1 is processed; global loads and stores share one
  // counter, so each tile still waits for the previous tile's stores.  Only the last tile has rows
  // past Q; the stores of a tile share one validity test (a whole tile is past the end of a
  // periodic domain, or not).
  const unsigned hoff = static_cast<unsigned>(h) * 4u * sbytes + static_cast<unsigned>(j) * 4u;
  const u32x4_t* __restrict__ rtab = T.rebuild;
  if constexpr (kRebLds) rtab = reb_lds;
  u32x4_t th[KR], tl[KR];
#pragma unroll
  for (int kk = 0; kk < KR; ++kk) {
    th[kk] = rtab[kk * 64 + lane];
    tl[kk] = rtab[S::REB_VEC + kk * 64 + lane];
  }
#pragma unroll
  for (int tau = 0; tau < S::QTILES; ++tau) {
    const int tn = tau + 1 < S::QTILES ? tau + 1 : tau;
    const long long an = static_cast<long long>(tn) * KR * 64 + lane;
    u32x4_t nh[KR], nl[KR];
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) {
      nh[kk] = rtab[an + kk * 64];
      nl[kk] = rtab[S::REB_VEC + an + kk * 64];
    }
    __builtin_amdgcn_sched_barrier(0);
    f32x16_t big0, big1, c0 = f32x16_t{}, c1 = f32x16_t{};
    big0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(th[0]), B1[0][0], f32x16_t{}, 0, 0, 0);
    big1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(th[0]), B1[1][0], f32x16_t{}, 0, 0, 0);
#pragma unroll
    for (int kk = KR - 1; kk >= 1; --kk) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(th[kk]), B1[0][kk], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(th[kk]), B1[1][kk], c1, 0, 0, 0);
    }
#pragma unroll
    for (int kk = KR - 1; kk >= 0; --kk) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(th[kk]), B2[0][kk], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(th[kk]), B2[1][kk], c1, 0, 0, 0);
    }
#pragma unroll
    for (int kk = KR - 1; kk >= 0; --kk) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(tl[kk]), B1[0][kk], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(tl[kk]), B1[1][kk], c1, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      c0[v] = big0[v] + c0[v];
      c1[v] = big1[v] + c1[v];
    }
    float* __restrict__ base0 = fdst + static_cast<size_t>(32 * tau) * A.stride + D.off + tstart[0];
    float* __restrict__ base1 = fdst + static_cast<size_t>(32 * tau) * A.stride + D.off + tstart[1];
    if (tau + 1 < S::QTILES) {
      if (valid[0]) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
          store_pop<!SHOCK>(base0 + static_cast<size_t>(8 * (v / 4) + (v % 4)) * A.stride, hoff, c0[v]);
      }
      if (valid[1]) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
          store_pop<!SHOCK>(base1 + static_cast<size_t>(8 * (v / 4) + (v % 4)) * A.stride, hoff, c1[v]);
      }
    } else {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = 8 * (v / 4) + (v % 4);   // row of the lower half-wave in the tile
        const bool qok = 32 * tau + r + 4 * h < S::Q;
        if (qok && valid[0]) store_pop<!SHOCK>(base0 + static_cast<size_t>(r) * A.stride, hoff, c0[v]);
        if (qok && valid[1]) store_pop<!SHOCK>(base1 + static_cast<size_t>(r) * A.stride, hoff, c1[v]);
      }
    }
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) {
      th[kk] = nh[kk];
      tl[kk] = nl[kk];
    }
  }
}

}  // namespace lbsmrt
