// Member definitions of Launch<Q1, N> (capi_internal.hpp); included only by the launch units,
// each of which instantiates one pair.
#pragma once
#include <algorithm>

#include "capi_internal.hpp"

namespace lbsmrt {

template <int Q1, int N>
template <int PREC>
void Launch<Q1, N>::step_p(lbsmrt_ctx* c, const StepArgs& A, const float* src, float* dst, hipStream_t s) {
    // additive collision: FP64 contractions, one lane per node
    if constexpr (kFull) {
      if (PREC == kPrecFp64 && c->additive && c->shock) {
        hipLaunchKernelGGL((k_collide_stream<Q1, N, true, kPrecFp64, 1, true>), dim3(c->n_blocks), dim3(c->block), 0,
                           s, c->L, A, src, dst);
        return;
      }
      if (PREC == kPrecFp64 && c->additive) {
        hipLaunchKernelGGL((k_collide_stream<Q1, N, false, kPrecFp64, 1, true>), dim3(c->n_blocks), dim3(c->block), 0,
                           s, c->L, A, src, dst);
        return;
      }
    }
    if (PREC == kPrecFp64 && c->shock && c->lpn == 16)
      hipLaunchKernelGGL((k_collide_stream<Q1, N, true, kPrecFp64, 16>), dim3(c->n_blocks), dim3(c->block), 0, s, c->L,
                         A, src, dst);
    else if (PREC == kPrecFp64 && c->shock && c->lpn == 8)
      hipLaunchKernelGGL((k_collide_stream<Q1, N, true, kPrecFp64, 8>), dim3(c->n_blocks), dim3(c->block), 0, s, c->L,
                         A, src, dst);
    else if (PREC == kPrecFp64 && c->shock && c->lpn == 4)
      hipLaunchKernelGGL((k_collide_stream<Q1, N, true, kPrecFp64, 4>), dim3(c->n_blocks), dim3(c->block), 0, s, c->L,
                         A, src, dst);
    else if (PREC == kPrecFp64 && c->shock && c->lpn == 2)
      hipLaunchKernelGGL((k_collide_stream<Q1, N, true, kPrecFp64, 2>), dim3(c->n_blocks), dim3(c->block), 0, s, c->L,
                         A, src, dst);
    else if (c->shock)
      hipLaunchKernelGGL((k_collide_stream<Q1, N, true, PREC>), dim3(c->n_blocks), dim3(c->block), 0, s, c->L, A, src,
                         dst);
    else
      hipLaunchKernelGGL((k_collide_stream<Q1, N, false, PREC>), dim3(c->n_blocks), dim3(c->block), 0, s, c->L, A, src,
                         dst);
  }

template <int Q1, int N>
void Launch<Q1, N>::step(lbsmrt_ctx* c, const StepArgs& A, const float* src, float* dst, hipStream_t s) {
    if constexpr (kFull) {
      if (c->precision == LBSMRT_FP32) {
        step_p<kPrecFp32>(c, A, src, dst, s);
        return;
      }
      if (c->precision == LBSMRT_SPLIT_BF16X3) {   // 256-item work-groups, 4 waves of 64 nodes
        if (c->shock)
          hipLaunchKernelGGL((k_collide_stream_bf16x3<Q1, N, true>), dim3(c->n_blocks), dim3(256), 0, s, c->L, A,
                             c->mfma, src, dst);
        else
          hipLaunchKernelGGL((k_collide_stream_bf16x3<Q1, N, false>), dim3(c->n_blocks), dim3(256), 0, s, c->L, A,
                             c->mfma, src, dst);
        return;
      }
    }
    step_p<kPrecFp64>(c, A, src, dst, s);
  }

template <int Q1, int N>
template <int PREC, bool SH, int LPN, bool FLOW>
const void* Launch<Q1, N>::persistent_fn() {
    return reinterpret_cast<const void*>(&k_collide_persistent<Q1, N, SH, PREC, LPN, FLOW>);
  }

template <int Q1, int N>
template <bool FLOW>
const void* Launch<Q1, N>::persistent_flow(const lbsmrt_ctx* c) {
    if (c->precision == LBSMRT_FP64_CONTRACT && c->shock && c->lpn == 8) return persistent_fn<kPrecFp64, true, 8, FLOW>();
    if (c->precision == LBSMRT_FP64_CONTRACT && c->shock && c->lpn == 4) return persistent_fn<kPrecFp64, true, 4, FLOW>();
    if (c->precision == LBSMRT_FP64_CONTRACT && c->shock && c->lpn == 2) return persistent_fn<kPrecFp64, true, 2, FLOW>();
    if (c->precision == LBSMRT_FP32)
      return c->shock ? persistent_fn<kPrecFp32, true, 1, FLOW>() : persistent_fn<kPrecFp32, false, 1, FLOW>();
    return c->shock ? persistent_fn<kPrecFp64, true, 1, FLOW>() : persistent_fn<kPrecFp64, false, 1, FLOW>();
  }

template <int Q1, int N>
const void* Launch<Q1, N>::persistent(const lbsmrt_ctx* c) {
    if constexpr (!kFull) {
      return nullptr;
    } else {
      if (c->precision == LBSMRT_SPLIT_BF16X3) return nullptr;
      return c->flow ? persistent_flow<true>(c) : persistent_flow<false>(c);
    }
  }

template <int Q1, int N>
void Launch<Q1, N>::moments(lbsmrt_ctx* c, const StepArgs& A, const float* f, double* out, unsigned mask, hipStream_t s) {
    if (c->shock)
      hipLaunchKernelGGL((k_moments<Q1, N, true>), dim3(c->n_blocks), dim3(c->block / c->lpn), 0, s, c->L, A, f, out, mask,
                         c->n_nodes);
    else
      hipLaunchKernelGGL((k_moments<Q1, N, false>), dim3(c->n_blocks), dim3(c->block / c->lpn), 0, s, c->L, A, f, out, mask,
                         c->n_nodes);
  }

template <int Q1, int N>
void Launch<Q1, N>::adjoint(lbsmrt_ctx* c, const StepArgs& A, const float* f_t, const float* lam_next, float* lam_t,
                            double* partial, double* stage, hipStream_t s) {
    if constexpr (!kFull) {
      return;
    } else {
      const int nb = adjoint_groups(c);
      if constexpr (N <= 4) {
        if (!c->shock && c->n_blocks_adjR > 0) {
          hipLaunchKernelGGL((k_adjoint<Q1, N, false, 1, kAdjRowBlock>), dim3(nb), dim3(kAdjRowBlock),
                             (adjoint_lds_bytes<N, 1, kAdjRowBlock>()), s, c->L, A, f_t, lam_next, lam_t, partial);
          hipLaunchKernelGGL(k_reduce_stage1, dim3(kReduceBlocks), dim3(256), 0, s, partial, nb, n_tau_slots(N),
                             stage);
          hipLaunchKernelGGL((k_reduce_tau<N>), dim3(1), dim3(kReduceBlocks), 0, s, stage, A.dtau);
          return;
        }
      }
      if (c->shock && c->lpn == 16)
        hipLaunchKernelGGL((k_adjoint<Q1, N, true, 16>), dim3(nb), dim3(kAdjBlock),
                           (adjoint_lds_bytes<N, 16, kAdjBlock>()), s, c->L, A, f_t, lam_next, lam_t, partial);
      else if (c->shock && c->lpn == 8)
        hipLaunchKernelGGL((k_adjoint<Q1, N, true, 8>), dim3(nb), dim3(kAdjBlock), (adjoint_lds_bytes<N, 8, kAdjBlock>()),
                           s, c->L, A, f_t, lam_next, lam_t, partial);
      else if (c->shock && c->lpn == 4)
        hipLaunchKernelGGL((k_adjoint<Q1, N, true, 4>), dim3(nb), dim3(kAdjBlock), (adjoint_lds_bytes<N, 4, kAdjBlock>()),
                           s, c->L, A, f_t, lam_next, lam_t, partial);
      else if (c->shock)
        hipLaunchKernelGGL((k_adjoint<Q1, N, true>), dim3(nb), dim3(kAdjBlock), (adjoint_lds_bytes<N, 1, kAdjBlock>()), s,
                           c->L, A, f_t, lam_next, lam_t, partial);
      else
        hipLaunchKernelGGL((k_adjoint<Q1, N, false>), dim3(nb), dim3(kAdjBlock), (adjoint_lds_bytes<N, 1, kAdjBlock>()),
                           s, c->L, A, f_t, lam_next, lam_t, partial);
      if (nb <= kSmallReduceRows) {
        hipLaunchKernelGGL((k_reduce_tau_rows<N>), dim3(1), dim3(kReduceBlocks), 0, s, partial, nb, A.dtau);
        return;
      }
      hipLaunchKernelGGL(k_reduce_stage1, dim3(kReduceBlocks), dim3(256), 0, s, partial, nb, n_tau_slots(N), stage);
      hipLaunchKernelGGL((k_reduce_tau<N>), dim3(1), dim3(kReduceBlocks), 0, s, stage, A.dtau);
    }
  }

template <int Q1, int N>
bool Launch<Q1, N>::allow_adjoint_lds() {
    if constexpr (!kFull) {
      return true;
    } else {
      auto raise = [](const void* fn, size_t bytes) {
        return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes)) ==
               hipSuccess;
      };
      return raise(reinterpret_cast<const void*>(&k_adjoint<Q1, N, true, 16>), adjoint_lds_bytes<N, 16, kAdjBlock>()) &&
             raise(reinterpret_cast<const void*>(&k_adjoint<Q1, N, true, 8>), adjoint_lds_bytes<N, 8, kAdjBlock>()) &&
             raise(reinterpret_cast<const void*>(&k_adjoint<Q1, N, true, 4>), adjoint_lds_bytes<N, 4, kAdjBlock>()) &&
             raise(reinterpret_cast<const void*>(&k_adjoint<Q1, N, true>), adjoint_lds_bytes<N, 1, kAdjBlock>()) &&
             raise(reinterpret_cast<const void*>(&k_adjoint<Q1, N, false>), adjoint_lds_bytes<N, 1, kAdjBlock>());
    }
  }

template <int Q1, int N>
bool Launch<Q1, N>::allow_row_adjoint() {
    if constexpr (N <= 4) {
      const int bytes = static_cast<int>(adjoint_lds_bytes<N, 1, kAdjRowBlock>());
      return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adjoint<Q1, N, false, 1, kAdjRowBlock>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, bytes) == hipSuccess;
    }
    return false;
  }

template <int Q1, int N>
void Launch<Q1, N>::loss_seed(lbsmrt_ctx* c, const StepArgs& A, const float* f, const double* target, const double* sc,
                        float* lam, hipStream_t s) {
    if constexpr (!kFull) {
      return;
    } else {
      if (c->shock)
        hipLaunchKernelGGL((k_loss_seed<Q1, N, true>), dim3(c->n_blocks_adj), dim3(64), 0, s, c->L, A, f, target,
                           c->n_nodes, sc[0], sc[1], sc[2], lam, c->d_partial);
      else
        hipLaunchKernelGGL((k_loss_seed<Q1, N, false>), dim3(c->n_blocks_adj), dim3(64), 0, s, c->L, A, f, target,
                           c->n_nodes, sc[0], sc[1], sc[2], lam, c->d_partial);
    }
  }

template <int Q1, int N>
int Launch<Q1, N>::ms_chunk(long long lines, int len) {
    const long long chunks = std::max(1LL, (kMsLanes + lines - 1) / lines);
    const long long rows = (len + chunks - 1) / chunks;
    const long long r = std::min(8LL, std::max(1LL, rows / kMsWindow));
    return static_cast<int>(r) * kMsWindow;
  }

template <int Q1, int N>
void Launch<Q1, N>::ms_step(lbsmrt_ctx* c, const MsGeom& G, const float* src, float* dst, float* t1, float* t2,
                      hipStream_t s) {
    if constexpr (!kFull) {
      return;
    } else {
      const long long lz = static_cast<long long>(G.nx) * G.ny, ly = static_cast<long long>(G.nx) * G.nz;
      const int Tz = ms_chunk(lz, G.nz), Ty = ms_chunk(ly, G.ny);
      hipLaunchKernelGGL((k_ms_pass_z<Q1, N>), dim3(static_cast<unsigned>((lz + 255) / 256), (G.nz + Tz - 1) / Tz),
                         dim3(256), 0, s, G, src, t1, Tz);
      hipLaunchKernelGGL((k_ms_pass_y<Q1, N>), dim3(static_cast<unsigned>((ly + 255) / 256), (G.ny + Ty - 1) / Ty),
                         dim3(256), 0, s, G, t1, t2, Ty);
      if (G.nx % 64 == 0 && G.k[0] == 0)
        hipLaunchKernelGGL((k_ms_pass_x_collide<Q1, N, true>), dim3((G.nx + 255) / 256, G.ny, G.nz), dim3(256), 0, s,
                           c->L, G, t2, dst);
      else
        hipLaunchKernelGGL((k_ms_pass_x_collide<Q1, N, false>), dim3((G.nx + 255) / 256, G.ny, G.nz), dim3(256), 0, s,
                           c->L, G, t2, dst);
    }
  }

template <int Q1, int N>
void Launch<Q1, N>::ms_line_step(lbsmrt_ctx* c, const StepArgs& A0, const float* src, float* dst, hipStream_t s) {
    if constexpr (!kFull) {
      // nine tap pairs: sixteen lanes per node (one tap pair each) when the context splits nodes
      // over four or more lanes (shock tubes), else one
      StepArgs A = A0;
      const bool split = c->lpn >= 4 && c->n_blocks_adj16 > 0;
      A.blocks = split ? c->d_blocks_adj16 : c->d_blocks_adj;
      const int nb = split ? c->n_blocks_adj16 : c->n_blocks_adj;
      if (split)
        hipLaunchKernelGGL((k_ms_line_collide<Q1, N, true, 16>), dim3(nb), dim3(kAdjBlock), 0, s, c->L, A,
                           c->d_ghost_m, src, dst);
      else if (c->shock)
        hipLaunchKernelGGL((k_ms_line_collide<Q1, N, true, 1>), dim3(nb), dim3(kAdjBlock), 0, s, c->L, A,
                           c->d_ghost_m, src, dst);
      else
        hipLaunchKernelGGL((k_ms_line_collide<Q1, N, false, 1>), dim3(nb), dim3(kAdjBlock), 0, s, c->L, A,
                           c->d_ghost_m, src, dst);
    } else {
      StepArgs A = A0;
      const bool split = c->lpn >= 4;
      A.blocks = split ? c->d_blocks_adj8 : c->d_blocks_adj;
      const int nb = split ? c->n_blocks_adj8 : c->n_blocks_adj;
      if (split && c->shock)
        hipLaunchKernelGGL((k_ms_line_collide<Q1, N, true, 8>), dim3(nb), dim3(kAdjBlock), 0, s, c->L, A,
                           c->d_ghost_m, src, dst);
      else if (split)
        hipLaunchKernelGGL((k_ms_line_collide<Q1, N, false, 8>), dim3(nb), dim3(kAdjBlock), 0, s, c->L, A,
                           c->d_ghost_m, src, dst);
      else if (c->shock)
        hipLaunchKernelGGL((k_ms_line_collide<Q1, N, true, 1>), dim3(nb), dim3(kAdjBlock), 0, s, c->L, A,
                           c->d_ghost_m, src, dst);
      else
        hipLaunchKernelGGL((k_ms_line_collide<Q1, N, false, 1>), dim3(nb), dim3(kAdjBlock), 0, s, c->L, A,
                           c->d_ghost_m, src, dst);
    }
  }

template <int Q1, int N>
bool Launch<Q1, N>::ms_taps_match(const lbsmrt_ctx* c) {
    const int p = Q1 / 2;
    for (int t = 0; t <= Taps1D<Q1>::p; ++t)
      if (c->e1[p + t] != Taps1D<Q1>::e[t]) return false;
    return true;
  }

template <int Q1, int N>
bool Launch<Q1, N>::ms_std_match(const lbsmrt_ctx* c) {
    auto close = [](double a, double b) { return std::fabs(a - b) <= 1e-13 * std::max(1.0, std::fabs(b)); };
    for (int t = 0; t <= Taps1D<Q1>::p; ++t)
      for (int n = 0; n <= N; ++n)
        if (!close(c->ms_tab.He[t][n], MsStdTables<Q1>::He[t][n]) || !close(c->ms_tab.Rw[t][n], MsStdTables<Q1>::Rw[t][n]))
          return false;
    return true;
  }

template <int Q1, int N>
void Launch<Q1, N>::ms_project(lbsmrt_ctx* c, const float* f, float* m, hipStream_t s) {
    const unsigned nb = static_cast<unsigned>((c->n_nodes + 255) / 256);
    hipLaunchKernelGGL((k_ms_project<Q1, N>), dim3(nb), dim3(256), 0, s, c->L, f, m, c->stride, c->n_nodes);
  }

template <int Q1, int N>
void Launch<Q1, N>::ms_expand(lbsmrt_ctx* c, const float* m, float* f, hipStream_t s) {
    const unsigned nb = static_cast<unsigned>((c->n_nodes + 255) / 256);
    hipLaunchKernelGGL((k_ms_expand<Q1, N>), dim3(nb), dim3(256), 0, s, c->L, m, f, c->stride, c->n_nodes);
  }

template <int Q1, int N>
void Launch<Q1, N>::ms_equilibrium_into(lbsmrt_ctx* c, const double* fields, long long count, float* m, long long stride,
                                  hipStream_t s) {
    const unsigned nb = static_cast<unsigned>((count + 255) / 256);
    hipLaunchKernelGGL((k_ms_equilibrium<N>), dim3(nb), dim3(256), 0, s, c->L, fields, count, m, stride);
  }

template <int Q1, int N>
void Launch<Q1, N>::ms_equilibrium(lbsmrt_ctx* c, const double* fields, float* m, hipStream_t s) {
    const unsigned nb = static_cast<unsigned>((c->n_nodes + 255) / 256);
    hipLaunchKernelGGL((k_ms_equilibrium<N>), dim3(nb), dim3(256), 0, s, c->L, fields, c->n_nodes, m, c->stride);
  }

template <int Q1, int N>
void Launch<Q1, N>::equilibrium(lbsmrt_ctx* c, const double* fields, long long count, float* f, long long stride,
                          hipStream_t s) {
    const int bs = 256;
    const long long nb = (count + bs - 1) / bs;
    hipLaunchKernelGGL((k_equilibrium<Q1, N>), dim3(static_cast<unsigned>(nb)), dim3(bs), 0, s, c->L, fields, count,
                       f, stride);
  }

}  // namespace lbsmrt
