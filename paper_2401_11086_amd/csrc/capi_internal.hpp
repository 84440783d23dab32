// Internals shared by the C-ABI translation unit and the per-(Q1, N) launch units: the context
// and the launch dispatch of one compiled (stencil, order) pair.  Each launch unit explicitly
// instantiates one Launch<Q1, N> (launch_impl.hpp holds the member definitions), so the kernels
// of the five pairs compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "adjoint_kernels.hpp"
#include "kernels.hpp"
#include "lbsmrt.h"
#include "mfma_bf16x3.hpp"
#include "moment_state.hpp"

struct lbsmrt_ctx {
  int device = -1;
  int Q1 = 0, N = 0, Q = 0, M = 0;
  double r = 0.0;
  double w1[17] = {};
  int e1[17] = {};
  lbsmrt::LatticeConst L{};
  std::vector<lbsmrt_domain> doms;
  std::vector<long long> dom_off;
  long long n_nodes = 0, stride = 0;
  bool shock = false;
  int block = 256;
  int lpn = 1;                       // lanes per node of the step kernel (1; 2, 4 or 8: shocks, FP64)
  int n_blocks = 0;
  int n_ghost = 0;
  lbsmrt::DomainDev* d_doms = nullptr;
  lbsmrt::BlockDev* d_blocks = nullptr;
  float* d_ghost = nullptr;
  double* d_ghost_fields = nullptr;
  int* d_err = nullptr;
  double* d_partial = nullptr;   // [n_blocks_adj][kTauCols] per-block partial sums
  lbsmrt::BlockDev* d_blocks_adj = nullptr;  // 64-item work-groups for the adjoint and the loss seed
  lbsmrt::BlockDev* d_blocks_adj4 = nullptr; // 16-node work-groups of the adjoint at four lanes per node
  lbsmrt::BlockDev* d_blocks_adj8 = nullptr; // 8-node work-groups of the adjoint at eight lanes per node
  lbsmrt::BlockDev* d_blocks_adj16 = nullptr; // 4-node work-groups at sixteen lanes per node: the adjoint
  int n_blocks_adj16 = 0;                     // and the 17-point line moment-state kernel (0: not used)
  int n_blocks_adj4 = 0, n_blocks_adj8 = 0;
  lbsmrt::BlockDev* d_blocks_adjR = nullptr; // 256-node work-groups of the adjoint on periodic domains
  int n_blocks_adjR = 0;             // (0: not used)
  bool lpn4_ok = false;              // lanes_per_node > 1 allowed: shock domains, FP64
                                     // contractions, state below 4 GiB
  double* d_stage = nullptr;         // [kReduceBlocks][kTauCols] first-stage column sums
  // launch mode of lbsmrt_step
  int mode = LBSMRT_LAUNCH_DIRECT;
  int persistent_grid = 0;           // resident work-groups of the persistent kernel
  // persistent launch on line domains: per-block progress instead of a grid-wide barrier
  bool flow = false;                 // every domain a line (ny = nz = 1)
  int2* d_nbr = nullptr;             // [n_blocks] the blocks each block pulls from (-1: none)
  unsigned* d_done = nullptr;        // [n_blocks] steps completed since the tables were built
  unsigned flow_spin_limit = 1u << 22;
  unsigned flow_skew = 0;
  hipGraphExec_t graph = nullptr;    // captured pair of steps for LBSMRT_LAUNCH_GRAPH
  const float* graph_a = nullptr;
  const float* graph_b = nullptr;
  int graph_pairs = 0;
  hipGraphExec_t ms_graph = nullptr; // the same for lbsmrt_step_moment_state (its two state buffers
  const float* ms_graph_a = nullptr; // and the work buffer it was captured with)
  const float* ms_graph_b = nullptr;
  const float* ms_graph_w = nullptr;
  int n_blocks_adj = 0;
  int precision = LBSMRT_FP32;
  bool additive = false;              // f* = g + R (a' - a) instead of the rebuild (regularized = 0)
  // moment-state form: one periodic domain (box passes) or line domains only (ny = nz = 1: the
  // x-stage alone), with a stencil whose taps are compiled
  bool ms_ok = false;
  bool ms_lines = false;
  float* d_ghost_m = nullptr;        // [M][n_ghost] moments of the end states (line domains)
  lbsmrt::MomentTables64 ms_tab{};
  // split-BF16x3 contractions: MFMA operand tables and conservation constants (one allocation)
  void* d_mfma = nullptr;
  lbsmrt::MfmaArgs mfma{};          // 1D tap tables, checked against the compiled ones
};

namespace lbsmrt {

// Work-groups of the adjoint launch, one row of dL/dtau partial sums each: the 256-node periodic
// grid when the context has one, else the grid of its lanes-per-node setting.
inline int adjoint_groups(const lbsmrt_ctx* c) {
  if (!c->shock && c->n_blocks_adjR > 0) return c->n_blocks_adjR;
  if (c->lpn == 16) return c->n_blocks_adj16;
  return c->lpn == 8 ? c->n_blocks_adj8 : (c->lpn == 4 ? c->n_blocks_adj4 : c->n_blocks_adj);
}

// Launch dispatch over the compiled (Q1, N) pairs.  The 17-point stencil (kFull false) has the
// forward step with FP64 contractions and the rebuilt collision, the moments, the equilibrium
// fill, and the moment-state form on line domains (one lane per node) with the state
// conversions; the API refuses the rest for it before dispatching.
template <int Q1, int N>
struct Launch {
  static constexpr bool kFull = Q1 <= 9;
  template <int PREC>
  static void step_p(lbsmrt_ctx* c, const StepArgs& A, const float* src, float* dst, hipStream_t s);
  static void step(lbsmrt_ctx* c, const StepArgs& A, const float* src, float* dst, hipStream_t s);
  template <int PREC, bool SH, int LPN, bool FLOW>
  static const void* persistent_fn();
  template <bool FLOW>
  static const void* persistent_flow(const lbsmrt_ctx* c);
  static const void* persistent(const lbsmrt_ctx* c);
  static void moments(lbsmrt_ctx* c, const StepArgs& A, const float* f, double* out, unsigned mask, hipStream_t s);
  // Adjoint step and its dL/dtau reduction: per-work-group partials (adjoint_groups(c) rows of
  // n_tau_slots(N)) in partial, the first-stage column sums (kReduceBlocks rows) in stage.
  static void adjoint(lbsmrt_ctx* c, const StepArgs& A, const float* f_t, const float* lam_next, float* lam_t,
                      double* partial, double* stage, hipStream_t s);
  // Raise the dynamic LDS limit of the 256-node periodic adjoint (N <= 4); false if refused.
  static bool allow_row_adjoint();
  // Raise the dynamic LDS limit of the 64-item adjoint work-groups to what they take
  // (adjoint_lds_bytes: above 64 KB with one lane per node at N = 5); false if refused.
  static bool allow_adjoint_lds();
  static void loss_seed(lbsmrt_ctx* c, const StepArgs& A, const float* f, const double* target, const double* sc,
                        float* lam, hipStream_t s);
  // Moment-state form.  Line chunk of the z and y passes: a multiple of the tap window W, as long
  // as possible (the W - 1 halo rows are read again per chunk) while the launch still has about
  // kMsLanes work-items (4 waves per SIMD of the chip), and at most 8 W.
  static constexpr int kMsWindow = 2 * Taps1D<Q1>::H + 1;
  static constexpr long long kMsLanes = 262144;
  static int ms_chunk(long long lines, int len);
  static void ms_step(lbsmrt_ctx* c, const MsGeom& G, const float* src, float* dst, float* t1, float* t2,
                      hipStream_t s);
  // Line domains: eight lanes per node (one tap pair each) when the context splits nodes over
  // four or more lanes (small tubes), else one.
  static void ms_line_step(lbsmrt_ctx* c, const StepArgs& A0, const float* src, float* dst, hipStream_t s);
  static bool ms_taps_match(const lbsmrt_ctx* c);
  // The context's tap tables agree with the compiled ones of passes z and y (with these taps the
  // quadrature is unique, so every entry is the same up to the rounding of the host arithmetic).
  static bool ms_std_match(const lbsmrt_ctx* c);
  static void ms_project(lbsmrt_ctx* c, const float* f, float* m, hipStream_t s);
  static void ms_expand(lbsmrt_ctx* c, const float* m, float* f, hipStream_t s);
  static void ms_equilibrium_into(lbsmrt_ctx* c, const double* fields, long long count, float* m, long long stride,
                                  hipStream_t s);
  static void ms_equilibrium(lbsmrt_ctx* c, const double* fields, float* m, hipStream_t s);
  static void equilibrium(lbsmrt_ctx* c, const double* fields, long long count, float* f, long long stride,
                          hipStream_t s);
};

// the compiled pairs (one launch unit each)
extern template struct Launch<7, 3>;
extern template struct Launch<7, 4>;
extern template struct Launch<9, 4>;
extern template struct Launch<9, 5>;
extern template struct Launch<17, 5>;

}  // namespace lbsmrt
