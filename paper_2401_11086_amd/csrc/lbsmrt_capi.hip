// C-ABI of the LB-SMRT library: context set-up, launches, error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "capi_internal.hpp"
#include "host_setup.hpp"
#include "mfma_tables.hpp"

using namespace lbsmrt;

// Reduction scratch of lbsmrt_step_adjoint_noalloc: the per-work-group dL/dtau partial sums
// followed by the first-stage column sums.  One copy per GPU, at its own address, held until the
// process ends; calls on one GPU share it.  Host code never passes this name to a kernel: it
// uses the address scratch_address returns for the device.
constexpr size_t kScratchDoubles = size_t(1) << 20;   // 8 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];


namespace {

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t e__ = (expr);                           \
    if (e__ != hipSuccess) return LBSMRT_E_HIP;        \
  } while (0)

double hermite_1d(int n, double x) {
  double h0 = 1.0, h1 = x;
  if (n == 0) return h0;
  for (int k = 1; k < n; ++k) {
    const double h2 = x * h1 - k * h0;
    h0 = h1;
    h1 = h2;
  }
  return h1;
}

bool supported(int Q1, int N) {
  return (Q1 == 7 && (N == 3 || N == 4)) || (Q1 == 9 && (N == 4 || N == 5)) || (Q1 == 17 && N == 5);
}

template <typename F>
void dispatch(int Q1, int N, F&& fn) {
  if (Q1 == 7 && N == 3) fn(Launch<7, 3>{});
  else if (Q1 == 7 && N == 4) fn(Launch<7, 4>{});
  else if (Q1 == 9 && N == 4) fn(Launch<9, 4>{});
  else if (Q1 == 9 && N == 5) fn(Launch<9, 5>{});
  else if (Q1 == 17 && N == 5) fn(Launch<17, 5>{});
}

StepArgs step_args(const lbsmrt_ctx* c) {
  StepArgs A;
  A.doms = c->d_doms;
  A.blocks = c->d_blocks;
  A.ghosts = c->d_ghost;
  A.n_ghost = c->n_ghost;
  A.stride = c->stride;
  A.err = c->d_err;
  return A;
}

void drop_graph(lbsmrt_ctx* c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  c->graph_a = c->graph_b = nullptr;
  if (c->ms_graph) (void)hipGraphExecDestroy(c->ms_graph);
  c->ms_graph = nullptr;
  c->ms_graph_a = c->ms_graph_b = c->ms_graph_w = nullptr;
}

// Capture 2 graph_pairs calls of step(t, stream) (t = 0, 1, ...) on a private stream into an
// executable graph; false if any stage fails.
template <class StepFn>
bool capture_steps(int n, hipGraphExec_t* out, StepFn step) {
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return false;
  hipGraph_t g = nullptr;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    for (int t = 0; t < n; ++t) step(t, cs);
    ok = hipStreamEndCapture(cs, &g) == hipSuccess;
  }
  if (ok) ok = hipGraphInstantiate(out, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  return ok;
}

void free_ctx(lbsmrt_ctx* c) {
  if (!c) return;
  if (c->device >= 0) (void)hipSetDevice(c->device);
  drop_graph(c);
  (void)hipFree(c->d_doms);
  (void)hipFree(c->d_blocks);
  (void)hipFree(c->d_ghost);
  (void)hipFree(c->d_ghost_fields);
  (void)hipFree(c->d_err);
  (void)hipFree(c->d_partial);
  (void)hipFree(c->d_blocks_adj);
  (void)hipFree(c->d_blocks_adj4);
  (void)hipFree(c->d_blocks_adj8);
  (void)hipFree(c->d_blocks_adj16);
  (void)hipFree(c->d_blocks_adjR);
  (void)hipFree(c->d_stage);
  (void)hipFree(c->d_ghost_m);
  (void)hipFree(c->d_mfma);
  (void)hipFree(c->d_nbr);
  (void)hipFree(c->d_done);
  delete c;
}

// Progress tables of the persistent launch on line domains for the current block table (blocks
// of c->block / c->lpn nodes): each block depends on its neighbours in its domain (periodic rings
// wrap), which must hold the whole pull reach max |e_j + k_x|.  False (and no tables) when a block
// is shorter than the reach, or a ring of more than three blocks ends in a block shorter than the
// reach (its neighbours would pull across it); the grid-barrier form is used then.
bool build_flow(lbsmrt_ctx* c) {
  (void)hipFree(c->d_nbr);
  (void)hipFree(c->d_done);
  c->d_nbr = nullptr;
  c->d_done = nullptr;
  int reach = 0;
  for (int j = 0; j < c->Q1; ++j) reach = std::max(reach, std::abs(c->e1[j] + c->L.k[0]));
  const int npb = c->block / c->lpn;
  if (npb < reach) return false;
  std::vector<int2> nbr;
  for (const lbsmrt_domain& d : c->doms) {
    const int nb = (d.nx + npb - 1) / npb;
    const int b0 = static_cast<int>(nbr.size());
    if (d.bc_x == 0 && nb > 3 && d.nx % npb != 0 && d.nx % npb < reach) return false;
    for (int i = 0; i < nb; ++i) {
      int prev = i > 0 ? b0 + i - 1 : -1, next = i + 1 < nb ? b0 + i + 1 : -1;
      if (d.bc_x == 0 && nb > 1) {
        if (prev < 0) prev = b0 + nb - 1;
        if (next < 0) next = b0;
      }
      if (prev == next) next = -1;
      nbr.push_back(int2{prev, next});
    }
  }
  if (static_cast<int>(nbr.size()) != c->n_blocks) return false;
  if (hipMalloc(&c->d_nbr, sizeof(int2) * nbr.size()) != hipSuccess ||
      hipMalloc(&c->d_done, sizeof(unsigned) * nbr.size()) != hipSuccess ||
      hipMemcpy(c->d_nbr, nbr.data(), sizeof(int2) * nbr.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(c->d_done, 0, sizeof(unsigned) * nbr.size()) != hipSuccess) {
    (void)hipFree(c->d_nbr);
    (void)hipFree(c->d_done);
    c->d_nbr = nullptr;
    c->d_done = nullptr;
    return false;
  }
  return true;
}

// Device address of scratch per device ordinal, looked up once per device with that device
// current (lbsmrt_init_lattice); nullptr until then or if the lookup failed.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Looks up the address of scratch on device dev, which must be current: E_HIP if
// hipGetSymbolAddress fails.  Ordinals from kMaxDevices on are skipped (their contexts cannot use
// the allocation-free entry point).
lbsmrt_status scratch_lookup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return LBSMRT_OK;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return LBSMRT_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return LBSMRT_E_HIP;
  g_scratch[dev] = static_cast<double*>(p);
  return LBSMRT_OK;
}

double* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[dev];
}

// Eligible contexts start with L lanes per node while nodes * L stays within 65536 work-items
// (1024 wavefronts, one per SIMD of the chip): 8 up to 8192 nodes, 4 up to 16384, else 1.
constexpr long long kSplitWorkItems = 65536;

// Work-group table: consecutive runs of `bs` nodes of each domain.
std::vector<BlockDev> block_table(const std::vector<lbsmrt_domain>& doms, int bs) {
  std::vector<BlockDev> bl;
  for (size_t i = 0; i < doms.size(); ++i) {
    const long long n = static_cast<long long>(doms[i].nx) * doms[i].ny * doms[i].nz;
    for (long long first = 0; first < n; first += bs) bl.push_back(BlockDev{static_cast<int>(i), static_cast<int>(first)});
  }
  return bl;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

lbsmrt_status validate_desc(const lbsmrt_lattice_desc* d) {
  if (!d) return LBSMRT_E_ARG;
  if (d->n_abscissa < 1 || d->n_abscissa > 8) return LBSMRT_E_ARG;
  if (d->order_N < 2 || d->order_N > kMaxN) return LBSMRT_E_ARG;
  if (d->regularized != 0 && d->regularized != 1) return LBSMRT_E_ARG;
  if (d->precision != LBSMRT_FP32 && d->precision != LBSMRT_FP64_CONTRACT && d->precision != LBSMRT_SPLIT_BF16X3)
    return LBSMRT_E_UNSUPPORTED;
  if (d->regularized == 0 && d->precision != LBSMRT_FP64_CONTRACT) return LBSMRT_E_UNSUPPORTED;
  if (!(d->rho_ref > 0.0)) return LBSMRT_E_ARG;
  for (int n = 2; n <= d->order_N; ++n)
    for (int m = 0; 2 * m <= n; ++m) {
      if (n == 2 && m == 1) continue;
      if (!(d->tau[n][m] > 0.0) || !std::isfinite(d->tau[n][m])) return LBSMRT_E_ARG;
    }
  return LBSMRT_OK;
}


lbsmrt_status adjoint_check(const lbsmrt_ctx* c, const float* f_t, const float* lam_next, const float* lam_t,
                            const double* dL_dtau) {
  if (!c || !f_t || !lam_next || !lam_t || !dL_dtau) return LBSMRT_E_ARG;
  if (c->Q1 > 9) return LBSMRT_E_UNSUPPORTED;   // no kernel for the 17-point stencil
  if (lam_t == lam_next || lam_t == f_t) return LBSMRT_E_ARG;
  if (c->additive) return LBSMRT_E_UNSUPPORTED;
  return LBSMRT_OK;
}

lbsmrt_status adjoint_launch(lbsmrt_ctx* c, const float* f_t, const float* lam_next, float* lam_t, double* dL_dtau,
                             double* partial, double* stage, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  StepArgs A = step_args(c);
  A.blocks = c->lpn == 16 ? c->d_blocks_adj16
             : (c->lpn == 8 ? c->d_blocks_adj8 : (c->lpn == 4 ? c->d_blocks_adj4 : c->d_blocks_adj));
  if (!c->shock && c->n_blocks_adjR > 0) A.blocks = c->d_blocks_adjR;
  A.dtau = dL_dtau;
  dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::adjoint(c, A, f_t, lam_next, lam_t, partial, stage, s); });
  return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
}

}  // namespace

extern "C" {

const char* lbsmrt_status_string(lbsmrt_status s) {
  switch (s) {
    case LBSMRT_OK: return "ok";
    case LBSMRT_E_ARG: return "invalid argument";
    case LBSMRT_E_QUADRATURE: return "no positive-weight quadrature for this stencil and degree";
    case LBSMRT_E_STATE: return "a node left rho > 0, 0 < theta < 2 (or became non-finite)";
    case LBSMRT_E_HIP: return "HIP runtime error";
    case LBSMRT_E_NOMEM: return "out of memory";
    case LBSMRT_E_UNSUPPORTED: return "unsupported configuration";
    case LBSMRT_E_LIMIT: return "problem too large for the fixed scratch of an allocation-free entry point";
    case LBSMRT_E_TIMEOUT: return "a persistent launch's wait for a neighbouring work-group gave up";
  }
  return "unknown status";
}

lbsmrt_status lbsmrt_solve_quadrature(int n_abscissa, const int* abscissa, int degree, double* r_out, double* w_out) {
  return solve_quadrature(abscissa, n_abscissa, degree, r_out, w_out);
}

lbsmrt_status lbsmrt_shock_states(double Ma, double gamma, double theta1, double theta2, double c_l, double* out) {
  return shock_states(Ma, gamma, theta1, theta2, c_l, out);
}

lbsmrt_status lbsmrt_init_lattice(const lbsmrt_lattice_desc* desc, const lbsmrt_domain* domains, int n_domains,
                                  void* stream, lbsmrt_ctx** out) {
  if (!out || !domains || n_domains < 1 || n_domains > 4096) return LBSMRT_E_ARG;
  *out = nullptr;
  lbsmrt_status st = validate_desc(desc);
  if (st != LBSMRT_OK) return st;
  const int p = desc->n_abscissa;
  const int Q1 = 2 * p + 1;
  if (!supported(Q1, desc->order_N)) return LBSMRT_E_UNSUPPORTED;
  // the 17-point stencil: forward step with FP64 contractions and the rebuilt collision only
  if (Q1 > 9 && (desc->precision != LBSMRT_FP64_CONTRACT || desc->regularized == 0)) return LBSMRT_E_UNSUPPORTED;

  double r = 0.0, w[17] = {};
  st = solve_quadrature(desc->abscissa, p, desc->degree, &r, w);
  if (st != LBSMRT_OK) return st;
  if (desc->degree < 2 * desc->order_N) return LBSMRT_E_ARG;  // eq:an needs a degree-2N rule

  lbsmrt_ctx* c = new (std::nothrow) lbsmrt_ctx();
  if (!c) return LBSMRT_E_NOMEM;
  c->Q1 = Q1;
  c->N = desc->order_N;
  c->Q = Q1 * Q1 * Q1;
  c->M = n_moments(c->N);
  c->r = r;
  c->precision = desc->precision;
  c->additive = desc->regularized == 0;
  for (int j = 0; j < Q1; ++j) {
    const int jj = j - p;  // -p..p
    const int a = jj == 0 ? 0 : (jj < 0 ? -desc->abscissa[-jj - 1] : desc->abscissa[jj - 1]);
    c->e1[j] = a;
    c->w1[j] = jj == 0 ? w[0] : w[(jj < 0 ? -jj : jj)];
  }
  // lattice constants
  LatticeConst& L = c->L;
  std::memset(&L, 0, sizeof(L));
  for (int j = 0; j < Q1; ++j) {
    L.e[j] = c->e1[j];
    const double cj = r * c->e1[j];
    double fact = 1.0;
    for (int n = 0; n <= c->N; ++n) {
      if (n > 0) fact *= n;
      const double h = hermite_1d(n, cj);
      L.He[j][n] = static_cast<float>(h);
      L.Rw[j][n] = static_cast<float>(c->w1[j] * h / fact);
      L.He64[j][n] = h;
      L.Rw64[j][n] = c->w1[j] * h / fact;
    }
  }
  dual_projection_table(L.Rw, L.He64, Q1, c->N, L.Hd);
  L.r = r;
  for (int k = 0; k < 3; ++k) L.k[k] = desc->shift_k[k];
  for (int n = 0; n <= kMaxN; ++n)
    for (int m = 0; m < 3; ++m) L.tau[n][m] = (n <= c->N && 2 * m <= n) ? desc->tau[n][m] : 1.0;
  L.tau[2][1] = 1.0;
  L.rho_ref = desc->rho_ref;
  L.tau_offset = desc->tau_offset_half ? 0.5 : 0.0;
  L.density_scaling = desc->tau_density_scaling ? 1 : 0;

  // domains, node space, block table
  c->doms.assign(domains, domains + n_domains);
  long long off = 0;
  std::vector<DomainDev> dd(n_domains);
  long long max_local = 0;
  for (int i = 0; i < n_domains; ++i) {
    const lbsmrt_domain& D = domains[i];
    if (D.nx < 1 || D.ny < 1 || D.nz < 1 || (D.bc_x != 0 && D.bc_x != 1)) { free_ctx(c); return LBSMRT_E_ARG; }
    const long long n = static_cast<long long>(D.nx) * D.ny * D.nz;
    if (D.bc_x == 1) {
      c->shock = true;
      if (!(D.rho_in > 0 && D.rho_out > 0 && D.theta_in > 0 && D.theta_in < 2 && D.theta_out > 0 && D.theta_out < 2)) {
        free_ctx(c);
        return LBSMRT_E_ARG;
      }
    }
    dd[i].off = off;
    dd[i].nx = D.nx; dd[i].ny = D.ny; dd[i].nz = D.nz;
    dd[i].bc_x = D.bc_x;
    dd[i].ghost = 2 * i;
    dd[i].pad = 0;
    if (D.tau_scale < 0.0 || !std::isfinite(D.tau_scale)) { free_ctx(c); return LBSMRT_E_ARG; }
    dd[i].tau_scale = D.tau_scale > 0.0 ? D.tau_scale : 1.0;
    c->dom_off.push_back(off);
    off += n;
    if (n > max_local) max_local = n;
  }
  c->n_nodes = off;
  if (off >= (1LL << 30)) { free_ctx(c); return LBSMRT_E_ARG; }   // 32-bit node offsets in the kernels
  c->stride = (off + 63) / 64 * 64;
  c->block = (max_local >= 4096) ? 256 : 64;
  if (c->precision == LBSMRT_SPLIT_BF16X3) {
    // the MFMA step takes 256-node work-groups of 32-node tiles, each inside one x row
    for (int i = 0; i < n_domains; ++i)
      if (domains[i].bc_x == 0 && domains[i].nx % 32 != 0) { free_ctx(c); return LBSMRT_E_UNSUPPORTED; }
    // 32-bit byte offsets inside one x-slab (Q1^2 population planes) and across 4 planes (stores)
    if (static_cast<long long>(c->Q1) * c->Q1 * c->stride * 4 >= (1LL << 32)) { free_ctx(c); return LBSMRT_E_UNSUPPORTED; }
    c->block = 256;
  }
  // Shock tubes with few nodes fill a small part of the GPU, and each wavefront's serial work
  // sets the step time: start with several lanes per node there (lbsmrt_set_launch can change it).
  // (the split kernels address a slab by a 32-bit byte offset from the start of f)
  c->lpn4_ok = c->shock && c->precision == LBSMRT_FP64_CONTRACT && !c->additive &&
               static_cast<long long>(c->Q) * c->stride * 4 < (1LL << 32);
  // nine or more x-slabs: sixteen lanes (one slab each on nine lanes) while the work-items stay
  // within kSplitWorkItems; seven slabs gain nothing beyond eight
  if (c->lpn4_ok)
    c->lpn = (Q1 >= 9 && off * 16 <= kSplitWorkItems) ? 16
             : (off * 8 <= kSplitWorkItems ? 8 : (off * 4 <= kSplitWorkItems ? 4 : 1));
  std::vector<BlockDev> bl = block_table(c->doms, c->block / c->lpn);
  c->n_blocks = static_cast<int>(bl.size());
  std::vector<BlockDev> bla = block_table(c->doms, kAdjBlock);
  c->n_blocks_adj = static_cast<int>(bla.size());
  std::vector<BlockDev> bla4, bla8;
  if (c->lpn4_ok) {
    bla4 = block_table(c->doms, kAdjBlock / 4);
    bla8 = block_table(c->doms, kAdjBlock / 8);
  }
  c->n_blocks_adj4 = static_cast<int>(bla4.size());
  c->n_blocks_adj8 = static_cast<int>(bla8.size());
  // sixteen lanes per node: the adjoint, and the 17-point stencil's line moment-state kernel
  // (nine tap pairs)
  std::vector<BlockDev> bla16;
  if (c->lpn4_ok) bla16 = block_table(c->doms, kAdjBlock / 16);
  c->n_blocks_adj16 = static_cast<int>(bla16.size());
  // periodic domains with N <= 4: 256-node adjoint work-groups when their LDS fits one work-group
  std::vector<BlockDev> blaR;
  if (!c->shock && c->N <= 4) {
    int dev = 0, max_lds = 0;
    const size_t need = 2 * sizeof(double) * c->M * kAdjRowBlock + sizeof(double) * n_tau_slots(c->N) * kAdjRowBlock;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        need <= static_cast<size_t>(max_lds)) {
      bool ok = true;
      dispatch(c->Q1, c->N, [&](auto l) { ok = decltype(l)::allow_row_adjoint(); });
      if (ok) blaR = block_table(c->doms, kAdjRowBlock);
    }
  }
  c->n_blocks_adjR = static_cast<int>(blaR.size());
  {
    bool ok = true;
    dispatch(c->Q1, c->N, [&](auto l) { ok = decltype(l)::allow_adjoint_lds(); });
    if (!ok) { free_ctx(c); return LBSMRT_E_HIP; }
  }
  const size_t partial_rows =
      static_cast<size_t>(std::max({c->n_blocks_adj, c->n_blocks_adj4, c->n_blocks_adj8, c->n_blocks_adj16,
                                    c->n_blocks_adjR}));
  c->n_ghost = 2 * n_domains;
  // moment-state form (lbsmrt_step_moment_state): the FP64 1D tables of the non-negative taps t,
  // K_{b a}(e_t) = He_b(c_t) Rw_a(c_t)
  dispatch(c->Q1, c->N, [&](auto l) { c->ms_ok = decltype(l)::ms_taps_match(c); });
  bool lines = true;
  for (int i = 0; i < n_domains; ++i) lines = lines && domains[i].ny == 1 && domains[i].nz == 1;
  c->ms_lines = c->ms_ok && lines && !c->additive;
  c->flow = false;   // set with the persistent launch (build_flow) for line domains
  c->ms_ok = c->ms_ok && !c->additive && (lines || (c->Q1 <= 9 && n_domains == 1 && domains[0].bc_x == 0));
  for (int t = 0; t <= p && t < kMsMaxTaps; ++t)
    for (int n = 0; n <= c->N; ++n) {
      c->ms_tab.He[t][n] = L.He64[p + t][n];
      c->ms_tab.Rw[t][n] = L.Rw64[p + t][n];
    }
  dispatch(c->Q1, c->N, [&](auto l) { c->ms_ok = c->ms_ok && decltype(l)::ms_std_match(c); });
  c->ms_lines = c->ms_lines && c->ms_ok;

  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&c->device) != hipSuccess) { free_ctx(c); return LBSMRT_E_HIP; }
  // device address of the allocation-free adjoint's scratch (looked up once per device)
  if (scratch_lookup(c->device) != LBSMRT_OK) { free_ctx(c); return LBSMRT_E_HIP; }
  auto fail = [&](lbsmrt_status code) { free_ctx(c); return code; };
  if (hipMalloc(&c->d_doms, sizeof(DomainDev) * dd.size()) != hipSuccess) return fail(LBSMRT_E_NOMEM);
  if (hipMalloc(&c->d_blocks, sizeof(BlockDev) * bl.size()) != hipSuccess) return fail(LBSMRT_E_NOMEM);
  if (hipMalloc(&c->d_ghost, sizeof(float) * c->Q * c->n_ghost) != hipSuccess) return fail(LBSMRT_E_NOMEM);
  if (hipMalloc(&c->d_ghost_fields, sizeof(double) * 5 * c->n_ghost) != hipSuccess) return fail(LBSMRT_E_NOMEM);
  if (hipMalloc(&c->d_err, sizeof(int)) != hipSuccess) return fail(LBSMRT_E_NOMEM);
  if (hipMalloc(&c->d_partial, sizeof(double) * kTauCols * partial_rows) != hipSuccess) return fail(LBSMRT_E_NOMEM);
  if (hipMalloc(&c->d_blocks_adj, sizeof(BlockDev) * bla.size()) != hipSuccess) return fail(LBSMRT_E_NOMEM);
  if (!bla4.empty() && hipMalloc(&c->d_blocks_adj4, sizeof(BlockDev) * bla4.size()) != hipSuccess)
    return fail(LBSMRT_E_NOMEM);
  if (!bla8.empty() && hipMalloc(&c->d_blocks_adj8, sizeof(BlockDev) * bla8.size()) != hipSuccess)
    return fail(LBSMRT_E_NOMEM);
  if (!bla16.empty() && hipMalloc(&c->d_blocks_adj16, sizeof(BlockDev) * bla16.size()) != hipSuccess)
    return fail(LBSMRT_E_NOMEM);
  if (!blaR.empty() && hipMalloc(&c->d_blocks_adjR, sizeof(BlockDev) * blaR.size()) != hipSuccess)
    return fail(LBSMRT_E_NOMEM);
  if (hipMalloc(&c->d_stage, sizeof(double) * kTauCols * kReduceBlocks) != hipSuccess) return fail(LBSMRT_E_NOMEM);
  if (c->ms_lines && hipMalloc(&c->d_ghost_m, sizeof(float) * c->M * c->n_ghost) != hipSuccess)
    return fail(LBSMRT_E_NOMEM);
  if (c->precision == LBSMRT_SPLIT_BF16X3) {
    // built for the stencils D1Q7 {0, +-1, +-2, +-3} and D1Q9 {0, +-1, +-2, +-3, +-5}
    bool std_taps = c->Q1 == 7 || c->Q1 == 9;
    for (int j = 0; std_taps && j < c->Q1; ++j)
      std_taps = c->e1[j] == (c->Q1 == 7 ? MfmaStencil<7>::e[j] : MfmaStencil<9>::e[j]);
    if (!std_taps) return fail(LBSMRT_E_UNSUPPORTED);
    MfmaHostTables mt;
    if (!build_mfma_tables(c->Q1, c->N, r, c->w1, c->e1, mt)) return fail(LBSMRT_E_QUADRATURE);
    const size_t pb = mt.proj.size() * 2, rb = mt.rebuild.size() * 2, cb = mt.cons.size() * sizeof(double);
    if (hipMalloc(&c->d_mfma, pb + rb + cb) != hipSuccess) return fail(LBSMRT_E_NOMEM);
    char* base = static_cast<char*>(c->d_mfma);
    if (hipMemcpy(base, mt.proj.data(), pb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + pb, mt.rebuild.data(), rb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + pb + rb, mt.cons.data(), cb, hipMemcpyHostToDevice) != hipSuccess)
      return fail(LBSMRT_E_HIP);
    c->mfma.proj = reinterpret_cast<const u32x4_t*>(base);
    c->mfma.rebuild = reinterpret_cast<const u32x4_t*>(base + pb);
    c->mfma.cons = reinterpret_cast<const double*>(base + pb + rb);
  }
  // ghost states: rows rho, ux, uy, uz, theta, columns (left_i, right_i)
  std::vector<double> gf(5 * c->n_ghost, 0.0);
  for (int i = 0; i < n_domains; ++i) {
    const lbsmrt_domain& D = domains[i];
    const bool sh = D.bc_x == 1;
    const double rin = sh ? D.rho_in : 1.0, rout = sh ? D.rho_out : 1.0;
    const double tin = sh ? D.theta_in : 1.0, tout = sh ? D.theta_out : 1.0;
    for (int side = 0; side < 2; ++side) {
      const int col = 2 * i + side;
      gf[0 * c->n_ghost + col] = side ? rout : rin;
      for (int k = 0; k < 3; ++k) gf[(1 + k) * c->n_ghost + col] = sh ? (side ? D.u_out[k] : D.u_in[k]) : r * L.k[k];
      gf[4 * c->n_ghost + col] = side ? tout : tin;
    }
  }
  if (hipMemcpyAsync(c->d_doms, dd.data(), sizeof(DomainDev) * dd.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(c->d_blocks, bl.data(), sizeof(BlockDev) * bl.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(c->d_blocks_adj, bla.data(), sizeof(BlockDev) * bla.size(), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      (!bla4.empty() && hipMemcpyAsync(c->d_blocks_adj4, bla4.data(), sizeof(BlockDev) * bla4.size(),
                                       hipMemcpyHostToDevice, s) != hipSuccess) ||
      (!bla8.empty() && hipMemcpyAsync(c->d_blocks_adj8, bla8.data(), sizeof(BlockDev) * bla8.size(),
                                       hipMemcpyHostToDevice, s) != hipSuccess) ||
      (!bla16.empty() && hipMemcpyAsync(c->d_blocks_adj16, bla16.data(), sizeof(BlockDev) * bla16.size(),
                                        hipMemcpyHostToDevice, s) != hipSuccess) ||
      (!blaR.empty() && hipMemcpyAsync(c->d_blocks_adjR, blaR.data(), sizeof(BlockDev) * blaR.size(),
                                       hipMemcpyHostToDevice, s) != hipSuccess) ||
      hipMemcpyAsync(c->d_ghost_fields, gf.data(), sizeof(double) * gf.size(), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemsetAsync(c->d_err, 0, sizeof(int), s) != hipSuccess)
    return fail(LBSMRT_E_HIP);
  dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::equilibrium(c, c->d_ghost_fields, c->n_ghost, c->d_ghost, c->n_ghost, s); });
  if (c->ms_lines)   // moments of the end states, [M][n_ghost]
    dispatch(c->Q1, c->N, [&](auto l) {
      decltype(l)::ms_equilibrium_into(c, c->d_ghost_fields, c->n_ghost, c->d_ghost_m, c->n_ghost, s);
    });
  if (hipGetLastError() != hipSuccess) return fail(LBSMRT_E_HIP);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(LBSMRT_E_HIP);
  *out = c;
  return LBSMRT_OK;
}

lbsmrt_status lbsmrt_get_info(const lbsmrt_ctx* c, lbsmrt_info* o) {
  if (!c || !o) return LBSMRT_E_ARG;
  std::memset(o, 0, sizeof(*o));
  o->Q = c->Q; o->Q1 = c->Q1; o->M = c->M; o->N = c->N;
  o->c_l = c->r;
  for (int j = 0; j < c->Q1; ++j) { o->w1d[j] = c->w1[j]; o->e1d[j] = c->e1[j]; }
  o->n_nodes = c->n_nodes;
  o->f_stride = c->stride;
  o->f_len = c->stride * c->Q;
  o->n_domains = static_cast<int>(c->doms.size());
  for (size_t i = 0; i < c->dom_off.size() && i < 64; ++i) o->domain_offset[i] = c->dom_off[i];
  return LBSMRT_OK;
}

lbsmrt_status lbsmrt_get_domain_offsets(const lbsmrt_ctx* c, long long* out, int capacity, int* n_written) {
  if (!c || !out || capacity < 1) return LBSMRT_E_ARG;
  const int n = static_cast<int>(std::min<size_t>(static_cast<size_t>(capacity), c->dom_off.size()));
  for (int i = 0; i < n; ++i) out[i] = c->dom_off[i];
  if (n_written) *n_written = n;
  return LBSMRT_OK;
}

lbsmrt_status lbsmrt_step(lbsmrt_ctx* c, float* f_a, float* f_b, int n_steps, void* stream) {
  if (!c || !f_a || !f_b || f_a == f_b || n_steps < 1) return LBSMRT_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const StepArgs A = step_args(c);
  auto direct = [&](int first_step, int count) {
    for (int t = first_step; t < first_step + count; ++t) {
      const float* src = (t & 1) ? f_b : f_a;
      float* dst = (t & 1) ? f_a : f_b;
      dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::step(c, A, src, dst, s); });
    }
  };
  if (c->mode == LBSMRT_LAUNCH_PERSISTENT) {
    const void* fn = nullptr;
    dispatch(c->Q1, c->N, [&](auto l) { fn = decltype(l)::persistent(c); });
    LatticeConst L = c->L;
    StepArgs Ac = A;
    float* fa = f_a;
    float* fb = f_b;
    int nb = c->n_blocks;
    int ns = n_steps;
    FlowArgs F{c->d_nbr, c->d_done, c->flow_spin_limit, c->flow_skew};
    void* args[] = {&L, &Ac, &fa, &fb, &nb, &ns, &F};
    if (hipLaunchCooperativeKernel(fn, dim3(c->persistent_grid), dim3(c->block), args, 0, s) != hipSuccess)
      return LBSMRT_E_HIP;
    return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
  }
  if (c->mode == LBSMRT_LAUNCH_GRAPH && n_steps >= 2 * c->graph_pairs) {
    if (!c->graph || c->graph_a != f_a || c->graph_b != f_b) {
      if (c->graph) (void)hipGraphExecDestroy(c->graph);
      c->graph = nullptr;
      const bool ok = capture_steps(2 * c->graph_pairs, &c->graph, [&](int t, hipStream_t cs) {
        const float* src = (t & 1) ? f_b : f_a;
        float* dst = (t & 1) ? f_a : f_b;
        dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::step(c, A, src, dst, cs); });
      });
      if (!ok) { drop_graph(c); return LBSMRT_E_HIP; }
      c->graph_a = f_a;
      c->graph_b = f_b;
    }
    const int per = 2 * c->graph_pairs;
    const int reps = n_steps / per;
    for (int r = 0; r < reps; ++r)
      if (hipGraphLaunch(c->graph, s) != hipSuccess) return LBSMRT_E_HIP;
    direct(0, n_steps - reps * per);   // an even number of steps has returned the state to f_a
    return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
  }
  direct(0, n_steps);
  return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
}

lbsmrt_status lbsmrt_set_launch(lbsmrt_ctx* c, int mode, int block_size, int graph_steps, int lanes_per_node) {
  if (!c) return LBSMRT_E_ARG;
  if (mode != LBSMRT_LAUNCH_DIRECT && mode != LBSMRT_LAUNCH_GRAPH && mode != LBSMRT_LAUNCH_PERSISTENT)
    return LBSMRT_E_ARG;
  if (block_size != 0 && block_size != 64 && block_size != 128 && block_size != 256) return LBSMRT_E_ARG;
  if (mode == LBSMRT_LAUNCH_GRAPH && (graph_steps < 2 || graph_steps > 4096 || (graph_steps & 1)))
    return LBSMRT_E_ARG;
  if (lanes_per_node != 0 && lanes_per_node != 1 && lanes_per_node != 2 && lanes_per_node != 4 && lanes_per_node != 8 &&
      lanes_per_node != 16)
    return LBSMRT_E_ARG;
  if (lanes_per_node > 1 && !c->lpn4_ok) return LBSMRT_E_UNSUPPORTED;
  if (mode == LBSMRT_LAUNCH_PERSISTENT && (c->additive || c->Q1 > 9 || c->precision == LBSMRT_SPLIT_BF16X3 ||
                                           (lanes_per_node != 0 ? lanes_per_node : c->lpn) == 16))
    return LBSMRT_E_UNSUPPORTED;
  if (c->precision == LBSMRT_SPLIT_BF16X3 && block_size != 0 && block_size != 256) return LBSMRT_E_UNSUPPORTED;
  if (hipSetDevice(c->device) != hipSuccess) return LBSMRT_E_HIP;
  drop_graph(c);
  const int bs = block_size != 0 ? block_size : c->block;
  const int lpn = lanes_per_node != 0 ? lanes_per_node : c->lpn;
  if (bs != c->block || lpn != c->lpn) {
    std::vector<BlockDev> bl = block_table(c->doms, bs / lpn);
    BlockDev* nb = nullptr;
    if (hipMalloc(&nb, sizeof(BlockDev) * bl.size()) != hipSuccess) return LBSMRT_E_NOMEM;
    if (hipMemcpy(nb, bl.data(), sizeof(BlockDev) * bl.size(), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(nb);
      return LBSMRT_E_HIP;
    }
    (void)hipFree(c->d_blocks);
    c->d_blocks = nb;
    c->n_blocks = static_cast<int>(bl.size());
    c->block = bs;
    c->lpn = lpn;
  }
  if (mode == LBSMRT_LAUNCH_PERSISTENT) {
    bool lines = true;
    for (const lbsmrt_domain& d : c->doms) lines = lines && d.ny == 1 && d.nz == 1;
    c->flow = lines && build_flow(c);
    const void* fn = nullptr;
    dispatch(c->Q1, c->N, [&](auto l) { fn = decltype(l)::persistent(c); });
    int per_cu = 0, cus = 0;
    if (!fn) return LBSMRT_E_UNSUPPORTED;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, c->block, 0) != hipSuccess) return LBSMRT_E_HIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
      return LBSMRT_E_HIP;
    if (per_cu < 1) return LBSMRT_E_UNSUPPORTED;
    c->persistent_grid = std::min(c->n_blocks, per_cu * cus);
  }
  c->graph_pairs = mode == LBSMRT_LAUNCH_GRAPH ? graph_steps / 2 : 0;
  c->mode = mode;
  return LBSMRT_OK;
}

lbsmrt_status lbsmrt_test_flow_wait(lbsmrt_ctx* c, unsigned spin_limit, unsigned skew) {
  if (!c || spin_limit == 0) return LBSMRT_E_ARG;
  c->flow_spin_limit = spin_limit;
  c->flow_skew = skew;
  return LBSMRT_OK;
}

lbsmrt_status lbsmrt_get_launch(const lbsmrt_ctx* c, int* mode, int* block_size, int* lanes_per_node) {
  if (!c) return LBSMRT_E_ARG;
  if (mode) *mode = c->mode;
  if (block_size) *block_size = c->block;
  if (lanes_per_node) *lanes_per_node = c->lpn;
  return LBSMRT_OK;
}

int lbsmrt_moment_rows(const lbsmrt_ctx* c, unsigned mask) {
  if (!c) return -1;
  int rows = 0;
  if (mask & LBSMRT_MOM_BASIC) rows += 5;
  if (mask & LBSMRT_MOM_SIGMA) rows += 6;
  if (mask & LBSMRT_MOM_Q) rows += 3;
  if (mask & LBSMRT_MOM_M3) rows += 10;
  if (c->N >= 4) {
    if (mask & LBSMRT_MOM_R41) rows += 6;
    if (mask & LBSMRT_MOM_R42) rows += 1;
  }
  if (mask & LBSMRT_MOM_DLOCAL) rows += c->M;
  if (mask & LBSMRT_MOM_ALAB) rows += c->M;
  return rows;
}

lbsmrt_status lbsmrt_moments(lbsmrt_ctx* c, const float* f, double* out, unsigned mask, void* stream) {
  if (!c || !f || !out || mask == 0 || (mask & ~0xFFu)) return LBSMRT_E_ARG;
  if (c->N < 4 && (mask & (LBSMRT_MOM_R41 | LBSMRT_MOM_R42))) return LBSMRT_E_ARG;
  if (c->N < 3 && (mask & (LBSMRT_MOM_Q | LBSMRT_MOM_M3))) return LBSMRT_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const StepArgs A = step_args(c);
  dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::moments(c, A, f, out, mask, s); });
  return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
}

lbsmrt_status lbsmrt_equilibrium(lbsmrt_ctx* c, const double* fields, float* f, void* stream) {
  if (!c || !fields || !f) return LBSMRT_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::equilibrium(c, fields, c->n_nodes, f, c->stride, s); });
  return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
}

lbsmrt_status lbsmrt_step_adjoint(lbsmrt_ctx* c, const float* f_t, const float* lam_next, float* lam_t,
                                  double* dL_dtau, void* stream) {
  const lbsmrt_status st = adjoint_check(c, f_t, lam_next, lam_t, dL_dtau);
  if (st != LBSMRT_OK) return st;
  return adjoint_launch(c, f_t, lam_next, lam_t, dL_dtau, c->d_partial, c->d_stage, stream);
}

lbsmrt_status lbsmrt_step_adjoint_noalloc(lbsmrt_ctx* c, const float* f_t, const float* lam_next, float* lam_t,
                                          double* dL_dtau, void* stream) {
  const lbsmrt_status st = adjoint_check(c, f_t, lam_next, lam_t, dL_dtau);
  if (st != LBSMRT_OK) return st;
  const size_t cols = static_cast<size_t>(n_tau_slots(c->N));
  if (cols * (static_cast<size_t>(adjoint_groups(c)) + kReduceBlocks) > kScratchDoubles) return LBSMRT_E_LIMIT;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBSMRT_E_HIP;
  if (dev != c->device) return LBSMRT_E_ARG;   // the context's device must be current
  double* base = scratch_address(dev);
  if (!base) return LBSMRT_E_UNSUPPORTED;   // device ordinal beyond the lookup table
  // partials first, then the stage rows; every row the reduction reads is written by this call
  return adjoint_launch(c, f_t, lam_next, lam_t, dL_dtau, base, base + cols * adjoint_groups(c), stream);
}

lbsmrt_status lbsmrt_loss_seed(lbsmrt_ctx* c, const float* f, const double* target, const double* scales, float* lam,
                               double* loss, void* stream) {
  if (!c || !f || !target || !scales || !lam || !loss || lam == f) return LBSMRT_E_ARG;
  if (c->Q1 > 9) return LBSMRT_E_UNSUPPORTED;   // no kernel for the 17-point stencil
  hipStream_t s = static_cast<hipStream_t>(stream);
  StepArgs A = step_args(c);
  A.blocks = c->d_blocks_adj;
  dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::loss_seed(c, A, f, target, scales, lam, s); });
  hipLaunchKernelGGL(k_reduce_stage1, dim3(kReduceBlocks), dim3(256), 0, s, c->d_partial, c->n_blocks_adj, 1,
                     c->d_stage);
  hipLaunchKernelGGL(k_reduce_loss, dim3(1), dim3(kReduceBlocks), 0, s, c->d_stage, loss, 0);
  return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
}

lbsmrt_status lbsmrt_set_tau(lbsmrt_ctx* c, const double* tau) {
  if (!c || !tau) return LBSMRT_E_ARG;
  for (int n = 2; n <= c->N; ++n)
    for (int m = 0; 2 * m <= n; ++m) {
      if (n == 2 && m == 1) continue;
      const double t = tau[n * 3 + m];
      if (!(t > 0.0) || !std::isfinite(t)) return LBSMRT_E_ARG;
    }
  for (int n = 2; n <= c->N; ++n)
    for (int m = 0; 2 * m <= n; ++m)
      if (!(n == 2 && m == 1)) c->L.tau[n][m] = tau[n * 3 + m];
  drop_graph(c);   // captured launches hold the old relaxation times
  return LBSMRT_OK;
}

lbsmrt_status lbsmrt_moment_state_len(const lbsmrt_ctx* c, long long* m_len, long long* work_len) {
  if (!c) return LBSMRT_E_ARG;
  if (m_len) *m_len = static_cast<long long>(c->M) * c->stride;
  if (work_len) *work_len = c->ms_lines ? 0 : 2LL * n_sym(c->N) * (c->N + 1) * c->stride;
  return LBSMRT_OK;
}

lbsmrt_status lbsmrt_equilibrium_moments(lbsmrt_ctx* c, const double* fields, float* m, void* stream) {
  if (!c || !fields || !m) return LBSMRT_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::ms_equilibrium(c, fields, m, s); });
  return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
}

lbsmrt_status lbsmrt_project_state(lbsmrt_ctx* c, const float* f, float* m, void* stream) {
  if (!c || !f || !m) return LBSMRT_E_ARG;
  const size_t fb = sizeof(float) * c->Q * c->stride, mb = sizeof(float) * c->M * c->stride;
  if (overlap(f, fb, m, mb)) return LBSMRT_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::ms_project(c, f, m, s); });
  return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
}

lbsmrt_status lbsmrt_expand_state(lbsmrt_ctx* c, const float* m, float* f, void* stream) {
  if (!c || !f || !m) return LBSMRT_E_ARG;
  const size_t fb = sizeof(float) * c->Q * c->stride, mb = sizeof(float) * c->M * c->stride;
  if (overlap(f, fb, m, mb)) return LBSMRT_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::ms_expand(c, m, f, s); });
  return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
}

lbsmrt_status lbsmrt_step_moment_state(lbsmrt_ctx* c, float* m_a, float* m_b, float* work, int n_steps,
                                       void* stream) {
  if (!c || !m_a || !m_b || n_steps < 1) return LBSMRT_E_ARG;
  if (!c->ms_ok) return LBSMRT_E_UNSUPPORTED;
  if (!c->ms_lines && !work) return LBSMRT_E_ARG;
  const size_t mb = sizeof(float) * c->M * c->stride;
  const size_t half = static_cast<size_t>(n_sym(c->N)) * (c->N + 1) * c->stride;   // floats per intermediate
  if (overlap(m_a, mb, m_b, mb)) return LBSMRT_E_ARG;
  if (!c->ms_lines && (overlap(m_a, mb, work, 2 * half * sizeof(float)) || overlap(m_b, mb, work, 2 * half * sizeof(float))))
    return LBSMRT_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const StepArgs A = step_args(c);
  MsGeom G{};
  if (!c->ms_lines) {
    const lbsmrt_domain& D = c->doms[0];
    G.nx = D.nx; G.ny = D.ny; G.nz = D.nz;
    for (int k = 0; k < 3; ++k) G.k[k] = c->L.k[k];
    G.stride = c->stride;
    G.tsc = D.tau_scale > 0.0 ? D.tau_scale : 1.0;
    G.err = c->d_err;
  }
  float* t1 = work;
  float* t2 = work ? work + half : nullptr;
  // step t of the call: line domains run the x-stage kernel, a periodic box its three passes
  auto one = [&](int t, hipStream_t st) {
    const float* src = (t & 1) ? m_b : m_a;
    float* dst = (t & 1) ? m_a : m_b;
    if (c->ms_lines)
      dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::ms_line_step(c, A, src, dst, st); });
    else
      dispatch(c->Q1, c->N, [&](auto l) { decltype(l)::ms_step(c, G, src, dst, t1, t2, st); });
  };
  int done = 0;
  if (c->mode == LBSMRT_LAUNCH_GRAPH && n_steps >= 2 * c->graph_pairs) {
    // the launch setting's graph mode: 2 graph_pairs steps captured once per (m_a, m_b, work)
    const float* w = c->ms_lines ? nullptr : work;
    if (!c->ms_graph || c->ms_graph_a != m_a || c->ms_graph_b != m_b || c->ms_graph_w != w) {
      if (c->ms_graph) (void)hipGraphExecDestroy(c->ms_graph);
      c->ms_graph = nullptr;
      if (!capture_steps(2 * c->graph_pairs, &c->ms_graph, one)) {
        c->ms_graph = nullptr;
        c->ms_graph_a = c->ms_graph_b = c->ms_graph_w = nullptr;
        return LBSMRT_E_HIP;
      }
      c->ms_graph_a = m_a;
      c->ms_graph_b = m_b;
      c->ms_graph_w = w;
    }
    const int per = 2 * c->graph_pairs;
    const int reps = n_steps / per;
    for (int r = 0; r < reps; ++r)
      if (hipGraphLaunch(c->ms_graph, s) != hipSuccess) return LBSMRT_E_HIP;
    done = reps * per;   // even: the state is back in m_a
  }
  for (int t = done; t < n_steps; ++t) one(t - done, s);
  return hipGetLastError() == hipSuccess ? LBSMRT_OK : LBSMRT_E_HIP;
}

lbsmrt_status lbsmrt_sync_status(lbsmrt_ctx* c, void* stream) {
  if (!c) return LBSMRT_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, c->d_err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h != 0) {
    HIP_TRY(hipMemsetAsync(c->d_err, 0, sizeof(int), s));
    HIP_TRY(hipStreamSynchronize(s));
    return (h & kErrTimeout) ? LBSMRT_E_TIMEOUT : LBSMRT_E_STATE;
  }
  return LBSMRT_OK;
}

void lbsmrt_destroy(lbsmrt_ctx* c) { free_ctx(c); }

}  // extern "C"
