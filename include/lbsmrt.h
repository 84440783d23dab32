/*
 * lbsmrt.h -- C ABI of the MI355X (gfx950) LB-SMRT collide-and-stream library.
 *
 * Method: Yan & Shan, "Lattice Boltzmann simulation of non-equilibrium flows
 * using spectral multiple-relaxation-time collision model" (arXiv 2401.11086).
 * One time step maps the post-collision populations f*_i(x) of every node to
 * the next ones: pull-stream g_i(x) = f*_i(x - s_i) with s_i = e_i + k
 * (Sec. 4.1, shifted stencil), project onto absolute Hermite moments (eq:an),
 * shift them to the local frame (u, theta) by the binomial transform (Sec. 3),
 * split each order n >= 2 into irreducible parts (App. A, eq:IrrDecomp), relax
 * part (n,m) by 1/tau_bar_nm (eq:SMRT), shift back and rebuild
 * f_i = w_i sum_alpha a_alpha He_alpha(c_i) / alpha!  (eq:fi with eq:hermite1's 1/n!).
 *
 * Conventions shared by every call:
 *  - Velocity set: tensor product of a symmetric 1D integer stencil
 *    {0, +-a_1, ..., +-a_p} scaled by the lattice constant c_l (Table 3).
 *    Population index q = (ix*Q1 + iy)*Q1 + iz, where ix, iy, iz index the 1D
 *    integers sorted ascending (-a_p, ..., 0, ..., a_p); Q = Q1^3.
 *  - Hermite multi-indices alpha = (a,b,c), |alpha| <= N, ordered by order n,
 *    then a descending, then b descending; M = (N+1)(N+2)(N+3)/6.
 *  - Nodes: domains are concatenated; inside a domain node = x + nx*(y + ny*z).
 *    Every f / lambda buffer is structure-of-arrays float32 [Q][f_stride]
 *    (f_stride >= total nodes, a multiple of 64), owned by the caller, in
 *    device memory.  Padding entries are never read or written.
 *  - Units: time step 1, velocities in sqrt(k_B T_0), cell size c_l; theta is
 *    the temperature over the reference temperature (validity needs
 *    0 < theta < 2, Sec. 4.1).
 *  - Streams: every call that touches the GPU enqueues its work on `stream`
 *    (a hipStream_t; NULL = the default stream) and returns without waiting,
 *    except lbsmrt_init_lattice and lbsmrt_sync_status, which wait.
 *  - Errors: argument errors are returned synchronously.  A node found outside
 *    the validity region (rho <= 0, theta <= 0, theta >= 2 or non-finite) sets
 *    a device-side flag; it is reported by the next lbsmrt_sync_status.
 *  - Threading: a context may be used from one host thread at a time.
 */
#ifndef LBSMRT_H
#define LBSMRT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbsmrt_ctx lbsmrt_ctx;

typedef enum {
  LBSMRT_OK = 0,
  LBSMRT_E_ARG = 1,          /* bad argument: null pointer, size, unsupported combination */
  LBSMRT_E_QUADRATURE = 2,   /* no real positive-weight rule for the stencil and degree */
  LBSMRT_E_STATE = 3,        /* a node left rho > 0, 0 < theta < 2, or became non-finite */
  LBSMRT_E_HIP = 4,          /* a HIP runtime call failed */
  LBSMRT_E_NOMEM = 5,        /* device or host allocation failed */
  LBSMRT_E_UNSUPPORTED = 6,  /* valid but not built: a (Q1, N) pair with no compiled kernel (built:
                                D1Q7 with N = 3, 4; D1Q9 with N = 4, 5; D1Q17 with N = 5), a
                                configuration the split-BF16x3 form does not take (see
                                lbsmrt_precision), regularized = 0 with FP32 contractions (or with
                                the adjoint, the persistent launch or the moment state), D1Q17 with
                                anything but the forward step, moments, equilibrium, the state
                                conversions and the moment state on line domains, in FP64
                                contractions with the rebuilt collision, or a launch setting the
                                context does not allow */
  LBSMRT_E_LIMIT = 7,        /* the problem exceeds the fixed scratch of an allocation-free entry
                                point (lbsmrt_step_adjoint_noalloc) */
  LBSMRT_E_TIMEOUT = 8       /* a persistent launch on line domains waited for a neighbouring
                                work-group longer than its bound and gave up (the state is then
                                invalid); reported by lbsmrt_sync_status */
} lbsmrt_status;

/* Arithmetic of the projection (eq:an) / rebuild (eq:fi) contractions.  The state f is float32 in
 * every mode; the conserved sums, frame shift, irreducible split and relaxation run in FP64.
 *  LBSMRT_FP32          sum-factorised FP32 contractions; the conserved moments (and the order-2
 *                       trace) are taken in FP64 through weights dual to the float32 rebuild table,
 *                       so a rebuilt node hands its mass, momentum and energy on exactly.
 *  LBSMRT_SPLIT_BF16X3  dense contractions on the matrix cores: each operand split into bf16 halves,
 *                       hi.hi + hi.lo + lo.hi products accumulated in FP32 (v_mfma_f32_32x32x16_bf16);
 *                       orders 0, 1 and the order-2 trace from FP64 sums, and the rebuild corrected
 *                       per node so that its conserved sums are exact.  Stencils D1Q7 {0, +-1, +-2,
 *                       +-3} and D1Q9 {0, +-1, +-2, +-3, +-5} only, the
 *                       rebuilt collision, one lane per node, 256-item work-groups, direct or graph
 *                       launches; every periodic domain needs nx % 32 == 0, and one x-slab of the
 *                       state (Q1^2 f_stride floats) must stay below 4 GiB (E_UNSUPPORTED otherwise).
 *  LBSMRT_FP64_CONTRACT sum-factorised FP64 contractions folded over +-e pairs: the rebuild conserves
 *                       mass, momentum and energy up to the float32 rounding of the stored f. */
typedef enum { LBSMRT_FP32 = 0, LBSMRT_SPLIT_BF16X3 = 1, LBSMRT_FP64_CONTRACT = 2 } lbsmrt_precision;

/* Velocity set and collision model (Sec. 4.2, Tables 3 and 4). */
typedef struct {
  int    n_abscissa;           /* p: number of positive 1D integers (3 for D1Q7, 4 for D1Q9) */
  int    abscissa[16];         /* sorted distinct positive integers, e.g. {1,2,3} or {1,2,3,5} */
  int    degree;               /* degree of exactness of the 1D rule (9 for D1Q7, 11 for D1Q9) */
  int    order_N;              /* Hermite truncation N (3 to 5; see LBSMRT_E_UNSUPPORTED for the pairs) */
  int    shift_k[3];           /* integer frame shift: ubar = c_l * k (Sec. 4.1) */
  double tau[6][3];            /* tau[n][m] in time steps at rho_ref, n = 2..N.  tau[2][1]
                                  is ignored: the (2,1) part vanishes by the definition of theta. */
  double rho_ref;              /* density at which tau[][] holds */
  int    tau_density_scaling;  /* 1: tau_nm(x) = tau_nm * rho_ref / rho(x) (viscosity ~ theta) */
  int    tau_offset_half;      /* 1: tau_bar = tau + 1/2 (trapezoidal discretisation); 0: tau_bar = tau */
  int    regularized;          /* 1: f* rebuilt from the M relaxed moments, f* = R a' (eq:fi, default);
                                  0: additive collision f* = g + R (a' - a), which keeps the part of
                                  the pulled g outside the Hermite span (needs LBSMRT_FP64_CONTRACT;
                                  one lane per node; reads g twice: 12 Q bytes per node-step) */
  int    precision;            /* lbsmrt_precision of the projection/reconstruction contractions */
} lbsmrt_lattice_desc;

/* One domain.  bc_x = 0: periodic in x, y, z.  bc_x = 1: a shock tube whose
 * x ends are held at the truncated Maxwellians of the (rho, u, theta) "in"
 * (left) and "out" (right) states; y and z stay periodic (Sec. 4.2). */
typedef struct {
  int    nx, ny, nz;
  int    bc_x;
  double rho_in, u_in[3], theta_in;     /* lab-frame velocity */
  double rho_out, u_out[3], theta_out;
  double tau_scale;                     /* multiplies every tau_nm in this domain (its own Knudsen
                                           number); 0 means 1 */
} lbsmrt_domain;

/* Sizes of a context, filled by lbsmrt_get_info. */
typedef struct {
  int       Q, Q1, M, N;
  double    c_l;               /* lattice constant r of the 1D rule */
  double    w1d[17];           /* 1D weights in the sorted-ascending order of the stencil */
  int       e1d[17];           /* 1D integers, sorted ascending */
  long long n_nodes;           /* total nodes over all domains */
  long long f_stride;          /* row stride of every [Q][f_stride] buffer */
  long long f_len;             /* Q * f_stride floats per f or lambda buffer */
  int       n_domains;
  long long domain_offset[64]; /* first node of each of the first 64 domains; every domain's
                                  offset is given by lbsmrt_get_domain_offsets */
} lbsmrt_info;

/* Build a context: solve the 1D quadrature (smallest positive-weight root),
 * build Hermite and relaxation tables, upload them and the ghost-state
 * equilibria of shock domains.  Waits for its own work on `stream`.
 * Ownership: the context owns its device tables until lbsmrt_destroy.
 * Errors: E_ARG (bad sizes, N outside 2..5, n_dom outside 1..4096),
 * E_QUADRATURE, E_UNSUPPORTED (no kernel for this Q1 and N), E_HIP, E_NOMEM. */
lbsmrt_status lbsmrt_init_lattice(const lbsmrt_lattice_desc* desc, const lbsmrt_domain* domains,
                                  int n_domains, void* stream, lbsmrt_ctx** out);

lbsmrt_status lbsmrt_get_info(const lbsmrt_ctx* ctx, lbsmrt_info* out);

/* First node of every domain, in the order the domains were given to lbsmrt_init_lattice
 * (domains are concatenated in node space, each x fastest).  out: host array of `capacity`
 * entries, filled with min(capacity, n_domains) offsets; *n_written (may be NULL) receives
 * that count.  E_ARG for a NULL ctx or out, or capacity < 1. */
lbsmrt_status lbsmrt_get_domain_offsets(const lbsmrt_ctx* ctx, long long* out, int capacity, int* n_written);

/* How lbsmrt_step issues its work (lbsmrt_set_launch):
 *  LBSMRT_LAUNCH_DIRECT      one kernel launch per step over all domains (default);
 *  LBSMRT_LAUNCH_GRAPH       replays a captured hipGraph of `graph_steps` launches (even), captured on
 *                            first use for a given (f_a, f_b) pair and recaptured when the pair, the
 *                            launch settings or the relaxation times change;
 *  LBSMRT_LAUNCH_PERSISTENT  one cooperative launch running all steps, work-groups resident and
 *                            striding over the node blocks.  When every domain is a line (ny = nz
 *                            = 1) a block starts step t as soon as the blocks it pulls from have
 *                            completed step t - 1 (per-block progress counters, each wait bounded:
 *                            LBSMRT_E_TIMEOUT if one gives up); otherwise, or when a block holds
 *                            fewer nodes than the pull reach max |e_j + k_x| (or a periodic line
 *                            of more than three blocks ends in such a block), a grid-wide barrier
 *                            separates the steps.  Results are the same either way. */
enum { LBSMRT_LAUNCH_DIRECT = 0, LBSMRT_LAUNCH_GRAPH = 1, LBSMRT_LAUNCH_PERSISTENT = 2 };

/* Choose the launch mode, the work-group size (64, 128 or 256 work-items; 0 keeps the current
 * one) and the lanes per node of the step kernel (1, 2, 4, 8 or 16; 0 keeps the current one).  With
 * L > 1 lanes, a group of L consecutive work-items shares each node: each gathers and stores every
 * L-th x-slab of the node's populations and the group sums its moments before the (replicated)
 * collision, so a work-group of B work-items updates B/L nodes.  That shortens each wavefront's
 * serial work when a context has few nodes (single shock tubes).  Results do not depend on the
 * mode or the work-group size; lanes_per_node > 1 changes the order of the FP64 projection sums
 * (results agree with 1 to FP64 rounding before the FP32 store).  The adjoint step uses the
 * same split when lanes_per_node is 4, 8 or 16 and one lane per node otherwise.  Synchronous.
 * E_ARG for an unknown mode, size, lanes_per_node or odd graph_steps; E_UNSUPPORTED for
 * lanes_per_node > 1 unless the context has shock domains, LBSMRT_FP64_CONTRACT and a state
 * below 4 GiB (Q * f_stride * 4 bytes) and the rebuilt collision, for the persistent mode of an
 * additive-collision context or with sixteen lanes per node, or if the persistent kernel cannot
 * be made resident.
 * A new context starts in direct mode with work-groups of 256 (64 if no domain reaches 4096
 * nodes) and one lane per node; an eligible context with at most 8192 nodes starts with eight
 * (sixteen up to 4096 nodes for D1Q9 and D1Q17), one with at most 16384 nodes with four. */
lbsmrt_status lbsmrt_set_launch(lbsmrt_ctx* ctx, int mode, int block_size, int graph_steps, int lanes_per_node);

/* Test hook of the persistent launch's bounded waits on line domains: polls before a wait gives
 * up (default 4194304, each poll followed by a short sleep) and a skew added to every wait's
 * target step (0 by default; a large skew makes every wait unreachable, so that the give-up path,
 * LBSMRT_E_TIMEOUT, can be exercised without a stalled work-group).  Takes effect at the next
 * launch.  E_ARG for a NULL ctx or spin_limit 0. */
lbsmrt_status lbsmrt_test_flow_wait(lbsmrt_ctx* ctx, unsigned spin_limit, unsigned skew);

/* The current launch settings (any output pointer may be NULL).  E_ARG for a NULL ctx. */
lbsmrt_status lbsmrt_get_launch(const lbsmrt_ctx* ctx, int* mode, int* block_size, int* lanes_per_node);

/* Advance n_steps >= 1 time steps (Sec. 3-4: stream, then SMRT collision).
 * Step t reads buffer A if t is even, B if odd, and writes the other one, so
 * after n_steps the state is in f_a if n_steps is even and in f_b if odd.
 * f_a != f_b, both [Q][f_stride] float32 device buffers.  Asynchronous. */
lbsmrt_status lbsmrt_step(lbsmrt_ctx* ctx, float* f_a, float* f_b, int n_steps, void* stream);

/* Moment fields of the pre-collision populations of state f (stream first),
 * the quantities plotted in Sec. 4.3.  out is float64 [rows][n_nodes] in
 * device memory; the rows of each selected group follow in bit order:
 *   LBSMRT_MOM_BASIC  5 rows: rho, u_x, u_y, u_z (lab frame), theta
 *   LBSMRT_MOM_SIGMA  6 rows: sigma = theta d^(2), components xx,xy,xz,yy,yz,zz
 *   LBSMRT_MOM_Q      3 rows: q = theta^(3/2)/2 tr d^(3)
 *   LBSMRT_MOM_M3    10 rows: m = d^(3,0)/D(3,0) in multi-index order
 *   LBSMRT_MOM_R41    6 rows: R^(4,1) = d^(4,1)/D(4,1) (needs N >= 4)
 *   LBSMRT_MOM_R42    1 row : R^(4,2) = d^(4,2)/D(4,2) (needs N >= 4)
 *   LBSMRT_MOM_DLOCAL M rows: local-frame moments d_beta (rho absorbed)
 *   LBSMRT_MOM_ALAB   M rows: lattice-frame moments a_alpha (eq:an)
 * lbsmrt_moment_rows gives the row count of a mask.  Asynchronous. */
enum {
  LBSMRT_MOM_BASIC = 1u, LBSMRT_MOM_SIGMA = 2u, LBSMRT_MOM_Q = 4u, LBSMRT_MOM_M3 = 8u,
  LBSMRT_MOM_R41 = 16u, LBSMRT_MOM_R42 = 32u, LBSMRT_MOM_DLOCAL = 64u, LBSMRT_MOM_ALAB = 128u
};
lbsmrt_status lbsmrt_moments(lbsmrt_ctx* ctx, const float* f, double* out, unsigned fields_mask,
                             void* stream);
int lbsmrt_moment_rows(const lbsmrt_ctx* ctx, unsigned fields_mask);

/* Truncated discrete Maxwellian f_i = w_i sum_alpha a^eq_alpha He_alpha(c_i)/alpha!
 * with a^eq_alpha = rho prod_k A_{alpha_k}(u_k - ubar_k, theta) (App. B closed form).
 * fields: float64 [5][n_nodes] device rows rho, u_x, u_y, u_z (lab frame), theta.
 * f: [Q][f_stride] float32 device buffer written for every node.  Asynchronous. */
lbsmrt_status lbsmrt_equilibrium(lbsmrt_ctx* ctx, const double* fields, float* f, void* stream);

/* Adjoint of one step f_{t+1} = Step(f_t; tau) (reverse mode of the same
 * stream + collision).  Given lam_next = dL/df_{t+1} it writes
 * lam_t = (df_{t+1}/df_t)^T lam_next and adds (d f_{t+1}/d tau_nm)^T lam_next
 * to dL_dtau[n][m] (float64 [6][3] in device memory, accumulated, fixed
 * summation order so results are reproducible).  f_t, lam_next, lam_t are
 * [Q][f_stride] float32 device buffers; lam_t must not alias the others.
 * E_UNSUPPORTED for an additive-collision context (regularized = 0).  Asynchronous. */
lbsmrt_status lbsmrt_step_adjoint(lbsmrt_ctx* ctx, const float* f_t, const float* lam_next,
                                  float* lam_t, double* dL_dtau, void* stream);

/* lbsmrt_step_adjoint without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, results and summation order as lbsmrt_step_adjoint (bit-identical lam_t and
 * dL_dtau increment); the dL/dtau reduction partials go to a fixed 8 MiB device array of the
 * library (one per GPU, held until the process ends) instead of the context's buffers.  It calls
 * no hipMalloc, hipFree or allocating library routine.
 * Limit: n_tau_slots * (G + 256) doubles <= 2^20, where n_tau_slots = 3, 6, 9 for N = 3, 4, 5 and
 * G is the adjoint's work-group count (nodes / 256 on periodic domains with N <= 4, else
 * nodes / 64 at one lane per node, nodes / 16 and nodes / 8 at four and eight lanes, each domain
 * rounded up): about 44 million nodes for a periodic box with N = 4 (256^3 fits) and 7.4 million
 * for N = 5.
 * Larger contexts get E_LIMIT.  The context's device must be the current device (else E_ARG).
 * Every call on one GPU shares the array, so calls that overlap on that GPU (other streams,
 * other threads, other contexts) race: serialise them.  Nothing in the array needs to start at
 * zero; each call writes every entry it reads.  Asynchronous. */
lbsmrt_status lbsmrt_step_adjoint_noalloc(lbsmrt_ctx* ctx, const float* f_t, const float* lam_next,
                                          float* lam_t, double* dL_dtau, void* stream);

/* Seed of the adjoint for the shock-profile misfit
 *   L = sum_x [ s_rho^2 (rho - rho*)^2 + s_theta^2 (theta - theta*)^2 + s_q^2 (q_x - q_x*)^2 ]
 * of the pre-collision moments of state f.  target: float64 [3][n_nodes] device
 * rows rho*, theta*, q_x*; scales: host [3].  Writes lam = dL/df ([Q][f_stride])
 * and L into *loss (float64, device).  Asynchronous. */
lbsmrt_status lbsmrt_loss_seed(lbsmrt_ctx* ctx, const float* f, const double* target,
                               const double* scales, float* lam, double* loss, void* stream);

/* Replace the relaxation times: tau[n*3 + m] = tau_nm at rho_ref for n = 2..N (the (2,1)
 * entry is ignored), as in lbsmrt_lattice_desc.tau.  Host-side; takes effect for work
 * enqueued afterwards.  E_ARG if an entry is not positive and finite. */
lbsmrt_status lbsmrt_set_tau(lbsmrt_ctx* ctx, const double* tau);

/* ---- moment-state form ---------------------------------------------------
 * With the regularised rebuild (eq:fi) the post-collision populations of a node are
 * f*_i = w_i sum_alpha a'_alpha He_alpha(c_i)/alpha!, fixed by its M moments a'.  A context
 * can therefore hold its state as the moments instead: m is float32 [M][f_stride] (moment
 * order of lbsmrt_moments' LBSMRT_MOM_ALAB rows: by order n, then a, then b descending).
 * lbsmrt_step_moment_state advances it by the same step as lbsmrt_step (pull stream, eq:an
 * projection, SMRT collision), written as a separable convolution of the moment fields
 * along z, y and x; the state moves M floats per node instead of Q.  On line domains
 * (ny = nz = 1: shock tubes, rings) the y and z stages are the identity, because the
 * quadrature is exact to degree 2N, and the step is the x-stage alone, with the moments of
 * the fixed end states as ghosts.  The taps run in FP64 with FP64 tables (each +-e pair of
 * sources folded in float32), so mass, momentum and energy are conserved up to the float32
 * rounding of m.  Results agree with lbsmrt_step on the expanded state up to float32 rounding
 * of m instead of f. */

/* Sizes of the moment-state buffers in floats: m_len = M * f_stride (one state) and
 * work_len (scratch of lbsmrt_step_moment_state, 2 (N+1)^2 (N+2)/2 rows of f_stride; 0 when
 * every domain is a line).
 * Either pointer may be NULL.  E_ARG for a NULL ctx. */
lbsmrt_status lbsmrt_moment_state_len(const lbsmrt_ctx* ctx, long long* m_len, long long* work_len);

/* Moments a^eq of the truncated Maxwellian (as lbsmrt_equilibrium) written to m.
 * fields: float64 [5][n_nodes] device rows; m: [M][f_stride] float32.  Any context.  Asynchronous. */
lbsmrt_status lbsmrt_equilibrium_moments(lbsmrt_ctx* ctx, const double* fields, float* m, void* stream);

/* Own-node projection m_alpha = sum_i f_i He_alpha(c_i) (eq:an without the stream; FP64
 * sums, stored as float32).  For a post-collision state this recovers a'.  Any context;
 * f and m must not overlap.  Asynchronous. */
lbsmrt_status lbsmrt_project_state(lbsmrt_ctx* ctx, const float* f, float* m, void* stream);

/* Rebuild f_i = w_i sum_alpha m_alpha He_alpha(c_i)/alpha! (eq:fi) for every node, giving
 * the population state that lbsmrt_step, lbsmrt_moments and lbsmrt_step_adjoint take.
 * Any context; f and m must not overlap.  Asynchronous. */
lbsmrt_status lbsmrt_expand_state(lbsmrt_ctx* ctx, const float* m, float* f, void* stream);

/* Advance a moment state n_steps >= 1 steps; buffers alternate as in lbsmrt_step (result in
 * m_a for even n_steps, in m_b for odd).  work: lbsmrt_moment_state_len's work_len floats of
 * caller-owned device memory, contents irrelevant (unused, may be NULL, when every domain is a
 * line); none of m_a, m_b, work may overlap.  E_UNSUPPORTED unless the context has exactly one
 * periodic domain (bc_x = 0) or only line domains (ny = nz = 1, any bc_x, any number), the
 * rebuilt collision, and the stencil D1Q7 {0, +-1, +-2, +-3} or D1Q9 {0, +-1, +-2, +-3, +-5}, or
 * on line domains D1Q17 {0, +-1..+-7, +-9} (Table 3's Ma 7 set).
 * The context's launch setting applies: in LBSMRT_LAUNCH_GRAPH mode `graph_steps` steps are
 * captured once per (m_a, m_b, work) and replayed (recaptured when any of them, the launch
 * settings or the relaxation times change); lanes_per_node >= 4 runs line domains with eight
 * lanes per node (sixteen for D1Q17: one tap pair per lane); the persistent mode launches
 * directly.  E_HIP if a capture fails.
 * Validity failures latch the flag read by lbsmrt_sync_status.  Asynchronous. */
lbsmrt_status lbsmrt_step_moment_state(lbsmrt_ctx* ctx, float* m_a, float* m_b, float* work, int n_steps,
                                       void* stream);

/* Wait for `stream` and report (and clear) the latched device state flag. */
lbsmrt_status lbsmrt_sync_status(lbsmrt_ctx* ctx, void* stream);

/* Free the context's device tables and the context (NULL is a no-op).  Call it while the HIP
 * runtime is alive: not from process-exit handlers that run after the runtime (or a profiler
 * attached to it) has shut down.  The caller's buffers are untouched. */
void lbsmrt_destroy(lbsmrt_ctx* ctx);
const char* lbsmrt_status_string(lbsmrt_status s);

/* ---- host-only helpers (no GPU) --------------------------------------- */

/* 1D rule r*{0, +-a_1..a_p} exact to `degree` for the unit Gaussian: writes
 * r and the p+1 weights (w_0, w_{a_1}, ..., w_{a_p}).  Smallest positive-weight
 * root (Table 3), solved in binary128 and rounded to double (the same bits on every host).
 * E_QUADRATURE if none exists, E_ARG on bad input. */
lbsmrt_status lbsmrt_solve_quadrature(int n_abscissa, const int* abscissa, int degree,
                                      double* r_out, double* w_out);

/* Normal-shock end states (eq:rankine, temperature ratio with Ma^2 in the
 * denominator, which is what reproduces Table 3), rho1 = 1.  Pass theta1 > 0,
 * or theta1 <= 0 and theta2 > 0.  out[8] = rho1, u1, theta1, rho2, u2, theta2,
 * (u1+u2)/2, and k = round(((u1+u2)/2)/c_l) as a double (if c_l > 0). */
lbsmrt_status lbsmrt_shock_states(double Ma, double gamma, double theta1, double theta2,
                                  double c_l, double* out);

#ifdef __cplusplus
}
#endif
#endif /* LBSMRT_H */
