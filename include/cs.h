/*
 * cs.h - contingency screening on one MI355X (gfx950).
 *
 * The per-contingency evaluation loop of "High-performance computing enabled
 * contingency analysis for modern power networks" (arXiv 2512.08465):
 *
 *   Section II.A   every N-1 and N-2 outage of lines, transformers and
 *                  generators (the list is the caller's; loads may be
 *                  outaged too);
 *   Section II.B.3 islanding check: connected subgraphs after the outage,
 *                  more than one is severe; the island with the largest
 *                  generation is solved;
 *   Section II.B.1 AC optimal power flow on that island: non-convergence or a
 *                  limit violation is severe.  Solved by a primal-dual
 *                  interior-point method, one dense LU-factorised KKT system
 *                  per Newton step;
 *   Section II.B.2 linearised state matrix at the OPF point and its full
 *                  eigenspectrum: an eigenvalue with non-negative real part is
 *                  severe; the minimum damping ratio is reported;
 *   Section II.C   eq. (1)-(3): F_i = lambda_i, F_ij = lambda_i lambda_j,
 *                  R_i = F_i S_i + sum_j F_ij S_ij over the list.
 *
 * Conventions
 *   - Every call returns an int status: CS_OK (0) or a negative CS_E* code.
 *     The message of the last failure on the calling thread is returned by
 *     cs_last_error().  Validation failures reject the whole call and write no
 *     output.  Islanding, OPF failure and instability are results, not errors.
 *   - Per-unit quantities on base_mva; angles in radians; times in seconds.
 *   - Component ids: [0, n_branch) branches, then [n_branch, n_branch+n_gen)
 *     generators, then loads.  An outage row (i, j) outages i and j; j = -1
 *     marks an N-1 outage, and (-1, -1) is the base case with nothing out
 *     (the reference operating point of Section II.A).
 *   - Buffers passed in are owned by the caller and only read during the call
 *     (cs_net_create copies the network to the device).
 *   - All device work runs on one HIP device chosen at cs_ctx_create.
 */
#ifndef CS_H
#define CS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CS_ABI_VERSION 10

enum {
  CS_OK = 0,
  CS_EINVAL = -1,   /* invalid argument (message names it)                   */
  CS_ENOMEM = -2,   /* host or device allocation failed                        */
  CS_EHBM = -3,     /* one scenario's workspace exceeds the HBM budget         */
  CS_EDEVICE = -4,  /* HIP runtime error                                       */
  CS_EUNSUPPORTED = -5, /* a model or size the library does not support      */
  CS_EAGAIN = -6,       /* serving: no room for the request right now          */
  CS_ETIMEDOUT = -7     /* serving: the request is not complete yet            */
};

/* CS_PREC_FP64: every step in FP64.  CS_PREC_MIXED: the KKT systems are
 * factorised in FP32 on the matrix cores and each Newton step refined in FP64
 * to the backward error of an FP64 solve (FP64 factorisation when that is not
 * reached); everything else, the state matrix and the eigenvalues included,
 * stays FP64. */
enum { CS_PREC_FP64 = 0, CS_PREC_MIXED = 1 };

/* cause bits of cs_result.cause (severity criteria of Section II.B) */
enum {
  CS_CAUSE_ISLAND = 1,      /* more than one island after the outage          */
  CS_CAUSE_OPF = 2,         /* OPF not converged (or not solvable)            */
  CS_CAUSE_LIMIT = 4,       /* converged OPF violates a limit by > 1e-6 p.u.  */
  CS_CAUSE_SSS = 8,         /* an eigenvalue with Re >= 0                     */
  CS_CAUSE_NUMERICAL = 16,  /* singular/non-finite KKT, divergence, QR failure */
  CS_CAUSE_PRUNED = 32      /* N-3 row taken as severe because a screened
                               sub-scenario is severe (cs_screen_n3_device) */
};

/* cs_result.opf_status */
enum { CS_OPF_CONVERGED = 0, CS_OPF_MAXIT = 1, CS_OPF_NUMERICAL = 2, CS_OPF_NOT_RUN = 3 };

/* cs_result.near: the decision lies close to a threshold (set only for a
 * converged OPF) */
enum { CS_NEAR_SSS = 1   /* |max Re| <= near_eps                              */,
       CS_NEAR_OPF = 2   /* converged with iters >= max_it - 2                */,
       CS_NEAR_LIMIT = 4 /* 1e-7 < max violation <= 1e-5: a decade either side
                            of the 1e-6 p.u. limit test                      */ };

/* dyn row of a synchronous generator (kind 0): H D Xd Xq Xd' Xq' Td0' Tq0' Rs
 * KA TA R Tg Tt (two-axis machine, first-order AVR, governor and turbine);
 * of a grid-following converter (kind 1): Kpp Kip Kpc Kic Lf Rf Cdc Kpdc Kidc
 * Vdc0 and 4 unused entries (PLL PI, current PI with an L filter, DC link
 * with a DC-voltage PI).  System base. */
#define CS_N_DYN 14

/* Network description, host structure-of-arrays (copied at cs_net_create). */
typedef struct {
  int32_t n_bus, n_branch, n_gen, n_load;
  int32_t ref_bus;            /* angle reference bus                          */
  double base_mva;            /* MVA base of the per-unit system (cost scale) */
  double f_hz;                /* nominal frequency                            */
  const double *vmin, *vmax;  /* [n_bus] voltage limits                        */
  const double *gs, *bs;      /* [n_bus] shunt conductance/susceptance         */
  const int32_t *br_from, *br_to;              /* [n_branch] bus ids          */
  const double *br_r, *br_x, *br_b;            /* series r, x; total charging */
  const double *br_rate;      /* rating |S| (p.u.); 0 = unconstrained          */
  const double *br_tap;       /* off-nominal tap on the from side; 0 means 1   */
  const double *br_shift;     /* phase shift (rad)                             */
  const int32_t *gen_bus;     /* [n_gen]                                       */
  const int32_t *gen_kind;    /* 0 synchronous generator, 1 grid-following
                                 converter (NULL: all 0)                     */
  const double *pmin, *pmax, *qmin, *qmax;     /* [n_gen] limits (p.u.)       */
  const double *c2, *c1, *c0; /* cost c2 (Sb P)^2 + c1 (Sb P) + c0, $/h        */
  const double *dyn;          /* [n_gen][CS_N_DYN], system base                */
  const int32_t *load_bus;    /* [n_load]                                      */
  const double *pd, *qd;      /* [n_load] constant power at the OPF stage      */
} cs_net_desc;

typedef struct {
  int32_t prec;        /* CS_PREC_FP64 (default) or CS_PREC_MIXED             */
  int32_t max_it;      /* IPM iteration cap (default 150)                     */
  double tol;          /* IPM termination tolerance (default 1e-8)            */
  double near_eps;     /* |max Re lambda| flagged as near (default 1e-6)      */
  size_t hbm_budget;   /* bytes of scenario workspace; 0 = context default    */
  int32_t batch;       /* scenario slots resident at once (slots are refilled
                          from the list as scenarios finish); 0 = as many as
                          the budget allows, at most the list length        */
  int32_t timing;      /* 1: time every kernel launch with HIP events on its
                          stream and accumulate cs_stats when the call ends  */
  int32_t overlap;     /* 1: the dynamic stage (state matrix, eigenvalues,
                          records) runs on a second stream beside the OPF
                          iterations of other slots, started as soon as the
                          list's OPF tail is smaller than what waits; 2: the
                          same, started at the end of a list only once the
                          OPF tail holds at most two systems per compute
                          unit; 0: one stream (default 0).  Other values:
                          CS_EINVAL.  Records are identical either way.     */
  int32_t refine_steps; /* CS_PREC_MIXED: FP64 refinement steps a Newton solve
                          may take to reach the backward error of an FP64
                          solve before that system is factorised in FP64
                          instead (default 4, 0..100; 0: the FP32 solution is
                          tested as it is)                                   */
  int32_t graph;       /* 0: every Newton step's kernels are launched from the
                          host (default); k = 1..64: the step's kernels
                          (KKT assembly, factorisation and solve, update) are
                          captured once per call into a HIP graph and the
                          graph is replayed k times per scheduling round,
                          between two host synchronisations.  Records are
                          identical either way.  Ignored when timing = 1.    */
  int32_t autotune;    /* 1: launch variants of the large-order LU are chosen
                          by timing them on the device at first use
                          (cs_autotune) and cached per (device, order,
                          precision) for the process; 0: defaults (default) */
} cs_opts;

/* Per-kernel accumulated device time of the calls made with opts.timing = 1
 * since the last cs_stats_reset.  units = matrices or scenarios processed. */
enum { CS_K_TOPOLOGY = 0, CS_K_KKT_ASSEMBLE, CS_K_KKT_LU, CS_K_IPM_UPDATE,
       CS_K_DYN_ASSEMBLE, CS_K_DYN_LU, CS_K_STATE_MATRIX, CS_K_EIG, CS_K_CLASSIFY,
       CS_K_RISK, CS_K_KKT_REFINE, CS_K_KKT_LU64, CS_K_COUNT };
/* CS_K_KKT_LU is the KKT factorisation in the call's precision (FP32 for
 * CS_PREC_MIXED); CS_K_KKT_REFINE the FP64 refinement (with the FP32
 * conversion) and CS_K_KKT_LU64 the FP64 fallback factorisations of the
 * mixed path (units = systems that needed one). */
typedef struct {
  double ms[CS_K_COUNT];          /* summed launch durations                 */
  int64_t launches[CS_K_COUNT];
  int64_t units[CS_K_COUNT];      /* e.g. KKT factorisations performed       */
  int64_t kkt_order;              /* order of the last KKT system factorised */
  int64_t dyn_order;              /* order of the last algebraic system      */
} cs_stats;

/* One record per scenario (48 bytes), the paper's per-scenario record. */
typedef struct {
  uint8_t severe;       /* S_c in {0, 1}                                     */
  uint8_t cause;        /* CS_CAUSE_* bits                                   */
  uint8_t opf_status;   /* CS_OPF_*                                          */
  uint8_t near;         /* CS_NEAR_* bits                                    */
  int16_t n_islands;    /* connected subgraphs after the outage              */
  int16_t opf_iters;    /* Newton steps taken                                */
  int32_t n_states;     /* order of the state matrix (0 if not built)        */
  int32_t reserved;
  double opf_cost;      /* $/h; NaN if the OPF did not run                   */
  double max_real_eig;  /* max Re lambda; NaN if not computed                */
  double min_damping;   /* min damping ratio of oscillatory modes (1 if none) */
  double max_violation; /* largest limit excess (p.u., <= 0 when feasible)   */
} cs_result;

typedef struct cs_ctx cs_ctx;
typedef struct cs_net cs_net;

void cs_opts_default(cs_opts* opts);

/* Create a context on HIP device `device`.  hbm_budget bounds the scenario
 * workspace of each call (0 = 48 GiB).  Errors: CS_EINVAL, CS_EDEVICE. */
int cs_ctx_create(int device, size_t hbm_budget, cs_ctx** out);
void cs_ctx_destroy(cs_ctx* ctx);

/* Validate the network and copy it to the device (Section II.B.3 step 1: the
 * numerical model the outages are applied to).  Errors: CS_EINVAL (sizes,
 * bus ids, self-loops, non-finite values, non-positive time constants or
 * divisor gains), CS_EUNSUPPORTED (another generator kind, more than 1024
 * dynamic states or a network beyond the on-chip working set), CS_ENOMEM,
 * CS_EDEVICE.  The largest state-matrix order of the network is
 * n_a = 7 (machines) + 8 (converters) - 1. */
int cs_net_create(cs_ctx* ctx, const cs_net_desc* desc, cs_net** out);
void cs_net_destroy(cs_net* net);

/* Screen n outages (host buffers).  outages: int32 [n][2]; lambda: failure
 * rates [n_comp] in 1/yr (>= 0, finite); opts may be NULL for defaults.
 * out: [n] records; risk: [n_comp] R_i (may be NULL).  R_i sums eq. (3) over
 * the list as given, in list order.  Errors: CS_EINVAL (component id out of
 * range, i == j, bad lambda), CS_EHBM, CS_ENOMEM, CS_EDEVICE. */
int cs_screen(cs_ctx* ctx, cs_net* net, const int32_t* outages, int64_t n,
              const double* lambda, const cs_opts* opts, cs_result* out,
              double* risk);

/* Same, with device-resident buffers (e.g. from torch) and a HIP stream
 * (NULL = the default stream).  The outage list is validated on the device
 * and an invalid entry fails the call with CS_EINVAL before any result is
 * written.  Returns after the work on `stream` completes. */
int cs_screen_device(cs_ctx* ctx, cs_net* net, const int32_t* d_outages,
                     int64_t n, const double* d_lambda, const cs_opts* opts,
                     cs_result* d_out, double* d_risk, void* stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): cs_screen_device with the scenario
 * workspace in a static device array of CS_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends, instead of
 * the context's workspace.  Same arguments, results and validation as
 * cs_screen_device; as many scenario slots as the array holds (refilled from
 * the list, so any list length works), further capped by opts->batch and
 * opts->hbm_budget.  No device or pinned memory is allocated and nothing is
 * freed.  Errors as cs_screen_device, plus CS_EHBM when one scenario's
 * workspace exceeds half the array (a network too large for it) and
 * CS_EINVAL for opts->timing = 1 (timing allocates).  Every call on one GPU
 * uses that GPU's single array, whatever the context: calls that overlap on
 * one GPU (other threads, other streams) race and must be serialised by the
 * caller. */
#define CS_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int cs_screen_device_noalloc(cs_ctx* ctx, cs_net* net, const int32_t* d_outages,
                             int64_t n, const double* d_lambda, const cs_opts* opts,
                             cs_result* d_out, double* d_risk, void* stream);

/* One scenario in full detail, for parity checks.  Host buffers:
 * vm, va [n_bus] (NaN outside the solved island), pg, qg [n_gen] (NaN when
 * out of service), eig_re, eig_im [n_a] with *n_eig set to the number
 * written, label [n_bus] (island label = smallest bus id of the island).
 * Any pointer except rec may be NULL. */
int cs_detail(cs_ctx* ctx, cs_net* net, const int32_t outage[2],
              const cs_opts* opts, cs_result* rec, double* vm, double* va,
              double* pg, double* qg, double* eig_re, double* eig_im,
              int32_t* n_eig, int32_t* label);

/* Kernel-level entry points (device buffers, for testing the dense kernels
 * alone).  Batched LU with partial pivoting of `batch` row-major n x n
 * matrices followed by the solve of nrhs right-hand sides stored as extra
 * columns: A is [batch][n][lda], lda >= n + nrhs, overwritten by the factors
 * (unit lower L below the diagonal, U on and above, rows in pivoted order)
 * and the solutions.  info[b] = 1 if matrix b hit an exactly zero pivot. */
int cs_dense_solve_batched(const cs_ctx* ctx, double* d_A, int32_t n,
                           int32_t nrhs, int32_t lda, int32_t batch,
                           int32_t* d_info, void* stream);

/* Eigenvalues of `batch` column-major n x n matrices (lda), overwritten by
 * their Hessenberg/Schur work; wr, wi: [batch][n].  info[b] = 1 if QR did
 * not converge.  Allocates a temporary device scratch of 512 n bytes per
 * matrix (the reduction's panel products); CS_ENOMEM if that fails.
 * Section II.B.2: the full eigenspectrum of the state matrix. */
int cs_eigvals_batched(const cs_ctx* ctx, double* d_A, int32_t n, int32_t lda,
                       int32_t batch, double* d_wr, double* d_wi,
                       int32_t* d_info, void* stream);

/* Parity/debug: run the OPF of one scenario for `iters` Newton steps, then
 * evaluate and assemble the KKT system at the point reached (Section II.B.1).
 * Host outputs, each may be NULL: K [nk][nk + 1] row-major (the last
 * column is the right-hand side; layout of the fixed-position KKT: theta,
 * V, Pg, Qg, then P and Q balance multipliers, with identity rows for
 * removed variables), x [2 n_bus + 2 n_gen], lam [2 n_bus],
 * z, mu [2 n_branch + 2 n_bus + 4 n_gen], metrics [8] (feasibility,
 * gradient, complementarity, cost change, barrier, last-pivot-zero flag, cost,
 * Newton steps taken), status (CS_OPF_*; CS_OPF_MAXIT
 * means still iterating), order (= nk). */
int cs_kkt_at(cs_ctx* ctx, cs_net* net, const int32_t outage[2], int32_t iters,
              double* K, double* x, double* lam, double* z, double* mu,
              double* metrics, int32_t* status, int32_t* order);

/* Parity/debug: screen n outages (host buffers, as cs_screen, no risk) and
 * also return every scenario's OPF operating point and spectrum
 * (Section II.B.1-II.B.2): vm, va [n][n_bus] and pg, qg [n][n_gen] (NaN
 * outside the solved island, for generators out of service, and for every
 * entry when the OPF did not run; the point reached is reported also when
 * the OPF did not converge), eig_re, eig_im [n][n_a] (NaN-padded)
 * with n_eig [n] values each (0 unless the OPF converged and the state
 * matrix was formed).  Errors as cs_screen. */
int cs_screen_detail(cs_ctx* ctx, cs_net* net, const int32_t* outages, int64_t n,
                     const cs_opts* opts, cs_result* out, double* vm, double* va,
                     double* pg, double* qg, double* eig_re, double* eig_im,
                     int32_t* n_eig);

/* Parity/debug: the linearised state matrix of Section II.B.2 at a given
 * operating point of one outage's main island, and its eigenvalues.  vm, va
 * [n_bus], pg, qg [n_gen] are host buffers over the whole network; only the
 * island's buses and its in-service generators are read (their values must
 * be finite, vm > 0).  A (may be NULL): [n][n] row-major, n = *n_states =
 * 7 (machines in the island) + 8 (converters) - 1, states per device in
 * ascending generator order, [delta, omega, Eq', Ed', Efd, Psv, Pm] for a
 * machine and [theta_p, x_pll, x_id, x_iq, i_d, i_q, v_dc, x_dc] for a
 * converter, with angles (delta, theta_p) relative to the first device's
 * (its angle state removed).  eig_re, eig_im [n] (may be NULL:
 * no eigenvalues computed).  Errors: CS_EINVAL (bad outage, no island with
 * a generator, non-finite point), CS_EDEVICE (singular algebraic system,
 * non-finite A, QR not converged; A is still written). */
int cs_dyn_at(cs_ctx* ctx, cs_net* net, const int32_t outage[2], const double* vm,
              const double* va, const double* pg, const double* qg, double* A,
              int32_t* n_states, double* eig_re, double* eig_im);

/* Higher-order contingencies (Section VI, N-k with k > 2).  Rows of three
 * ids: (i, j, k) outages three components, (i, j, -1) and (i, -1, -1) are
 * N-2 and N-1 rows, (-1, -1, -1) the base case; ids distinct, -1 only as
 * trailing padding.  Each row is screened exactly as by cs_screen_device
 * (Section II.B criteria on the main island); R_i adds F = lambda_i
 * lambda_j lambda_k for every severe triple containing i (independent
 * failures, as eq. (2)).  Arguments, validation and errors as
 * cs_screen_device with d_outages [n][3]. */
int cs_screen3_device(cs_ctx* ctx, cs_net* net, const int32_t* d_outages, int64_t n,
                      const double* d_lambda, const cs_opts* opts, cs_result* d_out,
                      double* d_risk, void* stream);

/* N-3 screening with pruning (Section V.C: reduce the search space before
 * the full AC evaluation).  A row of d_rows [n][3] is pruned, taken as severe
 * without being solved, when one of its singles or pairs is severe in an
 * already screened N-1/N-2 list (d_sub [n_sub][2] with its records
 * d_sub_rec): more outaged elements are read as never making a severe
 * contingency secure (exact for islanding by branches, the screening
 * assumption for the OPF and stability criteria).  Sub-scenarios absent from
 * the screened list prune nothing.  The other rows are screened as by
 * cs_screen3_device.  d_out [n] records in list order; a pruned row's record
 * has severe 1, cause CS_CAUSE_PRUNED, opf_status CS_OPF_NOT_RUN, n_islands
 * 0 and NaN values.  *n_solved (host, may be NULL) = rows solved.  d_risk
 * [n_comp] (may be NULL) sums F_c S_c over all rows, pruned ones included.
 * Errors as cs_screen3_device. */
int cs_screen_n3_device(cs_ctx* ctx, cs_net* net, const int32_t* d_rows, int64_t n,
                        const int32_t* d_sub, int64_t n_sub, const cs_result* d_sub_rec,
                        const double* d_lambda, const cs_opts* opts, cs_result* d_out,
                        double* d_risk, int64_t* n_solved, void* stream);

/* Risk Index variants over a screened list (Section II.C, eq. (1)-(3), with
 * the extensions Section V.C lists as future work).
 *   severity = CS_SEV_BINARY: S_c is the record's binary severity (eq. (3)).
 *   severity = CS_SEV_DAMPING: non-binary severity from the damping ratio:
 *     a scenario severe by any criterion keeps S_c = 1; a secure one gets
 *     S_c = clip((zeta_ref - min_damping) / zeta_ref, 0, 1).
 *   Common-cause failures: each tagged pair (i, j) adds its common-cause
 *     frequency to the N-2 frequency, F_ij = lambda_i lambda_j + rate(i, j)
 *     (both orders of the pair; a pair tagged twice adds both rates). */
enum { CS_SEV_BINARY = 0, CS_SEV_DAMPING = 1 };
typedef struct {
  int32_t severity;          /* CS_SEV_BINARY (default) or CS_SEV_DAMPING       */
  double zeta_ref;           /* CS_SEV_DAMPING: damping ratio at which a secure
                                scenario's severity reaches 0 (default 0.05, > 0) */
  int64_t n_cc;              /* common-cause pairs (default 0)                  */
  const int32_t* cc_pairs;   /* host [n_cc][2]: distinct valid component ids    */
  const double* cc_rate;     /* host [n_cc]: frequency of the common cause, 1/yr,
                                finite and >= 0                                 */
} cs_risk_opts;
void cs_risk_opts_default(cs_risk_opts* ropts);

/* R_i over a screened list from its records, with the severity and
 * common-cause options above (ropts NULL = binary, independent: the R_i of
 * cs_screen).  Device buffers: d_outages [n][2] and d_records [n] as given
 * to and returned by cs_screen_device, d_lambda [n_comp], d_risk [n_comp]
 * out; stream as cs_screen_device.  Sums run in list order (identical run to
 * run).  Errors: CS_EINVAL (bad row, rate or option), CS_ENOMEM, CS_EDEVICE. */
int cs_risk(cs_ctx* ctx, cs_net* net, const int32_t* d_outages, int64_t n,
            const cs_result* d_records, const double* d_lambda,
            const cs_risk_opts* ropts, double* d_risk, void* stream);

/* Monte-Carlo over the failure rates (Section V.C, uncertainty analysis):
 * R_i for each of n_samples rate vectors d_lambda_samples [n_samples][n_comp]
 * (device, drawn by the caller; finite and >= 0), as
 * R(lambda) = lambda o (S1 + S2 lambda) + C with the list's severities folded
 * into S1 (N-1), the symmetric S2 (N-2) and C (common-cause terms), the
 * product over all samples on the FP64 matrix cores.  Outputs (device, each
 * may be NULL): d_risk [n_samples][n_comp]; d_moments [n_comp][2] mean and
 * sample standard deviation of R_i; d_rank_q [n_comp][3] the 5%, 50% and 95%
 * quantiles of the component's rank over the samples (rank 0 = the largest
 * R; equal R ranked by component id; quantile q = the smallest rank whose
 * cumulative count reaches ceil(q n_samples / 100)).  n_comp <= 16384.
 * Errors as cs_risk. */
int cs_risk_mc(cs_ctx* ctx, cs_net* net, const int32_t* d_outages, int64_t n,
               const cs_result* d_records, const double* d_lambda_samples,
               int64_t n_samples, const cs_risk_opts* ropts, double* d_risk,
               double* d_moments, int32_t* d_rank_q, void* stream);

/* Serving (continuous batching).  A server owns B scenario slots of a
 * network and a host thread that runs them; requests (each an outage list
 * with its own failure rates) are admitted into a device ring of
 * queue_capacity scenarios and their scenarios join the slots as slots free
 * up, beside the work of every other request in flight.  Each scenario's
 * record is computed exactly as by cs_screen; a request's R_i is eq. (3)
 * over its own list.  opts (NULL = defaults) fixes tol, max_it, near_eps,
 * batch (slots) and hbm_budget for all requests; timing is not available.
 * Errors: CS_EHBM (one scenario's workspace exceeds the budget),
 * CS_ENOMEM, CS_EDEVICE.  The server keeps ctx and net in use until
 * destroyed; destroying it waits for the requests in flight. */
typedef struct cs_server cs_server;
typedef struct cs_req cs_req;
int cs_server_create(cs_ctx* ctx, cs_net* net, const cs_opts* opts,
                     int64_t queue_capacity, cs_server** out);
void cs_server_destroy(cs_server* srv);

/* A server for several networks (for instance a 118-bus and a 300-bus grid)
 * under one HBM budget: network i gets the part shares[i] / sum(shares) of
 * the budget (shares NULL = equal parts; each > 0 and finite) as its own
 * scenario slots (capped by opts->batch), its own ring of queue_capacity
 * scenarios and its own streams, fixed for the server's lifetime.  One host
 * thread steps every network's slots in turn, so that their kernels overlap
 * on the device.  Requests name their network (cs_submit_net) and share the
 * table of requests in flight; each record is cs_screen's on that network.
 * n_nets is 1 .. CS_SERVER_MAX_NETS, every network made on ctx's device.
 * Errors: CS_EINVAL, CS_EHBM (a network's part holds no scenario),
 * CS_ENOMEM, CS_EDEVICE.  cs_server_create is this call with one network. */
#define CS_SERVER_MAX_NETS 16
int cs_server_create_multi(cs_ctx* ctx, cs_net* const* nets, int n_nets,
                           const double* shares, const cs_opts* opts,
                           int64_t queue_capacity, cs_server** out);

/* Scenario slots of network net (index into the creation list) in the
 * server, or a negative error code. */
int cs_server_slots(const cs_server* srv, int net);

/* Admit a request: outages [n][2] and lambda [n_comp] (may be NULL: no risk)
 * are host buffers, copied before the call returns.  Returns CS_EAGAIN when
 * the ring or the request table is full right now (retry later), CS_EINVAL
 * on an invalid row or rate, or when n exceeds the ring capacity.  n = 0 is
 * a valid, immediately complete request. */
int cs_submit(cs_server* srv, const int32_t* outages, int64_t n, const double* lambda,
              cs_req** out);

/* As cs_submit, for a snapshot of the network whose loads differ: every
 * load d of the request's scenarios is load_scale[d] times the network's
 * (host [n_load], finite and >= 0, copied before the call returns; NULL =
 * the network's loads).  Records equal cs_screen's on a network created with
 * the scaled loads.  The real-time data stage of the operator tool of
 * Section V.E: each request screens the grid state it was taken at. */
int cs_submit_snapshot(cs_server* srv, const int32_t* outages, int64_t n,
                       const double* lambda, const double* load_scale, cs_req** out);

/* As cs_submit_snapshot for network net of the server (index into the list
 * given to cs_server_create_multi; component ids, n_comp and n_load are that
 * network's).  CS_EINVAL when net is out of range.  cs_submit and
 * cs_submit_snapshot are this call with net = 0. */
int cs_submit_net(cs_server* srv, int net, const int32_t* outages, int64_t n,
                  const double* lambda, const double* load_scale, cs_req** out);

/* Wait up to timeout_us microseconds (< 0: no limit) for a request; then
 * copy its records (out [n]) and R_i (risk [n_comp], if lambda was given;
 * either may be NULL) and its latency in seconds from admission to the last
 * record (may be NULL).  CS_ETIMEDOUT if it is not complete yet. */
int cs_wait(cs_req* req, int64_t timeout_us, cs_result* out, double* risk,
            double* latency_s);

/* Release a request (at any time; an unfinished one is dropped when it
 * completes). */
void cs_req_free(cs_req* req);

/* Autotuning of launch variants.  Times the batched LU's launch variants
 * for order n (one untimed, one timed launch each) on synthetic systems of
 * order n (dense, entries from a counter hash, so that pivoting interchanges
 * rows as on KKT systems; min(batch, 2048) of them up to order 1,024,
 * min(batch, 512) above) in the precision prec names (FP64, or FP32 for
 * CS_PREC_MIXED, the mixed form's main factorisation), keeps the fastest for
 * (ctx's device, n, precision) for the rest of the process and returns it in
 * *choice (may be NULL), with the milliseconds of each timed launch in
 * ms[CS_TUNE_VARIANTS] (may be NULL; entries without a variant NaN).
 * Orders up to 1,024 (the register-resident LU), ms[0..1]:
 *   4, 8          wavefronts per matrix: 256 threads with up to three panel
 *                 rows each (orders up to 768; two matrices per CU in FP64),
 *                 or 512 threads with two.  The factors are the same bits.
 * Orders above 1,024 (the large-order LU), ms[0..4]:
 *   16, 32, 64    right-looking with panels of that width (the trailing
 *                 matrix updated after every panel);
 *   1664, 3264    panels of 16 or 32 columns, left-looking inside groups of
 *                 64 (the trailing matrix updated once per group).
 * opts.autotune = 1 runs it for the KKT order at first use.  Allocates
 * temporary device memory (at most half the context's budget).  Errors:
 * CS_EINVAL, CS_EUNSUPPORTED (n > 4,096), CS_ENOMEM, CS_EDEVICE. */
#define CS_TUNE_VARIANTS 5
int cs_autotune(cs_ctx* ctx, int32_t n, int32_t prec, int32_t batch, int32_t* choice,
                double* ms);

/* Install a choice measured earlier (for instance in another process) for
 * (ctx's device, n, prec): one of the variants above for that order (4 only
 * up to order 768), or 0 to return to the default (up to order 768: 4 in
 * FP64, 8 in FP32; 769 to 1,024: 8; above: 32).  CS_EINVAL for any other
 * value. */
int cs_autotune_set(cs_ctx* ctx, int32_t n, int32_t prec, int32_t choice);

/* Copy / clear the context's kernel timing counters. */
int cs_stats_get(const cs_ctx* ctx, cs_stats* out);
int cs_stats_reset(cs_ctx* ctx);

const char* cs_last_error(void);
int cs_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CS_H */
