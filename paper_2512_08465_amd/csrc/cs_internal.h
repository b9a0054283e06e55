// Internal layouts shared by the HIP kernels and the host runtime.
//
// Device network: structure of arrays, resident for the lifetime of a cs_net.
// Scenario slots: every per-scenario quantity is an array indexed
// [slot * stride + i], so one workgroup per slot reads contiguous data.
//
// KKT layout (fixed positions, independent of the outage):
//   x   = [theta (nb), V (nb), Pg (ng), Qg (ng)]            nx  = 2nb + 2ng
//   lam = [P balance (nb), Q balance (nb)]                 neq = 2nb
//   K is nk x nk, nk = nx + neq, stored row-major (row stride ldk) with one
//   extra column holding the right-hand side and then the solution.  Variables and
//   equations that the outage removes (buses outside the main island, the
//   island's reference angle, generators out of service) become identity
//   rows/columns with a zero right-hand side, so their Newton step is zero.
// Inequalities (fixed positions): [|Sf|^2 (nl), |St|^2 (nl), Vmin (nb),
//   Vmax (nb), Pmin (ng), Pmax (ng), Qmin (ng), Qmax (ng)]; masked entries
//   have z = 1, mu = 0 and take no part in any sum.
// Dynamic algebraic system (same buffer as K after the OPF):
//   y = [Id (ng), Iq (ng), theta (nb), V (nb)], ny = 2ng + 2nb, row-major,
//   followed by 3ng right-hand-side columns: d g / d(delta_j, Eq'_j, Ed'_j).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cs {

constexpr int kDyn = 14;     // H D Xd Xq Xdp Xqp Td0p Tq0p Rs KA TA R Tg Tt
constexpr int kNsSg = 7;     // delta omega Eq' Ed' Efd Psv Pm
constexpr int kNsGfl = 8;    // theta_p x_pll x_id x_iq i_d i_q v_dc x_dc (converter)

// Slot life cycle.  A free slot (EMPTY) is given the next scenario of the
// list (NEW), islanded and set up (IPM), and leaves the interior-point loop
// either converged (DYN) or finished without a dynamic model (DONE).  The
// dynamic stage claims such slots in one step (DYN -> DYNB, DONE -> FIN),
// forms the state matrix (DYNB -> EIG, or FIN on a numerical failure), takes
// the eigenvalues, and writes the record, which frees the slot again.
enum Phase : int {
  PH_EMPTY = 0, PH_IPM = 1, PH_DYN = 2, PH_EIG = 3, PH_DONE = 4,
  PH_NEW = 5, PH_DYNB = 6, PH_FIN = 7, PH_COUNT = 8
};
enum OpfStatus : int { OPF_CONVERGED = 0, OPF_MAXIT = 1, OPF_NUMERICAL = 2, OPF_NOT_RUN = 3 };
enum Cause : int { C_ISLAND = 1, C_OPF = 2, C_LIMIT = 4, C_SSS = 8, C_NUMERICAL = 16 };
enum Near : int { N_SSS = 1, N_OPF = 2, N_LIMIT = 4 };

struct DevNet {
  int nb, nl, ng, nd, ref_bus;
  double base_mva, ws;
  const int* br_f;
  const int* br_t;
  const double* yff_re; const double* yff_im;
  const double* yft_re; const double* yft_im;
  const double* ytf_re; const double* ytf_im;
  const double* ytt_re; const double* ytt_im;
  const double* rate;
  const double* vmin; const double* vmax; const double* gs; const double* bs;
  const int* bus_br_ptr; const int* bus_br;        // incident branches, ascending id
  const int* bus_gen_ptr; const int* bus_gen;      // generators at each bus
  const int* bus_load_ptr; const int* bus_load;    // loads at each bus
  const int* gen_bus;
  const double* pmin; const double* pmax; const double* qmin; const double* qmax;
  const double* c2; const double* c1; const double* c0;
  const int* gen_kind;                             // 0 machine, 1 converter
  const double* dyn;                               // [ng][kDyn]; a converter's row:
                                                   // Kpp Kip Kpc Kic Lf Rf Cdc Kpdc
                                                   // Kidc Vdc0
  const int* load_bus; const double* pd; const double* qd;
};

struct SlotState {
  int scen;        // scenario index within the call (-1 = empty)
  int phase;       // Phase
  int status;      // OpfStatus
  int iters;       // Newton steps taken
  int n_islands, main_label, ref_bus, n_ineq;
  int job;         // 1 = factorise and solve in this scheduling step
  int singular;    // exactly zero pivot met in the last factorisation
  int n_states;    // order of the reduced state matrix
  int cause, near, qr_fail;
  int fp64_only;   // mixed precision: an FP32 solve of this scenario failed to refine
  double gamma, f, f_prev, max_viol, alpha, zeta;
  double metrics[4];
};

struct Slots {
  int B;                        // slots
  int nx, neq, nk, ldk, ni;     // KKT sizes
  int ny, ldy, nyc;             // dynamic algebraic system: ny, lda, columns
  int na, lda_a;                // state matrix max order and lda
  size_t k_stride;              // doubles per slot in K
  size_t a_stride;              // doubles per slot in A
  double* K;
  float* K32;                   // mixed precision: FP32 copy / factors of K, row stride ld32
  int ld32;
  size_t k32_stride;            // floats per slot in K32
  int* piv;                     // [B][max(nk, ny)]
  double* x; double* lam; double* z; double* mu;
  double* hv;                   // [B][ni] inequality values at the last evaluation
  double* jh;                   // [B][nl][8] flow-limit gradients, both ends

  int* label;                   // [B][nb]
  uint8_t* bus_on; uint8_t* br_on; uint8_t* gen_on;
  double* pd; double* qd;       // per-bus load in service [B][nb]
  double* A;                    // [B][a_stride]
  double* wr; double* wi;       // [B][na]
  SlotState* st;
  int* jobs;                    // [B + 2] job list of one launch (JobList)
};

// A device list of the slots that have work in a launch (written by
// launch_job_list: [0] their number, [1] set when that number exceeded
// grid, [2..] slot ids in ascending order) and the launch's workgroups, an
// upper bound on that number.  list == nullptr: one workgroup per slot.
// Listing the slots puts the workgroups with work first: the hardware
// dispatches workgroups in index order, and an idle slot's workgroup that
// waits for a free CU would hold back the busy ones behind it.
struct JobList {
  const int* list = nullptr;
  int grid = 0;
};
// workgroups of a per-slot launch over count slots
inline int job_grid(int count, const JobList& jl) {
  return jl.list ? (count < jl.grid ? count : jl.grid) : count;
}
// the slot of this workgroup, or -1 when it has none
__device__ inline int list_slot(const int* __restrict__ list, int count) {
  const int b = (int)blockIdx.x;
  if (list == nullptr) return b < count ? b : -1;
  return b < list[0] ? list[2 + b] : -1;
}

// Per-scenario detail written by k_classify when requested (parity checks):
// the operating point over the whole network (NaN outside the solved island or
// when the OPF did not run) and the spectrum (NaN-padded to na).
struct DetailOut {
  double* vm; double* va;       // [n][nb]
  double* pg; double* qg;       // [n][ng]
  double* eig_re; double* eig_im;   // [n][na]
  int* n_eig;                   // [n]
};

// Launch wrappers (one per kernel file).
// outage rows hold `width` ids each (2: N-1/N-2 lists, 3: N-3 lists), -1 pads
void launch_islands(const DevNet& net, const Slots& s, const int* outages,
                    int count, hipStream_t st, int width = 2);
// load_scale [requests][n_load] with item_req (ring position -> request):
// per-request load factors of a server (nullptr: the network's loads)
void launch_setup_k(const DevNet& net, const Slots& s, int count, const int* outages,
                    hipStream_t st, int width = 2, const double* load_scale = nullptr,
                    const int* item_req = nullptr);
void launch_opf_eval(const DevNet& net, const Slots& s, int count, double tol,
                     int max_it, hipStream_t st, const JobList& jl = JobList{});
void launch_opf_update(const DevNet& net, const Slots& s, int count,
                       double gamma_max, hipStream_t st, const JobList& jl = JobList{});
// batched LU + solve; with slot states, only slots with st.job == want_job
// in phase want_phase.  role (LuRole) picks the kernel symbol only.
enum LuRole : int { LU_KKT = 0, LU_DYN = 1, LU_KKT_FALLBACK = 2 };

void launch_lu_solve(double* A, size_t stride, int n, int ncols, int lda,
                     int* piv, int piv_stride, SlotState* st, int want_phase, int want_job,
                     int count, int* info, hipStream_t stream, int role = LU_KKT,
                     int max_jobs = -1, const JobList& jl = JobList{});
// orders above the register-resident kernel's limit (k_lu_big.hip)
// nb: launch variant, the panel width 16, 32 or 64, or 1664 / 3264 (panels of
// 16 / 32 in groups of 64); 0 = the autotuner's choice for (current device,
// n, precision), else 32
void launch_lu_big(double* A, size_t stride, int n, int ncols, int lda, int* piv,
                   int piv_stride, SlotState* st, int want_phase, int want_job, int count,
                   int* info, hipStream_t stream, int nb = 0);
void launch_lu_big_f32(float* A, size_t stride, int n, int ncols, int lda, int* piv,
                       int piv_stride, SlotState* st, int want_phase, int want_job, int count,
                       int* info, hipStream_t stream, int nb = 0);
// launch variant per (device, order, precision), 0 when not set: for orders
// up to lu_reg_order() the wavefronts per matrix of k_lu_solve (4 or 8), above
// it the panel code of k_lu_big
void lu_set_variant(int device, int n, bool f32, int v);
int lu_variant(int device, int n, bool f32);
void launch_tune_fill(void* A, bool f32, size_t stride, int n, int ncols, int lda, int count,
                      unsigned seed, hipStream_t stream);
void launch_lu_solve_f32(float* A, size_t stride, int n, int ncols, int lda,
                         int* piv, int piv_stride, SlotState* st, int want_phase, int want_job,
                         int count, int* info, hipStream_t stream,
                         const JobList& jl = JobList{});
void launch_dyn_assemble(const DevNet& net, const Slots& s, int count, hipStream_t st);
void launch_form_state(const DevNet& net, const Slots& s, int count, hipStream_t st);
// scr: scratch of eig_scratch_doubles(order) doubles per matrix, scr_stride
// doubles apart (the slot's KKT array in the engine)
void launch_eig(double* A, size_t stride, int lda, const int* n_per, int n_uniform,
                double* wr, double* wi, int w_stride, SlotState* st, int count,
                int* info, double* scr, size_t scr_stride, hipStream_t stream);
size_t eig_scratch_doubles(int n);
void launch_classify(const Slots& s, int count, double near_eps, int max_it,
                     void* results, const int* item_req, int* req_done,
                     const DetailOut* detail, int nb, int ng, hipStream_t st);
void launch_risk(const int* outages, long long n, const uint8_t* severe_src,
                 int sev_stride, const double* lam, int n_comp, double* risk,
                 hipStream_t st, int width = 2);
void launch_validate(const int* outages, long long n, int n_comp, int* bad,
                     hipStream_t st, int width = 2);
// sets bit 2 of *bad when a failure rate is negative or not finite
void launch_validate_rates(const double* lam, int n_comp, int* bad, hipStream_t st);
// Risk Index extensions (k_risk.hip)
void launch_sev_weights(const void* rec, long long n, int mode, double zeta_ref, double* w,
                        hipStream_t st);
void launch_cc_table(const int* pairs, const double* rate, long long n_cc, int n_comp, double* T,
                     hipStream_t st);
void launch_risk_weighted(const int* outages, long long n, const double* w, const double* lam,
                          const double* cc, int n_comp, double* risk, hipStream_t st);
void launch_risk_split(const int* outages, long long n, const double* w, const double* cc,
                       int n_comp, int ld, double* S1, double* S2, double* C, hipStream_t st);
void launch_risk_mc_gemm(const double* L, long long M, int n, const double* S1, const double* S2,
                         int ld, const double* C, double* R, hipStream_t st);
void launch_rank_hist(const double* R, long long M, int n, int* hist, hipStream_t st);
void launch_risk_summary(const double* R, long long M, int n, const int* hist, double* moments,
                         int* rank_q, hipStream_t st);
// sets bit 2 of *bad when one of n values is negative or not finite
void launch_validate_values(const double* v, long long n, int* bad, hipStream_t st);

// N-3 pruning (k_prune.hip)
void launch_sub_severity(const int* sub, long long n2, const void* rec, int n_comp,
                         uint8_t* single, uint8_t* pair, hipStream_t st);
void launch_n3_prune(const int* rows, long long n3, int n_comp, const uint8_t* single,
                     const uint8_t* pair, uint8_t* keep, hipStream_t st);
size_t n3_select_bytes(long long n3);
int n3_select(void* tmp, size_t bytes, const uint8_t* keep, long long n3, long long* idx,
              long long* count, hipStream_t st);
void launch_gather_rows(const int* rows, const long long* idx, long long k, int* out,
                        hipStream_t st);
void launch_merge_n3(const uint8_t* keep, long long n3, const void* kept_rec, const long long* idx,
                     long long k, void* out, hipStream_t st);

// mixed-precision KKT solve
void launch_kkt_to_f32(const Slots& s, int count, hipStream_t st,
                       const JobList& jl = JobList{});
void launch_kkt_refine(const Slots& s, int count, int pstride, int max_it, hipStream_t st,
                       const JobList& jl = JobList{});
size_t kkt_refine_lds(int nk);

// slot scheduling
void launch_refill(const Slots& s, int count, unsigned long long* next, long long n_scen,
                   long long q_cap, hipStream_t st);
void launch_assign(const Slots& s, int count, hipStream_t st);
void launch_claim(const Slots& s, int count, hipStream_t st);
void launch_phase_counts(const Slots& s, int count, int* out, hipStream_t st);
void launch_gather_request(const int* q_out, const void* q_res, long long q0, int n,
                           long long q_cap, int* out, void* res, hipStream_t st);
void launch_fill_req(int* item_req, long long q0, int n, long long q_cap, int r, hipStream_t st);
void launch_count_jobs(const Slots& s, int count, int want, int* out, hipStream_t st);
// s.jobs = the slots among the first count with st.phase == want_phase and
// st.job == want_job (JOB_ANY: any job; JOB_NONZERO: job != 0), for a launch
// of grid workgroups
constexpr int JOB_ANY = -1, JOB_NONZERO = -2;
void launch_job_list(const Slots& s, int count, int want_phase, int want_job, int grid,
                     hipStream_t st);

}  // namespace cs
