// Severity and risk (Section II.B and Section II.C, eq. (1)-(3)).
//
// k_classify turns each scenario's islanding, OPF and eigenvalue outcome into
// the binary severity S_c and its cause bits: islands > 1; OPF not converged;
// a converged point violating a limit by more than 1e-6 p.u.; an eigenvalue
// with Re >= 0.  It also reports the largest real part and the minimum damping
// ratio -Re/|lambda| over oscillatory modes (|Im| > 1e-8 |lambda|; 1 if none).
//
// k_risk computes R_i = sum over the list of F_c S_c for every scenario c in
// which component i takes part, F_c = lambda_i (N-1) or lambda_i lambda_j
// (N-2).  One wavefront per component; each lane sums its strided share in
// list order and the lanes combine in a fixed butterfly, so R is identical run
// to run.
#include "cs_internal.h"
#include "../../include/cs.h"

namespace cs {

__global__ __launch_bounds__(64) void k_classify(Slots s, int count, double near_eps,
                                                 int max_it, cs_result* __restrict__ out,
                                                 const int* __restrict__ item_req,
                                                 int* __restrict__ req_done, DetailOut det,
                                                 int nb, int ng) {
  const int slot = blockIdx.x;
  if (slot >= count) return;
  SlotState& S = s.st[slot];
  const int lane = threadIdx.x;
  const int phase = S.phase;
  if (phase != PH_EIG && phase != PH_FIN) return;     // only slots claimed and finished
  const bool have_eig = (phase == PH_EIG) && (S.qr_fail == 0);
  double alpha = -__builtin_inf(), zeta = __builtin_inf();
  bool osc_any = false;
  if (have_eig) {
    const double* wr = s.wr + (size_t)slot * s.na;
    const double* wi = s.wi + (size_t)slot * s.na;
    for (int i = lane; i < S.n_states; i += 64) {
      const double re = wr[i], im = wi[i];
      alpha = fmax(alpha, re);
      const double mag = sqrt(re * re + im * im);
      if (fabs(im) > 1e-8 * mag) {
        osc_any = true;
        zeta = fmin(zeta, -re / mag);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      alpha = fmax(alpha, __shfl_xor(alpha, off, 64));
      zeta = fmin(zeta, __shfl_xor(zeta, off, 64));
    }
    osc_any = __any(osc_any);
  }
  if (det.vm != nullptr) {
    // detail of this scenario, before the record releases the slot
    const int sc = S.scen;
    const int status = S.status;
    const bool solved = status != OPF_NOT_RUN;
    const double nan = __builtin_nan("");
    const double* x = s.x + (size_t)slot * s.nx;
    const uint8_t* bus_on = s.bus_on + (size_t)slot * nb;
    const uint8_t* gen_on = s.gen_on + (size_t)slot * ng;
    for (int b = lane; b < nb; b += 64) {
      const bool on = solved && bus_on[b];
      det.va[(size_t)sc * nb + b] = on ? x[b] : nan;
      det.vm[(size_t)sc * nb + b] = on ? x[nb + b] : nan;
    }
    for (int g = lane; g < ng; g += 64) {
      const bool on = solved && gen_on[g];
      det.pg[(size_t)sc * ng + g] = on ? x[2 * nb + g] : nan;
      det.qg[(size_t)sc * ng + g] = on ? x[2 * nb + ng + g] : nan;
    }
    const int ne = (have_eig && status == OPF_CONVERGED) ? S.n_states : 0;
    const double* wr = s.wr + (size_t)slot * s.na;
    const double* wi = s.wi + (size_t)slot * s.na;
    for (int i = lane; i < s.na; i += 64) {
      det.eig_re[(size_t)sc * s.na + i] = i < ne ? wr[i] : nan;
      det.eig_im[(size_t)sc * s.na + i] = i < ne ? wi[i] : nan;
    }
    if (lane == 0) det.n_eig[sc] = ne;
  }
  if (lane != 0) return;
  int cause = S.cause;
  int nearf = 0;
  const int status = S.status;
  if (status != OPF_CONVERGED) cause |= C_OPF;
  if (status == OPF_NUMERICAL) cause |= C_NUMERICAL;
  double mv = __builtin_nan(""), ar = __builtin_nan(""), zr = __builtin_nan("");
  if (status == OPF_CONVERGED) {
    // converged within two steps of the cap: a solve rounded differently may
    // have ended at the cap instead
    if (S.iters >= max_it - 2) nearf |= N_OPF;
    mv = S.max_viol;
    if (mv > 1e-6) cause |= C_LIMIT;
    if (mv > 1e-7 && mv <= 1e-5) nearf |= N_LIMIT;   // a decade either side of the test
    if (phase == PH_EIG && S.qr_fail) cause |= C_NUMERICAL;
    if (have_eig) {
      ar = alpha;
      zr = osc_any ? zeta : 1.0;
      if (alpha >= 0.0) cause |= C_SSS;
      if (fabs(alpha) <= near_eps) nearf |= N_SSS;
    }
  }
  cs_result r;
  r.severe = cause != 0;
  r.cause = (uint8_t)cause;
  r.opf_status = (uint8_t)status;
  r.near = (uint8_t)nearf;
  r.n_islands = (int16_t)S.n_islands;
  r.opf_iters = (int16_t)(status == OPF_NOT_RUN ? 0 : S.iters);
  r.n_states = (status == OPF_CONVERGED) ? S.n_states : 0;
  r.reserved = 0;
  r.opf_cost = (status == OPF_NOT_RUN) ? __builtin_nan("") : S.f;
  r.max_real_eig = ar;
  r.min_damping = zr;
  r.max_violation = mv;
  out[S.scen] = r;
  // serving: one more record of this scenario's request is complete (the
  // record is visible device-wide before the count that announces it)
  if (req_done != nullptr) {
    __threadfence();
    atomicAdd(&req_done[item_req[S.scen]], 1);
  }
  // the record and every read of this slot precede its release: a refill
  // running on another stream may reuse the slot as soon as it sees EMPTY
  __threadfence();
  S.phase = PH_EMPTY;
}

void launch_classify(const Slots& s, int count, double near_eps, int max_it,
                     void* results, const int* item_req, int* req_done,
                     const DetailOut* detail, int nb, int ng, hipStream_t st) {
  if (count <= 0) return;
  DetailOut det{};
  if (detail) det = *detail;
  hipLaunchKernelGGL(k_classify, dim3(count), dim3(64), 0, st, s, count, near_eps,
                     max_it, reinterpret_cast<cs_result*>(results), item_req, req_done, det,
                     nb, ng);
}

__global__ __launch_bounds__(256) void k_risk(const int* __restrict__ outages, long long n,
                                              const uint8_t* __restrict__ sev, int sev_stride,
                                              const double* __restrict__ lam, int n_comp,
                                              double* __restrict__ risk, int width) {
  const int comp = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (comp >= n_comp) return;
  double acc = 0.0;
  for (long long c = lane; c < n; c += 64) {
    const int a = outages[width * c], b = outages[width * c + 1];
    const int d = width > 2 ? outages[width * c + 2] : -1;
    if ((a == comp || b == comp || d == comp) && sev[c * sev_stride]) {
      // eq. (1)-(2): the product of the outaged components' rates
      double f = (b < 0) ? lam[a] : lam[a] * lam[b];
      if (d >= 0) f *= lam[d];
      acc += f;
    }
  }
  for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) risk[comp] = acc;
}

void launch_risk(const int* outages, long long n, const uint8_t* severe_src,
                 int sev_stride, const double* lam, int n_comp, double* risk,
                 hipStream_t st, int width) {
  if (n_comp <= 0) return;
  hipLaunchKernelGGL(k_risk, dim3((n_comp + 3) / 4), dim3(256), 0, st, outages, n,
                     severe_src, sev_stride, lam, n_comp, risk, width);
}

// ------------------------------------------------------------- scheduling
// Give every free slot the next scenario of the list (one thread per slot;
// the order in which slots draw is irrelevant, each scenario's arithmetic
// depends on its own data only).  Scenario k of the stream of work sits at
// position k % q_cap of the list (a ring when serving).
__global__ void k_refill(SlotState* __restrict__ st, int count,
                         unsigned long long* __restrict__ next, long long n_scen, long long q_cap) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= count || st[slot].phase != PH_EMPTY) return;
  const unsigned long long k = atomicAdd(next, 1ull);
  if ((long long)k >= n_scen) {
    // give the number back: scenarios admitted later (serving) start at
    // n_scen, so the counter must end this launch at n_scen exactly
    atomicSub(next, 1ull);
    return;
  }
  st[slot].scen = (int)((long long)k % q_cap);
  st[slot].job = 0;
  st[slot].phase = PH_NEW;
}

// Slot i takes scenario i (single-scenario entry points).
__global__ void k_assign(SlotState* __restrict__ st, int count) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= count) return;
  st[slot].scen = slot;
  st[slot].job = 0;
  st[slot].phase = PH_NEW;
}

// Hand the slots that left the interior-point loop to the dynamic stage.
__global__ void k_claim(SlotState* __restrict__ st, int count) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= count) return;
  const int ph = st[slot].phase;
  if (ph == PH_DYN) st[slot].phase = PH_DYNB;
  else if (ph == PH_DONE) st[slot].phase = PH_FIN;
}

// out[p] = number of slots in phase p (p < PH_COUNT).
__global__ void k_phase_counts(const SlotState* __restrict__ st, int count,
                               int* __restrict__ out) {
  __shared__ int acc[PH_COUNT];
  if (threadIdx.x < PH_COUNT) acc[threadIdx.x] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    const int ph = st[i].phase;
    if (ph >= 0 && ph < PH_COUNT) atomicAdd(&acc[ph], 1);
  }
  __syncthreads();
  if (threadIdx.x < PH_COUNT) out[threadIdx.x] = acc[threadIdx.x];
}

// Number of interior-point slots with job == want (1: a KKT solve this
// round; 3: an FP64 fallback of the mixed-precision solve).
__global__ void k_count_jobs(const SlotState* __restrict__ st, int count, int want,
                             int* __restrict__ out) {
  __shared__ int acc;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  int c = 0;
  for (int i = threadIdx.x; i < count; i += blockDim.x)
    c += (st[i].job == want && st[i].phase == PH_IPM);
  atomicAdd(&acc, c);
  __syncthreads();
  if (threadIdx.x == 0) *out = acc;
}

__device__ inline bool job_matches(const SlotState& S, int want_phase, int want_job) {
  if (S.phase != want_phase) return false;
  return want_job == JOB_ANY || (want_job == JOB_NONZERO ? S.job != 0 : S.job == want_job);
}

// The slots of one stage with a given job, in ascending order (one
// workgroup of 1,024 threads, each scanning a contiguous range of slots):
// list[0] = their number m, list[2 + i] = the i-th; list[1] is set when m
// exceeds grid, the workgroups of the launch that reads the list (sticky
// until the caller clears it).
__global__ __launch_bounds__(1024) void k_job_list(const SlotState* __restrict__ st, int count,
                                                   int want_phase, int want_job, int grid,
                                                   int* __restrict__ list) {
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (count + 1023) / 1024;
  const int b0 = min(count, tid * per), b1 = min(count, b0 + per);
  int c = 0;
  for (int i = b0; i < b1; ++i) c += job_matches(st[i], want_phase, want_job);
  // inclusive scan of the counts over the wavefront, then over wavefronts
  int incl = c;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wave; ++w) base += wsum[w];
  int pos = base + incl - c;
  for (int i = b0; i < b1; ++i)
    if (job_matches(st[i], want_phase, want_job)) list[2 + pos++] = i;
  if (tid == 1023) {
    const int m = base + incl;
    list[0] = m;
    if (m > grid) list[1] = 1;
  }
}

void launch_job_list(const Slots& s, int count, int want_phase, int want_job, int grid,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_job_list, dim3(1), dim3(1024), 0, st, s.st, count, want_phase, want_job,
                     grid, s.jobs);
}

void launch_refill(const Slots& s, int count, unsigned long long* next, long long n_scen,
                   long long q_cap, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_refill, dim3((count + 255) / 256), dim3(256), 0, st, s.st, count, next,
                     n_scen, q_cap);
}

void launch_assign(const Slots& s, int count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_assign, dim3((count + 255) / 256), dim3(256), 0, st, s.st, count);
}

void launch_claim(const Slots& s, int count, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_claim, dim3((count + 255) / 256), dim3(256), 0, st, s.st, count);
}

void launch_phase_counts(const Slots& s, int count, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_phase_counts, dim3(1), dim3(1024), 0, st, s.st, count, out);
}

// Copy ring positions [q0, q0 + n) (mod q_cap) of the list and its records
// to contiguous buffers (a served request's risk reduction).
__global__ void k_gather_request(const int* __restrict__ q_out, const cs_result* __restrict__ q_res,
                                 long long q0, int n, long long q_cap, int* __restrict__ out,
                                 cs_result* __restrict__ res) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long k = (q0 + i) % q_cap;
  out[2 * i] = q_out[2 * k];
  out[2 * i + 1] = q_out[2 * k + 1];
  res[i] = q_res[k];
}

void launch_gather_request(const int* q_out, const void* q_res, long long q0, int n,
                           long long q_cap, int* out, void* res, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_request, dim3((n + 255) / 256), dim3(256), 0, st, q_out,
                     reinterpret_cast<const cs_result*>(q_res), q0, n, q_cap, out,
                     reinterpret_cast<cs_result*>(res));
}

// Set list positions [q0, q0 + n) (mod q_cap) to request index r.
__global__ void k_fill_req(int* __restrict__ item_req, long long q0, int n, long long q_cap, int r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) item_req[(q0 + i) % q_cap] = r;
}

void launch_fill_req(int* item_req, long long q0, int n, long long q_cap, int r, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_req, dim3((n + 255) / 256), dim3(256), 0, st, item_req, q0, n, q_cap, r);
}

void launch_count_jobs(const Slots& s, int count, int want, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_count_jobs, dim3(1), dim3(1024), 0, st, s.st, count, want, out);
}

}  // namespace cs
