// N-3 screening with pruning (Section VI names higher-order contingencies as
// future work; Section V.C asks for the search space to be reduced before the
// full AC evaluation).
//
// A triple of outaged components is pruned, i.e. taken as severe without
// being solved, when one of its sub-scenarios (a single component or a pair)
// is severe in an already screened N-1/N-2 list: losing more elements is
// read as never making a severe contingency secure.  For islanding by branch
// outages this holds exactly (removing more branches never reconnects a
// network); for the OPF and small-signal criteria it is the screening
// assumption, and pruned records carry their own cause bit.  Sub-scenarios
// absent from the screened list prune nothing.
//
// k_sub_severity marks the severe singles and pairs in two tables; k_n3_prune
// flags each row; the kept rows are compacted in list order (rocPRIM's
// select), screened by the ordinary engine, and the records of all rows are
// written in list order.
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "cs_internal.h"
#include "../../include/cs.h"

namespace cs {

__global__ void k_sub_severity(const int* __restrict__ sub, long long n2,
                               const cs_result* __restrict__ rec, int n_comp,
                               uint8_t* __restrict__ single, uint8_t* __restrict__ pair) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n2 || !rec[c].severe) return;
  const int a = sub[2 * c], b = sub[2 * c + 1];
  if (a < 0) return;                       // the base case prunes nothing
  // every writer stores the same value
  if (b < 0) {
    single[a] = 1;
  } else {
    pair[(size_t)a * n_comp + b] = 1;
    pair[(size_t)b * n_comp + a] = 1;
  }
}

void launch_sub_severity(const int* sub, long long n2, const void* rec, int n_comp,
                         uint8_t* single, uint8_t* pair, hipStream_t st) {
  if (n2 <= 0) return;
  const int t = 256;
  hipLaunchKernelGGL(k_sub_severity, dim3((unsigned)((n2 + t - 1) / t)), dim3(t), 0, st, sub, n2,
                     reinterpret_cast<const cs_result*>(rec), n_comp, single, pair);
}

// keep[r] = 1 when row r of the N-3 list must be solved
__global__ void k_n3_prune(const int* __restrict__ rows, long long n3, int n_comp,
                           const uint8_t* __restrict__ single, const uint8_t* __restrict__ pair,
                           uint8_t* __restrict__ keep) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n3) return;
  int id[3];
  int k = 0;
  for (int t = 0; t < 3; ++t) {
    const int v = rows[3 * r + t];
    if (v >= 0) id[k++] = v;
  }
  bool pruned = false;
  if (k >= 2)
    for (int t = 0; t < k; ++t) pruned |= single[id[t]] != 0;
  if (k == 3)
    pruned |= pair[(size_t)id[0] * n_comp + id[1]] || pair[(size_t)id[0] * n_comp + id[2]] ||
              pair[(size_t)id[1] * n_comp + id[2]];
  keep[r] = pruned ? 0 : 1;
}

void launch_n3_prune(const int* rows, long long n3, int n_comp, const uint8_t* single,
                     const uint8_t* pair, uint8_t* keep, hipStream_t st) {
  if (n3 <= 0) return;
  const int t = 256;
  hipLaunchKernelGGL(k_n3_prune, dim3((unsigned)((n3 + t - 1) / t)), dim3(t), 0, st, rows, n3,
                     n_comp, single, pair, keep);
}

// indices of the kept rows, in list order; *count = how many
size_t n3_select_bytes(long long n3) {
  size_t bytes = 0;
  rocprim::counting_iterator<long long> it(0);
  if (rocprim::select(nullptr, bytes, it, static_cast<const uint8_t*>(nullptr),
                      static_cast<long long*>(nullptr), static_cast<long long*>(nullptr),
                      (size_t)n3) != hipSuccess)
    return 0;
  return bytes;
}

int n3_select(void* tmp, size_t bytes, const uint8_t* keep, long long n3, long long* idx,
              long long* count, hipStream_t st) {
  rocprim::counting_iterator<long long> it(0);
  return rocprim::select(tmp, bytes, it, keep, idx, count, (size_t)n3, st) == hipSuccess ? 0 : -1;
}

__global__ void k_gather_rows(const int* __restrict__ rows, const long long* __restrict__ idx,
                              long long k, int* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const long long r = idx[i];
  for (int t = 0; t < 3; ++t) out[3 * i + t] = rows[3 * r + t];
}

void launch_gather_rows(const int* rows, const long long* idx, long long k, int* out,
                        hipStream_t st) {
  if (k <= 0) return;
  const int t = 256;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((k + t - 1) / t)), dim3(t), 0, st, rows, idx,
                     k, out);
}

// Pruned rows: severe, cause CS_CAUSE_PRUNED, nothing solved.
__global__ void k_pruned_records(const uint8_t* __restrict__ keep, long long n3,
                                 cs_result* __restrict__ out) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n3 || keep[r]) return;
  cs_result x;
  const double nan = __builtin_nan("");
  x.severe = 1;
  x.cause = CS_CAUSE_PRUNED;
  x.opf_status = CS_OPF_NOT_RUN;
  x.near = 0;
  x.n_islands = 0;
  x.opf_iters = 0;
  x.n_states = 0;
  x.reserved = 0;
  x.opf_cost = nan;
  x.max_real_eig = nan;
  x.min_damping = nan;
  x.max_violation = nan;
  out[r] = x;
}

__global__ void k_scatter_records(const cs_result* __restrict__ in, const long long* __restrict__ idx,
                                  long long k, cs_result* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  out[idx[i]] = in[i];
}

void launch_merge_n3(const uint8_t* keep, long long n3, const void* kept_rec, const long long* idx,
                     long long k, void* out, hipStream_t st) {
  const int t = 256;
  if (n3 > 0)
    hipLaunchKernelGGL(k_pruned_records, dim3((unsigned)((n3 + t - 1) / t)), dim3(t), 0, st, keep,
                       n3, reinterpret_cast<cs_result*>(out));
  if (k > 0)
    hipLaunchKernelGGL(k_scatter_records, dim3((unsigned)((k + t - 1) / t)), dim3(t), 0, st,
                       reinterpret_cast<const cs_result*>(kept_rec), idx, k,
                       reinterpret_cast<cs_result*>(out));
}

}  // namespace cs
