// Islanding check (Section II.B.3) and main-island choice (Section II.A):
// one wavefront per scenario.
//
// Connected components by union-find in LDS: every in-service branch hooks
// the root of the larger-indexed tree under the smaller one with a
// compare-and-swap that succeeds only on a root (retrying otherwise), so each
// tree's root is its smallest bus id and every component ends as one tree.
// Labels are the roots, i.e. the smallest bus id of the island, which makes
// them unique and comparable bit-for-bit with a graph search.  The island
// with the largest in-service generation capacity (sum of Pmax) is kept;
// ties go to the lowest label.  Its angle reference is the network's
// reference bus if inside, else the bus of its lowest-index in-service
// generator (-1 if it has none).
#include "cs_internal.h"

namespace cs {

__device__ inline int uf_find(volatile int* parent, int x) {
  int p = parent[x];
  while (p != x) {
    x = p;
    p = parent[x];
  }
  return x;
}

__global__ __launch_bounds__(64) void k_islands(DevNet net, Slots s,
                                                const int* __restrict__ outages,
                                                int width, int count) {
  const int slot = blockIdx.x;
  if (slot >= count || s.st[slot].phase != PH_NEW) return;
  extern __shared__ int parent[];
  __shared__ int roots_count;
  const int lane = threadIdx.x;
  const long long scen = s.st[slot].scen;
  // an outage row holds width ids (2: N-1/N-2 rows, 3: N-3 rows), -1 pads
  const int o0 = outages[width * scen], o1 = outages[width * scen + 1];
  const int o2 = width > 2 ? outages[width * scen + 2] : -1;
  const int nb = net.nb, nl = net.nl, ng = net.ng;
  const int gen0 = nl, load0 = nl + ng;
  for (int v = lane; v < nb; v += 64) parent[v] = v;
  __syncthreads();
  for (int l = lane; l < nl; l += 64) {
    if (l == o0 || l == o1 || l == o2) continue;
    int a = net.br_f[l], b = net.br_t[l];
    while (true) {
      a = uf_find(parent, a);
      b = uf_find(parent, b);
      if (a == b) break;
      if (a > b) { int t = a; a = b; b = t; }
      // hook root b under a; fails if b stopped being a root
      const int old = atomicCAS(&parent[b], b, a);
      if (old == b) break;
      b = old;
    }
  }
  __syncthreads();
  int* label = s.label + (size_t)slot * nb;
  int nroots = 0;
  for (int v = lane; v < nb; v += 64) {
    const int r = uf_find(parent, v);
    label[v] = r;
    nroots += (r == v);
  }
  for (int off = 32; off > 0; off >>= 1) nroots += __shfl_xor(nroots, off, 64);
  __syncthreads();
  // compress in LDS for the capacity scan
  for (int v = lane; v < nb; v += 64) parent[v] = uf_find(parent, v);
  __syncthreads();
  // main island: largest sum of Pmax of in-service generators
  int best = -1;
  double best_cap = -1.0;
  for (int r = 0; r < nb; ++r) {
    if (parent[r] != r) continue;           // uniform across lanes
    double cap = 0.0;
    for (int g = lane; g < ng; g += 64) {
      const bool on = (gen0 + g != o0) && (gen0 + g != o1) && (gen0 + g != o2);
      if (on && parent[net.gen_bus[g]] == r) cap += net.pmax[g];
    }
    for (int off = 32; off > 0; off >>= 1) cap += __shfl_xor(cap, off, 64);
    if (cap > best_cap) { best_cap = cap; best = r; }
  }
  // reference bus of the main island
  int ref = -1;
  if (parent[net.ref_bus] == best) {
    ref = net.ref_bus;
  } else {
    int cand = 0x7fffffff;
    for (int g = lane; g < ng; g += 64) {
      const bool on = (gen0 + g != o0) && (gen0 + g != o1) && (gen0 + g != o2);
      if (on && parent[net.gen_bus[g]] == best) cand = min(cand, g);
    }
    for (int off = 32; off > 0; off >>= 1) cand = min(cand, __shfl_xor(cand, off, 64));
    if (cand != 0x7fffffff) ref = net.gen_bus[cand];
  }
  (void)load0;
  if (lane == 0) {
    SlotState& S = s.st[slot];
    S.status = OPF_NOT_RUN;
    S.iters = 0;
    S.n_islands = nroots;
    S.main_label = best;
    S.ref_bus = ref;
    S.job = 0;
    S.singular = 0;
    S.n_states = 0;
    S.cause = (nroots > 1) ? C_ISLAND : 0;
    S.near = 0;
    S.qr_fail = 0;
    S.fp64_only = 0;
    S.alpha = __builtin_nan("");
    S.zeta = __builtin_nan("");
    S.max_viol = __builtin_nan("");
    S.f = __builtin_nan("");
    S.f_prev = __builtin_nan("");
  }
  (void)roots_count;
}

void launch_islands(const DevNet& net, const Slots& s, const int* outages,
                    int count, hipStream_t st, int width) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_islands, dim3(count), dim3(64), sizeof(int) * net.nb, st,
                     net, s, outages, width, count);
}

// outage list check: a row of width ids holds distinct valid ids followed by
// -1 padding (all -1 is the base case); the kernels only compare ids, never
// index with them
__global__ void k_validate(const int* __restrict__ outages, long long n,
                           int n_comp, int width, int* __restrict__ bad) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool ok = true, pad = false;
  for (int t = 0; t < width; ++t) {
    const int a = outages[width * i + t];
    if (a == -1) {
      pad = true;
      continue;
    }
    if (pad || a < 0 || a >= n_comp) ok = false;
    for (int u = 0; u < t; ++u)
      if (outages[width * i + u] == a) ok = false;
  }
  if (!ok) atomicOr(bad, 1);
}

void launch_validate(const int* outages, long long n, int n_comp, int* bad,
                     hipStream_t st, int width) {
  if (n <= 0) return;
  const int threads = 256;
  const long long blocks = (n + threads - 1) / threads;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(threads), 0, st,
                     outages, n, n_comp, width, bad);
}

// failure-rate check: finite and >= 0 (eq. (1)-(2) take them as frequencies)
__global__ void k_validate_rates(const double* __restrict__ lam, long long n,
                                 int* __restrict__ bad) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = lam[i];
  if (!(v >= 0.0) || !__builtin_isfinite(v)) atomicOr(bad, 2);
}

void launch_validate_values(const double* v, long long n, int* bad, hipStream_t st) {
  if (n <= 0) return;
  const int threads = 256;
  hipLaunchKernelGGL(k_validate_rates, dim3((unsigned)((n + threads - 1) / threads)),
                     dim3(threads), 0, st, v, n, bad);
}

void launch_validate_rates(const double* lam, int n_comp, int* bad, hipStream_t st) {
  launch_validate_values(lam, n_comp, bad, st);
}

}  // namespace cs
