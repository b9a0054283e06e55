// Mixed-precision KKT solve: the Newton system is factorised in FP32 on the
// matrix cores (k_lu_solve<float>) and its solution refined in FP64 against
// the FP64 matrix, with an FP64 factorisation as the fallback.
//
//   k_kkt_to_f32:   K32 = fl32(K), the augmented KKT system [K | r], for every
//                   slot that asked for a solve;
//   (FP32 LU + forward elimination + back substitution: x0 in K32's last column)
//   k_kkt_refine:   x = x0; repeat: r = b - K x in FP64; stop when the
//                   componentwise backward error max_i |r_i| / (|K| |x| + |b|)_i
//                   is at most 8 sqrt(n) eps_64 (rows of the KKT system differ
//                   in scale by many orders near the optimum, so a normwise
//                   test would let the small rows, the power balance, go
//                   unsolved); else solve L U d = P r with the FP32 factors
//                   and x += d.  At most max_it
//                   corrections; a slot that does not get there, or meets a
//                   non-finite value, is marked for the FP64 factorisation
//                   (job = 3), which then overwrites its right-hand side with
//                   the FP64 solution as in the plain path.
#include "cs_internal.h"

#include <float.h>

namespace cs {

constexpr int MX_THREADS = 512;
constexpr int MX_WAVES = MX_THREADS / 64;

__global__ __launch_bounds__(256) void k_kkt_to_f32(Slots s, int count,
                                                    const int* __restrict__ list) {
  const int slot = list_slot(list, count);
  if (slot < 0) return;
  SlotState& S = s.st[slot];
  if (S.phase != PH_IPM || S.job != 1) return;
  // the KKT system only gets worse conditioned as the barrier falls: once a
  // scenario needed the FP64 factorisation, it keeps using it
  if (S.fp64_only) {
    __syncthreads();
    if (threadIdx.x == 0) S.job = 3;
    return;
  }
  const int n = s.nk;
  const double* K = s.K + (size_t)slot * s.k_stride;
  float* F = s.K32 + (size_t)slot * s.k32_stride;
  // element e = r (n + 1) + c of the augmented system; eight loads of a
  // thread in flight together
  const int w = n + 1, tot = n * w;
  for (int e0 = threadIdx.x; e0 < tot; e0 += 8 * blockDim.x) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * blockDim.x;
      const int r = e / w, c = e - r * w;
      v[u] = (e < tot) ? K[(size_t)r * s.ldk + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * blockDim.x;
      const int r = e / w, c = e - r * w;
      if (e < tot) F[(size_t)r * s.ld32 + c] = (float)v[u];
    }
  }
}

// perm[i] = the row of the original system at position i after the
// factorisation's interchanges (applied in the order they were made)
__device__ void pivots_to_perm(const int* piv, int n, int* perm) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) perm[i] = i;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < n; ++j) {
      const int p = piv[j];
      if (p != j) {
        const int t = perm[j];
        perm[j] = perm[p];
        perm[p] = t;
      }
    }
  __syncthreads();
}

// The triangular solves work by 32-row blocks: the diagonal block is staged
// in LDS, one wavefront solves it (lane i holds y_i; each solved value is
// broadcast and eliminated from the other rows of the block), then every
// thread updates the rows outside the block.
constexpr int MX_BS = 32;

// y <- L^{-1} y, L unit lower triangular (row-major, below the diagonal of F)
__device__ void forward_f32(const float* __restrict__ F, int ld, int n, float* y, float* blk) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int b0 = 0; b0 < n; b0 += MX_BS) {
    const int bs = min(MX_BS, n - b0);
    for (int e = tid; e < MX_BS * MX_BS; e += MX_THREADS) {
      const int i = e / MX_BS, j = e % MX_BS;
      blk[e] = (i < bs && j < bs) ? F[(size_t)(b0 + i) * ld + b0 + j] : 0.f;
    }
    __syncthreads();
    if (wave == 0) {
      float v = (lane < bs) ? y[b0 + lane] : 0.f;
      for (int i = 0; i < bs; ++i) {
        const float yi = __shfl(v, i, 64);
        if (lane > i && lane < bs) v -= blk[lane * MX_BS + i] * yi;
      }
      if (lane < bs) y[b0 + lane] = v;
    }
    __syncthreads();
    for (int i = b0 + bs + tid; i < n; i += MX_THREADS) {
      const float* row = F + (size_t)i * ld + b0;
      // the block's entries all in flight before the first is used
      float f[MX_BS];
#pragma unroll
      for (int j = 0; j < MX_BS; ++j) f[j] = (j < bs) ? row[j] : 0.f;
      float acc = y[i];
#pragma unroll
      for (int j = 0; j < MX_BS; ++j)
        if (j < bs) acc -= f[j] * y[b0 + j];
      y[i] = acc;
    }
    __syncthreads();
  }
}

// y <- U^{-1} y, U upper triangular (on and above the diagonal of F), from
// the bottom block up
__device__ void backward_f32(const float* __restrict__ F, int ld, int n, float* y, float* blk) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = (n + MX_BS - 1) / MX_BS;
  for (int b = nblk - 1; b >= 0; --b) {
    const int b0 = b * MX_BS;
    const int bs = min(MX_BS, n - b0);
    for (int e = tid; e < MX_BS * MX_BS; e += MX_THREADS) {
      const int i = e / MX_BS, j = e % MX_BS;
      blk[e] = (i < bs && j < bs) ? F[(size_t)(b0 + i) * ld + b0 + j] : 0.f;
    }
    __syncthreads();
    if (wave == 0) {
      float v = (lane < bs) ? y[b0 + lane] : 0.f;
      for (int i = bs - 1; i >= 0; --i) {
        const float xi = __shfl(v, i, 64) / blk[i * MX_BS + i];
        if (lane == i) v = xi;
        if (lane < i) v -= blk[lane * MX_BS + i] * xi;
      }
      if (lane < bs) y[b0 + lane] = v;
    }
    __syncthreads();
    for (int i = tid; i < b0; i += MX_THREADS) {
      const float* row = F + (size_t)i * ld + b0;
      float f[MX_BS];
#pragma unroll
      for (int j = 0; j < MX_BS; ++j) f[j] = (j < bs) ? row[j] : 0.f;
      float acc = y[i];
#pragma unroll
      for (int j = 0; j < MX_BS; ++j)
        if (j < bs) acc -= f[j] * y[b0 + j];
      y[i] = acc;
    }
    __syncthreads();
  }
}

__device__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double m = red[0];
  for (int w = 1; w < MX_WAVES; ++w) m = fmax(m, red[w]);
  return m;
}

__global__ __launch_bounds__(MX_THREADS) void k_kkt_refine(Slots s, int count, int pstride,
                                                          int max_it,
                                                          const int* __restrict__ list) {
  const int slot = list_slot(list, count);
  if (slot < 0) return;
  SlotState& S = s.st[slot];
  if (S.phase != PH_IPM || S.job != 1) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = s.nk;
  double* K = s.K + (size_t)slot * s.k_stride;
  const float* F = s.K32 + (size_t)slot * s.k32_stride;
  const int* piv = s.piv + (size_t)slot * pstride;
  extern __shared__ __attribute__((aligned(16))) unsigned char mx_lds[];
  double* x = reinterpret_cast<double*>(mx_lds);     // [n]
  double* r = x + n;                                   // [n]
  float* y = reinterpret_cast<float*>(r + n);          // [n]
  int* perm = reinterpret_cast<int*>(y + n);           // [n]
  __shared__ double red[MX_WAVES];
  __shared__ float blk[MX_BS * MX_BS];
  __shared__ int s_ok;
  for (int i = tid; i < n; i += MX_THREADS) x[i] = (double)F[(size_t)i * s.ld32 + n];
  pivots_to_perm(piv, n, perm);
  bool ok = false;
  for (int it = 0; it <= max_it; ++it) {
    // r = b - K x and the componentwise backward error, one wavefront per row
    double berr = 0.0;
    for (int i = wave; i < n; i += MX_WAVES) {
      const double* row = K + (size_t)i * s.ldk;
      double acc = 0.0, den = 0.0;
      // the row's entries in groups of 8 per lane, loads of a group in flight
      // together
      for (int j0 = lane; j0 < n; j0 += 8 * 64) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = (j0 + 64 * u < n) ? row[j0 + 64 * u] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = j0 + 64 * u;
          if (j < n) {
            acc += a[u] * x[j];
            den += fabs(a[u]) * fabs(x[j]);
          }
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off, 64);
        den += __shfl_xor(den, off, 64);
      }
      const double bi = row[n];
      const double ri = bi - acc;
      den += fabs(bi);
      if (lane == 0) r[i] = ri;
      const double e = (ri == 0.0) ? 0.0 : ((den > 0.0) ? fabs(ri) / den : __builtin_inf());
      berr = fmax(berr, (e == e) ? e : __builtin_inf());
    }
    berr = block_max(berr, red);
    if (berr <= 8.0 * sqrt((double)n) * DBL_EPSILON) {
      ok = true;
      break;
    }
    if (it == max_it || !(berr < __builtin_inf())) break;
    // d = (LU)^{-1} P r in FP32, x += d
    for (int i = tid; i < n; i += MX_THREADS) y[i] = (float)r[perm[i]];
    __syncthreads();
    forward_f32(F, s.ld32, n, y, blk);
    backward_f32(F, s.ld32, n, y, blk);
    for (int i = tid; i < n; i += MX_THREADS) x[i] += (double)y[i];
    __syncthreads();
  }
  if (tid == 0) s_ok = ok;
  __syncthreads();
  if (s_ok) {
    for (int i = tid; i < n; i += MX_THREADS) K[(size_t)i * s.ldk + n] = x[i];
  } else if (tid == 0) {
    S.job = 3;             // FP64 factorisation of the untouched FP64 system
    S.fp64_only = 1;
  }
}

void launch_kkt_to_f32(const Slots& s, int count, hipStream_t st, const JobList& jl) {
  const int grid = job_grid(count, jl);
  if (grid <= 0) return;
  hipLaunchKernelGGL(k_kkt_to_f32, dim3(grid), dim3(256), 0, st, s, count, jl.list);
}

size_t kkt_refine_lds(int nk) {
  return (sizeof(double) * 2 + sizeof(float) + sizeof(int)) * (size_t)nk + 16;
}

void launch_kkt_refine(const Slots& s, int count, int pstride, int max_it, hipStream_t st,
                       const JobList& jl) {
  const int grid = job_grid(count, jl);
  if (grid <= 0) return;
  hipLaunchKernelGGL(k_kkt_refine, dim3(grid), dim3(MX_THREADS), kkt_refine_lds(s.nk), st, s,
                     count, pstride, max_it, jl.list);
}

}  // namespace cs
