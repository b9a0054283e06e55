// Batched dense LU with partial pivoting and solve for orders above the
// register-resident kernel's limit (k_dense.hip holds panels of up to 1,024
// rows in registers): one workgroup per matrix, the matrix in global memory.
//
// Blocked LU, panel width NB (16, 32 or 64), right-looking, or panels of 16
// or 32 columns left-looking inside groups of 64 (the autotuner's choice per
// order and precision; plain 32 by default), the same arithmetic contract as
// LAPACK's getrf (largest |a| pivot, ties to the lowest row, rows swapped
// across the whole augmented matrix, multipliers by division):
//   panel   column by column over the rows below the diagonal: a workgroup
//           argmax, the row interchange across every column, the scaling and
//           the rank-1 update of the panel's remaining columns;
//   U12     inv(L11) A12 for the panel's block row right of it (each thread
//           owns columns, L11 staged in LDS);
//   update  A22 -= L21 U12 on the matrix cores (v_mfma_f64_16x16x4f64, or
//           the FP32 step for the mixed-precision factorisation), 32 x 32
//           groups handed to the wavefronts in turn;
//   solve   U x = y for the right-hand-side columns by NB-row blocks from the
//           bottom (the forward substitution happened on the augmented
//           columns during the elimination).
// Its bound is the latency of the panel steps (four barriers per column);
// it serves the KKT systems of networks whose order exceeds 1,024.
#include "cs_internal.h"

#include <climits>

namespace cs {

constexpr int BIG_T = 512, BIG_W = BIG_T / 64;

template <class T> struct BigMfma;
template <> struct BigMfma<double> {
  typedef double acc __attribute__((ext_vector_type(4)));
  static __device__ inline acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator q of lane (li, lk) holds row lk + 4 q, column li
  static __device__ constexpr int row(int lk, int q) { return lk + 4 * q; }
};
template <> struct BigMfma<float> {
  typedef float acc __attribute__((ext_vector_type(4)));
  static __device__ inline acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator q of lane (li, lk) holds row 4 lk + q, column li
  static __device__ constexpr int row(int lk, int q) { return 4 * lk + q; }
};

template <class T>
__device__ inline bool big_better(T v, int i, T bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

#define AA(r, c) A[(size_t)(r) * lda + (c)]

// A[rlo:rhi, clo:chi] -= A[rlo:rhi, klo:klo+kn] A[klo:klo+kn, clo:chi]
// (kn <= KMAX) on the matrix cores, 32 x 32 groups handed to the wavefronts
// in turn
template <class T, int KMAX>
__device__ inline void big_update(T* __restrict__ A, int lda, int rlo, int rhi, int clo, int chi,
                                  int klo, int kn) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int gr = (rhi - rlo + 31) / 32, gc = (chi - clo + 31) / 32;
  for (int t = wave; t < gr * gc; t += BIG_W) {
    const int i0 = rlo + 32 * (t / gc), j0 = clo + 32 * (t % gc);
    typename BigMfma<T>::acc acc[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = i0 + 16 * ti + BigMfma<T>::row(lk, q), c = j0 + 16 * tj + li;
          acc[ti][tj][q] = (r < rhi && c < chi) ? AA(r, c) : T(0);
        }
#pragma unroll
    for (int kk = 0; kk < KMAX; kk += 4) {
      const int k = kk + lk;
      T a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int r = i0 + 16 * u + li, c = j0 + 16 * u + li;
        a[u] = (k < kn && r < rhi) ? -AA(r, klo + k) : T(0);
        b[u] = (k < kn && c < chi) ? AA(klo + k, c) : T(0);
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = BigMfma<T>::mac(a[ti], b[tj], acc[ti][tj]);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = i0 + 16 * ti + BigMfma<T>::row(lk, q), c = j0 + 16 * tj + li;
          if (r < rhi && c < chi) AA(r, c) = acc[ti][tj][q];
        }
  }
}

// rows g0+1 .. g0+m-1 of columns [clo, chi): forward substitution with the
// unit lower L held in Lg (rows and columns relative to g0), each thread
// owning columns (the column's values stay in the caches)
template <class T, int RANK>
__device__ inline void big_forward(T* __restrict__ A, int lda, int g0, int m, int clo, int chi,
                                   const T (*Lg)[RANK + 1]) {
  for (int c = clo + (int)threadIdx.x; c < chi; c += BIG_T)
    for (int r = 1; r < m; ++r) {
      T acc = AA(g0 + r, c);
      for (int t = 0; t < r; ++t) acc -= Lg[r][t] * AA(g0 + t, c);
      AA(g0 + r, c) = acc;
    }
}

// Panels of BIG_NB columns in groups of RANK columns (RANK a multiple of
// BIG_NB; RANK = BIG_NB is the plain right-looking form).  Inside a group the
// panels are left-looking: a panel first takes the group's earlier panels
// (its rows in the group by forward substitution with the group's L, its rows
// below by a rank k0 - g0 update), then is factorised; after the group the
// U12 rows of the whole group come from one forward substitution and the
// trailing matrix takes one rank-RANK update, so that it is read and written
// once per RANK columns instead of once per panel.  Two workgroups per CU
// (register budget of 128), so that one's panel latency overlaps the other's
// work.
template <class T, int BIG_NB, int RANK>
__global__ __launch_bounds__(BIG_T, 2) void k_lu_big(T* __restrict__ Abase, size_t stride, int n,
                                                  int ncols, int lda, int* __restrict__ pivbase,
                                                  int piv_stride, SlotState* __restrict__ st,
                                                  int want_phase, int want_job,
                                                  int* __restrict__ info) {
  static_assert(RANK % BIG_NB == 0 && RANK <= 64, "groups of whole panels, rank <= 64");
  const int slot = blockIdx.x;
  if (st != nullptr && (st[slot].job != want_job || st[slot].phase != want_phase)) return;
  T* __restrict__ A = Abase + (size_t)slot * stride;
  int* __restrict__ piv = pivbase + (size_t)slot * piv_stride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ T Lg[RANK][RANK + 1];         // the group's unit lower L (relative to g0)
  __shared__ T red_v[BIG_W];
  __shared__ int red_i[BIG_W];
  __shared__ int s_p, s_sing;
  __shared__ T s_d;
  __shared__ T ublk[BIG_NB][BIG_NB + 1];
  if (tid == 0) s_sing = 0;
  __syncthreads();
  for (int g0 = 0; g0 < n; g0 += RANK) {
    const int g1 = min(g0 + RANK, n);
    for (int k0 = g0; k0 < g1; k0 += BIG_NB) {
      const int kb = min(BIG_NB, g1 - k0);
      const int k1 = k0 + kb;
      if (k0 > g0) {
        // ---------------- the panel takes the group's earlier panels
        big_forward<T, RANK>(A, lda, g0, k0 - g0, k0, k1, Lg);
        __syncthreads();
        big_update<T, RANK>(A, lda, k0, n, k0, k1, g0, k0 - g0);
        __syncthreads();
      }
      // ---------------- panel
      for (int j = k0; j < k1; ++j) {
        T bv = T(-1);
        int bi = INT_MAX;
        for (int i = j + tid; i < n; i += BIG_T) {
          const T x = AA(i, j);
          // a NaN entry ranks above every number, so a row is always chosen
          const T a = (x == x) ? fabs(x) : T(HUGE_VAL);
          if (big_better(a, i, bv, bi)) {
            bv = a;
            bi = i;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const T v2 = __shfl_xor(bv, off, 64);
          const int i2 = __shfl_xor(bi, off, 64);
          if (big_better(v2, i2, bv, bi)) {
            bv = v2;
            bi = i2;
          }
        }
        if (lane == 0) {
          red_v[wave] = bv;
          red_i[wave] = bi;
        }
        __syncthreads();
        if (tid == 0) {
          T v = red_v[0];
          int p = red_i[0];
          for (int w = 1; w < BIG_W; ++w)
            if (big_better(red_v[w], red_i[w], v, p)) {
              v = red_v[w];
              p = red_i[w];
            }
          s_p = p;
          piv[j] = p;
        }
        __syncthreads();
        const int p = s_p;
        if (p != j)
          for (int c = tid; c < ncols; c += BIG_T) {
            const T a = AA(j, c), b = AA(p, c);
            AA(j, c) = b;
            AA(p, c) = a;
          }
        __syncthreads();
        if (tid == 0) {
          s_d = AA(j, j);
          if (s_d == T(0)) s_sing = 1;
        }
        __syncthreads();
        const T d = s_d;
        if (d != T(0)) {
          // multipliers, then the rank-1 update of the panel's other columns;
          // each thread owns its rows
          for (int i = j + 1 + tid; i < n; i += BIG_T) {
            const T l = AA(i, j) / d;
            AA(i, j) = l;
            for (int c = j + 1; c < k1; ++c) AA(i, c) -= l * AA(j, c);
          }
        }
        __syncthreads();
      }
      // the panel's rows of the group's L (final: later interchanges move
      // only rows below the panel)
      for (int e = tid; e < kb * (k1 - g0); e += BIG_T) {
        const int r = e / (k1 - g0), c = e % (k1 - g0);
        Lg[k0 - g0 + r][c] = AA(k0 + r, g0 + c);
      }
      __syncthreads();
    }
    if (g1 >= ncols) continue;
    // ---------------- U12 of the group's rows = inv(L11) A12 (L11 unit lower)
    big_forward<T, RANK>(A, lda, g0, g1 - g0, g1, ncols, Lg);
    __syncthreads();
    // ---------------- A22 -= L21 U12, rank g1 - g0
    big_update<T, RANK>(A, lda, g1, n, g1, ncols, g0, g1 - g0);
    __syncthreads();
  }
  // ---------------- U x = y, BIG_NB-row blocks from the bottom
  const int nrhs = ncols - n;
  for (int r1 = n; r1 > 0; r1 -= BIG_NB) {
    const int r0 = max(0, r1 - BIG_NB), bs = r1 - r0;
    for (int e = tid; e < bs * bs; e += BIG_T) {
      const int r = e / bs, c = e % bs;
      ublk[r][c] = AA(r0 + r, r0 + c);
    }
    __syncthreads();
    // the diagonal block: one thread per right-hand side
    for (int c = n + tid; c < ncols; c += BIG_T) {
      for (int r = bs - 1; r >= 0; --r) {
        T acc = AA(r0 + r, c);
        for (int t = r + 1; t < bs; ++t) acc -= ublk[r][t] * AA(r0 + t, c);
        AA(r0 + r, c) = acc / ublk[r][r];
      }
    }
    __syncthreads();
    // the rows above take the block's solution
    const long long work = (long long)r0 * nrhs;
    for (long long e = tid; e < work; e += BIG_T) {
      const int r = (int)(e / nrhs), c = n + (int)(e % nrhs);
      T acc = AA(r, c);
      for (int t = 0; t < bs; ++t) acc -= AA(r, r0 + t) * AA(r0 + t, c);
      AA(r, c) = acc;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (st != nullptr) st[slot].singular = s_sing;
    if (info != nullptr) info[slot] = s_sing;
  }
}
#undef AA

template <class T>
void launch_lu_big_t(T* A, size_t stride, int n, int ncols, int lda, int* piv, int piv_stride,
                     SlotState* st, int want_phase, int want_job, int count, int* info,
                     hipStream_t stream, int nb) {
  if (count <= 0) return;
  if (nb == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    nb = lu_variant(dev, n, sizeof(T) == 4);
  }
  auto k = nb == 16     ? k_lu_big<T, 16, 16>
           : nb == 64   ? k_lu_big<T, 64, 64>
           : nb == 1664 ? k_lu_big<T, 16, 64>
           : nb == 3264 ? k_lu_big<T, 32, 64>
                        : k_lu_big<T, 32, 32>;
  hipLaunchKernelGGL(k, dim3(count), dim3(BIG_T), 0, stream, A, stride, n, ncols, lda, piv,
                     piv_stride, st, want_phase, want_job, info);
}

void launch_lu_big(double* A, size_t stride, int n, int ncols, int lda, int* piv,
                   int piv_stride, SlotState* st, int want_phase, int want_job, int count,
                   int* info, hipStream_t stream, int nb) {
  launch_lu_big_t(A, stride, n, ncols, lda, piv, piv_stride, st, want_phase, want_job, count,
                  info, stream, nb);
}

void launch_lu_big_f32(float* A, size_t stride, int n, int ncols, int lda, int* piv,
                       int piv_stride, SlotState* st, int want_phase, int want_job, int count,
                       int* info, hipStream_t stream, int nb) {
  launch_lu_big_t(A, stride, n, ncols, lda, piv, piv_stride, st, want_phase, want_job, count,
                  info, stream, nb);
}

// Synthetic systems for timing: entries from a counter hash in [-1, 1)
// (dense random matrices, so that partial pivoting interchanges rows at
// almost every column, as it does on the KKT systems).
template <class T>
__global__ void k_tune_fill(T* __restrict__ A, size_t stride, int n, int ncols, int lda,
                            unsigned seed) {
  const int slot = blockIdx.x;
  T* a = A + (size_t)slot * stride;
  for (long long e = threadIdx.x; e < (long long)n * ncols; e += blockDim.x) {
    const int r = (int)(e / ncols), c = (int)(e % ncols);
    unsigned h = (unsigned)e * 2654435761u ^ (unsigned)slot * 40503u ^ seed;
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    a[(size_t)r * lda + c] = T((double)h * (2.0 / 4294967296.0) - 1.0);
  }
}

void launch_tune_fill(void* A, bool f32, size_t stride, int n, int ncols, int lda, int count,
                      unsigned seed, hipStream_t stream) {
  if (f32)
    hipLaunchKernelGGL(k_tune_fill<float>, dim3(count), dim3(256), 0, stream,
                       static_cast<float*>(A), stride, n, ncols, lda, seed);
  else
    hipLaunchKernelGGL(k_tune_fill<double>, dim3(count), dim3(256), 0, stream,
                       static_cast<double*>(A), stride, n, ncols, lda, seed);
}

}  // namespace cs
