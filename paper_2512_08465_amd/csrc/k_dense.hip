// Batched dense LU with partial pivoting and solve (one workgroup per matrix).
//
// Each Newton step of the OPF solves one dense KKT system, and the state
// matrix needs g_y^{-1} g_x; both go through this kernel.  The matrix is
// column-major [lda][ncols] with the right-hand sides as columns n..ncols-1
// (an augmented matrix), so the forward substitution falls out of the
// elimination and only the back substitution with U remains.
//
// Right-looking blocked LU, panel width NB:
//   1. the m x NB panel is staged in LDS and factorised there (pivot = first
//      largest |a| in the column, row swap, scale, rank-1 update);
//   2. the panel's row interchanges are applied to every other column, and the
//      NB x (ncols-k0-NB) block row is solved with the unit lower L11 (TRSM);
//   3. the trailing matrix is updated, A22 -= L21 U12, with FP64 MFMA
//      (v_mfma_f64_16x16x4f64), 16 x 16 tiles per wave, L21 read from LDS;
//      each tile is formed transposed so its rows map onto lanes.
// After the last panel, U x = y is solved by 16-row blocks from the bottom.
#include "cs_internal.h"

namespace cs {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int LU_NB = 16;
constexpr int LU_THREADS = 256;

__device__ inline void argmax_combine(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

__global__ __launch_bounds__(LU_THREADS) void k_lu_solve(
    double* __restrict__ Abase, size_t stride, int n, int ncols, int lda,
    int* __restrict__ pivbase, int piv_stride, SlotState* __restrict__ st,
    int* __restrict__ info) {
  const int slot = blockIdx.x;
  if (st != nullptr && st[slot].job == 0) return;
  double* __restrict__ A = Abase + (size_t)slot * stride;
  int* __restrict__ piv = pivbase + (size_t)slot * piv_stride;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  extern __shared__ double P[];          // panel, column-major, ld = ldp
  __shared__ double red_v[LU_THREADS / 64];
  __shared__ int red_i[LU_THREADS / 64];
  __shared__ int s_p;
  __shared__ int s_piv[LU_NB];
  __shared__ int s_sing;
  __shared__ double s_ub[LU_NB * LU_NB];
  const int ldp = n + 1;
  if (tid == 0) s_sing = 0;

  for (int k0 = 0; k0 < n; k0 += LU_NB) {
    const int kb = min(LU_NB, n - k0);
    const int m = n - k0;
    // ---- 1. stage the panel A[k0:n, k0:k0+kb] in LDS
    for (int c = 0; c < kb; ++c)
      for (int r = tid; r < m; r += LU_THREADS)
        P[r + ldp * c] = A[(size_t)(k0 + c) * lda + k0 + r];
    __syncthreads();
    // ---- factorise the panel
    for (int j = 0; j < kb; ++j) {
      double bv = -1.0;
      int bi = j;
      for (int r = j + tid; r < m; r += LU_THREADS) {
        double a = fabs(P[r + ldp * j]);
        if (a > bv) { bv = a; bi = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        double v2 = __shfl_xor(bv, off, 64);
        int i2 = __shfl_xor(bi, off, 64);
        argmax_combine(bv, bi, v2, i2);
      }
      if (lane == 0) { red_v[wave] = bv; red_i[wave] = bi; }
      __syncthreads();
      if (tid == 0) {
        double v = red_v[0];
        int i = red_i[0];
        for (int w = 1; w < LU_THREADS / 64; ++w) argmax_combine(v, i, red_v[w], red_i[w]);
        s_p = i;
        s_piv[j] = i;
        piv[k0 + j] = k0 + i;
      }
      __syncthreads();
      const int p = s_p;
      if (p != j && tid < kb) {
        double t = P[j + ldp * tid];
        P[j + ldp * tid] = P[p + ldp * tid];
        P[p + ldp * tid] = t;
      }
      __syncthreads();
      const double pv = P[j + ldp * j];
      if (pv == 0.0) {
        if (tid == 0) s_sing = 1;
      } else {
        const double inv = 1.0 / pv;
        for (int r = j + 1 + tid; r < m; r += LU_THREADS) {
          double l = P[r + ldp * j] * inv;
          P[r + ldp * j] = l;
          for (int c = j + 1; c < kb; ++c) P[r + ldp * c] -= l * P[j + ldp * c];
        }
      }
      __syncthreads();
    }
    // ---- write the factored panel back
    for (int c = 0; c < kb; ++c)
      for (int r = tid; r < m; r += LU_THREADS)
        A[(size_t)(k0 + c) * lda + k0 + r] = P[r + ldp * c];
    // ---- 2. interchanges on the other columns; TRSM on the block row
    for (int c = tid; c < ncols; c += LU_THREADS) {
      if (c >= k0 && c < k0 + kb) continue;
      double* col = A + (size_t)c * lda;
      for (int j = 0; j < kb; ++j) {
        const int p = s_piv[j];
        if (p != j) {
          double t = col[k0 + j];
          col[k0 + j] = col[k0 + p];
          col[k0 + p] = t;
        }
      }
      if (c >= k0 + kb) {
        double u[LU_NB];
#pragma unroll
        for (int j = 0; j < LU_NB; ++j) u[j] = (j < kb) ? col[k0 + j] : 0.0;
#pragma unroll
        for (int j = 0; j < LU_NB; ++j) {
#pragma unroll
          for (int i = j + 1; i < LU_NB; ++i)
            if (i < kb) u[i] -= P[i + ldp * j] * u[j];
        }
#pragma unroll
        for (int j = 0; j < LU_NB; ++j)
          if (j < kb) col[k0 + j] = u[j];
      }
    }
    __syncthreads();
    // ---- 3. trailing update A22 -= L21 * U12 on MFMA
    const int r0 = k0 + kb;
    const int rows = n - r0;
    const int cols = ncols - r0;
    if (rows > 0 && cols > 0) {
      const int tr = (rows + 15) >> 4;
      const int tc = (cols + 15) >> 4;
      const int ntiles = tr * tc;
      // The tile is computed transposed, C^T -= U12^T L21^T, so that the
      // accumulator layout of v_mfma_f64_16x16x4f64 (lane l, register q holds
      // D[l/16 + 4q][l%16]) puts C rows on lanes: lane l owns row i0 + l%16
      // of columns j0 + l/16 + 4q, and 16 lanes cover 16 consecutive doubles.
      const int li = lane & 15;
      const int lk = lane >> 4;
      for (int t = wave; t < ntiles; t += LU_THREADS / 64) {
        const int ti = t % tr;
        const int tj = t / tr;
        const int i0 = r0 + 16 * ti;
        const int j0 = r0 + 16 * tj;
        const int row = i0 + li;
        const bool rok = row < n;
        dbl4 acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int col = j0 + lk + 4 * q;
          acc[q] = (rok && col < ncols) ? A[(size_t)col * lda + row] : 0.0;
        }
        const int ucol = j0 + li;           // column of the U12 entry
        const bool uok = ucol < ncols;
        const double* up = A + (size_t)ucol * lda + k0;
        const double* lp = P + (row - k0);
#pragma unroll
        for (int kk = 0; kk < LU_NB / 4; ++kk) {
          const int k = 4 * kk + lk;
          double a = 0.0, b = 0.0;
          if (k < kb) {
            if (uok) a = -up[k];
            if (rok) b = lp[(size_t)ldp * k];
          }
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int col = j0 + lk + 4 * q;
          if (rok && col < ncols) A[(size_t)col * lda + row] = acc[q];
        }
      }
    }
    __syncthreads();
  }

  // ---- back substitution U x = y for the right-hand-side columns
  const int nrhs = ncols - n;
  if (nrhs > 0) {
    const int nblk = (n + LU_NB - 1) / LU_NB;
    for (int b = nblk - 1; b >= 0; --b) {
      const int b0 = b * LU_NB;
      const int bs = min(LU_NB, n - b0);
      for (int e = tid; e < LU_NB * LU_NB; e += LU_THREADS) {
        const int i = e % LU_NB, j = e / LU_NB;
        s_ub[e] = (i < bs && j < bs) ? A[(size_t)(b0 + j) * lda + b0 + i] : 0.0;
      }
      __syncthreads();
      for (int rc = tid; rc < nrhs; rc += LU_THREADS) {
        double* y = A + (size_t)(n + rc) * lda + b0;
        double v[LU_NB];
#pragma unroll
        for (int i = 0; i < LU_NB; ++i) v[i] = (i < bs) ? y[i] : 0.0;
#pragma unroll
        for (int i = LU_NB - 1; i >= 0; --i) {
          if (i < bs) {
            double s = v[i];
#pragma unroll
            for (int j = i + 1; j < LU_NB; ++j)
              if (j < bs) s -= s_ub[i + LU_NB * j] * v[j];
            v[i] = s / s_ub[i + LU_NB * i];
          }
        }
#pragma unroll
        for (int i = 0; i < LU_NB; ++i)
          if (i < bs) y[i] = v[i];
      }
      __syncthreads();
      // y[0:b0] -= U[0:b0, b0:b0+bs] x[b0:b0+bs]
      const int work = b0 * nrhs;
      for (int e = tid; e < work; e += LU_THREADS) {
        const int i = e % b0, rc = e / b0;
        double* y = A + (size_t)(n + rc) * lda;
        double s = y[i];
        for (int j = 0; j < bs; ++j) s -= A[(size_t)(b0 + j) * lda + i] * y[b0 + j];
        y[i] = s;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (st != nullptr) st[slot].singular = s_sing;
    if (info != nullptr) info[slot] = s_sing;
  }
}

void launch_lu_solve(double* A, size_t stride, int n, int ncols, int lda,
                     int* piv, int piv_stride, SlotState* st, int count,
                     int* info, hipStream_t stream) {
  if (count <= 0) return;
  const size_t lds = sizeof(double) * (size_t)LU_NB * (size_t)(n + 1);
  hipLaunchKernelGGL(k_lu_solve, dim3(count), dim3(LU_THREADS), lds, stream,
                     A, stride, n, ncols, lda, piv, piv_stride, st, info);
}

size_t lu_lds_bytes(int n) { return sizeof(double) * (size_t)LU_NB * (size_t)(n + 1); }

void lu_set_attrs(size_t bytes) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(k_lu_solve),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace cs
