// Batched dense LU with partial pivoting and solve (one workgroup per matrix).
//
// Each Newton step of the OPF solves one dense KKT system, and the state
// matrix needs g_y^{-1} g_x; both go through this kernel.  The matrix is
// row-major, rows of stride lda, with the right-hand sides stored as columns
// n..ncols-1 (an augmented matrix): the forward substitution falls out of the
// elimination and only the back substitution with U remains.
//
// Right-looking blocked LU with panel width NB = 16 and one panel of
// look-ahead, eight wavefronts per matrix.  The panel being factorised lives
// in LDS.  Per panel k (its factors in LDS, pivots known):
//   A. all waves: write the panel back, apply its row interchanges to every
//      other column (the panel's swaps compose to one permutation of at most
//      2 NB rows; each thread gathers its column's affected rows, then
//      scatters them), then form the block row U12 = inv(L11) A12 with MFMA
//      (inv(L11), the inverse of the panel's unit lower triangle, is built by
//      wave 0 with the panel);
//   B. all waves: update the next panel's NB columns with L21 U12, writing the
//      result straight into the LDS panel buffer;
//   C. wave 0 factorises that panel in LDS (pivot = first largest |a| in the
//      column, row swap, scale, rank-1 update; wavefront shuffles only, no
//      workgroup barrier), while the other waves update the rest of the
//      trailing matrix, A22 -= L21 U12, with FP64 MFMA (v_mfma_f64_16x16x4f64)
//      on 32 x 32 groups of four 16 x 16 tiles taken from a shared counter;
//      wave 0 joins the tile loop when its panel is done.
// After the last panel, U x = y is solved by 16-row blocks from the bottom.
#include "cs_internal.h"

#include <algorithm>

namespace cs {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int LU_NB = 16;
constexpr int LU_THREADS = 512;
constexpr int LU_WAVES = LU_THREADS / 64;
constexpr int PLD = LU_NB + 1;        // LDS row stride of the panel (bank spread)
constexpr int LU_NSW = 2 * LU_NB;     // rows a panel's interchanges can touch

__device__ inline void wave_sync() {
  // LDS accesses of one wavefront complete in issue order; this only stops
  // the compiler from moving memory operations across the point.
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline void argmax_combine(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

// Factorise the m x kb panel held in LDS (P, rows relative to the panel's
// first row r0) with one wavefront.  Pivots (relative) go to spiv[], absolute
// to piv[]; linv receives the inverse of the panel's unit lower triangle and
// sw[] the panel's net row permutation as (destination << 16 | source) pairs
// of relative rows, -1 for unused entries.  ridx[] is scratch of m ints.
__device__ void panel_factor(double* __restrict__ P, int m, int r0, int kb,
                             double* __restrict__ linv, int* __restrict__ spiv,
                             int* __restrict__ piv, int* __restrict__ ridx,
                             int* __restrict__ sw, int* sing, int lane) {
  for (int r = lane; r < m; r += 64) ridx[r] = r;
  wave_sync();
  for (int j = 0; j < kb; ++j) {
    double bv = -1.0;
    int bi = j;
    for (int r = j + lane; r < m; r += 64) {
      const double a = fabs(P[r * PLD + j]);
      if (a > bv) { bv = a; bi = r; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double v2 = __shfl_xor(bv, off, 64);
      const int i2 = __shfl_xor(bi, off, 64);
      argmax_combine(bv, bi, v2, i2);
    }
    const int p = bi;                 // uniform across the wavefront
    if (lane == 0) {
      spiv[j] = p;
      piv[r0 + j] = r0 + p;
    }
    if (p != j) {
      if (lane < kb) {
        const double t = P[j * PLD + lane];
        P[j * PLD + lane] = P[p * PLD + lane];
        P[p * PLD + lane] = t;
      } else if (lane == LU_NB) {
        const int t = ridx[j];
        ridx[j] = ridx[p];
        ridx[p] = t;
      }
    }
    wave_sync();
    const double pv = P[j * PLD + j];
    if (pv == 0.0) {
      if (lane == 0) *sing = 1;
    } else {
      const double inv = 1.0 / pv;
      for (int r = j + 1 + lane; r < m; r += 64) {
        double* row = P + r * PLD;
        const double l = row[j] * inv;
        row[j] = l;
        for (int c = j + 1; c < kb; ++c) row[c] -= l * P[j * PLD + c];
      }
    }
    wave_sync();
  }
  // net permutation: position t < kb now holds original row ridx[t]; a pivot
  // position q = spiv[t] >= kb holds ridx[q] (counted once if repeated)
  if (lane < LU_NB) {
    const int t = lane;
    int e0 = -1, e1 = -1;
    if (t < kb) {
      if (ridx[t] != t) e0 = (t << 16) | ridx[t];
      const int q = spiv[t];
      bool first = q >= kb;
      for (int u = 0; u < t; ++u) first = first && spiv[u] != q;
      if (first && ridx[q] != q) e1 = (q << 16) | ridx[q];
    }
    sw[2 * t] = e0;
    sw[2 * t + 1] = e1;
  }
  // inverse of the unit lower triangle L11 (kb x kb, identity-padded to 16):
  // lane j forms column j by forward substitution
  if (lane < LU_NB) {
    const int j = lane;
    for (int i = 0; i < LU_NB; ++i) {
      double v = (i == j) ? 1.0 : 0.0;
      if (i > j && i < kb) {
        v = 0.0;
        for (int k = j; k < i; ++k) v -= P[i * PLD + k] * linv[k * LU_NB + j];
      }
      linv[i * LU_NB + j] = v;
    }
  }
  wave_sync();
}

// C[i0:i0+16, j0:j0+16] - L21[i0:, k0:k0+kb] U12[k0:k0+kb, j0:] (global
// rows) for rows < n and columns < ncols; the result goes to the LDS panel
// buffer P (rows relative to j0, which is also the panel's first row)
__device__ inline void update_tile_to_panel(const double* __restrict__ A, int lda, int n,
                                            int ncols, int k0, int kb, int i0, int j0,
                                            double* __restrict__ P, int lane) {
  const int li = lane & 15, lk = lane >> 4;
  // accumulator layout of the f64 16x16x4 MFMA: lane l, register q holds
  // D[l/16 + 4q][l%16]; D is the tile itself, so 16 lanes cover 16
  // consecutive doubles of one row.
  const int col = j0 + li;
  const bool cok = col < ncols;
  dbl4 acc;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = i0 + lk + 4 * q;
    acc[q] = (cok && row < n) ? A[(size_t)row * lda + col] : 0.0;
  }
  const int arow = i0 + li;
  const bool aok = arow < n;
  const double* lrow = A + (size_t)arow * lda + k0;
  double a[LU_NB / 4], b[LU_NB / 4];
#pragma unroll
  for (int kk = 0; kk < LU_NB / 4; ++kk) {
    const int k = 4 * kk + lk;
    a[kk] = (k < kb && aok) ? -lrow[k] : 0.0;
    b[kk] = (k < kb && cok) ? A[(size_t)(k0 + k) * lda + col] : 0.0;
  }
#pragma unroll
  for (int kk = 0; kk < LU_NB / 4; ++kk)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], b[kk], acc, 0, 0, 0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = i0 + lk + 4 * q;
    if (cok && row < n) P[(row - j0) * PLD + li] = acc[q];
  }
}

// The same update on a 32 x 32 group of four tiles: all 32 loads of a lane
// are issued together and every L21 / U12 operand feeds two MFMAs.
__device__ inline void update_group(double* __restrict__ A, int lda, int n, int ncols,
                                    int k0, int kb, int i0, int j0, int lane) {
  const int li = lane & 15, lk = lane >> 4;
  dbl4 acc[2][2];
  int col[2];
  bool cok[2];
#pragma unroll
  for (int tj = 0; tj < 2; ++tj) {
    col[tj] = j0 + 16 * tj + li;
    cok[tj] = col[tj] < ncols;
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = i0 + 16 * ti + lk + 4 * q;
        acc[ti][tj][q] = (cok[tj] && row < n) ? A[(size_t)row * lda + col[tj]] : 0.0;
      }
  double a[2][LU_NB / 4], b[2][LU_NB / 4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti) {
    const int arow = i0 + 16 * ti + li;
    const double* lrow = A + (size_t)arow * lda + k0;
#pragma unroll
    for (int kk = 0; kk < LU_NB / 4; ++kk) {
      const int k = 4 * kk + lk;
      a[ti][kk] = (k < kb && arow < n) ? -lrow[k] : 0.0;
    }
  }
#pragma unroll
  for (int tj = 0; tj < 2; ++tj)
#pragma unroll
    for (int kk = 0; kk < LU_NB / 4; ++kk) {
      const int k = 4 * kk + lk;
      b[tj][kk] = (k < kb && cok[tj]) ? A[(size_t)(k0 + k) * lda + col[tj]] : 0.0;
    }
#pragma unroll
  for (int kk = 0; kk < LU_NB / 4; ++kk)
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti][kk], b[tj][kk], acc[ti][tj], 0, 0, 0);
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = i0 + 16 * ti + lk + 4 * q;
        if (cok[tj] && row < n) A[(size_t)row * lda + col[tj]] = acc[ti][tj][q];
      }
}

__global__ __launch_bounds__(LU_THREADS, 1) void k_lu_solve(
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

  extern __shared__ double P[];          // panel rows, stride PLD; then ridx
  int* ridx = reinterpret_cast<int*>(P + (size_t)PLD * n);
  __shared__ int s_piv[LU_NB];
  __shared__ int s_sw[LU_NSW];
  __shared__ int s_sing;
  __shared__ int s_tile;
  __shared__ double s_ub[LU_NB * LU_NB];
  __shared__ double s_linv[LU_NB * LU_NB];
  if (tid == 0) s_sing = 0;
  {
    const int kb = min(LU_NB, n);
    for (int e = tid; e < n * kb; e += LU_THREADS) {
      const int r = e / kb, c = e - r * kb;
      P[r * PLD + c] = A[(size_t)r * lda + c];
    }
  }
  __syncthreads();
  if (wave == 0)
    panel_factor(P, n, 0, min(LU_NB, n), s_linv, s_piv, piv, ridx, s_sw, &s_sing, lane);
  __syncthreads();

  for (int k0 = 0; k0 < n; k0 += LU_NB) {
    const int kb = min(LU_NB, n - k0);
    const int m = n - k0;
    const int r0 = k0 + kb;
    // ---- A: write the panel back, interchanges, TRSM of the block row
    for (int e = tid; e < m * kb; e += LU_THREADS) {
      const int r = e / kb, c = e - r * kb;
      A[(size_t)(k0 + r) * lda + k0 + c] = P[r * PLD + c];
    }
    {
      int sw[LU_NSW];
#pragma unroll
      for (int e = 0; e < LU_NSW; ++e) sw[e] = s_sw[e];
      for (int c = tid; c < ncols; c += LU_THREADS) {
        if (c >= k0 && c < r0) continue;
        double* colp = A + (size_t)k0 * lda + c;
        double v[LU_NSW];
#pragma unroll
        for (int e = 0; e < LU_NSW; ++e)
          v[e] = (sw[e] >= 0) ? colp[(size_t)(sw[e] & 0xffff) * lda] : 0.0;
#pragma unroll
        for (int e = 0; e < LU_NSW; ++e)
          if (sw[e] >= 0) colp[(size_t)(sw[e] >> 16) * lda] = v[e];
      }
    }
    __syncthreads();
    // U12 = inv(L11) A12 on MFMA, one 16-column tile per wavefront pass
    {
      const int li = lane & 15, lk = lane >> 4;
      const int ntc = (ncols - r0 + 15) >> 4;
      for (int t = wave; t < ntc; t += LU_WAVES) {
        const int col = r0 + 16 * t + li;
        const bool cok = col < ncols;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        double a[LU_NB / 4], b[LU_NB / 4];
#pragma unroll
        for (int kk = 0; kk < LU_NB / 4; ++kk) {
          const int k = 4 * kk + lk;
          a[kk] = s_linv[li * LU_NB + k];
          b[kk] = (cok && k < kb) ? A[(size_t)(k0 + k) * lda + col] : 0.0;
        }
#pragma unroll
        for (int kk = 0; kk < LU_NB / 4; ++kk)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], b[kk], acc, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = lk + 4 * q;
          if (cok && row < kb) A[(size_t)(k0 + row) * lda + col] = acc[q];
        }
      }
    }
    if (tid == 0) s_tile = 0;
    __syncthreads();
    if (r0 >= n) break;     // last panel: the right-hand sides were done by TRSM
    // ---- B: bring the next panel's columns up to date, into LDS
    const int kb2 = min(LU_NB, n - r0);
    const int tr = (n - r0 + 15) >> 4;
    for (int t = wave; t < tr; t += LU_WAVES)   // columns [r0, r0 + kb2) only
      update_tile_to_panel(A, lda, n, r0 + kb2, k0, kb, r0 + 16 * t, r0, P, lane);
    __syncthreads();
    // ---- C: wave 0 factorises the next panel; everyone updates the rest
    if (wave == 0)
      panel_factor(P, n - r0, r0, kb2, s_linv, s_piv, piv, ridx, s_sw, &s_sing, lane);
    const int c2 = r0 + kb2;
    if (c2 < ncols) {
      const int gr = (n - r0 + 31) >> 5;
      const int gc = (ncols - c2 + 31) >> 5;
      const int ngroups = gr * gc;
      while (true) {
        int t = 0;
        if (lane == 0) t = atomicAdd(&s_tile, 1);
        t = __shfl(t, 0, 64);
        if (t >= ngroups) break;
        const int ti = t % gr, tj = t / gr;
        update_group(A, lda, n, ncols, k0, kb, r0 + 32 * ti, c2 + 32 * tj, lane);
      }
    }
    __syncthreads();
  }

  // ---- back substitution U x = y for the right-hand-side columns, by
  // 16-row blocks from the bottom.  A wavefront solves a diagonal block for
  // one right-hand side at a time (lane i holds row i; x_i is broadcast and
  // eliminated from the rows above), the block solution is kept in LDS (the
  // panel buffer is free now), then every row above is updated.
  const int nrhs = ncols - n;
  if (nrhs > 0) {
    double* xs = P;                                 // [16][nrhs]
    const int nblk = (n + LU_NB - 1) / LU_NB;
    for (int b = nblk - 1; b >= 0; --b) {
      const int b0 = b * LU_NB;
      const int bs = min(LU_NB, n - b0);
      for (int e = tid; e < LU_NB * LU_NB; e += LU_THREADS) {
        const int i = e / LU_NB, j = e % LU_NB;
        s_ub[e] = (i < bs && j < bs) ? A[(size_t)(b0 + i) * lda + b0 + j] : 0.0;
      }
      __syncthreads();
      for (int rc = wave; rc < nrhs; rc += LU_WAVES) {
        double y = (lane < bs) ? A[(size_t)(b0 + lane) * lda + n + rc] : 0.0;
        for (int i = bs - 1; i >= 0; --i) {
          const double xi = __shfl(y, i, 64) / s_ub[i * LU_NB + i];
          if (lane == i) y = xi;
          if (lane < i) y -= s_ub[lane * LU_NB + i] * xi;
        }
        if (lane < bs) {
          xs[lane * nrhs + rc] = y;
          A[(size_t)(b0 + lane) * lda + n + rc] = y;
        }
      }
      __syncthreads();
      // y[0:b0] -= U[0:b0, b0:b0+bs] x[b0:b0+bs]
      const int work = b0 * nrhs;
      for (int e = tid; e < work; e += LU_THREADS) {
        const int i = e / nrhs, rc = e % nrhs;
        const double* urow = A + (size_t)i * lda + b0;
        double acc = A[(size_t)i * lda + n + rc];
        for (int j = 0; j < bs; ++j) acc -= urow[j] * xs[j * nrhs + rc];
        A[(size_t)i * lda + n + rc] = acc;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (st != nullptr) st[slot].singular = s_sing;
    if (info != nullptr) info[slot] = s_sing;
  }
}

// static LDS of k_lu_solve
constexpr size_t LU_STATIC_LDS =
    sizeof(int) * (LU_NB + LU_NSW + 2) + sizeof(double) * 2 * LU_NB * LU_NB;

// dynamic LDS: panel rows and their row-index scratch during the
// factorisation; a 16 x nrhs block during the solve
static size_t lu_dynamic_lds(int n, int nrhs) {
  return std::max(sizeof(double) * (size_t)PLD * (size_t)n + sizeof(int) * (size_t)n,
                  sizeof(double) * (size_t)LU_NB * (size_t)nrhs);
}

// total LDS one workgroup of k_lu_solve needs for order n and nrhs columns
size_t lu_lds_bytes(int n, int nrhs) { return lu_dynamic_lds(n, nrhs) + LU_STATIC_LDS; }

void launch_lu_solve(double* A, size_t stride, int n, int ncols, int lda,
                     int* piv, int piv_stride, SlotState* st, int count,
                     int* info, hipStream_t stream) {
  if (count <= 0) return;
  const size_t lds = lu_dynamic_lds(n, ncols - n);
  hipLaunchKernelGGL(k_lu_solve, dim3(count), dim3(LU_THREADS), lds, stream,
                     A, stride, n, ncols, lda, piv, piv_stride, st, info);
}



void lu_set_attrs(size_t bytes) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(k_lu_solve),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)(bytes - LU_STATIC_LDS));
}

}  // namespace cs
