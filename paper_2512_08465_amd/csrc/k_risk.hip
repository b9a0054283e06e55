// Risk Index extensions (Section II.C, eq. (1)-(3), with the extensions that
// Section V.C lists as future work):
//   - a per-scenario severity weight: the binary S_c of the record, or a
//     damping-based continuous severity for secure scenarios,
//     S_c = clip((zeta_ref - zeta_min) / zeta_ref, 0, 1);
//   - common-cause pairs: F_ij = lambda_i lambda_j + lambda_cc(i, j);
//   - Monte-Carlo over M sampled failure-rate vectors.  With S1_i the summed
//     weight of the N-1 scenarios of i, S2 the symmetric matrix of summed
//     N-2 weights and C_i = sum over i's N-2 scenarios of lambda_cc S_c,
//         R(lambda) = lambda o (S1 + S2 lambda) + C,
//     so the M samples are one dense product Lambda S2 (M x n x n) on the
//     matrix cores with the rest fused into its epilogue; then each
//     component's rank in every sample, its rank histogram and quantiles,
//     and the mean and standard deviation of its R.
// Every sum runs in a fixed order, so results are identical run to run.
#include "cs_internal.h"
#include "../../include/cs.h"

namespace cs {

typedef double dvec4 __attribute__((ext_vector_type(4)));

__global__ void k_sev_weights(const cs_result* __restrict__ rec, long long n, int mode,
                              double zeta_ref, double* __restrict__ w) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const cs_result r = rec[c];
  double v = r.severe ? 1.0 : 0.0;
  if (!r.severe && mode == CS_SEV_DAMPING) {
    const double z = r.min_damping;
    v = __builtin_isfinite(z) ? fmin(fmax((zeta_ref - z) / zeta_ref, 0.0), 1.0) : 0.0;
  }
  w[c] = v;
}

void launch_sev_weights(const void* rec, long long n, int mode, double zeta_ref, double* w,
                        hipStream_t st) {
  if (n <= 0) return;
  const int t = 256;
  hipLaunchKernelGGL(k_sev_weights, dim3((unsigned)((n + t - 1) / t)), dim3(t), 0, st,
                     reinterpret_cast<const cs_result*>(rec), n, mode, zeta_ref, w);
}

// Symmetric common-cause table [n_comp][n_comp] from tagged pairs, built by
// one thread per row so that every entry sums its pairs in list order.
__global__ void k_cc_table(const int* __restrict__ pairs, const double* __restrict__ rate,
                           long long n_cc, int n_comp, double* __restrict__ T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_comp) return;
  double* row = T + (size_t)i * n_comp;
  for (long long k = 0; k < n_cc; ++k) {
    const int a = pairs[2 * k], b = pairs[2 * k + 1];
    if (a == i) row[b] += rate[k];
    else if (b == i) row[a] += rate[k];
  }
}

void launch_cc_table(const int* pairs, const double* rate, long long n_cc, int n_comp, double* T,
                     hipStream_t st) {
  if (n_comp <= 0) return;
  hipLaunchKernelGGL(k_cc_table, dim3((n_comp + 255) / 256), dim3(256), 0, st, pairs, rate, n_cc,
                     n_comp, T);
}

// R_i for one rate vector: one wavefront per component; each lane sums its
// strided share of the list in order, then a fixed butterfly (as k_risk).
__global__ __launch_bounds__(256) void k_risk_weighted(const int* __restrict__ outages,
                                                       long long n, const double* __restrict__ w,
                                                       const double* __restrict__ lam,
                                                       const double* __restrict__ cc,
                                                       int n_comp, double* __restrict__ risk) {
  const int comp = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (comp >= n_comp) return;
  double acc = 0.0;
  for (long long c = lane; c < n; c += 64) {
    const int a = outages[2 * c], b = outages[2 * c + 1];
    if ((a == comp || b == comp) && w[c] != 0.0) {
      double f;
      if (b < 0) {
        f = lam[a];
      } else {
        f = lam[a] * lam[b];
        if (cc != nullptr) f += cc[(size_t)a * n_comp + b];
      }
      acc += f * w[c];
    }
  }
  for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) risk[comp] = acc;
}

void launch_risk_weighted(const int* outages, long long n, const double* w, const double* lam,
                          const double* cc, int n_comp, double* risk, hipStream_t st) {
  if (n_comp <= 0) return;
  hipLaunchKernelGGL(k_risk_weighted, dim3((n_comp + 3) / 4), dim3(256), 0, st, outages, n, w,
                     lam, cc, n_comp, risk);
}

// S1, S2 (row stride ld) and C from the list: thread i owns row i and adds
// the scenarios that contain component i in list order (the list passes
// through LDS in chunks shared by the workgroup).
constexpr int SPLIT_CHUNK = 1024;

__global__ __launch_bounds__(256) void k_risk_split(const int* __restrict__ outages, long long n,
                                                    const double* __restrict__ w,
                                                    const double* __restrict__ cc, int n_comp,
                                                    int ld, double* __restrict__ S1,
                                                    double* __restrict__ S2,
                                                    double* __restrict__ C) {
  __shared__ int ids[2 * SPLIT_CHUNK];
  __shared__ double ws[SPLIT_CHUNK];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s1 = 0.0, cacc = 0.0;
  double* row = S2 + (size_t)(i < n_comp ? i : 0) * ld;
  for (long long c0 = 0; c0 < n; c0 += SPLIT_CHUNK) {
    const int cnt = (int)((n - c0) < SPLIT_CHUNK ? (n - c0) : SPLIT_CHUNK);
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
      ids[2 * k] = outages[2 * (c0 + k)];
      ids[2 * k + 1] = outages[2 * (c0 + k) + 1];
      ws[k] = w[c0 + k];
    }
    __syncthreads();
    if (i < n_comp) {
      for (int k = 0; k < cnt; ++k) {
        const int a = ids[2 * k], b = ids[2 * k + 1];
        if (a != i && b != i) continue;
        const double wk = ws[k];
        if (wk == 0.0) continue;
        if (b < 0) {
          s1 += wk;
        } else {
          const int j = (a == i) ? b : a;
          row[j] += wk;
          if (cc != nullptr) cacc += cc[(size_t)a * n_comp + b] * wk;
        }
      }
    }
  }
  if (i < n_comp) {
    S1[i] = s1;
    C[i] = cacc;
  }
}

void launch_risk_split(const int* outages, long long n, const double* w, const double* cc,
                       int n_comp, int ld, double* S1, double* S2, double* C, hipStream_t st) {
  if (n_comp <= 0) return;
  hipLaunchKernelGGL(k_risk_split, dim3((n_comp + 255) / 256), dim3(256), 0, st, outages, n, w,
                     cc, n_comp, ld, S1, S2, C);
}

// R[m][i] = L[m][i] (S1[i] + sum_j L[m][j] S2[j][i]) + C[i] for all samples m.
// Workgroup: 64 x 64 outputs, four wavefronts of 32 x 32 (2 x 2 tiles of the
// 16 x 16 x 4 FP64 matrix-core step); the k dimension passes through LDS in
// slices of 16.  Operand convention of v_mfma_f64_16x16x4f64: lane (li, lk) =
// (lane % 16, lane / 16) supplies A[li][lk] and B[lk][li], and its four
// accumulators hold column li of rows lk + 4 q.
constexpr int MC_T = 64, MC_K = 16;

__global__ __launch_bounds__(256) void k_risk_mc_gemm(const double* __restrict__ L, long long M,
                                                      int n, const double* __restrict__ S1,
                                                      const double* __restrict__ S2, int ld,
                                                      const double* __restrict__ C,
                                                      double* __restrict__ R) {
  __shared__ double As[MC_T][MC_K + 1];
  __shared__ double Bs[MC_K][MC_T + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const long long m0 = (long long)blockIdx.y * MC_T;
  const int i0 = blockIdx.x * MC_T;
  const int wr = 32 * (wave >> 1), wc = 32 * (wave & 1);
  dvec4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dvec4{0.0, 0.0, 0.0, 0.0};
  for (int j0 = 0; j0 < n; j0 += MC_K) {
    __syncthreads();
    for (int e = tid; e < MC_T * MC_K; e += 256) {
      const int r = e / MC_K, k = e % MC_K;
      const long long m = m0 + r;
      const int j = j0 + k;
      As[r][k] = (m < M && j < n) ? L[m * n + j] : 0.0;
    }
    for (int e = tid; e < MC_K * MC_T; e += 256) {
      const int k = e / MC_T, c = e % MC_T;
      const int j = j0 + k, i = i0 + c;
      Bs[k][c] = (j < n && i < n) ? S2[(size_t)j * ld + i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < MC_K; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = As[wr + 16 * t + li][kk + lk];
        b[t] = Bs[kk + lk][wc + 16 * t + li];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    }
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      const int i = i0 + wc + 16 * tj + li;
      if (i >= n) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long long m = m0 + wr + 16 * ti + lk + 4 * q;
        if (m < M) {
          const double lmi = L[m * n + i];
          R[m * n + i] = lmi * (S1[i] + acc[ti][tj][q]) + C[i];
        }
      }
    }
}

void launch_risk_mc_gemm(const double* L, long long M, int n, const double* S1, const double* S2,
                         int ld, const double* C, double* R, hipStream_t st) {
  if (M <= 0 || n <= 0) return;
  dim3 grid((n + MC_T - 1) / MC_T, (unsigned)((M + MC_T - 1) / MC_T));
  hipLaunchKernelGGL(k_risk_mc_gemm, grid, dim3(256), 0, st, L, M, n, S1, S2, ld, C, R);
}

// Rank of every component in sample m (0 = largest R, equal values by
// component id) into hist[i][rank]; one workgroup per sample, the sample's
// R in LDS.
__global__ __launch_bounds__(256) void k_rank_hist(const double* __restrict__ R, long long M,
                                                   int n, int* __restrict__ hist) {
  extern __shared__ double rrow[];
  const long long m = blockIdx.x;
  if (m >= M) return;
  for (int i = threadIdx.x; i < n; i += blockDim.x) rrow[i] = R[m * n + i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = rrow[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double u = rrow[j];
      rank += (u > v) || (u == v && j < i);
    }
    atomicAdd(&hist[(size_t)i * n + rank], 1);
  }
}

void launch_rank_hist(const double* R, long long M, int n, int* hist, hipStream_t st) {
  if (M <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_rank_hist, dim3((unsigned)M), dim3(256), sizeof(double) * (size_t)n, st, R,
                     M, n, hist);
}

// Per component: mean and sample standard deviation of R over the samples
// (sequential sums), and the rank quantiles q in {5, 50, 95} percent: the
// smallest rank whose cumulative count reaches ceil(q M / 100).
__global__ void k_risk_summary(const double* __restrict__ R, long long M, int n,
                               const int* __restrict__ hist, double* __restrict__ moments,
                               int* __restrict__ rank_q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (moments != nullptr) {
    double s = 0.0;
    for (long long m = 0; m < M; ++m) s += R[m * n + i];
    const double mean = s / (double)M;
    double v = 0.0;
    for (long long m = 0; m < M; ++m) {
      const double d = R[m * n + i] - mean;
      v += d * d;
    }
    moments[2 * i] = mean;
    moments[2 * i + 1] = M > 1 ? sqrt(v / (double)(M - 1)) : 0.0;
  }
  if (rank_q != nullptr) {
    const int qs[3] = {5, 50, 95};
    long long need[3];
    for (int k = 0; k < 3; ++k) {
      need[k] = (qs[k] * M + 99) / 100;
      if (need[k] < 1) need[k] = 1;
    }
    long long cum = 0;
    int k = 0;
    for (int r = 0; r < n && k < 3; ++r) {
      cum += hist[(size_t)i * n + r];
      while (k < 3 && cum >= need[k]) rank_q[3 * i + k++] = r;
    }
  }
}

void launch_risk_summary(const double* R, long long M, int n, const int* hist, double* moments,
                         int* rank_q, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_risk_summary, dim3((n + 255) / 256), dim3(256), 0, st, R, M, n, hist,
                     moments, rank_q);
}

}  // namespace cs
