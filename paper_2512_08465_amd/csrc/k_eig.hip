// Batched nonsymmetric eigenvalues (one workgroup per matrix).
//
// The small-signal test needs every eigenvalue of the state matrix.  Each
// matrix is reduced to upper Hessenberg form by Householder reflections in
// panels of 16 (one read-only pass over the trailing columns per reflector,
// one read-write update per panel on the matrix cores), then
// implicit QR sweeps run on the active window [lo, hi] until every 1x1 or
// 2x2 diagonal block has split off (eigenvalues only, so updates stay inside
// the window).  A sweep chases a chain of up to four double-shift bulges in
// blocks of 16 steps through a small diagonal block held in LDS and applies
// the accumulated reflectors to the rest of the window once per block, as
// small products on the FP64 matrix cores.
// Deflation: a subdiagonal entry is negligible when |h(k,k-1)| <= eps
// (|h(k-1,k-1)| + |h(k,k)|).  Every tenth sweep without deflation uses an
// exceptional shift.  The matrix lives in global memory (column-major, lda),
// with 64 n doubles of global scratch per matrix for the reduction's panel
// products; the reflector vectors, the reduction's partial sums, the chased
// block and the shift computation live in LDS.
#include "cs_internal.h"
#include <float.h>

namespace cs {

constexpr int EIG_THREADS = 256;
constexpr int EIG_NMAX = 1024;

__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < EIG_THREADS / 64; ++w) s += red[w];
  return s;
}

__device__ inline int block_max_int(int v, int* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  int s = red[0];
  for (int w = 1; w < EIG_THREADS / 64; ++w) s = max(s, red[w]);
  return s;
}

// eigenvalues of [[a, b], [c, d]]
__device__ inline void eig2x2(double a, double b, double c, double d,
                              double& r1, double& i1, double& r2, double& i2) {
  const double p = 0.5 * (a - d);
  const double bc = b * c;
  const double disc = p * p + bc;
  if (disc >= 0.0) {
    const double s = sqrt(disc);
    const double zz = p + copysign(s, p);
    if (zz == 0.0) {
      r1 = r2 = d;
    } else {
      r1 = d + zz;
      r2 = d - bc / zz;
    }
    i1 = i2 = 0.0;
  } else {
    r1 = r2 = d + p;
    i1 = sqrt(-disc);
    i2 = -i1;
  }
}

constexpr int EIG_NW = EIG_THREADS / 64;
constexpr int EIG_CG = 8;                   // row chunks of 64 loaded together

// Blocked Householder reduction to upper Hessenberg form (compact WY:
// Dongarra, Hammarling and Sorensen; the panel recurrences as in LAPACK's
// gehrd).  Reflector j of the panel starting at column k0 (column c = k0 + j)
// is H_j = I - tau_j v_j v_j^T with v_j = 1 at row c + 1, zero above; the
// panel's product is Q = I - V T V^T.  Per reflector:
//   1. column c is brought up to date: the right-hand part of the panel's
//      earlier reflectors, h -= Y V[c, :]^T (Y = A V T, all rows), then the
//      left-hand part on rows k0+1.., h -= V (T^T (V^T h));
//   2. the reflector is formed from rows c+1.. of h (v stored below the
//      subdiagonal of column c until the panel ends);
//   3. one read-only pass over the columns right of c of the panel-start
//      matrix A gives y = A v (all rows) and z[col] = v^T A[:, col] for the
//      columns right of the panel;
//   4. Y[:, j] = tau (y - Y (V^T v)), and column j of T.
// After the panel, with M = V^T Y, every column right of the panel takes
//   A[:, col] -= Y a + V w,  a = V[col, :]^T,  w = T^T (z[col] - M a)
// in one read-write pass, a K = 32 product on the FP64 matrix cores.  The
// trailing columns are thus read once per reflector and read and written once
// per panel of HB_NB reflectors, instead of read and written once per
// reflector.  Scratch (global, per matrix, 4 HB_NB n doubles): Y, z and the
// right-hand operand [a; w] of the panel's update.  LDS: the column or the
// reflector (n), the wavefronts' partial products (EIG_NW n), T, M and small
// vectors.
constexpr int HB_NB = 16;
static_assert(HB_NB == 16 && EIG_THREADS == 256, "16 x 16 panel products, one entry per thread");
typedef double EigMfma __attribute__((ext_vector_type(4)));

size_t eig_scratch_doubles(int n) { return 4 * (size_t)HB_NB * (size_t)n; }

// entry (row i, reflector l) of the panel's V: 1 at row k0 + l + 1, the
// stored vector below it, 0 above
__device__ inline double vget(const double* __restrict__ H, int lda, int k0, int l, int i) {
  const int c = k0 + l;
  return i == c + 1 ? 1.0 : (i > c + 1 ? H[(size_t)c * lda + i] : 0.0);
}

// out[l] = sum_i V[i][l] x[i] for l < j: 16 row groups of threads per l,
// partials in part[16][16] added in a fixed order
__device__ inline void panel_dots(const double* __restrict__ H, int lda, int k0, int j,
                                  const double* __restrict__ x, int n, double* part,
                                  double* out) {
  const int tid = threadIdx.x, l = tid & 15, g = tid >> 4;
  double acc = 0.0;
  if (l < j) {
#pragma unroll 4
    for (int i = k0 + l + 1 + g; i < n; i += 16) acc += vget(H, lda, k0, l, i) * x[i];
  }
  part[g * 16 + l] = acc;
  __syncthreads();
  if (tid < j) {
    double s = 0.0;
#pragma unroll
    for (int gg = 0; gg < 16; ++gg) s += part[gg * 16 + tid];
    out[tid] = s;
  }
  __syncthreads();
}

size_t eig_hess_lds_doubles(int n) {
  return (size_t)(1 + EIG_NW) * n + 2 * HB_NB * HB_NB + EIG_NW * 256 + 2 * HB_NB;
}

__device__ void hessenberg(double* __restrict__ H, int n, int lda, double* __restrict__ lds,
                           double* red, double* __restrict__ scr) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#define HH(i, j) H[(size_t)(j) * lda + (i)]
  double* hc = lds;                          // [n] column c, then v_j by row
  double* pn = hc + n;                       // [EIG_NW][n] partial y per wavefront
  double* Tm = pn + EIG_NW * n;              // [HB_NB][HB_NB] T, row-major
  double* Mm = Tm + HB_NB * HB_NB;           // [HB_NB][HB_NB] M = V^T Y
  double* part = Mm + HB_NB * HB_NB;         // [EIG_NW][16][16] partial sums
  double* sv1 = part + EIG_NW * 16 * 16;     // [HB_NB]
  double* sv2 = sv1 + HB_NB;                 // [HB_NB]
  double* Ys = scr;                          // [HB_NB][n], column l at l * n
  double* Zs = Ys + HB_NB * (size_t)n;       // [HB_NB][n]
  double* Bs = Zs + HB_NB * (size_t)n;       // [2 HB_NB][n]: a (rows 0..15), w (16..31)
  __shared__ double s_tau, s_beta, s_scale;
  for (int k0 = 0; k0 < n - 2; k0 += HB_NB) {
    const int kb = min(HB_NB, n - 2 - k0);
    const int cfirst = k0 + kb;              // first column right of the panel
    for (int e = tid; e < HB_NB * HB_NB; e += EIG_THREADS) Tm[e] = 0.0;
    for (int j = 0; j < kb; ++j) {
      const int c = k0 + j;
      // ---- 1. column c up to date
      for (int i = tid; i < n; i += EIG_THREADS) hc[i] = HH(i, c);
      if (j > 0) {
        if (tid < j) sv1[tid] = vget(H, lda, k0, tid, c);   // row c of V
        __syncthreads();
        for (int i = tid; i < n; i += EIG_THREADS) {
          double acc = hc[i];
          for (int l = 0; l < j; ++l) acc -= Ys[(size_t)l * n + i] * sv1[l];
          hc[i] = acc;
        }
        __syncthreads();
        panel_dots(H, lda, k0, j, hc, n, part, sv2);          // V^T h
        if (tid < j) {
          double a = 0.0;
          for (int m = 0; m <= tid; ++m) a += Tm[m * HB_NB + tid] * sv2[m];
          sv1[tid] = a;                                       // T^T (V^T h)
        }
        __syncthreads();
        for (int i = k0 + 1 + tid; i < n; i += EIG_THREADS) {
          double acc = hc[i];
          for (int l = 0; l < j; ++l) acc -= vget(H, lda, k0, l, i) * sv1[l];
          hc[i] = acc;
        }
      }
      __syncthreads();
      // ---- 2. the reflector from rows c+1.. (LAPACK's convention: v = 1
      // at row c + 1, beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta)
      double p2 = 0.0;
      for (int i = c + 2 + tid; i < n; i += EIG_THREADS) p2 += hc[i] * hc[i];
      const double sig2 = block_sum(p2, red);
      if (tid == 0) {
        const double alpha = hc[c + 1];
        if (sig2 == 0.0) {
          s_tau = 0.0;
          s_beta = alpha;
          s_scale = 0.0;
        } else {
          const double beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
          s_tau = (beta - alpha) / beta;
          s_beta = beta;
          s_scale = 1.0 / (alpha - beta);
        }
      }
      __syncthreads();
      const double tau = s_tau, beta = s_beta, scale = s_scale;
      // column c is final above row c + 2; v is kept below the subdiagonal
      // until the panel ends, and in hc (by row) for the pass
      for (int i = tid; i < n; i += EIG_THREADS) {
        const double hv = hc[i];
        const double v = (i <= c) ? 0.0 : (i == c + 1 ? 1.0 : hv * scale);
        HH(i, c) = (i <= c) ? hv : (i == c + 1 ? beta : v);
        hc[i] = v;
      }
      __syncthreads();
      // ---- 3. one read-only pass over columns c+1..n-1: y = A v, and
      // z[col] = v^T A[:, col] right of the panel.  Columns go to the
      // wavefronts (two per pass), lanes run over the rows.
      {
        double* pw = pn + wave * n;
        for (int i = lane; i < n; i += 64) pw[i] = 0.0;
        for (int j0 = c + 1 + wave; j0 < n; j0 += 2 * EIG_NW) {
          const double* cj[2];
          double vj[2], t[2];
          bool jok[2];
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            const int jj = j0 + p * EIG_NW;
            jok[p] = jj < n;
            cj[p] = H + (size_t)(jok[p] ? jj : j0) * lda;
            vj[p] = jok[p] ? hc[jj] : 0.0;
            t[p] = 0.0;
          }
          for (int i0 = 0; i0 < n; i0 += 64 * EIG_CG) {
            double hv[2][EIG_CG];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
              for (int q = 0; q < EIG_CG; ++q) {
                const int i = i0 + 64 * q + lane;
                hv[p][q] = (jok[p] && i < n) ? cj[p][i] : 0.0;
              }
#pragma unroll
            for (int q = 0; q < EIG_CG; ++q) {
              const int i = i0 + 64 * q + lane;
              if (i < n) {
                const double vi = hc[i];
                double pacc = 0.0;
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                  pacc += hv[p][q] * vj[p];
                  t[p] += vi * hv[p][q];
                }
                pw[i] += pacc;
              }
            }
          }
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            const int jj = j0 + p * EIG_NW;
            double tp = t[p];
            for (int off = 32; off > 0; off >>= 1) tp += __shfl_xor(tp, off, 64);
            if (lane == 0 && jok[p] && jj >= cfirst) Zs[(size_t)j * n + jj] = tp;
          }
        }
      }
      __syncthreads();
      // ---- 4. Y[:, j] = tau (y - Y (V^T v)); column j of T
      panel_dots(H, lda, k0, j, hc, n, part, sv2);            // t = V^T v
      for (int i = tid; i < n; i += EIG_THREADS) {
        double y = 0.0;
#pragma unroll
        for (int w = 0; w < EIG_NW; ++w) y += pn[w * n + i];
        for (int l = 0; l < j; ++l) y -= Ys[(size_t)l * n + i] * sv2[l];
        Ys[(size_t)j * n + i] = tau * y;
      }
      if (tid < j) {
        double a = 0.0;
        for (int m = tid; m < j; ++m) a += Tm[tid * HB_NB + m] * sv2[m];
        Tm[tid * HB_NB + j] = -tau * a;
      }
      if (tid == 0) Tm[j * HB_NB + j] = tau;
      __syncthreads();
    }
    // ---- M = V^T Y (kb x kb) on the matrix cores: each wavefront takes every
    // fourth group of four rows (A[li][lk] = V[i][li], B[lk][li] = Y[i][li],
    // i = k0 + 1 + 4 s + lk); the four partial products are added in order
    {
      const int li = lane & 15, lk = lane >> 4;
      EigMfma acc = {0.0, 0.0, 0.0, 0.0};
      const int nsteps = (n - k0 - 1 + 3) / 4;
      for (int st = wave; st < nsteps; st += EIG_NW) {
        const int i = k0 + 1 + 4 * st + lk;
        const bool ok = i < n && li < kb;
        const double av = ok ? vget(H, lda, k0, li, i) : 0.0;
        const double bv = ok ? Ys[(size_t)li * n + i] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) part[wave * 256 + (lk + 4 * q) * 16 + li] = acc[q];
      __syncthreads();
      double m = 0.0;
#pragma unroll
      for (int w = 0; w < EIG_NW; ++w) m += part[w * 256 + tid];
      Mm[tid] = m;                              // tid = l * 16 + m
    }
    __syncthreads();
    // ---- the right-hand operand of the panel's update, per column right of
    // the panel: a = V[col, :]^T, w = T^T (z - M a)
    // (a goes to Bs, r = z - M a replaces z in Zs, then w = T^T r: the
    // thread's own global words, no private arrays)
    for (int col = cfirst + tid; col < n; col += EIG_THREADS) {
      for (int m = 0; m < HB_NB; ++m)
        Bs[(size_t)m * n + col] = (m < kb) ? vget(H, lda, k0, m, col) : 0.0;
      for (int l = 0; l < kb; ++l) {
        double r = Zs[(size_t)l * n + col];
        for (int m = 0; m < kb; ++m) r -= Mm[l * HB_NB + m] * Bs[(size_t)m * n + col];
        Zs[(size_t)l * n + col] = r;
      }
      for (int l = 0; l < HB_NB; ++l) {
        double w = 0.0;
        if (l < kb)
          for (int m = 0; m <= l; ++m) w += Tm[m * HB_NB + l] * Zs[(size_t)m * n + col];
        Bs[(size_t)(HB_NB + l) * n + col] = w;
      }
    }
    __syncthreads();
    // ---- A[:, col] -= [Y | V] [a; w] for every column right of the panel,
    // on the matrix cores in transposed form (out^T = [a; w]^T [Y | V]^T) so
    // that a lane's accumulators are 16 consecutive rows of 4 columns: lane
    // (li, lk) supplies A'[li][lk] = B[k][col0 + li] and B'[lk][li] =
    // [Y | V][row0 + li][k], k = 4 kk + lk; accumulator q is row row0 + li of
    // column col0 + lk + 4 q.
    {
      const int li = lane & 15, lk = lane >> 4;
      const int nrt = (n + 15) / 16, nct = (n - cfirst + 15) / 16;
      for (int rt = wave; rt < nrt; rt += EIG_NW) {
        const int row = 16 * rt + li;
        const bool rok = row < n;
        double bf[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const int k = 4 * kk + lk;
          double v = 0.0;
          if (rok) {
            if (k < HB_NB) v = (k < kb) ? Ys[(size_t)k * n + row] : 0.0;
            else v = (k - HB_NB < kb) ? vget(H, lda, k0, k - HB_NB, row) : 0.0;
          }
          bf[kk] = v;
        }
        for (int ct = 0; ct < nct; ++ct) {
          const int colb = cfirst + 16 * ct;
          double af[8];
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            const int k = 4 * kk + lk, col = colb + li;
            const bool kok = (k < HB_NB) ? (k < kb) : (k - HB_NB < kb);
            af[kk] = (kok && col < n) ? -Bs[(size_t)k * n + col] : 0.0;
          }
          EigMfma acc;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int col = colb + lk + 4 * q;
            acc[q] = (rok && col < n) ? HH(row, col) : 0.0;
          }
#pragma unroll
          for (int kk = 0; kk < 8; ++kk)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[kk], bf[kk], acc, 0, 0, 0);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int col = colb + lk + 4 * q;
            if (rok && col < n) HH(row, col) = acc[q];
          }
        }
      }
    }
    __syncthreads();
    // ---- the panel's columns: zero below the subdiagonal (v no longer needed)
    for (int l = 0; l < kb; ++l)
      for (int i = k0 + l + 2 + tid; i < n; i += EIG_THREADS) HH(i, k0 + l) = 0.0;
    __syncthreads();
  }
#undef HH
}

// Francis QR in blocks, with a chain of up to QR_KMAX double-shift bulges
// per sweep (small-bulge multishift: Braman, Byers and Mathias, SIMAX 2002).
//
// Bulge b of the chain is introduced at the top of the window [lo, hi] three
// positions behind bulge b-1 and chased to the bottom; at chain step t it
// sits at position p_b = lo + t - 3 b.  One wavefront owns each bulge and the
// wavefronts move in lockstep: at every chain step all of them first form
// their reflectors and apply them from the left (their rows are disjoint),
// then, after a barrier, from the right (their columns are disjoint).  This
// keeps the order of the sequential chase for every entry except the 3 x 3
// corners a trailing bulge's left and a leading bulge's right reflector both
// touch, where the two commute.
//
// A block covers QR_NB chain steps; everything those steps touch inside the
// window lies in the index range [c0, c1] (plus row c1 + 1, which the
// leading bulge's right-hand update reaches).  That diagonal block is held in
// LDS while the reflectors are accumulated into U; afterwards the rest of
// the window gets them in one pass each:
//   rows c0..c1, columns c1+1..hi:  H <- U^T H
//   rows lo..c0-1, columns c0..c1:  H <- H U
// Shifts: the eigenvalues of the window's trailing 2 QR_KMAX square block
// (one wavefront runs a plain double-shift QR on it in LDS), complex pairs as
// (2 Re, |.|^2), real ones sorted and paired in order; the two eigenvalues of
// the trailing 2 x 2 block (one bulge) for windows below QR_MS_MIN, when the
// small QR fails, and on every tenth sweep without deflation, which uses an
// exceptional shift instead.
constexpr int QR_NB = 16;
constexpr int QR_KMAX = 4;                       // bulges per chain (<= wavefronts)
constexpr int QR_MS_MIN = 4 * QR_KMAX;           // smallest window for a chain
constexpr int QR_D = QR_NB + 3 * QR_KMAX;        // largest block order
constexpr int QR_LD = QR_D + 1;                  // LDS row stride of the block and of U
constexpr int QR_NS = 2 * QR_KMAX;               // order of the shift block
constexpr int QR_SLD = QR_NS + 1;
// LDS of the QR phase (doubles): block (QR_D + 1 rows), U, shift block, its
// eigenvalues, the shift pairs
constexpr int QR_LDS = (QR_D + 1) * QR_LD + QR_D * QR_LD + QR_NS * QR_SLD + 2 * QR_NS + 2 * QR_KMAX;
static_assert(QR_KMAX <= EIG_NW, "one wavefront per bulge");
static_assert(QR_D + 1 <= 64, "block rows fit a wavefront");
static_assert(QR_D <= 32, "the off-block products take K = 32");

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Double-shift QR on a small Hessenberg matrix S (m <= QR_NS, row stride
// QR_SLD) by one wavefront: lanes run over the columns of a left update and
// the rows of a right update; every lane takes the same control decisions
// from the shared values.  Returns 0 on success.
__device__ int small_francis(double* S, int m, double* wr, double* wi) {
  const int lane = threadIdx.x & 63;
  const double eps = DBL_EPSILON;
#define SS(i, j) S[(i) * QR_SLD + (j)]
  int hi = m - 1, its = 0, total = 0;
  while (hi >= 0) {
    if (hi == 0) {
      if (lane == 0) { wr[0] = SS(0, 0); wi[0] = 0.0; }
      break;
    }
    int lo = 0;
    for (int k = hi; k >= 1; --k) {
      const double s = fabs(SS(k - 1, k - 1)) + fabs(SS(k, k));
      const double sub = fabs(SS(k, k - 1));
      if (sub <= eps * s || sub == 0.0) { lo = k; break; }
    }
    if (lo == hi) {
      if (lane == 0) { wr[hi] = SS(hi, hi); wi[hi] = 0.0; }
      hi -= 1;
      its = 0;
      continue;
    }
    if (lo == hi - 1) {
      if (lane == 0) {
        double r1, i1, r2, i2;
        eig2x2(SS(hi - 1, hi - 1), SS(hi - 1, hi), SS(hi, hi - 1), SS(hi, hi), r1, i1, r2, i2);
        wr[hi - 1] = r1; wi[hi - 1] = i1;
        wr[hi] = r2; wi[hi] = i2;
      }
      hi -= 2;
      its = 0;
      continue;
    }
    ++its;
    if (++total > 30 * m) return 1;
    double s_sum, s_prod;
    if (its % 10 == 0) {
      const double w = fabs(SS(hi, hi - 1)) + fabs(SS(hi - 1, hi - 2));
      s_sum = 1.5 * w;
      s_prod = w * w;
    } else {
      s_sum = SS(hi - 1, hi - 1) + SS(hi, hi);
      s_prod = SS(hi - 1, hi - 1) * SS(hi, hi) - SS(hi - 1, hi) * SS(hi, hi - 1);
    }
    double x = SS(lo, lo) * SS(lo, lo) + SS(lo, lo + 1) * SS(lo + 1, lo) - s_sum * SS(lo, lo) + s_prod;
    double y = SS(lo + 1, lo) * (SS(lo, lo) + SS(lo + 1, lo + 1) - s_sum);
    double z = SS(lo + 1, lo) * SS(lo + 2, lo + 1);
    for (int k = lo; k <= hi - 1; ++k) {
      const bool three = k < hi - 1;
      if (k > lo) {
        x = SS(k, k - 1);
        y = SS(k + 1, k - 1);
        z = three ? SS(k + 2, k - 1) : 0.0;
      }
      const double nv = three ? sqrt(x * x + y * y + z * z) : sqrt(x * x + y * y);
      wave_sync();
      if (nv != 0.0) {
        const double v0 = x + copysign(nv, x), v1 = y, v2 = three ? z : 0.0;
        const double t = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
        const int c = max(lo, k - 1) + lane;
        if (c <= hi) {
          const double a0 = SS(k, c), a1 = SS(k + 1, c), a2 = three ? SS(k + 2, c) : 0.0;
          const double sv = t * (v0 * a0 + v1 * a1 + v2 * a2);
          double b0 = a0 - sv * v0, b1 = a1 - sv * v1, b2 = a2 - sv * v2;
          if (k > lo && c == k - 1) { b0 = -copysign(nv, x); b1 = 0.0; b2 = 0.0; }
          SS(k, c) = b0;
          SS(k + 1, c) = b1;
          if (three) SS(k + 2, c) = b2;
        }
        wave_sync();
        const int r = lo + lane;
        if (r <= min(k + 3, hi)) {
          const double a0 = SS(r, k), a1 = SS(r, k + 1), a2 = three ? SS(r, k + 2) : 0.0;
          const double sv = t * (a0 * v0 + a1 * v1 + a2 * v2);
          SS(r, k) = a0 - sv * v0;
          SS(r, k + 1) = a1 - sv * v1;
          if (three) SS(r, k + 2) = a2 - sv * v2;
        }
        wave_sync();
      }
    }
  }
#undef SS
  return 0;
}

// The shift pairs of one sweep into pairs[0 .. 2k); returns k (1 .. QR_KMAX).
// All threads of the workgroup call it.
__device__ int sweep_shifts(const double* __restrict__ H, int lda, int lo, int hi, int its,
                            double* S, double* swr, double* swi, double* pairs, int* ired) {
  const int tid = threadIdx.x, wave = tid >> 6;
#define HH(i, j) H[(size_t)(j) * lda + (i)]
  const int m = hi - lo + 1;
  if (its % 10 != 0 && m >= QR_MS_MIN) {
    const int b0 = hi - QR_NS + 1;
    for (int e = tid; e < QR_NS * QR_NS; e += EIG_THREADS) {
      const int r = e / QR_NS, c = e - r * QR_NS;
      S[r * QR_SLD + c] = (r <= c + 1) ? HH(b0 + r, b0 + c) : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      const int fail = small_francis(S, QR_NS, swr, swi);
      if ((tid & 63) == 0) ired[0] = fail;
    }
    __syncthreads();
    const int fail = ired[0];
    __syncthreads();
    if (!fail) {
      if (tid == 0) {
        // complex pairs first; the real shifts, sorted in place at the front
        // of swr, then paired in order
        int k = 0, nre = 0;
        for (int i = 0; i < QR_NS; ++i) {
          const double re = swr[i], im = swi[i];
          if (im > 0.0) {
            pairs[2 * k] = 2.0 * re;
            pairs[2 * k + 1] = re * re + im * im;
            ++k;
          } else if (im == 0.0) {
            int j = nre++;
            for (; j > 0 && swr[j - 1] > re; --j) swr[j] = swr[j - 1];
            swr[j] = re;
          }
        }
        for (int i = 0; i + 1 < nre; i += 2) {
          pairs[2 * k] = swr[i] + swr[i + 1];
          pairs[2 * k + 1] = swr[i] * swr[i + 1];
          ++k;
        }
        ired[1] = k;
      }
      __syncthreads();
      const int k = ired[1];
      __syncthreads();
      if (k >= 1) return k;
    }
  }
  if (tid == 0) {
    if (its % 10 == 0) {
      const double w = fabs(HH(hi, hi - 1)) + fabs(HH(hi - 1, hi - 2));
      pairs[0] = 1.5 * w;
      pairs[1] = w * w;
    } else {
      const double a = HH(hi - 1, hi - 1), b = HH(hi - 1, hi);
      const double c = HH(hi, hi - 1), d = HH(hi, hi);
      pairs[0] = a + d;
      pairs[1] = a * d - b * c;
    }
  }
  __syncthreads();
#undef HH
  return 1;
}

// One chain step of bulge (wavefront) at position p, left half: form the
// reflector (introducing the bulge from its shift pair at p == lo) and apply
// it to rows p..p+2 of the block; the bulge column becomes exactly
// (-sign(x) |(x,y,z)|, 0, 0).  Returns false when the reflector is trivial.
__device__ inline bool chase_left(double* D, int c0, int d, int lo, int hi, int p,
                                  double s_sum, double s_prod, double& v0, double& v1,
                                  double& v2, double& t, bool& three) {
  const int lane = threadIdx.x & 63;
  const int j = p - c0;
  three = p < hi - 1;
  double x, y, z;
  if (p == lo) {
    const double h00 = D[j * QR_LD + j], h01 = D[j * QR_LD + j + 1];
    const double h10 = D[(j + 1) * QR_LD + j], h11 = D[(j + 1) * QR_LD + j + 1];
    x = h00 * h00 + h01 * h10 - s_sum * h00 + s_prod;
    y = h10 * (h00 + h11 - s_sum);
    z = three ? h10 * D[(j + 2) * QR_LD + j + 1] : 0.0;
  } else {
    x = D[j * QR_LD + j - 1];
    y = D[(j + 1) * QR_LD + j - 1];
    z = three ? D[(j + 2) * QR_LD + j - 1] : 0.0;
  }
  const double nv = three ? sqrt(x * x + y * y + z * z) : sqrt(x * x + y * y);
  if (nv == 0.0) return false;
  v0 = x + copysign(nv, x);
  v1 = y;
  v2 = three ? z : 0.0;
  t = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
  const int q = max(lo, p - 1) - c0;
  if (lane >= q && lane < d) {
    double* pp = D + j * QR_LD + lane;
    const double a0 = pp[0], a1 = pp[QR_LD], a2 = three ? pp[2 * QR_LD] : 0.0;
    const double sv = t * (v0 * a0 + v1 * a1 + v2 * a2);
    double b0 = a0 - sv * v0, b1 = a1 - sv * v1, b2 = a2 - sv * v2;
    if (p > lo && lane == j - 1) {
      b0 = -copysign(nv, x);
      b1 = 0.0;
      b2 = 0.0;
    }
    pp[0] = b0;
    pp[QR_LD] = b1;
    if (three) pp[2 * QR_LD] = b2;
  }
  return true;
}

// Right half: columns p..p+2 of the block rows c0..min(p+3, hi), and of U.
__device__ inline void chase_right(double* D, double* U, int c0, int d, int hi, int p,
                                   double v0, double v1, double v2, double t, bool three) {
  const int lane = threadIdx.x & 63;
  const int j = p - c0;
  const int rl = min(p + 3, hi) - c0;
  if (lane <= rl) {
    double* pp = D + lane * QR_LD + j;
    const double a0 = pp[0], a1 = pp[1], a2 = three ? pp[2] : 0.0;
    const double sv = t * (a0 * v0 + a1 * v1 + a2 * v2);
    pp[0] = a0 - sv * v0;
    pp[1] = a1 - sv * v1;
    if (three) pp[2] = a2 - sv * v2;
  }
  if (lane < d) {
    double* pp = U + lane * QR_LD + j;
    const double a0 = pp[0], a1 = pp[1], a2 = three ? pp[2] : 0.0;
    const double sv = t * (a0 * v0 + a1 * v1 + a2 * v2);
    pp[0] = a0 - sv * v0;
    pp[1] = a1 - sv * v1;
    if (three) pp[2] = a2 - sv * v2;
  }
}

// one sweep with k bulges over the window [lo, hi] (hi - lo >= 2)
__device__ void francis_sweep(double* __restrict__ H, int lda, int lo, int hi, int k,
                              const double* __restrict__ pairs, double* __restrict__ D,
                              double* __restrict__ U) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#define HH(i, j) H[(size_t)(j) * lda + (i)]
  const int T = (hi - 1 - lo) + 3 * (k - 1) + 1;       // chain steps
  const double s_sum = wave < k ? pairs[2 * wave] : 0.0;
  const double s_prod = wave < k ? pairs[2 * wave + 1] : 0.0;
  for (int t0 = 0; t0 < T; t0 += QR_NB) {
    const int t1 = min(t0 + QR_NB, T);
    const int pmin = max(lo, lo + t0 - 3 * (k - 1));
    const int pmax = min(hi - 1, lo + t1 - 1);
    const int c0 = max(lo, pmin - 1);
    const int c1 = min(hi, pmax + 2);
    const int d = c1 - c0 + 1;
    const int dr = d + (c1 < hi ? 1 : 0);
    for (int e = tid; e < dr * d; e += EIG_THREADS) {
      const int r = e / d, c = e - r * d;
      D[r * QR_LD + c] = HH(c0 + r, c0 + c);
    }
    // the whole QR_D x QR_D tile: the off-block products read every entry
    for (int e = tid; e < QR_D * QR_D; e += EIG_THREADS) {
      const int r = e / QR_D, c = e - r * QR_D;
      U[r * QR_LD + c] = (r == c && r < d) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (k == 1) {
      // one bulge: wavefront 0 alone, wavefront-level synchronisation
      if (wave == 0)
        for (int t = t0; t < t1; ++t) {
          const int p = lo + t;
          double v0, v1, v2, tt;
          bool three;
          const bool app = chase_left(D, c0, d, lo, hi, p, s_sum, s_prod, v0, v1, v2, tt, three);
          wave_sync();
          if (app) chase_right(D, U, c0, d, hi, p, v0, v1, v2, tt, three);
          wave_sync();
        }
    } else {
      for (int t = t0; t < t1; ++t) {
        const int p = lo + t - 3 * wave;
        const bool act = wave < k && p >= lo && p <= hi - 1;
        double v0 = 0.0, v1 = 0.0, v2 = 0.0, tt = 0.0;
        bool three = false, app = false;
        if (act) app = chase_left(D, c0, d, lo, hi, p, s_sum, s_prod, v0, v1, v2, tt, three);
        __syncthreads();
        if (app) chase_right(D, U, c0, d, hi, p, v0, v1, v2, tt, three);
        __syncthreads();
      }
    }
    __syncthreads();
    for (int e = tid; e < dr * d; e += EIG_THREADS) {
      const int r = e / d, c = e - r * d;
      HH(c0 + r, c0 + c) = D[r * QR_LD + c];
    }
    // The off-block products on the matrix cores (v_mfma_f64_16x16x4f64;
    // lane (li, lk) supplies A[li][lk] and B[lk][li], and accumulator q holds
    // row lk + 4 q, column li of the 16 x 16 tile).  The block's order is at
    // most QR_D = 28 <= 32, so the products have K = 32 with U zero beyond d.
    //   rows c0..c1, columns c1+1..hi:  H <- U^T H  (16-column tiles)
    //   rows lo..c0-1, columns c0..c1:  H <- H U    (16-row tiles)
    {
      const int li = lane & 15, lk = lane >> 4;
      const int nct = c1 < hi ? (hi - c1 + 15) / 16 : 0;      // U^T H tiles
      const int nrt = (c0 - lo + 15) / 16;                     // H U tiles
      if (nct > 0 && wave < nct) {
        // U^T fragments: A[16 ti + li][4 kk + lk] = U[4 kk + lk][16 ti + li]
        double ua[2][8];
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            const int r = 4 * kk + lk, c = 16 * ti + li;
            ua[ti][kk] = (r < QR_D && c < QR_D) ? U[r * QR_LD + c] : 0.0;
          }
        for (int t = wave; t < nct; t += EIG_NW) {
          const int col = c1 + 1 + 16 * t + li;
          const bool cok = col <= hi;
          double bv[8];
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            const int r = 4 * kk + lk;
            bv[kk] = (cok && r < d) ? HH(c0 + r, col) : 0.0;
          }
          EigMfma acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[0][kk], bv[kk], acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[1][kk], bv[kk], acc[1], 0, 0, 0);
          }
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int r = 16 * ti + lk + 4 * q;
              if (cok && r < d) HH(c0 + r, col) = acc[ti][q];
            }
        }
      }
      if (nrt > 0) {
        // U fragments: B[4 kk + lk][16 tj + li] = U[4 kk + lk][16 tj + li]
        const int w0 = nct % EIG_NW;                 // continue the waves' turns
        const int wv = (wave - w0 + EIG_NW) % EIG_NW;
        if (wv < nrt) {
          double ub[2][8];
#pragma unroll
          for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
              const int r = 4 * kk + lk, c = 16 * tj + li;
              ub[tj][kk] = (r < QR_D && c < QR_D) ? U[r * QR_LD + c] : 0.0;
            }
          for (int t = wv; t < nrt; t += EIG_NW) {
            const int row = lo + 16 * t + li;
            const bool rok = row < c0;
            double av[8];
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
              const int c = 4 * kk + lk;
              av[kk] = (rok && c < d) ? HH(row, c0 + c) : 0.0;
            }
            EigMfma acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
              acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], ub[0][kk], acc[0], 0, 0, 0);
              acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[kk], ub[1][kk], acc[1], 0, 0, 0);
            }
            const int rbase = lo + 16 * t;
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int r = rbase + lk + 4 * q, c = 16 * tj + li;
                if (r < c0 && c < d) HH(r, c0 + c) = acc[tj][q];
              }
          }
        }
      }
    }
    __syncthreads();
  }
#undef HH
}

// Francis QR on Hessenberg H; returns 0 on success.  lds holds QR_LDS
// doubles.
__device__ int francis(double* __restrict__ H, int n, int lda,
                       double* __restrict__ wr, double* __restrict__ wi,
                       int* ired, double* lds) {
  const int tid = threadIdx.x;
  const double eps = DBL_EPSILON;
  double* D = lds;
  double* U = D + (QR_D + 1) * QR_LD;
  double* S = U + QR_D * QR_LD;
  double* swr = S + QR_NS * QR_SLD;
  double* swi = swr + QR_NS;
  double* pairs = swi + QR_NS;
  int hi = n - 1;
  int its = 0;
  int total = 0;
  const int max_total = 40 * n + 100;
#define HH(i, j) H[(size_t)(j) * lda + (i)]
  while (hi >= 0) {
    if (hi == 0) {
      if (tid == 0) { wr[0] = HH(0, 0); wi[0] = 0.0; }
      hi = -1;
      break;
    }
    // deflation point: largest k in [1, hi] with a negligible subdiagonal
    int cand = 0;
    for (int k = 1 + tid; k <= hi; k += EIG_THREADS) {
      double s = fabs(HH(k - 1, k - 1)) + fabs(HH(k, k));
      double sub = fabs(HH(k, k - 1));
      if (sub <= eps * s || sub == 0.0) cand = max(cand, k);
    }
    const int lo = block_max_int(cand, ired);
    if (lo > 0 && tid == 0) HH(lo, lo - 1) = 0.0;
    __syncthreads();
    if (lo == hi) {
      if (tid == 0) { wr[hi] = HH(hi, hi); wi[hi] = 0.0; }
      hi -= 1;
      its = 0;
      __syncthreads();
      continue;
    }
    if (lo == hi - 1) {
      if (tid == 0) {
        double r1, i1, r2, i2;
        eig2x2(HH(hi - 1, hi - 1), HH(hi - 1, hi), HH(hi, hi - 1), HH(hi, hi), r1, i1, r2, i2);
        wr[hi - 1] = r1; wi[hi - 1] = i1;
        wr[hi] = r2; wi[hi] = i2;
      }
      hi -= 2;
      its = 0;
      __syncthreads();
      continue;
    }
    ++its;
    ++total;
    if (total > max_total) return 1;
    const int k = sweep_shifts(H, lda, lo, hi, its, S, swr, swi, pairs, ired);
    francis_sweep(H, lda, lo, hi, k, pairs, D, U);
  }
#undef HH
  return 0;
}

// four waves per SIMD: the register budget (128) admits four workgroups per CU
__global__ __launch_bounds__(EIG_THREADS, 4) void k_eig(
    double* __restrict__ Abase, size_t stride, int lda,
    const SlotState* __restrict__ st, int n_uniform, int nmax, double* __restrict__ wrb,
    double* __restrict__ wib, int w_stride, int* __restrict__ info,
    double* __restrict__ scrbase, size_t scr_stride) {
  const int slot = blockIdx.x;
  int n = n_uniform;
  if (st != nullptr) {
    if (st[slot].phase != PH_EIG) return;
    n = st[slot].n_states;
  }
  if (n <= 0 || n > EIG_NMAX || n > nmax) return;
  extern __shared__ double eig_lds[];
  __shared__ double red[EIG_THREADS / 64];
  __shared__ int ired[EIG_THREADS / 64];
  double* H = Abase + (size_t)slot * stride;
  double* wr = wrb + (size_t)slot * w_stride;
  double* wi = wib + (size_t)slot * w_stride;
  hessenberg(H, n, lda, eig_lds, red, scrbase + (size_t)slot * scr_stride);
  __syncthreads();
  // the QR phase reuses the reduction's LDS
  const int fail = francis(H, n, lda, wr, wi, ired, eig_lds);
  if (threadIdx.x == 0 && info != nullptr) info[slot] = fail;
  if (threadIdx.x == 0 && st != nullptr) const_cast<SlotState*>(st)[slot].qr_fail = fail;
}

size_t eig_hess_lds(int nmax) {
  return sizeof(double) * std::max<size_t>(eig_hess_lds_doubles(nmax), QR_LDS);
}

void launch_eig(double* A, size_t stride, int lda, const int* /*n_per*/,
                int n_uniform, double* wr, double* wi, int w_stride,
                SlotState* st, int count, int* info, double* scr, size_t scr_stride,
                hipStream_t stream) {
  if (count <= 0) return;
  // the dynamic LDS is sized for the largest order a slot can have (the
  // eigenvalue arrays have that many entries per slot)
  const int nmax = n_uniform > 0 ? n_uniform : w_stride;
  hipLaunchKernelGGL(k_eig, dim3(count), dim3(EIG_THREADS), eig_hess_lds(nmax), stream, A,
                     stride, lda, st, n_uniform, nmax, wr, wi, w_stride, info, scr, scr_stride);
}

void eig_set_attrs(size_t bytes) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(k_eig),
                      hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)std::min(bytes - 8 * 1024, eig_hess_lds(EIG_NMAX)));
}

}  // namespace cs
