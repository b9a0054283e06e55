// Batched nonsymmetric eigenvalues (one workgroup per matrix).
//
// The small-signal test needs every eigenvalue of the state matrix.  Each
// matrix is reduced to upper Hessenberg form by Householder reflections, one
// read-write pass over the trailing columns per reflector (the two-sided
// update of one step fused with the products the next step needs), then
// Francis implicit double-shift QR sweeps run on the active window [lo, hi]
// until every 1x1 or 2x2 diagonal block has split off (eigenvalues only, so
// updates stay inside the window).  A sweep chases its bulge in blocks of 16
// steps through a small diagonal block held in LDS and applies the
// accumulated reflectors to the rest of the window once per block.
// Deflation: a subdiagonal entry is negligible when |h(k,k-1)| <= eps
// (|h(k-1,k-1)| + |h(k,k)|).  Every tenth sweep without deflation uses an
// exceptional shift.  The matrix lives in global memory (column-major, lda);
// the reflector vectors, the reduction's partial sums and the chased block
// live in LDS.
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

// Householder reduction to upper Hessenberg form with one read-write pass
// over the matrix per reflector.  Step k uses P_k = I - tau u u^T on indices
// k+1..n-1 (u from column k below the diagonal).  With B = H[:, k+1:],
// p = B u and s = tau B[k+1:, :]^T u, both taken from H before the step, the
// two-sided update P_k H P_k is the rank-2 change
//   H[i][k+1+j] -= a_i s_j + w_i u_j,   a_i = u_{i-k-1} (i > k, else 0),
//   w_i = tau (p_i - a_i (s . u)),
// so one pass can apply step k and, on the values it has just written,
// gather p and s for step k+1 (whose reflector comes from column k+1, which
// is brought up to date first).  Columns are shared out to the wavefronts,
// lanes run over the rows: s of a column is a wavefront sum, p a per-lane
// partial per wavefront (kept in LDS), added in a fixed order.
// LDS (dynamic, 9 n doubles): u, s, w of the current step, un, sn of the
// next, and the NW partials of the next p.
constexpr int EIG_NW = EIG_THREADS / 64;
constexpr int EIG_CG = 8;                   // row chunks of 64 loaded together

size_t eig_hess_lds(int nmax) { return sizeof(double) * 9 * (size_t)nmax; }

__device__ void hessenberg(double* __restrict__ H, int n, int lda, double* __restrict__ lds,
                           double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* u = lds;
  double* sv = u + n;
  double* w = sv + n;
  double* un = w + n;
  double* sn = un + n;
  double* pn = sn + n;            // [EIG_NW][n]
  double tau = 0.0;
  __shared__ double s_x0;
  for (int k = -1; k <= n - 3; ++k) {
    const bool upd = k >= 0 && tau != 0.0;   // step k changes H
    const bool nxt = k + 1 <= n - 3;         // a reflector for column k+1
    // ---- column k+1: step k's update, then the next reflector from it
    double* c1 = H + (size_t)(k + 1) * lda;
    double part = 0.0;
    for (int i = tid; i < n; i += EIG_THREADS) {
      double h = c1[i];
      if (upd) h -= ((i > k) ? u[i - k - 1] * sv[0] : 0.0) + w[i] * u[0];
      if (i >= k + 2 && nxt) {
        un[i - k - 2] = h;
        part += h * h;
      } else {
        c1[i] = h;
      }
    }
    double taun = 0.0, alpha = 0.0;
    if (nxt) {
      const double sig2 = block_sum(part, red);   // barriers: un[] complete
      if (tid == 0) s_x0 = un[0];
      __syncthreads();
      const double x0 = s_x0;
      if (sig2 != 0.0) {
        const double sig = sqrt(sig2);
        alpha = -copysign(sig, x0);
        taun = 1.0 / (sig * (sig + fabs(x0)));
        if (tid == 0) un[0] = x0 - alpha;
      }
      for (int i = k + 2 + tid; i < n; i += EIG_THREADS) c1[i] = (i == k + 2) ? alpha : 0.0;
    }
    __syncthreads();
    // ---- one pass over columns k+2..n-1: apply step k, gather p and s of
    // step k+1 from the updated values
    if (upd || nxt) {
      double* pw = pn + wave * n;   // this wavefront's partial p (lane-owned rows)
      if (nxt)
        for (int i = lane; i < n; i += 64) pw[i] = 0.0;
      // two columns per pass of a wavefront (j and j + EIG_NW), all their
      // loads in flight together
      for (int j0 = k + 2 + wave; j0 < n; j0 += 2 * EIG_NW) {
        double* cj[2];
        double sj[2], uj[2], unj[2], t[2];
        bool jok[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int j = j0 + p * EIG_NW;
          jok[p] = j < n;
          cj[p] = H + (size_t)(jok[p] ? j : j0) * lda;
          sj[p] = (upd && jok[p]) ? sv[j - k - 1] : 0.0;
          uj[p] = (upd && jok[p]) ? u[j - k - 1] : 0.0;
          unj[p] = (nxt && jok[p]) ? un[j - k - 2] : 0.0;
          t[p] = 0.0;
        }
        for (int i0 = 0; i0 < n; i0 += 64 * EIG_CG) {
          double hv[2][EIG_CG];
#pragma unroll
          for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int c = 0; c < EIG_CG; ++c) {
              const int i = i0 + 64 * c + lane;
              hv[p][c] = (jok[p] && i < n) ? cj[p][i] : 0.0;
            }
#pragma unroll
          for (int c = 0; c < EIG_CG; ++c) {
            const int i = i0 + 64 * c + lane;
            if (i < n) {
              const double ai = (upd && i > k) ? u[i - k - 1] : 0.0;
              const double wi = upd ? w[i] : 0.0;
              const double uni = (nxt && i >= k + 2) ? un[i - k - 2] : 0.0;
              double pacc = 0.0;
#pragma unroll
              for (int p = 0; p < 2; ++p) {
                if (jok[p]) {
                  double h = hv[p][c];
                  if (upd) {
                    h -= ai * sj[p] + wi * uj[p];
                    cj[p][i] = h;
                  }
                  pacc += h * unj[p];
                  t[p] += uni * h;
                }
              }
              if (nxt) pw[i] += pacc;
            }
          }
        }
        if (nxt) {
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            double tp = t[p];
            for (int off = 32; off > 0; off >>= 1) tp += __shfl_xor(tp, off, 64);
            if (lane == 0 && jok[p]) sn[j0 + p * EIG_NW - k - 2] = taun * tp;
          }
        }
      }
    }
    __syncthreads();
    if (!nxt) break;
    // ---- step k+1's w from p (the partials in a fixed order) and s . u
    double dot = 0.0;
    for (int j = tid; j < n - k - 2; j += EIG_THREADS) dot += sn[j] * un[j];
    const double cdot = block_sum(dot, red);
    for (int i = tid; i < n; i += EIG_THREADS) {
      double pi = 0.0;
#pragma unroll
      for (int v = 0; v < EIG_NW; ++v) pi += pn[v * n + i];
      const double ai = (i > k + 1) ? un[i - k - 2] : 0.0;
      w[i] = taun * (pi - ai * cdot);
    }
    double* t1 = u; u = un; un = t1;
    double* t2 = sv; sv = sn; sn = t2;
    tau = taun;
    __syncthreads();
  }
}

// Bulge chasing in blocks.  A block covers QR_NB consecutive bulge steps
// k0 .. kend-1; every row and column those steps touch inside the window
// lies in the index range [c0, c1] (plus the row c1 + 1, which the last
// step's right-hand update reaches).  That diagonal block is chased in LDS by
// one wavefront while the reflectors are accumulated into U (P_k0 ... P_kend-1);
// afterwards the rest of the window gets them in one pass each:
//   rows c0..c1, columns c1+1..hi:  H <- U^T H
//   rows lo..c0-1, columns c0..c1:  H <- H U
constexpr int QR_NB = 16;
constexpr int QR_D = QR_NB + 3;      // block order
constexpr int QR_LD = QR_D + 1;      // LDS row stride of the block and of U

// one Francis double-shift sweep over the window [lo, hi] (hi - lo >= 2)
__device__ void francis_sweep(double* __restrict__ H, int lda, int lo, int hi,
                              double x, double y, double z,
                              double* __restrict__ D, double* __restrict__ U) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#define HH(i, j) H[(size_t)(j) * lda + (i)]
  for (int k0 = lo; k0 <= hi - 1; k0 += QR_NB) {
    const int kend = min(k0 + QR_NB, hi);        // steps k0 .. kend-1
    const int c0 = max(lo, k0 - 1);
    const int c1 = min(kend + 1, hi);
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
    if (wave == 0) {
      for (int k = k0; k < kend; ++k) {
        const int j = k - c0;
        const bool three = k < hi - 1;
        if (k > lo) {
          x = D[j * QR_LD + j - 1];
          y = D[(j + 1) * QR_LD + j - 1];
          z = three ? D[(j + 2) * QR_LD + j - 1] : 0.0;
        }
        const double nv = three ? sqrt(x * x + y * y + z * z) : sqrt(x * x + y * y);
        if (nv != 0.0) {
          const double v0 = x + copysign(nv, x), v1 = y, v2 = three ? z : 0.0;
          const double t = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
          // from the left: rows j..j+2, columns max(lo, k-1) .. c1; the
          // bulge column k-1 becomes exactly (-sign(x) |(x,y,z)|, 0, 0)
          const int q = max(lo, k - 1) - c0;
          if (lane >= q && lane < d) {
            double* p = D + j * QR_LD + lane;
            const double a0 = p[0], a1 = p[QR_LD], a2 = three ? p[2 * QR_LD] : 0.0;
            const double sv = t * (v0 * a0 + v1 * a1 + v2 * a2);
            double b0 = a0 - sv * v0, b1 = a1 - sv * v1, b2 = a2 - sv * v2;
            if (k > lo && lane == j - 1) {
              b0 = -copysign(nv, x);
              b1 = 0.0;
              b2 = 0.0;
            }
            p[0] = b0;
            p[QR_LD] = b1;
            if (three) p[2 * QR_LD] = b2;
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          // from the right: columns j..j+2, rows c0 .. min(k+3, hi); and U
          const int rl = min(k + 3, hi) - c0;
          if (lane <= rl) {
            double* p = D + lane * QR_LD + j;
            const double a0 = p[0], a1 = p[1], a2 = three ? p[2] : 0.0;
            const double sv = t * (a0 * v0 + a1 * v1 + a2 * v2);
            p[0] = a0 - sv * v0;
            p[1] = a1 - sv * v1;
            if (three) p[2] = a2 - sv * v2;
          }
          if (lane < d) {
            double* p = U + lane * QR_LD + j;
            const double a0 = p[0], a1 = p[1], a2 = three ? p[2] : 0.0;
            const double sv = t * (a0 * v0 + a1 * v1 + a2 * v2);
            p[0] = a0 - sv * v0;
            p[1] = a1 - sv * v1;
            if (three) p[2] = a2 - sv * v2;
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < dr * d; e += EIG_THREADS) {
      const int r = e / d, c = e - r * d;
      HH(c0 + r, c0 + c) = D[r * QR_LD + c];
    }
    // rows c0..c1 right of the block: H <- U^T H, one thread per column
    for (int cc = c1 + 1 + tid; cc <= hi; cc += EIG_THREADS) {
      double* col = H + (size_t)cc * lda + c0;
      double a[QR_D];
#pragma unroll
      for (int i = 0; i < QR_D; ++i) a[i] = (i < d) ? col[i] : 0.0;
#pragma nounroll
      for (int i = 0; i < d; ++i) {
        double sv = 0.0;
#pragma unroll
        for (int r = 0; r < QR_D; ++r) sv += U[r * QR_LD + i] * a[r];
        col[i] = sv;
      }
    }
    // rows lo..c0-1 of the block's columns: H <- H U, one thread per row
    for (int rr = lo + tid; rr < c0; rr += EIG_THREADS) {
      double* row = H + (size_t)c0 * lda + rr;
      double a[QR_D];
#pragma unroll
      for (int i = 0; i < QR_D; ++i) a[i] = (i < d) ? row[(size_t)i * lda] : 0.0;
#pragma nounroll
      for (int jj = 0; jj < d; ++jj) {
        double sv = 0.0;
#pragma unroll
        for (int i = 0; i < QR_D; ++i) sv += a[i] * U[i * QR_LD + jj];
        row[(size_t)jj * lda] = sv;
      }
    }
    __syncthreads();
  }
#undef HH
}

// Francis double-shift QR on Hessenberg H; returns 0 on success.
__device__ int francis(double* __restrict__ H, int n, int lda,
                       double* __restrict__ wr, double* __restrict__ wi,
                       int* ired, double* D, double* U) {
  const int tid = threadIdx.x;
  const double eps = DBL_EPSILON;
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
    double s_sum, s_prod;
    if (its % 10 == 0) {
      const double w = fabs(HH(hi, hi - 1)) + fabs(HH(hi - 1, hi - 2));
      s_sum = 1.5 * w;
      s_prod = w * w;
    } else {
      const double a = HH(hi - 1, hi - 1), b = HH(hi - 1, hi);
      const double c = HH(hi, hi - 1), d = HH(hi, hi);
      s_sum = a + d;
      s_prod = a * d - b * c;
    }
    const double x = HH(lo, lo) * HH(lo, lo) + HH(lo, lo + 1) * HH(lo + 1, lo) - s_sum * HH(lo, lo) + s_prod;
    const double y = HH(lo + 1, lo) * (HH(lo, lo) + HH(lo + 1, lo + 1) - s_sum);
    const double z = HH(lo + 1, lo) * HH(lo + 2, lo + 1);
    __syncthreads();
    francis_sweep(H, lda, lo, hi, x, y, z, D, U);
  }
#undef HH
  return 0;
}

__global__ __launch_bounds__(EIG_THREADS) void k_eig(
    double* __restrict__ Abase, size_t stride, int lda,
    const SlotState* __restrict__ st, int n_uniform, int nmax, double* __restrict__ wrb,
    double* __restrict__ wib, int w_stride, int* __restrict__ info) {
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
  __shared__ double qd[(QR_D + 1) * QR_LD];
  __shared__ double qu[QR_D * QR_LD];
  double* H = Abase + (size_t)slot * stride;
  double* wr = wrb + (size_t)slot * w_stride;
  double* wi = wib + (size_t)slot * w_stride;
  hessenberg(H, n, lda, eig_lds, red);
  // zero below the subdiagonal (the reduction leaves exact zeros already)
  const int fail = francis(H, n, lda, wr, wi, ired, qd, qu);
  if (threadIdx.x == 0 && info != nullptr) info[slot] = fail;
  if (threadIdx.x == 0 && st != nullptr) const_cast<SlotState*>(st)[slot].qr_fail = fail;
}

void launch_eig(double* A, size_t stride, int lda, const int* /*n_per*/,
                int n_uniform, double* wr, double* wi, int w_stride,
                SlotState* st, int count, int* info, hipStream_t stream) {
  if (count <= 0) return;
  // the dynamic LDS is sized for the largest order a slot can have (the
  // eigenvalue arrays have that many entries per slot)
  const int nmax = n_uniform > 0 ? n_uniform : w_stride;
  hipLaunchKernelGGL(k_eig, dim3(count), dim3(EIG_THREADS), eig_hess_lds(nmax), stream, A,
                     stride, lda, st, n_uniform, nmax, wr, wi, w_stride, info);
}

void eig_set_attrs(size_t bytes) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(k_eig),
                      hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)std::min(bytes - 8 * 1024, eig_hess_lds(EIG_NMAX)));
}

}  // namespace cs
