// Batched dense LU with partial pivoting and solve (one workgroup per matrix).
//
// Each Newton step of the OPF solves one dense KKT system, and the state
// matrix needs g_y^{-1} g_x; both go through this kernel.  The matrix is
// row-major, rows of stride lda, with the right-hand sides stored as columns
// n..ncols-1 (an augmented matrix): the forward substitution falls out of the
// elimination and only the back substitution with U remains.
//
// Right-looking blocked LU, panel width NB = 32, four or eight wavefronts per
// matrix (LuGeo), panels taken in pairs so that the trailing matrix is updated
// once per pair with rank 64.  Per pair (panels [k0, k1) and [k1, k2)):
//   B1. the first panel's columns are brought up to date by the previous
//       pair (A -= L21 U12 on MFMA), passed through LDS in 16-column chunks
//       and loaded into registers: thread t holds panel rows t, t + THREADS
//       (and t + 2 THREADS with four wavefronts, while the panel needs it);
//   P1. that panel is factorised in registers by all threads.  Rows are never
//       moved while it runs: each keeps its LAPACK position (the position it
//       would occupy after the interchanges so far) and a "pivoted" flag.  Per
//       column: a wavefront argmax of |a| on DPP (ties to the lower position),
//       each wavefront publishes its candidate and the candidate's row in LDS,
//       one barrier, every thread picks the winner and eliminates with that
//       row.  Finally every row is written to its position;
//   C.  the rest of the previous pair's trailing update (rows from k0,
//       columns from k1) on the matrix cores (v_mfma_f64_16x16x4f64, or
//       v_mfma_f32_16x16x4f32 for the FP32 factorisation of the mixed-
//       precision solve), 32 x 32 groups of four 16 x 16 tiles taken from an
//       LDS counter, -U12 staged in LDS;
//   A1. the first panel's row interchanges applied to every other column (the
//       swaps compose to one permutation of at most 2 NB rows: each wavefront
//       gathers its columns' affected rows, then scatters them), fused with
//       the block row U12 = inv(L11) A12 on MFMA;
//   B2, P2. the second panel, brought up to date by the first, factorised;
//   A2. its interchanges and U12 rows, which right of the pair still lack the
//       first panel's update: that comes in through M = inv(L11_2) L_top,1.
// After the last pair, U x = y is solved by 32-row blocks from the bottom.
#include "cs_internal.h"

#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <tuple>

namespace cs {

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

// The 16 x 16 x 4 matrix-core step for each element type.  Operands: lane
// (li, lk) = (lane % 16, lane / 16) gives A[li][lk] and B[lk][li]; its four
// accumulator registers hold column li of rows row(lk, 0..3).
template <class T> struct Mfma;
template <> struct Mfma<double> {
  typedef dvec4 acc;
  static __device__ inline acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ constexpr int row(int lk, int q) { return lk + 4 * q; }
};
template <> struct Mfma<float> {
  typedef fvec4 acc;
  static __device__ inline acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ constexpr int row(int lk, int q) { return 4 * lk + q; }
};

constexpr int LU_NB = 32;             // panel width
constexpr int LU_CW = 16;             // columns per LDS transposition chunk
// LDS chunk layout: row r, column c (< 16) at r * 17 + c (the padding
// spreads a column over the banks for the row-wise reads)
constexpr int PLD = LU_CW + 1;
__device__ inline int chunk_at(int r, int c) { return r * PLD + c; }
constexpr int LU_KK = LU_NB / 4;      // k-steps of the 16x16x4 MFMA per panel
constexpr int LU_KU = 2 * LU_NB;     // rank of the trailing update (a panel pair)

// Launch geometry: W wavefronts per matrix.  Every element goes through the
// same operations in the same order whatever W is (pivot ties go to the lower
// position, each MFMA tile and group covers the same rows and columns), so the
// factors do not depend on it.
//   W = 8: 512 threads, panel rows tid and tid + 512 (orders up to 1,024); the
//          16-column chunk of the panel update holds every row below the
//          first panel.
//   W = 4: 256 threads, three panel rows per thread (orders up to 768); the
//          chunk holds 256 rows at a time.  In FP64 two workgroups fit a CU
//          (registers and LDS), so that one matrix's latency-bound panel runs
//          beside another matrix's trailing update.
template <int W>
struct LuGeo {
  static constexpr int WAVES = W;
  static constexpr int THREADS = 64 * W;
  static constexpr int R = W == 8 ? 2 : 3;            // panel rows per thread
  static constexpr int MAX_N = R * THREADS;
  static constexpr int PASS_ROWS = W == 8 ? MAX_N : THREADS;   // chunk rows per pass
  // smallest chunk area: the pair's coupling term (two 32 x 32 blocks) and
  // staged U12 rows (64 rows of 33 columns; W = 4: of 97, three groups of 32
  // columns per staging pass)
  static constexpr int MIN_CHUNK = W == 8 ? (LU_NB + 1) * LU_KU : (3 * 32 + 1) * LU_KU;
};
constexpr int LU_MAX_N = LuGeo<8>::MAX_N;
// elements of the chunk area of the dynamic LDS: a 16-column chunk of (a pass
// of) the panel rows below the first panel, or the staged U12 rows of the
// trailing update, or the two 32 x 32 blocks of the pair's coupling term
template <int W>
__host__ __device__ inline int chunk_elems(int n) {
  // the chunk holds rows below the first panel (at most n - 32)
  const int rows = n - LU_NB < LuGeo<W>::PASS_ROWS ? n - LU_NB : LuGeo<W>::PASS_ROWS;
  const int c = PLD * rows;
  return c > LuGeo<W>::MIN_CHUNK ? c : LuGeo<W>::MIN_CHUNK;
}
// columns of U12 staged per pass of the trailing update (a multiple of 32;
// the staged rows have a stride of cols + 1 elements)
template <int W>
__device__ inline int u_stage_cols(int n) {
  return ((chunk_elems<W>(n) / LU_KU - 1) / 32) * 32;
}

// static LDS of the kernel
template <class T, int W>
struct LuShared {
  T rows[LU_NB * LU_NB];        // pivot rows of the panel: [L11 | U11]; U block in the solve
  T linv[LU_NB * LU_NB];        // inv(L11), row-major
  // per panel column (two buffers, alternating): each wavefront's pivot
  // candidate, |value| and LAPACK position, and the candidate's whole row
  T slot[2][W][LU_NB];
  T cand_v[2][W];
  int cand_pos[2][W];
  int piv[LU_NB];               // relative pivot positions of the panel
  int bq[LU_NB];                // interchanged rows below the panel's top: position, -1 unused
  int bs[LU_NB];                //   and the position its new content comes from
  int sing, tile;
};

template <class T>
__device__ inline bool better(T v, int pos, T bv, int bpos) {
  return v > bv || (v == bv && pos < bpos);
}

// Per-thread state of the panel factorisation.
template <class T, int W>
struct PanelRows {
  static constexpr int R = LuGeo<W>::R;
  T v[R][LU_NB];           // panel row tid + THREADS s, columns of the panel
  int pos[R];              // its LAPACK position within the panel
  bool live[R];            // not yet chosen as a pivot
};

// Cross-lane moves within a 16-lane row of the wavefront (DPP), for 32-bit
// and 64-bit values.
// (rows outside ROWS keep their own value)
template <int CTRL, int ROWS = 0xF>
__device__ inline int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS = 0xF>
__device__ inline float dpp_move(float v) {
  return __builtin_bit_cast(float, dpp_move<CTRL, ROWS>(__builtin_bit_cast(int, v)));
}
template <int CTRL, int ROWS = 0xF>
__device__ inline double dpp_move(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = dpp_move<CTRL, ROWS>((int)(unsigned)(u & 0xffffffffu));
  const int hi = dpp_move<CTRL, ROWS>((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ inline int read_lane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline float read_lane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ inline double read_lane(double v, int l) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffu), l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
template <class T, int CTRL, int ROWS = 0xF>
__device__ inline void amax_step(T& bv, int& bp) {
  const T v2 = dpp_move<CTRL, ROWS>(bv);
  const int p2 = dpp_move<CTRL, ROWS>(bp);
  if (better(v2, p2, bv, bp)) {
    bv = v2;
    bp = p2;
  }
}
// DPP controls: lane pairs, lane quads, 8-lane halves mirrored, 16-lane rows
// mirrored (after these four every lane of a row holds the row's best); then
// lane 15 of rows 0 and 2 to rows 1 and 3, and lane 31 to rows 2 and 3, after
// which lane 63 holds the wavefront's best
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;
constexpr int DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;
// the same with the candidate's wavefront carried along
template <class T, int CTRL>
__device__ inline void choose_step(T& bv, int& bp, int& bw) {
  const T v2 = dpp_move<CTRL>(bv);
  const int p2 = dpp_move<CTRL>(bp);
  const int w2 = dpp_move<CTRL>(bw);
  if (better(v2, p2, bv, bp)) {
    bv = v2;
    bp = p2;
    bw = w2;
  }
}

// One column J of the panel factorisation (J is a compile-time constant so
// that every register index is static).  One workgroup barrier: each
// wavefront publishes its best candidate (|value|, LAPACK position) and that
// candidate's whole row in the column's LDS buffer; after the barrier every
// thread picks the winner, applies the interchange to the positions of its
// own rows (the winner takes position J, the row at position J takes the
// winner's) and eliminates with the winner's row.  The two buffers alternate
// between columns, so a buffer is rewritten only after the next barrier.
template <class T, int W, int NR, int J>
__device__ __attribute__((always_inline)) inline void panel_column(
    PanelRows<T, W>& R, int m, int r0, int* __restrict__ piv, LuShared<T, W>& S, int tid) {
  // FP32: the wavefront index as a scalar, so that the candidate's LDS
  // address is formed on the scalar unit instead of occupying a vector
  // register
  const int lane = tid & 63;
  const int wave = sizeof(T) == 4 ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6;
  constexpr int BUF = J & 1;
  // --- candidates: largest |a| in column J among rows not yet pivoted
  T bv = T(-1);
  int bp = INT_MAX;
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    // a NaN entry ranks above every number, so a row is always chosen
    const T x = R.v[s][J];
    const T a = (x == x) ? fabs(x) : T(HUGE_VAL);
    if (R.live[s] && better(a, R.pos[s], bv, bp)) {
      bv = a;
      bp = R.pos[s];
    }
  }
  amax_step<T, DPP_XOR1>(bv, bp);
  amax_step<T, DPP_XOR2>(bv, bp);
  amax_step<T, DPP_HALF_MIRROR>(bv, bp);
  amax_step<T, DPP_MIRROR>(bv, bp);
  amax_step<T, DPP_BCAST15, 0xA>(bv, bp);
  amax_step<T, DPP_BCAST31, 0xC>(bv, bp);
  bv = read_lane(bv, 63);
  bp = read_lane(bp, 63);
  if (lane == 0) {
    S.cand_v[BUF][wave] = bv;
    S.cand_pos[BUF][wave] = bp;
  }
  // (only columns J.. are needed by the elimination; the whole pivot rows
  // go to S.rows at the end of the panel)
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    if (R.live[s] && R.pos[s] == bp) {
#pragma unroll
      for (int c = J; c < LU_NB; ++c) S.slot[BUF][wave][c] = R.v[s][c];
    }
  }
  __syncthreads();
  // --- the winner (ties to the lower position, as LAPACK).  The order is
  // total, so the winner does not depend on the order of the reduction.
  int bw;
  if constexpr (sizeof(T) == 4) {
    // every lane reads the W candidates (the same LDS words for all
    // lanes, at fixed addresses) and reduces them in wavefront order: no
    // per-lane address stays live across the columns (in the FP32 kernel,
    // whose register budget is 128, such an address was spilled and
    // reloaded in every column)
    T cv = S.cand_v[BUF][0];
    int cp = S.cand_pos[BUF][0], cw = 0;
#pragma unroll
    for (int w = 1; w < W; ++w) {
      const T v2 = S.cand_v[BUF][w];
      const int p2 = S.cand_pos[BUF][w];
      if (better(v2, p2, cv, cp)) {
        cv = v2;
        cp = p2;
        cw = w;
      }
    }
    bv = read_lane(cv, 0);
    bp = read_lane(cp, 0);
    bw = read_lane(cw, 0);
  } else {
    // lanes 0..W-1 of every wavefront take the W candidates and reduce
    // them on DPP (measured faster in FP64 than the form above)
    T cv = T(-1);
    int cp = INT_MAX, cw = 0;
    if (lane < W) {
      cv = S.cand_v[BUF][lane];
      cp = S.cand_pos[BUF][lane];
      cw = lane;
    }
    choose_step<T, DPP_XOR1>(cv, cp, cw);
    choose_step<T, DPP_XOR2>(cv, cp, cw);
    if constexpr (W > 4) choose_step<T, DPP_HALF_MIRROR>(cv, cp, cw);
    bv = read_lane(cv, 0);
    bp = read_lane(cp, 0);
    bw = read_lane(cw, 0);
  }
  const T* prow = S.slot[BUF][bw];
  // LAPACK interchanges positions J and bp
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    if (R.live[s]) {
      if (R.pos[s] == bp) {
        R.live[s] = false;
        R.pos[s] = J;
      } else if (R.pos[s] == J) {
        R.pos[s] = bp;
      }
    }
  }
  if (tid == 0) {
    S.piv[J] = bp;
    piv[r0 + J] = r0 + bp;
    if (bv == T(0)) S.sing = 1;
  }
  // --- scale and rank-1 update of the rows not yet pivoted
  const T pv = prow[J];
  if (pv != T(0)) {
    const T inv = T(1) / pv;
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      if (R.live[s]) {
        const T l = R.v[s][J] * inv;
        R.v[s][J] = l;
#pragma unroll
        for (int c = J + 1; c < LU_NB; ++c) R.v[s][c] -= l * prow[c];
      }
    }
  }
}

template <class T, int W, int NR, int J>
struct PanelColumns {
  static __device__ __attribute__((always_inline)) inline void run(
      PanelRows<T, W>& R, int m, int r0, int kb, int* piv, LuShared<T, W>& S, int tid) {
    if (J < kb) {
      panel_column<T, W, NR, J>(R, m, r0, piv, S, tid);
      PanelColumns<T, W, NR, J + 1>::run(R, m, r0, kb, piv, S, tid);
    }
  }
};
template <class T, int W, int NR>
struct PanelColumns<T, W, NR, LU_NB> {
  static __device__ __attribute__((always_inline)) inline void run(
      PanelRows<T, W>&, int, int, int, int*, LuShared<T, W>&, int) {}
};

// Factorise the m x kb panel whose rows sit in R.v (row tid + THREADS s of the
// panel, relative to its first row r0, s < NR: m <= NR * THREADS) with all
// threads of the workgroup.
// Rows are never moved while it runs: each keeps its LAPACK position (the
// position it would occupy after the interchanges so far) and a "pivoted"
// flag.  Writes the factored rows to A at their pivoted positions, the
// pivots to piv[] (absolute) and S.piv (relative), L11/U11 to S.rows,
// inv(L11) to S.linv and the rows interchanged below the panel's top to
// S.bq / S.bs, and in ridx[t] (LDS, m ints) the row, relative to r0, that
// ends up at position t.
template <class T, int W, int NR>
__device__ __attribute__((always_inline)) inline void factor_panel(
    PanelRows<T, W>& R, int m, int r0, int kb, T* __restrict__ A, int lda,
    int* __restrict__ piv, int* __restrict__ ridx, LuShared<T, W>& S, int tid) {
  constexpr int NT = LuGeo<W>::THREADS;
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    R.pos[s] = tid + NT * s;
    R.live[s] = R.pos[s] < m;
  }
  __syncthreads();
  PanelColumns<T, W, NR, 0>::run(R, m, r0, kb, piv, S, tid);
  // every row to its pivoted position (columns r0 .. r0+kb); ridx[t] = the
  // row (relative to r0) that ends up at position t; the pivot rows also to
  // S.rows ([L11 | U11])
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int r = tid + NT * s;
    if (r < m) {
      ridx[R.pos[s]] = r;
      if (R.pos[s] < kb) {
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) S.rows[R.pos[s] * LU_NB + c] = R.v[s][c];
      }
      T* dst = A + (size_t)(r0 + R.pos[s]) * lda + r0;
#pragma unroll
      for (int c = 0; c < LU_NB; ++c)
        if (c < kb) dst[c] = R.v[s][c];
    }
  }
  __syncthreads();
  // net permutation: position t < kb now holds the row that was at
  // position ridx[t]; a pivot position q = piv[t] >= kb holds ridx[q]
  // (listed once if repeated)
  if (tid < LU_NB) {
    const int t = tid;
    int q = -1, src = 0;
    if (t < kb) {
      const int p = S.piv[t];
      bool first = p >= kb;
      for (int u = 0; u < t; ++u) first = first && S.piv[u] != p;
      if (first && ridx[p] != p) {
        q = p;
        src = ridx[p];
      }
    }
    S.bq[t] = q;
    S.bs[t] = src;
  }
  // inv(L11), identity-padded to NB: thread j forms column j by forward
  // substitution in registers
  if (tid >= 64 && tid < 64 + LU_NB) {
    const int j = tid - 64;
    T x[LU_NB];
#pragma unroll
    for (int i = 0; i < LU_NB; ++i) {
      T v = (i == j) ? T(1) : T(0);
      if (i < kb) {
#pragma unroll
        for (int k = 0; k < i; ++k) v -= S.rows[i * LU_NB + k] * x[k];
      }
      x[i] = (i < j) ? T(0) : v;
    }
#pragma unroll
    for (int i = 0; i < LU_NB; ++i) S.linv[i * LU_NB + j] = x[i];
  }
}

// C[i0:i0+16, j0:j0+16] - L21[i0:, k0:k0+kb] U12[k0:k0+kb, j0:] (global
// rows, kb <= 64) for rows < n and columns < ncols, written to the LDS chunk
// buffer (rows relative to r0, columns relative to j0)
template <class T>
__device__ inline void update_tile_to_lds(const T* __restrict__ A, int lda, int n,
                                          int ncols, int k0, int kb, int i0, int j0, int r0,
                                          T* __restrict__ P, int lane) {
  const int li = lane & 15, lk = lane >> 4;
  // the accumulator is the tile itself: register q of lane (li, lk) holds
  // column li of row Mfma<T>::row(lk, q)
  const int col = j0 + li;
  const bool cok = col < ncols;
  typename Mfma<T>::acc acc;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = i0 + Mfma<T>::row(lk, q);
    acc[q] = (cok && row < n) ? A[(size_t)row * lda + col] : T(0);
  }
  const int arow = i0 + li;
  const bool aok = arow < n;
  // rank kb <= 64, by halves of 32
  for (int h = 0; h < kb; h += LU_NB) {
    const T* lrow = A + (size_t)arow * lda + k0 + h;
    T a[LU_KK], b[LU_KK];
#pragma unroll
    for (int kk = 0; kk < LU_KK; ++kk) {
      const int k = h + 4 * kk + lk;
      a[kk] = (k < kb && aok) ? lrow[4 * kk + lk] : T(0);
      b[kk] = (k < kb && cok) ? A[(size_t)(k0 + k) * lda + col] : T(0);
    }
    // negated only once every load is in flight (a use right after each load
    // would make it wait for that load alone)
#pragma unroll
    for (int kk = 0; kk < LU_KK; ++kk)
      acc = Mfma<T>::mac(-a[kk], b[kk], acc);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = i0 + Mfma<T>::row(lk, q);
    if (cok && row < n) P[chunk_at(row - r0, li)] = acc[q];
  }
}

// The trailing update on a 32 x 32 group of four tiles, in place: all loads
// of a lane are issued together and every L21 / U12 operand feeds two MFMAs.
// -U12 comes from its copy in LDS (Us: row k of the panel's U12 at k * ldu,
// columns relative to the staged first column c0), so that the L21 operands
// go from memory straight into the MFMAs.
template <class T>
__device__ inline void update_group(T* __restrict__ A, int lda, int n, int ncols,
                                    int k0, int kb, int i0, int j0, const T* __restrict__ Us,
                                    int ldu, int c0, int lane) {
  const int li = lane & 15, lk = lane >> 4;
  typename Mfma<T>::acc acc[2][2];
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
        const int row = i0 + 16 * ti + Mfma<T>::row(lk, q);
        acc[ti][tj][q] = (cok[tj] && row < n) ? A[(size_t)row * lda + col[tj]] : T(0);
      }
  // rank kb <= 64, by halves of 32
  for (int h = 0; h < kb; h += LU_NB) {
    T a[2][LU_KK], b[2][LU_KK];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti) {
      const int arow = i0 + 16 * ti + li;
      const T* lrow = A + (size_t)arow * lda + k0 + h;
#pragma unroll
      for (int kk = 0; kk < LU_KK; ++kk) {
        const int k = h + 4 * kk + lk;
        a[ti][kk] = (k < kb && arow < n) ? lrow[4 * kk + lk] : T(0);
      }
    }
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int kk = 0; kk < LU_KK; ++kk) {
        const int k = h + 4 * kk + lk;
        b[tj][kk] = (k < kb && cok[tj]) ? Us[k * ldu + col[tj] - c0] : T(0);
      }
#pragma unroll
    for (int kk = 0; kk < LU_KK; ++kk)
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = Mfma<T>::mac(a[ti][kk], b[tj][kk], acc[ti][tj]);
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = i0 + 16 * ti + Mfma<T>::row(lk, q);
        if (cok[tj] && row < n) A[(size_t)row * lda + col[tj]] = acc[ti][tj][q];
      }
}

// Back substitution U x = y for the right-hand-side columns n..ncols-1 (the
// forward substitution was done on them during the elimination), by 32-row
// blocks from the bottom.  A wavefront solves a diagonal block for one
// right-hand side at a time (lane i holds row i; x_i is broadcast by a
// scalar read of lane i and eliminated from the rows above), the block
// solution is kept in LDS (xs, 32 x nrhs; ub, 32 x 32 with row i's column j
// at i * 32 + (j ^ i), so that the 32 lanes' reads of one column fall in
// different banks), then every row above is updated.
constexpr int LU_BS = 32;
template <class T, int W>
__device__ void back_substitute(T* __restrict__ A, int lda, int n, int ncols, T* xs, T* ub,
                                int tid) {
  constexpr int NT = LuGeo<W>::THREADS;
  const int lane = tid & 63, wave = tid >> 6;
  const int nrhs = ncols - n;
  if (nrhs <= 0) return;
  const int nblk = (n + LU_BS - 1) / LU_BS;
  for (int b = nblk - 1; b >= 0; --b) {
    const int b0 = b * LU_BS;
    const int bs = min(LU_BS, n - b0);
    for (int e = tid; e < LU_BS * LU_BS; e += NT) {
      const int i = e / LU_BS, j = e % LU_BS;
      ub[i * LU_BS + (j ^ i)] = (i < bs && j < bs) ? A[(size_t)(b0 + i) * lda + b0 + j] : T(0);
    }
    __syncthreads();
    for (int rc = wave; rc < nrhs; rc += W) {
      T y = (lane < bs) ? A[(size_t)(b0 + lane) * lda + n + rc] : T(0);
      for (int i = bs - 1; i >= 0; --i) {
        const T xi = read_lane(y, i) / ub[i * LU_BS];      // the diagonal: (i ^ i) = 0
        if (lane == i) y = xi;
        if (lane < i) y -= ub[lane * LU_BS + (i ^ lane)] * xi;
      }
      if (lane < bs) {
        xs[lane * nrhs + rc] = y;
        A[(size_t)(b0 + lane) * lda + n + rc] = y;
      }
    }
    __syncthreads();
    // y[0:b0] -= U[0:b0, b0:b0+bs] x[b0:b0+bs]
    const int work = b0 * nrhs;
    for (int e = tid; e < work; e += NT) {
      const int i = e / nrhs, rc = e - i * nrhs;
      const T* urow = A + (size_t)i * lda + b0;
      // the block's U entries all in flight before the first is used
      T u[LU_BS];
#pragma unroll
      for (int j = 0; j < LU_BS; ++j) u[j] = (j < bs) ? urow[j] : T(0);
      T acc = A[(size_t)i * lda + n + rc];
#pragma unroll
      for (int j = 0; j < LU_BS; ++j)
        if (j < bs) acc -= u[j] * xs[j * nrhs + rc];
      A[(size_t)i * lda + n + rc] = acc;
    }
    __syncthreads();
  }
}

// Panel columns [k0, k0 + kb) of rows k0.. into the registers R: straight
// from memory when no update is pending (kbp = 0), else after the update by
// L21 / U12 of columns [kp, kp + kbp) (MFMA), passed through the LDS chunk
// buffer P in 16-column chunks, PASS_ROWS rows at a time.  Rows tid + THREADS s
// for s < NR (n - k0 <= NR * THREADS).
template <class T, int W, int NR>
__device__ inline void load_panel(PanelRows<T, W>& R, const T* __restrict__ A, int lda, int n,
                                  int k0, int kb, int kp, int kbp, T* __restrict__ P, int tid) {
  constexpr int NT = LuGeo<W>::THREADS, PR = LuGeo<W>::PASS_ROWS;
  constexpr int NPASS = (NR * NT + PR - 1) / PR;
  const int lane = tid & 63, wave = tid >> 6;
  const int m = n - k0;
  if (kbp == 0) {
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      const int r = tid + NT * s;
#pragma unroll
      for (int c = 0; c < LU_NB; ++c)
        R.v[s][c] = (r < m && c < kb) ? A[(size_t)(k0 + r) * lda + k0 + c] : T(0);
    }
    return;
  }
#pragma unroll
  for (int ch = 0; ch < LU_NB; ch += LU_CW) {
    if (ch < kb) {
      const int cend = k0 + min(kb, ch + LU_CW);
#pragma unroll
      for (int p = 0; p < NPASS; ++p) {
        // rows [p0, p0 + PR) of the panel (a multiple of 16 apart); the
        // condition is the same for the whole workgroup
        const int p0 = p * PR;
        if (p0 < m) {
          const int t0 = p0 >> 4, t1 = (min(m, p0 + PR) + 15) >> 4;
          for (int t = t0 + wave; t < t1; t += W)
            update_tile_to_lds(A, lda, n, cend, kp, kbp, k0 + 16 * t, k0 + ch, k0 + p0, P, lane);
          __syncthreads();
#pragma unroll
          for (int s = 0; s < NR; ++s) {
            if (s * NT >= p0 && s * NT < p0 + PR) {
              const int r = tid + NT * s;
#pragma unroll
              for (int c = 0; c < LU_CW; ++c)
                R.v[s][ch + c] = (r < m && ch + c < kb) ? P[chunk_at(r - p0, c)] : T(0);
            }
          }
          __syncthreads();
        } else {
#pragma unroll
          for (int s = 0; s < NR; ++s)
            if (s * NT >= p0 && s * NT < p0 + PR)
#pragma unroll
              for (int c = 0; c < LU_CW; ++c) R.v[s][ch + c] = T(0);
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < NR; ++s)
#pragma unroll
        for (int c = 0; c < LU_CW; ++c) R.v[s][ch + c] = T(0);
    }
  }
}

// Rows i0.. and columns c1.. of A take the update by L21 / U12 of columns
// [kp, kp + kbp), kbp <= 64.  The U12 rows are staged, negated, in the LDS
// chunk area P, a block of columns per pass, so that every 32 x 32 group
// reads them from there and its L21 operands go from memory straight into
// the MFMAs; groups are handed out by an LDS ticket counter.
template <class T, int W>
__device__ inline void trailing_update(T* __restrict__ A, int lda, int n, int ncols, int kp,
                                       int kbp, int i0, int c1, T* __restrict__ P,
                                       LuShared<T, W>& S, int tid) {
  constexpr int NT = LuGeo<W>::THREADS;
  const int lane = tid & 63;
  const int gr = (n - i0 + 31) >> 5;
  const int cap = u_stage_cols<W>(n);
  for (int c0 = c1; c0 < ncols; c0 += cap) {
    const int w = min(cap, ncols - c0);
    const int ldu = w + 1;
    if (tid == 0) S.tile = 0;
    // eight loads in flight per thread before any of them is used
    const int tot = kbp * w;
    for (int e0 = 0; e0 < tot; e0 += 8 * NT) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * NT + tid;
        const int r = e / w, c = e - r * w;
        v[u] = (e < tot) ? A[(size_t)(kp + r) * lda + c0 + c] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * NT + tid;
        const int r = e / w, c = e - r * w;
        if (e < tot) P[r * ldu + c] = -v[u];
      }
    }
    __syncthreads();
    const int gc = (w + 31) >> 5;
    const int ngroups = gr * gc;
    while (true) {
      int t = 0;
      if (lane == 0) t = atomicAdd(&S.tile, 1);
      t = __shfl(t, 0, 64);
      if (t >= ngroups) break;
      // consecutive tickets walk along a row block: the waves working at the
      // same time share its L21 rows in L2
      const int ti = t / gc, tj = t % gc;
      update_group(A, lda, n, ncols, kp, kbp, i0 + 32 * ti, c0 + 32 * tj, P, ldu, c0, lane);
    }
    __syncthreads();
  }
}

// The interchanges of the panel [k0, k0 + kb) outside its own columns, fused
// with U12 = inv(L11) A12 right of it.  A wavefront takes 16 columns: it
// gathers the kb rows that end up on top (position t comes from position
// ridx[t]) and the interchanged rows below, then writes the latter back and
// the former either as they are (columns left of the panel) or multiplied by
// inv(L11) (to the right).  With Mneg (LDS, 32 x 32, row-major), the right
// side also takes + Mneg U[kc .. kc + kbc) (rows of an earlier panel's U12).
template <class T, int W>
__device__ inline void interchange_trsm(T* __restrict__ A, int lda, int ncols, int k0, int kb,
                                        const int* __restrict__ ridx, const LuShared<T, W>& S,
                                        const T* __restrict__ Mneg, int kc, int kbc, int tid) {
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = k0 + kb;
  const int ntl = k0 >> 4;                       // tiles left of the panel
  const int ntr = (ncols - r0 + 15) >> 4;        // tiles right of it
  int top[LU_KK], bq[LU_KK], bsrc[LU_KK];
#pragma unroll
  for (int kk = 0; kk < LU_KK; ++kk) {
    const int k = 4 * kk + lk;
    top[kk] = (k < kb) ? ridx[k] : k;
    bq[kk] = S.bq[k];
    bsrc[kk] = S.bs[k];
  }
  for (int t = wave; t < ntl + ntr; t += W) {
    const bool right = t >= ntl;
    const int col = right ? r0 + 16 * (t - ntl) + li : 16 * t + li;
    const bool cok = col < ncols;
    const T* colp = A + (size_t)k0 * lda + col;
    T b[LU_KK], v[LU_KK], uc[LU_KK];
#pragma unroll
    for (int kk = 0; kk < LU_KK; ++kk) {
      const int k = 4 * kk + lk;
      b[kk] = (cok && k < kb) ? colp[(size_t)top[kk] * lda] : T(0);
      v[kk] = (cok && bq[kk] >= 0) ? colp[(size_t)bsrc[kk] * lda] : T(0);
      uc[kk] = (Mneg != nullptr && right && cok && k < kbc) ? A[(size_t)(kc + k) * lda + col]
                                                             : T(0);
    }
    // lanes write rows that other lanes of this wavefront read: every load
    // has returned before the first store
    __builtin_amdgcn_s_waitcnt(0);
    T* colw = A + (size_t)k0 * lda + col;
#pragma unroll
    for (int kk = 0; kk < LU_KK; ++kk)
      if (cok && bq[kk] >= 0) colw[(size_t)bq[kk] * lda] = v[kk];
    if (!right) {
#pragma unroll
      for (int kk = 0; kk < LU_KK; ++kk) {
        const int k = 4 * kk + lk;
        if (cok && k < kb) colw[(size_t)k * lda] = b[kk];
      }
    } else {
      typename Mfma<T>::acc acc[2] = {{T(0), T(0), T(0), T(0)}, {T(0), T(0), T(0), T(0)}};
#pragma unroll
      for (int kk = 0; kk < LU_KK; ++kk)
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
          acc[ti] = Mfma<T>::mac(S.linv[(16 * ti + li) * LU_NB + 4 * kk + lk], b[kk], acc[ti]);
      if (Mneg != nullptr) {
#pragma unroll
        for (int kk = 0; kk < LU_KK; ++kk)
#pragma unroll
          for (int ti = 0; ti < 2; ++ti)
            acc[ti] = Mfma<T>::mac(Mneg[(16 * ti + li) * LU_NB + 4 * kk + lk], uc[kk], acc[ti]);
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 16 * ti + Mfma<T>::row(lk, q);
          if (cok && row < kb) colw[(size_t)row * lda] = acc[ti][q];
        }
    }
  }
}

// Load (B) and factorise (P) the panel [k0, k0 + kb) after the pending update
// by columns [kp, kp + kbp).  Four wavefronts: the panel's height picks two or
// three rows per thread.
template <class T, int W>
__device__ __attribute__((always_inline)) inline void panel_step(
    PanelRows<T, W>& R, T* __restrict__ A, int lda, int n, int k0, int kb, int kp,
    int kbp, T* __restrict__ P, int* __restrict__ piv, int* __restrict__ ridx,
    LuShared<T, W>& S, int tid) {
  constexpr int NR = LuGeo<W>::R, NT = LuGeo<W>::THREADS;
  if constexpr (NR == 3) {
    if (n - k0 > 2 * NT) {
      load_panel<T, W, 3>(R, A, lda, n, k0, kb, kp, kbp, P, tid);
      factor_panel<T, W, 3>(R, n - k0, k0, kb, A, lda, piv, ridx, S, tid);
      return;
    }
    load_panel<T, W, 2>(R, A, lda, n, k0, kb, kp, kbp, P, tid);
    factor_panel<T, W, 2>(R, n - k0, k0, kb, A, lda, piv, ridx, S, tid);
  } else {
    load_panel<T, W, NR>(R, A, lda, n, k0, kb, kp, kbp, P, tid);
    factor_panel<T, W, NR>(R, n - k0, k0, kb, A, lda, piv, ridx, S, tid);
  }
}

// Wavefronts per SIMD the register budget is cut for.  FP64: two (eight
// wavefronts: one workgroup of 512 threads or two of 256 per CU; the panel
// rows fill the registers).  FP32: four (two workgroups of 512 threads or four
// of 256 per CU), so that one workgroup's latency-bound panel steps overlap
// another's work.
template <class T>
struct LuWavesPerEu { static constexpr int value = sizeof(T) == 4 ? 4 : 2; };

// ROLE only names the instantiation (LuRole): the KKT systems, the dynamic
// algebraic systems and the FP64 fallback of the mixed-precision solve run
// the same code under their own kernel symbols, so that a profiler's
// per-kernel statistics separate them.
template <class T, int ROLE, int W>
__global__ __launch_bounds__(64 * W, LuWavesPerEu<T>::value) void k_lu_solve(
    T* __restrict__ Abase, size_t stride, int n, int ncols, int lda,
    int* __restrict__ pivbase, int piv_stride, SlotState* __restrict__ st,
    int want_phase, int want_job, int* __restrict__ info, const int* __restrict__ list) {
  // one slot per workgroup: the workgroup's own index, or with a job list
  // (list[0] slots, ids from list[2]) the list's entry, so that the
  // workgroups with work are the first ones dispatched
  int slot = blockIdx.x;
  if (list != nullptr) {
    if ((int)blockIdx.x >= list[0]) return;
    slot = list[2 + blockIdx.x];
  }
  // with slot states: only the slots of one stage that asked for this solve
  if (st != nullptr && (st[slot].job != want_job || st[slot].phase != want_phase)) return;
  T* __restrict__ A = Abase + (size_t)slot * stride;
  int* __restrict__ piv = pivbase + (size_t)slot * piv_stride;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  extern __shared__ __attribute__((aligned(16))) unsigned char lu_lds[];
  T* P = reinterpret_cast<T*>(lu_lds);   // a 16-column chunk (chunk_at); then ridx
  int* ridx = reinterpret_cast<int*>(P + chunk_elems<W>(n));
  __shared__ LuShared<T, W> S;
  if (tid == 0) {
    S.sing = 0;
    S.tile = 0;
  }
  __syncthreads();
  PanelRows<T, W> R;
  constexpr int NT = LuGeo<W>::THREADS;
  // Panels are taken in pairs: the trailing update is applied once per pair
  // with rank 64, which halves the passes over the trailing matrix.
  int kp = 0, kbp = 0;                   // previous pair: columns [kp, kp + kbp)
  for (int k0 = 0; k0 < n; k0 += LU_KU) {
    const int kb1 = min(LU_NB, n - k0);
    const int k1 = k0 + kb1;
    const int kb2 = max(0, min(LU_NB, n - k1));
    const int k2 = k1 + kb2;
    // ---- B1: first panel's columns into registers, after the previous
    // pair's update
    // ---- P1 (with four wavefronts, the third row of each thread only while
    // the panel is taller than 512 rows: the registers of the shorter panels'
    // columns then need no spill slots)
    panel_step(R, A, lda, n, k0, kb1, kp, kbp, P, piv, ridx, S, tid);
    // ---- C: the rest of the previous pair's update (rows from k0, columns
    // right of the first panel), independent of the first panel's factors
    if (kbp > 0 && k1 < ncols) trailing_update(A, lda, n, ncols, kp, kbp, k0, k1, P, S, tid);
    __syncthreads();
    // ---- A1: the first panel's interchanges, U12 of its rows
    interchange_trsm(A, lda, ncols, k0, kb1, ridx, S, (const T*)nullptr, 0, 0, tid);
    __syncthreads();
    if (kb2 > 0) {
      // ---- B2, P2: the second panel after the first panel's update
      panel_step(R, A, lda, n, k1, kb2, k0, kb1, P, piv, ridx, S, tid);
      __syncthreads();
      // ---- A2: the second panel's interchanges; the U12 rows of its top
      // rows right of the pair still lack the first panel's update, so
      //   U12_2 = inv(L11_2) (A_top - L_top,1 U12_1)
      //         = inv(L11_2) A_top - M U12_1,   M = inv(L11_2) L_top,1
      // with L_top,1 the first panel's columns of the rows that the second
      // panel brings to its top (read before A2 moves them).  -M goes to LDS.
      T* Mneg = P + LU_NB * LU_NB;
      if (k2 < ncols) {
        {
          // both elements of a thread in flight together
          T v[LU_NB * LU_NB / NT];
#pragma unroll
          for (int u = 0; u < LU_NB * LU_NB / NT; ++u) {
            const int e = u * NT + tid;
            const int t = e / LU_NB, c = e - t * LU_NB;
            v[u] = (t < kb2 && c < kb1) ? A[(size_t)(k1 + ridx[t]) * lda + k0 + c] : T(0);
          }
#pragma unroll
          for (int u = 0; u < LU_NB * LU_NB / NT; ++u) P[u * NT + tid] = v[u];
        }
        __syncthreads();
        for (int e = tid; e < LU_NB * LU_NB; e += NT) {
          const int i = e / LU_NB, c = e - i * LU_NB;
          T acc = T(0);
#pragma unroll 8
          for (int l = 0; l < LU_NB; ++l) acc += S.linv[i * LU_NB + l] * P[l * LU_NB + c];
          Mneg[e] = -acc;
        }
        __syncthreads();
      }
      interchange_trsm(A, lda, ncols, k1, kb2, ridx, S, (const T*)Mneg, k0, kb1, tid);
      __syncthreads();
    }
    kp = k0;
    kbp = kb1 + kb2;
  }

  back_substitute<T, W>(A, lda, n, ncols, P, S.rows, tid);
  if (tid == 0) {
    if (st != nullptr) st[slot].singular = S.sing;
    if (info != nullptr) info[slot] = S.sing;
  }
}

// static LDS of k_lu_solve
template <class T, int W>
constexpr size_t lu_static_lds() { return sizeof(LuShared<T, W>); }

// dynamic LDS: the chunk area (a 16-column chunk of panel rows, or staged
// U12 rows) and the panel's row-index scratch during the factorisation; a
// 32 x nrhs block during the solve
template <class T, int W>
static size_t lu_dynamic_lds(int n, int nrhs) {
  return std::max(sizeof(T) * (size_t)chunk_elems<W>(n) + sizeof(int) * (size_t)n,
                  sizeof(T) * (size_t)LU_BS * (size_t)nrhs);
}

// total LDS one workgroup of the FP64 k_lu_solve needs for order n and nrhs
// columns, whichever geometry runs it (the FP32 one needs less), with room
// for the compiler's padding of the static part; orders above LU_MAX_N go to
// k_lu_big, whose LDS is static and small
size_t lu_lds_bytes(int n, int nrhs) {
  if (n > LU_MAX_N) return 0;
  size_t b = lu_dynamic_lds<double, 8>(n, nrhs) + lu_static_lds<double, 8>();
  if (n <= LuGeo<4>::MAX_N)
    b = std::max(b, lu_dynamic_lds<double, 4>(n, nrhs) + lu_static_lds<double, 4>());
  return b + 256;
}

// largest order the batched LU entry points take: k_lu_solve up to LU_MAX_N
// (panel rows in registers), k_lu_big above
int lu_max_order() { return 4096; }

// largest order the register-resident kernel takes
int lu_reg_order() { return LU_MAX_N; }

// largest order its four-wavefront geometry takes
int lu_reg_order_w4() { return LuGeo<4>::MAX_N; }

// launch variant per (device, order, precision), set by the autotuner or by
// hand: for k_lu_solve the wavefronts per matrix (4 or 8), for k_lu_big its
// panel code; 0 = not set
static std::mutex g_var_m;
static std::map<std::tuple<int, int, int>, int> g_var;

void lu_set_variant(int device, int n, bool f32, int v) {
  std::lock_guard<std::mutex> lk(g_var_m);
  g_var[std::make_tuple(device, n, f32 ? 1 : 0)] = v;
}

int lu_variant(int device, int n, bool f32) {
  std::lock_guard<std::mutex> lk(g_var_m);
  auto it = g_var.find(std::make_tuple(device, n, f32 ? 1 : 0));
  return it == g_var.end() ? 0 : it->second;
}

// compute units of a device (cached per device)
static int device_cus(int dev) {
  static std::mutex m;
  static std::map<int, int> cus;
  std::lock_guard<std::mutex> lk(m);
  auto it = cus.find(dev);
  if (it != cus.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n = 0;
  cus[dev] = n;
  return n;
}

// wavefronts per matrix for order n: the variant table, else four in FP64
// where the order allows (measured 4-5% faster on the order-580 KKT systems,
// 7% on the order-344 algebraic ones) and eight in FP32 (where four, with its
// four workgroups per CU, spilled and ran a third slower).  max_jobs, when
// known (>= 0), bounds the matrices that have work in the launch: with at most
// one per compute unit no second matrix shares a CU to overlap the panel's
// latency, and eight wavefronts take one matrix 20-25% faster (measured at
// orders 580 and 344 with 16 to 256 systems per launch; 4 is ahead from 320).
// Both geometries give the same bits.
static int lu_waves_for(int n, bool f32, int max_jobs = -1) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int v = lu_variant(dev, n, f32);
  if (v == 8 || n > LuGeo<4>::MAX_N) return 8;
  if (v == 4) return 4;
  if (f32) return 8;
  if (max_jobs >= 0 && max_jobs <= device_cus(dev)) return 8;
  return 4;
}

// launch variant that lu_waves_for picks for order n
int lu_reg_waves(int n, bool f32) { return lu_waves_for(n, f32); }

// grid workgroups: count (one per slot), or with a job list (JobList) the
// list's bound on the slots that have work
template <class T, int ROLE, int W>
static void lu_launch_w(T* A, size_t stride, int n, int ncols, int lda, int* piv,
                        int piv_stride, SlotState* st, int want_phase, int want_job, int count,
                        int* info, hipStream_t stream, const JobList& jl) {
  const size_t lds = lu_dynamic_lds<T, W>(n, ncols - n);
  const int grid = jl.list ? std::min(count, jl.grid) : count;
  if (grid <= 0) return;
  hipLaunchKernelGGL((k_lu_solve<T, ROLE, W>), dim3(grid), dim3(LuGeo<W>::THREADS), lds,
                     stream, A, stride, n, ncols, lda, piv, piv_stride, st, want_phase, want_job,
                     info, jl.list);
}

template <class T, int ROLE>
static void lu_launch(T* A, size_t stride, int n, int ncols, int lda, int* piv, int piv_stride,
                      SlotState* st, int want_phase, int want_job, int count, int* info,
                      hipStream_t stream, int max_jobs = -1, const JobList& jl = JobList{}) {
  if (lu_waves_for(n, sizeof(T) == 4, max_jobs) == 4)
    lu_launch_w<T, ROLE, 4>(A, stride, n, ncols, lda, piv, piv_stride, st, want_phase, want_job,
                            count, info, stream, jl);
  else
    lu_launch_w<T, ROLE, 8>(A, stride, n, ncols, lda, piv, piv_stride, st, want_phase, want_job,
                            count, info, stream, jl);
}

void launch_lu_solve(double* A, size_t stride, int n, int ncols, int lda,
                     int* piv, int piv_stride, SlotState* st, int want_phase, int want_job,
                     int count, int* info, hipStream_t stream, int role, int max_jobs,
                     const JobList& jl) {
  if (count <= 0) return;
  if (n > LU_MAX_N) {
    launch_lu_big(A, stride, n, ncols, lda, piv, piv_stride, st, want_phase, want_job, count,
                  info, stream);
    return;
  }
  if (role == LU_DYN)
    lu_launch<double, LU_DYN>(A, stride, n, ncols, lda, piv, piv_stride, st, want_phase,
                              want_job, count, info, stream, max_jobs, jl);
  else if (role == LU_KKT_FALLBACK)
    lu_launch<double, LU_KKT_FALLBACK>(A, stride, n, ncols, lda, piv, piv_stride, st,
                                       want_phase, want_job, count, info, stream, max_jobs, jl);
  else
    lu_launch<double, LU_KKT>(A, stride, n, ncols, lda, piv, piv_stride, st, want_phase,
                              want_job, count, info, stream, max_jobs, jl);
}

void launch_lu_solve_f32(float* A, size_t stride, int n, int ncols, int lda,
                         int* piv, int piv_stride, SlotState* st, int want_phase, int want_job,
                         int count, int* info, hipStream_t stream, const JobList& jl) {
  if (count <= 0) return;
  if (n > LU_MAX_N) {
    launch_lu_big_f32(A, stride, n, ncols, lda, piv, piv_stride, st, want_phase, want_job, count,
                      info, stream);
    return;
  }
  lu_launch<float, LU_KKT>(A, stride, n, ncols, lda, piv, piv_stride, st, want_phase, want_job,
                           count, info, stream, -1, jl);
}

// the dynamic LDS limit of a kernel: what is left of `bytes` beside its
// static LDS as the compiler laid it out (which may pad the struct)
template <class T, int ROLE, int W>
static void lu_set_attr(size_t bytes) {
  const void* f = reinterpret_cast<const void*>(k_lu_solve<T, ROLE, W>);
  hipFuncAttributes fa;
  size_t fixed = lu_static_lds<T, W>();
  if (hipFuncGetAttributes(&fa, f) == hipSuccess) fixed = std::max(fixed, fa.sharedSizeBytes);
  hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(bytes - fixed));
}

void lu_set_attrs(size_t bytes) {
  lu_set_attr<double, LU_KKT, 8>(bytes);
  lu_set_attr<double, LU_DYN, 8>(bytes);
  lu_set_attr<double, LU_KKT_FALLBACK, 8>(bytes);
  lu_set_attr<float, LU_KKT, 8>(bytes);
  lu_set_attr<double, LU_KKT, 4>(bytes);
  lu_set_attr<double, LU_DYN, 4>(bytes);
  lu_set_attr<double, LU_KKT_FALLBACK, 4>(bytes);
  lu_set_attr<float, LU_KKT, 4>(bytes);
}

}  // namespace cs
