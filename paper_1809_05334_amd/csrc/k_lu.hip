// Diagonal-block preconditioner of Sec. 2.3 (Eq. 6): LU factorisation with
// partial pivoting of each material-domain block A_dd (the substitutions that
// apply A_dd^{-1} inside GMRES are in k_trsv.hip).
//
// Right-looking blocked LU on a row-major complex block (leading dimension
// ld), in FP64 (dz) or, for the mixed-precision path, FP32 (fz): per panel of
// nb columns, a column-by-column panel factorisation (pivot search, row swap
// inside the panel, scale, rank-1 update), the panel's row swaps applied to
// the other columns, a triangular solve for the U12 block row, and the
// trailing update A22 -= L21 U12 on the matrix cores (v_mfma_f64_16x16x4f64
// or v_mfma_f32_16x16x4f32, four real products per complex product).  Every
// kernel body is a template on the element type with one __global__ wrapper
// per type (suffix _z: FP64, _c: FP32).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vie {

typedef double v4d __attribute__((ext_vector_type(4)));

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double cabs1(dz a) { return fabs(a.re) + fabs(a.im); }
__device__ __forceinline__ double cabs1(fz a) { return (double)(fabsf(a.re) + fabsf(a.im)); }

// copy the diagonal block Z[start:start+n, start:start+n] into A (ld lda);
// in mixed precision the FP32 far part here, the near part by k_add_near
template <typename C>
__device__ __forceinline__ void copy_block_body(const ZOut &Z, int64_t start, int n, C *__restrict__ A, int64_t lda) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int r = blockIdx.y; r < n; r += gridDim.y) {   // rows grid-strided: gridDim.y is capped by the host
    const int64_t idx = (start + r) * Z.ld + start + c;
    A[(int64_t)r * lda + c] = Z.Z ? cx<C>::of(Z.Z[idx]) : cx<C>::of(Z.Zs[idx]);
  }
}

// A += the FP64 near entries of the diagonal block (one thread per row; the
// sum is formed in FP64 and rounded once)
template <typename C>
__device__ __forceinline__ void add_near_body(const ZOut &Z, int64_t start, int n, C *__restrict__ A, int64_t lda) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t m = start + r;
  for (int64_t e = Z.rowptr[m]; e < Z.rowptr[m + 1]; ++e) {
    const int64_t c = Z.cols[e] - start;
    if (c >= 0 && c < n) A[(int64_t)r * lda + c] = cx<C>::of(to_dz(A[(int64_t)r * lda + c]) + Z.vals[e]);
  }
}

__global__ void k_copy_block_z(ZOut Z, int64_t start, int n, dz *A, int64_t lda) { copy_block_body(Z, start, n, A, lda); }
__global__ void k_copy_block_c(ZOut Z, int64_t start, int n, fz *A, int64_t lda) { copy_block_body(Z, start, n, A, lda); }
__global__ void k_add_near_z(ZOut Z, int64_t start, int n, dz *A, int64_t lda) { add_near_body(Z, start, n, A, lda); }
__global__ void k_add_near_c(ZOut Z, int64_t start, int n, fz *A, int64_t lda) { add_near_body(Z, start, n, A, lda); }

// ------------------------------------------------------------ panel
// Every launch below advances the factorisations of up to kLuMaxDom domains
// at the same global column (domain d's thread blocks start at
// st.d[d].first_block); a domain takes part while the column lies inside it.

__device__ __forceinline__ int lu_domain(const LuStep &st) {
  int d = 0;
  while (d + 1 < st.ndom && (int)blockIdx.x >= st.d[d + 1].first_block) ++d;
  return d;
}

// better pivot candidate: larger |re| + |im|, ties to the smaller row
__device__ __forceinline__ bool piv_better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// Swap rows j and p inside the panel columns [k0, k0 + jb) and store the
// reciprocal pivot (or flag a zero pivot); `tid`/`nthr` stride the columns.
template <typename C>
__device__ __forceinline__ void pivot_finish(const LuDom &D, int j, int k0, int jb, int p, double pv, int tid,
                                             int nthr) {
  typedef typename cx<C>::R R;
  C *A = (C *)D.A;
  if (p != j)
    for (int c = k0 + tid; c < k0 + jb; c += nthr) {
      const C t = A[(int64_t)j * D.ld + c];
      A[(int64_t)j * D.ld + c] = A[(int64_t)p * D.ld + c];
      A[(int64_t)p * D.ld + c] = t;
    }
  __syncthreads();
  if (tid == 0) {
    D.ipiv[j] = p;
    C *rp = (C *)D.rpiv;
    if (!(pv > 0.0)) {
      if (*D.info == 0) *D.info = j + 1;
      *rp = cx<C>::make(0, 0);
    } else {
      const C d = A[(int64_t)j * D.ld + j];
      const R den = d.re * d.re + d.im * d.im;
      *rp = cx<C>::make(d.re / den, -d.im / den);
    }
  }
}

// Pivot of the first column j = k0 of a panel: one thread block per domain.
template <typename C>
__device__ __forceinline__ void lu_pivot_body(const LuStep &st) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const LuDom &D = st.d[blockIdx.x];
  const C *A = (const C *)D.A;
  const int j = st.j, k0 = st.k0, n = D.n, jb = min(kLuNB, n - k0);
  const int tid = threadIdx.x;
  double best = -1.0;
  int bi = n;
  for (int i = j + tid; i < n; i += 1024) {
    const double v = cabs1(A[(int64_t)i * D.ld + j]);
    if (piv_better(v, i, best, bi)) {
      best = v;
      bi = i;
    }
  }
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s && piv_better(sv[tid + s], si[tid + s], sv[tid], si[tid])) {
      sv[tid] = sv[tid + s];
      si[tid] = si[tid + s];
    }
    __syncthreads();
  }
  pivot_finish<C>(D, j, k0, jb, si[0], sv[0], tid, 1024);
}

// Column j of the panel: scale it below the diagonal, apply the rank-1 update
// to the rest of the panel (columns j+1 .. k0+jb-1).  kColT adjacent lanes
// share a row (lane t takes columns j+1+t, j+1+t+kColT, ...), kColRows rows
// per thread block.  When column j+1 is inside the panel, each thread block
// also reduces its rows' pivot candidates in column j+1 into part; the last
// block of the domain to finish (agent-scope acq_rel counter; nothing waits
// on it) picks the pivot of column j+1, swaps it into place inside the panel,
// stores the reciprocal pivot and puts the counter back to zero.
template <typename C>
__device__ __forceinline__ void lu_col_body(const LuStep &st) {
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ int last;
  const int d = lu_domain(st);
  const LuDom &D = st.d[d];
  const int j = st.j, k0 = st.k0, n = D.n, jb = min(kLuNB, n - k0);
  const int blk = blockIdx.x - D.first_block;
  const int tid = threadIdx.x;
  const int t = tid % kColT;
  const int i = j + 1 + blk * kColRows + tid / kColT;
  const bool next = j + 1 < k0 + jb;
  double v = -1.0;
  if (i < n) {
    C *row = (C *)D.A + (int64_t)i * D.ld;
    const C *prow = (const C *)D.A + (int64_t)j * D.ld;
    // the kColT lanes of a row are adjacent lanes of one wave: all read row[j]
    // before lane t == 0 stores the multiplier
    const C l = row[j] * (*(const C *)D.rpiv);
    if (t == 0) row[j] = l;
    for (int c = j + 1 + t; c < k0 + jb; c += kColT) row[c] = row[c] - l * prow[c];
    if (next && t == 0) v = cabs1(row[j + 1]);
  }
  if (!next) return;
  const int nb = (n - j - 1 + kColRows - 1) / kColRows;
  sv[tid] = v;
  si[tid] = (i < n && t == 0) ? i : n;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s && piv_better(sv[tid + s], si[tid + s], sv[tid], si[tid])) {
      sv[tid] = sv[tid + s];
      si[tid] = si[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    D.pval[blk] = sv[0];
    D.pidx[blk] = si[0];
    __threadfence();
    const int old = __hip_atomic_fetch_add(D.counter, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = old == nb - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double best = -1.0;
  int bi = n;
  for (int q = tid; q < nb; q += 256) {
    const double pv = D.pval[q];
    const int pi = D.pidx[q];
    if (piv_better(pv, pi, best, bi)) {
      best = pv;
      bi = pi;
    }
  }
  __syncthreads();
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s && piv_better(sv[tid + s], si[tid + s], sv[tid], si[tid])) {
      sv[tid] = sv[tid + s];
      si[tid] = si[tid + s];
    }
    __syncthreads();
  }
  pivot_finish<C>(D, j + 1, k0, jb, si[0], sv[0], tid, 256);
  if (tid == 0) __hip_atomic_store(D.counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Apply the panel's row swaps to a set of columns (st.all_cols): those
// outside the panel (column pivoting), all of them (tournament pivoting), only
// [c_lo, c_hi) (mode 2: the blocks start at c_lo), or all but [c_lo, c_hi)
// (mode 3).  A pair's swaps can so be applied to its own panels first and to
// the other columns later, in the same order.
template <typename C>
__device__ __forceinline__ void lu_swap_body(const LuStep &st) {
  const LuDom &D = st.d[lu_domain(st)];
  C *A = (C *)D.A;
  const int k0 = st.k0, n = D.n, jb = min(kLuNB, n - k0);
  const int m = st.all_cols;
  const int c = (m == 2 ? st.c_lo : 0) + (blockIdx.x - D.first_block) * 256 + threadIdx.x;
  if (c >= n) return;
  if (m == 0 && c >= k0 && c < k0 + jb) return;
  if (m == 2 && c >= st.c_hi) return;
  if (m == 3 && c >= st.c_lo && c < st.c_hi) return;
  for (int j = k0; j < k0 + jb; ++j) {
    const int p = D.ipiv[j];
    if (p != j) {
      const C t = A[(int64_t)j * D.ld + c];
      A[(int64_t)j * D.ld + c] = A[(int64_t)p * D.ld + c];
      A[(int64_t)p * D.ld + c] = t;
    }
  }
}

// U12 = L11^{-1} A12 (L11 unit lower, jb <= 64) for the columns right of the
// panel (or those of them in [c_lo, c_hi)), kColRows columns per thread
// block: L11 staged in LDS, kColT lanes per column (lane t owns the rows
// i = t (mod kColT) of its column), the dot products of the forward
// substitution split over the lanes and combined by shuffles.
template <typename C>
__device__ __forceinline__ void lu_trsm_body(const LuStep &st) {
  __shared__ C Lt[kLuNB][kLuNB + 1];
  const LuDom &D = st.d[lu_domain(st)];
  const int k0 = st.k0, n = D.n, jb = min(kLuNB, n - k0);
  const int64_t ld = D.ld;
  C *A = (C *)D.A;
  const int tid = threadIdx.x;
  for (int e = tid; e < jb * jb; e += 256) {
    const int r = e / jb, c = e - r * jb;
    Lt[r][c] = A[(int64_t)(k0 + r) * ld + k0 + c];
  }
  __syncthreads();
  constexpr int kPer = kLuNB / kColT;
  const int t = tid % kColT;
  const int cbeg = st.c_hi > 0 ? max(st.c_lo, k0 + jb) : k0 + jb, cend = st.c_hi > 0 ? min(st.c_hi, n) : n;
  const int c = cbeg + (blockIdx.x - D.first_block) * kColRows + tid / kColT;
  const bool ok = c < cend;
  C x[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u)
    x[u] = (ok && kColT * u + t < jb) ? A[(int64_t)(k0 + kColT * u + t) * ld + c] : cx<C>::make(0, 0);
#pragma clang loop unroll(full)
  for (int i = 1; i < kLuNB; ++i) {
    if (i < jb) {
      C s = cx<C>::make(0, 0);
#pragma clang loop unroll(full)
      for (int u = 0; u < kPer; ++u)
        if (kColT * u < i && kColT * u + t < i) s = s + Lt[i][kColT * u + t] * x[u];
      s.re += __shfl_xor(s.re, 1);
      s.im += __shfl_xor(s.im, 1);
      s.re += __shfl_xor(s.re, 2);
      s.im += __shfl_xor(s.im, 2);
      if (t == i % kColT) x[i / kColT] = x[i / kColT] - s;
    }
  }
  if (ok)
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (kColT * u + t < jb) A[(int64_t)(k0 + kColT * u + t) * ld + c] = x[u];
}

// ------------------------------------------------------------ tournament panel
// The pivot rows of a panel are chosen by a reduction tree (tournament
// pivoting) instead of one global search per column:
//   * a leaf thread block runs Gaussian elimination with partial pivoting on
//     a slice of the panel's rows and keeps the kLuNB rows it chose;
//   * up to TsCfg::fan sibling candidate sets are merged by the same elimination
//     on their original rows; the last sibling to finish (agent-scope acq_rel
//     counter of the parent node, put back to zero by that sibling; nothing
//     waits on it) does the merge and climbs on;
//   * the block that reaches the root holds the winners in pivot order and
//     the LU factors of the panel restricted to them: it writes the row swaps
//     (LAPACK order, as the column-by-column panel) and that factored
//     kLuNB x kLuNB top block.
// After the swaps (k_lu_swap over every column), k_lu_tfin stores the top
// block and forms L21 = A21 U11^-1 for the rows below.  The result is an LU
// factorisation P A = L U like partial pivoting's, with pivots chosen per
// panel by the tournament; elimination inside a node is sequential, so the
// tree depth (the panel height over the leaf slice, in powers of the fan-in)
// sets the panel's latency.
//
// Inside a node the rows stay in registers: TsCfg::lpr lanes per row, lane t
// owning the contiguous columns [t W, (t+1) W), W = kLuNB / lpr.  Rows are not
// moved: a pivot row is marked used and its step recorded.  Each step takes
// one barrier: every wave publishes its best candidate (a 64-bit key of the
// magnitude and the row) and that row's remaining columns in LDS,
// double-buffered by the step's parity, and every thread then picks the
// winner of the waves.
template <typename C> struct TsCfg;
template <> struct TsCfg<dz> {
  static constexpr int lpr = kTsLprZ, fan = kTsFanZ, rows = kTsRowsZ;
};
template <> struct TsCfg<fz> {
  static constexpr int lpr = kTsLprC, fan = kTsFanC, rows = kTsRowsC;
};
template <typename C>
struct TsShared {
  static constexpr int kFan = TsCfg<C>::fan, kRows = TsCfg<C>::rows, kLpr = TsCfg<C>::lpr,
                       kThreads = kRows * kLpr, kWaves = kThreads / 64, kW = kLuNB / kLpr;
  C crow[2][kWaves][kLuNB];           // each wave's best candidate row, by step parity
  unsigned long long key[2][kWaves];
  int rid[kRows];                     // the node's rows (rows of the domain)
  int order[kLuNB];                   // node rows in pivot order
  int zero;                           // first zero pivot of the last elimination (1-based), 0 if none
  int flag;
  int nv[kFan];                       // valid candidates of each child
};

template <typename C>
__device__ __forceinline__ C cinv(C d) {
  typedef typename cx<C>::R R;
  const R den = d.re * d.re + d.im * d.im;
  if (!(den > R(0))) return cx<C>::make(0, 0);
  const R s = R(1) / den;
  return cx<C>::make(d.re * s, -d.im * s);
}

// x - l p as four fused multiply-adds
template <typename C>
__device__ __forceinline__ C fms(C x, C l, C p) {
  return cx<C>::make(fma(-l.im, -p.im, fma(-l.re, p.re, x.re)), fma(-l.im, p.re, fma(-l.re, p.im, x.im)));
}

// Pivot key: the magnitude rounded to FP32 (its bits order like the value)
// above the complement of the row, so a larger key is a larger magnitude, ties
// to the smaller row; 0 = no candidate.
__device__ __forceinline__ unsigned long long ts_key(double v, int r) {
  return ((unsigned long long)__float_as_uint((float)v) << 32) | (unsigned)(0x7fffffff - r);
}
__device__ __forceinline__ int ts_key_row(unsigned long long k) { return 0x7fffffff - (int)(k & 0xffffffffu); }

// Maximum of a 64-bit key over the wave, returned to every lane: DPP lane
// permutations inside each row of 16 lanes (quad swaps, half-row and row
// mirrors), then the four row maxima read out of lanes 0, 16, 32, 48.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long k) {
  unsigned long long o;
  o = dpp64<0xb1>(k);    // quad_perm [1,0,3,2]
  k = o > k ? o : k;
  o = dpp64<0x4e>(k);    // quad_perm [2,3,0,1]
  k = o > k ? o : k;
  o = dpp64<0x141>(k);   // row_half_mirror
  k = o > k ? o : k;
  o = dpp64<0x140>(k);   // row_mirror
  k = o > k ? o : k;
  unsigned long long m = readlane64(k, 0);
  o = readlane64(k, 16);
  m = o > m ? o : m;
  o = readlane64(k, 32);
  m = o > m ? o : m;
  o = readlane64(k, 48);
  return o > m ? o : m;
}

// This lane's columns of its row (row tid / lpr of S.rid, m valid rows; a
// row outside the domain is read as zeros).
template <typename C>
__device__ __forceinline__ void ts_load(const TsShared<C> &S, const C *__restrict__ A, int64_t ld, int n, int k0,
                                        int m, int jb, C (&x)[TsShared<C>::kW]) {
  constexpr int L = TsShared<C>::kLpr, W = TsShared<C>::kW;
  const int r = threadIdx.x / L, t = threadIdx.x % L;
  const int g = r < m ? S.rid[r] : -1;
  const bool ok = g >= 0 && g < n;
  const C *row = A + (int64_t)(ok ? g : 0) * ld + k0 + t * W;
#pragma unroll
  for (int i = 0; i < W; ++i) x[i] = (ok && t * W + i < jb) ? row[i] : cx<C>::make(0, 0);
}

// Partial-pivoting elimination of the m x jb matrix held in x (m <= kRows
// rows, S.rid): on return S.order[0 .. min(m, jb)) lists the pivot rows in
// order, *step is this row's pivot step (-1 if none) and x holds L\U of the
// panel restricted to the pivot rows.  Step j works on column j in block
// b = (j mod W) / 8 of its owner lane o = j / W; the owner keeps column j in
// the first register of that block by rotating the block one register per
// step, so every register index is static with only the loop over blocks
// unrolled (the loop over the 8 steps of a block is not: small code).
template <typename C>
__device__ __forceinline__ void ts_gepp(TsShared<C> &S, C (&x)[TsShared<C>::kW], int m, int jb, int *step) {
  constexpr int L = TsShared<C>::kLpr, W = TsShared<C>::kW, NB = W / 8;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = tid / L, t = tid % L;
  const bool valid = r < m;
  const int steps = min(m, jb);
  bool used = false;
  int zero = 0;
  *step = -1;
#pragma unroll
  for (int o = 0; o < L; ++o) {
    const bool owner = t == o;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j0 = o * W + 8 * b;
      if (j0 >= steps) break;
#pragma clang loop unroll(disable)
      for (int jt = 0; jt < 8; ++jt) {
        const int j = j0 + jt;
        if (j < steps) {
          const int buf = j & 1;
          // the non-owner lanes of a row carry no candidate (key 0)
          const unsigned long long k =
              wave_max_u64((owner && valid && !used) ? ts_key(cabs1(x[8 * b]), r) : 0ull);
          if (k != 0ull && r == ts_key_row(k)) {   // the wave's best row: columns j .. kLuNB-1
            C *dst = S.crow[buf][wave];
            if (owner) {
#pragma unroll
              for (int kk = 0; kk < 8; ++kk)
                if (kk + jt < 8) dst[j0 + kk + jt] = x[8 * b + kk];
#pragma unroll
              for (int bb = b + 1; bb < NB; ++bb)
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) dst[o * W + 8 * bb + kk] = x[8 * bb + kk];
            } else if (t > o) {
#pragma unroll
              for (int i = 0; i < W; ++i) dst[t * W + i] = x[i];
            }
          }
          if (lane == 0) S.key[buf][wave] = k;
          __syncthreads();
          unsigned long long best = S.key[buf][0];
          int wb = 0;
#pragma unroll
          for (int w = 1; w < TsShared<C>::kWaves; ++w) {
            const unsigned long long kw = S.key[buf][w];
            if (kw > best) {
              best = kw;
              wb = w;
            }
          }
          const int p = ts_key_row(best);
          const bool nonzero = (best >> 32) != 0ull;
          if (!nonzero && zero == 0) zero = j + 1;
          if (r == p) {   // the pivot row: not updated any more
            used = true;
            *step = j;
          }
          if (tid == 0) S.order[j] = best != 0ull ? p : -1;
          const C *prow = S.crow[buf][wb];
          const C lraw = x[8 * b] * cinv(prow[j]);
          C l = lraw;
          if (L > 1) l = cx<C>::make(__shfl(lraw.re, (lane & ~(L - 1)) | o), __shfl(lraw.im, (lane & ~(L - 1)) | o));
          if (valid && !used && nonzero) {
            if (owner) {
              C pv[8];
#pragma unroll
              for (int kk = 1; kk < 8; ++kk) pv[kk] = prow[j0 + min(kk + jt, 7)];
#pragma unroll
              for (int kk = 1; kk < 8; ++kk)
                if (kk + jt < 8) x[8 * b + kk] = fms(x[8 * b + kk], l, pv[kk]);
#pragma unroll
              for (int bb = b + 1; bb < NB; ++bb) {
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) pv[kk] = prow[o * W + 8 * bb + kk];
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) x[8 * bb + kk] = fms(x[8 * bb + kk], l, pv[kk]);
              }
              x[8 * b] = l;
            } else if (t > o) {
#pragma unroll
              for (int bb = 0; bb < NB; ++bb) {
                C pv[8];
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) pv[kk] = prow[t * W + 8 * bb + kk];
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) x[8 * bb + kk] = fms(x[8 * bb + kk], l, pv[kk]);
              }
            }
          }
        }
        // the owner rotates its block: column j + 1 to the front (after 8
        // steps the block is back in column order)
        if (owner) {
          const C f = x[8 * b];
#pragma unroll
          for (int kk = 0; kk < 7; ++kk) x[8 * b + kk] = x[8 * b + kk + 1];
          x[8 * b + 7] = f;
        }
      }
    }
  }
  __syncthreads();   // S.order complete; the LDS rows may be reused
  if (tid == 0) S.zero = zero;
}

// The row of the domain chosen at step j of the last elimination, -1 if the
// record is out of range (a defect the root reports through info).
template <typename C>
__device__ __forceinline__ int ts_winner(const TsShared<C> &S, int j, int m) {
  const int o = S.order[j];
  return (o >= 0 && o < m) ? S.rid[o] : -1;
}

template <typename C>
__device__ __forceinline__ void lu_tsel_body(const LuStep &st) {
  __shared__ TsShared<C> S;
  constexpr int kRows = TsShared<C>::kRows, kFan = TsShared<C>::kFan;
  const int d = lu_domain(st);
  const LuDom &D = st.d[d];
  const C *A = (const C *)D.A;
  const int k0 = st.k0, n = D.n, jb = min(kLuNB, n - k0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int q = blockIdx.x - D.first_block;
  C x[TsShared<C>::kW];
  int step;
  // leaf: rows k0 + q kRows ...
  const int r0 = k0 + q * kRows;
  int m = min(kRows, n - r0);
  if (tid < m) S.rid[tid] = r0 + tid;
  __syncthreads();
  int cnt = (n - k0 + kRows - 1) / kRows;   // nodes on this level
  int base = 0;                             // first node id of this level
  // one elimination per node this block takes: its leaf, then each merge
  for (;;) {
    ts_load(S, A, D.ld, n, k0, m, jb, x);
    ts_gepp(S, x, m, jb, &step);
    bool merged = false;
    while (cnt > 1 && !merged) {
      const int nc = min(m, jb);
      const int first = q & ~(kFan - 1), nchild = min(kFan, cnt - first);
      const int pbase = base + cnt, parent = pbase + q / kFan;
      if (nchild > 1) {
        // candidate lists pass between thread blocks through agent-scope
        // atomic stores and loads; the last of the siblings to finish merges
        if (tid < kLuNB)
          __hip_atomic_store(D.cand + (int64_t)(base + q) * kLuNB + tid, tid < nc ? ts_winner(S, tid, m) : -1,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        __syncthreads();
        if (tid == 0) {
          const int old = __hip_atomic_fetch_add(D.tcnt + parent, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
          S.flag = old == nchild - 1;
          if (S.flag) __hip_atomic_store(D.tcnt + parent, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (!S.flag) return;   // a sibling merges
        __threadfence();
        // the children are consecutive nodes; wave w < nchild loads child w,
        // compacted in child order with empty entries dropped
        int *c0 = D.cand + (int64_t)(base + first) * kLuNB;
        const int rr = wave < nchild ? __hip_atomic_load(c0 + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
        const unsigned long long vm = __ballot(rr >= 0);
        if (lane == 0 && wave < kFan) S.nv[wave] = wave < nchild ? __popcll(vm) : 0;
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave && w < kFan; ++w) off += S.nv[w];
        if (rr >= 0) S.rid[off + __popcll(vm & ((1ull << lane) - 1ull))] = rr;
        m = 0;
        for (int w = 0; w < kFan; ++w) m += S.nv[w];
        __syncthreads();
        merged = true;
      }   // else alone in its group: its candidates go up unchanged
      base = pbase;
      cnt = (cnt + kFan - 1) / kFan;
      q /= kFan;
    }
    if (!merged) break;   // cnt == 1: this block holds the root
  }
  // root: the pivot rows in S.order, their LU in the registers of their lanes
  {
    constexpr int L = TsShared<C>::kLpr, W = TsShared<C>::kW;
    C *T = (C *)D.tblk;
    const int t = tid % L;
    if (step >= 0)
#pragma unroll
      for (int i = 0; i < W; ++i)
        if (t * W + i < jb) T[step * kLuNB + t * W + i] = x[i];
  }
  // LAPACK-order swaps, by wave 0 alone: step j swaps position k0+j with the
  // current position of winner j.  Lane e holds entry e of the list of rows
  // that left their positions (dr) and where they are now (dp); lane j keeps
  // the swap of step j.
  if (wave == 0) {
    int dr = -1, dp = -1, nd = 0, ipv = 0;
    bool bad = false;
    for (int j = 0; j < jb; ++j) {
      const int w = ts_winner(S, j, m), tgt = k0 + j;
      bad = bad || w < k0 || w >= n;
      const unsigned long long fw = __ballot(dr == w), fy = __ballot(dp == tgt);
      const int iw = fw ? __ffsll((long long)fw) - 1 : -1, iy = fy ? __ffsll((long long)fy) - 1 : -1;
      const int p = iw >= 0 ? __builtin_amdgcn_readlane(dp, iw) : w;
      if (lane == j) ipv = p;
      if (p != tgt) {
        const int y = iy >= 0 ? __builtin_amdgcn_readlane(dr, iy) : tgt;   // the row now at tgt moves to p
        if (lane == iw) dp = tgt;
        if (iy >= 0) {
          if (lane == iy) dp = p;
        } else {
          if (lane == nd) {
            dr = y;
            dp = p;
          }
          ++nd;
        }
      }
    }
    if (bad) {   // never expected: keep the factorisation in bounds and report it
      if (lane < jb) D.ipiv[k0 + lane] = k0 + lane;
      if (lane == 0) *D.info = -1;
    } else {
      if (lane < jb) D.ipiv[k0 + lane] = ipv;
      if (lane == 0 && S.zero && *D.info == 0) *D.info = k0 + S.zero;
    }
  }
}

// Store the factored top block (thread block 0 of the domain) and solve
// x U11 = a for every row below it, kColT lanes per row: lane t owns the
// columns j = t (mod kColT), the dot products are split over the lanes and
// combined by shuffles.
template <typename C>
__device__ __forceinline__ void lu_tfin_body(const LuStep &st) {
  __shared__ C U[kLuNB][kLuNB + 1];
  __shared__ C rinv[kLuNB];
  const LuDom &D = st.d[lu_domain(st)];
  const int k0 = st.k0, n = D.n, jb = min(kLuNB, n - k0);
  const int blk = blockIdx.x - D.first_block;
  const int tid = threadIdx.x;
  const C *T = (const C *)D.tblk;
  C *A = (C *)D.A;
  for (int e = tid; e < jb * jb; e += 256) {
    const int r = e / jb, c = e - r * jb;
    U[r][c] = T[r * kLuNB + c];
  }
  __syncthreads();
  if (tid < jb) rinv[tid] = cinv(U[tid][tid]);
  if (blk == 0)
    for (int e = tid; e < jb * jb; e += 256) {
      const int r = e / jb, c = e - r * jb;
      A[(int64_t)(k0 + r) * D.ld + k0 + c] = U[r][c];
    }
  __syncthreads();
  constexpr int kPer = kLuNB / kColT;
  const int t = tid % kColT;
  const int i = k0 + jb + blk * kColRows + tid / kColT;
  const bool ok = i < n;
  C *row = A + (int64_t)(ok ? i : 0) * D.ld + k0;
  C x[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) x[u] = (ok && kColT * u + t < jb) ? row[kColT * u + t] : cx<C>::make(0, 0);
#pragma clang loop unroll(full)
  for (int j = 0; j < kLuNB; ++j) {
    if (j < jb) {
      C s = cx<C>::make(0, 0);
#pragma clang loop unroll(full)
      for (int u = 0; u < kPer; ++u)
        if (kColT * u < j && kColT * u + t < j) s = s + x[u] * U[kColT * u + t][j];
      s.re += __shfl_xor(s.re, 1);
      s.im += __shfl_xor(s.im, 1);
      s.re += __shfl_xor(s.re, 2);
      s.im += __shfl_xor(s.im, 2);
      if (t == j % kColT) x[j / kColT] = (x[j / kColT] - s) * rinv[j];
    }
  }
  if (ok)
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (kColT * u + t < jb) row[kColT * u + t] = x[u];
}

// A22 -= L21 U12 on the matrix cores.  Tile 64 x 64 per block of 4 waves
// (2 x 2 waves of 32 x 32, each 2 x 2 MFMA tiles of 16 x 16); K = jb <= 64
// staged through LDS in chunks of 16, the next chunk's loads in flight while
// the current one is multiplied.  Every global load is unconditional, from
// an address clamped into the block, with out-of-range values zeroed: a load
// under a branch is waited for inside the branch.
//   v_mfma_f64_16x16x4f64 operand layout (lane l): A[i = l%16][k = l/16],
//   B[k = l/16][j = l%16]; result register r holds D[i = 4*r + l/16][j = l%16].
//   v_mfma_f32_16x16x4f32: the same operands; result register r holds
//   D[i = 4*(l/16) + r][j = l%16].
constexpr int kGemmKC = 16;

template <typename C> struct Mfma;
template <> struct Mfma<dz> {
  typedef double R;
  typedef v4d Acc;
  static __device__ __forceinline__ Acc mma(R a, R b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int r, int lane) { return 4 * r + (lane >> 4); }
};
template <> struct Mfma<fz> {
  typedef float R;
  typedef v4f Acc;
  static __device__ __forceinline__ Acc mma(R a, R b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int r, int lane) { return 4 * (lane >> 4) + r; }
};

template <typename C>
__device__ __forceinline__ void lu_gemm_body(const LuStep &st) {
  typedef typename Mfma<C>::R R;
  typedef typename Mfma<C>::Acc Acc;
  constexpr int kPerA = 64 * kGemmKC / 256, kPerB = kGemmKC * 64 / 256;
  __shared__ R Ar[64][kGemmKC + 1], Ai[64][kGemmKC + 1];
  __shared__ R Br[kGemmKC][64 + 1], Bi[kGemmKC][64 + 1];
  const LuDom &D = st.d[lu_domain(st)];
  const int k0 = st.k0, n = D.n, jb = min(kLuNB, n - k0);
  const int64_t ld = D.ld;
  C *__restrict__ A = (C *)D.A;
  const int nt = (n - k0 - jb + 63) / 64;     // tiles per side of A22
  const int nc = st.gcols > 0 ? min(st.gcols, nt - st.gcol0) : nt - st.gcol0;   // column tiles of this launch
  const int tile = blockIdx.x - D.first_block;
  const int r0 = k0 + jb + (tile / nc) * 64;  // rows of A22
  const int c0 = k0 + jb + (st.gcol0 + tile % nc) * 64;  // cols of A22
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  Acc cre[2][2], cim[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = Acc{0, 0, 0, 0};
      cim[a][b] = Acc{0, 0, 0, 0};
    }
  // L21[r0.., k0+kc..] (64 x KC) and U12[k0+kc.., c0..] (KC x 64) of chunk kc
  C va[kPerA], vb[kPerB];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int u = 0; u < kPerA; ++u) {
      const int e = tid + 256 * u, i = e / kGemmKC, k = e % kGemmKC;
      va[u] = A[(int64_t)min(r0 + i, n - 1) * ld + k0 + min(kc + k, jb - 1)];
    }
#pragma unroll
    for (int u = 0; u < kPerB; ++u) {
      const int e = tid + 256 * u, k = e / 64, j = e % 64;
      vb[u] = A[(int64_t)(k0 + min(kc + k, jb - 1)) * ld + min(c0 + j, n - 1)];
    }
  };
  fetch(0);
  for (int kc = 0; kc < jb; kc += kGemmKC) {
    __syncthreads();   // the previous chunk's shared reads are done
#pragma unroll
    for (int u = 0; u < kPerA; ++u) {
      const int e = tid + 256 * u, i = e / kGemmKC, k = e % kGemmKC;
      const bool ok = r0 + i < n && kc + k < jb;
      Ar[i][k] = ok ? va[u].re : R(0);
      Ai[i][k] = ok ? va[u].im : R(0);
    }
#pragma unroll
    for (int u = 0; u < kPerB; ++u) {
      const int e = tid + 256 * u, k = e / 64, j = e % 64;
      const bool ok = kc + k < jb && c0 + j < n;
      Br[k][j] = ok ? vb[u].re : R(0);
      Bi[k][j] = ok ? vb[u].im : R(0);
    }
    __syncthreads();
    fetch(min(kc + kGemmKC, jb - 1));   // the next chunk (clamped; unused past the end)
    __builtin_amdgcn_sched_barrier(0);  // keep its loads ahead of the products
#pragma unroll
    for (int kk = 0; kk < kGemmKC; kk += 4) {
      const int ka = kk + (lane >> 4);
      R are[2], aim[2], bre[2], bim[2];
      for (int a = 0; a < 2; ++a) {
        const int i = wr * 32 + a * 16 + (lane & 15);
        are[a] = Ar[i][ka];
        aim[a] = Ai[i][ka];
      }
      for (int b = 0; b < 2; ++b) {
        const int j = wc * 32 + b * 16 + (lane & 15);
        bre[b] = Br[ka][j];
        bim[b] = Bi[ka][j];
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          cre[a][b] = Mfma<C>::mma(are[a], bre[b], cre[a][b]);
          cre[a][b] = Mfma<C>::mma(-aim[a], bim[b], cre[a][b]);
          cim[a][b] = Mfma<C>::mma(are[a], bim[b], cim[a][b]);
          cim[a][b] = Mfma<C>::mma(aim[a], bre[b], cim[a][b]);
        }
    }
  }
  // A22 -= C, half a wave tile at a time: its eight loads first, then the
  // stores of the in-range entries
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    C old[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = r0 + wr * 32 + a * 16 + Mfma<C>::row(r, lane);
        const int gj = c0 + wc * 32 + b * 16 + (lane & 15);
        old[b][r] = A[(int64_t)min(gi, n - 1) * ld + min(gj, n - 1)];
      }
    __builtin_amdgcn_sched_barrier(0);  // the loads stay together, ahead of the stores
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = r0 + wr * 32 + a * 16 + Mfma<C>::row(r, lane);
        const int gj = c0 + wc * 32 + b * 16 + (lane & 15);
        if (gi < n && gj < n)
          A[(int64_t)gi * ld + gj] = cx<C>::make(old[b][r].re - cre[a][b][r], old[b][r].im - cim[a][b][r]);
      }
  }
}

__global__ __launch_bounds__(256) void k_lu_gemm_z(LuStep st) { lu_gemm_body<dz>(st); }
__global__ __launch_bounds__(256) void k_lu_gemm_c(LuStep st) { lu_gemm_body<fz>(st); }

// Trailing update after a pair of panels: A22 -= [L21_a L21_b] [U12_a; U12_b]
// with K = 2 kLuNB = 128 (the panels at k0 and k0 + 64 both factored and
// their U rows solved), rows and columns from k0 + 128.  Twice the K of the
// single-panel update halves the read-modify-write of A22 per flop.  Tiles
// of TM x TN (FP32: 128 x 128, FP64: 128 x 64) per block of 8 waves (WR x WC),
// each wave MB x NB MFMA tiles of 16 x 16; K staged through LDS in chunks of
// 16 with the next chunk's loads in flight.
//
// Tile order: each domain's blocks are padded to a multiple of 8 and its
// first block is a multiple of 8, so block b runs on XCD b % 8 (workgroups
// go to the XCDs in turn); XCD x takes the tiles [x q, (x + 1) q) of the
// domain's sequence (q = tiles / 8, rounded up), and the sequence walks
// groups of 8 column tiles row by row, so the 64 or so blocks an XCD holds at
// once share 8 row panels of L21 and 8 column panels of U12 in its L2.
template <typename C> struct Gemm2Cfg;
template <> struct Gemm2Cfg<fz> { static constexpr int TM = 128, TN = 128, WR = 2, WC = 4; };
template <> struct Gemm2Cfg<dz> { static constexpr int TM = 128, TN = 64, WR = 4, WC = 2; };
constexpr int kGemm2K = 2 * kLuNB, kGemm2Group = 8;

template <typename C>
__device__ __forceinline__ void lu_gemm2_body(const LuStep &st) {
  typedef typename Mfma<C>::R R;
  typedef typename Mfma<C>::Acc Acc;
  constexpr int TM = Gemm2Cfg<C>::TM, TN = Gemm2Cfg<C>::TN, WR = Gemm2Cfg<C>::WR, WC = Gemm2Cfg<C>::WC;
  constexpr int WM = TM / WR, WN = TN / WC, MB = WM / 16, NB = WN / 16, NT = kGemm2Threads;
  static_assert(WR * WC * 64 == NT, "one wave per wave tile");
  constexpr int kPerA = TM * kGemmKC / NT, kPerB = kGemmKC * TN / NT;
  __shared__ R As[2][TM][kGemmKC + 1];   // [0]: real, [1]: imaginary parts
  __shared__ R Bs[2][kGemmKC][TN + 1];
  const LuDom &D = st.d[lu_domain(st)];
  const int k0 = st.k0, n = D.n, base = k0 + kGemm2K;
  const int64_t ld = D.ld;
  C *__restrict__ A = (C *)D.A;
  const int nr = (n - base + TM - 1) / TM, ntc = (n - base + TN - 1) / TN;
  const int nc = st.gcols > 0 ? min(st.gcols, ntc - st.gcol0) : ntc - st.gcol0;
  const int total = nr * nc, q = (total + 7) / 8;
  const int b = blockIdx.x - D.first_block;
  const int t = (b & 7) * q + (b >> 3);
  if (t >= total) return;
  const int g = t / (kGemm2Group * nr), rem = t - g * kGemm2Group * nr;
  const int gw = min(kGemm2Group, nc - g * kGemm2Group);
  const int r0 = base + (rem / gw) * TM;
  const int c0 = base + (st.gcol0 + g * kGemm2Group + rem % gw) * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  Acc cre[MB][NB], cim[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      cre[a][c] = Acc{0, 0, 0, 0};
      cim[a][c] = Acc{0, 0, 0, 0};
    }
  // L21[r0.., k0+kc..] (TM x KC) and U12[k0+kc.., c0..] (KC x TN); K = 128 <= n - k0.
  // Thread tid loads A rows ar + u (NT / KC), column ak, and B rows bk + u (NT / TN),
  // column bj: uniform bases with 32-bit offsets (a tile spans < 2^31 / ld rows),
  // fixed per thread except for uniform steps, and LDS slots at constant
  // distances from one address per operand.
  constexpr int kRowStepA = NT / kGemmKC, kRowStepB = NT / TN;
  const uint32_t ld32 = (uint32_t)ld, rmax = (uint32_t)(n - 1 - r0), cmax = (uint32_t)(n - 1 - c0);
  const int ar = tid / kGemmKC, ak = tid % kGemmKC, bk = tid / TN, bj = tid % TN;
  const C *__restrict__ Ab = A + (int64_t)r0 * ld + k0;
  const C *__restrict__ Bb = A + (int64_t)k0 * ld + c0;
  uint32_t aoff[kPerA];
#pragma unroll
  for (int u = 0; u < kPerA; ++u) aoff[u] = min((uint32_t)(ar + u * kRowStepA), rmax) * ld32 + ak;
  const uint32_t boff = bk * ld32 + min((uint32_t)bj, cmax);
  bool aok[kPerA];
#pragma unroll
  for (int u = 0; u < kPerA; ++u) aok[u] = (uint32_t)(ar + u * kRowStepA) <= rmax;
  const bool bok = (uint32_t)bj <= cmax;
  R *const sa = &As[0][ar][ak];
  R *const sb = &Bs[0][bk][bj];
  constexpr int kAim = TM * (kGemmKC + 1), kBim = kGemmKC * (TN + 1);   // imaginary - real part
  C va[kPerA], vb[kPerB];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int u = 0; u < kPerA; ++u) va[u] = Ab[aoff[u] + kc];
#pragma unroll
    for (int u = 0; u < kPerB; ++u) vb[u] = Bb[boff + (uint32_t)(kc + u * kRowStepB) * ld32];
  };
  const R *const la = &As[0][wr * WM + (lane & 15)][lane >> 4];
  const R *const lb = &Bs[0][lane >> 4][wc * WN + (lane & 15)];
  fetch(0);
  for (int kc = 0; kc < kGemm2K; kc += kGemmKC) {
    __syncthreads();   // the previous chunk's shared reads are done
#pragma unroll
    for (int u = 0; u < kPerA; ++u) {
      sa[u * kRowStepA * (kGemmKC + 1)] = aok[u] ? va[u].re : R(0);
      sa[u * kRowStepA * (kGemmKC + 1) + kAim] = aok[u] ? va[u].im : R(0);
    }
#pragma unroll
    for (int u = 0; u < kPerB; ++u) {
      sb[u * kRowStepB * (TN + 1)] = bok ? vb[u].re : R(0);
      sb[u * kRowStepB * (TN + 1) + kBim] = bok ? vb[u].im : R(0);
    }
    __syncthreads();
    fetch(min(kc + kGemmKC, kGemm2K - kGemmKC));   // the next chunk (the last one again at the end, unused)
    __builtin_amdgcn_sched_barrier(0);  // keep its loads ahead of the products
#pragma unroll
    for (int kk = 0; kk < kGemmKC; kk += 4) {
      R are[MB], aim[MB], bre[NB], bim[NB];
#pragma unroll
      for (int a = 0; a < MB; ++a) {
        are[a] = la[a * 16 * (kGemmKC + 1) + kk];
        aim[a] = la[a * 16 * (kGemmKC + 1) + kk + kAim];
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        bre[c] = lb[kk * (TN + 1) + c * 16];
        bim[c] = lb[kk * (TN + 1) + c * 16 + kBim];
      }
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) cre[a][c] = Mfma<C>::mma(are[a], bre[c], cre[a][c]);
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) cim[a][c] = Mfma<C>::mma(are[a], bim[c], cim[a][c]);
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) cre[a][c] = Mfma<C>::mma(-aim[a], bim[c], cre[a][c]);
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c) cim[a][c] = Mfma<C>::mma(aim[a], bre[c], cim[a][c]);
    }
  }
  // A22 -= C, one MFMA row of the wave tile at a time: its loads first, then
  // the stores of the in-range entries
  C *__restrict__ Cb = A + (int64_t)r0 * ld + c0;
#pragma unroll
  for (int a = 0; a < MB; ++a) {
    C old[NB][4];
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = wr * WM + a * 16 + Mfma<C>::row(r, lane), j = wc * WN + c * 16 + (lane & 15);
        old[c][r] = Cb[min(i, rmax) * ld32 + min(j, cmax)];
      }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = wr * WM + a * 16 + Mfma<C>::row(r, lane), j = wc * WN + c * 16 + (lane & 15);
        if (i <= rmax && j <= cmax)
          Cb[i * ld32 + j] = cx<C>::make(old[c][r].re - cre[a][c][r], old[c][r].im - cim[a][c][r]);
      }
  }
}

__global__ __launch_bounds__(kGemm2Threads, 4) void k_lu_gemm2_z(LuStep st) { lu_gemm2_body<dz>(st); }
__global__ __launch_bounds__(kGemm2Threads, 4) void k_lu_gemm2_c(LuStep st) { lu_gemm2_body<fz>(st); }

__global__ __launch_bounds__(1024) void k_lu_pivot_z(LuStep st) { lu_pivot_body<dz>(st); }
__global__ __launch_bounds__(1024) void k_lu_pivot_c(LuStep st) { lu_pivot_body<fz>(st); }
__global__ __launch_bounds__(256) void k_lu_col_z(LuStep st) { lu_col_body<dz>(st); }
__global__ __launch_bounds__(256) void k_lu_col_c(LuStep st) { lu_col_body<fz>(st); }
__global__ __launch_bounds__(256) void k_lu_swap_z(LuStep st) { lu_swap_body<dz>(st); }
__global__ __launch_bounds__(256) void k_lu_swap_c(LuStep st) { lu_swap_body<fz>(st); }
__global__ __launch_bounds__(256) void k_lu_trsm_z(LuStep st) { lu_trsm_body<dz>(st); }
__global__ __launch_bounds__(256) void k_lu_trsm_c(LuStep st) { lu_trsm_body<fz>(st); }
__global__ __launch_bounds__(TsShared<dz>::kThreads) void k_lu_tsel_z(LuStep st) { lu_tsel_body<dz>(st); }
__global__ __launch_bounds__(TsShared<fz>::kThreads) void k_lu_tsel_c(LuStep st) { lu_tsel_body<fz>(st); }
__global__ __launch_bounds__(256) void k_lu_tfin_z(LuStep st) { lu_tfin_body<dz>(st); }
__global__ __launch_bounds__(256) void k_lu_tfin_c(LuStep st) { lu_tfin_body<fz>(st); }

}  // namespace vie
