// Diagonal-block preconditioner of Sec. 2.3 (Eq. 6): LU factorisation with
// partial pivoting of each material-domain block A_dd, and the forward/back
// substitutions that apply A_dd^{-1} inside GMRES.
//
// Right-looking blocked LU on a row-major complex FP64 block (leading
// dimension ld): per panel of nb columns, a column-by-column panel
// factorisation (pivot search, row swap inside the panel, scale, rank-1
// update), the panel's row swaps applied to the other columns, a triangular
// solve for the U12 block row, and the trailing update A22 -= L21 U12 on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64, four real products per complex
// product).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vie {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double cabs1(dz a) { return fabs(a.re) + fabs(a.im); }

// copy the diagonal block Z[start:start+n, start:start+n] into A (ld lda)
__global__ void k_copy_block(const dz *__restrict__ Z, int64_t ldz, int64_t start, int n, dz *__restrict__ A,
                             int64_t lda) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c < n) A[(int64_t)r * lda + c] = Z[(start + r) * ldz + start + c];
}

// ------------------------------------------------------------ panel
// Pivot search in column j (rows j..n-1), swap rows j and p inside the panel
// columns [k0, k0+jb), store ipiv[j] = p and the reciprocal pivot.
__global__ __launch_bounds__(1024) void k_lu_pivot(dz *__restrict__ A, int64_t ld, int n, int j, int k0, int jb,
                                                   int32_t *__restrict__ ipiv, dz *__restrict__ rpiv,
                                                   int32_t *__restrict__ info) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const int tid = threadIdx.x;
  double best = -1.0;
  int bi = n;
  for (int i = j + tid; i < n; i += 1024) {
    const double v = cabs1(A[(int64_t)i * ld + j]);
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s) {
      const double o = sv[tid + s];
      const int oi = si[tid + s];
      if (o > sv[tid] || (o == sv[tid] && oi < si[tid])) {
        sv[tid] = o;
        si[tid] = oi;
      }
    }
    __syncthreads();
  }
  const int p = si[0];
  const double pv = sv[0];
  if (tid == 0) ipiv[j] = p;
  if (p != j)
    for (int c = k0 + tid; c < k0 + jb; c += 1024) {
      const dz t = A[(int64_t)j * ld + c];
      A[(int64_t)j * ld + c] = A[(int64_t)p * ld + c];
      A[(int64_t)p * ld + c] = t;
    }
  __syncthreads();
  if (tid == 0) {
    if (!(pv > 0.0)) {
      if (*info == 0) *info = j + 1;
      *rpiv = mk(0.0, 0.0);
    } else {
      const dz d = A[(int64_t)j * ld + j];
      const double den = d.re * d.re + d.im * d.im;
      *rpiv = mk(d.re / den, -d.im / den);
    }
  }
}

// Scale column j below the diagonal and apply the rank-1 update to the rest
// of the panel (columns j+1 .. k0+jb-1).
__global__ __launch_bounds__(256) void k_lu_col(dz *__restrict__ A, int64_t ld, int n, int j, int k0, int jb,
                                                const dz *__restrict__ rpiv) {
  const int i = j + 1 + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dz *row = A + (int64_t)i * ld;
  const dz *prow = A + (int64_t)j * ld;
  const dz l = row[j] * (*rpiv);
  row[j] = l;
  for (int c = j + 1; c < k0 + jb; ++c) row[c] = row[c] - l * prow[c];
}

// Apply the panel's row swaps to the columns outside the panel.
__global__ __launch_bounds__(256) void k_lu_swap(dz *__restrict__ A, int64_t ld, int n, int k0, int jb,
                                                 const int32_t *__restrict__ ipiv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || (c >= k0 && c < k0 + jb)) return;
  for (int j = k0; j < k0 + jb; ++j) {
    const int p = ipiv[j];
    if (p != j) {
      const dz t = A[(int64_t)j * ld + c];
      A[(int64_t)j * ld + c] = A[(int64_t)p * ld + c];
      A[(int64_t)p * ld + c] = t;
    }
  }
}

// U12 = L11^{-1} A12 (L11 unit lower, jb <= 64): one wave per 64 columns, the
// column block lives in LDS.
__global__ __launch_bounds__(64) void k_lu_trsm(dz *__restrict__ A, int64_t ld, int n, int k0, int jb) {
  __shared__ dz tile[64][65];
  const int lane = threadIdx.x;
  const int c = k0 + jb + blockIdx.x * 64 + lane;
  const bool ok = c < n;
  for (int i = 0; i < jb; ++i) tile[i][lane] = ok ? A[(int64_t)(k0 + i) * ld + c] : mk(0, 0);
  for (int i = 1; i < jb; ++i) {
    const dz *Lr = A + (int64_t)(k0 + i) * ld + k0;
    dz s = tile[i][lane];
    for (int l = 0; l < i; ++l) s = s - Lr[l] * tile[l][lane];
    tile[i][lane] = s;
  }
  if (ok)
    for (int i = 1; i < jb; ++i) A[(int64_t)(k0 + i) * ld + c] = tile[i][lane];
}

// A22 -= L21 U12 on the matrix cores.  Tile 64 x 64 per block of 4 waves
// (2 x 2 waves of 32 x 32, each 2 x 2 MFMA tiles of 16 x 16); K = jb <= 64
// staged through LDS in chunks of 16.
//   v_mfma_f64_16x16x4f64 operand layout (lane l): A[i = l%16][k = l/16],
//   B[k = l/16][j = l%16]; result register r holds D[i = 4*r + l/16][j = l%16].
constexpr int kGemmKC = 16;

__global__ __launch_bounds__(256) void k_lu_gemm(dz *__restrict__ A, int64_t ld, int n, int k0, int jb) {
  __shared__ double Ar[64][kGemmKC + 1], Ai[64][kGemmKC + 1];
  __shared__ double Br[kGemmKC][64 + 1], Bi[kGemmKC][64 + 1];
  const int r0 = k0 + jb + blockIdx.y * 64;   // rows of A22
  const int c0 = k0 + jb + blockIdx.x * 64;   // cols of A22
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  v4d cre[2][2], cim[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = v4d{0, 0, 0, 0};
      cim[a][b] = v4d{0, 0, 0, 0};
    }
  for (int kc = 0; kc < jb; kc += kGemmKC) {
    __syncthreads();
    // stage L21[r0.., k0+kc..] (64 x KC) and U12[k0+kc.., c0..] (KC x 64)
    for (int e = tid; e < 64 * kGemmKC; e += 256) {
      const int i = e / kGemmKC, k = e % kGemmKC;
      const int gr = r0 + i, gk = kc + k;
      dz v = mk(0, 0);
      if (gr < n && gk < jb) v = A[(int64_t)gr * ld + k0 + gk];
      Ar[i][k] = v.re;
      Ai[i][k] = v.im;
    }
    for (int e = tid; e < kGemmKC * 64; e += 256) {
      const int k = e / 64, j = e % 64;
      const int gk = kc + k, gc = c0 + j;
      dz v = mk(0, 0);
      if (gk < jb && gc < n) v = A[(int64_t)(k0 + gk) * ld + gc];
      Br[k][j] = v.re;
      Bi[k][j] = v.im;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGemmKC; kk += 4) {
      const int ka = kk + (lane >> 4);
      double are[2], aim[2], bre[2], bim[2];
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
          cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[a], bre[b], cre[a][b], 0, 0, 0);
          cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-aim[a], bim[b], cre[a][b], 0, 0, 0);
          cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[a], bim[b], cim[a][b], 0, 0, 0);
          cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim[a], bre[b], cim[a][b], 0, 0, 0);
        }
    }
  }
  // A22 -= C
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int gi = r0 + wr * 32 + a * 16 + 4 * r + (lane >> 4);
        const int gj = c0 + wc * 32 + b * 16 + (lane & 15);
        if (gi < n && gj < n) {
          dz *p = A + (int64_t)gi * ld + gj;
          const dz v = *p;
          *p = mk(v.re - cre[a][b][r], v.im - cim[a][b][r]);
        }
      }
}

// ------------------------------------------------------------ apply
// perm[i] = original row now at position i, from the sequential swaps ipiv.
__global__ void k_lu_perm(int n, const int32_t *__restrict__ ipiv, int32_t *__restrict__ perm) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int j = 0; j < n; ++j) {
    const int p = ipiv[j];
    const int t = perm[j];
    perm[j] = perm[p];
    perm[p] = t;
  }
}

// z[i] = v[perm[i]] for one block (offset `off` in the global vectors)
__global__ void k_permute(int n, int64_t off, const int32_t *__restrict__ perm, const dz *__restrict__ v,
                          dz *__restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[off + i] = v[off + perm[i]];
}

// Inverses of the nb x nb diagonal blocks of L (unit lower) and U (upper),
// computed once per factorisation and stored TRANSPOSED: block b of DT holds
// inv(T_bb)^T row-major (nb x nb), T_bb the diagonal block at row b*nb.  One
// thread block per diagonal block; thread j forms column j of the inverse
// (row j of DT, contiguous) by substitution.
__global__ __launch_bounds__(128) void k_diag_inv(const dz *__restrict__ F, int64_t ld, int n, int nb, int lower,
                                                  dz *__restrict__ DT) {
  const int b = blockIdx.x;
  const int b0 = b * nb;
  const int m = min(nb, n - b0);
  const int j = threadIdx.x;
  if (j >= nb) return;
  dz *X = DT + ((int64_t)b * nb + j) * nb;   // X[i] = inv(T)[i][j]
  for (int i = 0; i < nb; ++i) X[i] = mk(0, 0);
  if (j >= m) return;
  const dz *T = F + (int64_t)b0 * ld + b0;
  if (lower) {
    X[j] = mk(1, 0);
    for (int i = j + 1; i < m; ++i) {
      dz s = mk(0, 0);
      for (int l = j; l < i; ++l) s = s + T[(int64_t)i * ld + l] * X[l];
      X[i] = mk(0, 0) - s;
    }
  } else {
    auto inv = [](dz d) {
      const double den = d.re * d.re + d.im * d.im;
      return mk(d.re / den, -d.im / den);
    };
    X[j] = inv(T[(int64_t)j * ld + j]);
    for (int i = j - 1; i >= 0; --i) {
      dz s = mk(0, 0);
      for (int l = i + 1; l <= j; ++l) s = s + T[(int64_t)i * ld + l] * X[l];
      X[i] = mk(0, 0) - s * inv(T[(int64_t)i * ld + i]);
    }
  }
}

__device__ __forceinline__ dz wave_sum(dz v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o);
    v.im += __shfl_xor(v.im, o);
  }
  return v;
}

// One block-column step of a blocked triangular solve.  On entry rows
// [b0, b0+m) of rhs are final.  Every thread block (16 waves) forms
// z_b = inv(T_bb) rhs_b: the 128 x 128 product with the transposed inverse
// is split eight ways per row (16 independent, coalesced loads per thread),
// thread block 0 stores z_b into sol, and each block then subtracts
// T[i, b0:b0+m] z_b from its 64 rows still to be solved (below the block for
// L, above it for U), four rows per wave with all loads issued together.
constexpr int kTrsvBlockRows = 64;

__global__ __launch_bounds__(1024) void k_trsv_step(const dz *__restrict__ F, int64_t ld, int n, int b0, int m,
                                                    int lower, const dz *__restrict__ DT, dz *__restrict__ rhs,
                                                    dz *__restrict__ sol) {
  __shared__ dz xb[kTrsvNB];
  __shared__ dz part[8][kTrsvNB];
  __shared__ dz zb[kTrsvNB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < kTrsvNB) xb[tid] = tid < m ? rhs[b0 + tid] : mk(0, 0);
  __syncthreads();
  {
    const int r = tid & (kTrsvNB - 1), h = tid >> 7;   // h = 0..7: columns 16 h .. 16 h + 15
    const dz *col = DT + (int64_t)(h * 16) * kTrsvNB + r;
    dz d[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) d[l] = col[(int64_t)l * kTrsvNB];
    dz s0 = mk(0, 0), s1 = mk(0, 0);
#pragma unroll
    for (int l = 0; l < 16; l += 2) {
      s0 = s0 + d[l] * xb[h * 16 + l];
      s1 = s1 + d[l + 1] * xb[h * 16 + l + 1];
    }
    part[h][r] = s0 + s1;
  }
  __syncthreads();
  if (tid < kTrsvNB) {
    dz z = part[0][tid];
#pragma unroll
    for (int h = 1; h < 8; ++h) z = z + part[h][tid];
    zb[tid] = tid < m ? z : mk(0, 0);
    if (blockIdx.x == 0 && tid < m) sol[b0 + tid] = z;
  }
  __syncthreads();
  int rlo, rhi;
  if (lower) {
    rlo = b0 + m + blockIdx.x * kTrsvBlockRows;
    rhi = min(n, rlo + kTrsvBlockRows);
  } else {
    rlo = blockIdx.x * kTrsvBlockRows;
    rhi = min(b0, rlo + kTrsvBlockRows);
  }
  const dz z0 = zb[lane], z1 = zb[lane + 64];
  const int i0 = rlo + 4 * wave;
  dz s[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + q;
    s[q] = mk(0, 0);
    if (i < rhi) {
      const dz *Fi = F + (int64_t)i * ld + b0;
      if (lane < m) s[q] = Fi[lane] * z0;
      if (lane + 64 < m) s[q] = s[q] + Fi[lane + 64] * z1;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) s[q] = wave_sum(s[q]);
  if (lane < 4 && i0 + lane < rhi) {
    const dz v = lane == 0 ? s[0] : lane == 1 ? s[1] : lane == 2 ? s[2] : s[3];
    rhs[i0 + lane] = rhs[i0 + lane] - v;
  }
}

}  // namespace vie
