// GMRES building blocks (Sec. 3): dense complex matrix-vector product,
// classical Gram-Schmidt (applied twice) against the Krylov basis, norms,
// Givens rotations on the Hessenberg matrix, and the final small solve.
// All in FP64.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vie {

__device__ __forceinline__ dz wsum(dz v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o);
    v.im += __shfl_xor(v.im, o);
  }
  return v;
}
__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// y = Z x  (or y = b - Z x when b != nullptr).  Z row-major, N x ld.
// A block of 4 waves owns 4*RPW consecutive rows; x is staged through LDS in
// chunks shared by the block, Z is streamed once with non-temporal loads.
// With NV = 2 one pass over Z serves two vectors (the two polarisations of a
// paired solve); each vector's sums run in the same order as with NV = 1.
// Loads are unconditional (rows past N read row N-1 and are never stored,
// staging reads past the chunk are clamped into it): a load under a branch is
// waited for inside the branch, which would serialise a wave's loads.
constexpr int kMvChunk = 1024;

// x chunk [c0, c0+len) of each vector into xs (vector q at q*kMvChunk):
// every load first, as two-double vectors held in registers (copies of the
// complex struct were kept in scratch memory), then the shared stores
typedef double v2d __attribute__((ext_vector_type(2)));
static_assert(kMvChunk == 4 * 256, "four staging loads per thread and vector");
template <int NV>
__device__ __forceinline__ void stage_x(const MvVecs &v, int64_t c0, int len, dz *xs) {
  static_assert(NV == 1 || NV == 2, "one or two vectors");
  const int tid = threadIdx.x;
  const int i0 = min(tid, len - 1), i1 = min(tid + 256, len - 1), i2 = min(tid + 512, len - 1),
            i3 = min(tid + 768, len - 1);
  const v2d *x = reinterpret_cast<const v2d *>(v.x[0] + c0);
  const v2d a0 = x[i0], a1 = x[i1], a2 = x[i2], a3 = x[i3];
  v2d b0 = a0, b1 = a1, b2 = a2, b3 = a3;
  if constexpr (NV == 2) {
    const v2d *y = reinterpret_cast<const v2d *>(v.x[1] + c0);
    b0 = y[i0];
    b1 = y[i1];
    b2 = y[i2];
    b3 = y[i3];
  }
  __syncthreads();   // the previous chunk's shared reads are done
  v2d *o = reinterpret_cast<v2d *>(xs);
  if (tid < len) o[tid] = a0;
  if (tid + 256 < len) o[tid + 256] = a1;
  if (tid + 512 < len) o[tid + 512] = a2;
  if (tid + 768 < len) o[tid + 768] = a3;
  if constexpr (NV == 2) {
    if (tid < len) o[kMvChunk + tid] = b0;
    if (tid + 256 < len) o[kMvChunk + tid + 256] = b1;
    if (tid + 512 < len) o[kMvChunk + tid + 512] = b2;
    if (tid + 768 < len) o[kMvChunk + tid + 768] = b3;
  }
  __syncthreads();
}

template <int RPW, int NV>
__device__ __forceinline__ void matvec_body(const dz *__restrict__ Z, int64_t ld, int64_t N, const MvVecs &v,
                                            dz *xs, int blk) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = ((int64_t)blk * 4 + wave) * RPW;
  double are[NV][RPW], aim[NV][RPW];
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int r = 0; r < RPW; ++r) are[q][r] = aim[q][r] = 0.0;
  const double *Zd = reinterpret_cast<const double *>(Z);
  for (int64_t c0 = 0; c0 < N; c0 += kMvChunk) {
    const int len = (int)min<int64_t>(kMvChunk, N - c0);
    stage_x<NV>(v, c0, len, xs);
    for (int cc = lane; cc < len; cc += 64) {
      double zr[RPW], zi[RPW];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int64_t o = 2 * (min(row0 + r, N - 1) * ld + c0 + cc);
        zr[r] = __builtin_nontemporal_load(Zd + o);
        zi[r] = __builtin_nontemporal_load(Zd + o + 1);
      }
      dz xv[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) xv[q] = xs[q * kMvChunk + cc];
#pragma unroll
      for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          are[q][r] = fma(zr[r], xv[q].re, fma(-zi[r], xv[q].im, are[q][r]));
          aim[q][r] = fma(zr[r], xv[q].im, fma(zi[r], xv[q].re, aim[q][r]));
        }
    }
  }
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int r = 0; r < RPW; ++r) {
      const double sr = wsum(are[q][r]), si = wsum(aim[q][r]);
      const int64_t row = row0 + r;
      if (lane == 0 && row < N) {
        const dz *b = v.b[q];
        if (b) v.y[q][row] = mk(b[row].re - sr, b[row].im - si);
        else v.y[q][row] = mk(sr, si);
      }
    }
}

#define VIE_MATVEC(R)                                                                                           \
  __global__ __launch_bounds__(256) void k_matvec_r##R(const dz *__restrict__ Z, int64_t ld, int64_t N,         \
                                                       const dz *__restrict__ x, const dz *__restrict__ b,      \
                                                       dz *__restrict__ y) {                                    \
    __shared__ dz xs[kMvChunk];                                                                                 \
    const MvVecs v{{x, nullptr}, {b, nullptr}, {y, nullptr}};                                                   \
    matvec_body<R, 1>(Z, ld, N, v, xs, blockIdx.x);                                                                         \
  }                                                                                                             \
  __global__ __launch_bounds__(256) void k_matvec2_r##R(const dz *__restrict__ Z, int64_t ld, int64_t N,        \
                                                        MvVecs v) {                                             \
    __shared__ dz xs[2 * kMvChunk];                                                                             \
    matvec_body<R, 2>(Z, ld, N, v, xs, blockIdx.x);                                                                         \
  }
VIE_MATVEC(2)
VIE_MATVEC(4)
VIE_MATVEC(8)

// y = Z x (or b - Z x) for the mixed-precision operator Z = Zs + Zn: Zs the
// complex-FP32 dense far part (row-major, ld a multiple of 8), Zn the FP64
// near part in CSR.  Arithmetic and accumulation in FP64.  Same row mapping
// as k_matvec; each lane streams two adjacent FP32 entries (16 bytes) per
// row, then the wave adds its rows' near entries.
typedef float v4f __attribute__((ext_vector_type(4)));

template <int RPW, int NV>
__device__ __forceinline__ void matvec_mixed_body(const fz *__restrict__ Zs, int64_t ld, int64_t N,
                                                  const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ cols, const dz *__restrict__ vals,
                                                  const MvVecs &v, dz *xs, int blk) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = ((int64_t)blk * 4 + wave) * RPW;
  double are[NV][RPW], aim[NV][RPW];
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int r = 0; r < RPW; ++r) are[q][r] = aim[q][r] = 0.0;
  for (int64_t c0 = 0; c0 < N; c0 += kMvChunk) {
    const int len = (int)min<int64_t>(kMvChunk, N - c0);
    stage_x<NV>(v, c0, len, xs);
    for (int cc = 2 * lane; cc < len; cc += 128) {
      v4f z[RPW];
#pragma unroll
      for (int r = 0; r < RPW; ++r)
        z[r] = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(Zs + min(row0 + r, N - 1) * ld + c0 + cc));
      dz x0[NV], x1[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        x0[q] = xs[q * kMvChunk + cc];
        x1[q] = cc + 1 < len ? xs[q * kMvChunk + cc + 1] : mk(0, 0);
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          are[q][r] = fma((double)z[r][0], x0[q].re, fma(-(double)z[r][1], x0[q].im, are[q][r]));
          aim[q][r] = fma((double)z[r][0], x0[q].im, fma((double)z[r][1], x0[q].re, aim[q][r]));
          are[q][r] = fma((double)z[r][2], x1[q].re, fma(-(double)z[r][3], x1[q].im, are[q][r]));
          aim[q][r] = fma((double)z[r][2], x1[q].im, fma((double)z[r][3], x1[q].re, aim[q][r]));
        }
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int64_t row = row0 + r;
    if (row < N)
      for (int64_t e = rowptr[row] + lane; e < rowptr[row + 1]; e += 64) {
        const dz nv = vals[e];
        const int c = cols[e];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const dz xv = v.x[q][c];
          are[q][r] = fma(nv.re, xv.re, fma(-nv.im, xv.im, are[q][r]));
          aim[q][r] = fma(nv.re, xv.im, fma(nv.im, xv.re, aim[q][r]));
        }
      }
  }
#pragma unroll
  for (int q = 0; q < NV; ++q)
    for (int r = 0; r < RPW; ++r) {
      const double sr = wsum(are[q][r]), si = wsum(aim[q][r]);
      const int64_t row = row0 + r;
      if (lane == 0 && row < N) {
        const dz *b = v.b[q];
        if (b) v.y[q][row] = mk(b[row].re - sr, b[row].im - si);
        else v.y[q][row] = mk(sr, si);
      }
    }
}

#define VIE_MATVEC_MIXED(R)                                                                                     \
  __global__ __launch_bounds__(256) void k_matvec_mixed_r##R(                                                   \
      const fz *__restrict__ Zs, int64_t ld, int64_t N, const int64_t *__restrict__ rowptr,                     \
      const int32_t *__restrict__ cols, const dz *__restrict__ vals, const dz *__restrict__ x,                  \
      const dz *__restrict__ b, dz *__restrict__ y) {                                                           \
    __shared__ dz xs[kMvChunk];                                                                                 \
    const MvVecs v{{x, nullptr}, {b, nullptr}, {y, nullptr}};                                                   \
    matvec_mixed_body<R, 1>(Zs, ld, N, rowptr, cols, vals, v, xs, blockIdx.x);                                              \
  }                                                                                                             \
  __global__ __launch_bounds__(256) void k_matvec2_mixed_r##R(                                                  \
      const fz *__restrict__ Zs, int64_t ld, int64_t N, const int64_t *__restrict__ rowptr,                     \
      const int32_t *__restrict__ cols, const dz *__restrict__ vals, MvVecs v) {                                \
    __shared__ dz xs[2 * kMvChunk];                                                                             \
    matvec_mixed_body<R, 2>(Zs, ld, N, rowptr, cols, vals, v, xs, blockIdx.x);                                              \
  }
VIE_MATVEC_MIXED(2)
VIE_MATVEC_MIXED(4)
VIE_MATVEC_MIXED(8)

// y[k] = sum_{i<nv} V_i[k] c[i]
__global__ __launch_bounds__(256) void k_combine(const dz *__restrict__ V, int64_t ldv, int nv,
                                                 const dz *__restrict__ c, dz *__restrict__ y, int64_t N) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  dz s = mk(0, 0);
  // eight basis entries in flight at a time; the sum runs in i order
  for (int i0 = 0; i0 < nv; i0 += 8) {
    double vr[8], vi[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const dz v = V[(int64_t)min(i0 + g, nv - 1) * ldv + k];
      vr[g] = v.re;
      vi[g] = v.im;
    }
#pragma unroll
    for (int g = 0; g < 8; ++g)
      if (i0 + g < nv) s = s + mk(vr[g], vi[g]) * c[i0 + g];
  }
  y[k] = s;
}

// partial squared norms per block
__global__ __launch_bounds__(256) void k_norm2(const dz *__restrict__ w, int64_t N, double *__restrict__ part) {
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = min<int64_t>(N, lo + chunk);
  double s = 0;
  for (int64_t k = lo + tid; k < hi; k += 256) s = fma(w[k].re, w[k].re, fma(w[k].im, w[k].im, s));
  s = wsum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (tid == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// out = sqrt(sum part)
__global__ void k_norm_reduce(const double *__restrict__ part, int nblk, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0;
  for (int b0 = 0; b0 < nblk; b0 += 16) {   // sixteen loads in flight, summed in order
    double p[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) p[u] = part[min(b0 + u, nblk - 1)];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (b0 + u < nblk) s += p[u];
  }
  *out = sqrt(s);
}

// v = w / *nrm  (or v = w * scale when nrm == nullptr)
__global__ void k_scale(const dz *__restrict__ w, const double *__restrict__ nrm, dz *__restrict__ v, int64_t N) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double s = 1.0 / *nrm;
  v[k] = s * w[k];
}

__global__ void k_axpy(dz *__restrict__ x, const dz *__restrict__ u, int64_t N) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) x[k] = x[k] + u[k];
}

// 1 / Z_mm (one thread per row).  Z_mm sums the dense entry (FP64, or the
// FP32 far part) and the row's CSR slot for column m when there is a near
// part; a zero diagonal (no physical operator has one) leaves the row unscaled.
__global__ void k_jacobi_diag(int64_t N, ZOut Z, dz *__restrict__ dinv) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  dz d = mk(0.0, 0.0);
  if (Z.Z) d = Z.Z[m * Z.ld + m];
  if (Z.Zs) d = mk((double)Z.Zs[m * Z.ld + m].re, (double)Z.Zs[m * Z.ld + m].im);
  if (Z.rowptr) {
    int64_t lo = Z.rowptr[m], hi = Z.rowptr[m + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (Z.cols[mid] < m) lo = mid + 1;
      else hi = mid;
    }
    if (lo < Z.rowptr[m + 1] && Z.cols[lo] == m) d = d + Z.vals[lo];
  }
  const double den = d.re * d.re + d.im * d.im;
  dinv[m] = den > 0.0 ? mk(d.re / den, -d.im / den) : mk(1.0, 0.0);
}

__global__ void k_jacobi_apply(int64_t N, const dz *__restrict__ dinv, const dz *__restrict__ v, dz *__restrict__ z) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m < N) z[m] = dinv[m] * v[m];
}

__global__ void k_fill_const(dz *__restrict__ x, int64_t N, double re, double im) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) x[k] = mk(re, im);
}

__global__ void k_copy(dz *__restrict__ d, const dz *__restrict__ s, int64_t N) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) d[k] = s[k];
}

// ------------------------------------------------------------ Arnoldi step
// The kernels of one Arnoldi step read the column index j from device memory
// (*jd), so the step issues the same launches for every j and can be
// captured once in a HIP graph and replayed.  k_jinc advances *jd at the end
// of the step.

// vin = V_j
__global__ void k_arn_begin(const dz *__restrict__ V, int64_t ldv, const int *__restrict__ jd, dz *__restrict__ vin,
                            int64_t N) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) vin[k] = V[(int64_t)(*jd) * ldv + k];
}

// partial inner products with V_0 .. V_j (k_dots with nv = j + 1): block
// (x, y) sums chunk x of N for basis vectors 8 y .. 8 y + 7; the grid's y
// extent covers the largest j (blocks past V_j return at once), so every
// group of eight runs at the same time and the launch is the same for every j
__global__ __launch_bounds__(256) void k_dots_j(const dz *__restrict__ V, int64_t ldv, const int *__restrict__ jd,
                                                const dz *__restrict__ w, int64_t N, dz *__restrict__ part) {
  // eight basis vectors per block: their loads are in flight together and one
  // barrier serves the eight block sums (each sum as for one vector)
  constexpr int G = 8;
  __shared__ dz red[G][4];
  const int nv = *jd + 1;
  const int i0 = blockIdx.y * G;
  if (i0 >= nv) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = min<int64_t>(N, lo + chunk);
  {
    double sr[G], si[G];
#pragma unroll
    for (int g = 0; g < G; ++g) sr[g] = si[g] = 0.0;
    for (int64_t k = lo + tid; k < hi; k += 256) {
      const dz ww = w[k];
      double vr[G], vi[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const dz v = V[(int64_t)min(i0 + g, nv - 1) * ldv + k];
        vr[g] = v.re;
        vi[g] = v.im;
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        sr[g] = fma(vr[g], ww.re, fma(vi[g], ww.im, sr[g]));
        si[g] = fma(vr[g], ww.im, fma(-vi[g], ww.re, si[g]));
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const double a = wsum(sr[g]), b = wsum(si[g]);
      if (lane == 0) red[g][wave] = mk(a, b);
    }
    __syncthreads();
    if (tid < G && i0 + tid < nv)
      part[(int64_t)blockIdx.x * nv + i0 + tid] = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
  }
}

// s_i = sum_b part[b][i]; y_i = s_i; H[i][j] = s_i (pass 0) or += s_i (pass 1)
__global__ void k_dots_reduce_j(const dz *__restrict__ part, int nblk, const int *__restrict__ jd,
                                dz *__restrict__ H, int ldh, dz *__restrict__ y, int pass) {
  const int j = *jd, nv = j + 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  dz s = mk(0, 0);
  for (int b0 = 0; b0 < nblk; b0 += 16) {   // sixteen loads in flight, summed in order
    double pr[16], pi[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const dz p = part[(int64_t)min(b0 + u, nblk - 1) * nv + i];
      pr[u] = p.re;
      pi[u] = p.im;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (b0 + u < nblk) s = s + mk(pr[u], pi[u]);
  }
  dz *h = H + (int64_t)j * ldh;
  h[i] = pass ? h[i] + s : s;
  y[i] = s;
}

// w[k] -= sum_{i<=j} V_i[k] c[i]
__global__ __launch_bounds__(256) void k_update_j(const dz *__restrict__ V, int64_t ldv, const int *__restrict__ jd,
                                                  const dz *__restrict__ c, dz *__restrict__ w, int64_t N) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int nv = *jd + 1;
  dz s = w[k];
  // eight basis entries in flight at a time; the updates run in i order
  for (int i0 = 0; i0 < nv; i0 += 8) {
    double vr[8], vi[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const dz v = V[(int64_t)min(i0 + g, nv - 1) * ldv + k];
      vr[g] = v.re;
      vi[g] = v.im;
    }
#pragma unroll
    for (int g = 0; g < 8; ++g)
      if (i0 + g < nv) s = s - mk(vr[g], vi[g]) * c[i0 + g];
  }
  w[k] = s;
}

// V_{j+1} = w / *nrm
__global__ void k_scale_j(const dz *__restrict__ w, const double *__restrict__ nrm, dz *__restrict__ V, int64_t ldv,
                          const int *__restrict__ jd, int64_t N) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double s = 1.0 / *nrm;
  V[(int64_t)(*jd + 1) * ldv + k] = s * w[k];
}

__global__ void k_jset(int *__restrict__ jd, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *jd = v;
}

__global__ void k_jinc(int *__restrict__ jd) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *jd = *jd + 1;
}

// GMRES state on the device: H (ldh x m, column j holds h_{0..j+1, j}),
// Givens cosines (real) and sines (complex), g (m+1).
// Arnoldi column j: h[0..j] from CGS2, hn = ||w||.  Apply the previous
// rotations to column j, form the new one, update g, write |g[j+1]|.
__device__ void givens_step(dz *__restrict__ H, int ldh, int j, double hnv, double *__restrict__ cs,
                            dz *__restrict__ sn, dz *__restrict__ g, double *__restrict__ res) {
  dz *h = H + (int64_t)j * ldh;
  h[j + 1] = mk(hnv, 0.0);
  for (int i = 0; i < j; ++i) {
    // [c  s; -conj(s) c] acting on (h_i, h_{i+1})
    const dz a = h[i], b = h[i + 1];
    h[i] = cs[i] * a + sn[i] * b;
    h[i + 1] = cs[i] * b - conjz(sn[i]) * a;
  }
  const dz a = h[j], b = h[j + 1];
  const double na = sqrt(a.re * a.re + a.im * a.im), nb = sqrt(b.re * b.re + b.im * b.im);
  double c;
  dz s;
  if (na == 0.0) {
    c = 0.0;
    s = mk(1.0, 0.0);
    h[j] = b;
  } else {
    const double t = sqrt(na * na + nb * nb);
    c = na / t;
    const dz al = mk(a.re / na, a.im / na);       // a / |a|
    s = (1.0 / t) * (al * conjz(b));              // alpha conj(b) / t
    h[j] = al * mk(t, 0.0);
  }
  h[j + 1] = mk(0.0, 0.0);
  cs[j] = c;
  sn[j] = s;
  const dz gj = g[j];
  g[j] = c * gj;
  g[j + 1] = mk(0, 0) - conjz(s) * gj;
  *res = sqrt(g[j + 1].re * g[j + 1].re + g[j + 1].im * g[j + 1].im);
}

// k_givens for the j in *jd; also records |g[j+1]| in hist[j]
__global__ void k_givens_j(dz *__restrict__ H, int ldh, const int *__restrict__ jd, const double *__restrict__ hn,
                           double *__restrict__ cs, dz *__restrict__ sn, dz *__restrict__ g,
                           double *__restrict__ hist) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int j = *jd;
  givens_step(H, ldh, j, *hn, cs, sn, g, hist + j);
}

// y = R^{-1} g for the leading k x k upper triangle of H (single thread).
__global__ void k_backsolve(const dz *__restrict__ H, int ldh, int k, const dz *__restrict__ g, dz *__restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    dz s = g[i];
    for (int l = i + 1; l < k; ++l) s = s - H[(int64_t)l * ldh + i] * y[l];
    const dz d = H[(int64_t)i * ldh + i];
    const double den = d.re * d.re + d.im * d.im;
    y[i] = mk((s.re * d.re + s.im * d.im) / den, (s.im * d.re - s.re * d.im) / den);
  }
}

// g = (beta, 0, ..., 0)
__global__ void k_ginit(dz *__restrict__ g, int m1, const double *__restrict__ beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m1) g[i] = i == 0 ? mk(*beta, 0.0) : mk(0.0, 0.0);
}

// ------------------------------------------------------------ fused batch
// The Arnoldi step of many cells at once (one GMRES process per cell): each
// kernel's grid is the concatenation of the cells' grids (pre[c] .. pre[c+1]
// are cell c's blocks), and a cell whose flag act[c] is 0 skips the step.
// Per cell the arithmetic is that of the single-cell kernels, with the
// two-stage reductions over nred blocks of the cell.

__device__ __forceinline__ int cell_of(const int *__restrict__ pre, int nc, int b) {
  int lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

#define VIE_CELL_BEGIN                                \
  const int c_ = cell_of(pre, nc, (int)blockIdx.x);   \
  if (!act[c_]) return;                               \
  const KryCell &K = cells[c_];                       \
  const int lb = (int)blockIdx.x - pre[c_];

// vin = V_j
__global__ void k_b_arn_begin(const KryCell *__restrict__ cells, const int *__restrict__ pre, int nc,
                              const int *__restrict__ act) {
  VIE_CELL_BEGIN
  const int64_t k = (int64_t)lb * blockDim.x + threadIdx.x;
  if (k < K.N) K.vin[k] = K.V[(int64_t)(*K.jd) * K.ldv + k];
}

// rhs of the triangular solves: tmp[off + i] = vin[off + perm[off + i]] per domain
__global__ void k_b_permute(const KryCell *__restrict__ cells, const int *__restrict__ pre, int nc,
                            const int *__restrict__ act) {
  VIE_CELL_BEGIN
  const int64_t k = (int64_t)lb * blockDim.x + threadIdx.x;
  if (k >= K.N) return;
  int64_t off = 0;
  for (int d = 1; d < K.ndom; ++d)
    if (k >= K.dstart[d]) off = K.dstart[d];
  K.tmp[k] = K.vin[off + K.perm[k]];
}

// w = Z z (the operator of the cell's precision); z = vin when unpreconditioned
__global__ __launch_bounds__(256) void k_b_matvec(const KryCell *__restrict__ cells, const int *__restrict__ pre, int nc,
                                                  const int *__restrict__ act) {
  __shared__ dz xs[kMvChunk];
  VIE_CELL_BEGIN
  const MvVecs v{{K.precond ? K.vin : K.z, nullptr}, {nullptr, nullptr}, {K.w, nullptr}};
  // rows per wave: the cell's autotuned shape
  if (K.Z) {
    if (K.rpw == 2) matvec_body<2, 1>(K.Z, K.ld, K.N, v, xs, lb);
    else if (K.rpw == 8) matvec_body<8, 1>(K.Z, K.ld, K.N, v, xs, lb);
    else matvec_body<4, 1>(K.Z, K.ld, K.N, v, xs, lb);
  } else {
    if (K.rpw == 2) matvec_mixed_body<2, 1>(K.Zs, K.ld, K.N, K.rowptr, K.cols, K.vals, v, xs, lb);
    else if (K.rpw == 8) matvec_mixed_body<8, 1>(K.Zs, K.ld, K.N, K.rowptr, K.cols, K.vals, v, xs, lb);
    else matvec_mixed_body<4, 1>(K.Zs, K.ld, K.N, K.rowptr, K.cols, K.vals, v, xs, lb);
  }
}

// partial inner products with V_0 .. V_j: local block (x, y) = chunk x of the
// cell's nred, basis vectors 8 y .. 8 y + 7
__global__ __launch_bounds__(256) void k_b_dots_j(const KryCell *__restrict__ cells, const int *__restrict__ pre, int nc,
                                                  const int *__restrict__ act) {
  constexpr int G = 8;
  __shared__ dz red[G][4];
  VIE_CELL_BEGIN
  const int nv = *K.jd + 1;
  const int bx = lb % K.nred, by = lb / K.nred;
  const int i0 = by * G;
  if (i0 >= nv) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t N = K.N, ldv = K.ldv;
  const int64_t chunk = (N + K.nred - 1) / K.nred;
  const int64_t lo = bx * chunk, hi = min<int64_t>(N, lo + chunk);
  double sr[G], si[G];
#pragma unroll
  for (int g = 0; g < G; ++g) sr[g] = si[g] = 0.0;
  for (int64_t k = lo + tid; k < hi; k += 256) {
    const dz ww = K.w[k];
    double vr[G], vi[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const dz v = K.V[(int64_t)min(i0 + g, nv - 1) * ldv + k];
      vr[g] = v.re;
      vi[g] = v.im;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      sr[g] = fma(vr[g], ww.re, fma(vi[g], ww.im, sr[g]));
      si[g] = fma(vr[g], ww.im, fma(-vi[g], ww.re, si[g]));
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const double a = wsum(sr[g]), b = wsum(si[g]);
    if (lane == 0) red[g][wave] = mk(a, b);
  }
  __syncthreads();
  if (tid < G && i0 + tid < nv)
    K.dpart[(int64_t)bx * nv + i0 + tid] = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
}

// s_i = sum_b part[b][i]; y_i = s_i; H[i][j] = s_i (pass 0) or += s_i (pass 1)
__global__ void k_b_dots_reduce_j(const KryCell *__restrict__ cells, const int *__restrict__ pre, int nc,
                                  const int *__restrict__ act, int pass) {
  VIE_CELL_BEGIN
  const int j = *K.jd, nv = j + 1;
  const int i = lb * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  dz s = mk(0, 0);
  for (int b0 = 0; b0 < K.nred; b0 += 16) {
    double pr[16], pi[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const dz p = K.dpart[(int64_t)min(b0 + u, K.nred - 1) * nv + i];
      pr[u] = p.re;
      pi[u] = p.im;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (b0 + u < K.nred) s = s + mk(pr[u], pi[u]);
  }
  dz *h = K.H + (int64_t)j * K.ldh;
  h[i] = pass ? h[i] + s : s;
  K.y[i] = s;
}

// w -= sum_{i<=j} V_i y_i
__global__ __launch_bounds__(256) void k_b_update_j(const KryCell *__restrict__ cells, const int *__restrict__ pre,
                                                    int nc, const int *__restrict__ act) {
  VIE_CELL_BEGIN
  const int64_t k = (int64_t)lb * blockDim.x + threadIdx.x;
  if (k >= K.N) return;
  const int nv = *K.jd + 1;
  dz s = K.w[k];
  for (int i0 = 0; i0 < nv; i0 += 8) {
    double vr[8], vi[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const dz v = K.V[(int64_t)min(i0 + g, nv - 1) * K.ldv + k];
      vr[g] = v.re;
      vi[g] = v.im;
    }
#pragma unroll
    for (int g = 0; g < 8; ++g)
      if (i0 + g < nv) s = s - mk(vr[g], vi[g]) * K.y[i0 + g];
  }
  K.w[k] = s;
}

// partial squared norms of w over the cell's nred chunks
__global__ __launch_bounds__(256) void k_b_norm2(const KryCell *__restrict__ cells, const int *__restrict__ pre, int nc,
                                                 const int *__restrict__ act) {
  __shared__ double red[4];
  VIE_CELL_BEGIN
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t chunk = (K.N + K.nred - 1) / K.nred;
  const int64_t lo = lb * chunk, hi = min<int64_t>(K.N, lo + chunk);
  double s = 0;
  for (int64_t k = lo + tid; k < hi; k += 256) s = fma(K.w[k].re, K.w[k].re, fma(K.w[k].im, K.w[k].im, s));
  s = wsum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (tid == 0) K.npart[lb] = red[0] + red[1] + red[2] + red[3];
}

// per cell (one thread each): h_{j+1,j} = ||w|| from the partials, then the
// Givens update of column j (|g_{j+1}| into rhist[j])
__global__ void k_b_norm_givens(const KryCell *__restrict__ cells, int nc, const int *__restrict__ act) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc || !act[c]) return;
  const KryCell &K = cells[c];
  double s = 0;
  for (int b0 = 0; b0 < K.nred; b0 += 16) {
    double p[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) p[u] = K.npart[min(b0 + u, K.nred - 1)];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (b0 + u < K.nred) s += p[u];
  }
  const double hn = sqrt(s);
  K.scal[2] = hn;
  givens_step(K.H, K.ldh, *K.jd, hn, K.cs, K.sn, K.g, K.rhist + *K.jd);
}

// V_{j+1} = w / h_{j+1,j}
__global__ void k_b_scale_j(const KryCell *__restrict__ cells, const int *__restrict__ pre, int nc,
                            const int *__restrict__ act) {
  VIE_CELL_BEGIN
  const int64_t k = (int64_t)lb * blockDim.x + threadIdx.x;
  if (k >= K.N) return;
  const double s = 1.0 / K.scal[2];
  K.V[(int64_t)(*K.jd + 1) * K.ldv + k] = s * K.w[k];
}

// per cell: the step's residual estimate |g_{j+1}| into res[c], then j += 1
__global__ void k_b_jinc(const KryCell *__restrict__ cells, int nc, const int *__restrict__ act,
                         double *__restrict__ res) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc || !act[c]) return;
  const KryCell &K = cells[c];
  const int j = *K.jd;
  res[c] = K.rhist[j];
  *K.jd = j + 1;
}
#undef VIE_CELL_BEGIN

}  // namespace vie
