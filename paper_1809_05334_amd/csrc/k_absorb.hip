// Outputs of a solve: absorbed power per material domain (Sec. 3, Eq. 7) and
// the Floquet-mode reflectance / transmittance of the radiated field.
//
// On tetrahedron T, D/eps0 = sum_k c_k (r - v_k) with c_k = x_m psi s a_m / (3 V_T).
//   A_d = k0 / (cos th a b) * sum_{T in d} (-Im eps_T)/|eps_T|^2 int_T |D/eps0|^2 dV
// (4-point rule, exact for the quadratic integrand).  The polarisation
// P/eps0 = kappa D/eps0 radiates into order (p,q) with amplitude
//   e = (k0^2 v - k (k.v)) / (2 a b gamma),  v = int P/eps0 e^{j k.r} dV
// (14-point rule), k = (k_t,pq, +/- beta_pq).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vie {

constexpr int kMaxProp = 32;

__device__ __forceinline__ double bsum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// part[blockIdx.x * ndom + d] = sum over this block's tets in domain d;
// per_tet[t] (if given) = tet t's own term
__global__ __launch_bounds__(256) void k_absorb(int64_t nt, int ndom, const TetGeom *__restrict__ tg,
                                                const TetFace *__restrict__ t2f, const int32_t *__restrict__ dom,
                                                const QuadRules *__restrict__ qr, const dz *__restrict__ gsrc,
                                                const dz *__restrict__ inv_eps, const dz *__restrict__ x,
                                                double *__restrict__ part, double *__restrict__ per_tet) {
  __shared__ double red[4];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double val = 0.0;
  int d = -1;
  if (t < nt) {
    const TetGeom &g = tg[t];
    dz c[4];
    for (int k = 0; k < 4; ++k) c[k] = (1.0 / 3.0) * (x[t2f[4 * t + k].unknown] * gsrc[4 * t + k]);
    double s = 0;
    for (int q = 0; q < 4; ++q) {
      double r[3];
      for (int dd = 0; dd < 3; ++dd) {
        double a = 0;
        for (int k = 0; k < 4; ++k) a = fma(qr->tet4[q][k], g.v[k][dd], a);
        r[dd] = a;
      }
      double e2 = 0;
      for (int dd = 0; dd < 3; ++dd) {
        dz D = mk(0, 0);
        for (int k = 0; k < 4; ++k) axpy(D, r[dd] - g.v[k][dd], c[k]);
        e2 += D.re * D.re + D.im * D.im;
      }
      s = fma(0.25 * g.vol, e2, s);
    }
    val = s * inv_eps[t].im;   // (-Im eps)/|eps|^2 = Im(1/eps)
    d = dom[t];
    if (per_tet) per_tet[t] = val;
  }
  for (int dd = 0; dd < ndom; ++dd) {
    const double v = bsum(d == dd ? val : 0.0, red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * ndom + dd] = v;
  }
}

// Floquet projections: for nk wave vectors kv[3*i] (mode i),
// part[blockIdx.x * nk * 6 + 6 i + (2*comp + re/im)] of v_i = int kappa D e^{j k.r}.
__global__ __launch_bounds__(256) void k_project(int64_t nt, const TetGeom *__restrict__ tg,
                                                 const TetFace *__restrict__ t2f, const QuadRules *__restrict__ qr,
                                                 const dz *__restrict__ gsrc, const dz *__restrict__ kappa,
                                                 const dz *__restrict__ x, int nk, const double *__restrict__ kv,
                                                 double *__restrict__ part) {
  __shared__ double red[4];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = t < nt;
  dz c[4];
  TetGeom g;
  if (ok) {
    g = tg[t];
    const dz kp = kappa[t];
    for (int k = 0; k < 4; ++k) c[k] = (1.0 / 3.0) * (kp * (x[t2f[4 * t + k].unknown] * gsrc[4 * t + k]));
  }
  for (int i = 0; i < nk; ++i) {
    dz v[3] = {mk(0, 0), mk(0, 0), mk(0, 0)};
    if (ok) {
      for (int q = 0; q < 14; ++q) {
        double r[3];
        for (int dd = 0; dd < 3; ++dd) {
          double a = 0;
          for (int k = 0; k < 4; ++k) a = fma(qr->tet14[q][k], g.v[k][dd], a);
          r[dd] = a;
        }
        double sn, cs;
        sincos(kv[3 * i] * r[0] + kv[3 * i + 1] * r[1] + kv[3 * i + 2] * r[2], &sn, &cs);
        const dz ph = (qr->w14[q] * g.vol) * mk(cs, sn);
        for (int dd = 0; dd < 3; ++dd) {
          dz D = mk(0, 0);
          for (int k = 0; k < 4; ++k) axpy(D, r[dd] - g.v[k][dd], c[k]);
          v[dd] = v[dd] + D * ph;
        }
      }
    }
    for (int dd = 0; dd < 3; ++dd) {
      const double re = bsum(v[dd].re, red);
      const double im = bsum(v[dd].im, red);
      if (threadIdx.x == 0) {
        part[((int64_t)blockIdx.x * nk + i) * 6 + 2 * dd] = re;
        part[((int64_t)blockIdx.x * nk + i) * 6 + 2 * dd + 1] = im;
      }
    }
  }
}

// out[j] = sum_b part[b * width + j]
__global__ void k_reduce_cols(const double *__restrict__ part, int nblk, int width, double *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= width) return;
  double s = 0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * width + j];
  out[j] = s;
}

// The field at sample points inside the structure (the field maps of
// Sec. 3): on the tetrahedron T holding point i (tet[i], -1 if none),
// D/eps0 = sum_k c_k (r - v_k) as in k_absorb, and e[3i + d] = (D/eps0)_d / eps_T
// (zero outside).  One lane per point.
__global__ __launch_bounds__(256) void k_field(int64_t np, const double *__restrict__ pts,
                                               const int32_t *__restrict__ tet, const TetGeom *__restrict__ tg,
                                               const TetFace *__restrict__ t2f, const dz *__restrict__ gsrc,
                                               const dz *__restrict__ inv_eps, const dz *__restrict__ x,
                                               dz *__restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int32_t t = tet[i];
  dz D[3] = {mk(0, 0), mk(0, 0), mk(0, 0)};
  if (t >= 0) {
    const TetGeom &g = tg[t];
    for (int k = 0; k < 4; ++k) {
      const dz c = (1.0 / 3.0) * (x[t2f[4 * t + k].unknown] * gsrc[4 * t + k]);
      for (int d = 0; d < 3; ++d) axpy(D[d], pts[3 * i + d] - g.v[k][d], c);
    }
    const dz ie = inv_eps[t];
    for (int d = 0; d < 3; ++d) D[d] = D[d] * ie;
  }
  for (int d = 0; d < 3; ++d) e[3 * i + d] = D[d];
}

}  // namespace vie
