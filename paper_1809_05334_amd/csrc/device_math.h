// Device helpers of libvie: complex arithmetic, Chebyshev evaluation, the
// Ewald periodic Green's function (Sec. 2.2, Eqs. 3-4) from the per-fill
// tables, and the closed-form 1/R and R potentials of a triangle and a
// tetrahedron (extracted singular part of the kernel).
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace vie {

struct dz {
  double re, im;
};
__device__ __forceinline__ dz mk(double r, double i) { return dz{r, i}; }
__device__ __forceinline__ dz operator+(dz a, dz b) { return dz{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ dz operator-(dz a, dz b) { return dz{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ dz operator*(dz a, dz b) {
  return dz{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ dz operator*(double s, dz a) { return dz{s * a.re, s * a.im}; }
__device__ __forceinline__ dz operator*(dz a, double s) { return dz{s * a.re, s * a.im}; }
__device__ __forceinline__ dz conjz(dz a) { return dz{a.re, -a.im}; }
// acc += a * s (s real)
__device__ __forceinline__ void axpy(dz &acc, double s, dz a) {
  acc.re = fma(s, a.re, acc.re);
  acc.im = fma(s, a.im, acc.im);
}

// f(t) = sum_{k=0}^{deg} c_k T_k(t), c_0 already halved (Clenshaw recurrence).
__device__ __forceinline__ double clenshaw(const double *__restrict__ c, int deg, double t) {
  double b1 = 0.0, b2 = 0.0;
  const double t2 = t + t;
  for (int k = deg; k >= 1; --k) {
    double b0 = fma(t2, b1, c[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(t, b1, c[0] - b2);
}

// g_p at separation (dx, dy, dz) = r - r'.  When TOUCH is true, `mask` lists the
// lattice images (bit (m+1)*3 + (n+1)) whose 1/(4 pi R) part is integrated in
// closed form elsewhere; for those images the remainder H(x) E/(4 pi) is used,
// so the value returned is g_p - sum_touching e^{j kt.rho}/(4 pi R).
template <bool TOUCH>
__device__ __forceinline__ dz pgf_eval(const PgfTable *__restrict__ T, double dx, double dy, double dzv, int mask) {
  const double a = T->a, b = T->b, E = T->E;
  const double m0 = rint(dx * T->inv_a), n0 = rint(dy * T->inv_b);
  dx = fma(-m0, a, dx);
  dy = fma(-n0, b, dy);
  const int im0 = (int)m0, in0 = (int)n0;
  const double dz2 = dzv * dzv;

  // spatial series
  double sre = 0.0, sim = 0.0;
  const int nimg = T->nimg;
  for (int i = 0; i < nimg; ++i) {
    const PgfImage &I = T->img[i];
    const double X = fma((double)I.m, a, dx), Y = fma((double)I.n, b, dy);
    const double R2 = fma(X, X, fma(Y, Y, dz2));
    bool touch = false;
    if (TOUCH) {
      const int um = I.m - im0, un = I.n - in0;
      touch = um >= -1 && um <= 1 && un >= -1 && un <= 1 && ((mask >> ((um + 1) * 3 + (un + 1))) & 1);
    }
    double f;
    if (!touch) {
      const double rinv = rsqrt(R2);
      const double x = R2 * rinv * E;
      f = clenshaw(I.f, I.deg, fma(x - I.xa, I.xs, -1.0)) * rinv;
    } else {
      const double x = sqrt(R2) * E;
      f = clenshaw(I.h, I.hdeg, fma(x - I.xa, I.xs, -1.0)) * E;
    }
    sre = fma(I.cre, f, sre);
    sim = fma(I.cim, f, sim);
  }

  // spectral series, Floquet phases by recurrence in p and q
  const double tw = fma(dz2 * E * E, T->ws, -1.0);
  double s0, c0, s1, c1;
  sincos(-T->kx * dx, &s0, &c0);
  sincos(-T->two_pi_a * dx, &s1, &c1);
  const dz bx = mk(c1, s1);
  dz ex = mk(c0, s0) * conjz(bx * bx * bx * bx);  // p = -4
  sincos(-T->ky * dy, &s0, &c0);
  sincos(-T->two_pi_b * dy, &s1, &c1);
  const dz by = mk(c1, s1);
  const dz ey0 = mk(c0, s0) * conjz(by * by * by * by);  // q = -4
  double kre = 0.0, kim = 0.0;
  for (int p = 0; p < kPgfSide; ++p) {
    dz e = ex * ey0;
    for (int q = 0; q < kPgfSide; ++q) {
      const PgfMode &M = T->mode[p * kPgfSide + q];
      if (M.deg >= 0) {
        const double kr = clenshaw(M.kre, M.deg, tw);
        if (M.cplx) {
          const double ki = clenshaw(M.kim, M.deg, tw);
          kre += e.re * kr - e.im * ki;
          kim += e.re * ki + e.im * kr;
        } else {
          kre = fma(e.re, kr, kre);
          kim = fma(e.im, kr, kim);
        }
      }
      e = e * by;
    }
    ex = ex * bx;
  }
  const int pi = (im0 + 1) * 3 + (in0 + 1);
  const dz ph = mk(T->ph0re[pi], T->ph0im[pi]);
  return ph * mk(sre + kre, sim + kim);
}

// ---------------------------------------------------------------- potentials
__device__ __forceinline__ void sub3(const double *a, const double *b, double *o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
__device__ __forceinline__ double dot3(const double *a, const double *b) {
  return fma(a[0], b[0], fma(a[1], b[1], a[2] * b[2]));
}
__device__ __forceinline__ void cross3(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ void unit3(double *v) {
  const double s = rsqrt(dot3(v, v));
  v[0] *= s;
  v[1] *= s;
  v[2] *= s;
}

// Integrals of 1/|r - r'| and |r - r'| over the flat triangle (A, B, C) for the
// observation point r (polygon formulas: edge logarithms and angle terms).
__device__ inline void tri_potentials(const double *A, const double *B, const double *C, const double *r,
                                      double &iinv, double &ione) {
  const double *V[3] = {A, B, C};
  double e1[3], e2[3], nrm[3];
  sub3(B, A, e1);
  sub3(C, A, e2);
  cross3(e1, e2, nrm);
  unit3(nrm);
  double ra[3];
  sub3(r, A, ra);
  const double d = dot3(ra, nrm), ad = fabs(d);
  const double rho0[3] = {r[0] - d * nrm[0], r[1] - d * nrm[1], r[2] - d * nrm[2]};
  double sinv = 0.0, sedge = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double *Pm = V[i], *Pp = V[(i + 1) % 3], *Po = V[(i + 2) % 3];
    double l[3], w[3], u[3], tmp[3];
    sub3(Pp, Pm, l);
    unit3(l);
    sub3(Pm, Po, w);
    const double wl = dot3(w, l);
    u[0] = w[0] - wl * l[0];
    u[1] = w[1] - wl * l[1];
    u[2] = w[2] - wl * l[2];
    unit3(u);
    sub3(Pm, rho0, tmp);
    const double t = dot3(tmp, u);
    double pp[3], pm[3];
    sub3(Pp, r, pp);
    sub3(Pm, r, pm);
    const double lp = dot3(pp, l), lm = dot3(pm, l);
    const double Rp = sqrt(dot3(pp, pp)), Rm = sqrt(dot3(pm, pm));
    const double R02 = fma(t, t, d * d);
    double f = 0.0;
    if (t != 0.0) {
      const bool neg = lp < 0.0 && lm < 0.0;
      const double num = neg ? Rm - lm : Rp + lp;
      const double den = neg ? Rp - lp : Rm + lm;
      if (num > 0.0 && den > 0.0) f = log(num / den);
    }
    const double beta = atan2(t * lp, fma(ad, Rp, R02)) - atan2(t * lm, fma(ad, Rm, R02));
    sinv += t * f - ad * beta;
    sedge += t * (fma(R02, f, lp * Rp) - lm * Rm);
  }
  iinv = sinv;
  ione = (d * d * sinv + 0.5 * sedge) / 3.0;
}

// Integrals of 1/|r - r'| (P) and (r' - r)/|r - r'| (V1) over the tetrahedron
// with vertices v[4][3], via the divergence theorem over its faces.
__device__ inline void tet_potentials(const double (*v)[3], const double *r, double &P, double *V1) {
  const int F[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
  double c[3];
  for (int d = 0; d < 3; ++d) c[d] = 0.25 * (v[0][d] + v[1][d] + v[2][d] + v[3][d]);
  P = 0.0;
  V1[0] = V1[1] = V1[2] = 0.0;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double *A = v[F[f][0]], *B = v[F[f][1]], *C = v[F[f][2]];
    double e1[3], e2[3], n[3], ac[3];
    sub3(B, A, e1);
    sub3(C, A, e2);
    cross3(e1, e2, n);
    unit3(n);
    sub3(A, c, ac);
    if (dot3(ac, n) < 0.0) {
      n[0] = -n[0];
      n[1] = -n[1];
      n[2] = -n[2];
    }
    double iinv, ione;
    tri_potentials(A, B, C, r, iinv, ione);
    double ar[3];
    sub3(A, r, ar);
    P = fma(0.5 * dot3(ar, n), iinv, P);
    V1[0] = fma(ione, n[0], V1[0]);
    V1[1] = fma(ione, n[1], V1[1]);
    V1[2] = fma(ione, n[2], V1[2]);
  }
}

// touching-image mask of two vertex sets (canonical ids + packed offsets)
__device__ __forceinline__ int touch_mask(const int32_t *ct, const int32_t *ot, int nt_, const int32_t *cs,
                                          const int32_t *os, int ns) {
  int mask = 0;
  for (int i = 0; i < nt_; ++i)
    for (int j = 0; j < ns; ++j)
      if (ct[i] == cs[j]) {
        const int dm = (os[j] & 15) - (ot[i] & 15), dn = (os[j] >> 4) - (ot[i] >> 4);
        mask |= 1 << ((dm + 1) * 3 + (dn + 1));
      }
  return mask;
}

}  // namespace vie
