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
// complex FP32: storage of the mixed-precision Z and of FP32 block factors
struct fz {
  float re, im;
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
// 64-bit DPP lane move (CTRL: a row-local permutation) and lane read, as two
// 32-bit halves
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)v, (int)(unsigned)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(v >> 32), (int)(unsigned)(v >> 32), CTRL, 0xf, 0xf, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int lane) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}
// acc += a * b with each real product fused into the accumulator (four FMAs,
// no separate product to keep live)
__device__ __forceinline__ void cmac(dz &acc, dz a, dz b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}

__device__ __forceinline__ fz operator+(fz a, fz b) { return fz{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ fz operator-(fz a, fz b) { return fz{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ fz operator*(fz a, fz b) {
  return fz{fmaf(a.re, b.re, -a.im * b.im), fmaf(a.re, b.im, a.im * b.re)};
}

// complex element traits: real type, construction, conversions to and from FP64
template <typename C> struct cx;
template <> struct cx<dz> {
  typedef double R;
  static __device__ __forceinline__ dz make(double a, double b) { return dz{a, b}; }
  static __device__ __forceinline__ dz of(dz v) { return v; }
  static __device__ __forceinline__ dz of(fz v) { return dz{v.re, v.im}; }
};
template <> struct cx<fz> {
  typedef float R;
  static __device__ __forceinline__ fz make(float a, float b) { return fz{a, b}; }
  static __device__ __forceinline__ fz of(dz v) { return fz{(float)v.re, (float)v.im}; }
  static __device__ __forceinline__ fz of(fz v) { return v; }
};
__device__ __forceinline__ dz to_dz(dz v) { return v; }
__device__ __forceinline__ dz to_dz(fz v) { return dz{v.re, v.im}; }

// f(t) = sum_{k=0}^{deg} c_k T_k(t), c_0 already halved (Clenshaw recurrence).
// f(t) = sum_{k=0}^{K} c_k T_k(t) by the Clenshaw recurrence for a
// zero-padded coefficient run, K a multiple of 4: four steps per iteration
// with the next four coefficients fetched before the current ones are used.
__device__ __forceinline__ double clenshaw4(const double *__restrict__ c, int K, double t) {
  double b1 = 0.0, b2 = 0.0;
  const double t2 = t + t;
  if (K >= 4) {
    double c3 = c[K], c2 = c[K - 1], c1 = c[K - 2], c0 = c[K - 3];
#pragma unroll 1
    for (int k = K;; k -= 4) {
      const bool more = k >= 8;
      double d3 = 0.0, d2 = 0.0, d1 = 0.0, d0 = 0.0;
      if (more) {
        d3 = c[k - 4];
        d2 = c[k - 5];
        d1 = c[k - 6];
        d0 = c[k - 7];
      }
      double b0 = fma(t2, b1, c3 - b2);
      b2 = b1;
      b1 = b0;
      b0 = fma(t2, b1, c2 - b2);
      b2 = b1;
      b1 = b0;
      b0 = fma(t2, b1, c1 - b2);
      b2 = b1;
      b1 = b0;
      b0 = fma(t2, b1, c0 - b2);
      b2 = b1;
      b1 = b0;
      if (!more) break;
      c3 = d3;
      c2 = d2;
      c1 = d1;
      c0 = d0;
    }
  }
  return fma(t, b1, c[0] - b2);
}

// Packed lattice-sum table (layout written by the host: header, per-mode
// offsets, image records, mode records; see host.h).
namespace pk {
constexpr int E = 0, A = 1, B = 2, IA = 3, IB = 4, KX = 5, KY = 6, TPA = 7, TPB = 8, WS = 9, PHRE = 10, PHIM = 19,
              NIMG = 28, MODES = 32, ROWS = 116, IMAGES = 128;
}

// Stage the packed table into LDS (all threads of the block participate).
__device__ __forceinline__ void stage_table(const double *__restrict__ pack, int len, double *lds) {
  for (int i = threadIdx.x; i < len; i += blockDim.x) lds[i] = pack[i];
  __syncthreads();
}

__device__ __forceinline__ int ufirst(int v) { return __builtin_amdgcn_readfirstlane(v); }

// integer field of the packed table (value in the low 32 bits of the slot)
__device__ __forceinline__ int pint(double slot) { return ufirst(__double2loint(slot)); }

// 1/sqrt(x) for x > 0 (finite): hardware estimate refined by one third-order
// Householder step, r <- r (1 + e/2 + 3 e^2/8) with e = 1 - x r^2.
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * r, r, 1.0);
  return fma(r * e, fma(e, 0.375, 0.5), r);
}

// W Chebyshev series with the same coefficients c[0..K] (K even, zero-padded)
// at W arguments t[w]: interleaved Clenshaw recurrences, two coefficients per
// step, each coefficient read once for all W.
template <int W>
__device__ __forceinline__ void clenshaw_w(const double *__restrict__ c, int K, const double (&t)[W], double (&f)[W]) {
  double b1[W], b2[W], t2[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    b1[w] = b2[w] = 0.0;
    t2[w] = t[w] + t[w];
  }
  // four coefficients per pass, all read before the first is used, so one
  // read's latency is exposed per four coefficients rather than per two
  const auto pair = [&](double ck, double ck1) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const double bk = fma(t2[w], b1[w], ck - b2[w]);
      const double bk1 = fma(t2[w], bk, ck1 - b1[w]);
      b2[w] = bk;
      b1[w] = bk1;
    }
  };
  int k = K;
#pragma unroll 1
  for (; k >= 8; k -= 8) {
    const double c0 = c[k], c1 = c[k - 1], c2 = c[k - 2], c3 = c[k - 3];
    const double c4 = c[k - 4], c5 = c[k - 5], c6 = c[k - 6], c7 = c[k - 7];
    pair(c0, c1);
    pair(c2, c3);
    pair(c4, c5);
    pair(c6, c7);
  }
  if (k >= 4) {   // (K is a multiple of 4: what remains is 4 or 0)
    const double c0 = c[k], c1 = c[k - 1], c2 = c[k - 2], c3 = c[k - 3];
    pair(c0, c1);
    pair(c2, c3);
    k -= 4;
  }
#pragma unroll 1
  for (; k >= 2; k -= 2) pair(c[k], c[k - 1]);
#pragma unroll
  for (int w = 0; w < W; ++w) f[w] = fma(t[w], b1[w], c[0] - b2[w]);
}

// g_p at W separations d[w] = r - r'_w at once (one test point, W source
// points), from the packed table P.  The table entries are read once for
// all W separations and the W Clenshaw recurrences run interleaved.  When
// TOUCH is true, `mask` lists the lattice images (bit (m+1)*3 + (n+1)) whose
// 1/(4 pi R) part is integrated in closed form elsewhere; for those images
// the remainder H(x) E/(4 pi) is used, so the value returned is
// g_p - sum_touching e^{j kt.rho}/(4 pi R).
//
// REV (non-touching separations only): also g_p at -d[w] into rev[w].  For a
// real wavenumber every spatial image term is a real function of R times the
// image phase e^{j kt.rho_mn}, and the images (m, n), (-m, -n) share that
// function, so the spatial sum at -d is the conjugate of the one at d.  A
// spectral term e^{-j k_tpq.Delta} K_pq(z) has K_pq even in z and real for an
// evanescent order, so it too conjugates, except for the propagating orders,
// whose K_pq is complex.  Hence
//   g_p(-d) = conj(g_p(d)) + conj(ph0) 2j sum_{propagating} conj(e^{-j k_tpq.Delta}) Im K_pq(z),
// with ph0 the phase of the nearest-image shift (which flips with d).  The
// reverse value costs two FMAs per propagating order on top of g_p(d).
template <bool TOUCH, int W, bool REV = false>
__device__ __forceinline__ void pgf_eval_w(const double *__restrict__ P, const double (&d)[W][3], int mask,
                                           dz (&out)[W], dz *rev = nullptr) {
  const double a = P[pk::A], b = P[pk::B], E = P[pk::E];
  double dx[W], dy[W], dz2[W], sre[W], sim[W];
  int im0[W], in0[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const double m0 = rint(d[w][0] * P[pk::IA]), n0 = rint(d[w][1] * P[pk::IB]);
    dx[w] = fma(-m0, a, d[w][0]);
    dy[w] = fma(-n0, b, d[w][1]);
    dz2[w] = d[w][2] * d[w][2];
    im0[w] = (int)m0;
    in0[w] = (int)n0;
    sre[w] = 0.0;
    sim[w] = 0.0;
  }
  // spatial series
  const int nimg = pint(P[pk::NIMG]);
  int off = pk::IMAGES;
#pragma unroll 1
  for (int i = 0; i < nimg; ++i) {
    const double *R = P + off;
    const double ts = R[0], t0 = R[1], cre = R[2], cim = R[3];   // t = ts R + t0
    const int im = pint(R[4]), in = pint(R[5]), K = pint(R[6]);
    off += pint(R[7]);
    double t[W], sc[W];
    bool touch[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const double X = fma((double)im, a, dx[w]), Y = fma((double)in, b, dy[w]);
      const double R2 = fma(X, X, fma(Y, Y, dz2[w]));
      touch[w] = false;
      if (TOUCH) {
        const int um = im - im0[w], un = in - in0[w];
        touch[w] = um >= -1 && um <= 1 && un >= -1 && un <= 1 && ((mask >> ((um + 1) * 3 + (un + 1))) & 1);
      }
      double rinv, Rw;
      if (TOUCH) {   // a touching image can sit at R = 0 (its H fit is evaluated at x = 0)
        rinv = rsqrt(R2);
        Rw = R2 > 0.0 ? R2 * rinv : 0.0;
      } else {       // separations of non-touching elements never vanish
        rinv = rsqrt_pos(R2);
        Rw = R2 * rinv;
      }
      t[w] = fma(Rw, ts, t0);
      sc[w] = touch[w] ? E : rinv;
    }
    // W interleaved Clenshaw recurrences on the F coefficients
    double b1[W], b2[W];
#pragma unroll
    for (int w = 0; w < W; ++w) b1[w] = b2[w] = 0.0;
    const double *c = R + 8;
    // four coefficients per pass, read before the first is used (as in clenshaw_w)
    double t2[W];
#pragma unroll
    for (int w = 0; w < W; ++w) t2[w] = t[w] + t[w];
    const auto pair = [&](double ck, double ck1) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const double bk = fma(t2[w], b1[w], ck - b2[w]);
        const double bk1 = fma(t2[w], bk, ck1 - b1[w]);
        b2[w] = bk;
        b1[w] = bk1;
      }
    };
    int k = K;
#pragma unroll 1
    for (; k >= 8; k -= 8) {
      const double c0 = c[k], c1 = c[k - 1], c2 = c[k - 2], c3 = c[k - 3];
      const double c4 = c[k - 4], c5 = c[k - 5], c6 = c[k - 6], c7 = c[k - 7];
      pair(c0, c1);
      pair(c2, c3);
      pair(c4, c5);
      pair(c6, c7);
    }
    if (k >= 4) {   // (K is a multiple of 4: what remains is 4 or 0)
      const double c0 = c[k], c1 = c[k - 1], c2 = c[k - 2], c3 = c[k - 3];
      pair(c0, c1);
      pair(c2, c3);
      k -= 4;
    }
#pragma unroll 1
    for (; k >= 2; k -= 2) pair(c[k], c[k - 1]);
    double f[W];
#pragma unroll
    for (int w = 0; w < W; ++w) f[w] = fma(t[w], b1[w], c[0] - b2[w]);
    if (TOUCH) {
      bool any = false;
#pragma unroll
      for (int w = 0; w < W; ++w) any = any || touch[w];
      if (any) {
        // touching images use the H fit (extracted 1/(4 pi R))
        const double *Hb = R + 8 + K + 4;
        const int HK = pint(Hb[0]);
#pragma unroll
        for (int w = 0; w < W; ++w)
          if (touch[w]) f[w] = clenshaw4(Hb + 4, HK, t[w]);
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const double g = f[w] * sc[w];
      sre[w] = fma(cre, g, sre[w]);
      sim[w] = fma(cim, g, sim[w]);
    }
  }

  // spectral series: the W separations share every mode's coefficient reads
  // and run W interleaved Clenshaw recurrences in w = (z E)^2; the Floquet
  // phases e^{-j k_tpq . Delta_t} of each separation by recurrence in p and q
  double tw[W], kre[W], kim[W], cre_[W], cim_[W];
  dz erow[W], bx[W], by[W];   // erow: phase of (p, q = -4); steps in p and in q
  const bool kt0 = P[pk::KX] == 0.0 && P[pk::KY] == 0.0;   // normal incidence: e^{-j kt.Delta} = 1
#pragma unroll
  for (int w = 0; w < W; ++w) {
    tw[w] = fma(dz2[w] * E * E, P[pk::WS], -1.0);
    double s0, c0, s1, c1;
    sincos(-P[pk::TPA] * dx[w], &s1, &c1);
    bx[w] = mk(c1, s1);
    sincos(-P[pk::TPB] * dy[w], &s1, &c1);
    by[w] = mk(c1, s1);
    const dz bx4 = conjz(bx[w] * bx[w] * bx[w] * bx[w]), by4 = conjz(by[w] * by[w] * by[w] * by[w]);
    if (kt0) {
      erow[w] = bx4 * by4;   // (p, q) = (-4, -4)
    } else {
      sincos(-P[pk::KX] * dx[w], &s0, &c0);
      const dz ex = mk(c0, s0) * bx4;   // p = -4
      sincos(-P[pk::KY] * dy[w], &s0, &c0);
      erow[w] = ex * (mk(c0, s0) * by4);
    }
    kre[w] = 0.0;
    kim[w] = 0.0;
    cre_[w] = 0.0;
    cim_[w] = 0.0;
  }
  // rows of the grid: only the slots from the row's first to its last mode
  // (the phases of the slots below reached by the same products as before)
#pragma unroll 1
  for (int p = 0; p < kPgfSide; ++p) {
    const int rr = pint(P[pk::ROWS + p]);
    const int qlo = rr & 0xff, qend = rr >> 8;
    dz e[W];
#pragma unroll
    for (int w = 0; w < W; ++w) e[w] = erow[w];
#pragma unroll 1
    for (int q = 0; q < qlo; ++q) {
#pragma unroll
      for (int w = 0; w < W; ++w) e[w] = e[w] * by[w];
    }
#pragma unroll 1
    for (int q = qlo; q < qend; ++q) {
      const double slot = P[pk::MODES + p * kPgfSide + q];
      const int moff = pint(slot);
      if (moff > 0) {
        const double *M = P + moff;
        const int kc = ufirst(__double2hiint(slot));   // K | cplx << 16
        const int K = kc & 0xffff;
        double kr[W];
        clenshaw_w<W>(M + 4, K, tw, kr);
        if ((kc >> 16) != 0) {
          double ki[W];
          clenshaw_w<W>(M + 4 + K + 4, K, tw, ki);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            kre[w] += e[w].re * kr[w] - e[w].im * ki[w];
            kim[w] += e[w].re * ki[w] + e[w].im * kr[w];
            if (REV) {   // conj(e) Im K_pq of a propagating order
              cre_[w] = fma(e[w].re, ki[w], cre_[w]);
              cim_[w] = fma(-e[w].im, ki[w], cim_[w]);
            }
          }
        } else {
#pragma unroll
          for (int w = 0; w < W; ++w) {
            kre[w] = fma(e[w].re, kr[w], kre[w]);
            kim[w] = fma(e[w].im, kr[w], kim[w]);
          }
        }
      }
#pragma unroll
      for (int w = 0; w < W; ++w) e[w] = e[w] * by[w];
    }
#pragma unroll
    for (int w = 0; w < W; ++w) erow[w] = erow[w] * bx[w];
  }
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int pi = (im0[w] + 1) * 3 + (in0[w] + 1);
    const dz ph = mk(P[pk::PHRE + pi], P[pk::PHIM + pi]);
    out[w] = ph * mk(sre[w] + kre[w], sim[w] + kim[w]);
    if (REV) rev[w] = conjz(out[w]) + conjz(ph) * mk(-2.0 * cim_[w], 2.0 * cre_[w]);
  }
}

// single separation
template <bool TOUCH>
__device__ __forceinline__ dz pgf_eval(const double *__restrict__ P, double dx, double dy, double dzv, int mask) {
  const double d[1][3] = {{dx, dy, dzv}};
  dz o[1];
  pgf_eval_w<TOUCH, 1>(P, d, mask, o);
  return o[0];
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
#pragma unroll 1
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
