// Impedance-matrix fill of the periodic SWG VIE (Sec. 2.1, Eq. 2 with the
// periodic Green's function of Sec. 2.2, Eqs. 3-4), right-hand side, and a
// diagnostic evaluation of g_p.
//
// Galerkin terms for test tet T (local face k -> unknown m) and source tet S
// (local face l -> unknown n), u = r - c_T, u' = r' - c_S, p~ = v_k - c_T,
// q~ = v'_l - c_S:
//   Z_mn += alpha_Tk * beta_Sl * [ II g_p - (k0^2/9) II (u - p~).(u' - q~) g_p ]
//   alpha_Tk = chi s a_m / V_T,   beta_Sl = psi s a_n kappa_S / V_S,
// with the Bloch test/source phases chi = e^{+j kt.rho}, psi = e^{-j kt.rho} of
// a wall-shifted half.  Surface charges (sigma_n on interface/boundary faces)
// and the boundary term of half-SWG test faces add scalar-potential pairs of
// tetrahedra and faces.  The mass term <f_m, f_n/eps> is added with the
// self pair.
//
// Scatter: every launch covers a pair of tetrahedron colour classes (no two
// tetrahedra of a class share a face), so no two lanes of one launch touch
// the same Z entry; the read-modify-write needs no atomics and the result is
// deterministic.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vie {

static constexpr double kInv4Pi = 0.079577471545947667884;

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Z[m][n] += v into the destination of this fill (see ZOut).  In mixed
// precision a far contribution is added to the FP32 entry in FP64 and rounded
// once; a near one goes to its slot of the sorted CSR row.
__device__ __forceinline__ void zput(const ZOut &o, int64_t m, int64_t n, dz v, bool near) {
  if (o.Z) {
    dz *p = o.Z + m * o.ld + n;
    *p = *p + v;
  } else if (near) {
    int64_t lo = o.rowptr[m], hi = o.rowptr[m + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (o.cols[mid] < n) lo = mid + 1;
      else hi = mid;
    }
    if (lo < o.rowptr[m + 1] && o.cols[lo] == n) o.vals[lo] = o.vals[lo] + v;
  } else {
    fz *p = o.Zs + m * o.ld + n;
    const fz z = *p;
    *p = fz{(float)((double)z.re + v.re), (float)((double)z.im + v.im)};
  }
}

// ------------------------------------------------------------ per-fill coefficients
__global__ void k_prep(int64_t nt, const TetFace *__restrict__ t2f, const TetGeom *__restrict__ tg,
                       const double *__restrict__ area, const dz *__restrict__ eps_int, double kx, double ky,
                       double a, double b, dz *__restrict__ alpha, dz *__restrict__ gsrc, dz *__restrict__ kappa,
                       dz *__restrict__ inv_eps) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const dz e = eps_int[t];
  const double den = e.re * e.re + e.im * e.im;
  const dz ie = mk(e.re / den, -e.im / den);
  inv_eps[t] = ie;
  kappa[t] = mk(1.0 - ie.re, -ie.im);
  const double V = tg[t].vol;
  for (int k = 0; k < 4; ++k) {
    const TetFace f = t2f[4 * t + k];
    double s, c;
    sincos(kx * f.sx * a + ky * f.sy * b, &s, &c);
    const double w = f.sign * area[f.unknown] / V;
    alpha[4 * t + k] = mk(w * c, w * s);   // e^{+j kt.rho} s a / V
    gsrc[4 * t + k] = mk(w * c, -w * s);   // e^{-j kt.rho} s a / V
  }
}

// sigma_n = kappa(T+) - kappa(T-) for each surface-charge face slot
__global__ void k_sigma(int nc, const int32_t *__restrict__ ctp, const int32_t *__restrict__ ctm,
                        const dz *__restrict__ kappa, dz *__restrict__ sigma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  dz s = kappa[ctp[i]];
  if (ctm[i] >= 0) s = s - kappa[ctm[i]];
  sigma[i] = s;
}

__global__ void k_zero(dz *__restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = mk(0.0, 0.0);
}

// ------------------------------------------------------------ tet-pair moments
struct Moments {
  dz m0, mu[3], mv[3], muv;
};

__device__ __forceinline__ void moments_zero(Moments &M) {
  M.m0 = mk(0, 0);
  M.muv = mk(0, 0);
  for (int d = 0; d < 3; ++d) M.mu[d] = M.mv[d] = mk(0, 0);
}

// Scatter the 16 face-pair contributions of tet pair (T, S) into Z (TRANS:
// entry (m, n) goes to (n, m) of the output).
template <bool TRANS = false>
__device__ __forceinline__ void scatter_tt(const Moments &M, const TetGeom &gt, const TetGeom &gs,
                                           const TetFace *__restrict__ t2f, int T, int S,
                                           const dz *__restrict__ alpha, const dz *__restrict__ gsrc,
                                           const dz *__restrict__ kappa, double k0sq9, const ZOut &out,
                                           bool near) {
  const dz ks = kappa[S];
  double qv[4][3];
  dz bl[4];
  int64_t col[4];
  for (int l = 0; l < 4; ++l) {
    for (int d = 0; d < 3; ++d) qv[l][d] = gs.v[l][d] - gs.c[d];
    bl[l] = gsrc[4 * S + l] * ks;
    col[l] = t2f[4 * S + l].unknown;
  }
  for (int k = 0; k < 4; ++k) {
    double pk[3];
    for (int d = 0; d < 3; ++d) pk[d] = gt.v[k][d] - gt.c[d];
    // muv - p~.mv
    dz base = M.muv;
    for (int d = 0; d < 3; ++d) base = base - pk[d] * M.mv[d];
    const dz ak = alpha[4 * T + k];
    const int64_t row = t2f[4 * T + k].unknown;
    for (int l = 0; l < 4; ++l) {
      dz I = base;
      for (int d = 0; d < 3; ++d) I = I - qv[l][d] * M.mu[d];
      I = I + dot3(pk, qv[l]) * M.m0;
      const dz v = M.m0 - k0sq9 * I;
      if (TRANS) zput(out, col[l], row, (ak * bl[l]) * v, near);
      else zput(out, row, col[l], (ak * bl[l]) * v, near);
    }
  }
}

// Far tet pairs: 4 x 4 product rule.  One wave = one test tet x 64 source tets.
// sym > 0 writes the swapped pair's block (S, T) too (see the declaration).
// At normal incidence the lattice sum is even in the separation (the phases
// e^{-j kt.rho} are all 1), so the pair's moments also give those of the
// swapped pair.  At oblique incidence (rev) g_p at the reversed separations
// follows from g_p at the separations plus the propagating orders' term (see
// pgf_eval_w), and the swapped pair's moments are accumulated from it.
// REV: the swapped pair's moments are summed per lane in LDS (16 doubles
// after the table, one column per thread), not in registers, so that the
// kernel keeps two waves per SIMD without spilling.
template <bool REV>
__device__ __forceinline__ void tt_far_body(const double *__restrict__ pack, int packlen,
                                            const QuadRules *__restrict__ qr, const TetGeom *__restrict__ tg,
                                            const TetFace *__restrict__ t2f, const int32_t *__restrict__ test_list,
                                            int ntest, const int32_t *__restrict__ src_list, int nsrc,
                                            const dz *__restrict__ alpha, const dz *__restrict__ gsrc,
                                            const dz *__restrict__ kappa, double k0sq9, const ZOut &out,
                                            const ZOut &outT, int sym, int bx_, int by_) {
  extern __shared__ double s_tab[];
  // one list against itself: a block whose source positions all lie at or
  // below its test positions has nothing to do (the whole block returns)
  if (sym == 2 && bx_ * 64 + 63 <= by_ * 4) return;
  stage_table(pack, packlen, s_tab);
  const double *__restrict__ P = s_tab;
  double *__restrict__ mr = s_tab + ((packlen + 1) & ~1) + threadIdx.x;   // REV: entry e at mr[256 e]

  const int ti = uniform(by_ * 4 + (threadIdx.x >> 6));
  const int si = bx_ * 64 + (threadIdx.x & 63);
  if (ti >= ntest || si >= nsrc) return;
  if (sym == 2 && si <= ti) return;
  const int T = uniform(test_list[ti]);
  const int S = src_list[si];
  const TetGeom &gt = tg[T];
  double wq;
  double up[4][3], dc[3];
  {
    const TetGeom gs = tg[S];
    if (touch_mask(gt.canon, gt.off, 4, gs.canon, gs.off, 4)) return;  // touching pairs: k_tt_near
    wq = 0.25 * gs.vol;
    for (int d = 0; d < 3; ++d) dc[d] = gt.c[d] - gs.c[d];
    // source points relative to the source centroid
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double s = 0;
        for (int k = 0; k < 4; ++k) s = fma(qr->tet4[j][k], gs.v[k][d], s);
        up[j][d] = s - gs.c[d];
      }
  }
  const double wt = 0.25 * gt.vol;
  Moments M;
  moments_zero(M);
  if (REV)
    for (int e = 0; e < 16; ++e) mr[256 * e] = 0.0;
  // one test point against the four source points per lattice-sum call
#pragma unroll 1
  for (int i = 0; i < 4; ++i) {
    double u[3];
    for (int d = 0; d < 3; ++d) {
      double s = 0;
      for (int k = 0; k < 4; ++k) s = fma(qr->tet4[i][k], gt.v[k][d], s);
      u[d] = s - gt.c[d];
    }
    double sep[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int d = 0; d < 3; ++d) sep[j][d] = dc[d] + u[d] - up[j][d];
    dz g[4], gr[REV ? 4 : 1];
    pgf_eval_w<false, 4, REV>(P, sep, 0, g, gr);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const dz gw = (wt * wq) * g[j];
      M.m0 = M.m0 + gw;
      for (int d = 0; d < 3; ++d) {
        axpy(M.mu[d], u[d], gw);
        axpy(M.mv[d], up[j][d], gw);
      }
      axpy(M.muv, dot3(u, up[j]), gw);
    }
    if (REV) {
      // swapped pair (S, T): its test offsets are up_j, its source offsets u
      Moments R;
      moments_zero(R);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const dz grw = (wt * wq) * gr[j];
        R.m0 = R.m0 + grw;
        for (int d = 0; d < 3; ++d) {
          axpy(R.mu[d], up[j][d], grw);
          axpy(R.mv[d], u[d], grw);
        }
        axpy(R.muv, dot3(u, up[j]), grw);
      }
      mr[0] += R.m0.re;
      mr[256] += R.m0.im;
      for (int d = 0; d < 3; ++d) {
        mr[256 * (2 + 2 * d)] += R.mu[d].re;
        mr[256 * (3 + 2 * d)] += R.mu[d].im;
        mr[256 * (8 + 2 * d)] += R.mv[d].re;
        mr[256 * (9 + 2 * d)] += R.mv[d].im;
      }
      mr[256 * 14] += R.muv.re;
      mr[256 * 15] += R.muv.im;
    }
  }
  // the source geometry is read again here rather than held in registers
  // through the lattice sums (the empty asm hides the earlier load)
  const TetGeom *tgs = tg + S;
  asm volatile("" : "+v"(tgs));
  const TetGeom gs = *tgs;
  scatter_tt(M, gt, gs, t2f, T, S, alpha, gsrc, kappa, k0sq9, out, false);
  if (REV && sym) {
    Moments R;
    R.m0 = mk(mr[0], mr[256]);
    for (int d = 0; d < 3; ++d) {
      R.mu[d] = mk(mr[256 * (2 + 2 * d)], mr[256 * (3 + 2 * d)]);
      R.mv[d] = mk(mr[256 * (8 + 2 * d)], mr[256 * (9 + 2 * d)]);
    }
    R.muv = mk(mr[256 * 14], mr[256 * 15]);
    scatter_tt<true>(R, gs, gt, t2f, S, T, alpha, gsrc, kappa, k0sq9, outT, false);
  } else if (sym) {
    // (S, T) at kt = 0: test offsets and source offsets trade places
    Moments Ms;
    Ms.m0 = M.m0;
    Ms.muv = M.muv;
    for (int d = 0; d < 3; ++d) {
      Ms.mu[d] = M.mv[d];
      Ms.mv[d] = M.mu[d];
    }
    scatter_tt<true>(Ms, gs, gt, t2f, S, T, alpha, gsrc, kappa, k0sq9, outT, false);
  }
}

__global__ __launch_bounds__(256, 2) void k_tt_far(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                const TetGeom *__restrict__ tg, const TetFace *__restrict__ t2f,
                                                const int32_t *__restrict__ test_list, int ntest,
                                                const int32_t *__restrict__ src_list, int nsrc,
                                                const dz *__restrict__ alpha, const dz *__restrict__ gsrc,
                                                const dz *__restrict__ kappa, double k0sq9, ZOut out, ZOut outT,
                                                int sym) {
  tt_far_body<false>(pack, packlen, qr, tg, t2f, test_list, ntest, src_list, nsrc, alpha, gsrc, kappa, k0sq9, out,
                     outT, sym, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256, 2) void k_tt_far_rev(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                    const TetGeom *__restrict__ tg, const TetFace *__restrict__ t2f,
                                                    const int32_t *__restrict__ test_list, int ntest,
                                                    const int32_t *__restrict__ src_list, int nsrc,
                                                    const dz *__restrict__ alpha, const dz *__restrict__ gsrc,
                                                    const dz *__restrict__ kappa, double k0sq9, ZOut out, ZOut outT,
                                                    int sym) {
  tt_far_body<true>(pack, packlen, qr, tg, t2f, test_list, ntest, src_list, nsrc, alpha, gsrc, kappa, k0sq9, out,
                    outT, sym, blockIdx.x, blockIdx.y);
}

// Z[i][j] += Zt[j][i]: 32 x 32 tiles through shared memory, both sides read
// and written along rows.  In FP32 the sum is formed in FP64 and rounded once.
template <typename C>
__device__ __forceinline__ void transpose_add_body(C *__restrict__ Z, const C *__restrict__ Zt, int64_t N, int64_t ld) {
  __shared__ C tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
  const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
  // tile of Zt rows j0.., columns i0..
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + r, i = i0 + tx;
    if (j < N && i < N) tile[r][tx] = Zt[j * ld + i];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, j = j0 + tx;
    if (i < N && j < N) {
      const C a = Z[i * ld + j], b = tile[tx][r];
      Z[i * ld + j] = cx<C>::make((double)a.re + (double)b.re, (double)a.im + (double)b.im);
    }
  }
}
__global__ __launch_bounds__(256) void k_transpose_add_z(dz *Z, const dz *Zt, int64_t N, int64_t ld) {
  transpose_add_body(Z, Zt, N, ld);
}
__global__ __launch_bounds__(256) void k_transpose_add_c(fz *Z, const fz *Zt, int64_t N, int64_t ld) {
  transpose_add_body(Z, Zt, N, ld);
}

// Touching tet pairs: 14-point outer rule on T; per touching image the closed
// form int_S 1/R and int_S (r'-r)/R; 4-point inner rule for the remainder.
// The self pair also adds the mass term <f_m, f_n / eps_r>.  Sixteen lanes
// share a pair: lane q < 14 takes outer point q, the moments are summed
// across the 16 lanes by shuffles, and the pair's first lane scatters.
__device__ __forceinline__ dz shfl_xor_dz(dz v, int o) { return mk(__shfl_xor(v.re, o), __shfl_xor(v.im, o)); }

__device__ __forceinline__ void k_tt_near_body(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                 const TetGeom *__restrict__ tg, const TetFace *__restrict__ t2f,
                                                 const int32_t *__restrict__ lt, const int32_t *__restrict__ ls,
                                                 const int32_t *__restrict__ lmask, int npairs,
                                                 const dz *__restrict__ alpha, const dz *__restrict__ gsrc,
                                                 const dz *__restrict__ kappa, const dz *__restrict__ inv_eps,
                                                 double k0sq9, ZOut out, int bx_, int by_) {
  extern __shared__ double s_tab[];
  stage_table(pack, packlen, s_tab);
  const double *__restrict__ P = s_tab;

  const int gid = bx_ * blockDim.x + threadIdx.x;
  const int i = gid >> 4, q = gid & 15;
  const bool act = i < npairs;
  // lanes past the last pair stay in the shuffles below with zero moments
  const int ii = act ? i : npairs - 1;
  const int T = lt[ii], S = ls[ii], mask = lmask[ii];
  const TetGeom gt = tg[T];
  const TetGeom gs = tg[S];
  const double wq = 0.25 * gs.vol;
  Moments M;
  moments_zero(M);
  if (act && q < 14) {
    double r[3], u[3];
    for (int d = 0; d < 3; ++d) {
      double s = 0;
      for (int k = 0; k < 4; ++k) s = fma(qr->tet14[q][k], gt.v[k][d], s);
      r[d] = s;
      u[d] = s - gt.c[d];
    }
    const double w = qr->w14[q] * gt.vol;
    dz s0 = mk(0, 0), s1[3] = {mk(0, 0), mk(0, 0), mk(0, 0)};
#pragma unroll 1
    for (int b = 0; b < 9; ++b) {
      if (!((mask >> b) & 1)) continue;
      const int m = b / 3 - 1, n = b % 3 - 1;
      const double o[3] = {r[0] + m * P[pk::A], r[1] + n * P[pk::B], r[2]};
      double pot, V1[3];
      tet_potentials(gs.v, o, pot, V1);
      const dz ph = kInv4Pi * mk(P[pk::PHRE + b], -P[pk::PHIM + b]);  // e^{+j kt.rho}/(4 pi)
      s0 = s0 + pot * ph;
      for (int d = 0; d < 3; ++d) s1[d] = s1[d] + (V1[d] + (o[d] - gs.c[d]) * pot) * ph;
    }
    double sep[4][3], upj[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double t = 0;
        for (int k = 0; k < 4; ++k) t = fma(qr->tet4[j][k], gs.v[k][d], t);
        upj[j][d] = t - gs.c[d];
        sep[j][d] = r[d] - t;
      }
    dz g[4];
    pgf_eval_w<true, 4>(P, sep, mask, g);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      axpy(s0, wq, g[j]);
      for (int d = 0; d < 3; ++d) axpy(s1[d], wq * upj[j][d], g[j]);
    }
    axpy(M.m0, w, s0);
    for (int d = 0; d < 3; ++d) {
      axpy(M.mu[d], w * u[d], s0);
      axpy(M.mv[d], w, s1[d]);
    }
    dz us = mk(0, 0);
    for (int d = 0; d < 3; ++d) axpy(us, u[d], s1[d]);
    axpy(M.muv, w, us);
  }
  // sum the 16 lanes of the pair (fixed order: deterministic)
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
    M.m0 = M.m0 + shfl_xor_dz(M.m0, o);
    M.muv = M.muv + shfl_xor_dz(M.muv, o);
    for (int d = 0; d < 3; ++d) {
      M.mu[d] = M.mu[d] + shfl_xor_dz(M.mu[d], o);
      M.mv[d] = M.mv[d] + shfl_xor_dz(M.mv[d], o);
    }
  }
  if (!act || q != 0) return;
  scatter_tt(M, gt, gs, t2f, T, S, alpha, gsrc, kappa, k0sq9, out, true);
  if (T == S) {
    // mass <f_m, f_n / eps_r>: alpha_k gsrc_l / (9 eps) int_T (r - v_k).(r - v_l), 4-point rule (exact)
    const dz ie = inv_eps[T];
    for (int k = 0; k < 4; ++k) {
      const int64_t row = t2f[4 * T + k].unknown;
      for (int l = 0; l < 4; ++l) {
        double s = 0;
        for (int q = 0; q < 4; ++q) {
          double a2 = 0;
          for (int d = 0; d < 3; ++d) {
            double r = 0;
            for (int kk = 0; kk < 4; ++kk) r = fma(qr->tet4[q][kk], gt.v[kk][d], r);
            a2 = fma(r - gt.v[k][d], r - gt.v[l][d], a2);
          }
          s = fma(0.25 * gt.vol, a2, s);
        }
        zput(out, row, t2f[4 * T + l].unknown, (s / 9.0) * ((alpha[4 * T + k] * gsrc[4 * T + l]) * ie), true);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_tt_near(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                 const TetGeom *__restrict__ tg, const TetFace *__restrict__ t2f,
                                                 const int32_t *__restrict__ lt, const int32_t *__restrict__ ls,
                                                 const int32_t *__restrict__ lmask, int npairs,
                                                 const dz *__restrict__ alpha, const dz *__restrict__ gsrc,
                                                 const dz *__restrict__ kappa, const dz *__restrict__ inv_eps,
                                                 double k0sq9, ZOut out) {
  k_tt_near_body(pack, packlen, qr, tg, t2f, lt, ls, lmask, npairs, alpha, gsrc, kappa, inv_eps, k0sq9, out, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------ pairs with faces
// M0 = II g_p over (test tet T, face F).  Far: 4 x 3 rule.  Touching: outer
// 14-point rule on T, closed-form int_F 1/R per touching image, 3-point
// inner rule for the remainder.
__device__ dz pair_tet_face(const double *__restrict__ P, const QuadRules *__restrict__ qr, const TetGeom &gt,
                            const FaceGeom &f, int &mask) {
  mask = touch_mask(gt.canon, gt.off, 4, f.canon, f.off, 3);
  double fp[3][3];
  for (int j = 0; j < 3; ++j)
    for (int d = 0; d < 3; ++d) fp[j][d] = qr->tri3[j][0] * f.v[0][d] + qr->tri3[j][1] * f.v[1][d] + qr->tri3[j][2] * f.v[2][d];
  const double wf = f.area / 3.0;
  dz acc = mk(0, 0);
  if (!mask) {
    // one face point against the tet's four points per lattice-sum call
    double tp[4][3];
    for (int i = 0; i < 4; ++i)
      for (int d = 0; d < 3; ++d) {
        double s = 0;
        for (int k = 0; k < 4; ++k) s = fma(qr->tet4[i][k], gt.v[k][d], s);
        tp[i][d] = s;
      }
#pragma unroll 1
    for (int j = 0; j < 3; ++j) {
      double sep[4][3];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d) sep[i][d] = tp[i][d] - fp[j][d];
      dz g[4];
      pgf_eval_w<false, 4>(P, sep, 0, g);
      acc = acc + ((g[0] + g[1]) + (g[2] + g[3]));
    }
    return (0.25 * gt.vol * wf) * acc;
  }
#pragma unroll 1
  for (int q = 0; q < 14; ++q) {
    double r[3];
    for (int d = 0; d < 3; ++d) {
      double s = 0;
      for (int k = 0; k < 4; ++k) s = fma(qr->tet14[q][k], gt.v[k][d], s);
      r[d] = s;
    }
    dz s0 = mk(0, 0);
#pragma unroll 1
    for (int b = 0; b < 9; ++b) {
      if (!((mask >> b) & 1)) continue;
      const int m = b / 3 - 1, n = b % 3 - 1;
      const double o[3] = {r[0] + m * P[pk::A], r[1] + n * P[pk::B], r[2]};
      double iinv, ione;
      tri_potentials(f.v[0], f.v[1], f.v[2], o, iinv, ione);
      s0 = s0 + (kInv4Pi * iinv) * mk(P[pk::PHRE + b], -P[pk::PHIM + b]);
    }
    {
      double sep[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) sep[j][d] = r[d] - fp[j][d];
      dz g[3];
      pgf_eval_w<true, 3>(P, sep, mask, g);
      axpy(s0, wf, (g[0] + g[1]) + g[2]);
    }
    axpy(acc, qr->w14[q] * gt.vol, s0);
  }
  return acc;
}

// M0 = II g_p over (test face F, source tet S).  Touching: outer 7-point rule
// on F, closed-form int_S 1/R, 4-point inner rule for the remainder.
__device__ dz pair_face_tet(const double *__restrict__ P, const QuadRules *__restrict__ qr, const FaceGeom &f,
                            const TetGeom &gs, int &mask) {
  mask = touch_mask(f.canon, f.off, 3, gs.canon, gs.off, 4);
  double sp[4][3];
  for (int j = 0; j < 4; ++j)
    for (int d = 0; d < 3; ++d) {
      double s = 0;
      for (int k = 0; k < 4; ++k) s = fma(qr->tet4[j][k], gs.v[k][d], s);
      sp[j][d] = s;
    }
  const double ws = 0.25 * gs.vol;
  dz acc = mk(0, 0);
  if (!mask) {
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      double r[3];
      for (int d = 0; d < 3; ++d) r[d] = qr->tri3[i][0] * f.v[0][d] + qr->tri3[i][1] * f.v[1][d] + qr->tri3[i][2] * f.v[2][d];
      double sep[4][3];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) sep[j][d] = r[d] - sp[j][d];
      dz g[4];
      pgf_eval_w<false, 4>(P, sep, 0, g);
      acc = acc + ((g[0] + g[1]) + (g[2] + g[3]));
    }
    return (f.area / 3.0 * ws) * acc;
  }
#pragma unroll 1
  for (int q = 0; q < 7; ++q) {
    double r[3];
    for (int d = 0; d < 3; ++d) r[d] = qr->tri7[q][0] * f.v[0][d] + qr->tri7[q][1] * f.v[1][d] + qr->tri7[q][2] * f.v[2][d];
    dz s0 = mk(0, 0);
#pragma unroll 1
    for (int b = 0; b < 9; ++b) {
      if (!((mask >> b) & 1)) continue;
      const int m = b / 3 - 1, n = b % 3 - 1;
      const double o[3] = {r[0] + m * P[pk::A], r[1] + n * P[pk::B], r[2]};
      double pot, V1[3];
      tet_potentials(gs.v, o, pot, V1);
      s0 = s0 + (kInv4Pi * pot) * mk(P[pk::PHRE + b], -P[pk::PHIM + b]);
    }
    {
      double sep[4][3];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) sep[j][d] = r[d] - sp[j][d];
      dz g[4];
      pgf_eval_w<true, 4>(P, sep, mask, g);
      axpy(s0, ws, (g[0] + g[1]) + (g[2] + g[3]));
    }
    axpy(acc, qr->w7[q] * f.area, s0);
  }
  return acc;
}

// M0 = II g_p over (test face F, source face G).
__device__ dz pair_face_face(const double *__restrict__ P, const QuadRules *__restrict__ qr, const FaceGeom &f,
                             const FaceGeom &g, int &mask) {
  mask = touch_mask(f.canon, f.off, 3, g.canon, g.off, 3);
  double gp[3][3];
  for (int j = 0; j < 3; ++j)
    for (int d = 0; d < 3; ++d) gp[j][d] = qr->tri3[j][0] * g.v[0][d] + qr->tri3[j][1] * g.v[1][d] + qr->tri3[j][2] * g.v[2][d];
  const double wg = g.area / 3.0;
  dz acc = mk(0, 0);
  if (!mask) {
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      double r[3];
      for (int d = 0; d < 3; ++d) r[d] = qr->tri3[i][0] * f.v[0][d] + qr->tri3[i][1] * f.v[1][d] + qr->tri3[i][2] * f.v[2][d];
      double sep[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) sep[j][d] = r[d] - gp[j][d];
      dz g[3];
      pgf_eval_w<false, 3>(P, sep, 0, g);
      acc = acc + (g[0] + g[1]) + g[2];
    }
    return (f.area / 3.0 * wg) * acc;
  }
#pragma unroll 1
  for (int q = 0; q < 7; ++q) {
    double r[3];
    for (int d = 0; d < 3; ++d) r[d] = qr->tri7[q][0] * f.v[0][d] + qr->tri7[q][1] * f.v[1][d] + qr->tri7[q][2] * f.v[2][d];
    dz s0 = mk(0, 0);
#pragma unroll 1
    for (int b = 0; b < 9; ++b) {
      if (!((mask >> b) & 1)) continue;
      const int m = b / 3 - 1, n = b % 3 - 1;
      const double o[3] = {r[0] + m * P[pk::A], r[1] + n * P[pk::B], r[2]};
      double iinv, ione;
      tri_potentials(g.v[0], g.v[1], g.v[2], o, iinv, ione);
      s0 = s0 + (kInv4Pi * iinv) * mk(P[pk::PHRE + b], -P[pk::PHIM + b]);
    }
    {
      double sep[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) sep[j][d] = r[d] - gp[j][d];
      dz g[3];
      pgf_eval_w<true, 3>(P, sep, mask, g);
      axpy(s0, wg, (g[0] + g[1]) + g[2]);
    }
    axpy(acc, qr->w7[q] * f.area, s0);
  }
  return acc;
}

// Far rule of pair_tet_face with both separations from one lattice-sum
// evaluation: m0 = II g_p(r - r') (test tet, source face) and m0r the same
// with r - r' reversed (test face, source tet), by the reversed-separation
// form of pgf_eval_w (oblique incidence, non-touching pairs).
__device__ void pair_tet_face_far_rev(const double *__restrict__ P, const QuadRules *__restrict__ qr,
                                      const TetGeom &gt, const FaceGeom &f, dz &m0, dz &m0r) {
  double fp[3][3], tp[4][3];
  for (int j = 0; j < 3; ++j)
    for (int d = 0; d < 3; ++d) fp[j][d] = qr->tri3[j][0] * f.v[0][d] + qr->tri3[j][1] * f.v[1][d] + qr->tri3[j][2] * f.v[2][d];
  for (int i = 0; i < 4; ++i)
    for (int d = 0; d < 3; ++d) {
      double s = 0;
      for (int k = 0; k < 4; ++k) s = fma(qr->tet4[i][k], gt.v[k][d], s);
      tp[i][d] = s;
    }
  dz acc = mk(0, 0), accr = mk(0, 0);
#pragma unroll 1
  for (int j = 0; j < 3; ++j) {
    double sep[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int d = 0; d < 3; ++d) sep[i][d] = tp[i][d] - fp[j][d];
    dz g[4], gr[4];
    pgf_eval_w<false, 4, true>(P, sep, 0, g, gr);
    acc = acc + ((g[0] + g[1]) + (g[2] + g[3]));
    accr = accr + ((gr[0] + gr[1]) + (gr[2] + gr[3]));
  }
  const double w = 0.25 * gt.vol * (f.area / 3.0);
  m0 = w * acc;
  m0r = w * accr;
}

// test tet (colour class list) x surface-charge face: Z[m_k(T), n_F] -= alpha_Tk sigma_F M0.
// Far pairs only: the touching ones come from the host list (k_tet_face_near).
__device__ __forceinline__ void tet_face_pair(const double *__restrict__ P, const QuadRules *__restrict__ qr,
                                              const TetGeom &gt, const TetFace *__restrict__ t2f, int T,
                                              const FaceGeom &f, int fi, const dz *__restrict__ alpha,
                                              const dz *__restrict__ sigma, const ZOut &out) {
  int mask;
  const dz m0 = pair_tet_face(P, qr, gt, f, mask);
  const dz sm = sigma[fi] * m0;
  for (int k = 0; k < 4; ++k) zput(out, t2f[4 * T + k].unknown, f.unknown, mk(0, 0) - alpha[4 * T + k] * sm, mask != 0);
}

// The far rules of the two face kernels take the same 4 x 3 point pairs with
// the same weights, so the (tet T, face F) evaluation also gives the value
// M0' of (F as a half-SWG test face, T as source): at normal incidence
// (swap 1) the lattice sum is even and M0' = M0; at oblique incidence
// (swap 2) M0' comes from the reversed-separation form of the same lattice
// sum.  With swap set, each far pair with a half-SWG face writes that entry
// too, Z[m_F, n_l(T)] -= gsrc_Tl kappa_T M0', at the transposed position of
// outT (rows of T's unknowns, columns of faces: the same conflict-free
// pattern as the tet-face entries); the staging copy is added transposed
// after the fill's other kernels.
template <bool REV_ONLY = false>
__device__ __forceinline__ void k_tet_face_body(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                  const TetGeom *__restrict__ tg, const TetFace *__restrict__ t2f,
                                                  const int32_t *__restrict__ test_list, int ntest,
                                                  const FaceGeom *__restrict__ fg, int nface,
                                                  const dz *__restrict__ alpha, const dz *__restrict__ sigma,
                                                  const dz *__restrict__ gsrc, const dz *__restrict__ kappa,
                                                  ZOut out, ZOut outT, int swap, int bx_, int by_) {
  extern __shared__ double s_tab[];
  stage_table(pack, packlen, s_tab);
  const double *__restrict__ P = s_tab;

  const int ti = uniform(by_ * 4 + (threadIdx.x >> 6));
  const int fi = bx_ * 64 + (threadIdx.x & 63);
  if (ti >= ntest || fi >= nface) return;
  const int T = uniform(test_list[ti]);
  const TetGeom &gt = tg[T];
  const FaceGeom f = fg[fi];
  if (touch_mask(gt.canon, gt.off, 4, f.canon, f.off, 3)) return;
  int mask;
  dz m0, m0r;
  if (REV_ONLY || swap == 2) {
    pair_tet_face_far_rev(s_tab, qr, gt, f, m0, m0r);
  } else {
    m0 = pair_tet_face(s_tab, qr, gt, f, mask);
    m0r = m0;
  }
  const dz sm = sigma[fi] * m0;
  for (int k = 0; k < 4; ++k) zput(out, t2f[4 * T + k].unknown, f.unknown, mk(0, 0) - alpha[4 * T + k] * sm, false);
  if (swap && f.half) {
    const dz km = m0r * kappa[T];
    for (int l = 0; l < 4; ++l) zput(outT, t2f[4 * T + l].unknown, f.unknown, mk(0, 0) - gsrc[4 * T + l] * km, false);
  }
}

__global__ __launch_bounds__(256, 2) void k_tet_face(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                  const TetGeom *__restrict__ tg, const TetFace *__restrict__ t2f,
                                                  const int32_t *__restrict__ test_list, int ntest,
                                                  const FaceGeom *__restrict__ fg, int nface,
                                                  const dz *__restrict__ alpha, const dz *__restrict__ sigma,
                                                  const dz *__restrict__ gsrc, const dz *__restrict__ kappa,
                                                  ZOut out, ZOut outT, int swap) {
  k_tet_face_body<false>(pack, packlen, qr, tg, t2f, test_list, ntest, fg, nface, alpha, sigma, gsrc, kappa, out, outT,
                         swap == 2 ? 0 : swap, blockIdx.x, blockIdx.y);
}
// oblique incidence with the staging copy: the (face, tet) entries from the
// reversed separation (swap 2); a kernel of its own, whose registers the
// two-separation form does not take from k_tet_face
__global__ __launch_bounds__(256, 2) void k_tet_face_rev(const double *__restrict__ pack, int packlen,
                                                      const QuadRules *__restrict__ qr, const TetGeom *__restrict__ tg,
                                                      const TetFace *__restrict__ t2f,
                                                      const int32_t *__restrict__ test_list, int ntest,
                                                      const FaceGeom *__restrict__ fg, int nface,
                                                      const dz *__restrict__ alpha, const dz *__restrict__ sigma,
                                                      const dz *__restrict__ gsrc, const dz *__restrict__ kappa,
                                                      ZOut out, ZOut outT) {
  k_tet_face_body<true>(pack, packlen, qr, tg, t2f, test_list, ntest, fg, nface, alpha, sigma, gsrc, kappa, out, outT, 2,
                        blockIdx.x, blockIdx.y);
}

// touching (test tet, surface-charge face) pairs of one test colour, one lane each
__device__ __forceinline__ void k_tet_face_near_body(const double *__restrict__ pack, int packlen,
                                                       const QuadRules *__restrict__ qr, const TetGeom *__restrict__ tg,
                                                       const TetFace *__restrict__ t2f, const int32_t *__restrict__ pairs,
                                                       int npairs, const FaceGeom *__restrict__ fg,
                                                       const dz *__restrict__ alpha, const dz *__restrict__ sigma,
                                                       ZOut out, int bx_, int by_) {
  extern __shared__ double s_tab[];
  stage_table(pack, packlen, s_tab);
  const int i = bx_ * 256 + threadIdx.x;
  if (i >= npairs) return;
  const int T = pairs[2 * i], fi = pairs[2 * i + 1];
  const FaceGeom f = fg[fi];
  tet_face_pair(s_tab, qr, tg[T], t2f, T, f, fi, alpha, sigma, out);
}

__global__ __launch_bounds__(256, 2) void k_tet_face_near(const double *__restrict__ pack, int packlen,
                                                       const QuadRules *__restrict__ qr, const TetGeom *__restrict__ tg,
                                                       const TetFace *__restrict__ t2f, const int32_t *__restrict__ pairs,
                                                       int npairs, const FaceGeom *__restrict__ fg,
                                                       const dz *__restrict__ alpha, const dz *__restrict__ sigma,
                                                       ZOut out) {
  k_tet_face_near_body(pack, packlen, qr, tg, t2f, pairs, npairs, fg, alpha, sigma, out, blockIdx.x, blockIdx.y);
}

// half-SWG test face x source tet (colour class list): Z[m_F, n_l(S)] -= gsrc_Sl kappa_S M0.
// Far pairs only: the touching ones come from the host list (k_face_tet_near).
__device__ __forceinline__ void face_tet_pair(const double *__restrict__ P, const QuadRules *__restrict__ qr,
                                              const FaceGeom &f, const TetGeom &gs, const TetFace *__restrict__ t2f,
                                              int S, const dz *__restrict__ gsrc, const dz *__restrict__ kappa,
                                              const ZOut &out) {
  int mask;
  const dz m0 = pair_face_tet(P, qr, f, gs, mask) * kappa[S];
  for (int l = 0; l < 4; ++l) zput(out, f.unknown, t2f[4 * S + l].unknown, mk(0, 0) - gsrc[4 * S + l] * m0, mask != 0);
}

__device__ __forceinline__ void k_face_tet_body(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                  const FaceGeom *__restrict__ fg, const int32_t *__restrict__ half_list,
                                                  int nhalf, const TetGeom *__restrict__ tg,
                                                  const TetFace *__restrict__ t2f, const int32_t *__restrict__ src_list,
                                                  int nsrc, const dz *__restrict__ gsrc, const dz *__restrict__ kappa,
                                                  ZOut out, int bx_, int by_) {
  extern __shared__ double s_tab[];
  stage_table(pack, packlen, s_tab);
  const double *__restrict__ P = s_tab;

  const int hi = uniform(by_ * 4 + (threadIdx.x >> 6));
  const int si = bx_ * 64 + (threadIdx.x & 63);
  if (hi >= nhalf || si >= nsrc) return;
  const FaceGeom &f = fg[uniform(half_list[hi])];
  const int S = src_list[si];
  const TetGeom gs = tg[S];
  if (touch_mask(f.canon, f.off, 3, gs.canon, gs.off, 4)) return;
  face_tet_pair(s_tab, qr, f, gs, t2f, S, gsrc, kappa, out);
}

__global__ __launch_bounds__(256, 2) void k_face_tet(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                  const FaceGeom *__restrict__ fg, const int32_t *__restrict__ half_list,
                                                  int nhalf, const TetGeom *__restrict__ tg,
                                                  const TetFace *__restrict__ t2f, const int32_t *__restrict__ src_list,
                                                  int nsrc, const dz *__restrict__ gsrc, const dz *__restrict__ kappa,
                                                  ZOut out) {
  k_face_tet_body(pack, packlen, qr, fg, half_list, nhalf, tg, t2f, src_list, nsrc, gsrc, kappa, out, blockIdx.x, blockIdx.y);
}

// touching (half-SWG test face, source tet) pairs of one source colour, one lane each
__device__ __forceinline__ void k_face_tet_near_body(const double *__restrict__ pack, int packlen,
                                                       const QuadRules *__restrict__ qr, const FaceGeom *__restrict__ fg,
                                                       const int32_t *__restrict__ half_list,
                                                       const TetGeom *__restrict__ tg, const TetFace *__restrict__ t2f,
                                                       const int32_t *__restrict__ pairs, int npairs,
                                                       const dz *__restrict__ gsrc, const dz *__restrict__ kappa,
                                                       ZOut out, int bx_, int by_) {
  extern __shared__ double s_tab[];
  stage_table(pack, packlen, s_tab);
  const int i = bx_ * 256 + threadIdx.x;
  if (i >= npairs) return;
  const int hi = pairs[2 * i], S = pairs[2 * i + 1];
  const FaceGeom f = fg[half_list[hi]];
  const TetGeom gs = tg[S];
  face_tet_pair(s_tab, qr, f, gs, t2f, S, gsrc, kappa, out);
}

__global__ __launch_bounds__(256, 2) void k_face_tet_near(const double *__restrict__ pack, int packlen,
                                                       const QuadRules *__restrict__ qr, const FaceGeom *__restrict__ fg,
                                                       const int32_t *__restrict__ half_list,
                                                       const TetGeom *__restrict__ tg, const TetFace *__restrict__ t2f,
                                                       const int32_t *__restrict__ pairs, int npairs,
                                                       const dz *__restrict__ gsrc, const dz *__restrict__ kappa,
                                                       ZOut out) {
  k_face_tet_near_body(pack, packlen, qr, fg, half_list, tg, t2f, pairs, npairs, gsrc, kappa, out, blockIdx.x, blockIdx.y);
}

// half-SWG test face x surface-charge face: Z[m_F, n_G] += sigma_G M0.  With
// no dense part in the destination (the structured-grid operator, whose far
// pairs come from its FFT tables) only the touching pairs are written.
__device__ __forceinline__ void k_face_face_body(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                   const FaceGeom *__restrict__ fg,
                                                   const int32_t *__restrict__ half_list, int nhalf, int nface,
                                                   const dz *__restrict__ sigma, ZOut out, int bx_, int by_) {
  extern __shared__ double s_tab[];
  stage_table(pack, packlen, s_tab);
  const double *__restrict__ P = s_tab;

  const int hi = uniform(by_ * 4 + (threadIdx.x >> 6));
  const int gi = bx_ * 64 + (threadIdx.x & 63);
  if (hi >= nhalf || gi >= nface) return;
  const FaceGeom &f = fg[uniform(half_list[hi])];
  const FaceGeom g = fg[gi];
  int mask;
  const dz m0 = pair_face_face(s_tab, qr, f, g, mask);
  if (mask == 0 && !out.Z && !out.Zs) return;
  zput(out, f.unknown, g.unknown, sigma[gi] * m0, mask != 0);
}

__global__ __launch_bounds__(256, 2) void k_face_face(const double *__restrict__ pack, int packlen, const QuadRules *__restrict__ qr,
                                                   const FaceGeom *__restrict__ fg,
                                                   const int32_t *__restrict__ half_list, int nhalf, int nface,
                                                   const dz *__restrict__ sigma, ZOut out) {
  k_face_face_body(pack, packlen, qr, fg, half_list, nhalf, nface, sigma, out, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------------ fused multi-cell fill
// The segment of fused-grid block b (segments ordered by their first block).
template <class S>
__device__ __forceinline__ int seg_of(const S *__restrict__ segs, int nseg, int b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= b) lo = mid;
    else hi = mid - 1;
  }
  return uniform(lo);
}

#define VIE_SEG_BEGIN(S)                                  \
  const int s_ = seg_of(segs, nseg, (int)blockIdx.x);     \
  const S &A = segs[s_];                                  \
  const int lb_ = (int)blockIdx.x - A.first;              \
  const int bx = lb_ % A.gx, by = lb_ / A.gx;

__global__ __launch_bounds__(256, 2) void k_tt_far_seg(const FarSeg *__restrict__ segs, int nseg) {
  VIE_SEG_BEGIN(FarSeg)
  tt_far_body<false>(A.pack, A.packlen, A.qr, A.tg, A.t2f, A.test_list, A.ntest, A.src_list, A.nsrc, A.alpha, A.gsrc,
                     A.kappa, A.k0sq9, A.out, A.outT, A.sym, bx, by);
}
__global__ __launch_bounds__(256, 2) void k_tt_far_rev_seg(const FarSeg *__restrict__ segs, int nseg) {
  VIE_SEG_BEGIN(FarSeg)
  tt_far_body<true>(A.pack, A.packlen, A.qr, A.tg, A.t2f, A.test_list, A.ntest, A.src_list, A.nsrc, A.alpha, A.gsrc,
                    A.kappa, A.k0sq9, A.out, A.outT, A.sym, bx, by);
}
__global__ __launch_bounds__(256) void k_tt_near_seg(const NearSeg *__restrict__ segs, int nseg) {
  VIE_SEG_BEGIN(NearSeg)
  k_tt_near_body(A.pack, A.packlen, A.qr, A.tg, A.t2f, A.lt, A.ls, A.lmask, A.npairs, A.alpha, A.gsrc, A.kappa,
                 A.inv_eps, A.k0sq9, A.out, bx, by);
}
__global__ __launch_bounds__(256, 2) void k_tet_face_seg(const TetFaceSeg *__restrict__ segs, int nseg) {
  VIE_SEG_BEGIN(TetFaceSeg)
  k_tet_face_body(A.pack, A.packlen, A.qr, A.tg, A.t2f, A.test_list, A.ntest, A.fg, A.nface, A.alpha, A.sigma, A.gsrc,
                  A.kappa, A.out, A.outT, A.swap, bx, by);
}
__global__ __launch_bounds__(256, 2) void k_tet_face_near_seg(const TetFaceNearSeg *__restrict__ segs, int nseg) {
  VIE_SEG_BEGIN(TetFaceNearSeg)
  k_tet_face_near_body(A.pack, A.packlen, A.qr, A.tg, A.t2f, A.pairs, A.npairs, A.fg, A.alpha, A.sigma, A.out, bx, by);
}
__global__ __launch_bounds__(256, 2) void k_face_tet_seg(const FaceTetSeg *__restrict__ segs, int nseg) {
  VIE_SEG_BEGIN(FaceTetSeg)
  k_face_tet_body(A.pack, A.packlen, A.qr, A.fg, A.half_list, A.nhalf, A.tg, A.t2f, A.src_list, A.nsrc, A.gsrc,
                  A.kappa, A.out, bx, by);
}
__global__ __launch_bounds__(256, 2) void k_face_tet_near_seg(const FaceTetNearSeg *__restrict__ segs, int nseg) {
  VIE_SEG_BEGIN(FaceTetNearSeg)
  k_face_tet_near_body(A.pack, A.packlen, A.qr, A.fg, A.half_list, A.tg, A.t2f, A.pairs, A.npairs, A.gsrc, A.kappa,
                       A.out, bx, by);
}
__global__ __launch_bounds__(256, 2) void k_face_face_seg(const FaceFaceSeg *__restrict__ segs, int nseg) {
  VIE_SEG_BEGIN(FaceFaceSeg)
  k_face_face_body(A.pack, A.packlen, A.qr, A.fg, A.half_list, A.nhalf, A.nface, A.sigma, A.out, bx, by);
}
#undef VIE_SEG_BEGIN

// ------------------------------------------------------------ right-hand side
// b_m = sum_{T in m} chi s a_m/(3 V_T) int_T (r - p).E^i dV, 14-point rule;
// one thread per unknown (gathers its two halves, no write conflicts).
__global__ void k_rhs(int64_t N, const int32_t *__restrict__ utet, const int32_t *__restrict__ uk,
                      const TetGeom *__restrict__ tg, const QuadRules *__restrict__ qr, const dz *__restrict__ alpha,
                      double kix, double kiy, double kiz, double ex, double ey, double ez, dz *__restrict__ b) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  dz acc = mk(0, 0);
  for (int h = 0; h < 2; ++h) {
    const int T = utet[2 * m + h];
    if (T < 0) continue;
    const int k = uk[2 * m + h];
    const TetGeom &g = tg[T];
    dz s = mk(0, 0);
    for (int q = 0; q < 14; ++q) {
      double r[3];
      for (int d = 0; d < 3; ++d) {
        double t = 0;
        for (int kk = 0; kk < 4; ++kk) t = fma(qr->tet14[q][kk], g.v[kk][d], t);
        r[d] = t;
      }
      const double proj = (r[0] - g.v[k][0]) * ex + (r[1] - g.v[k][1]) * ey + (r[2] - g.v[k][2]) * ez;
      double sn, cs;
      sincos(-(kix * r[0] + kiy * r[1] + kiz * r[2]), &sn, &cs);
      axpy(s, qr->w14[q] * g.vol * proj, mk(cs, sn));
    }
    acc = acc + alpha[4 * T + k] * ((1.0 / 3.0) * s);
  }
  b[m] = acc;
}

// ------------------------------------------------------------ diagnostics
__global__ void k_pgf_probe(const double *__restrict__ pack, int packlen, const double *__restrict__ d, int64_t n,
                            dz *__restrict__ out) {
  extern __shared__ double s_tab[];
  stage_table(pack, packlen, s_tab);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = pgf_eval<false>(s_tab, d[3 * i], d[3 * i + 1], d[3 * i + 2], 0);
}

// gather Z entries (mixed precision: FP32 far part plus the FP64 near entry)
__global__ void k_gather(ZOut Z, const int64_t *__restrict__ rows, const int64_t *__restrict__ cols, int64_t k,
                         dz *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int64_t m = rows[i], n = cols[i];
  if (Z.Z) {
    out[i] = Z.Z[m * Z.ld + n];
    return;
  }
  const fz f = Z.Zs[m * Z.ld + n];
  dz v = mk(f.re, f.im);
  int64_t lo = Z.rowptr[m], hi = Z.rowptr[m + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (Z.cols[mid] < n) lo = mid + 1;
    else hi = mid;
  }
  if (lo < Z.rowptr[m + 1] && Z.cols[lo] == n) v = v + Z.vals[lo];
  out[i] = v;
}

}  // namespace vie
