// Structured-grid far operator (see grid.h): kernel tables from the lattice
// sums, the source fields of a vector, the per-frequency products and the
// far potentials tested against every unknown, plus the near part.
//
// Field layout: field c, point x + nx (y + ny z) at c nf + that index, z over
// the padded length pz; charge fields c = s (s < kGridSub), current fields
// c = kGridSub + kGridTetSub d + s (component d, tetrahedron sublattice s).
// Table: sublattice pair (s, s') at (s kGridSub + s') nf.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "grid.h"
#include "kernels.h"

namespace vie {

__device__ __forceinline__ dz cexpj(double t) {
  double s, c;
  sincos(t, &s, &c);
  return mk(c, s);
}

// Kernel table of one sublattice pair over the brick offsets (blockIdx.y =
// s kGridSub + s', or with `sym` the slot of a pair s <= s'): offset (dx, dy)
// taken in (-n/2, n/2] (the circulant kernel is periodic in it), dz = z for
// z < lz and z - pz above (z = lz unused).  At normal incidence (sym) g_p is
// even, so K(s', s, -d) = K(s, s', d): only the pairs s <= s' are stored, and
// the product reads K(s', s) at the reversed frequency.
//   K(s, s', d) = scale e^{+j kt.(dx hx, dy hy)} g_p(pos_s - pos_s' + d h),
// zero for corner-sharing pairs (any image) and for separations beyond the
// mesh's height (no element pair has them; the fits do not cover them).
__global__ __launch_bounds__(256) void k_grid_table(const double *__restrict__ pack, int packlen,
                                                    const GridGeom *__restrict__ gg, double kx, double ky,
                                                    double scale, int sym, dz *__restrict__ tab) {
  extern __shared__ double s_tab[];
  stage_table(pack, packlen, s_tab);
  const GridGeom &G = *gg;
  const int64_t nf = G.nf;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nf) return;
  const int sp = blockIdx.y;
  int s = sp / kGridSub, s2 = sp % kGridSub;
  if (sym) {   // slot sp of the pairs s <= s2, row by row
    s = 0;
    while (sp >= grid_sym_pair(s + 1, s + 1)) ++s;
    s2 = s + (sp - grid_sym_pair(s, s));
  }
  const int nx = G.nx, ny = G.ny;
  const int x = (int)(id % nx), y = (int)((id / nx) % ny), z = (int)(id / ((int64_t)nx * ny));
  dz out = mk(0.0, 0.0);
  if (z != G.lz) {
    const int dz_ = z < G.lz ? z : z - G.pz;
    const int dx = x <= nx / 2 ? x : x - nx, dy = y <= ny / 2 ? y : y - ny;
    bool touch = false;
    if (dz_ >= -1 && dz_ <= 1) {
      const int e = G.ent[s], e2 = G.ent[s2];
      for (int ox = -1; ox <= 1; ++ox) {
        if (((ox - x) % nx + nx) % nx) continue;
        for (int oy = -1; oy <= 1; ++oy) {
          if (((oy - y) % ny + ny) % ny) continue;
          touch = touch || G.touch[e][e2][(ox + 1) + 3 * (oy + 1) + 9 * (dz_ + 1)];
        }
      }
    }
    const double sx = G.pos[s][0] - G.pos[s2][0] + dx * G.h[0];
    const double sy = G.pos[s][1] - G.pos[s2][1] + dy * G.h[1];
    const double sz = G.pos[s][2] - G.pos[s2][2] + dz_ * G.h[2];
    if (!touch && fabs(sz) <= G.zspan * (1.0 + 1e-12)) {
      const dz g = pgf_eval<false>(s_tab, sx, sy, sz, 0);
      out = (scale * cexpj(kx * dx * G.h[0] + ky * dy * G.h[1])) * g;
    }
  }
  tab[(int64_t)sp * nf + id] = out;
}

// Source fields of the tetrahedra: per tetrahedron S (one thread) its charge
// w rho_S and current w (rho_S r'_j - sum_l b_l x_l v_l) at its four points,
// positions relative to its brick, modulated by e^{+j kt.o} (o: brick origin).
// Every (brick, type) holds at most one tetrahedron: no two threads write one
// slot.  The fields start cleared.
__global__ __launch_bounds__(256) void k_grid_gather_tet(int64_t nt, const GridGeom *__restrict__ gg,
                                                         const int32_t *__restrict__ gtet,
                                                         const TetGeom *__restrict__ tg,
                                                         const TetFace *__restrict__ t2f, const dz *__restrict__ gsrc,
                                                         const dz *__restrict__ kappa, const dz *__restrict__ x,
                                                         double kx, double ky, dz *__restrict__ fld) {
  const int64_t T = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (T >= nt) return;
  const GridGeom &G = *gg;
  const int64_t nf = G.nf;
  const int slot = gtet[2 * T], type = gtet[2 * T + 1];
  const int bx = slot % G.nx, by = (slot / G.nx) % G.ny, bz = slot / (G.nx * G.ny);
  const double o[3] = {G.org[0] + bx * G.h[0], G.org[1] + by * G.h[1], G.org[2] + bz * G.h[2]};
  const dz ks = kappa[T];
  dz rho = mk(0.0, 0.0), c[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  for (int l = 0; l < 4; ++l) {
    const dz bxl = (gsrc[4 * T + l] * ks) * x[t2f[4 * T + l].unknown];
    rho = rho + bxl;
    for (int d = 0; d < 3; ++d) c[d] = c[d] + (tg[T].v[l][d] - o[d]) * bxl;
  }
  const dz ph = cexpj(kx * bx * G.h[0] + ky * by * G.h[1]);
  const double w = 0.25 * tg[T].vol;
  const dz wr = (w * ph) * rho;
  for (int q = 0; q < 4; ++q) {
    const int s = 4 * type + q;
    fld[(int64_t)s * nf + slot] = wr;
    for (int d = 0; d < 3; ++d)
      fld[(int64_t)(kGridSub + kGridTetSub * d + s) * nf + slot] = (w * ph) * (G.pos[s][d] * rho - c[d]);
  }
}

// Source fields of the surface-charge faces: charge -(A/3) sigma x at each of
// the face's three points (one thread per face).
__global__ __launch_bounds__(256) void k_grid_gather_face(int nface, const GridGeom *__restrict__ gg,
                                                          const int32_t *__restrict__ gface,
                                                          const FaceGeom *__restrict__ fg,
                                                          const dz *__restrict__ sigma, const dz *__restrict__ x,
                                                          double kx, double ky, dz *__restrict__ fld) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nface) return;
  const GridGeom &G = *gg;
  const int bx = gface[4 * i], by = gface[4 * i + 1], bz = gface[4 * i + 2], type = gface[4 * i + 3];
  const int64_t slot = bx % G.nx + (int64_t)G.nx * (by % G.ny + (int64_t)G.ny * bz);
  const dz q = (-fg[i].area / 3.0 * cexpj(kx * bx * G.h[0] + ky * by * G.h[1])) * (sigma[i] * x[fg[i].unknown]);
  for (int p = 0; p < 3; ++p) fld[(int64_t)(kGridTetSub + 3 * type + p) * G.nf + slot] = q;
}

// Per-frequency products.  A block takes kGridTile frequencies and every
// test sublattice: the 132 source fields of the tile are staged in LDS once,
// and each table entry is read once from HBM (the 32 lanes of an s-group
// read kGridTile consecutive frequencies of one table row).  Thread t owns
// frequency t % kGridTile of the tile and the sublattices s = t / kGridTile
// + 8 i: the scalar potential from every charge field and, for tetrahedron
// sublattices, the vector potential from the current fields.
constexpr int kGridTile = 32;
template <bool SYM>
__device__ __forceinline__ void grid_mul_body(int64_t nf, int nx, int ny, int pz, const dz *__restrict__ tab,
                                              const dz *__restrict__ fin, dz *__restrict__ fout) {
  __shared__ dz sf[kGridFields][kGridTile];
  const int64_t f0 = (int64_t)blockIdx.x * kGridTile;
  const int nt = (int)min<int64_t>(kGridTile, nf - f0);
  for (int e = threadIdx.x; e < kGridFields * kGridTile; e += 256) {
    const int c = e / kGridTile, fi = e % kGridTile;
    sf[c][fi] = fi < nt ? fin[(int64_t)c * nf + f0 + fi] : mk(0.0, 0.0);
  }
  __syncthreads();
  const int fi = threadIdx.x % kGridTile, sg = threadIdx.x / kGridTile;
  if (fi >= nt) return;
  const int64_t f = f0 + fi;
  // (SYM) the reversed frequency -f: each coordinate negated modulo its length
  int64_t fr = f;
  if (SYM) {
    const int x = (int)(f % nx), y = (int)((f / nx) % ny), z = (int)(f / ((int64_t)nx * ny));
    fr = (nx - x) % nx + (int64_t)nx * ((ny - y) % ny + (int64_t)ny * ((pz - z) % pz));
  }
  // Table row of output s: without SYM the 60 pairs (s, s2) at f, one table
  // stride apart.  With SYM, for s2 < s the stored pair (s2, s) at -f (its
  // slot advances by kGridSub - s2 - 1 from s2 to s2 + 1), and for
  // s2 >= s the pairs (s, s2) at f, in consecutive slots.
  auto entry = [&](int s, int s2) -> const dz * {
    if (!SYM) return tab + ((int64_t)s * kGridSub + s2) * nf + f;
    return s2 < s ? tab + (int64_t)grid_sym_pair(s2, s) * nf + fr : tab + (int64_t)grid_sym_pair(s, s2) * nf + f;
  };
  for (int s = sg; s < kGridSub; s += 256 / kGridTile) {
    dz acc = mk(0.0, 0.0);
    if (SYM) {
      const dz *K = tab + (int64_t)s * nf + fr;   // slot of (0, s)
#pragma unroll 4
      for (int s2 = 0; s2 < s; ++s2) {
        acc = acc + *K * sf[s2][fi];
        K += (int64_t)(kGridSub - s2 - 1) * nf;   // (s2, s) -> (s2 + 1, s)
      }
      K = tab + (int64_t)grid_sym_pair(s, s) * nf + f;
#pragma unroll 4
      for (int s2 = s; s2 < kGridSub; ++s2, K += nf) acc = acc + *K * sf[s2][fi];
    } else {
      const dz *K = tab + (int64_t)s * kGridSub * nf + f;
#pragma unroll 4
      for (int s2 = 0; s2 < kGridSub; ++s2) acc = acc + K[(int64_t)s2 * nf] * sf[s2][fi];
    }
    fout[(int64_t)s * nf + f] = acc;
    if (s < kGridTetSub) {
      dz a0 = mk(0.0, 0.0), a1 = mk(0.0, 0.0), a2 = mk(0.0, 0.0);
#pragma unroll 4
      for (int s2 = 0; s2 < kGridTetSub; ++s2) {
        const dz k = *entry(s, s2);
        a0 = a0 + k * sf[kGridSub + s2][fi];
        a1 = a1 + k * sf[kGridSub + kGridTetSub + s2][fi];
        a2 = a2 + k * sf[kGridSub + 2 * kGridTetSub + s2][fi];
      }
      fout[(int64_t)(kGridSub + s) * nf + f] = a0;
      fout[(int64_t)(kGridSub + kGridTetSub + s) * nf + f] = a1;
      fout[(int64_t)(kGridSub + 2 * kGridTetSub + s) * nf + f] = a2;
    }
  }
}

__global__ __launch_bounds__(256) void k_grid_mul(int64_t nf, const dz *__restrict__ tab, const dz *__restrict__ fin,
                                                  dz *__restrict__ fout) {
  grid_mul_body<false>(nf, 1, 1, 1, tab, fin, fout);
}
__global__ __launch_bounds__(256) void k_grid_mul_sym(int64_t nf, int nx, int ny, int pz, const dz *__restrict__ tab,
                                                      const dz *__restrict__ fin, dz *__restrict__ fout) {
  grid_mul_body<true>(nf, nx, ny, pz, tab, fin, fout);
}

// y = Z x (or b - Z x), one wave per unknown m: lanes 0-7 the far
// potentials at the four points of each of m's tetrahedra (demodulated by
// e^{-j kt.o}), lanes 8-10 those at the three points of m's face when it is a
// half-SWG face, and all lanes m's row of the near part (CSR, FP64); the wave
// sum is written by lane 0.
__global__ __launch_bounds__(256) void k_grid_apply(
    int64_t N, const GridGeom *__restrict__ gg, const int32_t *__restrict__ gtet, const int32_t *__restrict__ gface,
    const int32_t *__restrict__ ghalf, const int32_t *__restrict__ utet, const int32_t *__restrict__ uk,
    const TetGeom *__restrict__ tg, const FaceGeom *__restrict__ fg, const dz *__restrict__ alpha,
    const dz *__restrict__ fout, double k0sq9, double kx, double ky, const int64_t *__restrict__ rowptr,
    const int32_t *__restrict__ cols, const dz *__restrict__ vals, const dz *__restrict__ x, const dz *__restrict__ b,
    dz *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= N) return;   // the whole wave
  const GridGeom &G = *gg;
  const int64_t nf = G.nf;
  dz acc = mk(0.0, 0.0);
  if (lane < 8) {
    const int h = lane >> 2, q = lane & 3;
    const int T = utet[2 * m + h];
    if (T >= 0) {
      const int k = uk[2 * m + h];
      const int slot = gtet[2 * T], type = gtet[2 * T + 1];
      const int bx = slot % G.nx, by = (slot / G.nx) % G.ny, bz = slot / (G.nx * G.ny);
      const int s = 4 * type + q;
      dz ra = mk(0.0, 0.0);
      for (int d = 0; d < 3; ++d) {
        const double vk = tg[T].v[k][d] - (G.org[d] + (d == 0 ? bx : d == 1 ? by : bz) * G.h[d]);
        ra = ra + (G.pos[s][d] - vk) * fout[(int64_t)(kGridSub + kGridTetSub * d + s) * nf + slot];
      }
      const dz ph = cexpj(-(kx * bx * G.h[0] + ky * by * G.h[1]));
      acc = ((0.25 * tg[T].vol) * alpha[4 * T + k]) * (ph * (fout[(int64_t)s * nf + slot] - k0sq9 * ra));
    }
  } else if (lane < 11) {
    const int i = ghalf[m];
    if (i >= 0) {
      const int bx = gface[4 * i], by = gface[4 * i + 1], bz = gface[4 * i + 2], type = gface[4 * i + 3];
      const int64_t slot = bx % G.nx + (int64_t)G.nx * (by % G.ny + (int64_t)G.ny * bz);
      acc = (-fg[i].area / 3.0 * cexpj(-(kx * bx * G.h[0] + ky * by * G.h[1]))) *
            fout[(int64_t)(kGridTetSub + 3 * type + (lane - 8)) * nf + slot];
    }
  }
  for (int64_t e = rowptr[m] + lane; e < rowptr[m + 1]; e += 64) acc = acc + vals[e] * x[cols[e]];
  for (int o = 32; o > 0; o >>= 1) {
    acc.re += __shfl_xor(acc.re, o);
    acc.im += __shfl_xor(acc.im, o);
  }
  if (lane == 0) y[m] = b ? b[m] - acc : acc;
}

}  // namespace vie
