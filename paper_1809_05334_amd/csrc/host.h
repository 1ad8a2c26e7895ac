// Host-side internals of libvie: mesh topology, quadrature rules, lattice-sum
// tables and the special functions used to build them.
#pragma once
#include <complex>
#include <string>
#include <vector>

#include "common.h"

namespace vie {

using zd = std::complex<double>;

struct MeshTopology {
  double a = 0, b = 0;
  int64_t nv = 0, nt = 0;
  int ndom = 0;
  std::vector<double> verts;        // 3*nv
  std::vector<int32_t> tets;        // 4*nt
  std::vector<int32_t> dom;         // nt
  std::vector<int32_t> canon;       // nv  canonical vertex id
  std::vector<int32_t> offx, offy;  // nv  lattice offset of each vertex
  std::vector<double> vol;          // nt
  double zmin = 0, zmax = 0;
  double max_diam = 0;              // largest tetrahedron diameter

  int64_t N = 0;                    // unknowns
  std::vector<int32_t> face_vid;    // 3N (as the face sits in T+)
  std::vector<int32_t> tplus, tminus, fdom, freep, freem;
  std::vector<int32_t> shx, shy;    // lattice shift of T-'s copy
  std::vector<double> area;         // N
  std::vector<TetFace> t2f;         // 4*nt
  std::vector<int32_t> charged;     // surface-charge faces (unknown ids), increasing
  std::vector<int64_t> dstart, dend;

  // conflict-free colouring of the tetrahedra (face-adjacent tets differ)
  int ncolors = 0;
  std::vector<int32_t> color;                     // nt
  std::vector<std::vector<int32_t>> color_tets;   // per colour, increasing
  // touching tet pairs, grouped by (colour(T), colour(T')): test, source, image mask
  std::vector<std::vector<int32_t>> near_t, near_s, near_mask;
  // touching (tet T, surface-charge face) pairs grouped by colour(T): T and the
  // face's position in `charged`, interleaved
  std::vector<std::vector<int32_t>> near_tf;
  // touching (half-SWG face, tet S) pairs grouped by colour(S): the face's
  // position among the half-SWG faces of `charged`, and S, interleaved
  std::vector<std::vector<int32_t>> near_ft;
};

// Returns "" on success, else an error message.
std::string build_topology(MeshTopology &t, const double *verts, int64_t nv, const int32_t *tets, int64_t nt,
                           const int32_t *tet_domain, int ndom, double a, double b);

// Sparsity pattern of the near (touching-pair) entries of Z, CSR with sorted
// rows (rowptr [N+1], cols [nnz]).
void build_near_pattern(const MeshTopology &t, std::vector<int64_t> &rowptr, std::vector<int32_t> &cols);

// Tetrahedron holding each of n points (3n doubles): the lowest index among
// those whose barycentric coordinates are all >= -1e-12, -1 if none.
void locate_points(const MeshTopology &t, const double *pts, int64_t n, int32_t *tet);

// Touching-image mask (bit (m+1)*3 + (n+1)) of two vertex sets given by canonical
// ids and packed offsets ((ox+2) | (oy+2) << 4).
inline int touching_mask(const int32_t *ct, const int32_t *ot, int nt_, const int32_t *cs, const int32_t *os,
                         int ns) {
  int mask = 0;
  for (int i = 0; i < nt_; ++i)
    for (int j = 0; j < ns; ++j)
      if (ct[i] == cs[j]) {
        int dm = (os[j] & 15) - (ot[i] & 15);
        int dn = (os[j] >> 4) - (ot[i] >> 4);
        mask |= 1 << ((dm + 1) * 3 + (dn + 1));
      }
  return mask;
}

void build_quadrature(QuadRules &q);

// Special functions (host, FP64): complex erfc and erfcx from their integral
// definitions evaluated by Gauss-Legendre quadrature.
zd erfc_c(zd z);
zd erfcx_c(zd z);
double erfi_r(double y);

// Ewald split and per-fill tables.  zspan = zmax - zmin of the mesh.
// Returns "" or an error; sets *wood_margin = min_{(p,q)!=(0,0)} |gamma_pq|/k0.
std::string build_pgf_table(PgfTable &tab, double a, double b, double zspan, double lambda, double theta,
                            double phi, double *wood_margin);

// Compact copy of the table for the kernels (staged into LDS): only the
// fitted coefficients of the significant terms, in doubles.  Layout:
//   [0..10)  E, a, b, 1/a, 1/b, kx, ky, 2pi/a, 2pi/b, ws
//   [10..19) Re phase0[9], [19..28) Im phase0[9], [28] nimg
//   [32..113) per mode (p,q) grid index: offset of its record or 0 (low
//             word), K | cplx << 16 (high word)
//   [116..125) per row p of the mode grid: q_lo | (q_hi + 1) << 8, the
//             first and last q with a mode (0 | 0 << 8: none)
//   image records from kPackImages on, each
//     [xa, xs, cre, cim, m, n, K, len] f[0..K] (pad to 4) [HK, 0, 0, 0] h[0..HK] (pad to 4)
//     (the H block only for touching classes; len = record length)
//   mode records [K, cplx, 0, 0] kre[0..K] (pad) kim[0..K] (pad, complex orders only)
// Integer fields (nimg, mode offsets, m, n, K, len, HK, cplx) hold the value in
// the low 32 bits of the double slot.
// K, HK are the degrees rounded up to a multiple of 4 (zero coefficients).
constexpr int kPackRows = 116;
constexpr int kPackImages = 128;
void pack_pgf_table(const PgfTable &tab, std::vector<double> &out);

}  // namespace vie
