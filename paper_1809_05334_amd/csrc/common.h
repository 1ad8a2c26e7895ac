// Plain data shared by the host code and the HIP kernels of libvie.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define VIE_HD __host__ __device__
#else
#define VIE_HD
#endif

namespace vie {

// ------------------------------------------------------------ lattice sums
// Ewald periodic Green's function tables for one (lambda, theta, phi, cell).
//
// g_p(Delta) = phase0(m0, n0) * [ sum_images c_mn F_mn(R E) / R  +  sum_modes e^{-j k_tpq . Delta_t} K_pq(w) ]
// with Delta_t wrapped to the nearest image (shift (m0, n0)), R = |Delta_w + rho_mn|,
// w = (Delta_z E)^2.  F_mn is the per-image Chebyshev fit of
//   F(x) = exp(y^2 - x^2) Re erfcx(x - j y),  y = k0 / (2E)
// on the image's range of x = R E; for touching images the kernel uses
//   H(x) = (F(x) - 1) / x   (so the extracted 1/(4 pi R) never cancels numerically).
// K_pq(w) is the Chebyshev fit (in w) of the spectral term of mode (p, q):
//   (1 / (4 a b gamma)) [e^{gamma z} erfc(gamma/2E + z E) + e^{-gamma z} erfc(gamma/2E - z E)].
constexpr int kPgfMaxDeg = 47;
constexpr int kPgfM = 4;                         // |m|,|n|,|p|,|q| <= 4
constexpr int kPgfSide = 2 * kPgfM + 1;          // 9
constexpr int kPgfTerms = kPgfSide * kPgfSide;   // 81

struct PgfImage {
  double xa, xs;        // t = (x - xa) * xs - 1 maps [xlo, xhi] to [-1, 1]
  double cre, cim;      // e^{j kt.rho_mn} / (4 pi)
  int m, n;             // lattice image
  int deg, hdeg;        // Chebyshev degrees of F and H (hdeg < 0: no H fit)
  double f[kPgfMaxDeg + 1];
  double h[kPgfMaxDeg + 1];
};

struct PgfMode {
  int p, q;
  int deg;                        // < 0: mode skipped (below significance)
  int cplx;                       // 1 for a propagating order (complex K)
  double kre[kPgfMaxDeg + 1];
  double kim[kPgfMaxDeg + 1];
};

struct PgfTable {
  double a, b, inv_a, inv_b;
  double E, k0, kx, ky;
  double two_pi_a, two_pi_b;      // 2 pi / a, 2 pi / b
  double ws;                      // t_w = w * ws - 1 maps [0, wmax] to [-1, 1]
  double ph0re[9], ph0im[9];      // e^{-j (kx m0 a + ky n0 b)}, index (m0+1)*3 + (n0+1)
  int nimg;               // significant images, compact list
  int pad0, pad1, pad2;
  PgfImage img[kPgfTerms];
  PgfMode mode[kPgfTerms]; // dense grid, index (p+4)*9 + (q+4); deg < 0: below significance
};

// ------------------------------------------------------------ quadrature
// Barycentric rules (weights sum to 1).  Far pairs: tet 4-pt (degree 2) x
// triangle 3-pt (degree 2).  Touching pairs: outer tet 14-pt / triangle 7-pt
// (degree 5) with closed-form inner integrals + the degree-2 inner rule for
// the remainder.
struct QuadRules {
  double tet4[4][4], w4[4];
  double tet14[14][4], w14[14];
  double tri3[3][3], w3[3];
  double tri7[7][3], w7[7];
};

// ------------------------------------------------------------ mesh tables
// Per tetrahedron (device, AoS): vertices, centroid, volume, canonical
// vertex ids and lattice offsets of its vertices (for the touching test).
struct TetGeom {
  double v[4][3];
  double c[3];
  double vol;
  int32_t canon[4];
  int32_t off[4];       // (ox + 2) | (oy + 2) << 4
};

// Surface-charge / half-SWG face element (the face as it sits in T+).
struct FaceGeom {
  double v[3][3];
  double area;
  int32_t unknown;
  int32_t canon[3];
  int32_t off[3];
  int32_t half;         // 1 for a half-SWG (structure boundary)
};

// Per (tet, local face k): unknown id, orientation sign and the lattice
// shift of this tet's copy of the face (0 for T+).
struct TetFace {
  int32_t unknown;
  int32_t sign;
  int32_t sx, sy;
};

struct cplx {
  double re, im;
};

}  // namespace vie
