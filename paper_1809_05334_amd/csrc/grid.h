// Structured-grid far operator: on a uniform Kuhn brick grid the far part of
// Z x is a sum of discrete convolutions over brick offsets, evaluated by FFT.
//
// Every far term of Z (Sec. 2.1, Eq. 2 with the far product rules: tet 4-point
// x tet 4-point, tet 4-point x face 3-point, face 3-point x face 3-point) is a
// point-to-point lattice sum g_p(r - r') (Sec. 2.2, Eqs. 3-4) weighted by
// per-point densities.  On a uniform grid whose bricks are all split the same
// way, the quadrature points fall on kGridSub sublattices (each tetrahedron
// type and point, each face type and point), and g_p between two sublattices
// depends only on the brick offset.  With the sources modulated by
// e^{+j kt.x} the kernel is exactly circulant in x and y (g_p(d + R) =
// e^{-j kt.R} g_p(d) for a lattice vector R) and Toeplitz in z (zero-padded to
// twice the number of layers), so one 3D FFT per field, a per-frequency
// product with the tabulated kernels and one inverse FFT give every far
// potential at every point.  Pairs that touch (share a vertex under some
// lattice image) are zero in the tables: their entries come from the near
// kernels, as in the dense fill.
//
// Per test tetrahedron T, local face k (unknown m), with scalar potential Phi
// and vector potential A at T's points r_i (weights w = V/4):
//   (Z x)_m += alpha_Tk w_T sum_i [ Phi(r_i) - (k0^2/9) (r_i - v_k).A(r_i) ]
// and per half-SWG test face F (weights A_F/3 at its points r_p):
//   (Z x)_m -= (A_F/3) sum_p Phi(r_p),
// with the sources
//   tetrahedron S, point j:  charge w_S rho_S,  current w_S sum_l b_l x_l (r'_j - v_l),
//   rho_S = sum_l b_l x_l,   b_l = gsrc_Sl kappa_S,
//   surface-charge face G, point q:  charge -(A_G/3) sigma_G x_G.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#ifndef __HIPCC__
#ifndef __host__
#define __host__
#define __device__
#endif
#endif

namespace vie {

constexpr int kGridTetTypes = 6;                        // Kuhn tetrahedra of a brick
constexpr int kGridFaceTypes = 12;                      // faces owned by a brick
constexpr int kGridEnt = kGridTetTypes + kGridFaceTypes;
constexpr int kGridTetSub = 4 * kGridTetTypes;          // tetrahedron point sublattices
constexpr int kGridSub = kGridTetSub + 3 * kGridFaceTypes;   // all point sublattices (60)
constexpr int kGridFields = kGridSub + 3 * kGridTetSub;  // charge fields + current fields (132)
constexpr int kGridSymPairs = kGridSub * (kGridSub + 1) / 2;   // pairs s <= s' (1,830)

// Slot of the pair (s, s'), s <= s', in a table stored for s <= s' only.
__host__ __device__ inline int grid_sym_pair(int s, int s2) { return s * kGridSub - s * (s - 1) / 2 + (s2 - s); }

// Geometry of the grid and its sublattices (device copy in the workspace).
struct GridGeom {
  int nx, ny, nz;        // bricks per period in x, y and layers in z
  int lz, pz;            // z slots (nz + 1: faces on the top plane) and padded z length (2 lz)
  int64_t nf;            // nx * ny * pz: points of one field
  double h[3];           // brick size
  double org[3];         // corner of brick (0, 0, 0)
  double zspan;          // zmax - zmin of the mesh
  double pos[kGridSub][3];   // point of each sublattice relative to its brick's origin
  int32_t ent[kGridSub];     // entity type of each sublattice (tetrahedra 0..5, faces 6..17)
  // touch[e][e'][o]: entity e of brick i and e' of brick i - o share a corner,
  // o = (ox + 1) + 3 (oy + 1) + 9 (oz + 1) with ox, oy, oz in {-1, 0, 1}
  uint8_t touch[kGridEnt][kGridEnt][27];
};

// Host side: the grid found in a mesh and the per-element maps the kernels use.
struct MeshTopology;
struct QuadRules;
struct GridHost {
  GridGeom g{};
  std::vector<int32_t> tet;    // per tetrahedron: slot x + nx (y + ny z) of its brick, type
  std::vector<int32_t> face;   // per surface-charge face: brick x, y, z (x = nx or y = ny on the far
                               // periodic wall, not wrapped), type
  std::vector<int32_t> half;   // per unknown: its surface-charge face slot for a half-SWG face, else -1
};

// Recognise a uniform Kuhn brick grid spanning the unit cell (every brick
// split along its (0,0,0)-(1,1,1) diagonal, at least two bricks per period)
// and fill G.  Returns "" or the reason the mesh is not such a grid.
std::string analyse_grid(const MeshTopology &t, const QuadRules &q, GridHost &G);

}  // namespace vie
