// Host analysis of a uniform Kuhn brick grid for the structured-grid far
// operator: grid spacing, the brick and type of every tetrahedron and
// surface-charge face, the sublattice points of the far product rules and the
// table of corner-sharing element pairs.
#include "grid.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "common.h"
#include "host.h"

namespace vie {

namespace {

// corner of a unit brick as a bit index x + 2 y + 4 z
inline int cbit(int x, int y, int z) { return x | (y << 1) | (z << 2); }
inline void cxyz(int b, int *c) {
  c[0] = b & 1;
  c[1] = (b >> 1) & 1;
  c[2] = (b >> 2) & 1;
}

// Distinct coordinates of the vertices along one axis, checked to be uniform.
std::string axis_grid(const std::vector<double> &v, double tol, double *org, double *h, int *n) {
  std::vector<double> s(v);
  std::sort(s.begin(), s.end());
  std::vector<double> u;
  for (double x : s)
    if (u.empty() || x - u.back() > tol) u.push_back(x);
  if (u.size() < 2) return "fewer than two grid planes";
  *org = u.front();
  *n = (int)u.size() - 1;
  *h = (u.back() - u.front()) / *n;
  for (size_t i = 0; i < u.size(); ++i)
    if (std::fabs(u[i] - (*org + i * *h)) > tol) return "grid planes are not evenly spaced";
  return "";
}

}  // namespace

std::string analyse_grid(const MeshTopology &t, const QuadRules &q, GridHost &G) {
  GridGeom &g = G.g;
  g = GridGeom{};
  if (t.nv == 0 || t.nt == 0) return "empty mesh";
  const double span = std::max({t.a, t.b, t.zmax - t.zmin});
  const double tol = 1e-9 * span;
  std::vector<double> ax[3];
  for (int d = 0; d < 3; ++d) {
    ax[d].resize(t.nv);
    for (int64_t i = 0; i < t.nv; ++i) ax[d][i] = t.verts[3 * i + d];
  }
  int n[3];
  for (int d = 0; d < 3; ++d) {
    std::string e = axis_grid(ax[d], tol, &g.org[d], &g.h[d], &n[d]);
    if (!e.empty()) return std::string("not a uniform grid in ") + "xyz"[d] + ": " + e;
  }
  if (std::fabs(n[0] * g.h[0] - t.a) > tol || std::fabs(n[1] * g.h[1] - t.b) > tol)
    return "the grid does not span the lattice periods";
  if (n[0] < 2 || n[1] < 2) return "fewer than two bricks per lattice period";
  g.nx = n[0];
  g.ny = n[1];
  g.nz = n[2];
  g.lz = g.nz + 1;
  g.pz = 2 * g.lz;
  g.nf = (int64_t)g.nx * g.ny * g.pz;
  g.zspan = t.zmax - t.zmin;

  // integer grid coordinates of every vertex
  std::vector<int32_t> iv(3 * t.nv);
  for (int64_t i = 0; i < t.nv; ++i)
    for (int d = 0; d < 3; ++d) {
      const double r = (t.verts[3 * i + d] - g.org[d]) / g.h[d];
      iv[3 * i + d] = (int32_t)std::lround(r);
      if (std::fabs(r - iv[3 * i + d]) * g.h[d] > tol) return "a vertex is off the grid";
    }

  // the six Kuhn tetrahedra of a brick: corners 000, e_p0, e_p0 + e_p1, 111
  // for each permutation p of the axes; their faces, shifted to the brick of
  // their lowest corner, give the twelve face types
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int tcorn[kGridTetTypes][4], tmask[kGridTetTypes];
  for (int p = 0; p < 6; ++p) {
    int c[3] = {0, 0, 0};
    tcorn[p][0] = 0;
    for (int k = 0; k < 3; ++k) {
      c[perms[p][k]] = 1;
      tcorn[p][k + 1] = cbit(c[0], c[1], c[2]);
    }
    tmask[p] = 0;
    for (int k = 0; k < 4; ++k) tmask[p] |= 1 << tcorn[p][k];
  }
  std::vector<int> fmasks;
  for (int p = 0; p < 6; ++p)
    for (int skip = 0; skip < 4; ++skip) {
      int lo[3] = {1, 1, 1}, cs[3][3], m = 0;
      for (int k = 0, j = 0; k < 4; ++k)
        if (k != skip) cxyz(tcorn[p][k], cs[j++]);
      for (int j = 0; j < 3; ++j)
        for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], cs[j][d]);
      for (int j = 0; j < 3; ++j) m |= 1 << cbit(cs[j][0] - lo[0], cs[j][1] - lo[1], cs[j][2] - lo[2]);
      if (std::find(fmasks.begin(), fmasks.end(), m) == fmasks.end()) fmasks.push_back(m);
    }
  std::sort(fmasks.begin(), fmasks.end());
  if ((int)fmasks.size() != kGridFaceTypes) return "internal: Kuhn face types";
  int fcorn[kGridFaceTypes][3];
  for (int f = 0; f < kGridFaceTypes; ++f)
    for (int b = 0, j = 0; b < 8; ++b)
      if (fmasks[f] >> b & 1) fcorn[f][j++] = b;

  // entity corner masks (tetrahedron types, then face types)
  int emask[kGridEnt];
  for (int e = 0; e < kGridTetTypes; ++e) emask[e] = tmask[e];
  for (int f = 0; f < kGridFaceTypes; ++f) emask[kGridTetTypes + f] = fmasks[f];

  // elements of the mesh: brick (lowest corner) and type
  auto locate = [&](const int32_t *vids, int nvert, int *brick, int *mask) {
    int lo[3] = {1 << 30, 1 << 30, 1 << 30};
    for (int k = 0; k < nvert; ++k)
      for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], iv[3 * vids[k] + d]);
    int m = 0;
    for (int k = 0; k < nvert; ++k) {
      int c[3];
      for (int d = 0; d < 3; ++d) c[d] = iv[3 * vids[k] + d] - lo[d];
      if (c[0] > 1 || c[1] > 1 || c[2] > 1) return false;
      m |= 1 << cbit(c[0], c[1], c[2]);
    }
    for (int d = 0; d < 3; ++d) brick[d] = lo[d];
    *mask = m;
    return true;
  };
  const int64_t nslot = (int64_t)g.nx * g.ny * g.nz;
  G.tet.assign(2 * t.nt, 0);
  std::vector<char> seen(nslot * kGridTetTypes, 0);
  for (int64_t e = 0; e < t.nt; ++e) {
    int br[3], m;
    if (!locate(&t.tets[4 * e], 4, br, &m)) return "a tetrahedron spans more than one brick";
    int type = -1;
    for (int p = 0; p < kGridTetTypes; ++p)
      if (tmask[p] == m) type = p;
    if (type < 0) return "a tetrahedron is not a Kuhn tetrahedron of its brick";
    if (br[0] >= g.nx || br[1] >= g.ny || br[2] >= g.nz) return "a tetrahedron lies outside the grid";
    const int64_t slot = br[0] + (int64_t)g.nx * (br[1] + (int64_t)g.ny * br[2]);
    if (seen[slot * kGridTetTypes + type]++) return "two tetrahedra share a brick and type";
    G.tet[2 * e] = (int32_t)slot;
    G.tet[2 * e + 1] = type;
  }
  const size_t nc = t.charged.size();
  G.face.assign(4 * std::max<size_t>(1, nc), 0);
  std::vector<char> fseen((int64_t)g.nx * g.ny * g.lz * kGridFaceTypes, 0);
  for (size_t i = 0; i < nc; ++i) {
    const int32_t f = t.charged[i];
    int br[3], m;
    if (!locate(&t.face_vid[3 * f], 3, br, &m)) return "a face spans more than one brick";
    int type = -1;
    for (int p = 0; p < kGridFaceTypes; ++p)
      if (fmasks[p] == m) type = p;
    if (type < 0) return "a face is not a face of the Kuhn split";
    if (br[0] > g.nx || br[1] > g.ny || br[2] > g.nz) return "a face lies outside the grid";
    const int64_t slot = br[0] % g.nx + (int64_t)g.nx * (br[1] % g.ny + (int64_t)g.ny * br[2]);
    if (fseen[slot * kGridFaceTypes + type]++) return "two surface-charge faces share a slot";
    for (int d = 0; d < 3; ++d) G.face[4 * i + d] = br[d];
    G.face[4 * i + 3] = type;
  }
  G.half.assign(std::max<int64_t>(1, t.N), -1);
  for (size_t i = 0; i < nc; ++i)
    if (t.tminus[t.charged[i]] < 0) G.half[t.charged[i]] = (int32_t)i;

  // sublattice points of the far rules, relative to the brick origin
  for (int p = 0; p < kGridTetTypes; ++p)
    for (int i = 0; i < 4; ++i) {
      const int s = 4 * p + i;
      for (int d = 0; d < 3; ++d) {
        double r = 0;
        for (int k = 0; k < 4; ++k) {
          int c[3];
          cxyz(tcorn[p][k], c);
          r += q.tet4[i][k] * c[d];
        }
        g.pos[s][d] = r * g.h[d];
      }
      g.ent[s] = p;
    }
  for (int f = 0; f < kGridFaceTypes; ++f)
    for (int i = 0; i < 3; ++i) {
      const int s = kGridTetSub + 3 * f + i;
      for (int d = 0; d < 3; ++d) {
        double r = 0;
        for (int k = 0; k < 3; ++k) {
          int c[3];
          cxyz(fcorn[f][k], c);
          r += q.tri3[i][k] * c[d];
        }
        g.pos[s][d] = r * g.h[d];
      }
      g.ent[s] = kGridTetTypes + f;
    }
  // corner sharing: e in brick i, e' in brick i - o share a corner when some
  // corner c of e and c' of e' have c' - c = o
  for (int e = 0; e < kGridEnt; ++e)
    for (int e2 = 0; e2 < kGridEnt; ++e2)
      for (int o = 0; o < 27; ++o) {
        const int od[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
        bool hit = false;
        for (int b = 0; b < 8 && !hit; ++b)
          for (int b2 = 0; b2 < 8 && !hit; ++b2) {
            if (!(emask[e] >> b & 1) || !(emask[e2] >> b2 & 1)) continue;
            int c[3], c2[3];
            cxyz(b, c);
            cxyz(b2, c2);
            hit = c2[0] - c[0] == od[0] && c2[1] - c[1] == od[1] && c2[2] - c[2] == od[2];
          }
        g.touch[e][e2][o] = hit ? 1 : 0;
      }
  return "";
}

}  // namespace vie
