// Host-side driver for the sanitizer test (tests/test_host_sanitize.py): runs
// the library's host C++ (mesh topology and validation, near-pair pattern,
// point location, quadrature rules, lattice-sum tables and their packing, the
// structured-grid analysis) on
// one mesh read from a binary file, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by g++ (no device code is involved).
//
// File layout (little endian): int64 nv, nt; int32 ndom; double a, b;
// double verts[3 nv]; int32 tets[4 nt]; int32 dom[nt].
// Prints: N, near-pattern entries, located points, and per illumination the
// number of significant images and modes and the packed table length.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "grid.h"
#include "host.h"

using namespace vie;

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t nv = 0, nt = 0;
  int32_t ndom = 0;
  double a = 0, b = 0;
  bool ok = std::fread(&nv, 8, 1, f) == 1 && std::fread(&nt, 8, 1, f) == 1 && std::fread(&ndom, 4, 1, f) == 1 &&
            std::fread(&a, 8, 1, f) == 1 && std::fread(&b, 8, 1, f) == 1;
  std::vector<double> verts(ok ? 3 * nv : 0);
  std::vector<int32_t> tets(ok ? 4 * nt : 0), dom(ok ? nt : 0);
  ok = ok && std::fread(verts.data(), 8, verts.size(), f) == verts.size() &&
       std::fread(tets.data(), 4, tets.size(), f) == tets.size() && std::fread(dom.data(), 4, dom.size(), f) == dom.size();
  std::fclose(f);
  if (!ok) return 2;

  MeshTopology t;
  std::string err = build_topology(t, verts.data(), nv, tets.data(), nt, dom.data(), ndom, a, b);
  if (!err.empty()) {
    std::printf("topology error: %s\n", err.c_str());
    return 3;
  }
  std::vector<int64_t> rowptr;
  std::vector<int32_t> cols;
  build_near_pattern(t, rowptr, cols);
  std::printf("N %lld nnz %lld colors %d\n", (long long)t.N, (long long)rowptr.back(), t.ncolors);

  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const int np = 2000;
  std::vector<double> pts(3 * np);
  for (int i = 0; i < np; ++i) {
    pts[3 * i] = U(rng) * a;
    pts[3 * i + 1] = U(rng) * b;
    pts[3 * i + 2] = t.zmin - 2.0 + U(rng) * (t.zmax - t.zmin + 4.0);
  }
  std::vector<int32_t> where(np);
  locate_points(t, pts.data(), np, where.data());
  int inside = 0;
  for (int32_t w : where) inside += w >= 0;
  std::printf("located %d of %d\n", inside, np);

  QuadRules q;
  build_quadrature(q);
  const double ill[3][3] = {{500.0, 0.0, 0.0}, {620.0, 0.6, 0.4}, {450.0, 1.1, 1.3}};
  for (const auto &il : ill) {
    PgfTable *tab = new PgfTable;
    double margin = 0;
    err = build_pgf_table(*tab, a, b, t.zmax - t.zmin, il[0], il[1], il[2], &margin);
    if (!err.empty()) {
      std::printf("table error: %s\n", err.c_str());
      delete tab;
      return 4;
    }
    std::vector<double> pack;
    pack_pgf_table(*tab, pack);
    int modes = 0;
    for (int i = 0; i < kPgfTerms; ++i) modes += tab->mode[i].deg >= 0;
    std::printf("table lambda %.0f: images %d modes %d packed %zu margin %.3f\n", il[0], tab->nimg, modes,
                pack.size(), margin);
    delete tab;
  }

  // structured-grid analysis: a uniform Kuhn grid or the reason it is not;
  // on a grid, the corner-sharing table is symmetric under swapping the two
  // elements and negating the offset, every element shares a corner with
  // itself, and every sublattice point lies in its brick
  GridHost G;
  err = analyse_grid(t, q, G);
  if (!err.empty()) {
    std::printf("grid none: %s\n", err.c_str());
    return 0;
  }
  for (int e = 0; e < kGridEnt; ++e) {
    if (!G.g.touch[e][e][13]) return 5;
    for (int e2 = 0; e2 < kGridEnt; ++e2)
      for (int o = 0; o < 27; ++o)
        if (G.g.touch[e][e2][o] != G.g.touch[e2][e][26 - o]) return 6;
  }
  for (int s = 0; s < kGridSub; ++s)
    for (int d = 0; d < 3; ++d)
      if (G.g.pos[s][d] < 0 || G.g.pos[s][d] > G.g.h[d]) return 7;
  int sharing = 0;
  for (int o = 0; o < 27; ++o) sharing += G.g.touch[0][0][o];
  std::printf("grid %d %d %d nf %lld faces %zu sharing %d\n", G.g.nx, G.g.ny, G.g.nz, (long long)G.g.nf,
              G.face.size() / 4, sharing);
  return 0;
}
