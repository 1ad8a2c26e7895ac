// SWG topology of a periodic tetrahedral unit cell (Sec. 2.1: one SWG unknown
// per face; Sec. 2.2: one unit cell with Bloch-periodic walls; Sec. 2.3:
// unknowns grouped by material domain).
//
// Readings (the paper leaves these open):
//  * faces on x = 0 / x = a (and y) are identified by translation into one
//    Bloch-periodic SWG; its T- is an in-cell tetrahedron plus a lattice shift;
//  * T+ is the lower tetrahedron index; structure-boundary faces are half-SWGs;
//  * a face's domain is the lower domain id of its tetrahedra; unknowns are
//    ordered by (domain, canonical vertex key) so each A_dd is contiguous;
//  * surface-charge faces: half-SWGs and faces between two domains;
//  * two elements touch under image (m, n) when the source shifted by
//    -(m a, n b) shares a vertex with the test element (integer test).
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <thread>
#include <unordered_map>

#include "host.h"

namespace vie {
namespace {

struct QKey {
  int64_t x, y, z;
  bool operator==(const QKey &o) const { return x == o.x && y == o.y && z == o.z; }
};
struct QKeyHash {
  size_t operator()(const QKey &k) const {
    uint64_t h = 1469598103934665603ull;
    for (int64_t v : {k.x, k.y, k.z}) {
      h ^= (uint64_t)v;
      h *= 1099511628211ull;
    }
    return (size_t)h;
  }
};

using FaceKey = std::array<int32_t, 7>;  // c0 < c1 < c2, rel offsets of v1, v2 to v0

struct FaceSlot {
  int32_t tet, k;
  int32_t vid[3];  // sorted by canonical id
  int32_t ox, oy;  // offset of the first vertex in this copy
};

}  // namespace

std::string build_topology(MeshTopology &t, const double *verts, int64_t nv, const int32_t *tets, int64_t nt,
                           const int32_t *tet_domain, int ndom, double a, double b) {
  if (nv <= 0 || nt <= 0 || ndom <= 0 || !(a > 0) || !(b > 0)) return "empty mesh or bad period";
  t = MeshTopology();
  t.a = a;
  t.b = b;
  t.nv = nv;
  t.nt = nt;
  t.ndom = ndom;
  t.verts.assign(verts, verts + 3 * nv);
  t.tets.assign(tets, tets + 4 * nt);
  t.dom.assign(tet_domain, tet_domain + nt);
  for (int64_t i = 0; i < 4 * nt; ++i)
    if (t.tets[i] < 0 || t.tets[i] >= nv) return "tetrahedron vertex id out of range";
  for (int64_t i = 0; i < nt; ++i)
    if (t.dom[i] < 0 || t.dom[i] >= ndom) return "domain id out of range";

  // ---- canonical vertices: a vertex on x = a (y = b) is the image of one on x = 0 (y = 0)
  const double tol = 1e-6 * std::max(a, b);
  t.offx.resize(nv);
  t.offy.resize(nv);
  std::vector<QKey> q(nv);
  t.zmin = 1e300;
  t.zmax = -1e300;
  for (int64_t i = 0; i < nv; ++i) {
    double x = verts[3 * i], y = verts[3 * i + 1], z = verts[3 * i + 2];
    if (x < -tol || x > a + tol || y < -tol || y > b + tol) return "vertex outside the unit cell";
    t.offx[i] = std::fabs(x - a) < tol ? 1 : 0;
    t.offy[i] = std::fabs(y - b) < tol ? 1 : 0;
    q[i] = QKey{(int64_t)std::llround((x - t.offx[i] * a) / tol), (int64_t)std::llround((y - t.offy[i] * b) / tol),
                (int64_t)std::llround(z / tol)};
    t.zmin = std::min(t.zmin, z);
    t.zmax = std::max(t.zmax, z);
  }
  std::unordered_map<QKey, int32_t, QKeyHash> rep;
  rep.reserve(nv * 2);
  for (int64_t i = 0; i < nv; ++i)
    if (t.offx[i] == 0 && t.offy[i] == 0) {
      if (!rep.emplace(q[i], (int32_t)i).second) return "duplicate vertex";
    }
  std::vector<int32_t> repv(nv);
  for (int64_t i = 0; i < nv; ++i) {
    auto it = rep.find(q[i]);
    if (it == rep.end()) return "vertex on a periodic wall has no partner on the opposite wall";
    repv[i] = it->second;
  }
  // canonical ids: rank of the representative's vertex id
  std::vector<int32_t> rank(nv, -1);
  int32_t nc = 0;
  for (int64_t i = 0; i < nv; ++i)
    if (t.offx[i] == 0 && t.offy[i] == 0) rank[i] = nc++;
  t.canon.resize(nv);
  for (int64_t i = 0; i < nv; ++i) t.canon[i] = rank[repv[i]];

  // ---- volumes, extent check
  t.vol.resize(nt);
  double scale3 = std::pow(std::max(a, b), 3);
  for (int64_t e = 0; e < nt; ++e) {
    const double *p[4];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < 4; ++k) {
      p[k] = &verts[3 * t.tets[4 * e + k]];
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], p[k][d]);
        hi[d] = std::max(hi[d], p[k][d]);
      }
    }
    double u[3], v[3], w[3];
    for (int d = 0; d < 3; ++d) {
      u[d] = p[1][d] - p[0][d];
      v[d] = p[2][d] - p[0][d];
      w[d] = p[3][d] - p[0][d];
    }
    double det = u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
                 u[2] * (v[0] * w[1] - v[1] * w[0]);
    if (std::fabs(det) <= 1e-12 * scale3) return "degenerate tetrahedron";
    t.vol[e] = std::fabs(det) / 6.0;
    if (hi[0] - lo[0] > 0.5 * a * (1 + 1e-9) || hi[1] - lo[1] > 0.5 * b * (1 + 1e-9))
      return "fewer than 2 cells per periodic direction";
    double diam = 0;
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j) {
        double s = 0;
        for (int d = 0; d < 3; ++d) s += (p[i][d] - p[j][d]) * (p[i][d] - p[j][d]);
        diam = std::max(diam, std::sqrt(s));
      }
    t.max_diam = std::max(t.max_diam, diam);
  }

  // ---- faces grouped by canonical key
  std::map<FaceKey, std::vector<FaceSlot>> groups;
  for (int64_t e = 0; e < nt; ++e)
    for (int k = 0; k < 4; ++k) {
      FaceSlot s;
      s.tet = (int32_t)e;
      s.k = k;
      int c = 0;
      for (int j = 0; j < 4; ++j)
        if (j != k) s.vid[c++] = t.tets[4 * e + j];
      std::sort(s.vid, s.vid + 3, [&](int32_t x, int32_t y) { return t.canon[x] < t.canon[y]; });
      s.ox = t.offx[s.vid[0]];
      s.oy = t.offy[s.vid[0]];
      FaceKey key = {t.canon[s.vid[0]],
                     t.canon[s.vid[1]],
                     t.canon[s.vid[2]],
                     t.offx[s.vid[1]] - s.ox,
                     t.offy[s.vid[1]] - s.oy,
                     t.offx[s.vid[2]] - s.ox,
                     t.offy[s.vid[2]] - s.oy};
      groups[key].push_back(s);
    }

  struct Rec {
    FaceKey key;
    int32_t fdom;
    FaceSlot p, m;
    bool full;
  };
  std::vector<Rec> recs;
  recs.reserve(groups.size());
  for (auto &kv : groups) {
    auto &v = kv.second;
    if (v.size() > 2) return "non-manifold face";
    std::sort(v.begin(), v.end(), [](const FaceSlot &x, const FaceSlot &y) { return x.tet < y.tet; });
    Rec r;
    r.key = kv.first;
    r.p = v[0];
    r.full = v.size() == 2;
    if (r.full) {
      r.m = v[1];
      r.fdom = std::min(t.dom[r.p.tet], t.dom[r.m.tet]);
    } else {
      // a lone face lying on a periodic wall means the mesh is not periodic
      for (int ax = 0; ax < 2; ++ax) {
        double L = ax == 0 ? a : b;
        bool lo = true, hi = true;
        for (int j = 0; j < 3; ++j) {
          double c = verts[3 * r.p.vid[j] + ax];
          lo = lo && std::fabs(c) < 1e-6 * L;
          hi = hi && std::fabs(c - L) < 1e-6 * L;
        }
        if (lo || hi) return "periodic wall face has no partner";
      }
      r.fdom = t.dom[r.p.tet];
    }
    recs.push_back(r);
  }
  std::sort(recs.begin(), recs.end(), [](const Rec &x, const Rec &y) {
    if (x.fdom != y.fdom) return x.fdom < y.fdom;
    return x.key < y.key;
  });
  const int64_t N = (int64_t)recs.size();
  t.N = N;
  t.face_vid.resize(3 * N);
  t.tplus.resize(N);
  t.tminus.resize(N);
  t.fdom.resize(N);
  t.freep.resize(N);
  t.freem.resize(N);
  t.shx.resize(N);
  t.shy.resize(N);
  t.area.resize(N);
  t.t2f.assign(4 * nt, TetFace{-1, 0, 0, 0});
  for (int64_t i = 0; i < N; ++i) {
    const Rec &r = recs[i];
    // face vertex ids as the face sits in T+, ordered by canonical id
    for (int j = 0; j < 3; ++j) t.face_vid[3 * i + j] = r.p.vid[j];
    t.tplus[i] = r.p.tet;
    t.fdom[i] = r.fdom;
    t.freep[i] = t.tets[4 * r.p.tet + r.p.k];
    const double *A = &verts[3 * t.face_vid[3 * i]], *B = &verts[3 * t.face_vid[3 * i + 1]],
                 *C = &verts[3 * t.face_vid[3 * i + 2]];
    double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, v[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double n0 = u[1] * v[2] - u[2] * v[1], n1 = u[2] * v[0] - u[0] * v[2], n2 = u[0] * v[1] - u[1] * v[0];
    t.area[i] = 0.5 * std::sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    t.t2f[4 * r.p.tet + r.p.k] = TetFace{(int32_t)i, 1, 0, 0};
    if (r.full) {
      t.tminus[i] = r.m.tet;
      t.freem[i] = t.tets[4 * r.m.tet + r.m.k];
      t.shx[i] = r.m.ox - r.p.ox;
      t.shy[i] = r.m.oy - r.p.oy;
      t.t2f[4 * r.m.tet + r.m.k] = TetFace{(int32_t)i, -1, t.shx[i], t.shy[i]};
    } else {
      t.tminus[i] = -1;
      t.freem[i] = -1;
      t.shx[i] = t.shy[i] = 0;
    }
    if (!r.full || t.dom[r.p.tet] != t.dom[r.m.tet]) t.charged.push_back((int32_t)i);
  }
  t.dstart.assign(ndom, 0);
  t.dend.assign(ndom, 0);
  for (int d = 0; d < ndom; ++d) {
    int64_t s = -1, e = -1;
    for (int64_t i = 0; i < N; ++i)
      if (t.fdom[i] == d) {
        if (s < 0) s = i;
        e = i + 1;
      }
    if (s >= 0) {
      t.dstart[d] = s;
      t.dend[d] = e;
    }
  }

  // ---- greedy colouring: tets sharing an unknown get different colours
  t.color.assign(nt, -1);
  for (int64_t e = 0; e < nt; ++e) {
    unsigned used = 0;
    for (int k = 0; k < 4; ++k) {
      int32_t f = t.t2f[4 * e + k].unknown;
      int32_t other = t.tplus[f] == e ? t.tminus[f] : t.tplus[f];
      if (other >= 0 && t.color[other] >= 0) used |= 1u << t.color[other];
    }
    int c = 0;
    while (used & (1u << c)) ++c;
    t.color[e] = c;
    t.ncolors = std::max(t.ncolors, c + 1);
  }
  t.color_tets.assign(t.ncolors, {});
  for (int64_t e = 0; e < nt; ++e) t.color_tets[t.color[e]].push_back((int32_t)e);

  // ---- touching tet pairs via the tets around each canonical vertex
  std::vector<std::vector<int32_t>> around(nc);
  for (int64_t e = 0; e < nt; ++e)
    for (int k = 0; k < 4; ++k) around[t.canon[t.tets[4 * e + k]]].push_back((int32_t)e);
  const int C = t.ncolors;
  t.near_t.assign(C * C, {});
  t.near_s.assign(C * C, {});
  t.near_mask.assign(C * C, {});
  std::vector<int32_t> cand;
  for (int64_t e = 0; e < nt; ++e) {
    cand.clear();
    for (int k = 0; k < 4; ++k)
      for (int32_t s : around[t.canon[t.tets[4 * e + k]]]) cand.push_back(s);
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    int32_t ct[4], ot[4];
    for (int k = 0; k < 4; ++k) {
      int32_t v = t.tets[4 * e + k];
      ct[k] = t.canon[v];
      ot[k] = (t.offx[v] + 2) | ((t.offy[v] + 2) << 4);
    }
    for (int32_t s : cand) {
      int32_t cs[4], os[4];
      for (int k = 0; k < 4; ++k) {
        int32_t v = t.tets[4 * s + k];
        cs[k] = t.canon[v];
        os[k] = (t.offx[v] + 2) | ((t.offy[v] + 2) << 4);
      }
      int mask = touching_mask(ct, ot, 4, cs, os, 4);
      if (!mask) continue;
      int g = t.color[e] * C + t.color[s];
      t.near_t[g].push_back((int32_t)e);
      t.near_s[g].push_back(s);
      t.near_mask[g].push_back(mask);
    }
  }

  // ---- touching (tet, surface-charge face) and (half-SWG face, tet) pairs:
  // the tets around the face's vertices (sharing a canonical vertex is
  // touching under some image)
  t.near_tf.assign(C, {});
  t.near_ft.assign(C, {});
  int32_t hidx = 0;
  for (size_t fi = 0; fi < t.charged.size(); ++fi) {
    const int32_t f = t.charged[fi];
    const bool half = t.tminus[f] < 0;
    cand.clear();
    for (int j = 0; j < 3; ++j)
      for (int32_t e : around[t.canon[t.face_vid[3 * f + j]]]) cand.push_back(e);
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    for (int32_t e : cand) {
      t.near_tf[t.color[e]].push_back(e);
      t.near_tf[t.color[e]].push_back((int32_t)fi);
      if (half) {
        t.near_ft[t.color[e]].push_back(hidx);
        t.near_ft[t.color[e]].push_back(e);
      }
    }
    if (half) ++hidx;
  }
  return "";
}

// Sparsity pattern of the entries that touching tetrahedron pairs reach:
// (m, n) with m a face of T, n a face of S, (T, S) touching under some
// lattice image (the self pair included).  Every singular or near-neighbour
// contribution of the fill (tet-tet, tet-face, face-tet, face-face) lands
// inside it, because a face touches a tetrahedron only if the face's own
// tetrahedron does.  Rows sorted, no duplicates.
void build_near_pattern(const MeshTopology &t, std::vector<int64_t> &rowptr, std::vector<int32_t> &cols) {
  const int64_t N = t.N;
  std::vector<int64_t> cnt(N + 1, 0);
  const size_t G = t.near_t.size();
  for (size_t g = 0; g < G; ++g)
    for (size_t i = 0; i < t.near_t[g].size(); ++i) {
      const int32_t T = t.near_t[g][i];
      for (int k = 0; k < 4; ++k) cnt[t.t2f[4 * T + k].unknown + 1] += 4;
    }
  for (int64_t m = 0; m < N; ++m) cnt[m + 1] += cnt[m];
  std::vector<int32_t> raw(cnt[N]);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (size_t g = 0; g < G; ++g)
    for (size_t i = 0; i < t.near_t[g].size(); ++i) {
      const int32_t T = t.near_t[g][i], S = t.near_s[g][i];
      for (int k = 0; k < 4; ++k) {
        const int32_t m = t.t2f[4 * T + k].unknown;
        for (int l = 0; l < 4; ++l) raw[pos[m]++] = t.t2f[4 * S + l].unknown;
      }
    }
  // sort and de-duplicate every row (rows split over host threads), then compact
  std::vector<int64_t> uniq(N, 0);
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int w = 0; w < nth; ++w)
    pool.emplace_back([&, w]() {
      for (int64_t m = w; m < N; m += nth) {
        auto b = raw.begin() + cnt[m], e = raw.begin() + cnt[m + 1];
        std::sort(b, e);
        uniq[m] = std::unique(b, e) - b;
      }
    });
  for (auto &th : pool) th.join();
  rowptr.assign(N + 1, 0);
  for (int64_t m = 0; m < N; ++m) rowptr[m + 1] = rowptr[m] + uniq[m];
  cols.resize(rowptr[N]);
  for (int64_t m = 0; m < N; ++m) std::copy(raw.begin() + cnt[m], raw.begin() + cnt[m] + uniq[m], cols.begin() + rowptr[m]);
}

// Tetrahedron holding each point: the lowest index among the tetrahedra
// whose barycentric coordinates of the point are all >= -1e-12, -1 if none.
// Candidates come from a uniform bin grid over the mesh's bounding box (bin
// edge about twice the mean tetrahedron edge); each tetrahedron is listed,
// in increasing order, in every bin its slightly padded bounding box meets.
void locate_points(const MeshTopology &t, const double *pts, int64_t n, int32_t *tet) {
  if (t.nt == 0) {
    std::fill(tet, tet + n, -1);
    return;
  }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < t.nv; ++v)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], t.verts[3 * v + d]);
      hi[d] = std::max(hi[d], t.verts[3 * v + d]);
    }
  double vol = 0;
  for (int64_t i = 0; i < t.nt; ++i) vol += t.vol[i];
  const double h = std::max(2.0 * std::cbrt(6.0 * vol / (double)t.nt), 1e-9);
  int nb[3];
  for (int d = 0; d < 3; ++d) nb[d] = (int)std::min<double>(512.0, std::floor((hi[d] - lo[d]) / h) + 1);
  auto bin_of = [&](int d, double x) { return std::max(0, std::min(nb[d] - 1, (int)std::floor((x - lo[d]) / h))); };
  const int64_t nbins = (int64_t)nb[0] * nb[1] * nb[2];
  std::vector<std::vector<int32_t>> bins(nbins);
  for (int64_t i = 0; i < t.nt; ++i) {
    double bl[3] = {1e300, 1e300, 1e300}, bh[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < 4; ++k)
      for (int d = 0; d < 3; ++d) {
        const double x = t.verts[3 * (int64_t)t.tets[4 * i + k] + d];
        bl[d] = std::min(bl[d], x);
        bh[d] = std::max(bh[d], x);
      }
    int b0[3], b1[3];
    for (int d = 0; d < 3; ++d) {
      const double pad = 1e-9 * (bh[d] - bl[d] + h);
      b0[d] = bin_of(d, bl[d] - pad);
      b1[d] = bin_of(d, bh[d] + pad);
    }
    for (int x = b0[0]; x <= b1[0]; ++x)
      for (int y = b0[1]; y <= b1[1]; ++y)
        for (int z = b0[2]; z <= b1[2]; ++z) bins[((int64_t)x * nb[1] + y) * nb[2] + z].push_back((int32_t)i);
  }
  for (int64_t p = 0; p < n; ++p) {
    const double *q = pts + 3 * p;
    tet[p] = -1;
    bool outside = false;
    for (int d = 0; d < 3; ++d) outside |= !(q[d] >= lo[d] - 1e-9 * h && q[d] <= hi[d] + 1e-9 * h);
    if (outside) continue;
    const auto &cand = bins[((int64_t)bin_of(0, q[0]) * nb[1] + bin_of(1, q[1])) * nb[2] + bin_of(2, q[2])];
    for (int32_t i : cand) {
      // barycentric coordinates: solve [v1-v0 v2-v0 v3-v0] l = q - v0 by Cramer's rule
      const double *v0 = &t.verts[3 * (int64_t)t.tets[4 * i]];
      double e[3][3], r[3];
      for (int k = 0; k < 3; ++k) {
        const double *vk = &t.verts[3 * (int64_t)t.tets[4 * i + k + 1]];
        for (int d = 0; d < 3; ++d) e[d][k] = vk[d] - v0[d];
      }
      for (int d = 0; d < 3; ++d) r[d] = q[d] - v0[d];
      auto det3 = [](const double m[3][3]) {
        return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
               m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
      };
      const double det = det3(e);
      double l[3], sum = 0;
      for (int k = 0; k < 3; ++k) {
        double m[3][3];
        for (int d = 0; d < 3; ++d)
          for (int c = 0; c < 3; ++c) m[d][c] = c == k ? r[d] : e[d][c];
        l[k] = det3(m) / det;
        sum += l[k];
      }
      if (l[0] >= -1e-12 && l[1] >= -1e-12 && l[2] >= -1e-12 && 1.0 - sum >= -1e-12) {
        tet[p] = i;
        break;
      }
    }
  }
}

}  // namespace vie
