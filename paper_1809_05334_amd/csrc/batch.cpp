// Fused solves of many independent unit cells (the batch entry points of
// include/vie.h): one fill launch per kernel family and colour pair for every
// cell, one block factorisation over every cell's domains, and GMRES with the
// Arnoldi steps of every cell in one launch sequence (optionally one captured
// HIP graph replayed per step).  Each cell keeps its own context and
// workspace; the batch holds only descriptor tables.  Per cell the arithmetic
// is that of the single-cell entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "context.h"

using namespace vie;

struct vie_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<vie_ctx *> cells;
  int precision = VIE_FP64;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  double *pin_res = nullptr;        // pinned: residual estimates / norms, one per cell
  int *pin_act = nullptr;           // pinned: Arnoldi-step flags, one per cell
  int pin_cap = 0;                  // cells the pinned buffers hold
  hipStream_t side = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_la = nullptr, ev_ts = nullptr;
  int graph = 1;                    // capture the fused Arnoldi step in a HIP graph
  hipGraphExec_t gexec = nullptr;
  int filled = 0, factored = 0;
  double t_fill = 0, t_factor = 0;
};

namespace {

int bfail(vie_batch *b, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (b) b->err = buf;
  return code;
}

#define BCK(expr)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return bfail(b, VIE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define BLAUNCHCK()                                                                                        \
  do {                                                                                                     \
    hipError_t e_ = hipGetLastError();                                                                     \
    if (e_ != hipSuccess) return bfail(b, VIE_EDEVICE, "kernel launch (line %d): %s", __LINE__, hipGetErrorString(e_)); \
  } while (0)

// a failure of one cell's context, reported on the batch
int cell_fail(vie_batch *b, int c, int rc) {
  return bfail(b, rc, "cell %d: %s", c, b->cells[c]->err.c_str());
}

// Bump allocator over the batch workspace: every table of one operation is
// built on the host, then uploaded in one copy.
struct Stage {
  std::vector<char> host;
  size_t add(const void *p, size_t n) {
    const size_t off = (host.size() + 255) & ~size_t(255);
    host.resize(off + n);
    if (n) std::memcpy(host.data() + off, p, n);
    return off;
  }
};

int upload(vie_batch *b, const Stage &st) {
  if (st.host.size() > b->ws_bytes)
    return bfail(b, VIE_ENOMEM, "batch workspace %zu bytes < %zu needed", b->ws_bytes, st.host.size());
  if (!st.host.empty()) BCK(hipMemcpyAsync(b->ws, st.host.data(), st.host.size(), hipMemcpyHostToDevice, b->stream));
  return VIE_OK;
}

void release_graph(vie_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
}

// ---------------------------------------------------------------- fill
// Segments of one fused launch for the cells that have work for it.
template <class S>
struct Launch {
  std::vector<S> segs;
  int blocks = 0;
  size_t lds = 0;
  void add(S s, int gx, int gy, size_t l) {
    if (gx <= 0 || gy <= 0) return;
    s.gx = gx;
    s.first = blocks;
    blocks += gx * gy;
    segs.push_back(s);
    lds = std::max(lds, l);
  }
};

}  // namespace

extern "C" {

int vie_batch_create(vie_batch **out, int device, void *hip_stream) {
  if (!out) return VIE_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return VIE_EDEVICE;
  vie_batch *b = new vie_batch();
  b->device = device;
  b->stream = (hipStream_t)hip_stream;
  BCK(hipSetDevice(device));
  BCK(hipEventCreate(&b->ev0));
  BCK(hipEventCreate(&b->ev1));
  BCK(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
  BCK(hipEventCreateWithFlags(&b->ev_la, hipEventDisableTiming));
  BCK(hipEventCreateWithFlags(&b->ev_ts, hipEventDisableTiming));
  *out = b;
  return VIE_OK;
}

int vie_batch_destroy(vie_batch *b) {
  if (!b) return VIE_OK;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  release_graph(b);
  if (b->pin_res) (void)hipHostFree(b->pin_res);
  if (b->pin_act) (void)hipHostFree(b->pin_act);
  if (b->side) {
    (void)hipStreamSynchronize(b->side);
    (void)hipStreamDestroy(b->side);
  }
  for (hipEvent_t e : {b->ev0, b->ev1, b->ev_la, b->ev_ts})
    if (e) (void)hipEventDestroy(e);
  delete b;
  return VIE_OK;
}

const char *vie_batch_last_error(const vie_batch *b) { return b ? b->err.c_str() : "null batch"; }

size_t vie_batch_workspace_bytes(int ncells) {
  if (ncells < 1) return 0;
  return (size_t)(4 << 20) + (size_t)ncells * (512 << 10);
}

int vie_batch_bind(vie_batch *b, vie_ctx *const *cells, int ncells, void *dev_ptr, size_t bytes) {
  if (!b) return VIE_EINVAL;
  if (!cells || ncells < 1) return bfail(b, VIE_EINVAL, "no cells");
  if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return bfail(b, VIE_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < vie_batch_workspace_bytes(ncells))
    return bfail(b, VIE_ENOMEM, "batch workspace %zu bytes < %zu", bytes, vie_batch_workspace_bytes(ncells));
  for (int c = 0; c < ncells; ++c) {
    vie_ctx *x = cells[c];
    if (!x || x->state < S_BOUND) return bfail(b, VIE_ESTATE, "cell %d has no bound workspace", c);
    if (x->device != b->device) return bfail(b, VIE_EINVAL, "cell %d is on another device", c);
    if (x->precision != cells[0]->precision) return bfail(b, VIE_EINVAL, "cells of mixed precisions");
    if (x->precision == VIE_GRID_FP64) return bfail(b, VIE_EINVAL, "cell %d uses the grid operator (not batched)", c);
    if (x->topo.ndom > kCellMaxDom) return bfail(b, VIE_EINVAL, "cell %d has more than %d domains", c, kCellMaxDom);
    for (int k = 0; k < c; ++k)
      if (cells[k] == x) return bfail(b, VIE_EINVAL, "cell %d repeats cell %d", c, k);
  }
  BCK(hipSetDevice(b->device));
  if (b->stream) BCK(hipStreamSynchronize(b->stream));
  release_graph(b);
  if (b->pin_cap < ncells) {
    if (b->pin_res) BCK(hipHostFree(b->pin_res));
    if (b->pin_act) BCK(hipHostFree(b->pin_act));
    b->pin_res = nullptr;
    b->pin_act = nullptr;
    BCK(hipHostMalloc((void **)&b->pin_res, 8 * (size_t)ncells, hipHostMallocDefault));
    BCK(hipHostMalloc((void **)&b->pin_act, 4 * (size_t)ncells, hipHostMallocDefault));
    b->pin_cap = ncells;
  }
  b->cells.assign(cells, cells + ncells);
  b->precision = cells[0]->precision;
  b->ws = (char *)dev_ptr;
  b->ws_bytes = bytes;
  b->filled = b->factored = 0;
  // every cell's work goes to the batch's stream from now on
  for (vie_ctx *x : b->cells) {
    if (x->stream != b->stream && x->stream) {
      hipError_t e = hipStreamSynchronize(x->stream);
      if (e != hipSuccess) return bfail(b, VIE_EDEVICE, "cell stream: %s", hipGetErrorString(e));
    }
    x->stream = b->stream;
  }
  return VIE_OK;
}

int vie_batch_set_option(vie_batch *b, int option, int value) {
  if (!b) return VIE_EINVAL;
  if (option == VIE_BATCH_GRAPH) {
    if (value != 0 && value != 1) return bfail(b, VIE_EINVAL, "graph: 0 or 1");
    if (value != b->graph) release_graph(b);
    b->graph = value;
    return VIE_OK;
  }
  return bfail(b, VIE_EINVAL, "unknown batch option %d", option);
}

// Sec. 2.1, Eq. 2 with g_p of Sec. 2.2, Eqs. 3-4, for every cell at its own
// (lambda, theta, phi) and permittivities: the lattice-sum tables of all cells
// fitted on host threads, then each fill kernel family launched once per
// colour pair (or colour) for all cells.
int vie_batch_fill(vie_batch *b, const double *lambda_nm, const double *theta, const double *phi,
                   const vie_c128 *const *eps_per_tet) {
  if (!b || b->cells.empty()) return b ? bfail(b, VIE_ESTATE, "no cells bound") : VIE_EINVAL;
  if (!lambda_nm || !theta || !phi || !eps_per_tet) return bfail(b, VIE_EINVAL, "null argument");
  BCK(hipSetDevice(b->device));
  const int nc = (int)b->cells.size();
  // host: the tables of every cell (each fit is itself spread over host threads)
  {
    std::vector<int> rc(nc, VIE_OK);
    const int nthr = std::max(1, std::min(nc, 4));
    std::vector<std::thread> th;
    for (int w = 0; w < nthr; ++w)
      th.emplace_back([&, w]() {
        for (int c = w; c < nc; c += nthr)
          rc[c] = fill_tables(b->cells[c], lambda_nm[c], theta[c], phi[c], eps_per_tet[c], b->precision);
      });
    for (auto &t : th) t.join();
    for (int c = 0; c < nc; ++c)
      if (rc[c]) return cell_fail(b, c, rc[c]);
  }
  BCK(hipEventRecord(b->ev0, b->stream));
  for (int c = 0; c < nc; ++c)
    if (int rc = fill_upload(b->cells[c])) return cell_fail(b, c, rc);
  // the fused launches: segment tables for every launch in one upload
  Stage st;
  struct Rec {
    size_t off;
    int nseg, blocks;
    size_t lds;
    int kind;
  };
  std::vector<Rec> recs;
  int maxC = 0;
  for (vie_ctx *x : b->cells) maxC = std::max(maxC, x->topo.ncolors);
  enum { K_FAR, K_FAR_REV, K_NEAR, K_TF, K_TFN, K_FT, K_FTN, K_FF };
  auto put = [&](const auto &L, int kind) {
    if (L.segs.empty()) return;
    recs.push_back({st.add(L.segs.data(), sizeof(L.segs[0]) * L.segs.size()), (int)L.segs.size(), L.blocks, L.lds,
                    kind});
  };
  auto P = [&](vie_ctx *x) {
    struct C {
      const double *pk;
      int pkl;
      const QuadRules *qr;
      const TetGeom *tg;
      const TetFace *t2f;
      const dz *alpha, *gsrc, *kappa, *inveps, *sigma;
      const FaceGeom *fg;
      const int32_t *colors, *half;
      ZOut zo, zt;
    } c;
    const Layout &L = x->L;
    c.pk = x->ptr<double>(L.pack);
    c.pkl = x->packlen;
    c.qr = x->ptr<QuadRules>(L.quad);
    c.tg = x->ptr<TetGeom>(L.tg);
    c.t2f = x->ptr<TetFace>(L.t2f);
    c.alpha = x->ptr<dz>(L.alpha);
    c.gsrc = x->ptr<dz>(L.gsrc);
    c.kappa = x->ptr<dz>(L.kappa);
    c.inveps = x->ptr<dz>(L.inveps);
    c.sigma = x->ptr<dz>(L.sigma);
    c.fg = x->ptr<FaceGeom>(L.fg);
    c.colors = x->ptr<int32_t>(L.colors);
    c.half = x->ptr<int32_t>(L.half);
    c.zo = zout(x);
    c.zt = zout_staging(x);
    return c;
  };
  // far tet pairs, per colour pair (ct, cs)
  for (int ct = 0; ct < maxC; ++ct)
    for (int cs = 0; cs < maxC; ++cs) {
      Launch<FarSeg> plain, rev;
      for (vie_ctx *x : b->cells) {
        const int C = x->topo.ncolors;
        if (ct >= C || cs >= C || (x->fill_sym && cs < ct)) continue;
        const auto c = P(x);
        const int nT = x->color_off[ct + 1] - x->color_off[ct], nS = x->color_off[cs + 1] - x->color_off[cs];
        FarSeg s{c.pk, c.pkl, c.qr, c.tg, c.t2f, c.colors + x->color_off[ct], nT, c.colors + x->color_off[cs], nS,
                 c.alpha, c.gsrc, c.kappa, x->fill_k0sq9, c.zo, c.zt, !x->fill_sym ? 0 : (ct == cs ? 2 : 1), 0, 0};
        if (x->fill_sym && x->fill_rev) rev.add(s, (int)nblk(nS, 64), (int)nblk(nT, 4), x->fill_lds + kFarRevLds);
        else plain.add(s, (int)nblk(nS, 64), (int)nblk(nT, 4), x->fill_lds);
      }
      put(plain, K_FAR);
      put(rev, K_FAR_REV);
    }
  // touching tet pairs, per colour pair
  for (int ct = 0; ct < maxC; ++ct)
    for (int cs = 0; cs < maxC; ++cs) {
      Launch<NearSeg> L;
      for (vie_ctx *x : b->cells) {
        const int C = x->topo.ncolors;
        if (ct >= C || cs >= C) continue;
        const int g = ct * C + cs;
        const int np = x->near_off[g + 1] - x->near_off[g];
        if (!np) continue;
        const auto c = P(x);
        NearSeg s{c.pk, c.pkl, c.qr, c.tg, c.t2f, x->ptr<int32_t>(x->L.near_t) + x->near_off[g],
                  x->ptr<int32_t>(x->L.near_s) + x->near_off[g], x->ptr<int32_t>(x->L.near_m) + x->near_off[g], np,
                  c.alpha, c.gsrc, c.kappa, c.inveps, x->fill_k0sq9, c.zo, 0, 0};
        L.add(s, (int)nblk(16 * (int64_t)np, 256), 1, x->fill_lds);
      }
      put(L, K_NEAR);
    }
  // face pairs: per test colour the far and touching (tet, face) pairs, per
  // source colour the (half-SWG face, tet) pairs, then the face-face pairs
  for (int ct = 0; ct < maxC; ++ct) {
    Launch<TetFaceSeg> tf;
    Launch<TetFaceNearSeg> tfn;
    for (vie_ctx *x : b->cells) {
      if (!x->nface || ct >= x->topo.ncolors) continue;
      const auto c = P(x);
      const int nT = x->color_off[ct + 1] - x->color_off[ct];
      TetFaceSeg s{c.pk, c.pkl, c.qr, c.tg, c.t2f, c.colors + x->color_off[ct], nT, c.fg, x->nface, c.alpha,
                   c.sigma, c.gsrc, c.kappa, c.zo, c.zt, x->fill_sym_face ? (x->fill_rev ? 2 : 1) : 0, 0, 0};
      tf.add(s, (int)nblk(x->nface, 64), (int)nblk(nT, 4), x->fill_lds);
      const int np = x->tf_off[ct + 1] - x->tf_off[ct];
      if (np) {
        TetFaceNearSeg n{c.pk, c.pkl, c.qr, c.tg, c.t2f,
                         (const int32_t *)x->ptr<int32_t>(x->L.near_tf) + 2 * (int64_t)x->tf_off[ct], np, c.fg,
                         c.alpha, c.sigma, c.zo, 0, 0};
        tfn.add(n, (int)nblk(np, 256), 1, x->fill_lds);
      }
    }
    put(tf, K_TF);
    put(tfn, K_TFN);
  }
  for (int cs = 0; cs < maxC; ++cs) {
    Launch<FaceTetSeg> ft;
    Launch<FaceTetNearSeg> ftn;
    for (vie_ctx *x : b->cells) {
      if (!x->nface || !x->nhalf || cs >= x->topo.ncolors) continue;
      const auto c = P(x);
      const int nS = x->color_off[cs + 1] - x->color_off[cs];
      if (!x->fill_sym_face) {
        FaceTetSeg s{c.pk, c.pkl, c.qr, c.fg, c.half, x->nhalf, c.tg, c.t2f, c.colors + x->color_off[cs], nS,
                     c.gsrc, c.kappa, c.zo, 0, 0};
        ft.add(s, (int)nblk(nS, 64), (int)nblk(x->nhalf, 4), x->fill_lds);
      }
      const int np = x->ft_off[cs + 1] - x->ft_off[cs];
      if (np) {
        FaceTetNearSeg n{c.pk, c.pkl, c.qr, c.fg, c.half, c.tg, c.t2f,
                         (const int32_t *)x->ptr<int32_t>(x->L.near_ft) + 2 * (int64_t)x->ft_off[cs], np, c.gsrc,
                         c.kappa, c.zo, 0, 0};
        ftn.add(n, (int)nblk(np, 256), 1, x->fill_lds);
      }
    }
    put(ft, K_FT);
    put(ftn, K_FTN);
  }
  {
    Launch<FaceFaceSeg> ff;
    for (vie_ctx *x : b->cells) {
      if (!x->nface || !x->nhalf) continue;
      const auto c = P(x);
      FaceFaceSeg s{c.pk, c.pkl, c.qr, c.fg, c.half, x->nhalf, x->nface, c.sigma, c.zo, 0, 0};
      ff.add(s, (int)nblk(x->nface, 64), (int)nblk(x->nhalf, 4), x->fill_lds);
    }
    put(ff, K_FF);
  }
  if (int rc = upload(b, st)) return rc;
  for (const Rec &r : recs) {
    const void *p = b->ws + r.off;
    const dim3 g(r.blocks), t(256);
    switch (r.kind) {
      case K_FAR: hipLaunchKernelGGL(k_tt_far_seg, g, t, r.lds, b->stream, (const FarSeg *)p, r.nseg); break;
      case K_FAR_REV: hipLaunchKernelGGL(k_tt_far_rev_seg, g, t, r.lds, b->stream, (const FarSeg *)p, r.nseg); break;
      case K_NEAR: hipLaunchKernelGGL(k_tt_near_seg, g, t, r.lds, b->stream, (const NearSeg *)p, r.nseg); break;
      case K_TF: hipLaunchKernelGGL(k_tet_face_seg, g, t, r.lds, b->stream, (const TetFaceSeg *)p, r.nseg); break;
      case K_TFN:
        hipLaunchKernelGGL(k_tet_face_near_seg, g, t, r.lds, b->stream, (const TetFaceNearSeg *)p, r.nseg);
        break;
      case K_FT: hipLaunchKernelGGL(k_face_tet_seg, g, t, r.lds, b->stream, (const FaceTetSeg *)p, r.nseg); break;
      case K_FTN:
        hipLaunchKernelGGL(k_face_tet_near_seg, g, t, r.lds, b->stream, (const FaceTetNearSeg *)p, r.nseg);
        break;
      case K_FF: hipLaunchKernelGGL(k_face_face_seg, g, t, r.lds, b->stream, (const FaceFaceSeg *)p, r.nseg); break;
    }
    BLAUNCHCK();
  }
  // (the segment tables must outlive the launches: the host copy is staged
  // before they run, and the next upload comes after a synchronisation)
  for (int c = 0; c < nc; ++c) {
    vie_ctx *x = b->cells[c];
    x->fstats.far_launches = 0;
    if (int rc = fill_finish(x, false)) return cell_fail(b, c, rc);
  }
  BCK(hipEventRecord(b->ev1, b->stream));
  BCK(hipEventSynchronize(b->ev1));
  float ms = 0;
  BCK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  b->t_fill = ms;
  for (vie_ctx *x : b->cells) {
    x->t_fill = ms;
    x->fstats.t_fill_ms = ms;
  }
  b->filled = 1;
  b->factored = 0;
  release_graph(b);
  return VIE_OK;
}

// Sec. 2.3, Eq. 6 for every cell: one panel loop over all cells' domains.
int vie_batch_factor(vie_batch *b) {
  if (!b || !b->filled) return b ? bfail(b, VIE_ESTATE, "vie_batch_factor before vie_batch_fill") : VIE_EINVAL;
  BCK(hipSetDevice(b->device));
  const int nc = (int)b->cells.size();
  std::vector<std::vector<LuDom>> per(nc);
  std::vector<LuDom> all;
  BCK(hipEventRecord(b->ev0, b->stream));
  for (int c = 0; c < nc; ++c) {
    if (int rc = factor_prepare(b->cells[c], per[c])) return cell_fail(b, c, rc);
    all.insert(all.end(), per[c].begin(), per[c].end());
  }
  vie_ctx *x0 = b->cells[0];
  if (int rc = factor_panels(x0, all, fp32_factors(x0), 0, b->stream, b->side, b->ev_la, b->ev_ts))
    return cell_fail(b, 0, rc);
  for (int c = 0; c < nc; ++c)
    if (int rc = factor_finish(b->cells[c], per[c])) return cell_fail(b, c, rc);
  BCK(hipEventRecord(b->ev1, b->stream));
  BCK(hipEventSynchronize(b->ev1));
  float ms = 0;
  BCK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  b->t_factor = ms;
  for (vie_ctx *x : b->cells) x->t_factor = ms;
  b->factored = 1;
  release_graph(b);
  return VIE_OK;
}

}  // extern "C"

namespace {

// The fused Arnoldi step's tables: the cells' descriptors, the block prefix
// of each grid shape, the step flags and residual estimates, and the merged
// plan of the triangular solves (every cell's domains per step).
struct StepPlan {
  size_t kc, pre_elem, pre_mv, pre_dots, pre_red, pre_norm, act, res, trsv;
  int tot_elem, tot_mv, tot_dots, tot_red, tot_norm;
  struct TStep {
    size_t off;
    int ndom, lower, blocks, chain, zend;   // reduction items first, solution items up to zend
  };
  std::vector<TStep> tsteps;
  bool precond = true;
};

int build_step_plan(vie_batch *b, StepPlan &sp) {
  const int nc = (int)b->cells.size();
  Stage st;
  std::vector<KryCell> kc(nc);
  std::vector<int> pe(nc + 1, 0), pm(nc + 1, 0), pd(nc + 1, 0), pr(nc + 1, 0), pn(nc + 1, 0);
  sp.precond = false;
  for (int c = 0; c < nc; ++c) {
    vie_ctx *x = b->cells[c];
    const Layout &L = x->L;
    const Layout::Kry &K = L.K[0];
    const int64_t N = x->topo.N;
    KryCell &k = kc[c];
    std::memset(&k, 0, sizeof(k));
    const ZOut zo = zout(x);
    k.Z = zo.Z;
    k.Zs = zo.Zs;
    k.rowptr = zo.rowptr;
    k.cols = zo.cols;
    k.vals = zo.vals;
    k.ld = L.ld;
    k.N = N;
    k.ldv = L.ldv;
    k.V = x->ptr<dz>(K.V);
    k.jd = x->ptr<int>(K.jd);
    k.vin = x->ptr<dz>(K.vin);
    k.z = x->ptr<dz>(K.vz);
    k.w = x->ptr<dz>(K.vw);
    k.tmp = x->ptr<dz>(K.vt);
    k.H = x->ptr<dz>(K.H);
    k.ldh = L.restart + 2;
    k.cs = x->ptr<double>(K.cs);
    k.sn = x->ptr<dz>(K.sn);
    k.g = x->ptr<dz>(K.g);
    k.y = x->ptr<dz>(K.y);
    k.rhist = x->ptr<double>(K.rhist);
    k.scal = x->ptr<double>(K.scal);
    k.dpart = x->ptr<dz>(K.dpart);
    k.npart = x->ptr<double>(K.npart);
    k.nred = (int)std::min<int64_t>(kRedBlocks, nblk(N, 256));
    k.perm = x->ptr<int32_t>(L.perm);
    k.ndom = x->topo.ndom;
    for (int d = 0; d < x->topo.ndom; ++d) k.dstart[d] = x->topo.dstart[d];
    k.precond = x->precond;
    k.rpw = x->mv_rpw;
    sp.precond = sp.precond || x->precond == 0;
    const int ngrp = (int)nblk(L.restart + 1, 8);
    pe[c + 1] = pe[c] + (int)nblk(N, 256);
    pm[c + 1] = pm[c] + (int)nblk(N, 4 * k.rpw);
    pd[c + 1] = pd[c] + k.nred * ngrp;
    pr[c + 1] = pr[c] + (int)nblk(L.restart + 1, 128);
    pn[c + 1] = pn[c] + k.nred;
  }
  sp.kc = st.add(kc.data(), sizeof(KryCell) * nc);
  sp.pre_elem = st.add(pe.data(), 4 * (nc + 1));
  sp.pre_mv = st.add(pm.data(), 4 * (nc + 1));
  sp.pre_dots = st.add(pd.data(), 4 * (nc + 1));
  sp.pre_red = st.add(pr.data(), 4 * (nc + 1));
  sp.pre_norm = st.add(pn.data(), 4 * (nc + 1));
  sp.tot_elem = pe[nc];
  sp.tot_mv = pm[nc];
  sp.tot_dots = pd[nc];
  sp.tot_red = pr[nc];
  sp.tot_norm = pn[nc];
  std::vector<int> zeros(nc, 0);
  sp.act = st.add(zeros.data(), 4 * nc);
  std::vector<double> zd(nc, 0.0);
  sp.res = st.add(zd.data(), 8 * nc);
  // merged triangular-solve plan: every cell's per-step domains (the same
  // entries as its own plan with one vector), step k of a sweep holding each
  // domain's step k; a domain's closing entry comes right after its last step
  sp.tsteps.clear();
  if (sp.precond) {
    std::vector<std::vector<TrsvDom>> steps[2];
    for (int c = 0; c < nc; ++c) {
      vie_ctx *x = b->cells[c];
      if (x->precond) continue;
      const Layout::Kry &K = x->L.K[0];
      dz *out = x->ptr<dz>(K.vz), *s1 = x->ptr<dz>(K.vt), *s2 = x->ptr<dz>(K.vu);
      const int save_kc = x->trsv_kc;
      x->trsv_kc = kTrsvSumCols;   // the fused kernel's work-item width
      const std::vector<TrsvStep> plan = trsv_plan(x, 1, &out, &s1, &s2);
      x->trsv_kc = save_kc;
      // each entry to its step in the merged plan: a regular entry of block bk
      // at the sweep's step for bk, a domain's closing entry right after its
      // own last step (its partial products are not touched in between)
      for (const TrsvStep &s : plan) {
        const int sw = s.lower ? 0 : 1;
        for (int i = 0; i < s.ndom; ++i) {
          TrsvDom D = s.d[i];
          D.active = (const int *)(b->ws + sp.act) + c;
          const int nbk = (D.n + kTrsvNB - 1) / kTrsvNB, bk = D.nb0 / kTrsvNB;
          const int k = D.nm == 0 ? nbk : (s.lower ? bk : nbk - 1 - bk);
          if ((int)steps[sw].size() <= k) steps[sw].resize(k + 1);
          steps[sw][k].push_back(D);
        }
      }
    }
    for (int sw = 0; sw < 2; ++sw)
      for (auto &v : steps[sw]) {
        if (v.empty()) continue;
        int total = 0, zend = 0;
        const int chain = trsv_number_items(v.data(), (int)v.size(), &zend, &total);
        sp.tsteps.push_back(
            {st.add(v.data(), sizeof(TrsvDom) * v.size()), (int)v.size(), sw == 0 ? 1 : 0, total, chain, zend});
      }
  }
  return upload(b, st);
}

// One fused Arnoldi step of every cell whose flag is set (Sec. 3 GMRES with
// the block preconditioner of Eq. 6 on the right).
int issue_step(vie_batch *b, const StepPlan &sp) {
  const int nc = (int)b->cells.size();
  const KryCell *kc = (const KryCell *)(b->ws + sp.kc);
  const int *act = (const int *)(b->ws + sp.act);
  auto pre = [&](size_t off) { return (const int *)(b->ws + off); };
  const dim3 t256(256);
  hipLaunchKernelGGL(k_b_arn_begin, dim3(sp.tot_elem), t256, 0, b->stream, kc, pre(sp.pre_elem), nc, act);
  if (sp.precond) {
    hipLaunchKernelGGL(k_b_permute, dim3(sp.tot_elem), t256, 0, b->stream, kc, pre(sp.pre_elem), nc, act);
    const bool f32 = b->precision == VIE_MIXED_FP32;
    for (const auto &s : sp.tsteps) {
      const TrsvDom *d = (const TrsvDom *)(b->ws + s.off);
      if (f32)
        hipLaunchKernelGGL(k_trsv_stepd_c, dim3(s.blocks), dim3(1024), 0, b->stream, d, s.ndom, s.lower, s.chain,
                           s.zend);
      else
        hipLaunchKernelGGL(k_trsv_stepd_z, dim3(s.blocks), dim3(1024), 0, b->stream, d, s.ndom, s.lower, s.chain,
                           s.zend);
    }
  }
  hipLaunchKernelGGL(k_b_matvec, dim3(sp.tot_mv), t256, 0, b->stream, kc, pre(sp.pre_mv), nc, act);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_b_dots_j, dim3(sp.tot_dots), t256, 0, b->stream, kc, pre(sp.pre_dots), nc, act);
    hipLaunchKernelGGL(k_b_dots_reduce_j, dim3(sp.tot_red), dim3(128), 0, b->stream, kc, pre(sp.pre_red), nc, act,
                       pass);
    hipLaunchKernelGGL(k_b_update_j, dim3(sp.tot_elem), t256, 0, b->stream, kc, pre(sp.pre_elem), nc, act);
  }
  hipLaunchKernelGGL(k_b_norm2, dim3(sp.tot_norm), t256, 0, b->stream, kc, pre(sp.pre_norm), nc, act);
  hipLaunchKernelGGL(k_b_norm_givens, dim3(nblk(nc, 64)), dim3(64), 0, b->stream, kc, nc, act);
  hipLaunchKernelGGL(k_b_scale_j, dim3(sp.tot_elem), t256, 0, b->stream, kc, pre(sp.pre_elem), nc, act);
  hipLaunchKernelGGL(k_b_jinc, dim3(nblk(nc, 64)), dim3(64), 0, b->stream, kc, nc, act, (double *)(b->ws + sp.res));
  BLAUNCHCK();
  return VIE_OK;
}

struct CellGmres {
  int pol = 0;
  double bnorm = 0, beta = 0, true_rel = 1;
  int iters = 0, restarts = 0, jdone = 0;
  bool converged = false, done = false, in_cycle = false, est_ok = false, stop = false;
};

}  // namespace

extern "C" {

int vie_batch_solve(vie_batch *b, const int *polarisation, double tol, int max_iter, int restart,
                    vie_solve_info *info) {
  if (!b || !b->factored) return b ? bfail(b, VIE_ESTATE, "vie_batch_solve before vie_batch_factor") : VIE_EINVAL;
  if (!polarisation || !(tol > 0) || max_iter < 1) return bfail(b, VIE_EINVAL, "bad arguments");
  BCK(hipSetDevice(b->device));
  const int nc = (int)b->cells.size();
  for (int c = 0; c < nc; ++c) {
    vie_ctx *x = b->cells[c];
    if (polarisation[c] != VIE_TE && polarisation[c] != VIE_TM) return bfail(b, VIE_EINVAL, "bad polarisation");
    if (x->precond == 2) return bfail(b, VIE_EINVAL, "cell %d: the point-Jacobi preconditioner is not batched", c);
    if (restart < 1 || restart > x->L.restart) return bfail(b, VIE_EINVAL, "restart exceeds cell %d's workspace", c);
  }
  BCK(hipStreamSynchronize(b->stream));   // the previous solve's tables are no longer read
  StepPlan sp;
  if (int rc = build_step_plan(b, sp)) return rc;
  release_graph(b);
  std::vector<CellGmres> P(nc);
  BCK(hipEventRecord(b->ev0, b->stream));
  // start: b, x = 0, r = b, ||b|| per cell
  for (int c = 0; c < nc; ++c) {
    vie_ctx *x = b->cells[c];
    const Layout::Kry &K = x->L.K[0];
    const int64_t N = x->topo.N;
    P[c].pol = polarisation[c];
    x->hist[0].clear();
    x->sol_k[0] = x->sol_k[1] = -1;
    launch_rhs(x, P[c].pol, x->ptr<dz>(K.vb));
    hipLaunchKernelGGL(k_zero, dim3(nblk(N, 256)), dim3(256), 0, b->stream, x->ptr<dz>(K.vx), N);
    hipLaunchKernelGGL(k_copy, dim3(nblk(N, 256)), dim3(256), 0, b->stream, x->ptr<dz>(K.vr),
                       (const dz *)x->ptr<dz>(K.vb), N);
    BLAUNCHCK();
    if (int rc = norm_to(x, 0, x->ptr<dz>(K.vr), N, x->ptr<double>(K.scal) + 0)) return cell_fail(b, c, rc);
    BCK(hipMemcpyAsync(b->pin_res + c, x->ptr<double>(K.scal) + 0, 8, hipMemcpyDeviceToHost, b->stream));
    BCK(hipMemcpyAsync(x->ptr<double>(K.scal) + 1, x->ptr<double>(K.scal) + 0, 8, hipMemcpyDeviceToDevice,
                       b->stream));
  }
  BCK(hipStreamSynchronize(b->stream));
  for (int c = 0; c < nc; ++c) {
    P[c].bnorm = P[c].beta = b->pin_res[c];
    if (!(P[c].bnorm > 0)) return bfail(b, VIE_EINVAL, "cell %d: zero right-hand side", c);
  }
  int *act_h = b->pin_act;
  int *act_d = (int *)(b->ws + sp.act);
  std::vector<int> act_prev(nc, -1);
  while (true) {
    // cycle starts: V_0 = r / beta, g = beta e_1, j = 0
    bool any = false;
    for (int c = 0; c < nc; ++c) {
      CellGmres &p = P[c];
      if (p.done) {
        act_h[c] = 0;
        continue;
      }
      if (!p.in_cycle) {
        vie_ctx *x = b->cells[c];
        const Layout::Kry &K = x->L.K[0];
        const int64_t N = x->topo.N;
        hipLaunchKernelGGL(k_scale, dim3(nblk(N, 256)), dim3(256), 0, b->stream, (const dz *)x->ptr<dz>(K.vr),
                           (const double *)(x->ptr<double>(K.scal) + 1), x->ptr<dz>(K.V), N);
        hipLaunchKernelGGL(k_ginit, dim3(1), dim3(256), 0, b->stream, x->ptr<dz>(K.g), restart + 1,
                           (const double *)(x->ptr<double>(K.scal) + 1));
        hipLaunchKernelGGL(k_jset, dim3(1), dim3(1), 0, b->stream, x->ptr<int>(K.jd), 0);
        BLAUNCHCK();
        p.in_cycle = true;
        p.jdone = 0;
        p.est_ok = p.stop = false;
      }
      act_h[c] = 1;
      any = true;
    }
    if (!any) break;
    bool changed = false;
    for (int c = 0; c < nc; ++c) changed = changed || act_h[c] != act_prev[c];
    if (changed) {
      BCK(hipMemcpyAsync(act_d, act_h, 4 * (size_t)nc, hipMemcpyHostToDevice, b->stream));
      for (int c = 0; c < nc; ++c) act_prev[c] = act_h[c];
    }
    // one fused Arnoldi step of every running cell (a captured graph replayed
    // per step in graph mode; the flags and j live in device memory)
    if (b->graph && b->stream) {
      if (!b->gexec) {
        hipGraph_t g = nullptr;
        BCK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        int rc = issue_step(b, sp);
        hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (rc) {
          if (g) (void)hipGraphDestroy(g);
          return rc;
        }
        if (e != hipSuccess) return bfail(b, VIE_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return bfail(b, VIE_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
      }
      BCK(hipGraphLaunch(b->gexec, b->stream));
    } else if (int rc = issue_step(b, sp)) {
      return rc;
    }
    BCK(hipMemcpyAsync(b->pin_res, b->ws + sp.res, 8 * (size_t)nc, hipMemcpyDeviceToHost, b->stream));
    BCK(hipStreamSynchronize(b->stream));
    // the decisions of the single-cell solver, per cell
    std::vector<int> ending;
    for (int c = 0; c < nc; ++c) {
      if (!act_h[c]) continue;
      CellGmres &p = P[c];
      const double res = b->pin_res[c];
      ++p.iters;
      ++p.jdone;
      b->cells[c]->hist[0].push_back(res / p.bnorm);
      if (res / p.bnorm <= tol) p.est_ok = p.stop = true;
      else if (p.iters >= max_iter) p.stop = true;
      if (p.stop || p.jdone >= restart) ending.push_back(c);
    }
    if (ending.empty()) continue;
    // cycle ends: x += M^-1 V y, r = b - Z x, beta = ||r|| (per cell)
    for (int c : ending) {
      vie_ctx *x = b->cells[c];
      const Layout &L = x->L;
      const Layout::Kry &K = L.K[0];
      const int64_t N = x->topo.N;
      dz *w = x->ptr<dz>(K.vw), *u = x->ptr<dz>(K.vu), *tv = x->ptr<dz>(K.vt), *zv = x->ptr<dz>(K.vz);
      hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(1), 0, b->stream, (const dz *)x->ptr<dz>(K.H), L.restart + 2,
                         P[c].jdone, (const dz *)x->ptr<dz>(K.g), x->ptr<dz>(K.y));
      hipLaunchKernelGGL(k_combine, dim3(nblk(N, 256)), dim3(256), 0, b->stream, (const dz *)x->ptr<dz>(K.V), L.ldv,
                         P[c].jdone, (const dz *)x->ptr<dz>(K.y), w, N);
      BLAUNCHCK();
      const dz *wv = w;
      if (x->precond == 0) {
        if (int rc = apply_minv_n(x, 1, &wv, &u, &tv, &zv)) return cell_fail(b, c, rc);
      } else {
        u = w;
      }
      hipLaunchKernelGGL(k_axpy, dim3(nblk(N, 256)), dim3(256), 0, b->stream, x->ptr<dz>(K.vx), (const dz *)u, N);
      BLAUNCHCK();
      if (int rc = matvec(x, x->ptr<dz>(K.vx), x->ptr<dz>(K.vb), x->ptr<dz>(K.vr))) return cell_fail(b, c, rc);
      if (int rc = norm_to(x, 0, x->ptr<dz>(K.vr), N, x->ptr<double>(K.scal) + 1)) return cell_fail(b, c, rc);
      BCK(hipMemcpyAsync(b->pin_res + c, x->ptr<double>(K.scal) + 1, 8, hipMemcpyDeviceToHost, b->stream));
    }
    BCK(hipStreamSynchronize(b->stream));
    for (int c : ending) {
      CellGmres &p = P[c];
      p.beta = b->pin_res[c];
      p.true_rel = p.beta / p.bnorm;
      p.in_cycle = false;
      if (p.true_rel <= tol || (p.est_ok && p.true_rel <= 10 * tol)) {
        p.converged = p.done = true;
      } else if (p.iters >= max_iter) {
        p.done = true;
      } else {
        ++p.restarts;
      }
    }
  }
  BCK(hipEventRecord(b->ev1, b->stream));
  BCK(hipEventSynchronize(b->ev1));
  float ms = 0;
  BCK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  int status = VIE_OK;
  for (int c = 0; c < nc; ++c) {
    vie_ctx *x = b->cells[c];
    x->sol_k[P[c].pol] = 0;
    x->last_pol = P[c].pol;
    x->state = S_SOLVED;
    if (info) {
      info[c].iters = P[c].iters;
      info[c].restarts = P[c].restarts;
      info[c].refine_steps = P[c].restarts + 1;
      info[c].true_rel_residual = P[c].true_rel;
      info[c].t_fill_ms = b->t_fill;
      info[c].t_factor_ms = b->t_factor;
      info[c].t_solve_ms = ms;
      info[c].converged = P[c].converged ? 1 : 0;
    }
    if (!P[c].converged && status == VIE_OK)
      status = bfail(b, VIE_ENOCONV, "cell %d: %d iterations, relative residual %.3e", c, P[c].iters, P[c].true_rel);
  }
  return status;
}

}  // extern "C"
