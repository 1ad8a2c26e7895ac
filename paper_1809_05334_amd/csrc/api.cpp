// C-ABI of libvie (include/vie.h): context state machine, workspace layout and
// the host orchestration of the fill, block factorisation, GMRES solve and
// absorption kernels.  All device work is issued on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "context.h"

using namespace vie;

namespace vie {

// The library's own workspace for callers that cannot allocate device memory
// (vie_bind_static_workspace).  Each device holds its own copy of the array
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (kept in g_static_ptr).
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

}  // namespace vie

static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace vie {

std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};      // device address of `scratch` on each device
vie_ctx *g_static_owner[kMaxDevices] = {};  // the context bound to it, if any

// Resolve the device address of the static workspace on ctx->device (the
// device must be current); once per device.
int resolve_static(vie_ctx *ctx) {
  if (ctx->device >= kMaxDevices) return VIE_OK;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_ptr[ctx->device]) return VIE_OK;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return fail(ctx, VIE_EDEVICE, "static workspace address: %s", hipGetErrorString(e));
  g_static_ptr[ctx->device] = p;
  return VIE_OK;
}

// ctx gives up the static workspace of its device (if it holds it).
void release_static(vie_ctx *ctx) {
  if (!ctx->static_ws || ctx->device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_owner[ctx->device] == ctx) g_static_owner[ctx->device] = nullptr;
  ctx->static_ws = false;
}


size_t nested_size(const std::vector<std::vector<int32_t>> &v) {
  size_t s = 0;
  for (const auto &x : v) s += x.size();
  return s;
}

Layout make_layout(const MeshTopology &t, int restart, int64_t nnear, int nface, int nhalf, int precision,
                   int64_t near_nnz, bool sym_fill, int64_t grid_nf) {
  Layout L;
  size_t off = 0;
  auto put = [&](Region &r, size_t bytes) {
    r.off = off;
    r.bytes = bytes;
    off = align256(off + std::max<size_t>(bytes, 1));
  };
  const int64_t N = t.N, nt = t.nt;
  put(L.tg, sizeof(TetGeom) * nt);
  put(L.t2f, sizeof(TetFace) * 4 * nt);
  put(L.area, 8 * N);
  put(L.dom, 4 * nt);
  put(L.fg, sizeof(FaceGeom) * std::max(1, nface));
  put(L.half, 4 * std::max(1, nhalf));
  put(L.ctp, 4 * std::max(1, nface));
  put(L.ctm, 4 * std::max(1, nface));
  put(L.utet, 8 * N);
  put(L.uk, 8 * N);
  put(L.colors, 4 * nt);
  put(L.near_t, 4 * std::max<int64_t>(1, nnear));
  put(L.near_s, 4 * std::max<int64_t>(1, nnear));
  put(L.near_m, 4 * std::max<int64_t>(1, nnear));
  put(L.near_tf, 4 * std::max<size_t>(1, nested_size(t.near_tf)));
  put(L.near_ft, 4 * std::max<size_t>(1, nested_size(t.near_ft)));
  put(L.quad, sizeof(QuadRules));
  put(L.pgf, sizeof(PgfTable));
  put(L.pack, 8 * (size_t)kMaxPack);
  put(L.eps, 16 * nt);
  put(L.alpha, 16 * 4 * nt);
  put(L.gsrc, 16 * 4 * nt);
  put(L.kappa, 16 * nt);
  put(L.inveps, 16 * nt);
  put(L.sigma, 16 * std::max(1, nface));
  L.ld = (N + 7) / 8 * 8;
  const bool mixed = precision == VIE_MIXED_FP32, grid = precision == VIE_GRID_FP64;
  // the grid operator keeps no dense Z (far part by FFT, near part in the CSR)
  put(L.Z, grid ? 0 : (mixed ? 8 : 16) * (size_t)N * L.ld);
  // staging for the transposed far blocks of a normal-incidence fill (VIE_OPT_SYM_FILL)
  if (sym_fill && !grid) put(L.Zt, (mixed ? 8 : 16) * (size_t)N * L.ld);
  const bool csr = mixed || grid;
  put(L.nrow, csr ? 8 * (size_t)(N + 1) : 0);
  put(L.ncol, csr ? 4 * (size_t)near_nnz : 0);
  put(L.nval, csr ? 16 * (size_t)near_nnz : 0);
  if (grid) {
    put(L.ggeo, sizeof(GridGeom));
    put(L.gtet, 8 * (size_t)nt);
    put(L.gface, 16 * (size_t)std::max(1, nface));
    put(L.ghalf, 4 * (size_t)std::max<int64_t>(1, N));
    put(L.gtab, 16 * (size_t)kGridSub * kGridSub * grid_nf);
    put(L.gin, 16 * (size_t)kGridFields * grid_nf);
    put(L.gout, 16 * (size_t)kGridFields * grid_nf);
  }
  L.fld.resize(t.ndom);
  L.foff.resize(t.ndom);
  int64_t fel = 0, npiv = 0;
  for (int d = 0; d < t.ndom; ++d) {
    int64_t n = grid ? 0 : t.dend[d] - t.dstart[d];   // (no block preconditioner with the grid operator)
    L.fld[d] = (n + 7) / 8 * 8;
    L.foff[d] = fel;
    fel += n * L.fld[d];
    npiv += n;
  }
  const size_t fes = mixed ? 8 : 16;   // factor element: complex FP32 in mixed precision
  put(L.F, fes * (size_t)std::max<int64_t>(1, fel));
  // per domain: the L then the U inverses of its diagonal blocks (block b at b nb^2, the
  // last one m x m), and the L then the U coupling blocks (nbk - 1 per sweep, nb^2 each)
  L.doff.resize(t.ndom);
  L.goff.resize(t.ndom);
  int64_t del = 0, gel = 0;
  for (int d = 0; d < t.ndom; ++d) {
    const int64_t n = grid ? 0 : t.dend[d] - t.dstart[d];
    const int64_t nbk = (n + kTrsvNB - 1) / kTrsvNB;
    L.doff[d] = del;
    L.goff[d] = gel;
    if (nbk == 0) continue;
    const int64_t mlast = n - (nbk - 1) * kTrsvNB;
    del += 2 * ((nbk - 1) * kTrsvNB * kTrsvNB + mlast * mlast);
    gel += 2 * (nbk - 1) * kTrsvNB * kTrsvNB;
  }
  put(L.dinv, fes * (size_t)std::max<int64_t>(1, del));
  put(L.gcpl, fes * (size_t)std::max<int64_t>(1, gel));
  put(L.trr, 16 * 4 * (size_t)kTrsvNB * std::max(1, t.ndom));   // r of a block: two buffers of two vectors per domain
  // chunk sums: per domain two buffers (steps alternate) of two vectors, kTrsvNB rows each
  L.boff.resize(t.ndom);
  int64_t bel = 0;
  for (int d = 0; d < t.ndom; ++d) {
    L.boff[d] = bel;
    if (!grid) bel += 4 * (int64_t)kTrsvNB * trsv_bsum_stride(t.dend[d] - t.dstart[d]);
  }
  put(L.tbsum, 16 * (size_t)std::max<int64_t>(1, bel));
  {
    int maxnbk = 1;
    for (int d = 0; d < t.ndom; ++d) maxnbk = std::max<int>(maxnbk, (int)((t.dend[d] - t.dstart[d] + kTrsvNB - 1) / kTrsvNB));
    const int chunks = (t.ndom + kTrsvMaxDom - 1) / kTrsvMaxDom;
    L.plan_steps = 2 * (maxnbk + 1) * std::max(1, chunks);   // two sweeps of maxnbk steps and a closing step
    put(L.plans, kMaxPlans * sizeof(TrsvStep) * (size_t)L.plan_steps);
  }
  put(L.ipiv, 4 * std::max<int64_t>(1, npiv));
  put(L.perm, 4 * std::max<int64_t>(1, npiv));
  int64_t npart = 0;
  for (int d = 0; d < t.ndom; ++d) npart += nblk(t.dend[d] - t.dstart[d], kColRows);
  put(L.rpiv, 16 * (size_t)std::max(1, t.ndom));
  put(L.info, 4 * std::max(1, t.ndom));
  put(L.lupv, 8 * (size_t)std::max<int64_t>(1, npart));
  put(L.lupi, 4 * (size_t)std::max<int64_t>(1, npart));
  put(L.lucnt, 4 * (size_t)std::max(1, t.ndom));
  // tournament pivoting: nodes of the tree of the first (tallest) panel, the
  // largest tree of the factorisation: leaves, then ceil(count / fan-in) per level
  int64_t nodes = 0;
  L.toff.assign(t.ndom, 0);
  for (int d = 0; d < t.ndom; ++d) {
    L.toff[d] = nodes;
    for (int64_t c = nblk(grid ? 1 : t.dend[d] - t.dstart[d], mixed ? kTsRowsC : kTsRowsZ);;
         c = (c + (mixed ? kTsFanC : kTsFanZ) - 1) / (mixed ? kTsFanC : kTsFanZ)) {
      nodes += c;
      if (c == 1) break;
    }
  }
  put(L.tcand, 4 * (size_t)kLuNB * std::max<int64_t>(1, nodes));
  put(L.ttcnt, 4 * (size_t)std::max<int64_t>(1, nodes));
  put(L.tblk, fes * (size_t)kLuNB * kLuNB * std::max(1, t.ndom));
  L.restart = restart;
  L.ldv = (N + 31) / 32 * 32;
  for (Layout::Kry &k : L.K) {
    put(k.V, 16 * (size_t)L.ldv * (restart + 1));
    put(k.H, 16 * (size_t)(restart + 2) * (restart + 1));
    put(k.cs, 8 * (restart + 1));
    put(k.sn, 16 * (restart + 1));
    put(k.g, 16 * (restart + 2));
    put(k.y, 16 * (restart + 1));
    for (Region *r : {&k.vb, &k.vx, &k.vw, &k.vz, &k.vu, &k.vr, &k.vt, &k.vin}) put(*r, 16 * N);
    put(k.jd, 256);
    put(k.rhist, 8 * (size_t)(restart + 1));
    put(k.dpart, 16 * (size_t)kRedBlocks * (restart + 1));
    put(k.npart, 8 * kRedBlocks);
    put(k.scal, 64);
  }
  put(L.jdiag, 16 * (size_t)std::max<int64_t>(1, N));
  put(L.apart, 8 * (size_t)nblk(nt, 256) * std::max(6 * 2 * 32, t.ndom));
  put(L.atet, 8 * (size_t)std::max<int64_t>(1, nt));
  put(L.kv, 8 * 3 * 2 * 32);
  // solver scratch; also the reduction target of the R/T projections (6 doubles per k-vector, <= 64)
  put(L.idx, std::max<size_t>(16 * (size_t)N, 8 * 6 * 64));
  L.total = off;
  return L;
}

int check(vie_ctx *ctx, State need, const char *what) {
  if (!ctx) return VIE_EINVAL;
  if (ctx->state < need) return fail(ctx, VIE_ESTATE, "%s called out of order", what);
  return VIE_OK;
}

// factor storage: complex FP32 in mixed precision, FP64 otherwise
bool fp32_factors(const vie_ctx *ctx) { return ctx->precision == VIE_MIXED_FP32; }
size_t factor_bytes(const vie_ctx *ctx) { return fp32_factors(ctx) ? 8 : 16; }
void *factor_ptr(vie_ctx *ctx, const Region &r, int64_t elem) {
  return ctx->ws + r.off + factor_bytes(ctx) * (size_t)elem;
}

void drop_graphs(vie_ctx *ctx) {
  ctx->plans.clear();
  for (int m = 0; m < 3; ++m) {
    for (hipGraphExec_t &g : ctx->gexec[m]) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
    ctx->gexec_steps[m] = 0;
  }
}

void ensure_near_pattern(vie_ctx *ctx) {
  if (ctx->npat) return;
  build_near_pattern(ctx->topo, ctx->nrow, ctx->ncol);
  ctx->npat = true;
}

// Grid analysis of the uploaded mesh (once per mesh): "" if it is a uniform
// Kuhn grid the structured-grid operator can take, else the reason.
const std::string &ensure_grid(vie_ctx *ctx) {
  if (!ctx->grid) {
    ctx->grid = new GridHost();
    ctx->grid_err = analyse_grid(ctx->topo, ctx->quad, *ctx->grid);
  }
  return ctx->grid_err;
}

void release_fft(vie_ctx *ctx) {
  if (ctx->fft_tab) (void)hipfftDestroy(ctx->fft_tab);
  if (ctx->fft_tab_sym) (void)hipfftDestroy(ctx->fft_tab_sym);
  if (ctx->fft_fld) (void)hipfftDestroy(ctx->fft_fld);
  ctx->fft_tab = ctx->fft_tab_sym = ctx->fft_fld = 0;
}

void release_grid(vie_ctx *ctx) {
  release_fft(ctx);
  delete ctx->grid;
  ctx->grid = nullptr;
  ctx->grid_err.clear();
}

ZOut zout(vie_ctx *ctx) {
  const Layout &L = ctx->L;
  ZOut o{};
  o.ld = L.ld;
  if (ctx->precision == VIE_MIXED_FP32 || ctx->precision == VIE_GRID_FP64) {
    // (the grid operator has no dense part; its fill launches no far-pair writer but k_face_face,
    // which then writes only the touching pairs)
    if (ctx->precision == VIE_MIXED_FP32) o.Zs = ctx->ptr<fz>(L.Z);
    o.rowptr = ctx->ptr<int64_t>(L.nrow);
    o.cols = ctx->ptr<int32_t>(L.ncol);
    o.vals = ctx->ptr<dz>(L.nval);
  } else {
    o.Z = ctx->ptr<dz>(L.Z);
  }
  return o;
}

// Structured-grid operator: y = Z x (or b - Z x): source fields, forward
// FFTs, per-frequency products with the kernel tables, inverse FFTs, then the
// far potentials and the near part per unknown.
int grid_matvec(vie_ctx *ctx, const dz *x, const dz *b, dz *y) {
  const Layout &L = ctx->L;
  const MeshTopology &t = ctx->topo;
  const int64_t nf = ctx->grid->g.nf;
  const GridGeom *gg = ctx->ptr<GridGeom>(L.ggeo);
  dz *fin = ctx->ptr<dz>(L.gin), *fout = ctx->ptr<dz>(L.gout);
  const double kx = ctx->fill_kx, ky = ctx->fill_ky;
  hipLaunchKernelGGL(k_zero, dim3(2048), dim3(256), 0, ctx->stream, fin, (int64_t)kGridFields * nf);
  hipLaunchKernelGGL(k_grid_gather_tet, dim3(nblk(t.nt, 256)), dim3(256), 0, ctx->stream, (int64_t)t.nt, gg,
                     (const int32_t *)ctx->ptr<int32_t>(L.gtet), (const TetGeom *)ctx->ptr<TetGeom>(L.tg),
                     (const TetFace *)ctx->ptr<TetFace>(L.t2f), (const dz *)ctx->ptr<dz>(L.gsrc),
                     (const dz *)ctx->ptr<dz>(L.kappa), x, kx, ky, fin);
  if (ctx->nface)
    hipLaunchKernelGGL(k_grid_gather_face, dim3(nblk(ctx->nface, 256)), dim3(256), 0, ctx->stream, ctx->nface, gg,
                       (const int32_t *)ctx->ptr<int32_t>(L.gface), (const FaceGeom *)ctx->ptr<FaceGeom>(L.fg),
                       (const dz *)ctx->ptr<dz>(L.sigma), x, kx, ky, fin);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "grid matvec: %s", hipGetErrorString(e));
  if (hipfftExecZ2Z(ctx->fft_fld, (hipfftDoubleComplex *)fin, (hipfftDoubleComplex *)fin, HIPFFT_FORWARD) !=
      HIPFFT_SUCCESS)
    return fail(ctx, VIE_EDEVICE, "grid matvec: forward FFT failed");
  const GridGeom &G = ctx->grid->g;
  if (ctx->grid_sym)
    hipLaunchKernelGGL(k_grid_mul_sym, dim3(nblk(nf, 32)), dim3(256), 0, ctx->stream, nf, G.nx, G.ny, G.pz,
                       (const dz *)ctx->ptr<dz>(L.gtab), (const dz *)fin, fout);
  else
    hipLaunchKernelGGL(k_grid_mul, dim3(nblk(nf, 32)), dim3(256), 0, ctx->stream, nf,
                       (const dz *)ctx->ptr<dz>(L.gtab), (const dz *)fin, fout);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "grid matvec: %s", hipGetErrorString(e));
  if (hipfftExecZ2Z(ctx->fft_fld, (hipfftDoubleComplex *)fout, (hipfftDoubleComplex *)fout, HIPFFT_BACKWARD) !=
      HIPFFT_SUCCESS)
    return fail(ctx, VIE_EDEVICE, "grid matvec: inverse FFT failed");
  hipLaunchKernelGGL(k_grid_apply, dim3(nblk(t.N, 4)), dim3(256), 0, ctx->stream, (int64_t)t.N, gg,
                     (const int32_t *)ctx->ptr<int32_t>(L.gtet), (const int32_t *)ctx->ptr<int32_t>(L.gface),
                     (const int32_t *)ctx->ptr<int32_t>(L.ghalf), (const int32_t *)ctx->ptr<int32_t>(L.utet),
                     (const int32_t *)ctx->ptr<int32_t>(L.uk), (const TetGeom *)ctx->ptr<TetGeom>(L.tg),
                     (const FaceGeom *)ctx->ptr<FaceGeom>(L.fg), (const dz *)ctx->ptr<dz>(L.alpha), (const dz *)fout,
                     ctx->fill_k0sq9, kx, ky, (const int64_t *)ctx->ptr<int64_t>(L.nrow),
                     (const int32_t *)ctx->ptr<int32_t>(L.ncol), (const dz *)ctx->ptr<dz>(L.nval), x, b, y);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "grid matvec: %s", hipGetErrorString(e));
  return VIE_OK;
}

// y = Z x, or y = b - Z x when b is given, with the bound precision's operator
int matvec(vie_ctx *ctx, const dz *x, const dz *b, dz *y) {
  if (ctx->precision == VIE_GRID_FP64) return grid_matvec(ctx, x, b, y);
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  const int R = ctx->mv_rpw;
  const dim3 grid(nblk(N, 4 * R)), blk(256);
  if (ctx->precision == VIE_MIXED_FP32) {
    const fz *Zs = ctx->ptr<fz>(L.Z);
    const int64_t *rp = ctx->ptr<int64_t>(L.nrow);
    const int32_t *cl = ctx->ptr<int32_t>(L.ncol);
    const dz *vl = ctx->ptr<dz>(L.nval);
    if (R == 2) hipLaunchKernelGGL(k_matvec_mixed_r2, grid, blk, 0, ctx->stream, Zs, L.ld, N, rp, cl, vl, x, b, y);
    else if (R == 8) hipLaunchKernelGGL(k_matvec_mixed_r8, grid, blk, 0, ctx->stream, Zs, L.ld, N, rp, cl, vl, x, b, y);
    else hipLaunchKernelGGL(k_matvec_mixed_r4, grid, blk, 0, ctx->stream, Zs, L.ld, N, rp, cl, vl, x, b, y);
  } else {
    const dz *Z = ctx->ptr<dz>(L.Z);
    if (R == 2) hipLaunchKernelGGL(k_matvec_r2, grid, blk, 0, ctx->stream, Z, L.ld, N, x, b, y);
    else if (R == 8) hipLaunchKernelGGL(k_matvec_r8, grid, blk, 0, ctx->stream, Z, L.ld, N, x, b, y);
    else hipLaunchKernelGGL(k_matvec_r4, grid, blk, 0, ctx->stream, Z, L.ld, N, x, b, y);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "matvec: %s", hipGetErrorString(e));
  return VIE_OK;
}

// y_q = Z x_q (or b_q - Z x_q) for two vectors in one pass over Z; each y_q
// is bitwise the single-vector result.
int matvec2(vie_ctx *ctx, const MvVecs &v) {
  if (ctx->precision == VIE_GRID_FP64) {
    for (int q = 0; q < 2; ++q)
      if (int rc = grid_matvec(ctx, v.x[q], v.b[q], v.y[q])) return rc;
    return VIE_OK;
  }
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  const int R = ctx->mv_rpw;
  const dim3 grid(nblk(N, 4 * R)), blk(256);
  if (ctx->precision == VIE_MIXED_FP32) {
    const fz *Zs = ctx->ptr<fz>(L.Z);
    const int64_t *rp = ctx->ptr<int64_t>(L.nrow);
    const int32_t *cl = ctx->ptr<int32_t>(L.ncol);
    const dz *vl = ctx->ptr<dz>(L.nval);
    if (R == 2) hipLaunchKernelGGL(k_matvec2_mixed_r2, grid, blk, 0, ctx->stream, Zs, L.ld, N, rp, cl, vl, v);
    else if (R == 8) hipLaunchKernelGGL(k_matvec2_mixed_r8, grid, blk, 0, ctx->stream, Zs, L.ld, N, rp, cl, vl, v);
    else hipLaunchKernelGGL(k_matvec2_mixed_r4, grid, blk, 0, ctx->stream, Zs, L.ld, N, rp, cl, vl, v);
  } else {
    const dz *Z = ctx->ptr<dz>(L.Z);
    if (R == 2) hipLaunchKernelGGL(k_matvec2_r2, grid, blk, 0, ctx->stream, Z, L.ld, N, v);
    else if (R == 8) hipLaunchKernelGGL(k_matvec2_r8, grid, blk, 0, ctx->stream, Z, L.ld, N, v);
    else hipLaunchKernelGGL(k_matvec2_r4, grid, blk, 0, ctx->stream, Z, L.ld, N, v);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "matvec: %s", hipGetErrorString(e));
  return VIE_OK;
}

}  // namespace vie

// ================================================================ C-ABI
extern "C" {

}  // extern "C"

namespace {

// Events, pinned staging and the static workspace's address of a new context.
int init_ctx(vie_ctx *ctx) {
  ctx->tab = new PgfTable();
  build_quadrature(ctx->quad);
  HIPCK(hipSetDevice(ctx->device));
  HIPCK(hipHostMalloc((void **)&ctx->pinned, 4096, hipHostMallocDefault));
  HIPCK(hipEventCreate(&ctx->ev0));
  HIPCK(hipEventCreate(&ctx->ev1));
  HIPCK(hipEventCreate(&ctx->ev2));
  HIPCK(hipEventCreate(&ctx->ev3));
  HIPCK(hipEventCreate(&ctx->ev4));
  if (int rc = resolve_static(ctx)) return rc;
  // the factorisation's side stream is created at its first use, so contexts
  // that only wait (a serving queue) hold no stream of their own
  HIPCK(hipEventCreateWithFlags(&ctx->ev_la, hipEventDisableTiming));
  HIPCK(hipEventCreateWithFlags(&ctx->ev_ts, hipEventDisableTiming));
  return VIE_OK;
}

}  // namespace

extern "C" {

int vie_create(vie_ctx **out, int device, void *hip_stream) {
  if (!out) return VIE_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return VIE_EDEVICE;
  vie_ctx *ctx = new vie_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (int rc = init_ctx(ctx)) {
    vie_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return VIE_OK;
}

int vie_set_stream(vie_ctx *ctx, void *hip_stream) {
  if (!ctx) return VIE_EINVAL;
  HIPCK(hipSetDevice(ctx->device));
  // before the workspace is bound the context has issued no device work
  if (ctx->state >= S_BOUND) HIPCK(hipStreamSynchronize(ctx->stream));
  ctx->stream = (hipStream_t)hip_stream;
  for (hipfftHandle h : {ctx->fft_tab, ctx->fft_tab_sym, ctx->fft_fld})
    if (h && hipfftSetStream(h, ctx->stream) != HIPFFT_SUCCESS) return fail(ctx, VIE_EDEVICE, "hipfftSetStream failed");
  return VIE_OK;
}

int vie_destroy(vie_ctx *ctx) {
  if (!ctx) return VIE_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  drop_graphs(ctx);
  release_static(ctx);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->pin_piv) (void)hipHostFree(ctx->pin_piv);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->ev2) (void)hipEventDestroy(ctx->ev2);
  if (ctx->ev3) (void)hipEventDestroy(ctx->ev3);
  if (ctx->ev4) (void)hipEventDestroy(ctx->ev4);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->ev_la) (void)hipEventDestroy(ctx->ev_la);
  if (ctx->ev_ts) (void)hipEventDestroy(ctx->ev_ts);
  for (hipEvent_t e : ctx->upd_ev) (void)hipEventDestroy(e);
  release_grid(ctx);
  delete ctx->tab;
  delete ctx;
  return VIE_OK;
}

const char *vie_last_error(const vie_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int vie_mesh_upload(vie_ctx *ctx, const double *verts_nm, int64_t nv, const int32_t *tets, int64_t nt,
                    const int32_t *tet_domain, int32_t ndom, double a_nm, double b_nm) {
  if (!ctx) return VIE_EINVAL;
  if (!verts_nm || !tets || !tet_domain) return fail(ctx, VIE_EINVAL, "null mesh array");
  std::string e = build_topology(ctx->topo, verts_nm, nv, tets, nt, tet_domain, ndom, a_nm, b_nm);
  if (!e.empty()) {
    ctx->state = S_NEW;
    return fail(ctx, VIE_EINVAL, "mesh: %s", e.c_str());
  }
  ctx->state = S_MESH;
  ctx->factored = false;
  ctx->ws = nullptr;
  // per-mesh host state of the previous mesh: the near-part pattern and the grid analysis
  ctx->npat = false;
  ctx->nrow.clear();
  ctx->ncol.clear();
  release_grid(ctx);
  return VIE_OK;
}

int64_t vie_num_unknowns(const vie_ctx *ctx) { return ctx && ctx->state >= S_MESH ? ctx->topo.N : -1; }

int vie_domain_ranges(const vie_ctx *ctx, int64_t *se) {
  if (!ctx || ctx->state < S_MESH || !se) return VIE_ESTATE;
  for (int d = 0; d < ctx->topo.ndom; ++d) {
    se[2 * d] = ctx->topo.dstart[d];
    se[2 * d + 1] = ctx->topo.dend[d];
  }
  return VIE_OK;
}

static int64_t total_near(const MeshTopology &t) {
  int64_t s = 0;
  for (auto &v : t.near_t) s += (int64_t)v.size();
  return s;
}

size_t vie_workspace_bytes(const vie_ctx *cctx, int precision, int restart) {
  if (!cctx || cctx->state < S_MESH || restart < 1) return 0;
  if (precision != VIE_FP64 && precision != VIE_MIXED_FP32 && precision != VIE_GRID_FP64) return 0;
  vie_ctx *ctx = const_cast<vie_ctx *>(cctx);
  int nhalf = 0;
  for (int32_t f : ctx->topo.charged)
    if (ctx->topo.tminus[f] < 0) ++nhalf;
  int64_t nnz = 0, gnf = 0;
  if (precision == VIE_GRID_FP64) {
    if (!ensure_grid(ctx).empty()) return 0;
    gnf = ctx->grid->g.nf;
  }
  if (precision == VIE_MIXED_FP32 || precision == VIE_GRID_FP64) {
    ensure_near_pattern(ctx);
    nnz = (int64_t)ctx->ncol.size();
  }
  return make_layout(ctx->topo, restart, total_near(ctx->topo), (int)ctx->topo.charged.size(), nhalf, precision, nnz,
                     ctx->sym_fill != 0, gnf)
      .total;
}

}  // extern "C"

namespace vie {

// Bind `bytes` of device memory at dev_ptr as the workspace and upload the
// mesh tables.  no_alloc: allocate nothing (no pinned host staging either;
// the pivot read-back then goes through pageable host memory).
int bind_impl(vie_ctx *ctx, void *dev_ptr, size_t bytes, int precision, int restart, bool no_alloc) {
  if (precision != VIE_FP64 && precision != VIE_MIXED_FP32 && (precision != VIE_GRID_FP64 || no_alloc))
    return fail(ctx, VIE_EINVAL, no_alloc ? "precision must be VIE_FP64 or VIE_MIXED_FP32"
                                          : "precision must be VIE_FP64, VIE_MIXED_FP32 or VIE_GRID_FP64");
  if (restart < 1 || restart > 1000) return fail(ctx, VIE_EINVAL, "restart must be in [1, 1000]");
  if (!dev_ptr || ((uintptr_t)dev_ptr & 255)) return fail(ctx, VIE_EINVAL, "workspace must be 256-byte aligned");
  HIPCK(hipSetDevice(ctx->device));
  const MeshTopology &t = ctx->topo;
  std::vector<int32_t> half;
  for (size_t i = 0; i < t.charged.size(); ++i)
    if (t.tminus[t.charged[i]] < 0) half.push_back((int32_t)i);
  ctx->nhalf = (int)half.size();
  ctx->nface = (int)t.charged.size();
  int64_t nnz = 0, gnf = 0;
  if (precision == VIE_GRID_FP64) {
    const std::string &ge = ensure_grid(ctx);
    if (!ge.empty()) return fail(ctx, VIE_EINVAL, "VIE_GRID_FP64 needs a uniform Kuhn brick grid: %s", ge.c_str());
    gnf = ctx->grid->g.nf;
  }
  if (precision == VIE_MIXED_FP32 || precision == VIE_GRID_FP64) {
    ensure_near_pattern(ctx);
    nnz = (int64_t)ctx->ncol.size();
  }
  Layout L = make_layout(t, restart, total_near(t), ctx->nface, ctx->nhalf, precision, nnz, ctx->sym_fill != 0, gnf);
  if (bytes < L.total) return fail(ctx, VIE_ENOMEM, "workspace %zu bytes < required %zu", bytes, L.total);
  if (ctx->pin_piv_n < t.N) {
    HIPCK(hipStreamSynchronize(ctx->stream));   // no upload of the permutation in flight
    if (no_alloc) {
      ctx->piv_host.resize(2 * (size_t)std::max<int64_t>(1, t.N));
    } else {
      if (ctx->pin_piv) HIPCK(hipHostFree(ctx->pin_piv));
      ctx->pin_piv = nullptr;
      ctx->pin_piv_n = 0;
      HIPCK(hipHostMalloc((void **)&ctx->pin_piv, 8 * (size_t)std::max<int64_t>(1, t.N), hipHostMallocDefault));
      ctx->pin_piv_n = t.N;
    }
  }
  drop_graphs(ctx);   // captured graphs hold pointers into the old workspace
  ctx->L = L;
  ctx->ws = (char *)dev_ptr;
  ctx->ws_bytes = bytes;
  ctx->precision = precision;

  // ---- host staging of the mesh tables
  std::vector<TetGeom> tg(t.nt);
  for (int64_t e = 0; e < t.nt; ++e) {
    TetGeom &g = tg[e];
    for (int d = 0; d < 3; ++d) g.c[d] = 0;
    for (int k = 0; k < 4; ++k) {
      int32_t v = t.tets[4 * e + k];
      for (int d = 0; d < 3; ++d) {
        g.v[k][d] = t.verts[3 * v + d];
        g.c[d] += 0.25 * t.verts[3 * v + d];
      }
      g.canon[k] = t.canon[v];
      g.off[k] = (t.offx[v] + 2) | ((t.offy[v] + 2) << 4);
    }
    g.vol = t.vol[e];
  }
  std::vector<FaceGeom> fg(std::max<size_t>(1, t.charged.size()));
  std::vector<int32_t> ctp(fg.size(), 0), ctm(fg.size(), -1);
  for (size_t i = 0; i < t.charged.size(); ++i) {
    int32_t f = t.charged[i];
    FaceGeom &g = fg[i];
    for (int j = 0; j < 3; ++j) {
      int32_t v = t.face_vid[3 * f + j];
      for (int d = 0; d < 3; ++d) g.v[j][d] = t.verts[3 * v + d];
      g.canon[j] = t.canon[v];
      g.off[j] = (t.offx[v] + 2) | ((t.offy[v] + 2) << 4);
    }
    g.area = t.area[f];
    g.unknown = f;
    g.half = t.tminus[f] < 0;
    ctp[i] = t.tplus[f];
    ctm[i] = t.tminus[f];
  }
  std::vector<int32_t> utet(2 * t.N, -1), uk(2 * t.N, 0);
  for (int64_t e = 0; e < t.nt; ++e)
    for (int k = 0; k < 4; ++k) {
      const TetFace &f = t.t2f[4 * e + k];
      int h = f.sign > 0 ? 0 : 1;
      utet[2 * f.unknown + h] = (int32_t)e;
      uk[2 * f.unknown + h] = k;
    }
  std::vector<int32_t> colors;
  ctx->color_off.assign(t.ncolors + 1, 0);
  for (int c = 0; c < t.ncolors; ++c) {
    ctx->color_off[c] = (int32_t)colors.size();
    colors.insert(colors.end(), t.color_tets[c].begin(), t.color_tets[c].end());
  }
  ctx->color_off[t.ncolors] = (int32_t)colors.size();
  std::vector<int32_t> nt_, ns_, nm_;
  const int C = t.ncolors;
  ctx->near_off.assign(C * C + 1, 0);
  for (int g = 0; g < C * C; ++g) {
    ctx->near_off[g] = (int32_t)nt_.size();
    nt_.insert(nt_.end(), t.near_t[g].begin(), t.near_t[g].end());
    ns_.insert(ns_.end(), t.near_s[g].begin(), t.near_s[g].end());
    nm_.insert(nm_.end(), t.near_mask[g].begin(), t.near_mask[g].end());
  }
  ctx->near_off[C * C] = (int32_t)nt_.size();

  auto up = [&](const Region &r, const void *src, size_t n) -> int {
    if (n == 0) return VIE_OK;
    HIPCK(hipMemcpyAsync(ctx->ws + r.off, src, n, hipMemcpyHostToDevice, ctx->stream));
    return VIE_OK;
  };
  int rc = 0;
  rc |= up(L.tg, tg.data(), sizeof(TetGeom) * t.nt);
  rc |= up(L.t2f, t.t2f.data(), sizeof(TetFace) * 4 * t.nt);
  rc |= up(L.area, t.area.data(), 8 * t.N);
  rc |= up(L.dom, t.dom.data(), 4 * t.nt);
  rc |= up(L.fg, fg.data(), sizeof(FaceGeom) * t.charged.size());
  rc |= up(L.half, half.data(), 4 * half.size());
  rc |= up(L.ctp, ctp.data(), 4 * t.charged.size());
  rc |= up(L.ctm, ctm.data(), 4 * t.charged.size());
  rc |= up(L.utet, utet.data(), 4 * utet.size());
  rc |= up(L.uk, uk.data(), 4 * uk.size());
  rc |= up(L.colors, colors.data(), 4 * colors.size());
  rc |= up(L.near_t, nt_.data(), 4 * nt_.size());
  rc |= up(L.near_s, ns_.data(), 4 * ns_.size());
  rc |= up(L.near_m, nm_.data(), 4 * nm_.size());
  std::vector<int32_t> tf_, ft_;
  ctx->tf_off.assign(C + 1, 0);
  ctx->ft_off.assign(C + 1, 0);
  for (int c = 0; c < C; ++c) {
    ctx->tf_off[c] = (int32_t)(tf_.size() / 2);
    ctx->ft_off[c] = (int32_t)(ft_.size() / 2);
    tf_.insert(tf_.end(), t.near_tf[c].begin(), t.near_tf[c].end());
    ft_.insert(ft_.end(), t.near_ft[c].begin(), t.near_ft[c].end());
  }
  ctx->tf_off[C] = (int32_t)(tf_.size() / 2);
  ctx->ft_off[C] = (int32_t)(ft_.size() / 2);
  rc |= up(L.near_tf, tf_.data(), 4 * tf_.size());
  rc |= up(L.near_ft, ft_.data(), 4 * ft_.size());
  rc |= up(L.quad, &ctx->quad, sizeof(QuadRules));
  if (precision == VIE_MIXED_FP32 || precision == VIE_GRID_FP64) {
    rc |= up(L.nrow, ctx->nrow.data(), 8 * ctx->nrow.size());
    rc |= up(L.ncol, ctx->ncol.data(), 4 * ctx->ncol.size());
  }
  release_fft(ctx);
  if (precision == VIE_GRID_FP64) {
    const GridHost &G = *ctx->grid;
    rc |= up(L.ggeo, &G.g, sizeof(GridGeom));
    rc |= up(L.gtet, G.tet.data(), 4 * G.tet.size());
    rc |= up(L.gface, G.face.data(), 4 * G.face.size());
    rc |= up(L.ghalf, G.half.data(), 4 * G.half.size());
    // batched 3D transforms over (z, y, x): the kernel tables and the fields
    // of one product (hipFFT allocates their work areas)
    int n3[3] = {G.g.pz, G.g.ny, G.g.nx};
    const int nf = (int)G.g.nf;
    if (hipfftPlanMany(&ctx->fft_tab, 3, n3, nullptr, 1, nf, nullptr, 1, nf, HIPFFT_Z2Z, kGridSub * kGridSub) !=
            HIPFFT_SUCCESS ||
        hipfftPlanMany(&ctx->fft_tab_sym, 3, n3, nullptr, 1, nf, nullptr, 1, nf, HIPFFT_Z2Z, kGridSymPairs) !=
            HIPFFT_SUCCESS ||
        hipfftPlanMany(&ctx->fft_fld, 3, n3, nullptr, 1, nf, nullptr, 1, nf, HIPFFT_Z2Z, kGridFields) !=
            HIPFFT_SUCCESS ||
        hipfftSetStream(ctx->fft_tab, ctx->stream) != HIPFFT_SUCCESS ||
        hipfftSetStream(ctx->fft_tab_sym, ctx->stream) != HIPFFT_SUCCESS ||
        hipfftSetStream(ctx->fft_fld, ctx->stream) != HIPFFT_SUCCESS) {
      release_fft(ctx);
      return fail(ctx, VIE_EDEVICE, "hipFFT plans for the grid operator could not be made");
    }
  }
  if (rc) return rc;
  // the panel and tournament counters start (and always end) at zero
  HIPCK(hipMemsetAsync(ctx->ws + L.lucnt.off, 0, L.lucnt.bytes, ctx->stream));
  HIPCK(hipMemsetAsync(ctx->ws + L.ttcnt.off, 0, L.ttcnt.bytes, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));   // host staging vectors go out of scope
  ctx->state = S_BOUND;
  ctx->factored = false;
  return VIE_OK;
}

}  // namespace vie

extern "C" {

int vie_bind_workspace(vie_ctx *ctx, void *dev_ptr, size_t bytes, int precision, int restart) {
  if (int r = check(ctx, S_MESH, "vie_bind_workspace")) return r;
  release_static(ctx);
  return bind_impl(ctx, dev_ptr, bytes, precision, restart, false);
}

int vie_bind_static_workspace(vie_ctx *ctx, int precision, int restart) {
  if (int r = check(ctx, S_MESH, "vie_bind_static_workspace")) return r;
  if (precision != VIE_FP64 && precision != VIE_MIXED_FP32)
    return fail(ctx, VIE_EINVAL, "precision must be VIE_FP64 or VIE_MIXED_FP32");
  if (restart < 1 || restart > 1000) return fail(ctx, VIE_EINVAL, "restart must be in [1, 1000]");
  if (ctx->device >= kMaxDevices) return fail(ctx, VIE_EINVAL, "no static workspace on device %d", ctx->device);
  const size_t need = vie_workspace_bytes(ctx, precision, restart);
  if (need == 0 || need > kStaticWorkspaceBytes)
    return fail(ctx, VIE_ENOMEM, "workspace of %zu bytes exceeds the library's static workspace (%zu bytes)", need,
                kStaticWorkspaceBytes);
  HIPCK(hipSetDevice(ctx->device));
  void *p = nullptr;
  vie_ctx *prev = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    p = g_static_ptr[ctx->device];
    prev = g_static_owner[ctx->device];
    g_static_owner[ctx->device] = ctx;
  }
  if (!p) return fail(ctx, VIE_EDEVICE, "static workspace address unresolved on device %d", ctx->device);
  if (prev && prev != ctx) {
    // the previous holder loses the workspace: let its issued work finish,
    // then any further call on it needs a new bind (VIE_ESTATE)
    if (prev->stream) HIPCK(hipStreamSynchronize(prev->stream));
    else HIPCK(hipDeviceSynchronize());
    prev->static_ws = false;
    prev->ws = nullptr;
    prev->factored = false;
    if (prev->state > S_MESH) prev->state = S_MESH;
  }
  ctx->static_ws = true;
  if (int rc = bind_impl(ctx, p, kStaticWorkspaceBytes, precision, restart, true)) {
    release_static(ctx);
    ctx->ws = nullptr;
    ctx->state = S_MESH;
    return rc;
  }
  return VIE_OK;
}

}  // extern "C"

namespace vie {

// Host-only part of a fill (no device work; any thread): the lattice-sum
// tables of (lambda, theta, phi) packed for the device, and the internal
// permittivities.  The previous fill's kernels may still read the device
// copies: fill_upload waits for them.
int fill_tables(vie_ctx *ctx, double lambda_nm, double theta, double phi, const vie_c128 *eps_per_tet, int precision) {
  if (int r = check(ctx, S_BOUND, "vie_fill")) return r;
  if (precision != ctx->precision) return fail(ctx, VIE_EINVAL, "precision does not match the bound workspace");
  if (!eps_per_tet || !(lambda_nm > 0) || !(std::fabs(theta) < 1.5533)) return fail(ctx, VIE_EINVAL, "bad fill arguments");
  const MeshTopology &t = ctx->topo;
  double margin = 0;
  std::string e = build_pgf_table(*ctx->tab, t.a, t.b, t.zmax - t.zmin, lambda_nm, theta, phi, &margin);
  if (!e.empty()) return fail(ctx, VIE_EINVAL, "%s", e.c_str());
  if (margin < 0.02) return fail(ctx, VIE_EWOOD, "Floquet order near grazing (margin %.3g < 0.02)", margin);
  ctx->lambda = lambda_nm;
  ctx->theta = theta;
  ctx->phi = phi;
  for (int64_t i = 0; i < t.nt; ++i) {
    const vie_c128 e = eps_per_tet[i];
    if (!std::isfinite(e.re) || !std::isfinite(e.im) || (e.re == 0 && e.im == 0))
      return fail(ctx, VIE_EINVAL, "permittivity of tetrahedron %lld is zero or not finite", (long long)i);
  }
  ctx->eps_int.resize(t.nt);
  for (int64_t i = 0; i < t.nt; ++i) ctx->eps_int[i] = dz{eps_per_tet[i].re, -eps_per_tet[i].im};
  pack_pgf_table(*ctx->tab, ctx->pack);
  if ((int)ctx->pack.size() > kMaxPack)
    return fail(ctx, VIE_EINVAL, "lattice-sum table needs %zu doubles (> %d)", ctx->pack.size(), kMaxPack);
  ctx->packlen = (int)ctx->pack.size();
  return VIE_OK;
}

int fill_prepare(vie_ctx *ctx, double lambda_nm, double theta, double phi, const vie_c128 *eps_per_tet, int precision) {
  if (int rc = fill_tables(ctx, lambda_nm, theta, phi, eps_per_tet, precision)) return rc;
  return fill_upload(ctx);
}

// Device part of a fill's preparation (after fill_tables): tables and
// permittivities uploaded, per-tetrahedron coefficients, Z (with its staging
// copy and near part) cleared; records ev0.  Decides the form of the far fill.
int fill_upload(vie_ctx *ctx) {
  HIPCK(hipSetDevice(ctx->device));
  const MeshTopology &t = ctx->topo;
  const Layout &L = ctx->L;
  const double lambda_nm = ctx->lambda, theta = ctx->theta, phi = ctx->phi;
  // the previous fill's kernels may still read the tables: wait before overwriting
  HIPCK(hipStreamSynchronize(ctx->stream));
  HIPCK(hipMemcpyAsync(ctx->ws + L.pgf.off, ctx->tab, sizeof(PgfTable), hipMemcpyHostToDevice, ctx->stream));
  HIPCK(hipMemcpyAsync(ctx->ws + L.pack.off, ctx->pack.data(), 8 * ctx->pack.size(), hipMemcpyHostToDevice,
                       ctx->stream));
  HIPCK(hipMemcpyAsync(ctx->ws + L.eps.off, ctx->eps_int.data(), 16 * t.nt, hipMemcpyHostToDevice, ctx->stream));
  HIPCK(hipEventRecord(ctx->ev0, ctx->stream));

  const TetGeom *tg = ctx->ptr<TetGeom>(L.tg);
  const TetFace *t2f = ctx->ptr<TetFace>(L.t2f);
  dz *alpha = ctx->ptr<dz>(L.alpha), *gsrc = ctx->ptr<dz>(L.gsrc), *kappa = ctx->ptr<dz>(L.kappa),
     *inveps = ctx->ptr<dz>(L.inveps), *sigma = ctx->ptr<dz>(L.sigma);
  const double k0 = 2 * M_PI / lambda_nm;
  const double kx = k0 * std::sin(theta) * std::cos(phi), ky = k0 * std::sin(theta) * std::sin(phi);
  ctx->fill_k0sq9 = k0 * k0 / 9.0;
  ctx->fill_kx = kx;
  ctx->fill_ky = ky;
  ctx->jdiag_ok = false;
  ctx->fill_lds = 8 * (size_t)ctx->packlen;

  hipLaunchKernelGGL(k_prep, dim3(nblk(t.nt, 256)), dim3(256), 0, ctx->stream, (int64_t)t.nt, t2f, tg,
                     ctx->ptr<double>(L.area), ctx->ptr<dz>(L.eps), kx, ky, t.a, t.b, alpha, gsrc, kappa, inveps);
  LAUNCHCK();
  if (ctx->nface)
    hipLaunchKernelGGL(k_sigma, dim3(nblk(ctx->nface, 256)), dim3(256), 0, ctx->stream, ctx->nface,
                       ctx->ptr<int32_t>(L.ctp), ctx->ptr<int32_t>(L.ctm), (const dz *)kappa, sigma);
  // With the staging bound (VIE_OPT_SYM_FILL) each unordered far tet pair is
  // evaluated once and also yields the swapped pair's block, gathered in Zt:
  // at normal incidence (kt = 0) the lattice sum is even in the separation;
  // at oblique incidence g_p at the reversed separations follows from the same
  // evaluation plus the propagating orders' term (rev).  Each far (tet,
  // half-SWG face) pair likewise yields the (face, tet) entry, by the same
  // two forms.  Zt is added transposed after the face kernels.
  const bool kt0 = kx == 0.0 && ky == 0.0;
  // (the oblique form keeps 32 KB per block of the swapped moments in LDS
  // beside the table; a table too large for both runs the plain fill)
  ctx->fill_sym = L.Zt.bytes > 0 && (kt0 || ctx->fill_lds + kFarRevLds <= 65536);
  ctx->fill_sym_face = ctx->fill_sym;
  ctx->fill_rev = kt0 ? 0 : 1;
  ctx->last_sym = ctx->fill_sym;
  if (ctx->fill_sym)
    hipLaunchKernelGGL(k_zero, dim3(4096), dim3(256), 0, ctx->stream, ctx->ptr<dz>(L.Zt), (int64_t)(L.Zt.bytes / 16));
  // clear Z (and the near part): the fill accumulates into it
  hipLaunchKernelGGL(k_zero, dim3(4096), dim3(256), 0, ctx->stream, ctx->ptr<dz>(L.Z), (int64_t)(L.Z.bytes / 16));
  if (L.nval.bytes)
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, ctx->stream, ctx->ptr<dz>(L.nval), (int64_t)(L.nval.bytes / 16));
  LAUNCHCK();
  return VIE_OK;
}

// The staging copy of Z as a fill destination (the swapped blocks).
ZOut zout_staging(vie_ctx *ctx) {
  ZOut zt = zout(ctx);
  if (ctx->fill_sym) {
    if (ctx->precision == VIE_MIXED_FP32) zt.Zs = ctx->ptr<fz>(ctx->L.Zt);
    else zt.Z = ctx->ptr<dz>(ctx->L.Zt);
  }
  return zt;
}

// One context's fill kernels: far tet pairs (all colour pairs), touching
// pairs, face pairs; events between the groups time each kernel family.
int fill_kernels(vie_ctx *ctx) {
  const MeshTopology &t = ctx->topo;
  const Layout &L = ctx->L;
  const double *pk_ = ctx->ptr<double>(L.pack);
  const int pkl = ctx->packlen;
  const size_t lds = ctx->fill_lds;
  const QuadRules *qr = ctx->ptr<QuadRules>(L.quad);
  const TetGeom *tg = ctx->ptr<TetGeom>(L.tg);
  const TetFace *t2f = ctx->ptr<TetFace>(L.t2f);
  const dz *alpha = ctx->ptr<dz>(L.alpha), *gsrc = ctx->ptr<dz>(L.gsrc), *kappa = ctx->ptr<dz>(L.kappa),
           *inveps = ctx->ptr<dz>(L.inveps), *sigma = ctx->ptr<dz>(L.sigma);
  const ZOut zo = zout(ctx), zt = zout_staging(ctx);
  const double k0sq9 = ctx->fill_k0sq9;
  const bool sym = ctx->fill_sym, sym_face = ctx->fill_sym_face;
  const int rev = ctx->fill_rev;
  const int C = t.ncolors;
  const int32_t *colors = ctx->ptr<int32_t>(L.colors);
  // the grid operator takes every far pair from its FFT tables (built below)
  const bool grid = ctx->precision == VIE_GRID_FP64;
  HIPCK(hipEventRecord(ctx->ev2, ctx->stream));
  int far_launches = 0;
  for (int ct = 0; ct < (grid ? 0 : C); ++ct)
    for (int cs = 0; cs < C; ++cs) {
      if (sym && cs < ct) continue;   // covered by the launch of (cs, ct)
      const int nT = ctx->color_off[ct + 1] - ctx->color_off[ct], nS = ctx->color_off[cs + 1] - ctx->color_off[cs];
      const int mode = !sym ? 0 : (ct == cs ? 2 : 1);
      if (sym && rev)
        hipLaunchKernelGGL(k_tt_far_rev, dim3(nblk(nS, 64), nblk(nT, 4)), dim3(256), lds + kFarRevLds, ctx->stream,
                           pk_, pkl, qr, tg, t2f, colors + ctx->color_off[ct], nT, colors + ctx->color_off[cs], nS,
                           alpha, gsrc, kappa, k0sq9, zo, zt, mode);
      else
        hipLaunchKernelGGL(k_tt_far, dim3(nblk(nS, 64), nblk(nT, 4)), dim3(256), lds, ctx->stream, pk_, pkl, qr, tg,
                           t2f, colors + ctx->color_off[ct], nT, colors + ctx->color_off[cs], nS, alpha, gsrc, kappa,
                           k0sq9, zo, zt, mode);
      LAUNCHCK();
      ++far_launches;
    }
  ctx->fstats.far_launches = far_launches;
  HIPCK(hipEventRecord(ctx->ev3, ctx->stream));
  for (int g = 0; g < C * C; ++g) {
    const int np = ctx->near_off[g + 1] - ctx->near_off[g];
    if (!np) continue;
    hipLaunchKernelGGL(k_tt_near, dim3(nblk(16 * (int64_t)np, 256)), dim3(256), lds, ctx->stream, pk_, pkl, qr, tg, t2f,
                       ctx->ptr<int32_t>(L.near_t) + ctx->near_off[g], ctx->ptr<int32_t>(L.near_s) + ctx->near_off[g],
                       ctx->ptr<int32_t>(L.near_m) + ctx->near_off[g], np, alpha, gsrc, kappa, inveps, k0sq9, zo);
    LAUNCHCK();
  }
  HIPCK(hipEventRecord(ctx->ev4, ctx->stream));
  if (ctx->nface) {
    const FaceGeom *fg = ctx->ptr<FaceGeom>(L.fg);
    // per test colour: the far pairs, then the touching ones from their list
    // (one lane each, so no wave mixes the two kinds)
    for (int ct = 0; ct < C; ++ct) {
      const int nT = ctx->color_off[ct + 1] - ctx->color_off[ct];
      if (grid)
        ;
      else if (sym_face && rev)
        hipLaunchKernelGGL(k_tet_face_rev, dim3(nblk(ctx->nface, 64), nblk(nT, 4)), dim3(256), lds, ctx->stream, pk_, pkl,
                           qr, tg, t2f, colors + ctx->color_off[ct], nT, fg, ctx->nface, alpha, sigma, gsrc, kappa, zo, zt);
      else
        hipLaunchKernelGGL(k_tet_face, dim3(nblk(ctx->nface, 64), nblk(nT, 4)), dim3(256), lds, ctx->stream, pk_, pkl, qr,
                           tg, t2f, colors + ctx->color_off[ct], nT, fg, ctx->nface, alpha, sigma, gsrc, kappa, zo, zt,
                           sym_face ? 1 : 0);
      const int np = ctx->tf_off[ct + 1] - ctx->tf_off[ct];
      if (np)
        hipLaunchKernelGGL(k_tet_face_near, dim3(nblk(np, 256)), dim3(256), lds, ctx->stream, pk_, pkl, qr, tg, t2f,
                           (const int32_t *)ctx->ptr<int32_t>(L.near_tf) + 2 * (int64_t)ctx->tf_off[ct], np, fg,
                           alpha, sigma, zo);
      LAUNCHCK();
    }
    if (ctx->nhalf) {
      for (int cs = 0; cs < C; ++cs) {
        const int nS = ctx->color_off[cs + 1] - ctx->color_off[cs];
        if (!sym_face && !grid)   // (with the staging the far pairs came from k_tet_face)
          hipLaunchKernelGGL(k_face_tet, dim3(nblk(nS, 64), nblk(ctx->nhalf, 4)), dim3(256), lds, ctx->stream, pk_, pkl,
                             qr, fg, ctx->ptr<int32_t>(L.half), ctx->nhalf, tg, t2f, colors + ctx->color_off[cs], nS,
                             gsrc, kappa, zo);
        const int np = ctx->ft_off[cs + 1] - ctx->ft_off[cs];
        if (np)
          hipLaunchKernelGGL(k_face_tet_near, dim3(nblk(np, 256)), dim3(256), lds, ctx->stream, pk_, pkl, qr, fg,
                             ctx->ptr<int32_t>(L.half), tg, t2f,
                             (const int32_t *)ctx->ptr<int32_t>(L.near_ft) + 2 * (int64_t)ctx->ft_off[cs], np, gsrc,
                             kappa, zo);
        LAUNCHCK();
      }
      hipLaunchKernelGGL(k_face_face, dim3(nblk(ctx->nface, 64), nblk(ctx->nhalf, 4)), dim3(256), lds, ctx->stream, pk_,
                         pkl, qr, fg, ctx->ptr<int32_t>(L.half), ctx->nhalf, ctx->nface, sigma, zo);
      LAUNCHCK();
    }
  }
  if (grid) {
    // kernel tables of every sublattice pair (at normal incidence, where g_p
    // is even, of the pairs s <= s' only), scaled by 1/nf for the
    // unnormalised inverse transform, then transformed in place
    const int64_t nf = ctx->grid->g.nf;
    const bool sym = ctx->fill_kx == 0.0 && ctx->fill_ky == 0.0;
    ctx->grid_sym = sym;
    dz *tab = ctx->ptr<dz>(L.gtab);
    hipLaunchKernelGGL(k_grid_table, dim3(nblk(nf, 256), sym ? kGridSymPairs : kGridSub * kGridSub), dim3(256), lds,
                       ctx->stream, pk_, pkl, (const GridGeom *)ctx->ptr<GridGeom>(L.ggeo), ctx->fill_kx, ctx->fill_ky,
                       1.0 / (double)nf, sym ? 1 : 0, tab);
    LAUNCHCK();
    if (hipfftExecZ2Z(sym ? ctx->fft_tab_sym : ctx->fft_tab, (hipfftDoubleComplex *)tab, (hipfftDoubleComplex *)tab,
                      HIPFFT_FORWARD) != HIPFFT_SUCCESS)
      return fail(ctx, VIE_EDEVICE, "grid operator: FFT of the kernel tables failed");
  }
  return VIE_OK;
}

// End of a fill: the staging copy added transposed, ev1, the work counts
// (and, when `timed`, each kernel family's time from the events of
// fill_kernels); the context becomes S_FILLED.
int fill_finish(vie_ctx *ctx, bool timed) {
  const MeshTopology &t = ctx->topo;
  const Layout &L = ctx->L;
  const bool sym = ctx->fill_sym;
  const int rev = ctx->fill_rev;
  if (sym) {
    const dim3 tg2(nblk(t.N, 32), nblk(t.N, 32));
    if (ctx->precision == VIE_MIXED_FP32)
      hipLaunchKernelGGL(k_transpose_add_c, tg2, dim3(256), 0, ctx->stream, ctx->ptr<fz>(L.Z),
                         (const fz *)ctx->ptr<fz>(L.Zt), (int64_t)t.N, L.ld);
    else
      hipLaunchKernelGGL(k_transpose_add_z, tg2, dim3(256), 0, ctx->stream, ctx->ptr<dz>(L.Z),
                         (const dz *)ctx->ptr<dz>(L.Zt), (int64_t)t.N, L.ld);
    LAUNCHCK();
  }
  HIPCK(hipEventRecord(ctx->ev1, ctx->stream));
  HIPCK(hipEventSynchronize(ctx->ev1));
  vie_fill_stats &st = ctx->fstats;
  if (timed) {
    float ms = 0, mfar = 0, mnear = 0, mface = 0;
    HIPCK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    HIPCK(hipEventElapsedTime(&mfar, ctx->ev2, ctx->ev3));
    HIPCK(hipEventElapsedTime(&mnear, ctx->ev3, ctx->ev4));
    HIPCK(hipEventElapsedTime(&mface, ctx->ev4, ctx->ev1));
    ctx->t_fill = ms;
    st.t_fill_ms = ms;
    st.t_far_ms = mfar;
    st.t_near_ms = mnear;
    st.t_face_ms = mface;
  }
  // algorithmic work of the far tet-pair kernel (cost model, FMA = 2 FLOPs):
  // per point pair: separation and wrap 12; per image 27 + 3 deg (X, Y, R^2,
  // rsqrt counted as 8, the fit argument from R, Clenshaw, scale,
  // accumulate); spectral set-up 212 (four sincos counted as 40 each, phase
  // powers; 132 at normal incidence, where the two sincos of kt vanish); per
  // mode 13 + 3 deg (twice the Clenshaw for a complex order); final phase 6.
  // Per tet pair:
  // 16 point pairs + 1200 for moments and the 16-entry scatter (+ 1200 for
  // the swapped pair's scatter when one evaluation serves both).  At oblique
  // incidence one evaluation serving both also forms g_p at the reversed
  // separations (per point pair 4 per propagating order + 10) and the swapped
  // pair's moments (16 x 36 per tet pair).
  double pp = 12 + (rev ? 212 : 132) + 6;
  const PgfTable &tb = *ctx->tab;
  for (int i = 0; i < tb.nimg; ++i) pp += 27 + 3 * tb.img[i].deg;
  int nmodes = 0, ncplx = 0;
  for (int i = 0; i < kPgfTerms; ++i)
    if (tb.mode[i].deg >= 0) {
      ++nmodes;
      ncplx += tb.mode[i].cplx ? 1 : 0;
      pp += 13 + 3 * tb.mode[i].deg * (tb.mode[i].cplx ? 2 : 1) + (tb.mode[i].cplx ? 4 : 0);
    }
  if (sym && rev) pp += 10 + 4 * ncplx;
  int64_t nnear = 0;
  for (auto &v : t.near_t) nnear += (int64_t)v.size();
  // pairs evaluated (near-ness is symmetric and includes every self pair)
  st.far_pairs = sym ? (t.nt * t.nt - nnear) / 2 : t.nt * t.nt - nnear;
  st.near_pairs = nnear;
  st.face_pairs = (int64_t)t.nt * ctx->nface + (int64_t)ctx->nhalf * t.nt + (int64_t)ctx->nhalf * ctx->nface;
  st.far_symmetric = sym ? 1 : 0;
  st.point_pair_flops = pp;
  st.far_flops = (double)st.far_pairs * (16.0 * pp + (sym ? 2400.0 : 1200.0) + (sym && rev ? 16.0 * 36 : 0.0));
  if (ctx->precision == VIE_GRID_FP64) {
    // no far pair is evaluated: the far part lives in the FFT tables; only the
    // touching face pairs of the face-face kernel write anything
    st.far_pairs = 0;
    st.far_flops = 0;
    st.face_pairs = (int64_t)ctx->nhalf * ctx->nface;
  }
  st.nimg = tb.nimg;
  st.nmode = nmodes;
  ctx->state = S_FILLED;
  ctx->factored = false;
  return VIE_OK;
}

}  // namespace vie

extern "C" {

int vie_fill(vie_ctx *ctx, double lambda_nm, double theta, double phi, const vie_c128 *eps_per_tet, int precision) {
  if (int rc = fill_prepare(ctx, lambda_nm, theta, phi, eps_per_tet, precision)) return rc;
  if (int rc = fill_kernels(ctx)) return rc;
  return fill_finish(ctx, true);
}

// ---------------------------------------------------------------- factor
}  // extern "C"

namespace vie {

enum LuKernel { LU_PIVOT, LU_COL, LU_SWAP, LU_TRSM, LU_GEMM, LU_GEMM2, LU_TSEL, LU_TFIN };

// One launch of an LU kernel (FP32 factors if f32) on stream sm over every
// domain with blocks_of(d) > 0 thread blocks (kLuMaxDom domains per launch;
// more domains take more launches).  (GEMM: column tiles gcol0 .. gcol0 +
// gcols - 1 of the trailing matrix, gcols <= 0 for all from gcol0.)
template <typename BlocksOf>
void lu_launch(bool f32, hipStream_t sm, LuKernel k, const std::vector<LuDom> &doms, int j, int k0, BlocksOf blocks_of,
               int all_cols = 0, int gcol0 = 0, int gcols = 0, int c_lo = 0, int c_hi = 0) {
  LuStep st{};
  st.j = j;
  st.k0 = k0;
  st.all_cols = all_cols;
  st.gcol0 = gcol0;
  st.gcols = gcols;
  st.c_lo = c_lo;
  st.c_hi = c_hi;
  int total = 0;
  auto flush = [&]() {
    if (st.ndom == 0) return;
    switch (k) {
      case LU_PIVOT:
        if (f32) hipLaunchKernelGGL(k_lu_pivot_c, dim3(total), dim3(1024), 0, sm, st);
        else hipLaunchKernelGGL(k_lu_pivot_z, dim3(total), dim3(1024), 0, sm, st);
        break;
      case LU_COL:
        if (f32) hipLaunchKernelGGL(k_lu_col_c, dim3(total), dim3(256), 0, sm, st);
        else hipLaunchKernelGGL(k_lu_col_z, dim3(total), dim3(256), 0, sm, st);
        break;
      case LU_SWAP:
        if (f32) hipLaunchKernelGGL(k_lu_swap_c, dim3(total), dim3(256), 0, sm, st);
        else hipLaunchKernelGGL(k_lu_swap_z, dim3(total), dim3(256), 0, sm, st);
        break;
      case LU_TRSM:
        if (f32) hipLaunchKernelGGL(k_lu_trsm_c, dim3(total), dim3(256), 0, sm, st);
        else hipLaunchKernelGGL(k_lu_trsm_z, dim3(total), dim3(256), 0, sm, st);
        break;
      case LU_GEMM:
        if (f32) hipLaunchKernelGGL(k_lu_gemm_c, dim3(total), dim3(256), 0, sm, st);
        else hipLaunchKernelGGL(k_lu_gemm_z, dim3(total), dim3(256), 0, sm, st);
        break;
      case LU_GEMM2:
        if (f32) hipLaunchKernelGGL(k_lu_gemm2_c, dim3(total), dim3(kGemm2Threads), 0, sm, st);
        else hipLaunchKernelGGL(k_lu_gemm2_z, dim3(total), dim3(kGemm2Threads), 0, sm, st);
        break;
      case LU_TSEL:
        if (f32) hipLaunchKernelGGL(k_lu_tsel_c, dim3(total), dim3(kTsRowsC * kTsLprC), 0, sm, st);
        else hipLaunchKernelGGL(k_lu_tsel_z, dim3(total), dim3(kTsRowsZ * kTsLprZ), 0, sm, st);
        break;
      case LU_TFIN:
        if (f32) hipLaunchKernelGGL(k_lu_tfin_c, dim3(total), dim3(256), 0, sm, st);
        else hipLaunchKernelGGL(k_lu_tfin_z, dim3(total), dim3(256), 0, sm, st);
        break;
    }
    st.ndom = 0;
    total = 0;
  };
  for (size_t d = 0; d < doms.size(); ++d) {
    const int nb = blocks_of((int)d);
    if (nb <= 0) continue;
    st.d[st.ndom] = doms[d];
    st.d[st.ndom].first_block = total;
    total += nb;
    if (++st.ndom == kLuMaxDom) flush();
  }
  flush();
}

}  // namespace vie

extern "C" {

}  // extern "C"

namespace vie {

// The domain descriptors of the block factorisation (Sec. 2.3, Eq. 6) and
// each diagonal block A_dd copied (with the FP64 near part in mixed
// precision) into the factor storage; records ev0.
int factor_prepare(vie_ctx *ctx, std::vector<LuDom> &doms) {
  if (int r = check(ctx, S_FILLED, "vie_precond_factor")) return r;
  if (ctx->precision == VIE_GRID_FP64)
    return fail(ctx, VIE_EINVAL, "VIE_GRID_FP64 stores no diagonal blocks to factor (solve with VIE_OPT_PRECOND 1)");
  // the factors of an earlier factorisation of this fill are overwritten from
  // here on: until this one succeeds, no solve or apply may use them
  ctx->factored = false;
  const MeshTopology &t = ctx->topo;
  for (int d = 0; d < t.ndom; ++d)
    if (t.dend[d] - t.dstart[d] > (int64_t)kTrsvChunksMax * kTrsvSumCols)
      return fail(ctx, VIE_EINVAL, "domain %d has %lld unknowns; the block preconditioner takes at most %d", d,
                  (long long)(t.dend[d] - t.dstart[d]), kTrsvChunksMax * kTrsvSumCols);
  HIPCK(hipSetDevice(ctx->device));
  const Layout &L = ctx->L;
  const ZOut zo = zout(ctx);
  const bool f32 = fp32_factors(ctx);
  int32_t *ipiv = ctx->ptr<int32_t>(L.ipiv), *info = ctx->ptr<int32_t>(L.info);
  HIPCK(hipEventRecord(ctx->ev0, ctx->stream));
  HIPCK(hipMemsetAsync(info, 0, 4 * t.ndom, ctx->stream));
  ctx->upd_n = 0;
  doms.assign(t.ndom, LuDom{});
  int64_t poff = 0, pvoff = 0;
  for (int d = 0; d < t.ndom; ++d) {
    const int n = (int)(t.dend[d] - t.dstart[d]);
    LuDom &D = doms[d];
    D.A = factor_ptr(ctx, L.F, L.foff[d]);
    D.ld = L.fld[d];
    D.n = n;
    D.ipiv = ipiv + poff;
    D.info = info + d;
    D.rpiv = ctx->ws + L.rpiv.off + 16 * (size_t)d;
    D.pval = ctx->ptr<double>(L.lupv) + pvoff;
    D.pidx = ctx->ptr<int32_t>(L.lupi) + pvoff;
    D.counter = ctx->ptr<int>(L.lucnt) + d;
    D.cand = ctx->ptr<int32_t>(L.tcand) + L.toff[d] * kLuNB;
    D.tcnt = ctx->ptr<int>(L.ttcnt) + L.toff[d];
    D.tblk = factor_ptr(ctx, L.tblk, (int64_t)d * kLuNB * kLuNB);
    poff += n;
    pvoff += nblk(n, kColRows);
    if (n == 0) continue;
    const dim3 cg(nblk(n, 256), std::min(n, 32768)), ng(nblk(n, 256)), b256(256);
    if (f32) {
      hipLaunchKernelGGL(k_copy_block_c, cg, b256, 0, ctx->stream, zo, (int64_t)t.dstart[d], n, (fz *)D.A, D.ld);
      if (!zo.Z) hipLaunchKernelGGL(k_add_near_c, ng, b256, 0, ctx->stream, zo, (int64_t)t.dstart[d], n, (fz *)D.A, D.ld);
    } else {
      hipLaunchKernelGGL(k_copy_block_z, cg, b256, 0, ctx->stream, zo, (int64_t)t.dstart[d], n, (dz *)D.A, D.ld);
      if (!zo.Z) hipLaunchKernelGGL(k_add_near_z, ng, b256, 0, ctx->stream, zo, (int64_t)t.dstart[d], n, (dz *)D.A, D.ld);
    }
    LAUNCHCK();
  }
  return VIE_OK;
}

// Right-looking blocked LU of every domain in `doms` (any number of
// contexts' domains, all FP32 or all FP64 factors), advanced together on
// `stream`.
//
// Tournament pivoting (lu_pivot 0) takes the panels two at a time, so that
// the bulk trailing update has K = 128 (k_lu_gemm2).  A pair at k0 (panels
// a = [k0, k0+64), b = [k0+64, k0+128)) is done in two phases:
//   * panels: a's tournament, its row swaps on the pair's columns, L21 and
//     the U12 rows of a over b's columns; a's update of b's columns; b's
//     tournament, its swaps on the pair's columns, L21;
//   * rest: both panels' swaps on every other column (a's, then b's), a's
//     U12 right of the pair, a's update of b's rows right of the pair (a
//     64-row strip), b's U12; then every row and column right of the pair
//     takes both panels' update at once.
// The panel phase of the next pair touches only the next pair's columns, so
// it runs on the side stream while the bulk update of the current pair runs
// (after that update's first 128 columns, the next pair's, are done); the
// rest phase waits for it.  Column-by-column partial pivoting (lu_pivot 1)
// advances one panel at a time with the K = 64 update.
int factor_panels(vie_ctx *ctx, std::vector<LuDom> &doms, bool f32, int lu_pivot, hipStream_t stream,
                  hipStream_t side, hipEvent_t ev_la, hipEvent_t ev_ts) {
  int maxn = 0;
  for (const LuDom &D : doms) maxn = std::max(maxn, D.n);
  const int ts_rows = f32 ? kTsRowsC : kTsRowsZ;
  auto tsel = [&](int kp, hipStream_t sm) {
    lu_launch(f32, sm, LU_TSEL, doms, kp, kp, [&](int d) { return doms[d].n > kp ? (int)nblk(doms[d].n - kp, ts_rows) : 0; });
  };
  auto jb_of = [&](int d, int k0) { return std::min(kLuNB, doms[d].n - k0); };
  // single-panel update tiles of domain d at panel k0: row tiles (all, or grows)
  // x column tiles gcol0 .. (gcols <= 0: to the end)
  auto gemm_blocks = [&](int d, int k0, int gcol0, int gcols, int grows = 0) {
    const int rest = doms[d].n > k0 ? doms[d].n - k0 - std::min(kLuNB, doms[d].n - k0) : 0;
    const int nt = (int)((rest + 63) / 64);
    const int nc = gcols > 0 ? std::min(gcols, nt - gcol0) : nt - gcol0;
    const int nr = grows > 0 ? std::min(grows, nt) : nt;
    return rest > 0 && nc > 0 ? nr * nc : 0;
  };
  // row swaps of panel k0 on the columns that mode (k_lu_swap) selects
  auto swap_blocks = [&](int k0, int mode, int c_lo, int c_hi) {
    return [&, k0, mode, c_lo, c_hi](int d) {
      const int n = doms[d].n;
      if (n <= k0) return 0;
      if (mode == 2) return (int)nblk(std::max(0, std::min(c_hi, n) - c_lo), 256);
      return (int)nblk(n, 256);
    };
  };
  auto tfin_blocks = [&](int k0) {
    return [&, k0](int d) {
      if (doms[d].n <= k0) return 0;
      const int rest = doms[d].n - k0 - jb_of(d, k0);
      return rest > 0 ? (int)nblk(rest, kColRows) : 1;
    };
  };
  // U12 of panel k0 on the columns [c_lo, c_hi) right of it (c_hi <= 0: all of them)
  auto trsm_blocks = [&](int k0, int c_lo = 0, int c_hi = 0) {
    return [&, k0, c_lo, c_hi](int d) {
      const int n = doms[d].n;
      if (n <= k0) return 0;
      const int beg = c_hi > 0 ? std::max(c_lo, k0 + jb_of(d, k0)) : k0 + jb_of(d, k0);
      const int end = c_hi > 0 ? std::min(c_hi, n) : n;
      return end > beg ? (int)nblk(end - beg, kColRows) : 0;
    };
  };
  if (lu_pivot == 0) {
    const int tm = 128, tn = f32 ? 128 : 64;   // k_lu_gemm2 tile
    // pair-update tiles of domain d at k0 (column tiles gcol0 .., gcols <= 0: to the end), padded to 8
    auto gemm2_blocks = [&](int d, int k0, int gcol0, int gcols) {
      const int rest = doms[d].n - k0 - 2 * kLuNB;
      if (rest <= 0) return 0;
      const int nr = (rest + tm - 1) / tm, ntc = (rest + tn - 1) / tn;
      const int nc = gcols > 0 ? std::min(gcols, ntc - gcol0) : ntc - gcol0;
      return nc > 0 ? 8 * (int)nblk(nr * nc, 8) : 0;
    };
    // each bulk update between an event pair of ctx's pool (its device time)
    auto timed_gemm2 = [&](int k0, int gcol0, int gcols) -> int {
      if ((int)ctx->upd_ev.size() < 2 * (ctx->upd_n + 1)) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCK(hipEventCreate(&e0));
        HIPCK(hipEventCreate(&e1));
        ctx->upd_ev.push_back(e0);
        ctx->upd_ev.push_back(e1);
      }
      HIPCK(hipEventRecord(ctx->upd_ev[2 * ctx->upd_n], stream));
      lu_launch(f32, stream, LU_GEMM2, doms, k0, k0, [&](int d) { return gemm2_blocks(d, k0, gcol0, gcols); }, 0, gcol0,
                gcols);
      HIPCK(hipEventRecord(ctx->upd_ev[2 * ctx->upd_n + 1], stream));
      ++ctx->upd_n;
      return VIE_OK;
    };
    constexpr int kBig = 1 << 30;
    auto panels = [&](int k0, hipStream_t sm) {
      const int kb = k0 + kLuNB, pe = k0 + 2 * kLuNB;
      tsel(k0, sm);
      lu_launch(f32, sm, LU_SWAP, doms, k0, k0, swap_blocks(k0, 2, k0, pe), 2, 0, 0, k0, pe);
      lu_launch(f32, sm, LU_TFIN, doms, k0, k0, tfin_blocks(k0));
      if (kb < maxn) {
        lu_launch(f32, sm, LU_TRSM, doms, k0, k0, trsm_blocks(k0, kb, pe), 0, 0, 0, kb, pe);
        lu_launch(f32, sm, LU_GEMM, doms, k0, k0, [&](int d) { return gemm_blocks(d, k0, 0, 1); }, 0, 0, 1);
        tsel(kb, sm);
        lu_launch(f32, sm, LU_SWAP, doms, kb, kb, swap_blocks(kb, 2, k0, pe), 2, 0, 0, k0, pe);
        lu_launch(f32, sm, LU_TFIN, doms, kb, kb, tfin_blocks(kb));
      }
    };
    auto rest = [&](int k0) {
      const int kb = k0 + kLuNB, pe = k0 + 2 * kLuNB;
      lu_launch(f32, stream, LU_SWAP, doms, k0, k0, swap_blocks(k0, 3, k0, pe), 3, 0, 0, k0, pe);
      if (kb < maxn) lu_launch(f32, stream, LU_SWAP, doms, kb, kb, swap_blocks(kb, 3, k0, pe), 3, 0, 0, k0, pe);
      lu_launch(f32, stream, LU_TRSM, doms, k0, k0, trsm_blocks(k0, pe, kBig), 0, 0, 0, pe, kBig);
      if (kb < maxn) {
        lu_launch(f32, stream, LU_GEMM, doms, k0, k0, [&](int d) { return gemm_blocks(d, k0, 1, 0, 1); }, 0, 1, 0);
        lu_launch(f32, stream, LU_TRSM, doms, kb, kb, trsm_blocks(kb, pe, kBig), 0, 0, 0, pe, kBig);
      }
    };
    panels(0, stream);
    for (int k0 = 0; k0 < maxn; k0 += 2 * kLuNB) {
      const int next = k0 + 2 * kLuNB;
      if (k0 > 0) HIPCK(hipStreamWaitEvent(stream, ev_ts, 0));   // this pair's panels, factored on the side stream
      rest(k0);
      if (next < maxn) {
        if (int rc = timed_gemm2(k0, 0, 2 * kLuNB / tn)) return rc;   // the next pair's columns first
        HIPCK(hipEventRecord(ev_la, stream));
        HIPCK(hipStreamWaitEvent(side, ev_la, 0));
        panels(next, side);
        HIPCK(hipEventRecord(ev_ts, side));
        if (int rc = timed_gemm2(k0, 2 * kLuNB / tn, 0)) return rc;
      }
      LAUNCHCK();
    }
    return VIE_OK;
  }
  for (int k0 = 0; k0 < maxn; k0 += kLuNB) {
    lu_launch(f32, stream, LU_PIVOT, doms, k0, k0, [&](int d) { return doms[d].n > k0 ? 1 : 0; });
    for (int j = k0; j < k0 + kLuNB && j < maxn; ++j)
      lu_launch(f32, stream, LU_COL, doms, j, k0, [&](int d) {
        const int n = doms[d].n;
        return (n > k0 && j < k0 + jb_of(d, k0) && n - j - 1 > 0) ? (int)nblk(n - j - 1, kColRows) : 0;
      });
    lu_launch(f32, stream, LU_SWAP, doms, k0, k0, swap_blocks(k0, 0, 0, 0));
    lu_launch(f32, stream, LU_TRSM, doms, k0, k0, trsm_blocks(k0));
    lu_launch(f32, stream, LU_GEMM, doms, k0, k0, [&](int d) { return gemm_blocks(d, k0, 0, 0); });
    LAUNCHCK();
  }
  return VIE_OK;
}

// After the panels: the inverses of the 256-row diagonal blocks of L and U and
// the coupling blocks of the triangular solves, the pivots read back (zero pivot: VIE_ESINGULAR), each block's row
// permutation built on the host and uploaded; the context becomes S_FACTORED.
int factor_finish(vie_ctx *ctx, const std::vector<LuDom> &doms) {
  const MeshTopology &t = ctx->topo;
  const Layout &L = ctx->L;
  const bool f32 = fp32_factors(ctx);
  int32_t *ipiv = ctx->ptr<int32_t>(L.ipiv), *perm = ctx->ptr<int32_t>(L.perm), *info = ctx->ptr<int32_t>(L.info);
  for (int d = 0; d < t.ndom; ++d) {
    const int n = doms[d].n;
    if (n == 0) continue;
    const int nbk = (n + kTrsvNB - 1) / kTrsvNB;
    const int64_t mlast = n - (int64_t)(nbk - 1) * kTrsvNB;
    void *DL = factor_ptr(ctx, L.dinv, L.doff[d]);
    void *DU = factor_ptr(ctx, L.dinv, L.doff[d] + (int64_t)(nbk - 1) * kTrsvNB * kTrsvNB + mlast * mlast);
    void *GL = factor_ptr(ctx, L.gcpl, L.goff[d]);
    void *GU = factor_ptr(ctx, L.gcpl, L.goff[d] + (int64_t)(nbk - 1) * kTrsvNB * kTrsvNB);
    const dim3 ig(nbk, kTrsvNB / kInvColsH), ib(4 * kInvColsH);   // kInvColsH columns of one inverse per block
    const dim3 cg(nbk - 1, (kTrsvNB / 64) * (kTrsvNB / 64)), cb(256);   // 64 x 64 tiles of each coupling block
    if (f32) {
      const fz *A = (const fz *)doms[d].A;
      hipLaunchKernelGGL(k_diag_inv_c, ig, ib, 0, ctx->stream, A, doms[d].ld, n, kTrsvNB, 1, (fz *)DL);
      hipLaunchKernelGGL(k_diag_inv_c, ig, ib, 0, ctx->stream, A, doms[d].ld, n, kTrsvNB, 0, (fz *)DU);
      if (nbk > 1) {
        hipLaunchKernelGGL(k_trsv_coupling_c, cg, cb, 0, ctx->stream, A, doms[d].ld, n, 1, (const fz *)DL, (fz *)GL);
        hipLaunchKernelGGL(k_trsv_coupling_c, cg, cb, 0, ctx->stream, A, doms[d].ld, n, 0, (const fz *)DU, (fz *)GU);
      }
    } else {
      const dz *A = (const dz *)doms[d].A;
      hipLaunchKernelGGL(k_diag_inv_z, ig, ib, 0, ctx->stream, A, doms[d].ld, n, kTrsvNB, 1, (dz *)DL);
      hipLaunchKernelGGL(k_diag_inv_z, ig, ib, 0, ctx->stream, A, doms[d].ld, n, kTrsvNB, 0, (dz *)DU);
      if (nbk > 1) {
        hipLaunchKernelGGL(k_trsv_coupling_z, cg, cb, 0, ctx->stream, A, doms[d].ld, n, 1, (const dz *)DL, (dz *)GL);
        hipLaunchKernelGGL(k_trsv_coupling_z, cg, cb, 0, ctx->stream, A, doms[d].ld, n, 0, (const dz *)DU, (dz *)GU);
      }
    }
    LAUNCHCK();
  }
  HIPCK(hipEventRecord(ctx->ev1, ctx->stream));
  HIPCK(hipMemcpyAsync(ctx->pinned, info, 4 * t.ndom, hipMemcpyDeviceToHost, ctx->stream));
  // pivots and permutation staged in pinned memory, or pageable memory after a no-allocation bind
  int32_t *stage = ctx->pin_piv_n >= t.N ? ctx->pin_piv : ctx->piv_host.data();
  HIPCK(hipMemcpyAsync(stage, ipiv, 4 * (size_t)t.N, hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  float ms = 0;
  HIPCK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  ctx->t_factor = ms;
  {
    vie_factor_stats &fs = ctx->facstats;
    fs = vie_factor_stats{};
    fs.t_factor_ms = ms;
    for (int i = 0; i < ctx->upd_n; ++i) {
      float e = 0;
      HIPCK(hipEventElapsedTime(&e, ctx->upd_ev[2 * i], ctx->upd_ev[2 * i + 1]));
      fs.t_update_ms += e;
    }
    fs.update_launches = ctx->upd_n;
    for (const LuDom &D : doms) {
      const double n = D.n;
      fs.factor_flops += 8.0 / 3.0 * n * n * n;
      if (ctx->upd_n)
        for (int64_t k0 = 0; k0 + 2 * kLuNB < D.n; k0 += 2 * kLuNB) {
          const double m = (double)(D.n - k0 - 2 * kLuNB);
          fs.update_flops += 8.0 * m * m * (2 * kLuNB);
        }
    }
  }
  const int32_t *inf = reinterpret_cast<const int32_t *>(ctx->pinned);
  for (int d = 0; d < t.ndom; ++d)
    if (inf[d] < 0) return fail(ctx, VIE_EDEVICE, "tournament pivoting of block %d chose a row outside the panel", d);
    else if (inf[d]) return fail(ctx, VIE_ESINGULAR, "zero pivot in block %d at column %d", d, inf[d] - 1);
  // row permutation of each block from its swaps (sequential by nature: done
  // on the host from the pivots read back, then uploaded for the applies)
  int32_t *hp = stage + t.N;
  for (int d = 0; d < t.ndom; ++d) {
    const int64_t o = t.dstart[d], n = t.dend[d] - t.dstart[d];
    const int32_t *ip = stage + o;
    int32_t *pm = hp + o;
    for (int64_t i = 0; i < n; ++i) pm[i] = (int32_t)i;
    for (int64_t j = 0; j < n; ++j) {
      const int32_t p = ip[j];
      if (p < j || p >= n) return fail(ctx, VIE_EDEVICE, "pivot %d of column %lld in block %d out of range", p,
                                      (long long)j, d);
      std::swap(pm[j], pm[p]);
    }
  }
  HIPCK(hipMemcpyAsync(perm, hp, 4 * (size_t)t.N, hipMemcpyHostToDevice, ctx->stream));
  ctx->state = S_FACTORED;
  ctx->factored = true;
  return VIE_OK;
}

}  // namespace vie

extern "C" {

int vie_precond_factor(vie_ctx *ctx) {
  std::vector<LuDom> doms;
  if (int rc = factor_prepare(ctx, doms)) return rc;
  if (!ctx->side) HIPCK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
  if (int rc = factor_panels(ctx, doms, fp32_factors(ctx), ctx->lu_pivot, ctx->stream, ctx->side, ctx->ev_la,
                             ctx->ev_ts))
    return rc;
  return factor_finish(ctx, doms);
}

}  // extern "C"

// ---------------------------------------------------------------- solve
namespace vie {

// The step list of the blocked triangular solves (L sweep, then U sweep) for
// nv (1 or 2) right-hand sides; step k advances every domain (kTrsvMaxDom per
// entry) by one diagonal block, so the step count follows the largest domain.
// Step k of a domain with nbk blocks (numbered in the sweep's order) solves
// block k and forms the chunk sums of block k + 1 over the blocks <= k - 2,
// in work items of ctx->trsv_kc columns.
std::vector<TrsvStep> trsv_plan(vie_ctx *ctx, int nv, dz *const *out, dz *const *s1, dz *const *s2) {
  const MeshTopology &t = ctx->topo;
  const Layout &L = ctx->L;
  const int kc = ctx->trsv_kc;
  int maxnbk = 0;
  for (int d = 0; d < t.ndom; ++d) maxnbk = std::max(maxnbk, (int)((t.dend[d] - t.dstart[d] + kTrsvNB - 1) / kTrsvNB));
  // r of a block: per domain two buffers (steps alternate) of two vectors
  dz *rr = ctx->ptr<dz>(L.trr);
  auto rbuf = [&](int d, int k) { return rr + ((int64_t)d * 4 + 2 * (k & 1)) * kTrsvNB; };
  // chunk sums: the same alternation, in the domain's region of L.tbsum
  dz *bsum = ctx->ptr<dz>(L.tbsum);
  auto bbuf = [&](int d, int k) {
    const int64_t n = t.dend[d] - t.dstart[d];
    return bsum + L.boff[d] + (int64_t)(k & 1) * 2 * kTrsvNB * trsv_bsum_stride(n);
  };
  std::vector<TrsvStep> plan;
  // L sweep: rhs s1, solution s2; U sweep: rhs s2, solution out.
  for (int lower = 1; lower >= 0; --lower) {
    // steps 0 .. maxnbk-1 advance the solves; step maxnbk stores each
    // domain's last diagonal block
    for (int k = 0; k <= maxnbk; ++k) {
      TrsvStep st{};
      st.lower = lower;
      auto push = [&]() {
        if (st.ndom == 0) return;
        st.chain_blocks = trsv_number_items(st.d, st.ndom, &st.z_end, &st.total_blocks);
        plan.push_back(st);
        st = TrsvStep{};
        st.lower = lower;
      };
      for (int d = 0; d < t.ndom; ++d) {
        const int n = (int)(t.dend[d] - t.dstart[d]);
        const int nbk = (n + kTrsvNB - 1) / kTrsvNB;
        if (nbk == 0 || (k >= nbk && k < maxnbk)) continue;
        const int64_t off = t.dstart[d];
        const int64_t mlast = n - (int64_t)(nbk - 1) * kTrsvNB;
        const int64_t isz = (int64_t)(nbk - 1) * kTrsvNB * kTrsvNB + mlast * mlast;   // inverses of one sweep
        TrsvDom &D = st.d[st.ndom];
        D.F = factor_ptr(ctx, L.F, L.foff[d]);
        D.ld = L.fld[d];
        D.n = n;
        for (int q = 0; q < nv; ++q) {
          D.rhs[q] = (lower ? s1[q] : s2[q]) + off;
          D.sol[q] = (lower ? s2[q] : out[q]) + off;
        }
        D.bst = trsv_bsum_stride(n);
        // inverse of matrix block b of this sweep, and its coupling block (L: b >= 1, U: b <= nbk - 2)
        auto invof = [&](int b) {
          return factor_ptr(ctx, L.dinv, L.doff[d] + (lower ? 0 : isz) + (int64_t)b * kTrsvNB * kTrsvNB);
        };
        auto cplof = [&](int b) {
          const int64_t slot = lower ? b - 1 : (nbk - 1) + b;
          return factor_ptr(ctx, L.gcpl, L.goff[d] + slot * kTrsvNB * kTrsvNB);
        };
        if (k == maxnbk) {
          // the end of the domain's sweep: the solution of its last block
          const int bk = lower ? nbk - 1 : 0;
          D.pb0 = bk * kTrsvNB;
          D.pm = std::min(kTrsvNB, n - D.pb0);
          D.cb0 = D.cm = D.nb0 = D.nm = 0;
          D.rin = rbuf(d, nbk - 1);
          D.rout = nullptr;
          D.INV = invof(bk);
          D.G = D.F;   // (unused: no reduction items)
          D.gld = 0;
          D.bsum_in = D.bsum_out = bbuf(d, 0);
          if (++st.ndom == kTrsvMaxDom) push();
          continue;
        }
        // step k reduces block bk; blocks bk -+ 1 and bk -+ 2 (in the sweep's order) come before it
        D.rin = rbuf(d, k - 1);
        D.rout = rbuf(d, k);
        const int bk = lower ? k : nbk - 1 - k;
        const int dir = lower ? -1 : 1;
        D.nb0 = bk * kTrsvNB;
        D.nm = std::min(kTrsvNB, n - D.nb0);
        D.pb0 = k >= 1 ? (bk + dir) * kTrsvNB : 0;
        D.pm = k >= 1 ? std::min(kTrsvNB, n - D.pb0) : 0;
        D.cb0 = k >= 2 ? (bk + 2 * dir) * kTrsvNB : 0;
        D.cm = k >= 2 ? std::min(kTrsvNB, n - D.cb0) : 0;
        // (k = 0: no previous block; G then reads one valid entry, masked)
        D.G = k >= 1 ? cplof(bk) : D.F;
        D.gld = k >= 1 ? kTrsvNB : 0;
        D.INV = invof(k >= 1 ? bk + dir : bk);
        // block k's chunk sums over the blocks <= k - 3, from step k - 1
        D.bsum_in = bbuf(d, k - 1);
        const int kin = k >= 3 ? (lower ? (k - 2) * kTrsvNB : n - (nbk + 2 - k) * kTrsvNB) : 0;
        D.nci = (kin + kTrsvSumCols - 1) / kTrsvSumCols;
        // block k + 1's chunk sums over the blocks <= k - 2 (columns [bc0, bc0 + bk))
        D.bsum_out = bbuf(d, k);
        if (k >= 2 && k + 1 < nbk) {
          const int tb = lower ? k + 1 : nbk - 2 - k;
          D.br0 = tb * kTrsvNB;
          D.brm = std::min(kTrsvNB, n - D.br0);
          D.bc0 = lower ? 0 : (nbk + 1 - k) * kTrsvNB;
          D.bk = lower ? (k - 1) * kTrsvNB : n - D.bc0;
          D.nrg = (D.brm + 15) / 16;
          D.nco = (D.bk + kc - 1) / kc;
        }
        if (++st.ndom == kTrsvMaxDom) push();
      }
      push();
    }
  }
  return plan;
}

void launch_trsv_step(vie_ctx *ctx, const TrsvStep &st, int nv) {
  const dim3 g(st.total_blocks), b(1024);
  const bool w = ctx->trsv_kc == 2048;
  if (nv == 2) {
    if (fp32_factors(ctx)) {
      if (w) hipLaunchKernelGGL(k_trsv_step2_c_k2048, g, b, 0, ctx->stream, st);
      else hipLaunchKernelGGL(k_trsv_step2_c_k1024, g, b, 0, ctx->stream, st);
    } else {
      if (w) hipLaunchKernelGGL(k_trsv_step2_z_k2048, g, b, 0, ctx->stream, st);
      else hipLaunchKernelGGL(k_trsv_step2_z_k1024, g, b, 0, ctx->stream, st);
    }
    return;
  }
  if (fp32_factors(ctx)) {
    if (w) hipLaunchKernelGGL(k_trsv_step_c_k2048, g, b, 0, ctx->stream, st);
    else hipLaunchKernelGGL(k_trsv_step_c_k1024, g, b, 0, ctx->stream, st);
  } else {
    if (w) hipLaunchKernelGGL(k_trsv_step_z_k2048, g, b, 0, ctx->stream, st);
    else hipLaunchKernelGGL(k_trsv_step_z_k1024, g, b, 0, ctx->stream, st);
  }
}

const void *coop_kernel(const vie_ctx *ctx) {
  const bool w = ctx->trsv_kc == 2048;
  if (fp32_factors(ctx)) return w ? (const void *)k_trsv_coop_c_k2048 : (const void *)k_trsv_coop_c_k1024;
  return w ? (const void *)k_trsv_coop_z_k2048 : (const void *)k_trsv_coop_z_k1024;
}

// Run the plan as one cooperative launch: the plan is uploaded once per
// (vectors, variant) and cached in the workspace; the grid is the number of
// thread blocks that are co-resident on the device (the runtime refuses a
// larger cooperative grid).
int launch_trsv_coop(vie_ctx *ctx, const std::vector<TrsvStep> &plan, const dz *v, const dz *out, const dz *s1,
                     const dz *s2) {
  const Layout &L = ctx->L;
  const void *kern = coop_kernel(ctx);
  if (ctx->coop_grid <= 0) {
    int per_cu = 0, cus = 0;
    HIPCK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 1024, 0));
    HIPCK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    ctx->coop_grid = std::max(1, per_cu) * std::max(1, cus);
  }
  if ((int)plan.size() > L.plan_steps) return fail(ctx, VIE_EINVAL, "triangular-solve plan too long");
  const vie_ctx::CoopPlan *cp = nullptr;
  for (const auto &p : ctx->plans)
    if (p.v == v && p.out == out && p.s1 == s1 && p.s2 == s2 && p.kc == ctx->trsv_kc) cp = &p;
  if (!cp) {
    if ((int)ctx->plans.size() == kMaxPlans) ctx->plans.clear();
    vie_ctx::CoopPlan p{v, out, s1, s2, ctx->trsv_kc, (int)plan.size(),
                        L.plans.off + ctx->plans.size() * sizeof(TrsvStep) * (size_t)L.plan_steps};
    HIPCK(hipMemcpyAsync(ctx->ws + p.off, plan.data(), sizeof(TrsvStep) * plan.size(), hipMemcpyHostToDevice,
                         ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));   // the host plan goes out of scope
    ctx->plans.push_back(p);
    cp = &ctx->plans.back();
  }
  const TrsvStep *dplan = reinterpret_cast<const TrsvStep *>(ctx->ws + cp->off);
  int nsteps = cp->nsteps;
  void *args[] = {(void *)&dplan, (void *)&nsteps};
  HIPCK(hipLaunchCooperativeKernel(kern, dim3(ctx->coop_grid), dim3(1024), args, 0, ctx->stream));
  return VIE_OK;
}

// z_q = M^{-1} v_q (q < nv, nv = 1 or 2) for the block-diagonal
// preconditioner: per domain, permute by the pivots, then L y = P v and
// U z = y by blocked triangular solves, either one launch per step (the launch
// count follows the largest domain; with nv = 2 each launch serves both
// vectors from one pass over the factors) or, for one vector, all steps in one
// cooperative launch (VIE_OPT_TRSV_COOP, not under graph capture).
int apply_minv_n(vie_ctx *ctx, int nv, const dz *const *v, dz *const *out, dz *const *s1, dz *const *s2) {
  const MeshTopology &t = ctx->topo;
  const Layout &L = ctx->L;
  const int32_t *perm = ctx->ptr<int32_t>(L.perm);
  for (int q = 0; q < nv; ++q) {
    int64_t poff = 0;
    for (int d = 0; d < t.ndom; ++d) {
      const int n = (int)(t.dend[d] - t.dstart[d]);
      if (n > 0)
        hipLaunchKernelGGL(k_permute, dim3(nblk(n, 256)), dim3(256), 0, ctx->stream, n, (int64_t)t.dstart[d],
                           perm + poff, v[q], s1[q]);
      poff += n;
    }
  }
  if (ctx->trsv_coop && !ctx->capturing) {
    for (int q = 0; q < nv; ++q) {
      const std::vector<TrsvStep> plan = trsv_plan(ctx, 1, out + q, s1 + q, s2 + q);
      if (int rc = launch_trsv_coop(ctx, plan, v[q], out[q], s1[q], s2[q])) return rc;
    }
  } else {
    const std::vector<TrsvStep> plan = trsv_plan(ctx, nv, out, s1, s2);
    for (const TrsvStep &st : plan) launch_trsv_step(ctx, st, nv);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "preconditioner apply: %s", hipGetErrorString(e));
  return VIE_OK;
}

int apply_minv(vie_ctx *ctx, const dz *v, dz *out, dz *s1, dz *s2) { return apply_minv_n(ctx, 1, &v, &out, &s1, &s2); }

// dst = ||w|| with the partial sums in the scratch of Krylov process k
int norm_to(vie_ctx *ctx, int k, const dz *w, int64_t N, double *dst) {
  const Layout &L = ctx->L;
  hipLaunchKernelGGL(k_norm2, dim3(kRedBlocks), dim3(256), 0, ctx->stream, w, N, ctx->ptr<double>(L.K[k].npart));
  hipLaunchKernelGGL(k_norm_reduce, dim3(1), dim3(1), 0, ctx->stream, (const double *)ctx->ptr<double>(L.K[k].npart),
                     kRedBlocks, dst);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "norm: %s", hipGetErrorString(e));
  return VIE_OK;
}

int read_scalar(vie_ctx *ctx, const double *dev, double *host) {
  hipError_t e = hipMemcpyAsync(ctx->pinned, dev, 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "read-back: %s", hipGetErrorString(e));
  *host = ctx->pinned[0];
  return VIE_OK;
}

// Right-hand side <f_m, E^i> (Sec. 2.1) of the unit plane wave of the last
// fill's incidence in polarisation pol, into b.
void launch_rhs(vie_ctx *ctx, int pol, dz *b) {
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  const double k0 = 2 * M_PI / ctx->lambda;
  const double st = std::sin(ctx->theta), ct = std::cos(ctx->theta), sp = std::sin(ctx->phi), cp = std::cos(ctx->phi);
  const double kix = k0 * st * cp, kiy = k0 * st * sp, kiz = -k0 * ct;
  double ex, ey, ez;
  if (pol == VIE_TE) {
    ex = -sp;
    ey = cp;
    ez = 0;
  } else {
    ex = ct * cp;
    ey = ct * sp;
    ez = st;
  }
  hipLaunchKernelGGL(k_rhs, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, N, ctx->ptr<int32_t>(L.utet),
                     ctx->ptr<int32_t>(L.uk), ctx->ptr<TetGeom>(L.tg), ctx->ptr<QuadRules>(L.quad),
                     (const dz *)ctx->ptr<dz>(L.alpha), kix, kiy, kiz, ex, ey, ez, b);
}

// One Arnoldi step of right-preconditioned GMRES for each Krylov process in
// `mask` (bit k: process k), on the column j held in device memory (K[k].jd):
// z = M^-1 V_j, w = Z z, CGS2 against V_0..V_j into H[:, j], h_{j+1,j} =
// ||w||, Givens update of H and g (|g_{j+1}| into rhist[j]), V_{j+1} =
// w / h_{j+1,j}, j += 1.  With both processes the preconditioner apply and the
// matvec serve the two in one pass each; every other launch is per process,
// so a process computes the same bits as alone.  The launches do not depend on
// j, so steps can be captured in a graph and replayed.
int arnoldi_step(vie_ctx *ctx, int mask) {
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  const int ldh = L.restart + 2;
  int ks[2], np = 0;
  for (int k = 0; k < 2; ++k)
    if (mask >> k & 1) ks[np++] = k;
  const dz *vin[2];
  dz *z[2], *w[2], *tmp[2], *u[2];
  for (int i = 0; i < np; ++i) {
    const Layout::Kry &K = L.K[ks[i]];
    dz *vi = ctx->ptr<dz>(K.vin);
    vin[i] = vi;
    z[i] = ctx->ptr<dz>(K.vz);
    w[i] = ctx->ptr<dz>(K.vw);
    tmp[i] = ctx->ptr<dz>(K.vt);
    u[i] = ctx->ptr<dz>(K.vu);
    hipLaunchKernelGGL(k_arn_begin, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, (const dz *)ctx->ptr<dz>(K.V),
                       L.ldv, (const int *)ctx->ptr<int>(K.jd), vi, N);
  }
  if (ctx->precond == 0) {
    if (int rc = apply_minv_n(ctx, np, vin, z, tmp, u)) return rc;
  } else if (ctx->precond == 2) {
    for (int i = 0; i < np; ++i)
      hipLaunchKernelGGL(k_jacobi_apply, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, N,
                         (const dz *)ctx->ptr<dz>(L.jdiag), vin[i], z[i]);
  } else {
    for (int i = 0; i < np; ++i) z[i] = const_cast<dz *>(vin[i]);   // M = I: the product takes V_j itself
  }
  if (np == 2) {
    const MvVecs v{{z[0], z[1]}, {nullptr, nullptr}, {w[0], w[1]}};
    if (int rc = matvec2(ctx, v)) return rc;
  } else if (int rc = matvec(ctx, z[0], nullptr, w[0])) {
    return rc;
  }
  for (int i = 0; i < np; ++i) {
    const Layout::Kry &K = L.K[ks[i]];
    dz *V = ctx->ptr<dz>(K.V), *H = ctx->ptr<dz>(K.H), *g = ctx->ptr<dz>(K.g), *y = ctx->ptr<dz>(K.y);
    double *cs = ctx->ptr<double>(K.cs), *scal = ctx->ptr<double>(K.scal);
    dz *sn = ctx->ptr<dz>(K.sn), *part = ctx->ptr<dz>(K.dpart);
    int *jd = ctx->ptr<int>(K.jd);
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_dots_j, dim3(kRedBlocks, nblk(L.restart + 1, 8)), dim3(256), 0, ctx->stream, (const dz *)V, L.ldv,
                         (const int *)jd, (const dz *)w[i], N, part);
      hipLaunchKernelGGL(k_dots_reduce_j, dim3(nblk(L.restart + 1, 128)), dim3(128), 0, ctx->stream,
                         (const dz *)part, kRedBlocks, (const int *)jd, H, ldh, y, pass);
      hipLaunchKernelGGL(k_update_j, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, (const dz *)V, L.ldv,
                         (const int *)jd, (const dz *)y, w[i], N);
    }
    if (int rc = norm_to(ctx, ks[i], w[i], N, scal + 2)) return rc;   // scal[2] = h_{j+1,j}
    hipLaunchKernelGGL(k_givens_j, dim3(1), dim3(1), 0, ctx->stream, H, ldh, (const int *)jd,
                       (const double *)(scal + 2), cs, sn, g, ctx->ptr<double>(K.rhist));
    hipLaunchKernelGGL(k_scale_j, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, (const dz *)w[i],
                       (const double *)(scal + 2), V, L.ldv, (const int *)jd, N);
    hipLaunchKernelGGL(k_jinc, dim3(1), dim3(1), 0, ctx->stream, jd);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "Arnoldi step: %s", hipGetErrorString(e));
  return VIE_OK;
}

// Capture `steps` Arnoldi steps of the processes in `mask` on the context's
// stream into an executable graph.
int capture_steps(vie_ctx *ctx, int mask, int steps, hipGraphExec_t *out) {
  hipGraph_t graph = nullptr;
  HIPCK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  ctx->capturing = true;   // no cooperative launches inside a captured graph
  int rc = VIE_OK;
  for (int q = 0; q < steps && rc == VIE_OK; ++q) rc = arnoldi_step(ctx, mask);
  ctx->capturing = false;
  hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(ctx, VIE_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  return VIE_OK;
}

// Issue `steps` Arnoldi steps of the processes in `mask`: replay a captured
// graph (one per process set and step count) when graph mode is on.
int issue_steps(vie_ctx *ctx, int mask, int steps) {
  if (ctx->graph_steps > 0 && ctx->stream == nullptr)
    return fail(ctx, VIE_EINVAL, "graph capture needs a non-null stream (VIE_OPT_GRAPH_STEPS)");
  if (ctx->graph_steps <= 0) {
    for (int q = 0; q < steps; ++q)
      if (int rc = arnoldi_step(ctx, mask)) return rc;
    return VIE_OK;
  }
  const int m = mask - 1;
  hipGraphExec_t *ge = steps == 1 ? &ctx->gexec[m][1] : &ctx->gexec[m][0];
  if (steps != 1 && ctx->gexec_steps[m] != steps) {
    if (ctx->gexec[m][0]) (void)hipGraphExecDestroy(ctx->gexec[m][0]);
    ctx->gexec[m][0] = nullptr;
    ctx->gexec_steps[m] = steps;
  }
  if (!*ge)
    if (int rc = capture_steps(ctx, mask, steps, ge)) return rc;
  HIPCK(hipGraphLaunch(*ge, ctx->stream));
  return VIE_OK;
}

// One restarted GMRES process: Krylov workspace K[k], polarisation pol.
struct Gmres {
  int k = 0, pol = 0;
  double bnorm = 0, beta = 0, true_rel = 1;
  int iters = 0, restarts = 0;
  bool converged = false, done = false;
  int jdone = 0;             // Arnoldi columns of the current cycle
  bool est_ok = false, stop = false;
};

// Restarted right-preconditioned GMRES (Sec. 3) for np (1 or 2) processes in
// lockstep, x0 = 0.  A restart cycle runs Arnoldi steps for every process that
// has not stopped; a process stops at its own converged estimate or at the
// cycle's end, and the others go on without it.  Each process takes the same
// decisions, on the same values, as it would alone.
int gmres(vie_ctx *ctx, int np, Gmres *P, double tol, int max_iter, int restart) {
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  const int ldh = L.restart + 2;
  for (int i = 0; i < np; ++i) {
    const Layout::Kry &K = L.K[P[i].k];
    dz *b = ctx->ptr<dz>(K.vb), *x = ctx->ptr<dz>(K.vx), *r = ctx->ptr<dz>(K.vr);
    ctx->hist[P[i].k].clear();
    launch_rhs(ctx, P[i].pol, b);
    hipLaunchKernelGGL(k_zero, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, x, N);
    hipLaunchKernelGGL(k_copy, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, r, (const dz *)b, N);
    LAUNCHCK();
    if (int rc = norm_to(ctx, P[i].k, r, N, ctx->ptr<double>(K.scal) + 0)) return rc;   // scal[0] = ||b||
  }
  for (int i = 0; i < np; ++i) {
    double *scal = ctx->ptr<double>(L.K[P[i].k].scal);
    if (int rc = read_scalar(ctx, scal + 0, &P[i].bnorm)) return rc;
    if (!(P[i].bnorm > 0)) return fail(ctx, VIE_EINVAL, "zero right-hand side");
    HIPCK(hipMemcpyAsync(scal + 1, scal + 0, 8, hipMemcpyDeviceToDevice, ctx->stream));   // scal[1] = beta
    P[i].beta = P[i].bnorm;
  }
  const int G = std::max(1, ctx->graph_steps);
  while (true) {
    int cyc = 0;   // processes in this restart cycle
    for (int i = 0; i < np; ++i) {
      Gmres &p = P[i];
      if (p.done) continue;
      cyc |= 1 << i;
      const Layout::Kry &K = L.K[p.k];
      // V0 = r / beta ; g = beta e1 ; j = 0
      hipLaunchKernelGGL(k_scale, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, (const dz *)ctx->ptr<dz>(K.vr),
                         (const double *)(ctx->ptr<double>(K.scal) + 1), ctx->ptr<dz>(K.V), N);
      hipLaunchKernelGGL(k_ginit, dim3(1), dim3(256), 0, ctx->stream, ctx->ptr<dz>(K.g), restart + 1,
                         (const double *)(ctx->ptr<double>(K.scal) + 1));
      hipLaunchKernelGGL(k_jset, dim3(1), dim3(1), 0, ctx->stream, ctx->ptr<int>(K.jd), 0);
      LAUNCHCK();
      p.jdone = 0;
      p.est_ok = p.stop = false;
    }
    if (!cyc) break;
    // Arnoldi steps in launches of up to G steps; the residual estimates of a
    // launch are read back together.  Steps past the converged one are
    // harmless: the update below uses only the first jdone columns.
    for (int j = 0; j < restart;) {
      int run = 0, mask = 0;
      for (int i = 0; i < np; ++i)
        if ((cyc >> i & 1) && !P[i].stop) {
          run |= 1 << i;
          mask |= 1 << P[i].k;
        }
      if (!run) break;
      const int steps = (ctx->graph_steps > 0 && j + G <= restart) ? G : 1;
      if (int rc = issue_steps(ctx, mask, steps)) return rc;
      for (int i = 0; i < np; ++i)
        if (run >> i & 1)
          HIPCK(hipMemcpyAsync(ctx->pinned + 64 * i, ctx->ptr<double>(L.K[P[i].k].rhist) + j, 8 * steps,
                               hipMemcpyDeviceToHost, ctx->stream));
      HIPCK(hipStreamSynchronize(ctx->stream));
      for (int i = 0; i < np; ++i) {
        if (!(run >> i & 1)) continue;
        Gmres &p = P[i];
        for (int q = 0; q < steps; ++q) {
          const double res = ctx->pinned[64 * i + q];
          ++p.iters;
          p.jdone = j + q + 1;
          ctx->hist[p.k].push_back(res / p.bnorm);
          if (res / p.bnorm <= tol) {
            p.est_ok = p.stop = true;
            break;
          }
          if (p.iters >= max_iter) {
            p.stop = true;
            break;
          }
        }
      }
      j += steps;
    }
    // x += M^{-1} V y, then the true residual r = b - Z x
    int nc = 0;
    const dz *wv[2];
    dz *uv[2], *tv[2], *zv[2];
    MvVecs rv{};
    for (int i = 0; i < np; ++i) {
      if (!(cyc >> i & 1)) continue;
      const Layout::Kry &K = L.K[P[i].k];
      dz *w = ctx->ptr<dz>(K.vw);
      hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(1), 0, ctx->stream, (const dz *)ctx->ptr<dz>(K.H), ldh,
                         P[i].jdone, (const dz *)ctx->ptr<dz>(K.g), ctx->ptr<dz>(K.y));
      hipLaunchKernelGGL(k_combine, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, (const dz *)ctx->ptr<dz>(K.V),
                         L.ldv, P[i].jdone, (const dz *)ctx->ptr<dz>(K.y), w, N);
      LAUNCHCK();
      wv[nc] = w;
      uv[nc] = ctx->ptr<dz>(K.vu);
      tv[nc] = ctx->ptr<dz>(K.vt);
      zv[nc] = ctx->ptr<dz>(K.vz);
      rv.x[nc] = ctx->ptr<dz>(K.vx);
      rv.b[nc] = ctx->ptr<dz>(K.vb);
      rv.y[nc] = ctx->ptr<dz>(K.vr);
      ++nc;
    }
    if (ctx->precond == 0) {
      if (int rc = apply_minv_n(ctx, nc, wv, uv, tv, zv)) return rc;
    } else if (ctx->precond == 2) {
      for (int q = 0; q < nc; ++q)
        hipLaunchKernelGGL(k_jacobi_apply, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, N,
                           (const dz *)ctx->ptr<dz>(L.jdiag), wv[q], uv[q]);
    } else {
      for (int q = 0; q < nc; ++q) uv[q] = const_cast<dz *>(wv[q]);   // M = I: x += V y
    }
    for (int q = 0; q < nc; ++q)
      hipLaunchKernelGGL(k_axpy, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, const_cast<dz *>(rv.x[q]),
                         (const dz *)uv[q], N);
    if (nc == 2) {
      if (int rc = matvec2(ctx, rv)) return rc;
    } else if (int rc = matvec(ctx, rv.x[0], rv.b[0], rv.y[0])) {
      return rc;
    }
    for (int i = 0; i < np; ++i) {
      if (!(cyc >> i & 1)) continue;
      Gmres &p = P[i];
      double *scal = ctx->ptr<double>(L.K[p.k].scal);
      if (int rc = norm_to(ctx, p.k, ctx->ptr<dz>(L.K[p.k].vr), N, scal + 1)) return rc;
      if (int rc = read_scalar(ctx, scal + 1, &p.beta)) return rc;
      p.true_rel = p.beta / p.bnorm;
      if (p.true_rel <= tol || (p.est_ok && p.true_rel <= 10 * tol)) {
        p.converged = p.done = true;
      } else if (p.iters >= max_iter) {
        p.done = true;
      } else {
        ++p.restarts;
      }
    }
  }
  return VIE_OK;
}

int solve_args(vie_ctx *ctx, double tol, int max_iter, int restart) {
  if (!(tol > 0) || max_iter < 1) return fail(ctx, VIE_EINVAL, "bad tol / max_iter");
  if (restart < 1 || restart > ctx->L.restart)
    return fail(ctx, VIE_EINVAL, "restart %d exceeds the bound workspace (%d)", restart, ctx->L.restart);
  return VIE_OK;
}

// Run np GMRES processes and fill info[np]; t_solve_ms is the wall time of
// the whole run (shared by a pair).
int run_solve(vie_ctx *ctx, int np, Gmres *P, double tol, int max_iter, int restart, vie_solve_info *info) {
  HIPCK(hipSetDevice(ctx->device));
  ctx->sol_k[0] = ctx->sol_k[1] = -1;
  HIPCK(hipEventRecord(ctx->ev0, ctx->stream));
  if (int rc = gmres(ctx, np, P, tol, max_iter, restart)) return rc;
  HIPCK(hipEventRecord(ctx->ev1, ctx->stream));
  HIPCK(hipEventSynchronize(ctx->ev1));
  float ms = 0;
  HIPCK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  for (int i = 0; i < np; ++i) {
    ctx->sol_k[P[i].pol] = P[i].k;
    if (info) {
      info[i].iters = P[i].iters;
      info[i].restarts = P[i].restarts;
      info[i].refine_steps = P[i].restarts + 1;
      info[i].true_rel_residual = P[i].true_rel;
      info[i].t_fill_ms = ctx->t_fill;
      info[i].t_factor_ms = ctx->t_factor;
      info[i].t_solve_ms = ms;
      info[i].converged = P[i].converged ? 1 : 0;
    }
  }
  ctx->last_pol = P[np - 1].pol;
  ctx->state = S_SOLVED;
  for (int i = 0; i < np; ++i)
    if (!P[i].converged)
      return fail(ctx, VIE_ENOCONV, "GMRES (%s): %d iterations, relative residual %.3e",
                  P[i].pol == VIE_TE ? "TE" : "TM", P[i].iters, P[i].true_rel);
  return VIE_OK;
}

}  // namespace vie

// Before a solve: the point-Jacobi scaling of this fill (once) when that
// preconditioner is chosen; the grid operator solves with M = diag(Z) or
// M = I and plain launches (its FFTs are not captured into the Arnoldi-step
// graphs).
static int solve_setup(vie_ctx *ctx) {
  if (ctx->precond == 2 && !ctx->jdiag_ok) {
    HIPCK(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_jacobi_diag, dim3(nblk(ctx->topo.N, 256)), dim3(256), 0, ctx->stream, (int64_t)ctx->topo.N,
                       zout(ctx), ctx->ptr<dz>(ctx->L.jdiag));
    LAUNCHCK();
    ctx->jdiag_ok = true;
  }
  if (ctx->precision != VIE_GRID_FP64) return VIE_OK;
  if (ctx->precond == 0)
    return fail(ctx, VIE_EINVAL, "VIE_GRID_FP64 has no block preconditioner: set VIE_OPT_PRECOND to 2 or 1");
  if (ctx->graph_steps > 0) return fail(ctx, VIE_EINVAL, "VIE_GRID_FP64 runs without graph-captured steps");
  return VIE_OK;
}

extern "C" {

int vie_solve(vie_ctx *ctx, int pol, double tol, int max_iter, int restart, vie_solve_info *info) {
  if (int r = check(ctx, S_FILLED, "vie_solve")) return r;
  if (int r = solve_setup(ctx)) return r;
  if (!ctx->precond && !ctx->factored)
    return fail(ctx, VIE_ESTATE, "vie_solve: the block preconditioner needs vie_precond_factor after the fill");
  if (pol != VIE_TE && pol != VIE_TM) return fail(ctx, VIE_EINVAL, "polarisation must be VIE_TE or VIE_TM");
  if (int r = solve_args(ctx, tol, max_iter, restart)) return r;
  Gmres P[1];
  P[0].k = 0;
  P[0].pol = pol;
  return run_solve(ctx, 1, P, tol, max_iter, restart, info);
}

int vie_solve_pair(vie_ctx *ctx, double tol, int max_iter, int restart, vie_solve_info *info) {
  if (int r = check(ctx, S_FILLED, "vie_solve_pair")) return r;
  if (int r = solve_setup(ctx)) return r;
  if (!ctx->precond && !ctx->factored)
    return fail(ctx, VIE_ESTATE, "vie_solve_pair: the block preconditioner needs vie_precond_factor after the fill");
  if (int r = solve_args(ctx, tol, max_iter, restart)) return r;
  Gmres P[2];
  P[0].k = 0;
  P[0].pol = VIE_TE;
  P[1].k = 1;
  P[1].pol = VIE_TM;
  return run_solve(ctx, 2, P, tol, max_iter, restart, info);
}

// ---------------------------------------------------------------- outputs
int vie_absorption(vie_ctx *ctx, double *absorptance, double *R, double *T) {
  if (int r = check(ctx, S_SOLVED, "vie_absorption")) return r;
  return vie_absorption_pol(ctx, ctx->last_pol, absorptance, R, T);
}

int vie_absorption_per_tet(vie_ctx *ctx, int pol, double *per_tet) {
  if (int r = check(ctx, S_SOLVED, "vie_absorption_per_tet")) return r;
  if (pol < 0) pol = ctx->last_pol;
  if (pol != VIE_TE && pol != VIE_TM) return fail(ctx, VIE_EINVAL, "polarisation must be VIE_TE, VIE_TM or -1");
  if (ctx->sol_k[pol] < 0) return fail(ctx, VIE_ESTATE, "the last solve did not cover this polarisation");
  if (!per_tet) return fail(ctx, VIE_EINVAL, "null output");
  HIPCK(hipSetDevice(ctx->device));
  const MeshTopology &t = ctx->topo;
  const Layout &L = ctx->L;
  const dz *xsol = ctx->ptr<dz>(L.K[ctx->sol_k[pol]].vx);
  const unsigned nb = nblk(t.nt, 256);
  double *dev = ctx->ptr<double>(L.atet);
  hipLaunchKernelGGL(k_absorb, dim3(nb), dim3(256), 0, ctx->stream, (int64_t)t.nt, t.ndom, ctx->ptr<TetGeom>(L.tg),
                     ctx->ptr<TetFace>(L.t2f), ctx->ptr<int32_t>(L.dom), ctx->ptr<QuadRules>(L.quad),
                     (const dz *)ctx->ptr<dz>(L.gsrc), (const dz *)ctx->ptr<dz>(L.inveps), xsol,
                     ctx->ptr<double>(L.apart), dev);
  LAUNCHCK();
  HIPCK(hipMemcpyAsync(per_tet, dev, 8 * (size_t)t.nt, hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  const double k0 = 2 * M_PI / ctx->lambda;
  const double scale = k0 / (std::cos(ctx->theta) * t.a * t.b);
  for (int64_t i = 0; i < t.nt; ++i) per_tet[i] *= scale;
  return VIE_OK;
}

int vie_sample_field(vie_ctx *ctx, int pol, const double *points, int64_t npts, vie_c128 *e, int32_t *tet) {
  if (int r = check(ctx, S_SOLVED, "vie_sample_field")) return r;
  if (pol < 0) pol = ctx->last_pol;
  if (pol != VIE_TE && pol != VIE_TM) return fail(ctx, VIE_EINVAL, "polarisation must be VIE_TE, VIE_TM or -1");
  if (ctx->sol_k[pol] < 0) return fail(ctx, VIE_ESTATE, "the last solve did not cover this polarisation");
  if (npts < 0 || (npts > 0 && (!points || !e))) return fail(ctx, VIE_EINVAL, "bad arguments");
  if (npts == 0) return VIE_OK;
  const MeshTopology &t = ctx->topo;
  const Layout &L = ctx->L;
  std::vector<int32_t> hostTet(npts);
  locate_points(t, points, npts, hostTet.data());
  if (tet) std::copy(hostTet.begin(), hostTet.end(), tet);
  // points, their tetrahedra and the field staged in the Krylov-basis region (clobbers it), in chunks
  const int64_t cap = (int64_t)((L.K[0].V.bytes - 1024) / 80);
  if (cap < 1) return fail(ctx, VIE_ENOMEM, "no staging space");
  HIPCK(hipSetDevice(ctx->device));
  const dz *xsol = ctx->ptr<dz>(L.K[ctx->sol_k[pol]].vx);
  for (int64_t s0 = 0; s0 < npts; s0 += cap) {
    const int64_t m = std::min(cap, npts - s0);
    char *base = ctx->ws + L.K[0].V.off;
    double *dp = reinterpret_cast<double *>(base);
    int32_t *dt = reinterpret_cast<int32_t *>(base + align256(24 * (size_t)m));
    dz *de = reinterpret_cast<dz *>(base + align256(24 * (size_t)m) + align256(4 * (size_t)m));
    HIPCK(hipMemcpyAsync(dp, points + 3 * s0, 24 * m, hipMemcpyHostToDevice, ctx->stream));
    HIPCK(hipMemcpyAsync(dt, hostTet.data() + s0, 4 * m, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_field, dim3(nblk(m, 256)), dim3(256), 0, ctx->stream, m, (const double *)dp,
                       (const int32_t *)dt, ctx->ptr<TetGeom>(L.tg), ctx->ptr<TetFace>(L.t2f),
                       (const dz *)ctx->ptr<dz>(L.gsrc), (const dz *)ctx->ptr<dz>(L.inveps), xsol, de);
    LAUNCHCK();
    HIPCK(hipMemcpyAsync(e + 3 * s0, de, 48 * m, hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
  }
  return VIE_OK;
}

int vie_absorption_pol(vie_ctx *ctx, int pol, double *absorptance, double *R, double *T) {
  if (int r = check(ctx, S_SOLVED, "vie_absorption_pol")) return r;
  if (pol != VIE_TE && pol != VIE_TM) return fail(ctx, VIE_EINVAL, "polarisation must be VIE_TE or VIE_TM");
  if (ctx->sol_k[pol] < 0) return fail(ctx, VIE_ESTATE, "the last solve did not cover this polarisation");
  if (!absorptance) return fail(ctx, VIE_EINVAL, "null output");
  HIPCK(hipSetDevice(ctx->device));
  const MeshTopology &t = ctx->topo;
  const Layout &L = ctx->L;
  const dz *xsol = ctx->ptr<dz>(L.K[ctx->sol_k[pol]].vx);
  const unsigned nb = nblk(t.nt, 256);
  double *part = ctx->ptr<double>(L.apart);
  double *out = ctx->ptr<double>(L.idx);
  hipLaunchKernelGGL(k_absorb, dim3(nb), dim3(256), 0, ctx->stream, (int64_t)t.nt, t.ndom, ctx->ptr<TetGeom>(L.tg),
                     ctx->ptr<TetFace>(L.t2f), ctx->ptr<int32_t>(L.dom), ctx->ptr<QuadRules>(L.quad),
                     (const dz *)ctx->ptr<dz>(L.gsrc), (const dz *)ctx->ptr<dz>(L.inveps), xsol,
                     part, nullptr);
  hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(256), 0, ctx->stream, (const double *)part, (int)nb, t.ndom, out);
  LAUNCHCK();
  std::vector<double> h(t.ndom);
  HIPCK(hipMemcpyAsync(h.data(), out, 8 * t.ndom, hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  const double k0 = 2 * M_PI / ctx->lambda;
  const double scale = k0 / (std::cos(ctx->theta) * t.a * t.b);
  for (int d = 0; d < t.ndom; ++d) absorptance[d] = h[d] * scale;

  if (R || T) {
    const double kx = k0 * std::sin(ctx->theta) * std::cos(ctx->phi), ky = k0 * std::sin(ctx->theta) * std::sin(ctx->phi);
    std::vector<double> kvh;
    std::vector<double> beta;
    std::vector<int> isz;
    // every propagating Floquet order (|kt_pq| < k0 needs |2 pi p / a| < k0 + |kx|)
    const int pmax = (int)std::ceil((k0 + std::fabs(kx)) * t.a / (2 * M_PI));
    const int qmax = (int)std::ceil((k0 + std::fabs(ky)) * t.b / (2 * M_PI));
    for (int p = -pmax; p <= pmax; ++p)
      for (int q = -qmax; q <= qmax; ++q) {
        double tx = kx + 2 * M_PI * p / t.a, ty = ky + 2 * M_PI * q / t.b;
        double kt2 = tx * tx + ty * ty;
        if (kt2 >= k0 * k0) continue;
        if (std::abs(p) > kPgfM || std::abs(q) > kPgfM || (int)beta.size() >= 32)
          return fail(ctx, VIE_EINVAL, "propagating Floquet order (%d, %d) beyond the %d orders R/T can sum", p, q,
                      (int)beta.size());
        double bz = std::sqrt(k0 * k0 - kt2);
        for (int s : {+1, -1}) {
          kvh.push_back(tx);
          kvh.push_back(ty);
          kvh.push_back(s * bz);
        }
        beta.push_back(bz);
        isz.push_back(p == 0 && q == 0);
      }
    const int nk = (int)kvh.size() / 3;
    HIPCK(hipMemcpyAsync(ctx->ptr<double>(L.kv), kvh.data(), 8 * kvh.size(), hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_project, dim3(nb), dim3(256), 0, ctx->stream, (int64_t)t.nt, ctx->ptr<TetGeom>(L.tg),
                       ctx->ptr<TetFace>(L.t2f), ctx->ptr<QuadRules>(L.quad), (const dz *)ctx->ptr<dz>(L.gsrc),
                       (const dz *)ctx->ptr<dz>(L.kappa), xsol, nk,
                       (const double *)ctx->ptr<double>(L.kv), part);
    hipLaunchKernelGGL(k_reduce_cols, dim3(nblk(6 * nk, 256)), dim3(256), 0, ctx->stream, (const double *)part, (int)nb,
                       6 * nk, out);
    LAUNCHCK();
    std::vector<double> v(6 * nk);
    HIPCK(hipMemcpyAsync(v.data(), out, 8 * v.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
    const double st = std::sin(ctx->theta), ct = std::cos(ctx->theta), sp = std::sin(ctx->phi), cp = std::cos(ctx->phi);
    double e_inc[3];
    if (pol == VIE_TE) {
      e_inc[0] = -sp;
      e_inc[1] = cp;
      e_inc[2] = 0;
    } else {
      e_inc[0] = ct * cp;
      e_inc[1] = ct * sp;
      e_inc[2] = st;
    }
    const double beta00 = k0 * ct;
    double Rs = 0, Ts = 0;
    for (int i = 0; i < nk; ++i) {
      const int mode = i / 2;
      const bool up = (i % 2) == 0;
      zd vv[3];
      for (int d = 0; d < 3; ++d) vv[d] = zd(v[6 * i + 2 * d], v[6 * i + 2 * d + 1]);
      const double *k = &kvh[3 * i];
      zd kdotv = k[0] * vv[0] + k[1] * vv[1] + k[2] * vv[2];
      zd gam(0, beta[mode]);
      zd e[3];
      for (int d = 0; d < 3; ++d) e[d] = (k0 * k0 * vv[d] - k[d] * kdotv) / (2 * t.a * t.b * gam);
      if (!up && isz[mode])
        for (int d = 0; d < 3; ++d) e[d] += e_inc[d];
      double p2 = std::norm(e[0]) + std::norm(e[1]) + std::norm(e[2]);
      if (up) Rs += p2 * beta[mode] / beta00;
      else Ts += p2 * beta[mode] / beta00;
    }
    if (R) *R = Rs;
    if (T) *T = Ts;
  }
  return VIE_OK;
}

// ---------------------------------------------------------------- diagnostics
int vie_export_faces(const vie_ctx *c, int32_t *face_vid, int32_t *tplus, int32_t *tminus, int32_t *dom) {
  if (!c || c->state < S_MESH) return VIE_ESTATE;
  const MeshTopology &t = c->topo;
  if (face_vid) std::memcpy(face_vid, t.face_vid.data(), 4 * 3 * t.N);
  if (tplus) std::memcpy(tplus, t.tplus.data(), 4 * t.N);
  if (tminus) std::memcpy(tminus, t.tminus.data(), 4 * t.N);
  if (dom) std::memcpy(dom, t.fdom.data(), 4 * t.N);
  return VIE_OK;
}

int vie_read_Z(const vie_ctx *cctx, const int64_t *rows, const int64_t *cols, int64_t k, vie_c128 *out) {
  vie_ctx *ctx = const_cast<vie_ctx *>(cctx);
  if (int r = check(ctx, S_FILLED, "vie_read_Z")) return r;
  if (ctx->precision == VIE_GRID_FP64) return fail(ctx, VIE_EINVAL, "VIE_GRID_FP64 stores no Z (vie_apply_Z gives Z x)");
  if (!rows || !cols || !out || k < 0) return fail(ctx, VIE_EINVAL, "bad arguments");
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  HIPCK(hipSetDevice(ctx->device));
  // rows, cols and values staged through the Krylov-basis region (clobbers it)
  const int64_t cap = (int64_t)((L.K[0].V.bytes - 512) / 32);
  if (cap < 1) return fail(ctx, VIE_ENOMEM, "no staging space");
  int64_t *ri = ctx->ptr<int64_t>(L.K[0].V);
  for (int64_t s = 0; s < k; s += cap) {
    const int64_t n = std::min(cap, k - s);
    for (int64_t i = 0; i < n; ++i)
      if (rows[s + i] < 0 || rows[s + i] >= N || cols[s + i] < 0 || cols[s + i] >= N)
        return fail(ctx, VIE_EINVAL, "index out of range");
    dz *o = reinterpret_cast<dz *>(ctx->ws + L.K[0].V.off + align256(16 * (size_t)n));
    HIPCK(hipMemcpyAsync(ri, rows + s, 8 * n, hipMemcpyHostToDevice, ctx->stream));
    HIPCK(hipMemcpyAsync(ri + n, cols + s, 8 * n, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_gather, dim3(nblk(n, 256)), dim3(256), 0, ctx->stream, zout(ctx),
                       (const int64_t *)ri, (const int64_t *)(ri + n), n, o);
    LAUNCHCK();
    HIPCK(hipMemcpyAsync(out + s, o, 16 * n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
  }
  return VIE_OK;
}

static int read_vec(const vie_ctx *cctx, const Region &r, vie_c128 *dst) {
  vie_ctx *ctx = const_cast<vie_ctx *>(cctx);
  if (int rc = check(ctx, S_SOLVED, "read-back")) return rc;
  if (!dst) return fail(ctx, VIE_EINVAL, "null output");
  HIPCK(hipSetDevice(ctx->device));
  HIPCK(hipMemcpyAsync(dst, ctx->ws + r.off, 16 * ctx->topo.N, hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  return VIE_OK;
}

static int read_pol(const vie_ctx *cctx, int pol, bool rhs, vie_c128 *dst) {
  vie_ctx *ctx = const_cast<vie_ctx *>(cctx);
  if (!ctx) return VIE_EINVAL;
  if (int rc = check(ctx, S_SOLVED, "read-back")) return rc;
  if (pol != VIE_TE && pol != VIE_TM) return fail(ctx, VIE_EINVAL, "polarisation must be VIE_TE or VIE_TM");
  const int k = ctx->sol_k[pol];
  if (k < 0) return fail(ctx, VIE_ESTATE, "the last solve did not cover this polarisation");
  return read_vec(ctx, rhs ? ctx->L.K[k].vb : ctx->L.K[k].vx, dst);
}
int vie_read_rhs(const vie_ctx *ctx, vie_c128 *b) { return ctx ? read_pol(ctx, ctx->last_pol, true, b) : VIE_EINVAL; }
int vie_read_solution(const vie_ctx *ctx, vie_c128 *x) {
  return ctx ? read_pol(ctx, ctx->last_pol, false, x) : VIE_EINVAL;
}
int vie_read_solution_pol(const vie_ctx *ctx, int pol, vie_c128 *x) { return read_pol(ctx, pol, false, x); }

int vie_pgf_eval(vie_ctx *ctx, const double *delta, int64_t n, vie_c128 *out) {
  if (int r = check(ctx, S_FILLED, "vie_pgf_eval")) return r;
  const Layout &L = ctx->L;
  if (!delta || !out || n < 0) return fail(ctx, VIE_EINVAL, "bad arguments");
  // points and values staged in the Krylov-basis region (clobbers it), in chunks
  const int64_t cap = (int64_t)((L.K[0].V.bytes - 512) / 40);
  if (cap < 1) return fail(ctx, VIE_ENOMEM, "no staging space");
  HIPCK(hipSetDevice(ctx->device));
  double *d = ctx->ptr<double>(L.K[0].V);
  for (int64_t s = 0; s < n; s += cap) {
    const int64_t m = std::min(cap, n - s);
    dz *o = reinterpret_cast<dz *>(ctx->ws + L.K[0].V.off + align256(24 * (size_t)m));
    HIPCK(hipMemcpyAsync(d, delta + 3 * s, 24 * m, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_pgf_probe, dim3(nblk(m, 256)), dim3(256), 8 * (size_t)ctx->packlen, ctx->stream,
                       (const double *)ctx->ptr<double>(L.pack), ctx->packlen, (const double *)d, m, o);
    LAUNCHCK();
    HIPCK(hipMemcpyAsync(out + s, o, 16 * m, hipMemcpyDeviceToHost, ctx->stream));
    HIPCK(hipStreamSynchronize(ctx->stream));
  }
  return VIE_OK;
}

int vie_get_factor_stats(const vie_ctx *ctx, vie_factor_stats *out) {
  if (!ctx || !out) return VIE_EINVAL;
  if (!ctx->factored) return VIE_ESTATE;
  *out = ctx->facstats;
  return VIE_OK;
}

int vie_get_fill_stats(const vie_ctx *ctx, vie_fill_stats *out) {
  if (!ctx || !out) return VIE_EINVAL;
  if (ctx->state < S_FILLED) return VIE_ESTATE;
  *out = ctx->fstats;
  return VIE_OK;
}

int vie_apply_Z(vie_ctx *ctx, const vie_c128 *x, vie_c128 *y) {
  if (int r = check(ctx, S_FILLED, "vie_apply_Z")) return r;
  if (!x || !y) return fail(ctx, VIE_EINVAL, "null vector");
  HIPCK(hipSetDevice(ctx->device));
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  dz *xd = ctx->ptr<dz>(L.K[0].vz), *yd = ctx->ptr<dz>(L.K[0].vw);   // Krylov scratch (clobbered)
  HIPCK(hipMemcpyAsync(xd, x, 16 * (size_t)N, hipMemcpyHostToDevice, ctx->stream));
  if (int rc = matvec(ctx, xd, nullptr, yd)) return rc;
  HIPCK(hipMemcpyAsync(y, yd, 16 * (size_t)N, hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  return VIE_OK;
}

int vie_bench_matvec(vie_ctx *ctx, int reps, double *ms_per_matvec) {
  if (int r = check(ctx, S_FILLED, "vie_bench_matvec")) return r;
  if (reps < 1 || !ms_per_matvec) return fail(ctx, VIE_EINVAL, "bad arguments");
  HIPCK(hipSetDevice(ctx->device));
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  dz *x = ctx->ptr<dz>(L.K[0].vz), *y = ctx->ptr<dz>(L.K[0].vw);
  hipLaunchKernelGGL(k_fill_const, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, x, N, 1.0, 0.5);
  LAUNCHCK();
  HIPCK(hipEventRecord(ctx->ev2, ctx->stream));
  for (int r = 0; r < reps; ++r)
    if (int rc = matvec(ctx, x, nullptr, y)) return rc;
  HIPCK(hipEventRecord(ctx->ev3, ctx->stream));
  HIPCK(hipEventSynchronize(ctx->ev3));
  float ms = 0;
  HIPCK(hipEventElapsedTime(&ms, ctx->ev2, ctx->ev3));
  *ms_per_matvec = ms / reps;
  return VIE_OK;
}

int vie_precond_apply(vie_ctx *ctx, const vie_c128 *v, vie_c128 *z) {
  if (int r = check(ctx, S_FACTORED, "vie_precond_apply")) return r;
  if (!ctx->factored) return fail(ctx, VIE_ESTATE, "vie_precond_apply needs vie_precond_factor after the fill");
  if (!v || !z) return fail(ctx, VIE_EINVAL, "null vector");
  HIPCK(hipSetDevice(ctx->device));
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  dz *in = ctx->ptr<dz>(L.K[0].vw), *out = ctx->ptr<dz>(L.K[0].vz);
  HIPCK(hipMemcpyAsync(in, v, 16 * N, hipMemcpyHostToDevice, ctx->stream));
  if (int rc = apply_minv(ctx, in, out, ctx->ptr<dz>(L.K[0].vu), ctx->ptr<dz>(L.K[0].vr))) return rc;
  HIPCK(hipMemcpyAsync(z, out, 16 * N, hipMemcpyDeviceToHost, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  return VIE_OK;
}

int vie_set_option(vie_ctx *ctx, int option, int value) {
  if (!ctx) return VIE_EINVAL;
  switch (option) {
    case VIE_OPT_GRAPH_STEPS:
      if (value < 0 || value > 64) return fail(ctx, VIE_EINVAL, "graph steps must be in [0, 64]");
      if (value != ctx->graph_steps) drop_graphs(ctx);
      ctx->graph_steps = value;
      return VIE_OK;
    case VIE_OPT_MATVEC_ROWS:
      if (value != 2 && value != 4 && value != 8) return fail(ctx, VIE_EINVAL, "matvec rows per wave: 2, 4 or 8");
      if (value != ctx->mv_rpw) drop_graphs(ctx);
      ctx->mv_rpw = value;
      return VIE_OK;
    case VIE_OPT_TRSV_COOP:
      if (value != 0 && value != 1) return fail(ctx, VIE_EINVAL, "cooperative triangular solves: 0 or 1");
      ctx->trsv_coop = value;
      return VIE_OK;
    case VIE_OPT_LU_PIVOT:
      if (value != 0 && value != 1) return fail(ctx, VIE_EINVAL, "LU pivoting: 0 (tournament) or 1 (partial)");
      ctx->lu_pivot = value;
      return VIE_OK;
    case VIE_OPT_SYM_FILL:
      if (value != 0 && value != 1) return fail(ctx, VIE_EINVAL, "symmetric fill: 0 or 1");
      if (ctx->state >= S_BOUND) return fail(ctx, VIE_ESTATE, "VIE_OPT_SYM_FILL is set before the workspace is bound");
      ctx->sym_fill = value;
      return VIE_OK;
    case VIE_OPT_PRECOND:
      if (value < 0 || value > 2)
        return fail(ctx, VIE_EINVAL, "preconditioner: 0 (block-diagonal LU), 1 (none) or 2 (point Jacobi)");
      if (value != ctx->precond) drop_graphs(ctx);
      ctx->precond = value;
      return VIE_OK;
    case VIE_OPT_TRSV_CHUNK:
      if (value != 1024 && value != 2048) return fail(ctx, VIE_EINVAL, "trsv chunk width: 1024 or 2048 columns");
      if (value != ctx->trsv_kc) drop_graphs(ctx);
      ctx->trsv_kc = value;
      return VIE_OK;
  }
  return fail(ctx, VIE_EINVAL, "unknown option %d", option);
}

int vie_get_option(const vie_ctx *ctx, int option, int *value) {
  if (!ctx || !value) return VIE_EINVAL;
  switch (option) {
    case VIE_OPT_GRAPH_STEPS: *value = ctx->graph_steps; return VIE_OK;
    case VIE_OPT_MATVEC_ROWS: *value = ctx->mv_rpw; return VIE_OK;
    case VIE_OPT_TRSV_CHUNK: *value = ctx->trsv_kc; return VIE_OK;
    case VIE_OPT_TRSV_COOP: *value = ctx->trsv_coop; return VIE_OK;
    case VIE_OPT_LU_PIVOT: *value = ctx->lu_pivot; return VIE_OK;
    case VIE_OPT_SYM_FILL: *value = ctx->sym_fill; return VIE_OK;
    case VIE_OPT_PRECOND: *value = ctx->precond; return VIE_OK;
  }
  return VIE_EINVAL;
}

int vie_autotune(vie_ctx *ctx, int reps, vie_tuning *out) {
  if (int r = check(ctx, S_FACTORED, "vie_autotune")) return r;
  if (!ctx->factored) return fail(ctx, VIE_ESTATE, "vie_autotune needs vie_precond_factor after the fill");
  if (reps < 1) return fail(ctx, VIE_EINVAL, "reps must be >= 1");
  HIPCK(hipSetDevice(ctx->device));
  const Layout &L = ctx->L;
  const int64_t N = ctx->topo.N;
  dz *x = ctx->ptr<dz>(L.K[0].vz), *y = ctx->ptr<dz>(L.K[0].vw);
  hipLaunchKernelGGL(k_fill_const, dim3(nblk(N, 256)), dim3(256), 0, ctx->stream, x, N, 1.0, 0.5);
  LAUNCHCK();
  vie_tuning t{};
  auto time_it = [&](auto &&issue, double *ms_out) -> int {
    if (int rc = issue()) return rc;   // warm-up
    HIPCK(hipEventRecord(ctx->ev2, ctx->stream));
    for (int r = 0; r < reps; ++r)
      if (int rc = issue()) return rc;
    HIPCK(hipEventRecord(ctx->ev3, ctx->stream));
    HIPCK(hipEventSynchronize(ctx->ev3));
    float ms = 0;
    HIPCK(hipEventElapsedTime(&ms, ctx->ev2, ctx->ev3));
    *ms_out = ms / reps;
    return VIE_OK;
  };
  // products for one vector and for two (paired solves): the pick
  // minimises the sum of the two
  const int mv_opts[3] = {2, 4, 8}, tr_opts[2] = {1024, 2048};
  double best = 1e300;
  int pick = ctx->mv_rpw;
  MvVecs v2{};
  v2.x[0] = v2.x[1] = x;
  v2.y[0] = y;
  v2.y[1] = ctx->ptr<dz>(L.K[1].vw);
  for (int i = 0; i < 3; ++i) {
    ctx->mv_rpw = mv_opts[i];
    if (int rc = time_it([&]() { return matvec(ctx, x, nullptr, y); }, &t.matvec_ms[i])) return rc;
    if (int rc = time_it([&]() { return matvec2(ctx, v2); }, &t.matvec_ms[3 + i])) return rc;
    if (t.matvec_ms[i] + t.matvec_ms[3 + i] < best) {
      best = t.matvec_ms[i] + t.matvec_ms[3 + i];
      pick = mv_opts[i];
    }
  }
  ctx->mv_rpw = pick;
  // triangular solves for one vector and for two (paired solves): the pick
  // minimises the sum of the two
  best = 1e300;
  pick = ctx->trsv_kc;
  for (int i = 0; i < 2; ++i) {
    ctx->trsv_kc = tr_opts[i];
    const Layout::Kry &A = L.K[0], &B = L.K[1];
    const dz *v2[2] = {x, x};
    dz *o2[2] = {ctx->ptr<dz>(A.vu), ctx->ptr<dz>(B.vu)}, *t2[2] = {ctx->ptr<dz>(A.vt), ctx->ptr<dz>(B.vt)},
       *r2[2] = {ctx->ptr<dz>(A.vr), ctx->ptr<dz>(B.vr)};
    if (int rc = time_it([&]() { return apply_minv(ctx, x, o2[0], t2[0], r2[0]); }, &t.apply_ms[i])) return rc;
    if (int rc = time_it([&]() { return apply_minv_n(ctx, 2, v2, o2, t2, r2); }, &t.apply_ms[2 + i])) return rc;
    if (t.apply_ms[i] + t.apply_ms[2 + i] < best) {
      best = t.apply_ms[i] + t.apply_ms[2 + i];
      pick = tr_opts[i];
    }
  }
  ctx->trsv_kc = pick;
  drop_graphs(ctx);
  t.matvec_rows = ctx->mv_rpw;
  t.trsv_chunk = ctx->trsv_kc;
  if (out) *out = t;
  return VIE_OK;
}

int vie_residual_history(const vie_ctx *ctx, double *hist, int cap) {
  if (!ctx || !hist || cap < 0) return VIE_EINVAL;
  const int k = ctx->sol_k[ctx->last_pol];
  if (k < 0) return 0;
  const std::vector<double> &h = ctx->hist[k];
  int n = std::min<int>(cap, (int)h.size());
  for (int i = 0; i < n; ++i) hist[i] = h[i];
  return n;
}

}  // extern "C"
