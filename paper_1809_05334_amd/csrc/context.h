// Internal state of a libvie context (the opaque vie_ctx of include/vie.h)
// and the host helpers shared by the single-context entry points (api.cpp)
// and the fused multi-cell batch (batch.cpp).  Not part of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/vie.h"
#include "device_math.h"
#include "grid.h"
#include "host.h"
#include "kernels.h"

namespace vie {

enum State { S_NEW = 0, S_MESH = 1, S_BOUND = 2, S_FILLED = 3, S_FACTORED = 4, S_SOLVED = 5 };

constexpr int kMaxPack = 8192;     // doubles of the packed lattice-sum table (64 KB of LDS)
constexpr int kRedBlocks = 240;   // blocks of the two-stage reductions
constexpr int kMaxPlans = 4;      // cached cooperative triangular-solve plans per context

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Region {
  size_t off = 0, bytes = 0;
};

struct Layout {
  Region tg, t2f, area, dom, fg, half, ctp, ctm, utet, uk, colors, near_t, near_s, near_m, near_tf, near_ft, quad, pgf,
      pack;
  Region eps, alpha, gsrc, kappa, inveps, sigma;
  Region Z, Zt, nrow, ncol, nval, F, ipiv, perm, rpiv, info, lupv, lupi, lucnt, tcand, ttcnt, tblk, dinv, gcpl, trr, tbsum,
      plans;
  // structured-grid operator (VIE_GRID_FP64): geometry, element maps, kernel
  // tables (kGridSub^2 x nf), source and potential fields (kGridFields x nf)
  Region ggeo, gtet, gface, ghalf, gtab, gin, gout;
  Region jdiag;   // 1 / Z_mm of the last fill (point-Jacobi preconditioner)
  int plan_steps = 0;   // TrsvStep entries of one cooperative plan
  // one GMRES process per polarisation of a paired solve (K[0] alone otherwise)
  struct Kry {
    Region V, H, cs, sn, g, y, vb, vx, vw, vz, vu, vr, vt, vin, dpart, npart, scal, jd, rhist;
  } K[2];
  Region apart, atet, kv, idx;
  size_t total = 0;
  int64_t ld = 0;
  std::vector<int64_t> fld, foff;  // per-domain factor leading dim and offset (elements)
  std::vector<int64_t> doff;       // per-domain offset of the diagonal-block inverses (elements)
  std::vector<int64_t> goff;       // per-domain offset of the coupling blocks (elements)
  std::vector<int64_t> boff;       // per-domain offset of the triangular solves' chunk sums (elements)
  std::vector<int64_t> toff;       // per-domain offset of the tournament tree nodes (nodes)
  int restart = 0;
  int64_t ldv = 0;
};

}  // namespace vie

using namespace vie;

struct vie_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  State state = S_NEW;
  std::string err;
  MeshTopology topo;
  QuadRules quad;
  Layout L;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  int precision = VIE_FP64;
  // fill parameters
  double lambda = 0, theta = 0, phi = 0;
  PgfTable *tab = nullptr;          // host copy (heap, large)
  std::vector<dz> eps_int;
  std::vector<double> pack;         // packed lattice-sum table of the last fill
  int packlen = 0;
  std::vector<int32_t> near_off;    // offsets of the near lists per colour pair
  std::vector<int32_t> tf_off, ft_off;   // offsets (in pairs) of the touching tet-face / face-tet lists per colour
  int mv_rpw = 4;                   // matvec rows per wave (2, 4, 8)
  int trsv_kc = 2048;               // triangular-solve chunk width in columns (1024, 2048)
  int graph_steps = 0;              // Arnoldi steps per captured graph (0: plain launches)
  int trsv_coop = 0;                // triangular solves as one cooperative launch per apply
  int lu_pivot = 0;                 // 0: tournament pivoting per panel, 1: partial pivoting column by column
  int precond = 0;                  // 0: block-diagonal LU preconditioner, 1: none (M = I)
  bool factored = false;            // the factors belong to the current fill (a solve with M = I
                                    // reaches S_SOLVED without them)
  int sym_fill = 0;                 // the next bind reserves the transposed-block staging of normal-incidence fills
  bool last_sym = false;            // the last fill used it
  bool capturing = false;           // a graph capture is in progress on the stream
  int coop_grid = 0;                // co-resident thread blocks of the cooperative kernel
  struct CoopPlan {
    const void *v, *out, *s1, *s2;
    int kc, nsteps;
    size_t off;                     // byte offset of the plan in the workspace
  };
  std::vector<CoopPlan> plans;
  // captured Arnoldi steps per Krylov process set (K[0], K[1], both):
  // [0] graph_steps steps, [1] one step (tail of a restart cycle)
  hipGraphExec_t gexec[3][2] = {};
  int gexec_steps[3] = {};
  std::vector<int64_t> nrow;        // near-part CSR pattern (mixed precision), built on first use
  std::vector<int32_t> ncol;
  bool npat = false;
  std::vector<int32_t> color_off;
  int nhalf = 0, nface = 0;
  int last_pol = 0;                 // polarisation of the last solve (the TM one of a pair)
  int sol_k[2] = {-1, -1};          // Krylov process holding the last TE / TM solution, -1: none
  std::vector<double> hist[2];      // residual estimates of each Krylov process's last solve
  double *pinned = nullptr;         // small pinned host buffer for scalar read-backs
  int32_t *pin_piv = nullptr;       // pinned: the pivots read back [N], the row permutation [N]
  int64_t pin_piv_n = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr, ev4 = nullptr;
  std::vector<int32_t> piv_host;     // pivot read-back staging when no pinned buffer is allocated
  bool static_ws = false;            // bound to the library's own workspace (vie_bind_static_workspace)
  // block LU look-ahead: the next panel's tournament on a stream of its own
  // (default priority) while the rest of the trailing update runs
  hipStream_t side = nullptr;
  hipEvent_t ev_la = nullptr, ev_ts = nullptr;
  vie_fill_stats fstats{};
  // timing of the factorisation's K = 128 trailing updates: one event pair per
  // launch (pool grown on demand), pairs used by the last factorisation
  std::vector<hipEvent_t> upd_ev;
  int upd_n = 0;
  vie_factor_stats facstats{};
  // the fill in progress (set by fill_prepare): one evaluation per unordered
  // far pair, the (face, tet) entries from the tet-face kernel, the
  // reversed-separation form, the table's LDS bytes, k0^2 / 9
  bool fill_sym = false, fill_sym_face = false;
  int fill_rev = 0;
  size_t fill_lds = 0;
  double fill_k0sq9 = 0;
  double fill_kx = 0, fill_ky = 0;  // transverse wavevector of the fill
  // structured-grid operator: the mesh's grid analysis (built on first use,
  // per mesh; grid_err holds why the mesh is not a uniform Kuhn grid) and the
  // hipFFT plans of the bound workspace
  GridHost *grid = nullptr;
  std::string grid_err;
  hipfftHandle fft_tab = 0, fft_fld = 0, fft_tab_sym = 0;
  bool grid_sym = false;            // the tables hold the pairs s <= s' only (normal incidence)
  bool jdiag_ok = false;            // jdiag holds the last fill's 1 / Z_mm
  double t_fill = 0, t_factor = 0;

  template <class T>
  T *ptr(const Region &r) const {
    return reinterpret_cast<T *>(ws + r.off);
  }
};

namespace vie {

// Record a failure on the context and return its code.
inline int fail(vie_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

// defined in api.cpp
int check(vie_ctx *ctx, State need, const char *what);
ZOut zout(vie_ctx *ctx);
bool fp32_factors(const vie_ctx *ctx);
void *factor_ptr(vie_ctx *ctx, const Region &r, int64_t elem);
void launch_rhs(vie_ctx *ctx, int pol, dz *b);
int matvec(vie_ctx *ctx, const dz *x, const dz *b, dz *y);
int apply_minv_n(vie_ctx *ctx, int nv, const dz *const *v, dz *const *out, dz *const *s1, dz *const *s2);
int norm_to(vie_ctx *ctx, int k, const dz *w, int64_t N, double *dst);
std::vector<TrsvStep> trsv_plan(vie_ctx *ctx, int nv, dz *const *out, dz *const *s1, dz *const *s2);
int fill_tables(vie_ctx *ctx, double lambda_nm, double theta, double phi, const vie_c128 *eps_per_tet, int precision);
int fill_upload(vie_ctx *ctx);
int fill_prepare(vie_ctx *ctx, double lambda_nm, double theta, double phi, const vie_c128 *eps_per_tet, int precision);
ZOut zout_staging(vie_ctx *ctx);
int fill_kernels(vie_ctx *ctx);
int fill_finish(vie_ctx *ctx, bool timed);
int factor_prepare(vie_ctx *ctx, std::vector<LuDom> &doms);
int factor_panels(vie_ctx *ctx, std::vector<LuDom> &doms, bool f32, int lu_pivot, hipStream_t stream, hipStream_t side,
                  hipEvent_t ev_la, hipEvent_t ev_ts);
int factor_finish(vie_ctx *ctx, const std::vector<LuDom> &doms);

}  // namespace vie

#define HIPCK(expr)                                                                            \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(ctx, VIE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCK()                                                                                        \
  do {                                                                                                    \
    hipError_t e_ = hipGetLastError();                                                                    \
    if (e_ != hipSuccess) return fail(ctx, VIE_EDEVICE, "kernel launch (line %d): %s", __LINE__, hipGetErrorString(e_)); \
  } while (0)

