// Declarations of the libvie kernels launched from the host orchestration.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_math.h"
#include "grid.h"

namespace vie {

// Destination of the fill.  VIE_FP64: everything into the FP64 dense Z.
// VIE_MIXED_FP32: far contributions into the complex-FP32 dense Zs, the
// contributions of touching pairs (singular extraction, mass) into the FP64
// CSR near part (rowptr/cols/vals over the touching-pair pattern).
struct ZOut {
  dz *Z;
  fz *Zs;
  int64_t ld;
  const int64_t *rowptr;
  const int32_t *cols;
  dz *vals;
};

// fill (k_fill.hip)
__global__ void k_prep(int64_t nt, const TetFace *t2f, const TetGeom *tg, const double *area, const dz *eps_int,
                       double kx, double ky, double a, double b, dz *alpha, dz *gsrc, dz *kappa, dz *inv_eps);
__global__ void k_sigma(int nc, const int32_t *ctp, const int32_t *ctm, const dz *kappa, dz *sigma);
__global__ void k_zero(dz *p, int64_t n);
// sym: 0 every pair of the two lists, writing Z; 1 the same, also writing the
// transposed pair's block into outT (stored untransposed); 2 (one list twice)
// only pairs with source position > test position, both blocks as for 1.
// k_tt_far: the swapped block from the same moments (kt = 0 only);
// k_tt_far_rev (any incidence): from g_p at the reversed separations, with
// 16 doubles per thread of dynamic LDS after the table (kFarRevLds bytes).
__global__ void k_tt_far(const double *pack, int packlen, const QuadRules *qr, const TetGeom *tg, const TetFace *t2f,
                         const int32_t *test_list, int ntest, const int32_t *src_list, int nsrc, const dz *alpha,
                         const dz *gsrc, const dz *kappa, double k0sq9, ZOut out, ZOut outT, int sym);
__global__ void k_tt_far_rev(const double *pack, int packlen, const QuadRules *qr, const TetGeom *tg,
                             const TetFace *t2f, const int32_t *test_list, int ntest, const int32_t *src_list, int nsrc,
                             const dz *alpha, const dz *gsrc, const dz *kappa, double k0sq9, ZOut out, ZOut outT,
                             int sym);
constexpr int kFarRevLds = 16 * 256 * 8 + 8;
// Fused fill of many cells (the batch): one launch runs one fill kernel for
// every cell that has work for it.  Each segment holds the arguments of one
// cell's launch; it covers the fused grid's blocks [first, first + gx * gy)
// and its local block (bx, by) = ((b - first) % gx, (b - first) / gx).
// Segments are ordered by `first`.  The dynamic LDS of the launch is the
// largest of its cells' lattice-sum tables.
struct FarSeg {
  const double *pack; int packlen; const QuadRules *qr; const TetGeom *tg; const TetFace *t2f;
  const int32_t *test_list; int ntest; const int32_t *src_list; int nsrc;
  const dz *alpha, *gsrc, *kappa; double k0sq9; ZOut out, outT; int sym, gx, first;
};
struct NearSeg {
  const double *pack; int packlen; const QuadRules *qr; const TetGeom *tg; const TetFace *t2f;
  const int32_t *lt, *ls, *lmask; int npairs; const dz *alpha, *gsrc, *kappa, *inv_eps; double k0sq9; ZOut out;
  int gx, first;
};
struct TetFaceSeg {
  const double *pack; int packlen; const QuadRules *qr; const TetGeom *tg; const TetFace *t2f;
  const int32_t *test_list; int ntest; const FaceGeom *fg; int nface; const dz *alpha, *sigma, *gsrc, *kappa;
  ZOut out, outT; int swap, gx, first;
};
struct TetFaceNearSeg {
  const double *pack; int packlen; const QuadRules *qr; const TetGeom *tg; const TetFace *t2f;
  const int32_t *pairs; int npairs; const FaceGeom *fg; const dz *alpha, *sigma; ZOut out; int gx, first;
};
struct FaceTetSeg {
  const double *pack; int packlen; const QuadRules *qr; const FaceGeom *fg; const int32_t *half_list; int nhalf;
  const TetGeom *tg; const TetFace *t2f; const int32_t *src_list; int nsrc; const dz *gsrc, *kappa; ZOut out;
  int gx, first;
};
struct FaceTetNearSeg {
  const double *pack; int packlen; const QuadRules *qr; const FaceGeom *fg; const int32_t *half_list;
  const TetGeom *tg; const TetFace *t2f; const int32_t *pairs; int npairs; const dz *gsrc, *kappa; ZOut out;
  int gx, first;
};
struct FaceFaceSeg {
  const double *pack; int packlen; const QuadRules *qr; const FaceGeom *fg; const int32_t *half_list; int nhalf;
  int nface; const dz *sigma; ZOut out; int gx, first;
};
__global__ void k_tt_far_seg(const FarSeg *segs, int nseg);
__global__ void k_tt_far_rev_seg(const FarSeg *segs, int nseg);
__global__ void k_tt_near_seg(const NearSeg *segs, int nseg);
__global__ void k_tet_face_seg(const TetFaceSeg *segs, int nseg);
__global__ void k_tet_face_near_seg(const TetFaceNearSeg *segs, int nseg);
__global__ void k_face_tet_seg(const FaceTetSeg *segs, int nseg);
__global__ void k_face_tet_near_seg(const FaceTetNearSeg *segs, int nseg);
__global__ void k_face_face_seg(const FaceFaceSeg *segs, int nseg);
// Z[i][j] += Zt[j][i] for i, j < N (row-major, leading dimension ld)
__global__ void k_transpose_add_z(dz *Z, const dz *Zt, int64_t N, int64_t ld);
__global__ void k_transpose_add_c(fz *Z, const fz *Zt, int64_t N, int64_t ld);
__global__ void k_tt_near(const double *pack, int packlen, const QuadRules *qr, const TetGeom *tg, const TetFace *t2f,
                          const int32_t *lt, const int32_t *ls, const int32_t *lmask, int npairs, const dz *alpha,
                          const dz *gsrc, const dz *kappa, const dz *inv_eps, double k0sq9, ZOut out);
// swap = 1 (normal incidence, staging bound): a far pair with a half-SWG
// face also gives the (face, tet) entry, written transposed into outT
__global__ void k_tet_face(const double *pack, int packlen, const QuadRules *qr, const TetGeom *tg, const TetFace *t2f,
                           const int32_t *test_list, int ntest, const FaceGeom *fg, int nface, const dz *alpha,
                           const dz *sigma, const dz *gsrc, const dz *kappa, ZOut out, ZOut outT, int swap);
__global__ void k_tet_face_rev(const double *pack, int packlen, const QuadRules *qr, const TetGeom *tg,
                               const TetFace *t2f, const int32_t *test_list, int ntest, const FaceGeom *fg, int nface,
                               const dz *alpha, const dz *sigma, const dz *gsrc, const dz *kappa, ZOut out, ZOut outT);
__global__ void k_face_tet(const double *pack, int packlen, const QuadRules *qr, const FaceGeom *fg, const int32_t *half_list,
                           int nhalf, const TetGeom *tg, const TetFace *t2f, const int32_t *src_list, int nsrc,
                           const dz *gsrc, const dz *kappa, ZOut out);
// touching pairs from the host lists (lane = pair): (tet, surface-charge face
// index) and (half-SWG face position, tet), interleaved
__global__ void k_tet_face_near(const double *pack, int packlen, const QuadRules *qr, const TetGeom *tg,
                                const TetFace *t2f, const int32_t *pairs, int npairs, const FaceGeom *fg,
                                const dz *alpha, const dz *sigma, ZOut out);
__global__ void k_face_tet_near(const double *pack, int packlen, const QuadRules *qr, const FaceGeom *fg,
                                const int32_t *half_list, const TetGeom *tg, const TetFace *t2f, const int32_t *pairs,
                                int npairs, const dz *gsrc, const dz *kappa, ZOut out);
__global__ void k_face_face(const double *pack, int packlen, const QuadRules *qr, const FaceGeom *fg, const int32_t *half_list,
                            int nhalf, int nface, const dz *sigma, ZOut out);
__global__ void k_rhs(int64_t N, const int32_t *utet, const int32_t *uk, const TetGeom *tg, const QuadRules *qr,
                      const dz *alpha, double kix, double kiy, double kiz, double ex, double ey, double ez, dz *b);
__global__ void k_pgf_probe(const double *pack, int packlen, const double *d, int64_t n, dz *out);
__global__ void k_gather(ZOut Z, const int64_t *rows, const int64_t *cols, int64_t k, dz *out);

// block LU (k_lu.hip) and its application (k_trsv.hip)
constexpr int kTrsvNB = 512;                   // diagonal-block size of the triangular solves
constexpr int kInvColsH = 8192 / kTrsvNB;      // columns of one inverse per k_diag_inv block (128 KB of LDS)
// FP64 (_z) and FP32 (_c) factor storage
__global__ void k_copy_block_z(ZOut Z, int64_t start, int n, dz *A, int64_t lda);
__global__ void k_copy_block_c(ZOut Z, int64_t start, int n, fz *A, int64_t lda);
__global__ void k_add_near_z(ZOut Z, int64_t start, int n, dz *A, int64_t lda);
__global__ void k_add_near_c(ZOut Z, int64_t start, int n, fz *A, int64_t lda);
// The panel, swap, triangular-solve and trailing-update launches of the
// block LU advance up to kLuMaxDom domains at the same global column.
constexpr int kLuNB = 64;
constexpr int kColT = 4;        // lanes per row in the panel column kernel
constexpr int kColRows = 64;    // rows per thread block of the panel column kernel (256 / kColT)
constexpr int kLuMaxDom = 8;
constexpr int kGemm2Threads = 512;   // threads per block of the two-panel trailing update (k_lu_gemm2)
// Tournament nodes: 256 rows and four children per node; a row takes two
// lanes for FP64 factors (512 threads), one lane for FP32 (256 threads).
constexpr int kTsFanZ = 4, kTsFanC = 4;
constexpr int kTsRowsZ = kTsFanZ * kLuNB, kTsRowsC = kTsFanC * kLuNB;
constexpr int kTsLprZ = 2, kTsLprC = 1;
struct LuDom {
  void *A;            // the domain's block (dz or fz), row-major, leading dimension ld, factored in place
  int64_t ld;
  int n;
  int first_block;    // first thread block of this domain in the launch
  int32_t *ipiv;      // row swaps (LAPACK order)
  int32_t *info;      // first zero pivot (1-based), 0 if none, -1 if tournament pivoting went out of range
  void *rpiv;         // reciprocal of the current pivot (same element type as A)
  double *pval;       // per-thread-block pivot candidates (k_lu_col)
  int32_t *pidx;
  int *counter;       // zero between launches
  // tournament pivoting (k_lu_tsel / k_lu_tfin)
  int32_t *cand;      // candidate rows of each tree node, kLuNB per node (-1 = none)
  int *tcnt;          // per tree node: children that finished, zero between launches
  void *tblk;         // the panel's factored top block, kLuNB x kLuNB row-major (type of A)
};
struct LuStep {
  LuDom d[kLuMaxDom];
  int ndom, j, k0;    // current column and panel start
  int all_cols;       // k_lu_swap columns: 0 all but the panel's, 1 all, 2 only [c_lo, c_hi), 3 all but [c_lo, c_hi)
  int gcol0, gcols;   // k_lu_gemm: column tiles gcol0 .. gcol0 + gcols - 1 of A22 (gcols <= 0: to the end)
  int c_lo, c_hi;     // k_lu_swap column range (modes 2, 3); k_lu_trsm: columns [c_lo, c_hi) if c_hi > 0
};
#define VIE_DECL_LU(T)                       \
  __global__ void k_lu_pivot_##T(LuStep st); \
  __global__ void k_lu_col_##T(LuStep st);   \
  __global__ void k_lu_swap_##T(LuStep st);  \
  __global__ void k_lu_trsm_##T(LuStep st);  \
  __global__ void k_lu_gemm_##T(LuStep st);  \
  __global__ void k_lu_gemm2_##T(LuStep st); \
  __global__ void k_lu_tsel_##T(LuStep st);  \
  __global__ void k_lu_tfin_##T(LuStep st);
VIE_DECL_LU(z)
VIE_DECL_LU(c)
#undef VIE_DECL_LU
// (k_trsv.hip)
__global__ void k_permute(int n, int64_t off, const int32_t *perm, const dz *v, dz *z);
__global__ void k_diag_inv_z(const dz *F, int64_t ld, int n, int nb, int lower, dz *Dinv);
__global__ void k_diag_inv_c(const fz *F, int64_t ld, int n, int nb, int lower, fz *Dinv);
// coupling blocks G_b = T[b, p] inv(T_pp) of one domain's L (p = b - 1, b >= 1) or U
// (p = b + 1, b <= nbk - 2) sweep, each kTrsvNB x kTrsvNB (k_trsv.hip)
__global__ void k_trsv_coupling_z(const dz *F, int64_t ld, int n, int lower, const dz *INV, dz *G);
__global__ void k_trsv_coupling_c(const fz *F, int64_t ld, int n, int lower, const fz *INV, fz *G);
// One launch advances the blocked triangular solves of up to kTrsvMaxDom
// domains by one diagonal block each (k_trsv.hip).
constexpr int kTrsvGroupsH = kTrsvNB / 16;   // work items of 16 rows per diagonal block
constexpr int kTrsvMaxDom = 8;
// Row sums over the solved columns come in chunks of kTrsvSumCols columns
// (a work item covers kc = 1024 or 2048 columns, one or two chunks, with the
// same sums either way); a row's chunk sums are read by 64 lanes, two each,
// which bounds a domain at kTrsvChunksMax * kTrsvSumCols unknowns.
constexpr int kTrsvSumCols = 1024;
constexpr int kTrsvChunksMax = 128;
struct TrsvDom {
  const void *F;      // the domain's LU factors (dz or fz, row-major, leading dimension ld)
  const void *G;      // coupling block of block j: T[j, j-1] inv(T_{j-1,j-1}) (row-major, leading
                      // dimension gld = kTrsvNB, zero past its sizes; gld = 0 when j has no predecessor)
  const void *INV;    // inv(T_{j-1,j-1}) (pm x pm, row-major)
  const dz *rhs[2];   // right-hand sides, domain-local, per vector (read only)
  dz *sol[2];         // solutions, domain-local, per vector
  const dz *rin;      // r_{j-1}, the previous block's reduced right-hand side (vector q at q * kTrsvNB)
  dz *rout;           // r_j, written by this step
  // chunk sums over the solved columns: for row i of a block, chunk c of vector q at
  // q * kTrsvNB * bst + i * bst + c.  bsum_in holds nci chunks for this step's block
  // (written by the previous step); bsum_out receives those of the next block
  const dz *bsum_in;
  dz *bsum_out;
  int64_t ld;
  // blocks of the step: [cb0, cb0+cm) two back (solution in sol), [pb0, pb0+pm) the previous one
  // (its r in rin), [nb0, nb0+nm) the one reduced; nm = 0: only solve the previous block
  int n, cb0, cm, pb0, pm, nb0, nm, gld;
  // the next block's rows [br0, br0+brm) against the solved columns [bc0, bc0+bk):
  // nrg groups of 16 rows times nco work items of kc columns (brm = 0: none)
  int bst, nci, br0, brm, bc0, bk, nrg, nco;
  // the entry's work items: reduction items (block j) from first_block, solution
  // items (block j-1) from first_z, chunk-sum items from first_bulk; a step numbers
  // every entry's reduction items first, then the solution items, then the chunk sums
  int first_block, first_z, first_bulk;
  const int *active;  // (fused batch) the cell's flag: 0 skips the domain; nullptr always runs
};
// chunk sums per row of a domain of n unknowns (the row stride bst)
inline int trsv_bsum_stride(int64_t n) { return (int)std::max<int64_t>(1, (n + kTrsvSumCols - 1) / kTrsvSumCols); }
// work items of one domain's entry in a step
inline int trsv_chain_items(const TrsvDom &D) { return D.nm > 0 ? kTrsvGroupsH : 0; }
inline int trsv_z_items(const TrsvDom &D) { return D.pm > 0 ? kTrsvGroupsH : 0; }
inline int trsv_bulk_items(const TrsvDom &D) { return D.nm > 0 ? D.nrg * D.nco : 0; }
// first_block / first_z / first_bulk of entries d[0 .. nd) in that order; returns
// the reduction items, *zend the end of the solution items, *total every item
inline int trsv_number_items(TrsvDom *d, int nd, int *zend, int *total) {
  int c = 0;
  for (int i = 0; i < nd; ++i) {
    d[i].first_block = c;
    c += trsv_chain_items(d[i]);
  }
  int z = c;
  for (int i = 0; i < nd; ++i) {
    d[i].first_z = z;
    z += trsv_z_items(d[i]);
  }
  int b = z;
  for (int i = 0; i < nd; ++i) {
    d[i].first_bulk = b;
    b += trsv_bulk_items(d[i]);
  }
  *zend = z;
  *total = b;
  return c;
}
struct TrsvStep {
  TrsvDom d[kTrsvMaxDom];
  int ndom, lower;
  int chain_blocks;   // reduction items, numbered first
  int z_end;          // end of the solution items
  int total_blocks;   // thread blocks (work items) of the step over all its domains
};
// variants by factor type (_z FP64, _c FP32) and columns per work item
// (1024 or 2048, the same sums); vectors and arithmetic FP64.
// k_trsv_step2_*: two right-hand sides per pass over the factors (each
// vector's sums in the order of the one-vector kernel).
// k_trsv_coop_*: every step of a plan in one cooperative launch.
#define VIE_DECL_TRSV(T, K)                                  \
  __global__ void k_trsv_step_##T##_k##K(TrsvStep st);       \
  __global__ void k_trsv_step2_##T##_k##K(TrsvStep st);      \
  __global__ void k_trsv_coop_##T##_k##K(const TrsvStep *plan, int nsteps);
// k_trsv_stepd_*: one step of a batch's fused solves, one vector per cell,
// the step's domains (any number) read from device memory; work items of
// kTrsvSumCols columns
__global__ void k_trsv_stepd_z(const TrsvDom *doms, int ndom, int lower, int chain_blocks, int z_end);
__global__ void k_trsv_stepd_c(const TrsvDom *doms, int ndom, int lower, int chain_blocks, int z_end);
VIE_DECL_TRSV(z, 1024)
VIE_DECL_TRSV(z, 2048)
VIE_DECL_TRSV(c, 1024)
VIE_DECL_TRSV(c, 2048)
#undef VIE_DECL_TRSV

// Krylov (k_krylov.hip).  Matvec variants by rows per wave (2, 4, 8): a block
// of 4 waves owns 4 * RPW rows; the autotuner picks one per context.  The
// k_matvec2_* variants take two vectors through one pass over Z: y_q = Z x_q
// (or b_q - Z x_q when b_q is given), each sum in the order of the one-vector
// kernel.
// One cell's GMRES process in a batch's fused Arnoldi step (k_b_*): its
// operator, Krylov basis and work vectors, the reduction partials over nred
// blocks, and the row permutation of its block preconditioner.
constexpr int kCellMaxDom = 8;
struct KryCell {
  const dz *Z;                 // FP64 operator, or nullptr: the mixed operator below
  const fz *Zs; const int64_t *rowptr; const int32_t *cols; const dz *vals;
  int64_t ld, N, ldv;
  dz *V; int *jd; dz *vin, *z, *w, *tmp;
  dz *H; int ldh; double *cs; dz *sn, *g, *y; double *rhist, *scal;
  dz *dpart; double *npart; int nred;
  const int32_t *perm; int ndom; int64_t dstart[kCellMaxDom];
  int precond;                 // 1: no preconditioner (the product takes V_j itself)
  int rpw;                     // matvec rows per wave (2, 4, 8): 4 RPW rows per thread block
};
__global__ void k_b_arn_begin(const KryCell *cells, const int *pre, int nc, const int *act);
__global__ void k_b_permute(const KryCell *cells, const int *pre, int nc, const int *act);
__global__ void k_b_matvec(const KryCell *cells, const int *pre, int nc, const int *act);
__global__ void k_b_dots_j(const KryCell *cells, const int *pre, int nc, const int *act);
__global__ void k_b_dots_reduce_j(const KryCell *cells, const int *pre, int nc, const int *act, int pass);
__global__ void k_b_update_j(const KryCell *cells, const int *pre, int nc, const int *act);
__global__ void k_b_norm2(const KryCell *cells, const int *pre, int nc, const int *act);
__global__ void k_b_norm_givens(const KryCell *cells, int nc, const int *act);
__global__ void k_b_scale_j(const KryCell *cells, const int *pre, int nc, const int *act);
__global__ void k_b_jinc(const KryCell *cells, int nc, const int *act, double *res);

struct MvVecs {
  const dz *x[2];
  const dz *b[2];
  dz *y[2];
};
#define VIE_DECL_MATVEC(R)                                                                                      \
  __global__ void k_matvec_r##R(const dz *Z, int64_t ld, int64_t N, const dz *x, const dz *b, dz *y);           \
  __global__ void k_matvec_mixed_r##R(const fz *Zs, int64_t ld, int64_t N, const int64_t *rowptr,               \
                                      const int32_t *cols, const dz *vals, const dz *x, const dz *b, dz *y);    \
  __global__ void k_matvec2_r##R(const dz *Z, int64_t ld, int64_t N, MvVecs v);                                \
  __global__ void k_matvec2_mixed_r##R(const fz *Zs, int64_t ld, int64_t N, const int64_t *rowptr,              \
                                       const int32_t *cols, const dz *vals, MvVecs v);
VIE_DECL_MATVEC(2)
VIE_DECL_MATVEC(4)
VIE_DECL_MATVEC(8)
#undef VIE_DECL_MATVEC
__global__ void k_combine(const dz *V, int64_t ldv, int nv, const dz *c, dz *y, int64_t N);
__global__ void k_norm2(const dz *w, int64_t N, double *part);
__global__ void k_norm_reduce(const double *part, int nblk, double *out);
__global__ void k_scale(const dz *w, const double *nrm, dz *v, int64_t N);
__global__ void k_axpy(dz *x, const dz *u, int64_t N);
// point-Jacobi preconditioner: dinv = 1 / Z_mm from the stored operator (dense
// entry, or the FP32 dense part plus the CSR near part, or the CSR alone),
// and z = dinv v
__global__ void k_jacobi_diag(int64_t N, ZOut Z, dz *dinv);
__global__ void k_jacobi_apply(int64_t N, const dz *dinv, const dz *v, dz *z);
__global__ void k_copy(dz *d, const dz *s, int64_t N);
__global__ void k_fill_const(dz *x, int64_t N, double re, double im);
__global__ void k_backsolve(const dz *H, int ldh, int k, const dz *g, dz *y);
__global__ void k_ginit(dz *g, int m1, const double *beta);
// one Arnoldi step with the column index j read from device memory
__global__ void k_arn_begin(const dz *V, int64_t ldv, const int *jd, dz *vin, int64_t N);
__global__ void k_dots_j(const dz *V, int64_t ldv, const int *jd, const dz *w, int64_t N, dz *part);
__global__ void k_dots_reduce_j(const dz *part, int nblk, const int *jd, dz *H, int ldh, dz *y, int pass);
__global__ void k_update_j(const dz *V, int64_t ldv, const int *jd, const dz *c, dz *w, int64_t N);
__global__ void k_scale_j(const dz *w, const double *nrm, dz *V, int64_t ldv, const int *jd, int64_t N);
__global__ void k_givens_j(dz *H, int ldh, const int *jd, const double *hn, double *cs, dz *sn, dz *g, double *hist);
__global__ void k_jset(int *jd, int v);
__global__ void k_jinc(int *jd);

// outputs (k_absorb.hip)
// (per_tet, nullable: each tetrahedron's term before the domain sums)
__global__ void k_absorb(int64_t nt, int ndom, const TetGeom *tg, const TetFace *t2f, const int32_t *dom,
                         const QuadRules *qr, const dz *gsrc, const dz *inv_eps, const dz *x, double *part,
                         double *per_tet);
__global__ void k_project(int64_t nt, const TetGeom *tg, const TetFace *t2f, const QuadRules *qr, const dz *gsrc,
                          const dz *kappa, const dz *x, int nk, const double *kv, double *part);
__global__ void k_reduce_cols(const double *part, int nblk, int width, double *out);
__global__ void k_field(int64_t np, const double *pts, const int32_t *tet, const TetGeom *tg, const TetFace *t2f,
                        const dz *gsrc, const dz *inv_eps, const dz *x, dz *e);

// structured-grid far operator (k_grid.hip); grid (ceil(nf / 256), kGridSub^2, or
// kGridSymPairs with sym) for the table, ceil(nf / 32) blocks for the products (the _sym
// form reads tables of the pairs s <= s' only), ceil(N / 4) blocks (a wave per unknown)
// for the apply; 256 threads
__global__ void k_grid_table(const double *pack, int packlen, const GridGeom *gg, double kx, double ky, double scale,
                             int sym, dz *tab);
__global__ void k_grid_gather_tet(int64_t nt, const GridGeom *gg, const int32_t *gtet, const TetGeom *tg,
                                  const TetFace *t2f, const dz *gsrc, const dz *kappa, const dz *x, double kx,
                                  double ky, dz *fld);
__global__ void k_grid_gather_face(int nface, const GridGeom *gg, const int32_t *gface, const FaceGeom *fg,
                                   const dz *sigma, const dz *x, double kx, double ky, dz *fld);
__global__ void k_grid_mul(int64_t nf, const dz *tab, const dz *fin, dz *fout);
__global__ void k_grid_mul_sym(int64_t nf, int nx, int ny, int pz, const dz *tab, const dz *fin, dz *fout);
__global__ void k_grid_apply(int64_t N, const GridGeom *gg, const int32_t *gtet, const int32_t *gface,
                             const int32_t *ghalf, const int32_t *utet, const int32_t *uk, const TetGeom *tg,
                             const FaceGeom *fg, const dz *alpha, const dz *fout, double k0sq9, double kx, double ky,
                             const int64_t *rowptr, const int32_t *cols, const dz *vals, const dz *x, const dz *b,
                             dz *y);

}  // namespace vie
