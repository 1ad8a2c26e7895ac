/*
 * vie.h -- C-ABI of libvie: the periodic volume-integral-equation method of
 * moments for plasmonic thin-film cells, on one AMD Instinct MI355X (gfx950).
 *
 * Method (He, Gu, Sha, Chen, "Efficient Volumetric Method of Moments for
 * Modeling Plasmonic Thin-Film Solar Cells with Periodic Structures"):
 *   - VIE in the polarisation current, SWG basis, Galerkin testing
 *     (Sec. 2.1, Eqs. 1-2; contrast kappa = (eps_r - 1)/eps_r);
 *   - two-dimensional periodic Green's function with the incidence Bloch
 *     phase, evaluated with the Ewald split (Sec. 2.2, Eqs. 3-4);
 *   - material-domain block partition and block-diagonal preconditioner
 *     (Sec. 2.3, Eqs. 5-6), applied on the right inside GMRES (Sec. 3);
 *   - absorbed power Im(eps)|E|^2 per domain (Sec. 3, Eq. 7).
 *
 * Conventions shared by every entry point:
 *   - lengths in nm, angles in radians;
 *   - permittivities use the optics sign (Im eps >= 0 is lossy); internally
 *     the library works in exp(+j w t) (Sec. 2.1) with eps_int = conj(eps);
 *   - the incident plane wave arrives from +z with unit amplitude,
 *     k = k0 (sin th cos ph, sin th sin ph, -cos th); TE: E || (-sin ph, cos ph, 0),
 *     TM: E || (cos th cos ph, cos th sin ph, sin th);
 *   - every call returns VIE_OK (0) or a negative vie_status; the message of
 *     the last failure is available from vie_last_error().
 *
 * Memory: host inputs are copied before a call returns.  All device memory
 * a context uses lives in ONE workspace: caller-owned memory bound with
 * vie_bind_workspace (the library never allocates device memory itself), or
 * the library's fixed per-device workspace bound with
 * vie_bind_static_workspace.  The caller keeps its workspace alive until
 * vie_destroy or the next bind.
 * Work is issued on the stream given to vie_create; calls that return
 * results to host buffers synchronise that stream.
 *
 * Call order: create -> mesh_upload -> bind_workspace -> fill -> precond_factor
 * -> solve (any number of times, per polarisation) -> absorption.  A new fill
 * (new wavelength, angles or permittivities) invalidates the factor and the
 * solution.  Any other order returns VIE_ESTATE.  A context is not thread-safe;
 * distinct contexts may run concurrently on distinct streams.
 */
#ifndef VIE_H
#define VIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vie_ctx vie_ctx;

typedef struct {
  double re, im;
} vie_c128;

typedef enum {
  VIE_OK = 0,
  VIE_EINVAL = -1,     /* bad argument or bad mesh */
  VIE_ESTATE = -2,     /* call out of order */
  VIE_ENOMEM = -3,     /* workspace too small */
  VIE_ENOCONV = -4,    /* GMRES hit max_iter; solution and info still written */
  VIE_EWOOD = -5,      /* a Floquet order grazes the cell plane (Rayleigh-Wood anomaly) */
  VIE_ESINGULAR = -6,  /* zero pivot in a diagonal-block factorisation */
  VIE_EDEVICE = -7     /* HIP runtime error */
} vie_status;

enum { VIE_TE = 0, VIE_TM = 1 };

/* Storage precision of the impedance matrix.
 * VIE_FP64: Z dense in complex FP64 (16 bytes per entry).
 * VIE_MIXED_FP32: the far part of Z dense in complex FP32 (8 bytes per
 *   entry); every contribution of a touching element pair (singularity-
 *   extracted self and neighbour integrals, near-field Ewald remainders, the
 *   mass term) kept in FP64 in a sparse part over the touching-pair pattern.
 *   The block preconditioner is factored in FP32 (FP32 matrix cores) from
 *   that operator and its factors are stored in FP32.  Products with Z,
 *   preconditioner applications (FP32 factors read, FP64 arithmetic), the
 *   Krylov basis, Hessenberg/Givens updates and the true residual that closes
 *   every restart cycle run in FP64 on the mixed operator, so the solve
 *   converges to the tolerance of that operator; its difference from the FP64
 *   Z is the FP32 rounding of far entries.
 * VIE_GRID_FP64: structured-grid operator for a uniform Kuhn brick grid
 *   (every brick split along its (0,0,0)-(1,1,1) diagonal, at least two
 *   bricks per lattice period; vie_bind_workspace returns VIE_EINVAL for any
 *   other mesh).  Z is never stored: the near part is the FP64 sparse part
 *   above; the far part is applied by FFT.  Each far product-rule term is a
 *   lattice sum between quadrature points, and on such a grid the points fall
 *   on 60 sublattices whose kernels depend only on the brick offset
 *   (circulant in x and y after a Bloch modulation, Toeplitz in z).  The fill
 *   tabulates those kernels (60^2 x nx ny 2(nz+1) complex values) instead of
 *   the N^2 far entries; a product with Z costs two batched 3D FFTs of 132
 *   fields plus a per-frequency contraction.  Same Z as VIE_FP64 to
 *   rounding.  There is no block preconditioner (vie_precond_factor returns
 *   VIE_EINVAL; solve with VIE_OPT_PRECOND 2, point Jacobi, or 1), no vie_read_Z (vie_apply_Z
 *   gives Z x), no graph-captured steps, no batch and no static workspace.
 *   hipFFT allocates its plans' work areas at bind. */
enum { VIE_FP64 = 0, VIE_MIXED_FP32 = 1, VIE_GRID_FP64 = 2 };

typedef struct {
  int iters;                 /* total GMRES iterations (all restarts, all refinement steps) */
  int restarts;              /* GMRES restarts */
  int refine_steps;          /* restart cycles (restarts + 1), each closed by an FP64 true residual
                              * b - Z x of the stored operator.  In VIE_MIXED_FP32 that operator holds
                              * the far entries rounded to FP32: the cycles converge on it and do not
                              * refine toward the FP64 operator (the two differ by that rounding) */
  double true_rel_residual;  /* ||b - Z x|| / ||b|| recomputed in FP64 at the end */
  double t_fill_ms;          /* device time of the last vie_fill */
  double t_factor_ms;        /* device time of the last vie_precond_factor */
  double t_solve_ms;         /* device time of this vie_solve (of the pair for vie_solve_pair) */
  int converged;             /* 1 if the stopping test was met, 0 at max_iter */
} vie_solve_info;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t
 * (NULL = the device's null stream).  *out receives the handle. */
int vie_create(vie_ctx **out, int device, void *hip_stream);
int vie_destroy(vie_ctx *ctx);

/* Move the context to another stream of the same device (hipStream_t; NULL =
 * the null stream).  Once a workspace is bound it first waits for the work
 * already issued on the old stream; before that the context has issued no
 * device work, so a scheduler can prepare a context (mesh upload, workspace
 * query) and pick the stream the request will run on later. */
int vie_set_stream(vie_ctx *ctx, void *hip_stream);

/* Upload a tetrahedral mesh of ONE unit cell [0,a] x [0,b] x [zmin,zmax]
 * (Sec. 2.2: only one unit cell is modelled, the periodic Green's function
 * supplies the Bloch condition; Fig. 1 geometry).
 *   verts_nm   [3*nv]  vertex coordinates (x,y,z) in nm; vertices on the
 *                      x = a / y = b walls must have partners on x = 0 / y = 0
 *   tets       [4*nt]  0-based vertex ids of each tetrahedron (any orientation)
 *   tet_domain [nt]    material domain id in [0, ndom) (Sec. 2.3, Eq. 5 blocks);
 *                      a face between two domains belongs to the lower id
 *   a, b               periods along x and y (Sec. 2.2)
 * Builds the SWG unknowns (one per face; wall faces paired into Bloch-periodic
 * functions; top/bottom faces are half-SWGs), ordered domain-major.  Host-only:
 * no device work until the workspace is bound.  Errors: VIE_EINVAL for
 * degenerate or non-periodic meshes, or fewer than 2 cells per periodic
 * direction (every tetrahedron must span at most a/2 in x and b/2 in y). */
int vie_mesh_upload(vie_ctx *ctx, const double *verts_nm, int64_t nv, const int32_t *tets, int64_t nt,
                    const int32_t *tet_domain, int32_t ndom, double a_nm, double b_nm);

int64_t vie_num_unknowns(const vie_ctx *ctx);

/* starts_ends [2*ndom]: unknown range [start, end) of each domain's diagonal block. */
int vie_domain_ranges(const vie_ctx *ctx, int64_t *starts_ends);

/* Bytes of device workspace needed for `precision` and GMRES `restart`. */
size_t vie_workspace_bytes(const vie_ctx *ctx, int precision, int restart);

/* Bind caller-owned device memory (>= vie_workspace_bytes, 256-byte aligned)
 * and upload the mesh tables into it.  VIE_ENOMEM if too small. */
int vie_bind_workspace(vie_ctx *ctx, void *dev_ptr, size_t bytes, int precision, int restart);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bind the
 * library's own workspace instead of a caller-owned one, then use the context
 * exactly as after vie_bind_workspace.  The library holds one such workspace
 * per device, 64 MiB (VIE_STATIC_WORKSPACE_BYTES), from its first vie_create
 * on that device until the process ends; this call allocates nothing (no
 * device memory, no pinned host memory).  A mesh whose
 * vie_workspace_bytes(precision, restart) exceeds it gets VIE_ENOMEM (roughly
 * N <= 1,400 unknowns in FP64, 2,000 mixed, at restart 100).  Every context
 * on a device shares the one workspace, which keeps what the last holder
 * wrote: binding it to a context first waits for the previous holder's
 * stream, then takes the workspace from it (the previous holder's next call
 * returns VIE_ESTATE until it binds again).  Calls on two contexts that hold
 * it in turn must not overlap in time: they race on the same memory.
 * Errors as vie_bind_workspace, plus VIE_ENOMEM when the mesh does not fit. */
#define VIE_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int vie_bind_static_workspace(vie_ctx *ctx, int precision, int restart);

/* Fill Z (dense, complex, row-major, domain-major unknowns) for wavelength
 * lambda_nm, incidence (theta, phi) and per-tetrahedron permittivity
 * eps_per_tet [nt] (Sec. 2.1, Eq. 2 with the periodic Green's function of
 * Sec. 2.2, Eqs. 3-4).  precision: VIE_FP64 or VIE_MIXED_FP32 (must match the
 * bound workspace).  VIE_EWOOD if a non-specular Floquet order has
 * |gamma_pq| / k0 < 0.02; VIE_EINVAL if a permittivity is zero or not finite. */
int vie_fill(vie_ctx *ctx, double lambda_nm, double theta_rad, double phi_rad, const vie_c128 *eps_per_tet,
             int precision);

/* LU factorisation P A_dd = L U of every diagonal block A_dd (Sec. 2.3,
 * Eq. 6), with tournament pivoting per 64-column panel by default or partial
 * pivoting column by column (VIE_OPT_LU_PIVOT).  VIE_ESINGULAR on a zero
 * pivot (the message names the domain and the column); VIE_EINVAL if a
 * domain has more than 131,072 unknowns (the bound of the triangular solves'
 * row sums).  Any factors of an earlier call are void from the start of the
 * call: after a failure, vie_solve, vie_solve_pair and vie_precond_apply
 * return VIE_ESTATE until a factorisation succeeds (the no-preconditioner
 * option aside). */
int vie_precond_factor(vie_ctx *ctx);

/* Right-preconditioned restarted GMRES(restart) on Z M^-1 y = b, x = M^-1 y,
 * x0 = 0, for the incident polarisation `polarisation` (VIE_TE / VIE_TM),
 * stopping when the residual estimate falls below tol * ||b|| (Sec. 3).
 * The true FP64 residual is recomputed at the end (info->true_rel_residual).
 * VIE_ENOCONV after max_iter iterations (x and info still written).
 * `info` may be NULL. */
int vie_solve(vie_ctx *ctx, int polarisation, double tol, int max_iter, int restart, vie_solve_info *info);

/* Both polarisations of the incident wave at once (Sec. 3 solves TE and TM
 * for every incidence): two GMRES processes, TE and TM, run in lockstep and
 * share each pass over Z (matvec) and over the LU factors (preconditioner
 * apply), two vectors per pass.  Each process computes the same bits as
 * vie_solve for its polarisation; one that converges first drops out and the
 * other goes on alone.  info [2] (TE, TM; nullable): the shared wall time in
 * t_solve_ms of both.  Afterwards vie_absorption / vie_read_solution /
 * vie_residual_history refer to TM; vie_absorption_pol and
 * vie_read_solution_pol reach either.  VIE_ENOCONV if either stops at
 * max_iter (both solutions and info still written). */
int vie_solve_pair(vie_ctx *ctx, double tol, int max_iter, int restart, vie_solve_info *info);

/* Absorptance (absorbed / incident power) per domain of the last solution
 * (Sec. 3, Eq. 7, normalised by the incident power crossing one cell):
 *   A_d = k0 sum_{T in d} Im(eps_T) / |eps_T|^2 int_T |D/eps0|^2 dV / (cos th a b).
 * absorptance_per_domain [ndom]; R, T (nullable): reflectance and
 * transmittance summed over the propagating Floquet orders. */
int vie_absorption(vie_ctx *ctx, double *absorptance_per_domain, double *R, double *T);

/* The same for the solution of polarisation `polarisation` of the last
 * vie_solve or vie_solve_pair; VIE_ESTATE if that solve did not cover it. */
int vie_absorption_pol(vie_ctx *ctx, int polarisation, double *absorptance_per_domain, double *R, double *T);

/* Each tetrahedron's share of the absorptance of the last solution of
 * polarisation `polarisation` (-1: the last solve's), the term of Eq. 7 for
 * one tetrahedron with the same normalisation, so that the shares of a
 * domain's tetrahedra add up to its absorptance (up to summation order):
 *   per_tet[T] = k0 Im(1/eps_T) int_T |D/eps0|^2 dV / (cos th a b).
 * Divided by the tetrahedron's volume it is the absorption density whose
 * maps Sec. 3 shows (Fig. 5).  per_tet [number of tetrahedra], host memory,
 * mesh order.  VIE_ESTATE before a solve or for a polarisation the last solve
 * did not cover. */
int vie_absorption_per_tet(vie_ctx *ctx, int polarisation, double *per_tet);

/* The field of the last solution of polarisation `polarisation` (-1: the last
 * solve's) at points inside the structure, for field maps on a plane (Sec. 3,
 * the profiles behind Fig. 5): on the tetrahedron T holding a point, the SWG
 * expansion gives D/eps0 (Sec. 2.1) and
 *   e[3i + d] = (D/eps0)_d / eps_T,  the field E/E0 of a unit incident wave,
 * in the library's exp(+j w t) convention (conjugate for exp(-j w t)).
 * points [3 npts] (x, y, z in nm), host memory.  e [3 npts], host memory.
 * tet [npts] (nullable), host memory: the tetrahedron holding each point, the
 * lowest index when a point lies on a face shared by several, -1 when it lies
 * in none (e = 0 there).  Points are located on the host (a bin grid over
 * the mesh); the field is evaluated on the device, with the points staged
 * through the Krylov-basis region of the workspace, which this call
 * overwrites (a later solve starts its own basis).  VIE_ESTATE before a solve
 * or for a polarisation the last solve did not cover. */
int vie_sample_field(vie_ctx *ctx, int polarisation, const double *points, int64_t npts, vie_c128 *e,
                     int32_t *tet);

const char *vie_last_error(const vie_ctx *ctx);

/* ---------------------------------------------------------------- diagnostics
 * Read-back helpers used by tests; they synchronise the context's stream. */

/* Face table in unknown order: face_vid [3N] (vertex ids as the face sits in
 * T+), tplus [N], tminus [N] (-1 for a half-SWG), dom [N].  Any pointer may be NULL. */
int vie_export_faces(const vie_ctx *ctx, int32_t *face_vid, int32_t *tplus, int32_t *tminus, int32_t *dom);

/* out[i] = Z[rows[i], cols[i]] (FP64 value; in mixed precision the stored
 * FP32 far part plus the FP64 near part). */
int vie_read_Z(const vie_ctx *ctx, const int64_t *rows, const int64_t *cols, int64_t k, vie_c128 *out);

/* Right-hand side of the last solve's polarisation, and the last solution x [N]. */
int vie_read_rhs(const vie_ctx *ctx, vie_c128 *b);
int vie_read_solution(const vie_ctx *ctx, vie_c128 *x);
/* The last solution of polarisation `polarisation` (VIE_ESTATE if none). */
int vie_read_solution_pol(const vie_ctx *ctx, int polarisation, vie_c128 *x);

/* Evaluate g_p(r, r') (Sec. 2.2, Eqs. 3-4) on the device at n separations
 * delta_host [3n] = r - r', with the tables of the last vie_fill.
 * out [n].  Needs a bound workspace and a completed fill. */
int vie_pgf_eval(vie_ctx *ctx, const double *delta_host, int64_t n, vie_c128 *out);

/* z = M^{-1} v for the block-diagonal preconditioner of the last
 * vie_precond_factor (Sec. 2.3, Eq. 6: M = blockdiag(A_dd)); v, z [N] host
 * vectors in unknown order.  Clobbers the solver's work vectors but not the
 * last solution or right-hand side.  VIE_ESTATE before a factorisation. */
int vie_precond_apply(vie_ctx *ctx, const vie_c128 *v, vie_c128 *z);

/* ---------------------------------------------------------------- tuning
 * Launch shapes, graph capture, the pivoting of the block LU and the choice
 * of preconditioner.  Apart from VIE_OPT_LU_PIVOT and VIE_OPT_PRECOND none of
 * them changes a result: every variant computes the same sums in the same
 * order. */
enum {
  VIE_OPT_GRAPH_STEPS = 1,  /* Arnoldi steps per captured HIP graph, 0 = plain launches (default);
                             * residual estimates are read back once per graph launch, so a solve
                             * may run up to this many steps past convergence (unused).  Needs a
                             * non-null stream: vie_solve returns VIE_EINVAL on the null stream */
  VIE_OPT_MATVEC_ROWS = 2,  /* matvec rows per wave: 2, 4 (default) or 8 */
  VIE_OPT_TRSV_CHUNK = 3,   /* triangular-solve columns per update work item: 1024 or 2048 (default) */
  VIE_OPT_TRSV_COOP = 4,    /* 1: each preconditioner apply runs its triangular-solve steps in one
                             * cooperative launch with grid barriers between steps (not inside
                             * captured graphs); 0 (default): one
                             * launch per step.  Use 1 only where no other context's work needs
                             * the device at the same time (a cooperative grid holds every CU). */
  VIE_OPT_LU_PIVOT = 5,     /* row pivoting of the next vie_precond_factor: 0 (default) tournament
                             * pivoting, the pivot rows of each 64-column panel chosen by a
                             * reduction tree of partial-pivoting eliminations on 256-row slices;
                             * 1: partial pivoting column by column.  Both give P A = L U; the
                             * factors, and so the rounding of M^{-1} v, differ between them */
  VIE_OPT_SYM_FILL = 6,     /* 1: the workspace bound next also holds a second N x ld copy of Z's
                             * far part, and every fill evaluates each unordered far tetrahedron
                             * pair once, writing the swapped pair's block there and adding it
                             * transposed into Z.  At normal incidence (kt = 0) g_p is even in
                             * r - r'; at oblique incidence g_p(r' - r) is the conjugate of
                             * g_p(r - r') plus a term of the propagating Floquet orders (Sec. 2.2,
                             * Eqs. 3-4, real wavenumber), formed in the same lattice-sum
                             * evaluation.  Z differs only by rounding.  Set it before
                             * vie_workspace_bytes / vie_bind_workspace (VIE_ESTATE after);
                             * 0 (default): no staging */
  VIE_OPT_PRECOND = 7       /* preconditioner of the next vie_solve / vie_solve_pair: 0 (default)
                             * the block-diagonal M of the last vie_precond_factor (Sec. 2.3,
                             * Eq. 6); 1: none, M = I (GMRES on Z x = b, the reference against
                             * which Sec. 3 compares the block preconditioner), for which a
                             * completed fill suffices; 2: point Jacobi, M = diag(Z) of the last
                             * fill (also needs only the fill; not in the batch).  The iterations
                             * and the rounding of x differ between them */
};
int vie_set_option(vie_ctx *ctx, int option, int value);
int vie_get_option(const vie_ctx *ctx, int option, int *value);

typedef struct {
  double matvec_ms[6];   /* per product, rows per wave 2, 4, 8: one vector, then two */
  double apply_ms[4];    /* per preconditioner apply, work items of 1024 and 2048 columns: one
                          * vector, then two */
  int matvec_rows, trsv_chunk;   /* the picks, now set on the context */
} vie_tuning;

/* Autotuner: time each matvec and triangular-solve variant on this context's
 * operator and factors (reps timed runs after one warm-up, HIP events) and
 * keep the fastest.  Needs a completed factorisation; clobbers the solver's
 * work vectors but not the last solution.  `out` may be NULL. */
int vie_autotune(vie_ctx *ctx, int reps, vie_tuning *out);

/* ---------------------------------------------------------------- batch
 * Many independent unit cells solved together (the batched form of the
 * method: one (cell, wavelength, angles, polarisation) solve per cell, as in
 * Sec. 3's sweeps).  Each cell is an ordinary context (mesh uploaded,
 * workspace bound, all in the same precision) that keeps its own Z, factors
 * and Krylov basis; the batch launches each step of the method once for all
 * of them:
 *   - fill: the lattice-sum tables of every cell fitted on host threads, then
 *     one launch per fill kernel and colour pair (or colour) covering every
 *     cell, each cell's share of the grid described by a segment table;
 *   - factor: one blocked LU (Sec. 2.3, Eq. 6) advancing every cell's
 *     domains together, panel by panel;
 *   - solve: right-preconditioned GMRES (Sec. 3) with the Arnoldi steps of
 *     all cells in one launch sequence (fused matvec, triangular solves over
 *     every cell's domains, Gram-Schmidt, norms, Givens), replayed as one
 *     captured HIP graph per step (VIE_BATCH_GRAPH), each cell stepping until
 *     its own stopping test; restart updates per cell.
 * Per cell the results equal those of vie_fill / vie_precond_factor /
 * vie_solve on that context up to the summation order of the reductions.
 * After a batch solve each cell answers vie_absorption, vie_absorption_pol,
 * vie_read_solution as after vie_solve.  A batch issues all work on its own
 * stream; binding sets every cell's stream to it. */
typedef struct vie_batch vie_batch;
enum { VIE_BATCH_GRAPH = 1 };   /* 1 (default): capture the fused Arnoldi step once and replay it */
int vie_batch_create(vie_batch **out, int device, void *hip_stream);
int vie_batch_destroy(vie_batch *b);
const char *vie_batch_last_error(const vie_batch *b);
/* Device bytes of the batch's own tables (segment tables, descriptors, the
 * merged triangular-solve plan) for ncells cells. */
size_t vie_batch_workspace_bytes(int ncells);
/* cells [ncells]: bound contexts of one device and one precision, each used
 * by no other thread or batch while bound here; dev_ptr: caller-owned device
 * memory (>= vie_batch_workspace_bytes, 256-byte aligned). */
int vie_batch_bind(vie_batch *b, vie_ctx *const *cells, int ncells, void *dev_ptr, size_t bytes);
int vie_batch_set_option(vie_batch *b, int option, int value);
/* Per cell c: wavelength lambda_nm[c], incidence theta[c], phi[c] (radians),
 * permittivities eps_per_tet[c] (that cell's tetrahedra; optics sign). */
int vie_batch_fill(vie_batch *b, const double *lambda_nm, const double *theta, const double *phi,
                   const vie_c128 *const *eps_per_tet);
int vie_batch_factor(vie_batch *b);
/* polarisation [ncells]; info [ncells] (nullable; t_fill_ms, t_factor_ms,
 * t_solve_ms are the batch's).  VIE_ENOCONV if a cell stops at max_iter
 * (every cell's solution and info are still written). */
int vie_batch_solve(vie_batch *b, const int *polarisation, double tol, int max_iter, int restart,
                    vie_solve_info *info);

/* Residual history (estimate / ||b||) of the last solve; returns the count
 * written (at most cap). */
int vie_residual_history(const vie_ctx *ctx, double *hist, int cap);

/* Timing and work counts of the last vie_fill.  Device times come from HIP
 * events on the context's stream around each kernel family.  far_pairs counts
 * the tetrahedron pairs the far kernel evaluated (0 with VIE_GRID_FP64, whose
 * far part is tabulated per sublattice pair: the table build counts in
 * t_face_ms); far_flops is
 * the algorithmic work of the far tetrahedron-pair kernel under the cost model
 * stated in the library source (FMA = 2 FLOPs, per-term operation counts of
 * the lattice-sum evaluation with the fitted degrees of this fill). */
typedef struct {
  double t_fill_ms, t_far_ms, t_near_ms, t_face_ms;
  int64_t far_pairs, near_pairs, face_pairs, far_launches;
  double point_pair_flops, far_flops;
  int nimg, nmode;
  int far_symmetric;   /* 1: the far pairs were evaluated once per unordered pair (VIE_OPT_SYM_FILL) */
} vie_fill_stats;
int vie_get_fill_stats(const vie_ctx *ctx, vie_fill_stats *out);

/* Timing and work counts of the last vie_precond_factor (Sec. 2.3, Eq. 6).
 * t_update_ms sums the device times (HIP events on the context's stream around
 * each launch) of the bulk trailing updates that follow each pair of 64-column
 * panels (K = 128, tournament pivoting only; zero with VIE_OPT_LU_PIVOT = 1);
 * update_flops is their algorithmic work, 8 rows cols 128 real FLOPs per
 * domain and pair (four real products and four sums per complex multiply-add);
 * factor_flops = (8/3) sum_d n_d^3, the whole factorisation's.  VIE_ESTATE
 * before a factorisation. */
typedef struct {
  double t_factor_ms, t_update_ms;
  double update_flops, factor_flops;
  int64_t update_launches;
} vie_factor_stats;
int vie_get_factor_stats(const vie_ctx *ctx, vie_factor_stats *out);

/* Time `reps` back-to-back products y = Z x on the context's stream (HIP
 * events); *ms_per_matvec = average.  Needs a completed fill; uses the
 * solver's work vectors. */
int vie_bench_matvec(vie_ctx *ctx, int reps, double *ms_per_matvec);

/* y = Z x with the bound operator (any precision; Eq. 2's Z of the last
 * fill), x and y host arrays of N values.  Needs a completed fill; uses the
 * solver's work vectors (the stored solutions are kept). */
int vie_apply_Z(vie_ctx *ctx, const vie_c128 *x, vie_c128 *y);

#ifdef __cplusplus
}
#endif

#endif /* VIE_H */
